"""HPMC reference oracle -- TEST INFRASTRUCTURE ONLY.

A plain serial FP64 CPU implementation of the checkerboard hard-shape
Metropolis sweep (Anderson, Irrgang, Glotzer: "Scalable Metropolis Monte Carlo
for simulation of hard shapes", Sec. 2.1-2.5).  Only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import it.  It shares no code
with the GPU library; the C source is ``hpmc_oracle.c`` next to this file.

A species is a plain dict: ``dim``, ``shape`` ("disk" | "polygon" |
"polyhedron"), ``verts`` (n x dim, particle frame; polygons CCW),
``diameter`` (disks), ``d``, ``a``, ``p_rot``, ``rounds`` (0 = auto) and
``sweep_radius`` (polygons and polyhedra swept by a disk / ball; 0 = none).
Positions are (dim, N) float64 arrays (structure of arrays, canonical order),
orientations (2, N) for polygons (c, s) and (4, N) for polyhedra (w, x, y, z).
"""
from .oracle import (  # noqa: F401
    EVENT_NAMES,
    N_STATS,
    STAT_NAMES,
    build,
    count_overlaps,
    event_counts,
    grid,
    index,
    load_counting,
    overlap_full,
    npt_cycles,
    pair_histogram,
    scale_counts,
    scale_positions,
    pair_overlaps,
    philox4x32_10,
    philox4x32_10_many,
    reset_events,
    serial_metropolis,
    shape_info,
    sincos,
    sweep,
    u01,
)

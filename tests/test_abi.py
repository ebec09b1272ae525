"""CPU checks of the C ABI: the library loads, exports every symbol that
include/hpmc.h declares, and its host-side argument validation (grid rule,
shape checks) behaves as documented.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1509_04692_amd import _lib, inputs
from paper_1509_04692_amd.build import LIB_PATH

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "hpmc.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB_PATH):
        pytest.fail("libhpmc.so is not built (run python -m paper_1509_04692_amd.build)")
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpmc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_phase_trace_layout_matches_the_binding(lib):
    """The binding's phase list and kernel list size the buffer of
    hpmc_phase_trace: one word short is rejected before anything runs, the
    full size reaches the build check (the normal build has no clock)."""
    n = len(_lib.TRACED_KERNELS) * (len(_lib.PHASES) + 1)
    buf = (ctypes.c_uint64 * n)()
    assert lib.hpmc_phase_trace(buf, n - 1, 0) == -1
    assert lib.hpmc_phase_trace(buf, n, 0) == -7


def test_strerror(lib):
    assert lib.hpmc_strerror(0) == b"ok"
    assert b"overlap" in lib.hpmc_strerror(-3)
    assert lib.hpmc_strerror(-99) == b"unknown error"


def _args(species_list, Ns, Ls, precision=0, path=0, flags=0, L_max=None):
    n = len(species_list)
    keep = []
    sp_arr = (_lib.Species * n)()
    for r, sp in enumerate(species_list):
        s = sp_arr[r]
        s.dim, s.shape = sp["dim"], _lib.SHAPES[sp["shape"]]
        if sp["shape"] != "disk":
            v = np.ascontiguousarray(sp["verts"], dtype=np.float64)
            keep.append(v)
            s.n_verts = v.shape[0]
            s.verts = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.diameter = sp.get("diameter", 0.0)
        s.d, s.a, s.p_rot, s.rounds = sp["d"], sp["a"], sp["p_rot"], sp.get("rounds", 0)
        s.sweep_radius = sp.get("sweep_radius", 0.0)
    a = _lib.InitArgs()
    a.n_replicas = n
    a.species = sp_arr
    Narr = (ctypes.c_int32 * n)(*Ns)
    Larr = (ctypes.c_double * n)(*Ls)
    a.N, a.L = Narr, Larr
    a.precision, a.path, a.flags = precision, path, flags
    Lmax = None
    if L_max is not None:
        Lmax = (ctypes.c_double * n)(*L_max)
        a.L_max = Lmax
    return a, (keep, sp_arr, Narr, Larr, Lmax)


def ws_bytes(lib, *args, **kw):
    a, keep = _args(*args, **kw)
    out = ctypes.c_size_t()
    rc = lib.hpmc_workspace_bytes(ctypes.byref(a), ctypes.byref(out))
    return rc, out.value


def test_workspace_size_grows_with_the_system(lib):
    sp = inputs.pentagon_species()
    rc1, b1 = ws_bytes(lib, [sp], [4096], [63.70118630129784])
    rc2, b2 = ws_bytes(lib, [sp], [4194304], [2038.438])
    assert rc1 == rc2 == 0
    assert b2 > b1 > 0
    # global cell list: >= 4 B x (cells + 1) + 12 B per particle, and the
    # cell-sorted binary32 coordinates 8 B per particle (2D)
    assert b2 >= 4 * (2038 * 2038 + 1) + 20 * 4194304


def test_box_too_small_and_invalid_shapes(lib):
    disk = inputs.disk_species()
    assert ws_bytes(lib, [disk], [9], [3.9])[0] == -2
    assert ws_bytes(lib, [disk], [16], [4.1])[0] == 0
    cw = dict(inputs.pentagon_species(), verts=inputs.pentagon_species()["verts"][::-1].copy())
    assert ws_bytes(lib, [cw], [100], [20.0])[0] == -1  # clockwise polygon
    bad_rot = dict(disk, p_rot=0.5)
    assert ws_bytes(lib, [bad_rot], [100], [20.0])[0] == -1  # disks do not rotate
    nine = dict(inputs.pentagon_species(), verts=inputs.regular_polygon_vertices(9, 0.5))
    assert ws_bytes(lib, [nine], [100], [20.0])[0] == -1  # more than 8 polygon vertices
    assert ws_bytes(lib, [disk], [0], [20.0])[0] == -1
    assert ws_bytes(lib, [disk], [10], [20.0], precision=5)[0] == -1
    # queue entries carry 26-bit cell-list slots
    assert ws_bytes(lib, [disk], [1 << 26], [10000.0])[0] == -7
    assert ws_bytes(lib, [disk], [(1 << 26) - 1], [10000.0])[0] == 0


def test_persistent_path_limits(lib):
    sp = inputs.pentagon_species()
    # N beyond the 16-bit LDS member index cannot use the persistent path
    assert ws_bytes(lib, [sp], [70000], [400.0], path=2)[0] == -7
    assert ws_bytes(lib, [sp, sp], [4096, 4096], [63.7, 63.7], path=2)[0] == 0


def test_queue_variant_flags(lib):
    sp = inputs.pentagon_species()
    one = ([sp], [4096], [63.70118630129784])
    rc0, b0 = ws_bytes(lib, *one)
    rcr, br = ws_bytes(lib, *one, flags=_lib.QUEUE_FLAGS["register"])
    rcg, bg = ws_bytes(lib, *one, flags=_lib.QUEUE_FLAGS["global"])
    assert rc0 == rcr == rcg == 0
    assert br == b0  # the register queue needs no memory
    # global queue: 8 entries of 8 B per particle, 7 doubles + 4 words per cell
    assert bg - b0 >= 64 * 4096 + 72 * (62 * 62 + 1)
    both = _lib.QUEUE_FLAGS["register"] | _lib.QUEUE_FLAGS["global"]
    assert ws_bytes(lib, *one, flags=both)[0] == -1
    two = ([sp, sp], [4096, 4096], [63.7, 63.7])
    for q in ("register", "global"):
        assert ws_bytes(lib, *two, path=2, flags=_lib.QUEUE_FLAGS[q])[0] == -7  # grid path only
        assert ws_bytes(lib, *two, path=0, flags=_lib.QUEUE_FLAGS[q])[0] == 0   # auto: grid


def test_polygon_rotation_bound(lib):
    """Polygon rotation sizes above HPMC_MAX_POLYGON_ROTATION (0.75 rad) are
    rejected: the unnormalised 2D move is exact to rounding only below it."""
    with open(HEADER) as f:
        bound = float(re.search(r"#define HPMC_MAX_POLYGON_ROTATION ([0-9.]+)", f.read()).group(1))
    assert bound == 0.75
    sp = inputs.pentagon_species()
    assert ws_bytes(lib, [dict(sp, a=bound)], [1024], [32.0])[0] == 0
    assert ws_bytes(lib, [dict(sp, a=float(np.nextafter(bound, 1.0)))], [1024], [32.0])[0] == -1
    assert ws_bytes(lib, [dict(sp, a=float("nan"))], [1024], [32.0])[0] == -1
    # polyhedra renormalise their quaternion: no bound
    assert ws_bytes(lib, [dict(inputs.cube_species(), a=1.5)], [512], [12.0])[0] == 0


def test_sweep_radius_rules(lib):
    sph = inputs.sphere_species(1.0)
    assert ws_bytes(lib, [sph], [512], [8.75])[0] == 0           # one vertex, swept
    assert ws_bytes(lib, [dict(sph, sweep_radius=0.0)], [512], [8.75])[0] == -1
    assert ws_bytes(lib, [dict(sph, sweep_radius=-0.5)], [512], [8.75])[0] == -1
    pent = dict(inputs.pentagon_species(), sweep_radius=0.1)
    assert ws_bytes(lib, [pent], [1024], [32.0])[0] == 0           # a spheropolygon
    assert ws_bytes(lib, [inputs.spherocylinder_species()], [512], [16.5])[0] == 0
    stadium = inputs.stadium_species(1.0, 0.25)
    assert ws_bytes(lib, [stadium], [512], [40.0])[0] == 0         # two-vertex core
    assert ws_bytes(lib, [dict(stadium, sweep_radius=0.0)], [512], [40.0])[0] == -1
    dot = inputs.rounded_polygon_species([[0.0, 0.0]], 0.5)
    assert ws_bytes(lib, [dot], [512], [40.0])[0] == 0             # one-vertex core: a disk
    assert ws_bytes(lib, [dict(disk := inputs.disk_species(), sweep_radius=0.1)], [512], [40.0])[0] == -1
    assert disk["shape"] == "disk"
    # swept polygons run the wave queue only
    for q in ("register", "global"):
        assert ws_bytes(lib, [pent], [1024], [32.0], path=1, flags=_lib.QUEUE_FLAGS[q])[0] == -7
        assert ws_bytes(lib, [inputs.pentagon_species()], [1024], [32.0], path=1,
                        flags=_lib.QUEUE_FLAGS[q])[0] == 0


def test_box_growth_limit(lib):
    """Cell lists are sized for the largest box a volume move may reach."""
    sp = inputs.pentagon_species()
    L = 63.70118630129784
    rc0, b0 = ws_bytes(lib, [sp], [4096], [L])
    rc1, b1 = ws_bytes(lib, [sp], [4096], [L], L_max=[L])
    rc2, b2 = ws_bytes(lib, [sp], [4096], [L], L_max=[1.5 * L])
    assert rc0 == rc1 == rc2 == 0 and b0 == b1 and b2 > b1
    assert ws_bytes(lib, [sp], [4096], [L], L_max=[0.9 * L])[0] == -1  # below L
    assert ws_bytes(lib, [sp], [4096], [L], L_max=[float("inf")])[0] == -1

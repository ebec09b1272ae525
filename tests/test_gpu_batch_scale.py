"""GPU parity at the sizes the benchmark times.

* The headline batch exactly as bench.py builds it: 512 replicas of 4096
  pentagons (phi 0.60), mixed precision, persistent path, autotuned, then
  swept: every replica equals the oracle run with its replica word.
* The full heterogeneous screening batch (512 replicas, disks and
  pentagons, N in [64, 4096], phi in [0.30, 0.70]; two shape kinds launched
  concurrently on their own streams), autotuned and with positions forced
  out of LDS (residency 0).
* 4096 pentagons at the configuration's full 10^4 sweeps, bit for bit.
* Full-length runs too long for the oracle (32768 cubes, 1000 sweeps;
  4,194,304 pentagons, 100 sweeps) are checked by properties that hold at
  any length: no overlap afterwards, every attempted move counted exactly
  once as a cell reject, an overlap reject or an accept, attempted moves per
  sweep and round between half the cell count and the cell count (one move
  per non-empty cell), and rotations drawn with probability p_rot.  (The
  cell-reject fraction has the closed form 1 - (1 - d / 2w)^dim only with at
  most one particle per cell; these systems hold several.)
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1509_04692_amd import inputs

pytestmark = pytest.mark.gpu

PARITY = ("attempted", "attempted_rot", "cell_reject", "overlap_reject", "accept")


def announce(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _system(items, **kw):
    from paper_1509_04692_amd.system import System
    return System([c[0] for c in items], [c[1] for c in items], [c[2] for c in items],
                  [c[3] for c in items], [c[4] for c in items], **kw)


def _check_every_replica(system, items, seed, n_sweeps, t0=0):
    stats = system.stats()
    for r, (sp, N, L, pos, orient) in enumerate(items):
        ref_pos, ref_ori = pos.copy(), orient.copy()
        ref = oracle.sweep(sp, L, ref_pos, ref_ori, seed=seed, n_sweeps=n_sweeps, t0=t0, replica=r)
        assert [stats[r][k] for k in PARITY] == [int(x) for x in ref], r
        assert np.array_equal(system.positions(r), ref_pos), r
        if sp["shape"] != "disk":
            assert np.array_equal(system.orientations(r), ref_ori), r
    assert np.all(system.count_overlaps() == 0)


def test_headline_batch_equals_the_oracle():
    item = inputs.workload_pentagons(4096, 0.60)
    items = [item] * 512
    announce("512 x 4096 pentagons, mixed, persistent, autotuned")
    system = _system(items, precision="mixed", path="persistent")
    system.autotune(trial_sweeps=2)
    system.sweep(3, seed=1)
    _check_every_replica(system, items, 1, 3)


@pytest.mark.parametrize("residency", ["autotuned", "global"])
def test_screening_batch_equals_the_oracle(residency):
    items = inputs.screening_batch(512, seed=2026)
    announce(f"screening batch 512 replicas, mixed, persistent, {residency}")
    system = _system(items, precision="mixed", path="persistent")
    if residency == "autotuned":
        system.autotune(trial_sweeps=2)
    else:
        system.set_config(0)  # particle data in global memory
    system.sweep(2, seed=7)
    _check_every_replica(system, items, 7, 2)


def test_pentagons_global_residency_equals_the_oracle():
    items = [inputs.workload_pentagons(4096, 0.60)] * 8
    announce("8 x 4096 pentagons, fp64 and mixed, persistent, residency 0")
    for precision in ("fp64", "mixed"):
        system = _system(items, precision=precision, path="persistent")
        system.set_config(0)
        system.sweep(4, seed=3)
        _check_every_replica(system, items, 3, 4)
        del system


def test_pentagons_4096_ten_thousand_sweeps():
    sp, N, L, pos, orient = item = inputs.workload_pentagons(4096, 0.60)
    announce("4096 pentagons, 10^4 sweeps, mixed, grid, autotuned")
    system = _system([item], precision="mixed", path="grid")
    system.autotune(trial_sweeps=4)
    system.sweep(10000, seed=1)
    _check_every_replica(system, [item], 1, 10000)


@pytest.mark.parametrize("case", ["cubes_1000", "large_100"])
def test_full_length_properties(case):
    if case == "cubes_1000":
        item = inputs.workload_cubes(32768, 0.45)
        n_sweeps, path = 1000, "grid"
    else:
        item = inputs.workload_pentagons(4194304, 0.60)
        n_sweeps, path = 100, "grid"
    sp, N, L, pos, orient = item
    g = oracle.grid(sp, N, L)
    announce(f"{case}: N={N} {n_sweeps} sweeps, mixed, {path}")
    system = _system([item], precision="mixed", path=path)
    system.sweep(n_sweeps, seed=1)
    st = system.stats()[0]
    assert int(system.count_overlaps()[0]) == 0
    assert st["attempted"] == st["cell_reject"] + st["overlap_reject"] + st["accept"]
    # every sweep attempts one move per non-empty cell and round
    per = st["attempted"] / (n_sweeps * g["rounds"])
    assert 0.5 * g["n"] ** sp["dim"] < per <= g["n"] ** sp["dim"]
    p, n = sp["p_rot"], st["attempted"]
    assert abs(st["attempted_rot"] / n - p) < 5.0 * math.sqrt(p * (1 - p) / n)


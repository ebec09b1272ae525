"""Pins of the oracle's NPT volume move (the paper runs NVT and NPT, Sec. 1).

* Ideal-gas limit: with N particles that (almost) never overlap, volume moves
  uniform in V accepted with min(1, (V'/V)^N exp(-beta P dV)) sample the
  density V^N exp(-beta P V), a Gamma distribution: <V> = (N + 1) / beta P,
  Var V = (N + 1) / (beta P)^2.
* Box scaling: coordinates scale by one factor L'/L and stay in [0, L').
* Compression that would create an overlap is always rejected.
"""
import math

import numpy as np

import oracle
from paper_1509_04692_amd import inputs


def _batch_sem(x, nb=20):
    b = np.array_split(np.asarray(x), nb)
    m = np.array([v.mean() for v in b])
    return m.std(ddof=1) / math.sqrt(nb)


def test_ideal_gas_volume_distribution():
    sp = inputs.disk_species(0.05, d=0.1)
    N, L0, beta_p = 3, 2.0, 1.0
    rng = np.random.Generator(np.random.PCG64(71))
    pos = np.ascontiguousarray(rng.uniform(0.0, L0, size=(2, N)))
    u = inputs.box_move_uniforms(60000, seed=72)
    L, vols = L0, []
    for k in range(0, len(u), 10):
        L, _, _ = oracle.npt_cycles(sp, L, pos, None, seed=1, uniforms=u[k:k + 10],
                                    sweeps_per_cycle=0, beta_p=beta_p, delta_v=3.0, L_max=20.0)
        vols.append(L * L)
    v = np.array(vols[100:])
    # <V> = (N + 1) / beta P and <V^2> = (N + 1)(N + 2) / (beta P)^2
    want1, want2 = (N + 1) / beta_p, (N + 1) * (N + 2) / beta_p ** 2
    assert abs(v.mean() - want1) < 4 * _batch_sem(v) + 0.02, (v.mean(), _batch_sem(v))
    assert abs((v * v).mean() - want2) < 4 * _batch_sem(v * v) + 0.1, ((v * v).mean(),
                                                                       _batch_sem(v * v))


def test_scale_positions_and_wrap():
    rng = np.random.Generator(np.random.PCG64(73))
    L, L2 = 7.0, 5.5
    pos = np.ascontiguousarray(rng.uniform(0.0, L, size=(3, 1000)))
    pos[0, 0] = np.nextafter(L, 0.0)  # the largest coordinate below L
    want = pos * (L2 / L)
    want = np.where(want >= L2, want - L2, want)
    got = pos.copy()
    oracle.scale_positions(got, L, L2)
    assert np.array_equal(got, want)
    assert np.all((got >= 0.0) & (got < L2))


def test_compression_into_overlap_is_rejected():
    sp = inputs.disk_species(1.0, d=0.1)
    # a square lattice at spacing 1.02: any compression below 1/1.02 overlaps
    m, a = 8, 1.02
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), indexing="ij")).reshape(2, -1)
    pos = np.ascontiguousarray((g + 0.5) * a, dtype=np.float64)
    L = m * a
    u = np.array([[0.0, 0.0]])  # dV = -delta_v, always accepted by the exp test
    delta = L * L * (1 - (0.97) ** 2)
    L_after, _, acc = oracle.npt_cycles(sp, L, pos, None, 1, u, 0, 1.0, delta, L_max=100.0)
    assert acc == 0 and L_after == L
    delta = L * L * (1 - (0.995) ** 2)
    L_after, _, acc = oracle.npt_cycles(sp, L, pos, None, 1, u, 0, 1.0, delta, L_max=100.0)
    assert acc == 1 and abs(L_after - 0.995 * L) < 1e-9
    assert oracle.count_overlaps(sp, L_after, pos) == 0

"""The binary32 circumsphere pre-filter of the GPU scan never drops a pair
that the binary64 circumsphere test keeps.

The library's scan compares |r32|^2 with a threshold T computed on the host
(``scan_threshold`` in the HIP sources; restated below): r32 is the binary32
difference of a cell-sorted binary32 copy of the shifted-frame coordinate and
the trial point moved to the neighbour's periodic image.  Here the same
arithmetic is emulated with numpy on pairs placed just inside the
circumsphere, at the largest coordinates (worst binary32 rounding) and across
the periodic edges, and the binary64 test is the oracle's formula
(min image, then x^2 + y^2 (+ z^2)).
"""
import numpy as np
import pytest

U32, U64 = 2.0**-24, 2.0**-53


def scan_threshold(circ2, L, w, dim):
    e = 2.0 * (U32 + U64) * (2.0 * L + 3.0 * w)
    rho = np.sqrt(circ2) * (1.0 + 4.0 * U64) + np.sqrt(dim) * e
    t = rho * rho * (1.0 + 8.0 * U32)
    f = np.float32(t)
    if float(f) < t:
        f = np.nextafter(f, np.float32(np.inf))
    return f


def grid_coord(x, s, L):
    y = x - s
    return np.where(y < 0.0, y + L, y)


def prefilter_r2(xk, xn, s, L, n):
    """Binary32 |r|^2 as the kernel forms it (per-axis reference point of the
    neighbour's periodic image, fused square sum)."""
    inv_w = n / L
    yk, yn = grid_coord(xk, s, L), grid_coord(xn, s, L)
    ck = np.clip((yk * inv_w).astype(np.int64), 0, n - 1)
    cn = np.clip((yn * inv_w).astype(np.int64), 0, n - 1)
    dc = ck - cn
    ref = np.where(dc > 1, yn + L, np.where(dc < -1, yn - L, yn)).astype(np.float32)
    r = yk.astype(np.float32) - ref  # binary32 subtraction
    acc = (r[0].astype(np.float64) * r[0]).astype(np.float32)
    for a in range(1, r.shape[0]):
        acc = (r[a].astype(np.float64) * r[a] + acc.astype(np.float64)).astype(np.float32)
    return acc, np.abs(dc).max(axis=0)


def oracle_r2(xk, xn, L):
    r = xk - xn
    r = r - L * np.rint(r * (1.0 / L))
    r2 = r[0] * r[0] + r[1] * r[1]
    if r.shape[0] == 3:
        r2 = r2 + r[2] * r[2]
    return r2


@pytest.mark.parametrize("dim,L,dmax", [(2, 63.70118630129784, 1.0000000000000002),
                                        (2, 2038.438, 1.0000000000000002),
                                        (2, 20000.0, 0.2),
                                        (3, 40.31747359663594, 1.7320508075688774),
                                        (3, 131.0, 2.23606797749979)])
def test_prefilter_keeps_every_binary64_hit(dim, L, dmax):
    rng = np.random.default_rng(7)
    n = int(L / (dmax * (1.0 + 2.0**-30)))
    n -= n & 1
    w = L / n
    circ2 = dmax * dmax
    T = scan_threshold(circ2, L, w, dim)
    M = 400_000
    s = rng.uniform(0.0, w, size=(dim, 1))
    # trial points near the top of the box (largest coordinates) and anywhere
    xn = np.where(rng.random((dim, M)) < 0.5, L - rng.uniform(0.0, 2.0 * w, (dim, M)),
                  rng.uniform(0.0, L, (dim, M)))
    u = rng.normal(size=(dim, M))
    u /= np.linalg.norm(u, axis=0)
    rad = dmax * (1.0 - rng.uniform(0.0, 1e-4, size=M) ** 2)  # crowd the threshold
    xk = xn + rad * u
    xk = np.where(xk >= L, xk - L, np.where(xk < 0.0, xk + L, xk))
    keep = (xk >= 0.0).all(axis=0) & (xk < L).all(axis=0)
    xn, xk = xn[:, keep], xk[:, keep]
    r64 = oracle_r2(xk, xn, L)
    r32, _ = prefilter_r2(xk, xn, s, L, n)
    hit64 = r64 < circ2
    assert hit64.mean() > 0.5
    missed = hit64 & ~(r32 < T)
    assert not missed.any(), f"{missed.sum()} binary64 hits dropped by the pre-filter"
    # the band is thin where coordinates are small against the shape: pairs
    # 0.1% outside the circumsphere are filtered out (its relative width
    # grows like L / d_max)
    if L / dmax < 5000:
        assert float(T) < circ2 * 1.001**2


def test_threshold_is_a_tight_upper_bound():
    for L in (63.7, 2038.4):
        T = scan_threshold(1.0, L, 1.02, 2)
        assert 1.0 < float(T) < 1.0 + 64 * U32 * (2 * L + 3.06) * 2

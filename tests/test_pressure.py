"""Pins of the pair-separation histogram (oracle) and of the contact-value
pressure estimator (Sec. 4, Table 1)."""
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import oracle
from paper_1509_04692_amd import pressure


def test_oracle_histogram_square_lattice_shells():
    """Square lattice, spacing 1, 8 x 8 periodic: every particle has 4
    neighbours at 1, 4 at sqrt(2), 4 at 2, 8 at sqrt(5) -> 2N, 2N, 2N, 4N pairs."""
    m = 8
    xs, ys = np.meshgrid(np.arange(m) + 0.25, np.arange(m) + 0.5)
    pos = np.stack([xs.ravel(), ys.ravel()])
    N = pos.shape[1]
    edges2 = np.array([0.5, 1.5, 2.5, 3.5, 4.5, 5.5])
    got = oracle.pair_histogram(float(m), pos, edges2)
    assert list(got) == [2 * N, 2 * N, 0, 2 * N, 4 * N]



@pytest.mark.parametrize("dim", [2, 3])
def test_oracle_histogram_matches_periodic_kdtree(dim):
    rng = np.random.default_rng(4)
    N, L = 600, 9.0
    pos = rng.uniform(0.0, L, size=(dim, N))
    radii = np.array([0.3, 0.7, 1.0, 1.6, 2.2, 3.0])
    edges2 = np.concatenate([[0.0], radii ** 2])
    got = oracle.pair_histogram(L, pos, edges2)
    tree = cKDTree(pos.T, boxsize=L)
    cum = np.array([len(tree.query_pairs(r)) for r in radii])  # pairs with d <= r
    assert list(got) == list(np.diff(np.concatenate([[0], cum])))


def test_oracle_histogram_rejects_bad_edges():
    pos = np.zeros((2, 3))
    with pytest.raises(ValueError):
        oracle.pair_histogram(5.0, pos, np.array([1.0, 1.0, 2.0]))


def _shell_mean_g(coef, r0, r1, dim):
    """Exact shell average of the polynomial g(r) = sum coef[k] (r - 1)^k."""
    p = np.polynomial.Polynomial(coef)
    shift = np.polynomial.Polynomial([-1.0, 1.0])  # r - 1
    g = p(shift)
    jac = np.polynomial.Polynomial([0.0, 1.0]) if dim == 2 else np.polynomial.Polynomial([0, 0, 1.0])
    integ = (g * jac).integ()
    norm = jac.integ()
    return (integ(r1) - integ(r0)) / (norm(r1) - norm(r0))


@pytest.mark.parametrize("dim", [2, 3])
def test_contact_value_recovers_a_prescribed_profile(dim):
    coef = [6.676, -45.0, 300.0]
    N, L = 65536, 242.3
    edges = 1.0 + 0.0005 * np.arange(21)
    edges2 = edges ** 2
    g_avg = np.array([_shell_mean_g(coef, a, b, dim) for a, b in zip(edges[:-1], edges[1:])])
    ideal = 0.5 * N * (N - 1) * pressure.shell_measure(edges2, dim) / L ** dim
    g0, r_mid, g = pressure.contact_value(edges2, ideal * g_avg, N, L, 1.0, dim=dim, degree=2)
    assert np.allclose(g, g_avg, rtol=1e-12)
    assert abs(g0 - coef[0]) < 1e-5


def test_disk_pressure_virial_limits():
    # g = 1: second virial coefficient of hard disks, B2 = pi sigma^2 / 2
    N, L = 100, 1000.0
    rho = N / L ** 2
    assert math.isclose(pressure.disk_pressure(N, L, 1.0, 1.0), rho * (1 + 0.5 * math.pi * rho))
    # spheres: B2 = 2 pi sigma^3 / 3
    rho3 = N / L ** 3
    assert math.isclose(pressure.sphere_pressure(N, L, 1.0, 1.0), rho3 * (1 + 2 * math.pi / 3 * rho3))
    # the disk state point of Table 1: phi = 0.698, P* = 9.1707 <-> g(sigma+) = 6.676
    L698 = math.sqrt(65536 * math.pi / 4 / 0.698)
    assert abs(pressure.disk_pressure(65536, L698, 1.0, 6.676) - 9.1707) < 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_scale_route_recovers_the_contact_slope(dim):
    """Counts C(s) of pairs closer than sigma / (1 - s) for a prescribed
    g(r) = g0 + g1 (r - sigma), integrated exactly over the shells, give
    C'(0) = (N (N - 1) / 2V) S_dim sigma^dim g0 (S = 2 pi, 4 pi), hence
    beta P / rho = 1 + C'(0) / (dim N): the virial form of the contact route."""
    N, L, sigma, g0, g1 = 4096, 60.0 if dim == 2 else 20.0, 1.0, 6.0, -9.0
    V = L ** dim
    pref = 0.5 * N * (N - 1) / V
    s = 0.001 * np.arange(1, 21)
    r1 = sigma / (1.0 - s)
    if dim == 2:  # int 2 pi r g(r) dr
        F = lambda r: 2 * math.pi * ((g0 - g1 * sigma) * r ** 2 / 2 + g1 * r ** 3 / 3)
        slope = pref * 2 * math.pi * sigma ** 2 * g0
    else:         # int 4 pi r^2 g(r) dr
        F = lambda r: 4 * math.pi * ((g0 - g1 * sigma) * r ** 3 / 3 + g1 * r ** 4 / 4)
        slope = pref * 4 * math.pi * sigma ** 3 * g0
    counts = pref * (F(r1) - F(sigma))
    got = pressure.scale_slope(s, counts, degree=3)
    assert abs(got / slope - 1) < 1e-6
    rho = N / V
    contact = (pressure.disk_pressure(N, L, sigma, g0 * (N - 1) / N) if dim == 2
               else pressure.sphere_pressure(N, L, sigma, g0 * (N - 1) / N)) / rho
    assert abs(pressure.scale_pressure(N, dim, s, counts, degree=3) - contact) < 1e-6


def _table1():
    rows = {}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_pressures.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            shape, N, phi, serial, one_gpu = line.split()
            rows[shape] = (int(N), float(phi), float(serial.split("(")[0]))
    return rows


def test_validation_drivers_use_the_table_1_state_points():
    """The pressure and NPT checks run the paper's state points and compare
    with its serial values (tests/golden/table1_pressures.txt)."""
    import inspect
    from paper_1509_04692_amd import validate_npt, validate_pressure
    t = _table1()
    src = inspect.getsource(validate_pressure)
    for shape, key in (("disk", "disk"), ("sphere", "sphere"), ("truncated_oct", "trunc_oct")):
        N, phi, p = t[shape]
        assert f"{p}" in src and f"{N}" in src, shape
    npt_src = inspect.getsource(validate_npt)
    assert f'{t["disk"][2]}' in npt_src and f'{t["disk"][1]}' in npt_src
    # the disk state point maps to the contact value used by the pin above
    L = math.sqrt(t["disk"][0] * math.pi / 4 / t["disk"][1])
    assert abs(pressure.disk_pressure(t["disk"][0], L, 1.0, 6.676) - t["disk"][2]) < 1e-3

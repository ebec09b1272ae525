"""The library's certified binary32 overlap tests (mixed precision), built
for the host: the separating-axis filter for polygons and the XenoCollide
walk for polyhedra.  Every decision they certify must equal the oracle's
binary64 decision, and they must certify most pairs.

Pairs: random orientations, centre offsets inside the circumsphere distance,
half of them within 1e-10 .. 1e-2 (relative) of contact, found by bisection
on the oracle along the offset direction.  Shapes: pentagon, triangle and a
random 8-gon; cube, truncated octahedron and a random 40-vertex convex
polyhedron.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle
from paper_1509_04692_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _build(tmp_path_factory, defines=()):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    so = tmp_path_factory.mktemp("mpr32") / "libmpr32_host.so"
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O2", "-ffp-contract=off", "-fPIC",
                    "-shared", *defines, os.path.join(HERE, "certified32_host.hip"), "-o", str(so)],
                   check=True, capture_output=True)
    lib = ctypes.CDLL(str(so))
    P = ctypes.POINTER(ctypes.c_double)
    lib.mpr32_pairs.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.POINTER(ctypes.c_int32)]
    lib.sat32_pairs.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.POINTER(ctypes.c_int32),
                                ctypes.c_double, ctypes.c_int]
    return lib


@pytest.fixture(scope="module")
def mpr32(tmp_path_factory):
    return _build(tmp_path_factory)


def run32(lib, verts, r, qa, qb, fn="mpr32_pairs", *extra):
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    r, qa, qb = (np.ascontiguousarray(x, dtype=np.float64) for x in (r, qa, qb))
    out = np.zeros(len(r), dtype=np.int32)
    P = ctypes.POINTER(ctypes.c_double)
    rc = getattr(lib, fn)(verts.ctypes.data_as(P), len(verts), len(r), r.ctypes.data_as(P),
                         qa.ctypes.data_as(P), qb.ctypes.data_as(P),
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), *extra)
    assert rc == 0, rc
    return out


def random_polyhedron(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v * rng.uniform(0.6, 1.0, size=(n, 1))


def pairs(rng, sp, n):
    lib = oracle.load()
    dim = sp["dim"]
    nq = 2 if dim == 2 else 4
    R = np.sqrt((np.asarray(sp["verts"]) ** 2).sum(axis=1)).max()
    r, qa, qb = [], [], []
    for k in range(n):
        a, b = rng.normal(size=nq), rng.normal(size=nq)
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        d = rng.normal(size=dim)
        d /= np.linalg.norm(d)
        if k % 2:
            s = rng.uniform(0.0, 2.0 * R)
        else:
            lo, hi = 0.0, 2.0 * R
            for _ in range(40):
                mid = 0.5 * (lo + hi)
                if oracle.pair_overlaps(sp, d * mid, a, b, lib=lib):
                    lo = mid
                else:
                    hi = mid
            s = hi * (1.0 + rng.choice([-1.0, 1.0]) * 10.0 ** rng.uniform(-10, -2))
        r.append(d * s)
        qa.append(a)
        qb.append(b)
    return np.array(r), np.array(qa), np.array(qb)


def random_polygon(rng, n):
    ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, size=n))
    rad = rng.uniform(0.7, 1.0, size=n)
    v = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    from scipy.spatial import ConvexHull
    return v[ConvexHull(v).vertices]  # counter-clockwise, strictly convex


POLYGONS = {
    "pentagon": inputs.pentagon_species(),
    "triangle": dict(inputs.pentagon_species(), verts=inputs.regular_polygon_vertices(3, 0.5)),
    "random8": dict(inputs.pentagon_species(), verts=random_polygon(np.random.default_rng(5), 8)),
}


@pytest.mark.parametrize("name,symmetric", [("pentagon", 0), ("pentagon", 1), ("triangle", 0),
                                            ("triangle", 1), ("random8", 0)])
def test_certified_binary32_polygon_filter_equals_the_oracle(mpr32, name, symmetric):
    sp = POLYGONS[name]
    r, za, zb = pairs(np.random.default_rng(13), sp, 6000)
    got = run32(mpr32, sp["verts"], r, za, zb, "sat32_pairs", 1.0, symmetric)
    lib = oracle.load()
    ref = np.array([oracle.pair_overlaps(sp, r[i], za[i], zb[i], lib=lib) for i in range(len(r))])
    sure = got != 2
    assert (got[sure] == ref[sure]).all(), np.flatnonzero(sure & (got != ref))[:10]
    far = np.arange(len(r)) % 2 == 1
    assert sure[far].mean() > 0.999, sure[far].mean()
    assert sure.mean() > 0.6, sure.mean()
    assert ref.mean() > 0.2 and ref.mean() < 0.8


@pytest.mark.parametrize("symmetric", [0, 1])
def test_a_zero_polygon_margin_is_caught(mpr32, symmetric):
    """Sensitivity: with no certification margin the binary32 filter decides
    pairs it cannot resolve, and some differ from the oracle's."""
    sp = POLYGONS["pentagon"]
    r, za, zb = pairs(np.random.default_rng(13), sp, 6000)
    got = run32(mpr32, sp["verts"], r, za, zb, "sat32_pairs", 0.0, symmetric)
    lib = oracle.load()
    ref = np.array([oracle.pair_overlaps(sp, r[i], za[i], zb[i], lib=lib) for i in range(len(r))])
    sure = got != 2
    assert (got[sure] != ref[sure]).sum() > 10


def test_only_symmetric_polygons_take_the_symmetric_filter(mpr32):
    one = (np.zeros((1, 2)), np.array([[1.0, 0.0]]), np.array([[1.0, 0.0]]))
    run32(mpr32, POLYGONS["pentagon"]["verts"], *one, "sat32_pairs", 1.0, 1)
    with pytest.raises(AssertionError, match="-3"):
        run32(mpr32, POLYGONS["random8"]["verts"], *one, "sat32_pairs", 1.0, 1)


SHAPES = {
    "cube": inputs.cube_species(),
    "trunc_oct": inputs.truncated_octahedron_species(),
    "random40": dict(inputs.cube_species(), verts=random_polyhedron(np.random.default_rng(3), 40)),
}


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_certified_binary32_decisions_equal_the_oracle(mpr32, name):
    sp = SHAPES[name]
    rng = np.random.default_rng(11)
    r, qa, qb = pairs(rng, sp, 3000)
    got = run32(mpr32, sp["verts"], r, qa, qb)
    lib = oracle.load()
    ref = np.array([oracle.pair_overlaps(sp, r[i], qa[i], qb[i], lib=lib) for i in range(len(r))])
    sure = got != 2
    assert (got[sure] == ref[sure]).all(), np.flatnonzero(sure & (got != ref))[:10]
    # offsets uniform in the circumsphere distance: nearly all decided in
    # binary32.  Within 1e-2 of contact the portal closes in on a face of the
    # Minkowski difference, whose vertices tie in the support search, so many
    # of those go to binary64 (the choice of a tied vertex cannot be
    # certified).
    near, far = np.arange(len(r)) % 2 == 0, np.arange(len(r)) % 2 == 1
    assert sure[far].mean() > 0.9, sure[far].mean()
    assert sure[near].mean() > 0.05, sure[near].mean()
    assert ref.mean() > 0.2 and ref.mean() < 0.8


def test_coincident_centres_go_to_binary64(mpr32):
    sp = SHAPES["cube"]
    q = np.array([[1.0, 0.0, 0.0, 0.0]])
    assert run32(mpr32, sp["verts"], np.zeros((1, 3)), q, q)[0] == 2
    assert run32(mpr32, sp["verts"], np.array([[1e-9, 0.0, 0.0]]), q, q)[0] == 2


def test_a_shrunken_bound_is_caught(tmp_path_factory):
    """Sensitivity of the comparison above: with the error bounds scaled down
    by 1e-5 the walk certifies decisions that binary32 cannot resolve, and
    some of them differ from the oracle's."""
    bad = _build(tmp_path_factory, ["-DHPMC_MPR32_SLACK=1e-5f"])
    sp = SHAPES["trunc_oct"]
    r, qa, qb = pairs(np.random.default_rng(11), sp, 3000)
    got = run32(bad, sp["verts"], r, qa, qb)
    lib = oracle.load()
    ref = np.array([oracle.pair_overlaps(sp, r[i], qa[i], qb[i], lib=lib) for i in range(len(r))])
    sure = got != 2
    assert (got[sure] != ref[sure]).sum() > 10

"""Pins of the oracle's overlap tests (Sec. 2.3) against independent geometry.

* Disks: overlap iff the centre distance is below the diameter.
* Convex polygons (separating axes in the oracle) against the paper's own
  concave-polygon method -- any proper edge-pair intersection or any vertex
  strictly inside the other shape (Sec. 2.3) -- which is exact for convex
  polygons too; against dense point sampling (a common point proves overlap);
  and, for equal orientations, against the closed form "r_AB inside the
  Minkowski difference A (+) -A" (a decagon for pentagons).
* Convex polyhedra (XenoCollide in the oracle) against full 3D separating
  axes (all face normals plus all edge-edge cross products), against the
  closed form for axis-aligned unit cubes, and against point sampling.
* Spheropolyhedra: spheres and spherocylinders in closed form, rounded
  cubes against core separations and point sampling.
* Spheropolygons (cores overlapping or closer than twice the sweep radius in
  the oracle): one-vertex cores against the disk closed form, two-vertex
  cores against the segment distance, rounded polygons against the sampled
  signed separation of the cores (max over directions of the smallest
  projected vertex difference); monotone in the sweep radius, the plain
  polygon in its small limit, and the hard-disk chain bit for bit.
* Invariants: exchange symmetry and global rotation invariance.

Configurations whose separation or penetration is below 1e-9 are skipped:
there FP64 rounding may legitimately decide either way.
"""
import math

import numpy as np
import pytest
from scipy.spatial import ConvexHull

import oracle
from paper_1509_04692_amd import inputs

MARGIN = 1e-9


# -- 2D reference geometry -----------------------------------------------------

def rot2(z):
    c, s = z
    return np.array([[c, -s], [s, c]])


def world_polygon(verts, z, r):
    return verts @ rot2(z).T + np.asarray(r)


def orient2(a, b, p):
    return (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])


def inside_convex(poly, p):
    n = len(poly)
    return all(orient2(poly[k], poly[(k + 1) % n], p) > 0 for k in range(n))


def edges_or_vertices_overlap(PA, PB):
    """The paper's concave-polygon test: edge pairs and vertices inside."""
    na, nb = len(PA), len(PB)
    for i in range(na):
        p1, p2 = PA[i], PA[(i + 1) % na]
        for j in range(nb):
            q1, q2 = PB[j], PB[(j + 1) % nb]
            d1, d2 = orient2(q1, q2, p1), orient2(q1, q2, p2)
            d3, d4 = orient2(p1, p2, q1), orient2(p1, p2, q2)
            if d1 * d2 < 0 and d3 * d4 < 0:
                return True
    return any(inside_convex(PB, p) for p in PA) or any(inside_convex(PA, q) for q in PB)


def sat_gap_2d(PA, PB):
    """Largest separation along unit edge normals (> 0: apart, < 0: overlap)."""
    best = -np.inf
    for P in (PA, PB):
        n = len(P)
        for k in range(n):
            e = P[(k + 1) % n] - P[k]
            ax = np.array([e[1], -e[0]]) / np.hypot(*e)
            pa, pb = PA @ ax, PB @ ax
            best = max(best, pb.min() - pa.max(), pa.min() - pb.max())
    return best


def random_unit_complex(rng):
    t = rng.uniform(-math.pi, math.pi)
    return np.array([math.cos(t), math.sin(t)])


def polygon_cases(rng, n, R):
    for k in range(n):
        # mostly near contact (inradius-sum .. circumradius-sum), some anywhere
        rr = rng.uniform(1.5 * R, 2.1 * R) if k % 5 else rng.uniform(0, 2.2 * R)
        phi = rng.uniform(-math.pi, math.pi)
        r = np.array([rr * math.cos(phi), rr * math.sin(phi)])
        yield r, random_unit_complex(rng), random_unit_complex(rng)


@pytest.fixture(scope="module")
def pent():
    return inputs.pentagon_species()


def test_disk_overlap_closed_form():
    sp = inputs.disk_species(1.0)
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(3000):
        r = rng.uniform(-1.3, 1.3, size=2)
        d = math.hypot(*r)
        if abs(d - 1.0) < MARGIN:
            continue
        assert oracle.pair_overlaps(sp, r) == (d < 1.0)
    assert not oracle.pair_overlaps(sp, [1.0, 0.0])  # touching is not overlap
    assert oracle.pair_overlaps(sp, [0.0, 0.0])


def test_polygon_sat_matches_edge_and_vertex_test(pent):
    rng = np.random.Generator(np.random.PCG64(12))
    v = pent["verts"]
    checked = n_overlap = 0
    for r, za, zb in polygon_cases(rng, 3000, 0.5):
        PA, PB = world_polygon(v, za, [0, 0]), world_polygon(v, zb, r)
        if abs(sat_gap_2d(PA, PB)) < MARGIN:
            continue
        want = edges_or_vertices_overlap(PA, PB)
        assert oracle.overlap_full(pent, r, za, zb) == want, (r, za, zb)
        checked += 1
        n_overlap += want
    assert checked > 2500 and 0.2 < n_overlap / checked < 0.8


def test_polygon_sat_point_sampling(pent):
    """A sampled point strictly inside both polygons proves overlap."""
    rng = np.random.Generator(np.random.PCG64(13))
    v = pent["verts"]
    proved = 0
    for r, za, zb in polygon_cases(rng, 400, 0.5):
        PA, PB = world_polygon(v, za, [0, 0]), world_polygon(v, zb, r)
        pts = rng.uniform(-0.5, 0.5, size=(400, 2)) + 0.5 * r
        common = any(inside_convex(PA, p) and inside_convex(PB, p) for p in pts)
        if common:
            proved += 1
            assert oracle.overlap_full(pent, r, za, zb)
    assert proved > 50


def test_polygon_equal_orientation_decagon_closed_form(pent):
    v = pent["verts"]
    diff = (v[:, None, :] - v[None, :, :]).reshape(-1, 2)
    hull = ConvexHull(diff)
    assert len(hull.vertices) == 10  # A (+) -A of a regular pentagon is a decagon
    eq = hull.equations  # n . x + d <= 0 inside
    rng = np.random.Generator(np.random.PCG64(14))
    for _ in range(3000):
        r = rng.uniform(-1.05, 1.05, size=2)
        t = rng.uniform(-math.pi, math.pi)
        z = np.array([math.cos(t), math.sin(t)])
        r_world = rot2(z) @ r  # decagon is in the common body frame
        dist = eq[:, :2] @ r + eq[:, 2]
        if np.min(np.abs(dist)) < MARGIN:
            continue
        inside = bool(np.all(dist < 0))
        assert oracle.overlap_full(pent, r_world, z, z) == inside


def test_polygon_exchange_symmetry_and_rotation_invariance(pent):
    rng = np.random.Generator(np.random.PCG64(15))
    v = pent["verts"]
    for r, za, zb in polygon_cases(rng, 1500, 0.5):
        PA, PB = world_polygon(v, za, [0, 0]), world_polygon(v, zb, r)
        if abs(sat_gap_2d(PA, PB)) < MARGIN:
            continue
        base = oracle.overlap_full(pent, r, za, zb)
        assert oracle.overlap_full(pent, -r, zb, za) == base
        g = random_unit_complex(rng)
        gz = lambda z: np.array([g[0] * z[0] - g[1] * z[1], g[1] * z[0] + g[0] * z[1]])
        assert oracle.overlap_full(pent, rot2(g) @ r, gz(za), gz(zb)) == base


@pytest.mark.parametrize("flag", ["ORACLE_PLANT_SAT_SIGN", "ORACLE_PLANT_SAT_A_AXES_ONLY"])
def test_polygon_pins_detect_planted_mistakes(pent, planted, flag):
    lib = planted(flag)
    rng = np.random.Generator(np.random.PCG64(16))
    v = pent["verts"]
    mismatches = 0
    for r, za, zb in polygon_cases(rng, 1500, 0.5):
        PA, PB = world_polygon(v, za, [0, 0]), world_polygon(v, zb, r)
        if abs(sat_gap_2d(PA, PB)) < MARGIN:
            continue
        mismatches += oracle.overlap_full(pent, r, za, zb, lib=lib) != edges_or_vertices_overlap(PA, PB)
    assert mismatches > 0


# -- 3D reference geometry -----------------------------------------------------

def quat_matrix(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def random_quat(rng):
    q = rng.normal(size=4)
    return q / np.linalg.norm(q)


def hull_axes(P):
    h = ConvexHull(P)
    normals = h.equations[:, :3]
    edges = []
    for s in h.simplices:
        for a, b in ((0, 1), (1, 2), (2, 0)):
            edges.append(P[s[b]] - P[s[a]])
    return normals, np.array(edges), h


def sat_gap_3d(PA, PB):
    nA, eA, _ = hull_axes(PA)
    nB, eB, _ = hull_axes(PB)
    cross = np.cross(eA[:, None, :], eB[None, :, :]).reshape(-1, 3)
    nrm = np.linalg.norm(cross, axis=1)
    axes = np.concatenate([nA, nB, cross[nrm > 1e-9] / nrm[nrm > 1e-9, None]])
    pa, pb = PA @ axes.T, PB @ axes.T
    gaps = np.maximum(pb.min(axis=0) - pa.max(axis=0), pa.min(axis=0) - pb.max(axis=0))
    return float(gaps.max())


def polyhedron_cases(rng, n, R):
    for k in range(n):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        rr = rng.uniform(1.0 * R, 2.0 * R) if k % 5 else rng.uniform(0, 2.1 * R)
        yield d * rr, random_quat(rng), random_quat(rng)


SHAPES_3D = {"cube": inputs.cube_species(), "trunc_oct": inputs.truncated_octahedron_species(),
             "dodeca": inputs.dodecahedron_species()}


@pytest.mark.parametrize("name", sorted(SHAPES_3D))
def test_xenocollide_matches_3d_separating_axes(name):
    sp = SHAPES_3D[name]
    v = sp["verts"]
    R = float(np.max(np.linalg.norm(v, axis=1)))
    rng = np.random.Generator(np.random.PCG64(21))
    checked = n_overlap = 0
    for r, qa, qb in polyhedron_cases(rng, 1200, R):
        PA = v @ quat_matrix(qa).T
        PB = v @ quat_matrix(qb).T + r
        gap = sat_gap_3d(PA, PB)
        if abs(gap) < MARGIN:
            continue
        want = gap < 0
        assert oracle.overlap_full(sp, r, qa, qb) == want, (r, qa, qb, gap)
        checked += 1
        n_overlap += want
    assert checked > 1000 and 0.15 < n_overlap / checked < 0.85


def test_xenocollide_axis_aligned_cubes_closed_form():
    sp = SHAPES_3D["cube"]
    rng = np.random.Generator(np.random.PCG64(22))
    ident = [1.0, 0.0, 0.0, 0.0]
    for _ in range(3000):
        r = rng.uniform(-1.2, 1.2, size=3)
        if np.min(np.abs(np.abs(r) - 1.0)) < MARGIN:
            continue
        assert oracle.overlap_full(sp, r, ident, ident) == bool(np.all(np.abs(r) < 1.0)), r


@pytest.mark.parametrize("name", sorted(SHAPES_3D))
def test_xenocollide_point_sampling(name):
    sp = SHAPES_3D[name]
    v = sp["verts"]
    R = float(np.max(np.linalg.norm(v, axis=1)))
    rng = np.random.Generator(np.random.PCG64(23))
    proved = 0
    for r, qa, qb in polyhedron_cases(rng, 300, R):
        PA = v @ quat_matrix(qa).T
        PB = v @ quat_matrix(qb).T + r
        ea, eb = ConvexHull(PA).equations, ConvexHull(PB).equations
        pts = rng.uniform(-R, R, size=(3000, 3)) + 0.5 * r
        ina = np.all(pts @ ea[:, :3].T + ea[:, 3] < 0, axis=1)
        inb = np.all(pts @ eb[:, :3].T + eb[:, 3] < 0, axis=1)
        if np.any(ina & inb):
            proved += 1
            assert oracle.overlap_full(sp, r, qa, qb)
    assert proved > 40


@pytest.mark.parametrize("name", sorted(SHAPES_3D))
def test_xenocollide_exchange_symmetry_and_rotation_invariance(name):
    sp = SHAPES_3D[name]
    v = sp["verts"]
    R = float(np.max(np.linalg.norm(v, axis=1)))
    rng = np.random.Generator(np.random.PCG64(24))

    def qmul(p, q):
        w1, x1, y1, z1 = p
        w2, x2, y2, z2 = q
        return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                         w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                         w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    for r, qa, qb in polyhedron_cases(rng, 500, R):
        PA = v @ quat_matrix(qa).T
        PB = v @ quat_matrix(qb).T + r
        if abs(sat_gap_3d(PA, PB)) < MARGIN:
            continue
        base = oracle.overlap_full(sp, r, qa, qb)
        assert oracle.overlap_full(sp, -r, qb, qa) == base
        g = random_quat(rng)
        assert oracle.overlap_full(sp, quat_matrix(g) @ r, qmul(g, qa), qmul(g, qb)) == base


@pytest.mark.parametrize("flag", ["ORACLE_PLANT_MPR_TRANSPOSE", "ORACLE_PLANT_MPR_PORTAL"])
def test_xenocollide_pins_detect_planted_mistakes(planted, flag):
    lib = planted(flag)
    sp = SHAPES_3D["trunc_oct"]
    v = sp["verts"]
    R = float(np.max(np.linalg.norm(v, axis=1)))
    rng = np.random.Generator(np.random.PCG64(25))
    mismatches = 0
    for r, qa, qb in polyhedron_cases(rng, 600, R):
        PA = v @ quat_matrix(qa).T
        PB = v @ quat_matrix(qb).T + r
        gap = sat_gap_3d(PA, PB)
        if abs(gap) < MARGIN:
            continue
        mismatches += oracle.overlap_full(sp, r, qa, qb, lib=lib) != (gap < 0)
    assert mismatches > 0


# -- spheropolyhedra (hull swept by a ball; support gains s n/|n|) -------------

def _rand_unit(rng):
    d = rng.normal(size=3)
    return d / np.linalg.norm(d)


def test_sphere_closed_form():
    """One-vertex spheropolyhedron of sweep radius 1/2: the unit-diameter
    sphere, overlapping exactly when the centres are closer than 1."""
    sp = inputs.sphere_species(1.0)
    rng = np.random.Generator(np.random.PCG64(41))
    hits = 0
    for _ in range(3000):
        dist = rng.uniform(0.0, 1.3)
        if abs(dist - 1.0) < 1e-9:
            continue
        want = dist < 1.0
        assert oracle.overlap_full(sp, _rand_unit(rng) * dist, random_quat(rng), random_quat(rng)) == want
        hits += want
    assert 0.6 < hits / 3000 < 0.9


def segment_distance(p0, p1, q0, q1):
    """Distance between segments [p0, p1] and [q0, q1]: the convex quadratic
    |r + s d1 - t d2|^2 over the unit square is smallest at its interior
    critical point or on an edge, where the 1D minimiser is clamped."""
    d1, d2, r = p1 - p0, q1 - q0, p0 - q0
    a, e, b = d1 @ d1, d2 @ d2, d1 @ d2
    c, f = d1 @ r, d2 @ r
    cands = []
    m = np.array([[a, -b], [b, -e]])
    if abs(np.linalg.det(m)) > 1e-12:
        s, t = np.linalg.solve(m, [-c, -f])
        if 0.0 <= s <= 1.0 and 0.0 <= t <= 1.0:
            cands.append((s, t))
    for s in (0.0, 1.0):
        cands.append((s, float(np.clip((f + b * s) / e, 0.0, 1.0))))
    for t in (0.0, 1.0):
        cands.append((float(np.clip((b * t - c) / a, 0.0, 1.0)), t))
    return min(np.linalg.norm(r + s * d1 - t * d2) for s, t in cands)


def test_spherocylinder_closed_form():
    """Two-vertex spheropolyhedron: overlap exactly when the core segments are
    closer than twice the sweep radius."""
    sp = inputs.spherocylinder_species(1.0, 0.5)
    rng = np.random.Generator(np.random.PCG64(42))
    ax = np.array([0.0, 0.0, 0.5])
    checked = hits = 0
    for _ in range(3000):
        r = _rand_unit(rng) * rng.uniform(0.0, 2.2)
        qa, qb = random_quat(rng), random_quat(rng)
        ma, mb = quat_matrix(qa), quat_matrix(qb)
        dist = segment_distance(-ma @ ax, ma @ ax, r - mb @ ax, r + mb @ ax)
        if abs(dist - 1.0) < 1e-8:
            continue
        want = dist < 1.0
        assert oracle.overlap_full(sp, r, qa, qb) == want, (r, qa, qb, dist)
        checked += 1
        hits += want
    assert checked > 2900 and 0.2 < hits / checked < 0.8


def test_rounded_cube_bounds_and_sampling():
    """Rounded cubes: cores separated by more than twice the sweep radius on
    some axis never overlap; overlapping cores always do; a sample point
    within the sweep radius of both cores proves an overlap."""
    s = 0.1
    sp = inputs.rounded_cube_species(1.0, s)
    v = sp["verts"]
    rng = np.random.Generator(np.random.PCG64(43))
    apart = cores = proved = 0
    for _ in range(600):
        r = _rand_unit(rng) * rng.uniform(0.5, 2.0)
        qa, qb = random_quat(rng), random_quat(rng)
        ma, mb = quat_matrix(qa), quat_matrix(qb)
        gap = sat_gap_3d(v @ ma.T, v @ mb.T + r)
        got = oracle.overlap_full(sp, r, qa, qb)
        if gap > 2 * s + 1e-9:
            assert not got
            apart += 1
        elif gap < -1e-9:
            assert got
            cores += 1
        else:
            pts = rng.uniform(-1.0, 1.0, size=(4000, 3)) + 0.5 * r
            da = np.linalg.norm(np.maximum(np.abs(pts @ ma) - 0.5, 0.0), axis=1)
            db = np.linalg.norm(np.maximum(np.abs((pts - r) @ mb) - 0.5, 0.0), axis=1)
            if np.any((da < s - 1e-9) & (db < s - 1e-9)):
                assert got
                proved += 1
    assert apart > 50 and cores > 50 and proved > 10


def test_sweep_radius_shape_rules():
    sph = inputs.sphere_species(1.0)
    assert oracle.shape_info(sph)["R"] == math.nextafter(0.5, math.inf)
    rc = inputs.rounded_cube_species(1.0, 0.1)
    assert oracle.shape_info(rc)["R"] == math.nextafter(math.sqrt(0.75) + 0.1, math.inf)
    rp = inputs.rounded_pentagon_species(0.4, 0.1)
    assert oracle.shape_info(rp)["R"] == math.nextafter(0.4 + 0.1, math.inf)
    assert oracle.shape_info(inputs.stadium_species(1.0, 0.25))["R"] == math.nextafter(0.75, math.inf)
    with pytest.raises(ValueError):  # fewer than 4 vertices need a sweep radius
        oracle.shape_info(dict(inputs.spherocylinder_species(), sweep_radius=0.0))
    with pytest.raises(ValueError):  # fewer than 3 polygon vertices need one too
        oracle.shape_info(dict(inputs.stadium_species(), sweep_radius=0.0))
    with pytest.raises(ValueError):  # a swept core must still be convex
        oracle.shape_info(dict(rp, verts=rp["verts"][::-1].copy()))
    with pytest.raises(ValueError):
        oracle.shape_info(dict(inputs.cube_species(), sweep_radius=-0.1))


def test_sweep_pins_detect_a_one_sided_sweep(planted):
    lib = planted("ORACLE_PLANT_SWEEP_ONE_SIDED")
    sp = inputs.sphere_species(1.0)
    rng = np.random.Generator(np.random.PCG64(44))
    mismatches = 0
    for _ in range(300):
        dist = rng.uniform(0.0, 1.3)
        r = _rand_unit(rng) * dist
        mismatches += oracle.overlap_full(sp, r, random_quat(rng), random_quat(rng), lib=lib) != (dist < 1.0)
    assert mismatches > 0


# -- spheropolygons (core polygon swept by a disk of radius s) -----------------
#
# Independent reference: the signed separation of two convex cores,
# D = max over unit directions u of min over vertex pairs u . (b_j - a_k),
# the distance between the cores when they are apart and minus the
# penetration depth when they overlap; the swept shapes overlap exactly when
# D < 2 s.  Sampling u at NDIR angles gives a lower bound within
# (max vertex-pair distance) x (pi / NDIR) of D.

NDIR = 20000
_U = np.stack([np.cos(np.arange(NDIR) * (2 * math.pi / NDIR)),
               np.sin(np.arange(NDIR) * (2 * math.pi / NDIR))], axis=1)


def signed_separation(PA, PB):
    diff = (PB[:, None, :] - PA[None, :, :]).reshape(-1, 2)
    proj = diff @ _U.T
    err = float(np.linalg.norm(diff, axis=1).max()) * (math.pi / NDIR)
    return float(proj.min(axis=0).max()), err


def _random_z(rng):
    t = rng.uniform(0.0, 2.0 * math.pi)
    return np.array([math.cos(t), math.sin(t)])


def test_spheropolygon_one_vertex_is_a_disk():
    """One-vertex core swept by s = 1/2: the unit disk, overlapping exactly
    when the centres are closer than 1, whatever the orientations."""
    sp = inputs.rounded_polygon_species([[0.0, 0.0]], 0.5)
    rng = np.random.Generator(np.random.PCG64(51))
    hits = 0
    for _ in range(3000):
        dist = rng.uniform(0.0, 1.3)
        if abs(dist - 1.0) < 1e-9:
            continue
        want = dist < 1.0
        r = _random_z(rng) * dist
        assert oracle.overlap_full(sp, r, _random_z(rng), _random_z(rng)) == want
        hits += want
    assert 0.6 < hits / 3000 < 0.9


def test_stadium_closed_form():
    """Two-vertex core (a segment) swept by s: overlap exactly when the core
    segments are closer than 2 s (segment distance by the clamped quadratic
    above, crossing segments at distance 0)."""
    s = 0.25
    sp = inputs.stadium_species(1.0, s)
    rng = np.random.Generator(np.random.PCG64(52))
    h = np.array([0.5, 0.0])
    checked = hits = crossing = 0
    for _ in range(3000):
        r = _random_z(rng) * rng.uniform(0.0, 1.6)
        za, zb = _random_z(rng), _random_z(rng)
        ra, rb = rot2(za), rot2(zb)
        dist = segment_distance(-ra @ h, ra @ h, r - rb @ h, r + rb @ h)
        if abs(dist - 2 * s) < 1e-8:
            continue
        want = dist < 2 * s
        assert oracle.overlap_full(sp, r, za, zb) == want, (r, za, zb, dist)
        checked += 1
        hits += want
        crossing += dist < 1e-12
    assert checked > 2900 and 0.2 < hits / checked < 0.8 and crossing > 50


@pytest.mark.parametrize("verts, s", [
    (inputs.regular_polygon_vertices(5, 0.4), 0.1),
    (inputs.regular_polygon_vertices(3, 0.5), 0.05),
    (np.array([[-0.6, -0.2], [0.5, -0.3], [0.4, 0.25], [-0.3, 0.35]]), 0.15),
])
def test_rounded_polygons_against_signed_separation(verts, s):
    """Swept convex polygons against the sampled signed separation of their
    cores, over centre distances from deep overlap to well apart."""
    sp = inputs.rounded_polygon_species(verts, s)
    R = float(np.linalg.norm(verts, axis=1).max()) + s
    rng = np.random.Generator(np.random.PCG64(53))
    apart = overlap = near = 0
    for _ in range(600):
        r = _random_z(rng) * rng.uniform(0.0, 2.3 * R)
        za, zb = _random_z(rng), _random_z(rng)
        D, err = signed_separation(world_polygon(verts, za, [0.0, 0.0]), world_polygon(verts, zb, r))
        got = oracle.overlap_full(sp, r, za, zb)
        if D > 2 * s + 1e-12:  # the sampled D is a lower bound
            assert not got, (r, za, zb, D)
            apart += 1
        elif D < 2 * s - err - 1e-12:
            assert got, (r, za, zb, D)
            overlap += 1
            near += D > 0.0  # cores apart, swept disks meet
    assert apart > 80 and overlap > 150 and near > 30, (apart, overlap, near)


def test_spheropolygon_monotone_in_the_sweep_radius_and_its_limit():
    """A larger sweep radius never removes an overlap; a tiny one decides as
    the plain polygon wherever the cores are not within it of contact."""
    v = inputs.regular_polygon_vertices(5, 0.5)
    plain = inputs.pentagon_species(0.5)
    tiny = inputs.rounded_polygon_species(v, 1e-12)
    small = inputs.rounded_polygon_species(v, 0.05)
    large = inputs.rounded_polygon_species(v, 0.1)
    rng = np.random.Generator(np.random.PCG64(54))
    grew = same = 0
    for _ in range(2000):
        r = _random_z(rng) * rng.uniform(0.5, 1.3)
        za, zb = _random_z(rng), _random_z(rng)
        a, b = oracle.overlap_full(small, r, za, zb), oracle.overlap_full(large, r, za, zb)
        assert b or not a
        grew += b and not a
        gap = sat_gap_2d(world_polygon(v, za, [0.0, 0.0]), world_polygon(v, zb, r))
        if abs(gap) > 1e-9:
            assert oracle.overlap_full(tiny, r, za, zb) == oracle.overlap_full(plain, r, za, zb)
            same += 1
    assert grew > 50 and same > 1900


def test_spheropolygon_exchange_and_rotation_invariance():
    """Swapping the particles (r -> -r) and turning the whole pair by a
    common angle leave the decision unchanged away from contact."""
    v = inputs.regular_polygon_vertices(5, 0.4)
    s = 0.1
    sp = inputs.rounded_polygon_species(v, s)
    rng = np.random.Generator(np.random.PCG64(55))
    checked = 0
    for _ in range(800):
        r = _random_z(rng) * rng.uniform(0.3, 1.2)
        za, zb = _random_z(rng), _random_z(rng)
        D, err = signed_separation(world_polygon(v, za, [0.0, 0.0]), world_polygon(v, zb, r))
        if abs(D - 2 * s) < err + 1e-6:
            continue
        base = oracle.overlap_full(sp, r, za, zb)
        assert oracle.overlap_full(sp, -r, zb, za) == base
        g = _random_z(rng)
        rg = rot2(g)
        zag = np.array([g[0] * za[0] - g[1] * za[1], g[1] * za[0] + g[0] * za[1]])
        zbg = np.array([g[0] * zb[0] - g[1] * zb[1], g[1] * zb[0] + g[0] * zb[1]])
        assert oracle.overlap_full(sp, rg @ r, zag, zbg) == base
        checked += 1
    assert checked > 700


def test_one_vertex_spheropolygons_reproduce_hard_disks():
    """Without rotations, cores of one vertex swept by s are disks of
    diameter 2 s: the checkerboard chain of such a system equals the hard-disk
    chain bit for bit (same draws, same decisions |r|^2 < (2 s)^2)."""
    disk = inputs.disk_species(1.0, d=0.1)
    swept = inputs.rounded_polygon_species([[0.0, 0.0]], 0.5, d=0.1, a=0.0, p_rot=0.0)
    N, phi = 400, 0.55
    L, pos, _ = inputs.initial_state(disk, N, phi)
    assert oracle.grid(disk, N, L) == oracle.grid(swept, N, L)
    p1, p2 = pos.copy(), pos.copy()
    o1 = np.zeros((1, N))
    o2 = inputs.identity_orientations(swept, N)
    st1 = oracle.sweep(disk, L, p1, o1, seed=7, n_sweeps=20)
    st2 = oracle.sweep(swept, L, p2, o2, seed=7, n_sweeps=20)
    assert np.array_equal(p1, p2)
    assert np.array_equal(st1, st2)
    stat = dict(zip(oracle.STAT_NAMES, st1))
    assert stat["accept"] > 0 and stat["overlap_reject"] > 0


def test_spheropolygon_pins_detect_a_one_sided_sweep(planted):
    lib = planted("ORACLE_PLANT_SWEEP_ONE_SIDED")
    sp = inputs.rounded_polygon_species([[0.0, 0.0]], 0.5)
    rng = np.random.Generator(np.random.PCG64(56))
    mismatches = 0
    for _ in range(300):
        dist = rng.uniform(0.0, 1.3)
        r = _random_z(rng) * dist
        mismatches += oracle.overlap_full(sp, r, _random_z(rng), _random_z(rng), lib=lib) != (dist < 1.0)
    assert mismatches > 0


def test_spheropolygon_pins_detect_one_way_distances(planted):
    """Measuring only A's vertices against B's edges misses contacts where a
    vertex of B is nearest to an edge of A."""
    lib = planted("ORACLE_PLANT_SWEPT_ONE_WAY")
    v = inputs.regular_polygon_vertices(5, 0.4)
    s = 0.1
    sp = inputs.rounded_polygon_species(v, s)
    rng = np.random.Generator(np.random.PCG64(57))
    mismatches = 0
    for _ in range(400):
        r = _random_z(rng) * rng.uniform(0.6, 1.2)
        za, zb = _random_z(rng), _random_z(rng)
        D, err = signed_separation(world_polygon(v, za, [0.0, 0.0]), world_polygon(v, zb, r))
        if 0.0 < D < 2 * s - err - 1e-12:
            mismatches += not oracle.overlap_full(sp, r, za, zb, lib=lib)
    assert mismatches > 0


# -- volume-perturbation counts (pairs overlapping after shrinking by 1 - s) ---

def _random_state(dim, N, L, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.uniform(0.0, L, size=(dim, N)))


def test_scale_counts_of_spheres_closed_form():
    """One-vertex spheropolyhedra (unit spheres): pairs with
    |r| (1 - s) < 1 by numpy brute force over the minimum image."""
    sp = inputs.sphere_species(1.0)
    N, L = 300, 9.0
    pos = _random_state(3, N, L, 61)
    ori = inputs.identity_orientations(sp, N)
    s = np.array([0.0, 0.01, 0.05, 0.1, 0.3])
    d = pos[:, None, :] - pos[:, :, None]
    d -= L * np.rint(d / L)
    r = np.sqrt((d ** 2).sum(axis=0))[np.triu_indices(N, 1)]
    for f in 1.0 - s:
        assert np.min(np.abs(r * f - 1.0)) > 1e-9  # no ties in this sample
    want = [int(np.sum(r * (1.0 - x) < 1.0)) for x in s]
    assert list(oracle.scale_counts(sp, L, pos, ori, s)) == want
    assert want[0] < want[-1]


def test_scale_counts_of_aligned_cubes_closed_form():
    """Aligned unit cubes overlap exactly when every |r_a| (1 - s) < 1."""
    sp = inputs.cube_species(1.0)
    N, L = 250, 8.0
    pos = _random_state(3, N, L, 62)
    ori = inputs.identity_orientations(sp, N)
    s = np.array([0.0, 0.02, 0.1, 0.25])
    d = pos[:, None, :] - pos[:, :, None]
    d -= L * np.rint(d / L)
    iu = np.triu_indices(N, 1)
    a = np.abs(d[:, iu[0], iu[1]])
    want = []
    for x in s:
        m = np.max(a * (1.0 - x), axis=0)
        assert np.min(np.abs(m - 1.0)) > 1e-9
        want.append(int(np.sum(m < 1.0)))
    assert list(oracle.scale_counts(sp, L, pos, ori, s)) == want


def test_scale_counts_reject_bad_scales():
    sp = inputs.sphere_species(1.0)
    pos = _random_state(3, 10, 9.0, 63)
    ori = inputs.identity_orientations(sp, 10)
    for bad in ([0.1, 0.05], [1.0], [-0.01]):
        with pytest.raises(ValueError):
            oracle.scale_counts(sp, 9.0, pos, ori, bad)

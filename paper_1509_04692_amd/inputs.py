"""Seeded synthetic workloads: shape vertex tables, box sizes and initial states.

This module holds no step of the Monte Carlo method itself.  It only writes
down the systems the method runs on: particle-frame vertices of the shapes
(given once per type, as in the paper's job-script API, Fig. 1 and Sec. 2.3),
the periodic box length for a packing fraction, and non-overlapping lattice
starting configurations.  The GPU library and the reference oracle both take
their inputs from here; neither is imported by it.

Arrays: positions are (dim, N) float64 (structure of arrays), orientations
(2, N) float64 unit complex numbers (c, s) for polygons and (4, N) unit
quaternions (w, x, y, z) for polyhedra.
"""
import math

import numpy as np

INIT_SEED = 12345


# -- shapes --------------------------------------------------------------------

def regular_polygon_vertices(n_sides=5, circumradius=0.5):
    """Regular polygon, vertex 0 on +y, counter-clockwise."""
    k = np.arange(n_sides)
    ang = math.pi / 2 + 2 * math.pi * k / n_sides
    return np.stack([circumradius * np.cos(ang), circumradius * np.sin(ang)], axis=1)


def polygon_area(verts):
    x, y = verts[:, 0], verts[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def cube_vertices(edge=1.0):
    h = 0.5 * edge
    return np.array([[sx * h, sy * h, sz * h]
                     for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], dtype=np.float64)


def truncated_octahedron_vertices(edge=1.0):
    """All permutations of (0, +-1, +-2), scaled from edge sqrt(2) to `edge`."""
    pts = set()
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        for s1 in (-1, 1):
            for s2 in (-1, 1):
                base = [0.0, s1 * 1.0, s2 * 2.0]
                pts.add(tuple(base[p] for p in perm))
    v = np.array(sorted(pts), dtype=np.float64)
    return v * (edge / math.sqrt(2.0))


GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


def dodecahedron_vertices(edge=1.0):
    """Regular dodecahedron: the cube (+-1, +-1, +-1) and the cyclic
    permutations of (0, +-1/g, +-g), g the golden ratio (edge 2/g), scaled to
    `edge`."""
    g = GOLDEN
    pts = [(sx, sy, sz) for sx in (-1.0, 1.0) for sy in (-1.0, 1.0) for sz in (-1.0, 1.0)]
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            a, b = s1 / g, s2 * g
            pts += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    return np.array(pts, dtype=np.float64) * (edge * g / 2.0)


def dodecahedron_face_normals():
    """Unit outward normals of the 12 pentagonal faces: the cyclic
    permutations of (0, +-g, +-1), normalised (the dual icosahedron)."""
    g = GOLDEN
    out = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            base = np.array([0.0, s1 * g, s2 * 1.0])
            out += [np.roll(base, k) for k in range(3)]
    n = np.array(out)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


CUBE_VOLUME_PER_EDGE3 = 1.0
TRUNC_OCT_VOLUME_PER_EDGE3 = 8.0 * math.sqrt(2.0)
DODECA_VOLUME_PER_EDGE3 = (15.0 + 7.0 * math.sqrt(5.0)) / 4.0
DODECA_INRADIUS_PER_EDGE = GOLDEN ** 2 / (2.0 * math.sqrt(3.0 - GOLDEN))


def disk_species(diameter=1.0, d=0.1):
    return {"dim": 2, "shape": "disk", "diameter": float(diameter), "d": float(d),
            "a": 0.0, "p_rot": 0.0, "rounds": 0, "volume": math.pi * diameter ** 2 / 4}


def pentagon_species(circumradius=0.5, d=0.1, a=0.2, p_rot=0.5):
    v = regular_polygon_vertices(5, circumradius)
    return {"dim": 2, "shape": "polygon", "verts": v, "d": float(d), "a": float(a),
            "p_rot": float(p_rot), "rounds": 0, "volume": polygon_area(v)}


def cube_species(edge=1.0, d=0.08, a=0.1, p_rot=0.5):
    return {"dim": 3, "shape": "polyhedron", "verts": cube_vertices(edge), "d": float(d),
            "a": float(a), "p_rot": float(p_rot), "rounds": 0,
            "volume": CUBE_VOLUME_PER_EDGE3 * edge ** 3}


def truncated_octahedron_species(edge=1.0, d=0.08, a=0.1, p_rot=0.5):
    """Truncated octahedra; the face normals and offsets (6 squares at
    sqrt(2) edge, 8 hexagons at 3/sqrt(6) edge) serve the lattice starts only."""
    ax = np.vstack([np.eye(3), -np.eye(3)])
    diag = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                    dtype=np.float64) / math.sqrt(3.0)
    return {"dim": 3, "shape": "polyhedron", "verts": truncated_octahedron_vertices(edge),
            "d": float(d), "a": float(a), "p_rot": float(p_rot), "rounds": 0,
            "volume": TRUNC_OCT_VOLUME_PER_EDGE3 * edge ** 3,
            "face_normals": np.vstack([ax, diag]),
            "face_offsets": np.concatenate([np.full(6, math.sqrt(2.0) * edge),
                                            np.full(8, 3.0 / math.sqrt(6.0) * edge)])}


def dodecahedron_species(edge=1.0, d=0.08, a=0.1, p_rot=0.5):
    """Regular dodecahedra; the face normals and inradius are kept for the
    lattice start only (the method itself takes just the vertices)."""
    return {"dim": 3, "shape": "polyhedron", "verts": dodecahedron_vertices(edge),
            "d": float(d), "a": float(a), "p_rot": float(p_rot), "rounds": 0,
            "volume": DODECA_VOLUME_PER_EDGE3 * edge ** 3,
            "face_normals": dodecahedron_face_normals(),
            "inradius": DODECA_INRADIUS_PER_EDGE * edge}


# -- spheropolyhedra: a vertex hull swept by a ball (sweep_radius > 0) ----------

def sphere_species(diameter=1.0, d=0.1):
    """A sphere as the one-vertex spheropolyhedron (orientation irrelevant;
    rotation moves off)."""
    r = 0.5 * diameter
    return {"dim": 3, "shape": "polyhedron", "verts": np.zeros((1, 3)), "sweep_radius": r,
            "d": float(d), "a": 0.0, "p_rot": 0.0, "rounds": 0,
            "volume": 4.0 / 3.0 * math.pi * r ** 3}


def spherocylinder_species(length=1.0, radius=0.5, d=0.08, a=0.1, p_rot=0.5):
    """Segment of `length` along z swept by a ball of `radius`."""
    v = np.array([[0.0, 0.0, -0.5 * length], [0.0, 0.0, 0.5 * length]])
    return {"dim": 3, "shape": "polyhedron", "verts": v, "sweep_radius": float(radius),
            "d": float(d), "a": float(a), "p_rot": float(p_rot), "rounds": 0,
            "volume": math.pi * radius ** 2 * length + 4.0 / 3.0 * math.pi * radius ** 3}


def rounded_cube_species(edge=1.0, radius=0.1, d=0.08, a=0.1, p_rot=0.5):
    """Cube of `edge` swept by a ball of `radius`; volume by the Steiner
    formula V + S r + (pi/4) (sum of edge lengths x dihedral defects) r^2 +
    (4/3) pi r^3 = a^3 + 6 a^2 r + 3 pi a r^2 + (4/3) pi r^3."""
    return {"dim": 3, "shape": "polyhedron", "verts": cube_vertices(edge),
            "sweep_radius": float(radius), "d": float(d), "a": float(a),
            "p_rot": float(p_rot), "rounds": 0,
            "volume": edge ** 3 + 6 * edge ** 2 * radius + 3 * math.pi * edge * radius ** 2
            + 4.0 / 3.0 * math.pi * radius ** 3}


# -- spheropolygons: a convex polygon swept by a disk (sweep_radius > 0) ---------

def rounded_polygon_species(verts, radius, d=0.1, a=0.2, p_rot=0.5):
    """Core polygon `verts` (counter-clockwise; one vertex: a disk, two: a
    stadium) swept by a disk of `radius`.  Area by the Steiner formula
    A + P r + pi r^2, P the core's perimeter (twice the length of a segment)."""
    v = np.asarray(verts, dtype=np.float64).reshape(-1, 2)
    perim = float(np.sum(np.linalg.norm(np.roll(v, -1, axis=0) - v, axis=1)))
    core = polygon_area(v) if len(v) >= 3 else 0.0
    return {"dim": 2, "shape": "polygon", "verts": v, "sweep_radius": float(radius),
            "d": float(d), "a": float(a), "p_rot": float(p_rot), "rounds": 0,
            "volume": core + perim * radius + math.pi * radius ** 2}


def stadium_species(length=1.0, radius=0.25, d=0.1, a=0.2, p_rot=0.5):
    """Segment of `length` along x swept by a disk of `radius`."""
    return rounded_polygon_species([[-0.5 * length, 0.0], [0.5 * length, 0.0]], radius, d, a, p_rot)


def rounded_pentagon_species(circumradius=0.4, radius=0.1, d=0.1, a=0.2, p_rot=0.5):
    """Regular pentagon of `circumradius` swept by a disk of `radius`."""
    return rounded_polygon_species(regular_polygon_vertices(5, circumradius), radius, d, a, p_rot)


def box_length(N, particle_volume, phi, dim):
    """Side of the square / cubic periodic box holding N particles at phi."""
    return (N * particle_volume / phi) ** (1.0 / dim)


def aligned_extent(sp):
    """Width of the axis-aligned bounding box of one particle, per axis."""
    if sp["shape"] == "disk":
        return np.full(2, sp["diameter"])
    v = np.asarray(sp["verts"])
    return v.max(axis=0) - v.min(axis=0) + 2.0 * sp.get("sweep_radius", 0.0)


def identity_orientations(sp, N):
    if sp["shape"] == "polygon":
        o = np.zeros((2, N))
        o[0] = 1.0
        return o
    if sp["shape"] == "polyhedron":
        o = np.zeros((4, N))
        o[0] = 1.0
        return o
    return np.zeros((1, max(N, 1)))


# -- initial states ------------------------------------------------------------

def simple_lattice(sp, N, L, seed=INIT_SEED):
    """Aligned particles on a square / cubic lattice of m^dim >= N sites.

    If m^dim > N a seeded random subset of sites is occupied.  Raises if the
    lattice spacing does not clear the aligned bounding box (the particles
    would touch or overlap).
    """
    dim = sp["dim"]
    m = int(math.ceil(N ** (1.0 / dim) - 1e-9))
    while m ** dim < N:
        m += 1
    spacing = L / m
    if np.any(aligned_extent(sp) >= spacing * (1 - 1e-9)):
        raise ValueError(f"lattice spacing {spacing:.4f} too small for the shape")
    grids = np.meshgrid(*[np.arange(m)] * dim, indexing="ij")
    sites = np.stack([g.ravel(order="F") for g in grids], axis=0).astype(np.float64)
    if m ** dim > N:
        rng = np.random.Generator(np.random.PCG64(seed))
        keep = np.sort(rng.choice(m ** dim, size=N, replace=False))
        sites = sites[:, keep]
    pos = np.ascontiguousarray((sites + 0.5) * spacing)
    return pos, identity_orientations(sp, N)


def _check_aligned_lattice(sp, basis, a):
    """Raise unless aligned copies of the shape at every lattice vector of a
    cubic lattice (constant a, sites basis * a) are disjoint.

    Two aligned copies of a centrally symmetric convex body
    K = {x : n_f.x <= h_f} are disjoint exactly when their displacement t has
    max_f n_f.t / h_f > 2, so with face normals given every lattice vector
    shorter than the circumsphere diameter is checked against them; without,
    no lattice vector may be that short.
    """
    R = float(np.linalg.norm(sp["verts"], axis=1).max()) + sp.get("sweep_radius", 0.0)
    normals = sp.get("face_normals")
    if normals is not None:
        h = np.asarray(sp.get("face_offsets", np.full(len(normals), sp.get("inradius", 0.0))))
    rng3 = range(-2, 3)
    for i, j, k in ((i, j, k) for i in rng3 for j in rng3 for k in rng3):
        for b in basis:
            t = (np.array([i, j, k], dtype=np.float64) + b) * a
            dist = np.linalg.norm(t)
            if dist == 0.0 or dist > 2.0 * R * (1 + 1e-9):
                continue
            if normals is None or ((normals @ t) / h).max() <= 2.0 * (1 + 1e-9):
                raise ValueError(f"lattice constant {a:.4f} too small for the shape")


def _cubic_lattice_sites(basis, N, L, seed):
    m = 1
    while len(basis) * m ** 3 < N:
        m += 1
    a = L / m
    cells = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"),
                     axis=0).reshape(3, -1, order="F").T
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3).T.astype(np.float64)
    if sites.shape[1] > N:
        rng = np.random.Generator(np.random.PCG64(seed))
        keep = np.sort(rng.choice(sites.shape[1], size=N, replace=False))
        sites = sites[:, keep]
    return sites, a


_FCC = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
_BCC = np.array([[0, 0, 0], [0.5, 0.5, 0.5]])


def fcc_lattice(sp, N, L, seed=INIT_SEED):
    """Aligned particles on a face-centred cubic lattice of 4 m^3 >= N sites
    (a seeded random subset if larger); raises if aligned copies at the
    lattice vectors would overlap."""
    if sp["dim"] != 3:
        raise ValueError("fcc_lattice needs a 3D species")
    sites, a = _cubic_lattice_sites(_FCC, N, L, seed)
    _check_aligned_lattice(sp, _FCC, a)
    return np.ascontiguousarray((sites + 0.25) * a), identity_orientations(sp, N)


def bcc_lattice(sp, N, L, seed=INIT_SEED):
    """Aligned particles on a body-centred cubic lattice of 2 m^3 >= N sites
    (truncated octahedra tile space on it), checked like fcc_lattice."""
    if sp["dim"] != 3:
        raise ValueError("bcc_lattice needs a 3D species")
    sites, a = _cubic_lattice_sites(_BCC, N, L, seed)
    _check_aligned_lattice(sp, _BCC, a)
    return np.ascontiguousarray((sites + 0.25) * a), identity_orientations(sp, N)


# Up / down interlocked rows for regular pentagons: alternating columns hold
# pentagons rotated by pi, so neighbouring up / down edges are parallel.  For
# circumradius 0.5 the column pitch 2 r_in / cos(18 deg) = 0.8507 and the row
# pitch r_in + R = 0.9045 are the touching distances; both get a 0.5 %
# clearance.  Densest packing fraction reached: about 0.77.
_PENT_COL_PITCH = 0.8507 * 1.005
_PENT_ROW_PITCH = 0.9045 * 1.005


def pentagon_interlocked_lattice(sp, N, L, seed=INIT_SEED):
    R = float(np.max(np.hypot(sp["verts"][:, 0], sp["verts"][:, 1])))
    col = _PENT_COL_PITCH * R / 0.5
    row = _PENT_ROW_PITCH * R / 0.5
    mx = int(L // col)
    mx -= mx % 2
    if mx < 2:
        raise ValueError("box too small for an interlocked pentagon lattice")
    my = -(-N // mx)
    if L / my < row:
        raise ValueError("packing fraction too high for an interlocked pentagon lattice")
    ix, iy = np.meshgrid(np.arange(mx), np.arange(my), indexing="ij")
    ix, iy = ix.ravel(order="F"), iy.ravel(order="F")
    if mx * my > N:
        rng = np.random.Generator(np.random.PCG64(seed))
        keep = np.sort(rng.choice(mx * my, size=N, replace=False))
        ix, iy = ix[keep], iy[keep]
    pos = np.stack([(ix + 0.5) * (L / mx), (iy + 0.5) * (L / my)], axis=0)
    orient = np.zeros((2, N))
    orient[0] = np.where(ix % 2 == 0, 1.0, -1.0)
    return np.ascontiguousarray(pos), orient


def disk_triangular_lattice(sp, N, L, seed=INIT_SEED):
    """Disks on a staggered (triangular) lattice: rows alternately shifted by
    half a column pitch, an even number of rows so the stagger is periodic;
    every neighbour distance at least 1.0001 sigma."""
    sig = sp["diameter"] * 1.0001
    mx = int(L // sig)
    px = L / mx
    if px / 2 >= sig:
        raise ValueError("use the square lattice")
    py_min = math.sqrt(sig * sig - (px / 2) ** 2)
    my = int(L // py_min)
    my -= my % 2
    if my < 2 or mx * my < N:
        raise ValueError("packing fraction too high for a triangular disk lattice")
    ix, iy = np.meshgrid(np.arange(mx), np.arange(my), indexing="ij")
    ix, iy = ix.ravel(order="F"), iy.ravel(order="F")
    if mx * my > N:
        rng = np.random.Generator(np.random.PCG64(seed))
        keep = np.sort(rng.choice(mx * my, size=N, replace=False))
        ix, iy = ix[keep], iy[keep]
    x = (ix + 0.25 + 0.5 * (iy % 2)) * px
    pos = np.stack([x, (iy + 0.5) * (L / my)], axis=0)
    return np.ascontiguousarray(pos), identity_orientations(sp, N)


def initial_state(sp, N, phi, seed=INIT_SEED):
    """(L, pos, orient) of a valid starting configuration at packing fraction phi."""
    L = box_length(N, sp["volume"], phi, sp["dim"])
    try:
        pos, orient = simple_lattice(sp, N, L, seed)
    except ValueError:
        if sp["shape"] == "disk":
            pos, orient = disk_triangular_lattice(sp, N, L, seed)
        elif sp["shape"] == "polygon" and len(sp["verts"]) == 5 and not sp.get("sweep_radius"):
            pos, orient = pentagon_interlocked_lattice(sp, N, L, seed)
        elif sp["shape"] == "polyhedron":
            try:
                pos, orient = fcc_lattice(sp, N, L, seed)
            except ValueError:
                pos, orient = bcc_lattice(sp, N, L, seed)
        else:
            raise
    return L, pos, orient


def box_move_uniforms(n, seed=2028):
    """(n, 2) seeded uniforms in [0, 1) for n NPT volume moves (the proposal
    and the acceptance draw), a PCG64 stream shared by every implementation."""
    return np.random.Generator(np.random.PCG64(seed)).random((n, 2))


# -- workloads -----------------------------------------------------------------

def workload_disks_256():
    """2D hard disks, N=256, sigma=1, phi=0.50, square lattice, d=0.1."""
    sp = disk_species(1.0, d=0.1)
    L, pos, orient = initial_state(sp, 256, 0.50)
    return sp, 256, L, pos, orient


def workload_pentagons(N=4096, phi=0.60):
    """Regular pentagons, circumradius 0.5, d=0.1, a=0.2, p_rot=0.5."""
    sp = pentagon_species(0.5, d=0.1, a=0.2, p_rot=0.5)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def workload_cubes(N=32768, phi=0.45):
    sp = cube_species(1.0, d=0.08, a=0.1, p_rot=0.5)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def workload_truncated_octahedra(N=32768, phi=0.45):
    sp = truncated_octahedron_species(1.0, d=0.08, a=0.1, p_rot=0.5)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def workload_dodecahedra(N=4096, phi=0.50):
    """Regular dodecahedra, edge 1, the paper's second benchmark state (fluid
    at packing fraction 0.5, NVT); translation d=0.08, rotation a=0.1."""
    sp = dodecahedron_species(1.0, d=0.08, a=0.1, p_rot=0.5)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def workload_truncated_octahedra_solid(N=16000, phi=0.70):
    """The paper's truncated-octahedron validation state (Sec. 4, Table 1):
    BCC solid at packing fraction 0.7, aligned; small moves for the solid."""
    sp = truncated_octahedron_species(1.0, d=0.04, a=0.04, p_rot=0.5)
    L = box_length(N, sp["volume"], phi, 3)
    pos, orient = bcc_lattice(sp, N, L)
    return sp, N, L, pos, orient


def workload_spheres(N=4096, phi=0.40):
    sp = sphere_species(1.0, d=0.1)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def workload_spherocylinders(N=4096, phi=0.15):
    """Spherocylinders of aspect (length + 2 radius) / (2 radius) = 2 on a
    simple cubic lattice (whose pitch the long axis sets, hence the low
    packing fraction)."""
    sp = spherocylinder_species(1.0, 0.5, d=0.08, a=0.1, p_rot=0.5)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def workload_rounded_cubes(N=4096, phi=0.45):
    sp = rounded_cube_species(1.0, 0.1, d=0.08, a=0.1, p_rot=0.5)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def workload_rounded_pentagons(N=4096, phi=0.50):
    """Regular pentagons of core circumradius 0.4 swept by a disk of radius
    0.1 (outer circumradius 0.5, like the plain pentagons)."""
    sp = rounded_pentagon_species(0.4, 0.1, d=0.1, a=0.2, p_rot=0.5)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def workload_stadiums(N=4096, phi=0.30):
    """Stadiums: a unit segment swept by a disk of radius 0.25 (aspect
    (1 + 0.5) / 0.5 = 3), on a square lattice (whose pitch the long axis
    sets, hence the low packing fraction)."""
    sp = stadium_species(1.0, 0.25, d=0.1, a=0.2, p_rot=0.5)
    L, pos, orient = initial_state(sp, N, phi)
    return sp, N, L, pos, orient


def screening_manifest(n_replicas=512, seed=2026, n_lo=64, n_hi=4096, phi_lo=0.30,
                       phi_hi=0.70):
    """Heterogeneous batch: replica r even -> disks, odd -> pentagons; N and phi
    drawn uniformly from a seeded PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = rng.integers(n_lo, n_hi + 1, size=n_replicas)
    phis = rng.uniform(phi_lo, phi_hi, size=n_replicas)
    return [("disk" if r % 2 == 0 else "pentagon", int(Ns[r]), float(phis[r]))
            for r in range(n_replicas)]


def screening_batch(n_replicas=512, seed=2026, **kw):
    """Species, N, L, pos, orient lists of the heterogeneous screening batch."""
    out = []
    for kind, N, phi in screening_manifest(n_replicas, seed, **kw):
        sp = disk_species(1.0, d=0.1) if kind == "disk" else pentagon_species(0.5, 0.1, 0.2, 0.5)
        L, pos, orient = initial_state(sp, N, phi)
        out.append((sp, N, L, pos, orient))
    return out

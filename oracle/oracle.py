"""ctypes binding of the reference oracle (test infrastructure only).

Argument marshalling only: every computation happens in ``hpmc_oracle.c``.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hpmc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# Plain C with IEEE binary64 evaluation in source order: no contraction into
# fused multiply-adds, no fast-math reassociation.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared"]

STAT_NAMES = ("attempted", "attempted_rot", "cell_reject", "overlap_reject", "accept")
N_STATS = len(STAT_NAMES)
_SHAPES = {"disk": 0, "polygon": 1, "polyhedron": 2}

_lib = None
_lib_ops = None
_LIB_OPS_PATH = os.path.join(_HERE, "liboracle_ops.so")

# Event counters of the ORACLE_COUNT_OPS build, in the order of hpmc_oracle.c.
EVENT_NAMES = ("translate", "rotate2", "rotate3", "cand2", "cand3", "sat_setup", "sat_axis",
               "sat_frame_b", "mpr_setup", "mpr_support", "mpr_iter", "seg_setup", "seg_test")


def build(extra_flags=(), out_path=None):
    """Compile hpmc_oracle.c with gcc into a shared library; returns its path."""
    out = out_path or _LIB_PATH
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", out + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(out + ".tmp", out)
    return out


class _Species(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("shape", ctypes.c_int32),
        ("n_verts", ctypes.c_int32),
        ("verts", ctypes.POINTER(ctypes.c_double)),
        ("diameter", ctypes.c_double),
        ("d", ctypes.c_double),
        ("a", ctypes.c_double),
        ("p_rot", ctypes.c_double),
        ("rounds", ctypes.c_int32),
        ("sweep_radius", ctypes.c_double),
    ]


_P_D = ctypes.POINTER(ctypes.c_double)
_P_U32 = ctypes.POINTER(ctypes.c_uint32)
_P_I64 = ctypes.POINTER(ctypes.c_int64)


def _declare(lib):
    sp = ctypes.POINTER(_Species)
    lib.or_philox4x32_10.argtypes = [_P_U32, _P_U32, _P_U32]
    lib.or_philox4x32_10.restype = None
    lib.or_philox4x32_10_many.argtypes = [_P_U32, ctypes.c_int64, _P_U32, _P_U32]
    lib.or_philox4x32_10_many.restype = None
    lib.or_u01.argtypes = [ctypes.c_uint32]
    lib.or_u01.restype = ctypes.c_double
    lib.or_index.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.or_index.restype = ctypes.c_uint32
    lib.or_sincos.argtypes = [ctypes.c_double, _P_D, _P_D]
    lib.or_sincos.restype = None
    lib.or_shape_info.argtypes = [sp, _P_D]
    lib.or_shape_info.restype = ctypes.c_int
    lib.or_grid.argtypes = [sp, ctypes.c_int32, ctypes.c_double,
                            ctypes.POINTER(ctypes.c_int32), _P_D,
                            ctypes.POINTER(ctypes.c_int32)]
    lib.or_grid.restype = ctypes.c_int
    lib.or_overlap_full.argtypes = [sp, _P_D, _P_D, _P_D]
    lib.or_overlap_full.restype = ctypes.c_int
    lib.or_pair_overlaps.argtypes = [sp, _P_D, _P_D, _P_D]
    lib.or_pair_overlaps.restype = ctypes.c_int
    lib.or_pair_histogram.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _P_D, _P_D,
                                      ctypes.c_int32, _P_I64]
    lib.or_pair_histogram.restype = ctypes.c_int
    lib.or_scale_counts.argtypes = [sp, ctypes.c_int32, ctypes.c_double, _P_D, _P_D, _P_D,
                                    ctypes.c_int32, _P_I64]
    lib.or_scale_counts.restype = ctypes.c_int
    lib.or_scale_positions.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_double, _P_D]
    lib.or_scale_positions.restype = ctypes.c_int
    lib.or_count_overlaps.argtypes = [sp, ctypes.c_int32, ctypes.c_double, _P_D, _P_D]
    lib.or_count_overlaps.restype = ctypes.c_int64
    lib.or_sweep.argtypes = [sp, ctypes.c_int32, ctypes.c_double, _P_D, _P_D,
                             ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.c_uint64, _P_I64]
    lib.or_sweep.restype = ctypes.c_int
    lib.or_serial_metropolis.argtypes = [sp, ctypes.c_int32, ctypes.c_double, _P_D, _P_D,
                                         ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         _P_I64]
    lib.or_serial_metropolis.restype = ctypes.c_int


def _stale(lib_path):
    """True when the library is missing or older than the C source or header."""
    if not os.path.exists(lib_path):
        return True
    t = os.path.getmtime(lib_path)
    return any(os.path.getmtime(os.path.join(_HERE, f)) > t for f in ("hpmc_oracle.c", "hpmc_oracle.h"))


def load(path=None):
    """Load (building first if absent) the oracle library."""
    global _lib
    if path is not None:
        lib = ctypes.CDLL(path)
        _declare(lib)
        return lib
    if _lib is None:
        if _stale(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


def load_counting():
    """The event-counting build (ORACLE_COUNT_OPS), built on first use."""
    global _lib_ops
    if _lib_ops is None:
        if _stale(_LIB_OPS_PATH):
            build(extra_flags=["-DORACLE_COUNT_OPS"], out_path=_LIB_OPS_PATH)
        lib = ctypes.CDLL(_LIB_OPS_PATH)
        _declare(lib)
        lib.or_event_counts.restype = ctypes.POINTER(ctypes.c_int64)
        lib.or_n_events.restype = ctypes.c_int32
        assert lib.or_n_events() == len(EVENT_NAMES)
        _lib_ops = lib
    return _lib_ops


def event_counts(lib):
    """Copy of the event counters of a counting build, as a dict."""
    ptr = lib.or_event_counts()
    return {name: int(ptr[k]) for k, name in enumerate(EVENT_NAMES)}


def reset_events(lib):
    ptr = lib.or_event_counts()
    for k in range(len(EVENT_NAMES)):
        ptr[k] = 0


def _species(sp):
    """Marshal a species dict; returns (struct, keep-alive array)."""
    verts = np.ascontiguousarray(np.asarray(sp.get("verts", np.zeros((0, sp["dim"]))),
                                            dtype=np.float64))
    s = _Species()
    s.dim = int(sp["dim"])
    s.shape = _SHAPES[sp["shape"]]
    s.n_verts = int(verts.shape[0]) if verts.ndim == 2 else 0
    s.verts = verts.ctypes.data_as(_P_D) if verts.size else ctypes.cast(None, _P_D)
    s.diameter = float(sp.get("diameter", 0.0))
    s.d = float(sp.get("d", 0.0))
    s.a = float(sp.get("a", 0.0))
    s.p_rot = float(sp.get("p_rot", 0.0))
    s.rounds = int(sp.get("rounds", 0))
    s.sweep_radius = float(sp.get("sweep_radius", 0.0))
    return s, verts


def _dptr(a):
    return a.ctypes.data_as(_P_D)


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} failed with code {rc}")
    return rc


def philox4x32_10(ctr, key, lib=None):
    lib = lib or load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib.or_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def philox4x32_10_many(ctr, key, lib=None):
    """Philox4x32-10 of every row of an (n, 4) uint32 counter array."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros_like(ctr)
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    (lib or load()).or_philox4x32_10_many(ctr.ctypes.data_as(_P_U32), int(ctr.shape[0]), k,
                                          out.ctypes.data_as(_P_U32))
    return out


def u01(w, lib=None):
    return (lib or load()).or_u01(int(w))


def index(w, n, lib=None):
    return int((lib or load()).or_index(int(w), int(n)))


def sincos(delta, lib=None):
    c, s = ctypes.c_double(), ctypes.c_double()
    (lib or load()).or_sincos(float(delta), ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def shape_info(sp, lib=None):
    s, _keep = _species(sp)
    out = (ctypes.c_double * 4)()
    _check((lib or load()).or_shape_info(ctypes.byref(s), out), "shape_info")
    return {"R": out[0], "dmax": out[1], "circ2": out[2], "tol2": out[3]}


def grid(sp, N, L, lib=None):
    s, _keep = _species(sp)
    n, rounds, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check((lib or load()).or_grid(ctypes.byref(s), int(N), float(L), ctypes.byref(n),
                                   ctypes.byref(w), ctypes.byref(rounds)), "grid")
    return {"n": n.value, "w": w.value, "rounds": rounds.value}


def _q(q):
    a = np.zeros(4, dtype=np.float64)
    if q is not None:
        q = np.asarray(q, dtype=np.float64).ravel()
        a[: q.size] = q
    return a


def overlap_full(sp, r, qa=None, qb=None, lib=None):
    s, _keep = _species(sp)
    r = np.zeros(3) + np.pad(np.asarray(r, dtype=np.float64).ravel(), (0, 3))[:3]
    qa, qb = _q(qa), _q(qb)
    return bool(_check((lib or load()).or_overlap_full(ctypes.byref(s), _dptr(r), _dptr(qa),
                                                       _dptr(qb)), "overlap_full"))


def pair_overlaps(sp, r, qa=None, qb=None, lib=None):
    s, _keep = _species(sp)
    r = np.zeros(3) + np.pad(np.asarray(r, dtype=np.float64).ravel(), (0, 3))[:3]
    qa, qb = _q(qa), _q(qb)
    return bool(_check((lib or load()).or_pair_overlaps(ctypes.byref(s), _dptr(r), _dptr(qa),
                                                        _dptr(qb)), "pair_overlaps"))


def _state(sp, pos, orient):
    pos = np.asarray(pos)
    if pos.dtype != np.float64 or not pos.flags.c_contiguous or pos.shape[0] != sp["dim"]:
        raise ValueError("pos must be a C-contiguous (dim, N) float64 array")
    N = pos.shape[1]
    if orient is None:
        orient = np.zeros((1, max(N, 1)), dtype=np.float64)
    if orient.dtype != np.float64 or not orient.flags.c_contiguous:
        raise ValueError("orient must be C-contiguous float64")
    return N, pos, orient


def count_overlaps(sp, L, pos, orient=None, lib=None):
    s, _keep = _species(sp)
    N, pos, orient = _state(sp, pos, orient)
    return int(_check((lib or load()).or_count_overlaps(ctypes.byref(s), N, float(L), _dptr(pos),
                                                        _dptr(orient)), "count_overlaps"))


def pair_histogram(L, pos, edges2, lib=None):
    """Counts of unordered pairs with edges2[b] <= r^2 < edges2[b+1] (minimum
    image); pos is (dim, N) float64."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    edges2 = np.ascontiguousarray(edges2, dtype=np.float64)
    out = np.zeros(len(edges2) - 1, dtype=np.int64)
    _check((lib or load()).or_pair_histogram(pos.shape[0], pos.shape[1], float(L), _dptr(pos),
                                             _dptr(edges2), len(out),
                                             out.ctypes.data_as(_P_I64)), "pair_histogram")
    return out


def scale_counts(sp, L, pos, orient, scales, lib=None):
    """Unordered pairs overlapping once their separation is scaled by
    1 - scales[b], for each b (volume-perturbation pressure, Sec. 4)."""
    s, _keep = _species(sp)
    N, pos, orient = _state(sp, pos, orient)
    sc = np.ascontiguousarray(scales, dtype=np.float64)
    out = np.zeros(len(sc), dtype=np.int64)
    _check((lib or load()).or_scale_counts(ctypes.byref(s), N, float(L), _dptr(pos), _dptr(orient),
                                           _dptr(sc), len(sc), out.ctypes.data_as(_P_I64)),
           "scale_counts")
    return out


def scale_positions(pos, L, L_new, lib=None):
    """Scale (dim, N) positions in place from box L to box L_new."""
    _check((lib or load()).or_scale_positions(pos.shape[0], pos.shape[1], float(L), float(L_new),
                                              _dptr(pos)), "scale_positions")


def npt_cycles(sp, L, pos, orient, seed, uniforms, sweeps_per_cycle, beta_p, delta_v, L_max,
               t0=0, replica=0, lib=None):
    """Isothermal-isobaric chain: each cycle runs sweeps_per_cycle checkerboard
    sweeps, then one isotropic volume move V -> V + delta_v (2 u1 - 1) with
    the uniforms (u1, u2) of that cycle.  The move is rejected if V' <= 0,
    L' = V'^(1/dim) exceeds L_max or gives fewer than 4 cells per side, or
    (when shrinking) the scaled state has an overlapping pair; otherwise it
    is accepted with probability min(1, exp(arg)), arg = -beta_p dV +
    N ln(V'/V) (Frenkel & Smit's NPT volume move for hard particles): since
    u2 < 1, arg >= 0 always accepts, else u2 < exp(arg) decides.  pos/orient are updated in place;
    returns (L, sweep stats, accepted box moves)."""
    dim, N = sp["dim"], pos.shape[1]
    stats = np.zeros(N_STATS, dtype=np.int64)
    t, accepted = t0, 0
    for u1, u2 in uniforms:
        stats += sweep(sp, L, pos, orient, seed, sweeps_per_cycle, t0=t, replica=replica, lib=lib)
        t += sweeps_per_cycle
        V = L ** dim
        dV = delta_v * (2.0 * u1 - 1.0)
        V2 = V + dV
        if not V2 > 0.0:
            continue
        L2 = V2 ** (1.0 / dim)
        if L2 > L_max:
            continue
        try:
            grid(sp, N, L2, lib=lib)
        except ValueError:
            continue
        trial = pos.copy()
        scale_positions(trial, L, L2, lib=lib)
        if dV < 0.0 and count_overlaps(sp, L2, trial, orient, lib=lib) > 0:
            continue
        arg = -beta_p * dV + N * math.log(V2 / V)
        if not (arg >= 0.0 or u2 < math.exp(arg)):
            continue
        pos[...] = trial
        L = L2
        accepted += 1
    return L, stats, accepted


def sweep(sp, L, pos, orient, seed, n_sweeps, t0=0, replica=0, lib=None):
    """Run n_sweeps sweeps in place; returns the int64 stats of this call."""
    s, _keep = _species(sp)
    N, pos, orient = _state(sp, pos, orient)
    stats = np.zeros(N_STATS, dtype=np.int64)
    _check((lib or load()).or_sweep(ctypes.byref(s), N, float(L), _dptr(pos), _dptr(orient),
                                    int(seed), int(replica), int(t0), int(n_sweeps),
                                    stats.ctypes.data_as(_P_I64)), "sweep")
    return stats


def serial_metropolis(sp, L, pos, orient, seed, n_moves, move0=0, lib=None):
    s, _keep = _species(sp)
    N, pos, orient = _state(sp, pos, orient)
    stats = np.zeros(N_STATS, dtype=np.int64)
    _check((lib or load()).or_serial_metropolis(ctypes.byref(s), N, float(L), _dptr(pos),
                                                _dptr(orient), int(seed), int(move0),
                                                int(n_moves), stats.ctypes.data_as(_P_I64)),
           "serial_metropolis")
    return stats

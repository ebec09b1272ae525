"""ctypes binding of libhpmc.so (argument marshalling only).

The library is built in-tree by ``python -m paper_1509_04692_amd.build``.
Loading fails loudly when it is missing: there is no fallback
implementation.
"""
import ctypes
import os

from .build import LIB_PATH

HPMC_OK = 0
ERRORS = {
    -1: "invalid argument",
    -2: "box too small: fewer than 4 cells per side",
    -3: "initial configuration has overlapping particles",
    -4: "workspace too small",
    -5: "HIP runtime error",
    -6: "sweep counter would exceed 2^32",
    -7: "unsupported configuration",
    -8: "cell list overflow (overlapping state)",
}
SHAPES = {"disk": 0, "polygon": 1, "polyhedron": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
PATHS = {"auto": 0, "grid": 1, "persistent": 2}
STAT_FIELDS = ("attempted", "attempted_rot", "cell_reject", "overlap_reject", "accept",
               "pair_tests", "pair_fp64", "sweeps")

# Every symbol include/hpmc.h declares.
EXPORTS = ("hpmc_workspace_bytes", "hpmc_init", "hpmc_sweep", "hpmc_autotune", "hpmc_set_config",
           "hpmc_count_overlaps", "hpmc_pair_histogram", "hpmc_scale_counts", "hpmc_scale_box",
           "hpmc_restore_box", "hpmc_get_stats", "hpmc_reset_stats",
           "hpmc_sync_to_canonical", "hpmc_get_sweep", "hpmc_set_sweep", "hpmc_replica_info",
           "hpmc_uses_graph", "hpmc_graph_sweeps", "hpmc_volume_move", "hpmc_last_hip_error",
           "hpmc_destroy", "hpmc_strerror", "hpmc_phase_trace", "hpmc_sweep_static")
FLAG_NO_GRAPH = 1
QUEUE_FLAGS = {"wave": 0, "register": 2, "global": 4}  # HPMC_FLAG_*_QUEUE


class HpmcError(RuntimeError):
    def __init__(self, code, what, hip_error=0):
        msg = f"{what}: {ERRORS.get(code, 'unknown error')} (code {code})"
        if hip_error:
            msg += f", hipError_t {hip_error}"
        super().__init__(msg)
        self.code = code


class Species(ctypes.Structure):
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


class InitArgs(ctypes.Structure):
    _fields_ = [
        ("n_replicas", ctypes.c_int32),
        ("species", ctypes.POINTER(Species)),
        ("N", ctypes.POINTER(ctypes.c_int32)),
        ("L", ctypes.POINTER(ctypes.c_double)),
        ("precision", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("pos", ctypes.c_void_p),
        ("orient", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("flags", ctypes.c_int32),
        ("L_max", ctypes.POINTER(ctypes.c_double)),
    ]


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in STAT_FIELDS]


_lib = None


# order of the phase enum; the build_* phases split the persistent kernel's
# in-LDS cell-list build ("build" is then its clearing of the counts)
PHASES = ("build", "propose", "scan", "drain", "write", "barrier", "other",
          "build_count", "build_prefix", "build_scatter", "build_sort")
TRACED_KERNELS = ("k_batch", "k_update")


def load(path=None):
    """Load libhpmc.so; raises OSError if it has not been built.  The
    environment variable HPMC_LIBRARY names another build to load instead
    (the phase-trace build, lib/libhpmc_trace.so)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or os.environ.get("HPMC_LIBRARY") or LIB_PATH
    if not os.path.exists(p):
        raise OSError(f"{p} is missing: build it with python -m paper_1509_04692_amd.build")
    lib = ctypes.CDLL(p)
    st = ctypes.c_void_p
    lib.hpmc_workspace_bytes.argtypes = [ctypes.POINTER(InitArgs), ctypes.POINTER(ctypes.c_size_t)]
    lib.hpmc_init.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(InitArgs)]
    lib.hpmc_sweep.argtypes = [st, ctypes.c_uint64, ctypes.c_uint64]
    lib.hpmc_autotune.argtypes = [st, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int32)]
    lib.hpmc_set_config.argtypes = [st, ctypes.c_int32]
    lib.hpmc_uses_graph.argtypes = [st]
    lib.hpmc_count_overlaps.argtypes = [st, ctypes.POINTER(ctypes.c_uint64)]
    lib.hpmc_pair_histogram.argtypes = [st, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
    lib.hpmc_scale_counts.argtypes = [st, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
    lib.hpmc_scale_box.argtypes = [st, ctypes.c_int32, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_uint64)]
    lib.hpmc_restore_box.argtypes = [st, ctypes.c_int32]
    lib.hpmc_volume_move.argtypes = [st, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.hpmc_graph_sweeps.argtypes = [st, ctypes.POINTER(ctypes.c_uint64)]
    lib.hpmc_phase_trace.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32, ctypes.c_int32]
    lib.hpmc_sweep_static.argtypes = [ctypes.POINTER(InitArgs), ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.POINTER(Stats),
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.hpmc_get_stats.argtypes = [st, ctypes.POINTER(Stats)]
    lib.hpmc_reset_stats.argtypes = [st]
    lib.hpmc_sync_to_canonical.argtypes = [st]
    lib.hpmc_get_sweep.argtypes = [st, ctypes.POINTER(ctypes.c_uint64)]
    lib.hpmc_set_sweep.argtypes = [st, ctypes.c_uint64]
    lib.hpmc_replica_info.argtypes = [st, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.hpmc_last_hip_error.argtypes = [st]
    lib.hpmc_destroy.argtypes = [st]
    lib.hpmc_destroy.restype = None
    lib.hpmc_strerror.argtypes = [ctypes.c_int]
    lib.hpmc_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("hpmc_destroy", "hpmc_strerror"):
            getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib

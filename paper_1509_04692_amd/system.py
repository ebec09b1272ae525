"""Python front end of libhpmc: device buffers and streams come from PyTorch,
every step of the sweep runs in the library's HIP kernels.

    sys = System(species, N, L, pos, orient, precision="mixed")
    sys.sweep(1000, seed=1)           # like the paper's hoomd.run(n) (Fig. 1)
    sys.count_overlaps()              # system-level overlap check (Sec. 4)
    sys.stats()

``L_max`` (per replica, default L) bounds the box sides that volume moves
(``scale_box``, the NPT driver in ``npt.py``) may reach.

``queue`` picks how a pass schedules its full overlap tests: "wave" (the
block work queue, per wave64 in LDS; the default), or the paper's two
comparison variants "register" and "global" (grid path only).

``species`` is a dict (or one per replica) with keys dim, shape ("disk",
"polygon", "polyhedron"), verts (n x dim), diameter, d, a, p_rot, rounds and
(polygons and polyhedra) sweep_radius,
as produced by ``paper_1509_04692_amd.inputs``.
"""
import ctypes

import numpy as np

from . import _lib

_NCOMP = {"disk": 0, "polygon": 2, "polyhedron": 4}


def _as_list(x, n):
    if isinstance(x, (list, tuple)):
        if len(x) != n:
            raise ValueError("per-replica argument has the wrong length")
        return list(x)
    return [x] * n


def init_args(species, N, L, pos, orient, precision, path, stream, flags=0, L_max=None):
    """hpmc_init_args for replicas with the given species / N / L lists and
    device tensors pos / orient (replicas concatenated, hpmc.h layout).
    Returns (args, objects that must outlive the call)."""
    n_rep = len(species)
    keep = []
    sp_arr = (_lib.Species * n_rep)()
    for r, sp in enumerate(species):
        s = sp_arr[r]
        s.dim = int(sp["dim"])
        s.shape = _lib.SHAPES[sp["shape"]]
        if sp["shape"] != "disk":
            v = np.ascontiguousarray(np.asarray(sp["verts"], dtype=np.float64))
            keep.append(v)
            s.n_verts = v.shape[0]
            s.verts = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.diameter = float(sp.get("diameter", 0.0))
        s.d = float(sp.get("d", 0.0))
        s.a = float(sp.get("a", 0.0))
        s.p_rot = float(sp.get("p_rot", 0.0))
        s.rounds = int(sp.get("rounds", 0))
        s.sweep_radius = float(sp.get("sweep_radius", 0.0))
    N_arr = (ctypes.c_int32 * n_rep)(*[int(x) for x in N])
    L_arr = (ctypes.c_double * n_rep)(*[float(x) for x in L])
    args = _lib.InitArgs()
    args.n_replicas = n_rep
    args.species = sp_arr
    args.N = N_arr
    args.L = L_arr
    args.precision = _lib.PRECISIONS[precision]
    args.path = _lib.PATHS[path]
    args.pos = pos.data_ptr()
    args.orient = orient.data_ptr() if orient is not None else None
    args.stream = stream.cuda_stream
    args.flags = flags
    keep += [sp_arr, N_arr, L_arr]
    if L_max is not None:
        Lmax_arr = (ctypes.c_double * n_rep)(*[float(x) for x in L_max])
        args.L_max = Lmax_arr
        keep.append(Lmax_arr)
    return args, keep


def sweep_static(species, N, L, pos, orient, t0, n_sweeps, seed, precision="fp64", path="auto",
                 stream=None):
    """n_sweeps sweeps from sweep counter t0 through hpmc_sweep_static, the
    entry point that allocates no device memory: pos / orient are the
    caller's device tensors (float64, replicas concatenated, hpmc.h layout),
    updated in place.  Returns the per-replica counters of these sweeps."""
    import torch
    lib = _lib.load()
    n_rep = len(species)
    if stream is None:
        stream = torch.cuda.current_stream(pos.device)
    args, keep = init_args(species, N, L, pos, orient, precision, path, stream)
    out = (_lib.Stats * n_rep)()
    hip = ctypes.c_int32()
    rc = lib.hpmc_sweep_static(ctypes.byref(args), int(t0), int(n_sweeps), int(seed), out,
                               ctypes.byref(hip))
    del keep
    if rc != _lib.HPMC_OK:
        raise _lib.HpmcError(rc, "hpmc_sweep_static", hip.value)
    return [{f: int(getattr(out[r], f)) for f in _lib.STAT_FIELDS} for r in range(n_rep)]


def phase_trace(reset=False):
    """Per-wave phase clock of the trace build (HPMC_LIBRARY pointing at
    lib/libhpmc_trace.so): {kernel: {"waves": n, phase: cycles summed over
    waves}} since the last reset; synchronises the device."""
    lib = _lib.load()
    n = len(_lib.TRACED_KERNELS) * (len(_lib.PHASES) + 1)
    out = (ctypes.c_uint64 * n)()
    rc = lib.hpmc_phase_trace(out, n, 1 if reset else 0)
    if rc != _lib.HPMC_OK:
        raise _lib.HpmcError(rc, "hpmc_phase_trace")
    res, k = {}, 0
    for name in _lib.TRACED_KERNELS:
        d = {ph: int(out[k + j]) for j, ph in enumerate(_lib.PHASES)}
        d["waves"] = int(out[k + len(_lib.PHASES)])
        res[name] = d
        k += len(_lib.PHASES) + 1
    return res


class System:
    def __init__(self, species, N, L, pos, orient=None, precision="fp64", path="auto",
                 device="cuda", stream=None, graphs=True, queue="wave", L_max=None):
        import torch

        self._torch = torch
        self._lib = _lib.load()
        if isinstance(pos, (list, tuple)):
            n_rep = len(pos)
        else:
            n_rep = 1
            pos = [pos]
            orient = [orient]
        if orient is None:
            orient = [None] * n_rep
        self.n_replicas = n_rep
        self.species = _as_list(species, n_rep)
        self.N = [int(x) for x in _as_list(N, n_rep)]
        self.L = [float(x) for x in _as_list(L, n_rep)]
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("System needs a GPU device")

        pos_parts, ori_parts = [], []
        self._pos_off, self._ori_off = [], []
        po = oo = 0
        for r in range(n_rep):
            sp, Nr = self.species[r], self.N[r]
            p = np.ascontiguousarray(np.asarray(pos[r], dtype=np.float64))
            if p.shape != (sp["dim"], Nr):
                raise ValueError(f"replica {r}: pos must have shape (dim, N)")
            pos_parts.append(p.ravel())
            self._pos_off.append(po)
            po += p.size
            k = _NCOMP[sp["shape"]]
            self._ori_off.append(oo)
            if k:
                o = np.ascontiguousarray(np.asarray(orient[r], dtype=np.float64))
                if o.shape != (k, Nr):
                    raise ValueError(f"replica {r}: orient must have shape ({k}, N)")
                ori_parts.append(o.ravel())
                oo += o.size
        self.pos = torch.from_numpy(np.concatenate(pos_parts)).to(self.device)
        ori = np.concatenate(ori_parts) if ori_parts else np.zeros(1)
        self.orient = torch.from_numpy(ori).to(self.device)

        self.L_max = ([float(x) for x in _as_list(L_max, n_rep)] if L_max is not None
                      else list(self.L))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        if queue not in _lib.QUEUE_FLAGS:
            raise ValueError(f"queue must be one of {sorted(_lib.QUEUE_FLAGS)}")
        flags = (0 if graphs else _lib.FLAG_NO_GRAPH) | _lib.QUEUE_FLAGS[queue]
        args, self._keep = init_args(self.species, self.N, self.L, self.pos, self.orient, precision,
                                     path, stream, flags, self.L_max)
        nbytes = ctypes.c_size_t()
        self._check(self._lib.hpmc_workspace_bytes(ctypes.byref(args), ctypes.byref(nbytes)),
                    "hpmc_workspace_bytes")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        args.workspace = (base + 255) // 256 * 256
        args.workspace_bytes = nbytes.value
        self._args = args
        handle = ctypes.c_void_p()
        self._handle = None
        self._check(self._lib.hpmc_init(ctypes.byref(handle), ctypes.byref(args)), "hpmc_init")
        self._handle = handle
        self.precision = precision

    # -- calls -------------------------------------------------------------
    def _check(self, rc, what):
        if rc != _lib.HPMC_OK:
            # a failed hpmc_init leaves no state: NULL asks for its HIP error
            hip = self._lib.hpmc_last_hip_error(getattr(self, "_handle", None))
            raise _lib.HpmcError(rc, what, hip)

    def sweep(self, n_sweeps, seed):
        self._check(self._lib.hpmc_sweep(self._handle, int(n_sweeps), int(seed)), "hpmc_sweep")

    def autotune(self, trial_sweeps=8):
        """Time the launch configurations, keep the fastest; the state is
        restored exactly.  Returns the chosen lanes per cell (grid path) or
        LDS residency level (persistent path) in the low byte, plus 0x100
        when mixed-precision polyhedra walk in binary64."""
        cfg = ctypes.c_int32()
        self._check(self._lib.hpmc_autotune(self._handle, int(trial_sweeps), ctypes.byref(cfg)),
                    "hpmc_autotune")
        return cfg.value

    def set_config(self, config):
        """Apply a configuration in the encoding autotune() returns."""
        self._check(self._lib.hpmc_set_config(self._handle, int(config)), "hpmc_set_config")

    @property
    def uses_graph(self):
        return bool(self._lib.hpmc_uses_graph(self._handle))

    @property
    def graph_sweeps(self):
        """Sweeps run by replaying the captured hipGraph since init."""
        n = ctypes.c_uint64()
        self._check(self._lib.hpmc_graph_sweeps(self._handle, ctypes.byref(n)), "hpmc_graph_sweeps")
        return n.value

    def count_overlaps(self):
        out = (ctypes.c_uint64 * self.n_replicas)()
        self._check(self._lib.hpmc_count_overlaps(self._handle, out), "hpmc_count_overlaps")
        return np.array(out[:], dtype=np.uint64)

    def pair_histogram(self, edges2, r=0):
        """Counts of unordered pairs of replica r with edges2[b] <= |r|^2 <
        edges2[b+1] (minimum image); edges2 ascending squared distances."""
        e = np.ascontiguousarray(np.asarray(edges2, dtype=np.float64))
        out = (ctypes.c_uint64 * (len(e) - 1))()
        self._check(self._lib.hpmc_pair_histogram(self._handle, int(r),
                                                  e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                  len(e) - 1, out), "hpmc_pair_histogram")
        return np.array(out[:], dtype=np.uint64)

    def scale_counts(self, scales, r=0):
        """Pairs of replica r that overlap once every separation is scaled by
        1 - scales[b] (volume perturbation); scales ascending in [0, 1)."""
        sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64))
        out = (ctypes.c_uint64 * len(sc))()
        self._check(self._lib.hpmc_scale_counts(self._handle, int(r),
                                                sc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                len(sc), out), "hpmc_scale_counts")
        return np.array(out[:], dtype=np.uint64)

    def scale_box(self, r, L_new):
        """Scale replica r's box (and positions) to side L_new; returns the
        number of overlapping pairs after scaling.  restore_box(r) undoes it."""
        out = ctypes.c_uint64()
        self._check(self._lib.hpmc_scale_box(self._handle, int(r), float(L_new), ctypes.byref(out)),
                    "hpmc_scale_box")
        self._L_prev = getattr(self, "_L_prev", {})
        self._L_prev[r] = self.L[r]
        self.L[r] = float(L_new)
        return int(out.value)

    def restore_box(self, r):
        self._check(self._lib.hpmc_restore_box(self._handle, int(r)), "hpmc_restore_box")
        self.L[r] = self._L_prev.pop(r)

    def volume_move(self, r, u1, u2, beta_p, delta_v):
        """One isobaric volume move of replica r with the uniforms (u1, u2);
        returns True when accepted (the library decides and applies it)."""
        acc, L_after = ctypes.c_int32(), ctypes.c_double()
        self._check(self._lib.hpmc_volume_move(self._handle, int(r), float(u1), float(u2),
                                               float(beta_p), float(delta_v), ctypes.byref(acc),
                                               ctypes.byref(L_after)), "hpmc_volume_move")
        if acc.value:
            self._L_prev = getattr(self, "_L_prev", {})
            self._L_prev[r] = self.L[r]
        self.L[r] = L_after.value
        return bool(acc.value)

    def stats(self):
        out = (_lib.Stats * self.n_replicas)()
        self._check(self._lib.hpmc_get_stats(self._handle, out), "hpmc_get_stats")
        return [{f: int(getattr(out[r], f)) for f in _lib.STAT_FIELDS}
                for r in range(self.n_replicas)]

    def reset_stats(self):
        self._check(self._lib.hpmc_reset_stats(self._handle), "hpmc_reset_stats")

    @property
    def sweep_counter(self):
        t = ctypes.c_uint64()
        self._check(self._lib.hpmc_get_sweep(self._handle, ctypes.byref(t)), "hpmc_get_sweep")
        return t.value

    @sweep_counter.setter
    def sweep_counter(self, t):
        self._check(self._lib.hpmc_set_sweep(self._handle, int(t)), "hpmc_set_sweep")

    def replica_info(self, r=0):
        n, rounds, path = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.hpmc_replica_info(self._handle, r, ctypes.byref(n), ctypes.byref(rounds),
                                                ctypes.byref(path)), "hpmc_replica_info")
        return {"n": n.value, "rounds": rounds.value,
                "path": {v: k for k, v in _lib.PATHS.items()}[path.value]}

    def synchronize(self):
        self._check(self._lib.hpmc_sync_to_canonical(self._handle), "hpmc_sync_to_canonical")

    def positions(self, r=0):
        """(dim, N) float64 numpy copy of replica r."""
        self.synchronize()
        sp, Nr = self.species[r], self.N[r]
        o = self._pos_off[r]
        return self.pos[o:o + sp["dim"] * Nr].view(sp["dim"], Nr).cpu().numpy()

    def orientations(self, r=0):
        self.synchronize()
        sp, Nr = self.species[r], self.N[r]
        k = _NCOMP[sp["shape"]]
        if k == 0:
            return None
        o = self._ori_off[r]
        return self.orient[o:o + k * Nr].view(k, Nr).cpu().numpy()

    def close(self):
        if getattr(self, "_handle", None):
            self._lib.hpmc_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

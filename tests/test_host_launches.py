"""The library's host logic without a GPU: hpmc_init, hpmc_sweep,
hpmc_autotune, hpmc_count_overlaps and hpmc_volume_move run against a
host-only stand-in of the HIP runtime (tests/hip_runtime_stub.cpp, loaded
first in a fresh process) that checks every kernel launch and copy instead of
executing it.  Every pointer a kernel receives and every device side of a
copy must lie inside the caller's positions, orientations or workspace, and
every launch must have a non-empty grid -- so a host-side mistake that hands
a kernel a null or stray pointer fails here, on the CPU, before any GPU run."""
import os
import subprocess
import sys
import textwrap

import pytest

from paper_1509_04692_amd.build import LIB_PATH

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

DRIVER = textwrap.dedent(r"""
    import ctypes, sys
    import numpy as np
    stub = ctypes.CDLL(sys.argv[1], mode=ctypes.RTLD_GLOBAL)
    sys.path.insert(0, sys.argv[3])
    from paper_1509_04692_amd import _lib, inputs
    lib = _lib.load(sys.argv[2])
    lib.hpmc_destroy.argtypes = [ctypes.c_void_p]
    stub.stub_open_log(sys.argv[4].encode())
    def run(items, precision, path, flags=0):
        n = len(items)
        sp_arr = (_lib.Species * n)()
        keep = []
        for r, (sp, N, L, pos, ori) in enumerate(items):
            s = sp_arr[r]
            s.dim, s.shape = sp["dim"], _lib.SHAPES[sp["shape"]]
            if sp["shape"] != "disk":
                v = np.ascontiguousarray(sp["verts"], dtype=np.float64)
                keep.append(v)
                s.n_verts, s.verts = v.shape[0], v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            s.diameter = sp.get("diameter", 0.0)
            s.d, s.a, s.p_rot = sp["d"], sp["a"], sp["p_rot"]
            s.sweep_radius = sp.get("sweep_radius", 0.0)
        a = _lib.InitArgs()
        a.n_replicas, a.species = n, sp_arr
        a.N = (ctypes.c_int32 * n)(*[i[1] for i in items])
        a.L = (ctypes.c_double * n)(*[i[2] for i in items])
        a.L_max = (ctypes.c_double * n)(*[1.1 * i[2] for i in items])
        a.precision, a.path, a.flags = precision, path, flags
        nb = ctypes.c_size_t()
        assert lib.hpmc_workspace_bytes(ctypes.byref(a), ctypes.byref(nb)) == 0
        pos = np.concatenate([i[3].ravel() for i in items])
        ori = np.concatenate([i[4].ravel() for i in items if i[0]["shape"] != "disk"] or [np.zeros(1)])
        ws = np.zeros(nb.value // 8 + 64)
        base = (ws.ctypes.data + 255) // 256 * 256
        for buf in (pos, ori):
            stub.stub_add_region(ctypes.c_uint64(buf.ctypes.data), ctypes.c_uint64(buf.nbytes))
        stub.stub_add_region(ctypes.c_uint64(base), ctypes.c_uint64(nb.value))
        a.pos, a.orient, a.workspace, a.workspace_bytes = pos.ctypes.data, ori.ctypes.data, base, nb.value
        h = ctypes.c_void_p()
        assert lib.hpmc_init(ctypes.byref(h), ctypes.byref(a)) == 0
        assert lib.hpmc_sweep(h, 70, 1) == 0            # a whole persistent chunk and a remainder
        cfg = ctypes.c_int32()
        assert lib.hpmc_autotune(h, 1, ctypes.byref(cfg)) == 0
        out = (ctypes.c_uint64 * n)()
        assert lib.hpmc_count_overlaps(h, out) == 0
        acc, L2 = ctypes.c_int32(), ctypes.c_double()
        assert lib.hpmc_volume_move(h, 0, 0.9, 0.5, 1.0, 0.01 * items[0][2] ** items[0][0]["dim"],
                                    ctypes.byref(acc), ctypes.byref(L2)) == 0
        assert lib.hpmc_sweep(h, 2, 1) == 0
        lib.hpmc_destroy(h)
    run([inputs.workload_disks_256()], 0, 1)
    run([inputs.workload_pentagons(700, 0.6), inputs.workload_pentagons(400, 0.6),
         inputs.workload_disks_256(), inputs.workload_cubes(512, 0.45)], 1, 2)
    run([inputs.workload_pentagons(2048, 0.6)], 1, 1)
    run([inputs.workload_cubes(1000, 0.45)], 1, 1)
    run([inputs.workload_pentagons(1024, 0.6)], 0, 1, _lib.QUEUE_FLAGS["global"])
    run([inputs.workload_pentagons(1024, 0.6)], 0, 1, _lib.QUEUE_FLAGS["register"])
    run([inputs.workload_pentagons(20000, 0.6)], 1, 1)   # multi-kernel cell-list build
    run([inputs.workload_pentagons(4096, 0.6)] * 2, 1, 2)  # the headline replica: LDS near the limit
    run([inputs.workload_pentagons(4096, 0.6)] * 2, 0, 2)
    run(inputs.screening_batch(6, seed=2026, n_lo=3000, n_hi=4096), 1, 2)
    # spheropolygons: grid path (every lanes-per-cell candidate) and a batch
    # mixing them with plain polygons, stadiums and disks
    run([inputs.workload_rounded_pentagons(1500, 0.5)], 1, 1)
    run([inputs.workload_rounded_pentagons(900, 0.5), inputs.workload_stadiums(500, 0.25),
         inputs.workload_pentagons(600, 0.6), inputs.workload_disks_256()], 1, 2)
    # the scratch-free entry point: its workspace is the library's static array
    def run_static(items, precision, path):
        n = len(items)
        sp_arr = (_lib.Species * n)()
        keep = []
        for r, (sp, N, L, pos, ori) in enumerate(items):
            s = sp_arr[r]
            s.dim, s.shape = sp["dim"], _lib.SHAPES[sp["shape"]]
            if sp["shape"] != "disk":
                v = np.ascontiguousarray(sp["verts"], dtype=np.float64)
                keep.append(v)
                s.n_verts, s.verts = v.shape[0], v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            s.diameter = sp.get("diameter", 0.0)
            s.d, s.a, s.p_rot = sp["d"], sp["a"], sp["p_rot"]
        a = _lib.InitArgs()
        a.n_replicas, a.species = n, sp_arr
        a.N = (ctypes.c_int32 * n)(*[i[1] for i in items])
        a.L = (ctypes.c_double * n)(*[i[2] for i in items])
        a.precision, a.path = precision, path
        pos = np.concatenate([i[3].ravel() for i in items])
        ori = np.concatenate([i[4].ravel() for i in items if i[0]["shape"] != "disk"] or [np.zeros(1)])
        for buf in (pos, ori):
            stub.stub_add_region(ctypes.c_uint64(buf.ctypes.data), ctypes.c_uint64(buf.nbytes))
        a.pos, a.orient = pos.ctypes.data, ori.ctypes.data
        st = (_lib.Stats * n)()
        hip = ctypes.c_int32()
        assert lib.hpmc_sweep_static(ctypes.byref(a), 3, 70, 1, st, ctypes.byref(hip)) == 0
    run_static([inputs.workload_pentagons(700, 0.6), inputs.workload_disks_256()], 1, 2)
    run_static([inputs.workload_disks_256()], 0, 1)
    print("launches", stub.stub_launches(), "violations", stub.stub_violations())
""")


@pytest.fixture(scope="module")
def stub(tmp_path_factory):
    so = tmp_path_factory.mktemp("stub") / "libhip_runtime_stub.so"
    subprocess.run(["g++", "-O1", "-shared", "-fPIC", "-o", str(so), os.path.join(HERE, "hip_runtime_stub.cpp"),
                    f"-Wl,--version-script={os.path.join(HERE, 'hip_runtime_stub.map')}"],
                   check=True, capture_output=True)
    return str(so)


def test_every_launch_gets_valid_buffers(stub, tmp_path):
    if not os.path.exists(LIB_PATH):
        pytest.fail("libhpmc.so is not built (run python -m paper_1509_04692_amd.build)")
    log = tmp_path / "launches.log"
    res = subprocess.run([sys.executable, "-c", DRIVER, stub, LIB_PATH, ROOT, str(log)],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-3000:]
    last = res.stdout.strip().splitlines()[-1].split()
    launches, violations = int(last[1]), int(last[3])
    bad = [ln for ln in log.read_text().splitlines() if ln.startswith("VIOLATION")][:10]
    assert violations == 0, bad
    assert launches > 1000

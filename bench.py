#!/usr/bin/env python3
"""Trial moves per second of the checkerboard hard-shape sweep on one MI355X.

Default workload (the headline metric): 512 independent replicas of 4096
regular pentagons (circumradius 0.5, packing fraction 0.60, d = 0.1,
a = 0.2, p_rot = 0.5) in one persistent launch with the certified
mixed-precision overlap test, against the plain FP64 single-system path on
the same GPU.  One step is one sweep (N trial moves per replica) of every
replica.  Inputs are resident on the GPU before the timed region; trial
moves are counted on the device (attempted moves, cell rejects included).

Prints one JSON line.  Extra fields: the other three precision x batching
combinations, the re-checked pair fraction, the overlap count of the state
each timed run left, the sweeps that replayed the captured graph, a roofline
object for the timed kernel and the reference oracle timed on the host.  Each
configuration is timed --repeats times (default 5) over --steps sweeps;
`value` is the first of these runs and every run's rate is listed beside the
median.
"""
import argparse
import json
import math
import os
import platform
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X's published dense FP64 vector peak (an FMA counts as two flops).
FP64_PEAK_TFLOPS = 78.6
# One VALU operation per lane per clock: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
# (non-packed fp32 and fp64 issue at this rate): half the published figure,
# the ceiling for code whose operations are not FMAs.  Reported beside it.
VALU_ISSUE_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0
PERSISTENT_SWEEPS_PER_LAUNCH = 64  # HPMC_PERSISTENT_SWEEPS_PER_LAUNCH


def op_costs(nv):
    """Operations (+ - * / sqrt rint min max compare) of each counted event,
    from the pinned formulas of the sweep; nv = vertices of the shape."""
    return {
        "translate": 12,            # per axis; multiplied by dim below
        "rotate2": 43,              # angle 5 + sin/cos polynomial 32 + complex product 6
        "rotate3": 55,              # vector 15 + quaternion product 28 + norm 8 + 4 divisions
        "cand2": 14,                # 2 x min-image (5) + |r|^2 (3) + compare
        "cand3": 21,                # 3 x min-image (5) + |r|^2 (5) + compare
        "sat_setup": 12 + 8 * nv,   # relative rotation 6 + offset 6 + nv vertex maps
        "sat_axis": 5 * nv,         # nv projections (3) + min/max (2 (nv-1)) + 2 compares
        "sat_frame_b": 8 * nv,      # nv vertex maps into B's frame
        "mpr_setup": 169,           # relative rotation, two matrices, offset, first portal
        "mpr_support": 34 + 12 * nv,
        "mpr_iter": 55,
        "seg_setup": 15 + 8 * nv,   # relative rotation 6 + offset 6 + (s + s)^2 3 + nv vertex maps
        "seg_test": 16,             # one point-segment distance test (largest branch)
    }


def ops_per_move(events, attempted, dim, nv):
    c = op_costs(nv)
    total = 0
    for k, v in events.items():
        total += v * c[k] * (dim if k == "translate" else 1)
    return total / max(attempted, 1)


def workload(name):
    from paper_1509_04692_amd import inputs
    if name == "pentagons":
        sp, N, L, pos, ori = inputs.workload_pentagons(4096, 0.60)
        return {"desc": "regular pentagons N=4096 R=0.5 phi=0.60 d=0.1 a=0.2 p_rot=0.5",
                "items": [(sp, N, L, pos, ori)], "replicas": 512}
    if name == "pentagons676":
        sp, N, L, pos, ori = inputs.workload_pentagons(4096, 0.676)
        return {"desc": "regular pentagons N=4096 R=0.5 phi=0.676 d=0.1 a=0.2 p_rot=0.5",
                "items": [(sp, N, L, pos, ori)], "replicas": 512}
    if name == "disks":
        sp, N, L, pos, ori = inputs.workload_disks_256()
        return {"desc": "hard disks N=256 sigma=1 phi=0.50 d=0.1",
                "items": [(sp, N, L, pos, ori)], "replicas": 512}
    if name == "cubes":
        sp, N, L, pos, ori = inputs.workload_cubes(32768, 0.45)
        return {"desc": "cubes N=32768 edge 1 phi=0.45 d=0.08 a=0.1 p_rot=0.5",
                "items": [(sp, N, L, pos, ori)], "replicas": 1}
    if name == "trunc_oct":
        sp, N, L, pos, ori = inputs.workload_truncated_octahedra(32768, 0.45)
        return {"desc": "truncated octahedra N=32768 edge 1 phi=0.45 d=0.08 a=0.1 p_rot=0.5",
                "items": [(sp, N, L, pos, ori)], "replicas": 1}
    if name == "dodecahedra":
        sp, N, L, pos, ori = inputs.workload_dodecahedra(4096, 0.50)
        return {"desc": "regular dodecahedra N=4096 edge 1 phi=0.50 d=0.08 a=0.1 p_rot=0.5",
                "items": [(sp, N, L, pos, ori)], "replicas": 256}
    if name == "spherocylinders":
        sp, N, L, pos, ori = inputs.workload_spherocylinders(4096, 0.15)
        return {"desc": "spherocylinders N=4096 length 1 radius 0.5 phi=0.15 d=0.08 a=0.1 p_rot=0.5",
                "items": [(sp, N, L, pos, ori)], "replicas": 256}
    if name == "spheres":
        sp, N, L, pos, ori = inputs.workload_spheres(4096, 0.40)
        return {"desc": "spheres (one-vertex spheropolyhedra) N=4096 sigma=1 phi=0.40 d=0.1",
                "items": [(sp, N, L, pos, ori)], "replicas": 256}
    if name == "rounded_pentagons":
        sp, N, L, pos, ori = inputs.workload_rounded_pentagons(4096, 0.50)
        return {"desc": "spheropolygons: regular pentagons of core circumradius 0.4 swept by 0.1, "
                        "N=4096 phi=0.50 d=0.1 a=0.2 p_rot=0.5",
                "items": [(sp, N, L, pos, ori)], "replicas": 512}
    if name == "large":
        sp, N, L, pos, ori = inputs.workload_pentagons(4194304, 0.60)
        return {"desc": "regular pentagons N=4194304 R=0.5 phi=0.60 d=0.1 a=0.2 p_rot=0.5",
                "items": [(sp, N, L, pos, ori)], "replicas": 1}
    if name == "screening":
        batch = inputs.screening_batch(512, seed=2026)
        return {"desc": "512 replicas: even disks / odd pentagons, N ~ U[64,4096], "
                        "phi ~ U[0.30,0.70] (PCG64 seed 2026)",
                "items": batch, "replicas": None}
    raise SystemExit(f"unknown workload {name}")


def make_system(wl, precision, path, batched, queue="wave"):
    from paper_1509_04692_amd.system import System
    items = wl["items"]
    if wl["replicas"] is None:  # heterogeneous batch
        chosen = items if batched else items[:1]
    else:
        chosen = items * (wl["replicas"] if batched else 1)
    return System([c[0] for c in chosen], [c[1] for c in chosen], [c[2] for c in chosen],
                  [c[3] for c in chosen], [c[4] for c in chosen], precision=precision, path=path,
                  queue=queue)


def decode_config(cfg, path):
    """The fields of an hpmc_autotune configuration (include/hpmc.h)."""
    if cfg is None:
        return None
    return {("lds_residency" if path == "persistent" else "lanes_per_cell"): cfg & 0xff,
            "binary64_walk": bool(cfg & 0x100),
            "drain_at": (64, 32, 16, None)[(cfg >> 9) & 3],
            "work_group_size": ("default", "half", "quarter", None)[(cfg >> 11) & 3]}


def timed_run(system, steps, warmup, seed):
    """Warm up, then time exactly `steps` sweeps with HIP events on the
    library's stream, synchronised on both sides.  Returns the time, the
    counter differences and the sweeps of the timed call that replayed the
    captured graph."""
    import torch
    system.sweep(warmup, seed)
    torch.cuda.synchronize()
    before = system.stats()
    g0 = system.graph_sweeps
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(system.stream):
        start.record(system.stream)
        system.sweep(steps, seed)
        end.record(system.stream)
    torch.cuda.synchronize()
    after = system.stats()
    ms = start.elapsed_time(end)
    diff = {k: sum(a[k] - b[k] for a, b in zip(after, before)) for k in after[0] if k != "sweeps"}
    diff["graph_sweeps"] = system.graph_sweeps - g0
    return ms, diff


def cpu_baseline(wl, warmup, steps, budget_s=12.0):
    """The FP64 reference oracle on one host core, timed on replica 0 of the
    workload from its initial state, plus an event-counting run over the same
    sweeps the GPU timed (for the work-per-move figure)."""
    import oracle
    sp, N, L, pos, ori = wl["items"][0]
    p, o = pos.copy(), ori.copy()
    moves = 0
    t_sweep = 0
    t0 = time.perf_counter()
    chunk = max(1, int(2e5 // N))
    while time.perf_counter() - t0 < budget_s:
        st = oracle.sweep(sp, L, p, o, seed=1, n_sweeps=chunk, t0=t_sweep)
        moves += int(st[0])
        t_sweep += chunk
    dt = time.perf_counter() - t0
    # the separate serial one-move-at-a-time Metropolis reference, timed alongside
    p, o = pos.copy(), ori.copy()
    s_moves, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < budget_s / 4:
        oracle.serial_metropolis(sp, L, p, o, seed=1, n_moves=20000, move0=s_moves)
        s_moves += 20000
    s_dt = time.perf_counter() - t1
    lib = oracle.load_counting()
    p, o = pos.copy(), ori.copy()
    oracle.sweep(sp, L, p, o, seed=1, n_sweeps=warmup, lib=lib)
    oracle.reset_events(lib)
    n_count = min(steps, max(1, int(2e6 // N)))
    st = oracle.sweep(sp, L, p, o, seed=1, n_sweeps=n_count, t0=warmup, lib=lib)
    ev = oracle.event_counts(lib)
    nv = len(sp["verts"]) if "verts" in sp else 0
    opm = ops_per_move(ev, int(st[0]), sp["dim"], nv)
    cpu = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        cpu = next((l.split(":", 1)[1].strip() for l in out.splitlines() if "Model name" in l), cpu)
    except OSError:
        pass
    # all host cores: one oracle process per core, each on its own replica
    # word, started as fresh interpreters (no GPU state is inherited)
    n_proc = max(1, min(16, os.cpu_count() or 1))
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                               wl["name"], str(r), str(budget_s * 0.75)],
                              stdout=subprocess.PIPE, text=True) for r in range(n_proc)]
    all_moves, all_dt = 0, 0.0
    for pr in procs:
        out, _ = pr.communicate()
        res = json.loads(out.strip().splitlines()[-1])
        all_moves += res["moves"]
        all_dt = max(all_dt, res["seconds"])
    return {
        "value": moves / dt, "unit": "trial moves/s", "cores": 1, "kind": "oracle",
        "sample": f"replica 0 ({N} particles), sweeps 0..{t_sweep} from the initial state, "
                  f"{dt:.1f} s on one core of {cpu} (nproc {os.cpu_count()})",
        "all_cores": {"value": all_moves / all_dt, "cores": n_proc,
                      "sample": f"{n_proc} oracle processes, one replica word each, "
                                f"{all_dt:.1f} s"},
        "serial_metropolis": {"value": s_moves / s_dt, "cores": 1,
                              "sample": f"{s_moves} one-at-a-time moves of replica 0 from the "
                                        f"initial state, {s_dt:.1f} s"},
    }, opm, {k: v / max(int(st[0]), 1) for k, v in ev.items()}, n_count


def oracle_worker(name, replica, budget_s):
    """One oracle process of the all-cores leg: sweeps of the workload's first
    system with its own replica word for about budget_s seconds."""
    import oracle
    wl = workload(name)
    sp, N, L, pos, ori = wl["items"][0]
    p, o = pos.copy(), ori.copy()
    moves, t_sweep = 0, 0
    chunk = max(1, int(2e5 // N))
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        st = oracle.sweep(sp, L, p, o, seed=1, n_sweeps=chunk, t0=t_sweep, replica=replica)
        moves += int(st[0])
        t_sweep += chunk
    print(json.dumps({"moves": moves, "seconds": time.perf_counter() - t0}))


def _csrc_hash():
    """Hash of the device sources (every file of csrc/ but the host-side
    api.hip) with comments and blank lines removed, so that a recorded
    measurement stays valid across comment-only and host-only edits."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1509_04692_amd", "csrc", "*"))):
        if os.path.basename(f) == "api.hip":
            continue
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()


def recorded_counters():
    """The rocprofv3 counters recorded under profiles/ for the headline kernel
    (FETCH_SIZE / WRITE_SIZE over one launch of `launch_sweeps` sweeps, each
    scaled by the same counter's reading for a plain copy of known size;
    VALUBusy, VALUUtilization, waves per SIMD), or None when the kernel
    sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_k_batch_pentagons.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("csrc_sha256") != _csrc_hash():
        return None
    d["bytes_per_sweep"] = ((d["fetch_kib"] * d["fetch_factor"] + d["write_kib"] * d["write_factor"])
                            * 1024.0 / d["launch_sweeps"])
    return d


def _device_info():
    import torch
    p = torch.cuda.get_device_properties(0)
    keys = ("name", "gcnArchName", "multi_processor_count", "shared_memory_per_block",
            "shared_memory_per_block_optin", "shared_memory_per_multiprocessor", "L2_cache_size")
    return {k: getattr(p, k) for k in keys if hasattr(p, k)}


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--oracle-worker":
        oracle_worker(sys.argv[2], int(sys.argv[3]), float(sys.argv[4]))
        return 0
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1024, help="timed sweeps (64 per persistent launch, a remainder as one shorter launch)")
    ap.add_argument("--warmup", type=int, default=128, help="untimed sweeps first")
    ap.add_argument("--workload", default="pentagons",
                    choices=["pentagons", "pentagons676", "disks", "cubes", "trunc_oct", "dodecahedra",
                             "spheres", "spherocylinders", "rounded_pentagons", "large", "screening"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--queue", default="wave", choices=["wave", "register", "global"],
                    help="schedule of the full overlap tests (register/global: grid path, "
                         "single-system runs only; for comparison with the default)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of --steps sweeps per configuration (median reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--config", type=lambda x: int(x, 0), default=None,
                    help="apply this launch configuration (hpmc_set_config encoding) instead of autotuning")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized buffer once (calibrates HBM byte counters)")
    ap.add_argument("--phase-trace", action="store_true",
                    help="with HPMC_LIBRARY=<lib/libhpmc_trace.so>: report where each kernel's "
                         "waves spend their cycles over the timed runs (the clock reads slow the "
                         "kernels: not a timing run)")
    ap.add_argument("--only", default=None,
                    help="comma list of runs: mixed_batched,fp64_single,fp64_batched,mixed_single")
    args = ap.parse_args()
    if args.repeats < 1:
        ap.error("--repeats must be at least 1")
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(replicas shard across GPUs without communication; see the design notes).",
              file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        a = torch.arange(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "ok": bool(b[-1].item() == n - 1)}))
        return 0
    wl = workload(args.workload)
    wl["name"] = args.workload
    batched_ok = wl["replicas"] is None or wl["replicas"] > 1
    runs = ["mixed_batched", "fp64_single", "fp64_batched", "mixed_single"]
    if not batched_ok:
        runs = ["mixed_single", "fp64_single"]
    if args.queue != "wave":
        runs = ["mixed_single", "fp64_single"]
    if args.only:
        runs = [r for r in args.only.split(",") if r]
    results = {}
    for name in runs:
        precision, mode = name.split("_")
        batched = mode == "batched"
        path = "persistent" if batched else "grid"
        system = make_system(wl, precision, path, batched, args.queue)
        if args.config is not None:
            system.set_config(args.config)
            tuned = args.config
        else:
            tuned = system.autotune(trial_sweeps=8) if not args.no_autotune else None
        if args.phase_trace:
            from paper_1509_04692_amd.system import phase_trace
            system.sweep(args.warmup, args.seed)
            phase_trace(reset=True)
        ms, diff = timed_run(system, args.steps, 0 if args.phase_trace else args.warmup, args.seed)
        # further timed runs of the same length continue the chain; the line's
        # value stays the first one, the median of all is reported beside it
        rep = [diff["attempted"] / (ms * 1e-3)]
        for _ in range(args.repeats - 1):
            ms_k, diff_k = timed_run(system, args.steps, 0, args.seed)
            rep.append(diff_k["attempted"] / (ms_k * 1e-3))
        trace = None
        if args.phase_trace:
            trace = {}
            for kern, d in phase_trace(reset=True).items():
                total = sum(v for k, v in d.items() if k != "waves")
                if d["waves"]:
                    trace[kern] = {"waves": d["waves"], "cycles_per_wave": total / d["waves"],
                                   "fractions": {k: v / total for k, v in d.items() if k != "waves"}}
        # the state the timed sweeps left, checked outside the timed region
        overlaps = int(system.count_overlaps().sum())
        if overlaps:
            print(f"# {name}: {overlaps} overlapping pairs after the timed sweeps", file=sys.stderr)
        n_launch = (math.ceil(args.steps / PERSISTENT_SWEEPS_PER_LAUNCH) if path == "persistent"
                    else None)
        results[name] = {
            "value": diff["attempted"] / (ms * 1e-3),
            "ms_per_step": ms / args.steps,
            "replicas": system.n_replicas,
            "path": path,
            "acceptance": diff["accept"] / max(diff["attempted"], 1),
            "recheck_fraction": (diff["pair_fp64"] / diff["pair_tests"]
                                 if precision == "mixed" and diff["pair_tests"] else None),
            "moves": diff["attempted"],
            "pair_tests_per_move": diff["pair_tests"] / max(diff["attempted"], 1),
            "launches": n_launch,
            "autotuned": tuned,
            "tuned_config": decode_config(tuned, path),
            "graph": system.uses_graph,
            "graph_replayed_sweeps": diff["graph_sweeps"],
            "phase_trace": trace,
            "overlaps_after": overlaps,
            "ms_total": ms,
            "repeats": rep,
            "median_of_repeats": statistics.median(rep),
        }
        del system
        torch.cuda.synchronize()
        print(f"# {name}: {results[name]['value']:.4e} trial moves/s, "
              f"{results[name]['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)

    head = "mixed_batched" if "mixed_batched" in results else runs[0]
    h = results[head]
    cpu, opm, ev_per_move, n_count = (None, None, None, 0)
    if not args.no_cpu_baseline:
        cpu, opm, ev_per_move, n_count = cpu_baseline(wl, args.warmup, args.steps)
    roofline = None
    if opm is not None:
        if h["launches"]:
            launch_s = h["ms_total"] * 1e-3 / h["launches"]
            ops_per_launch = opm * h["moves"] / h["launches"]
        else:
            launch_s = h["ms_total"] * 1e-3
            ops_per_launch = opm * h["moves"]
        achieved = ops_per_launch / launch_s / 1e12
        traffic, rec = None, None
        if head == "mixed_batched" and args.workload == "pentagons" and h["launches"]:
            rec = recorded_counters()
        hbm = None
        if rec is not None:
            # counters of a recorded launch, per sweep, times the sweeps of an
            # average timed launch
            traffic = rec["bytes_per_sweep"] * args.steps / h["launches"]
            gbps = traffic / launch_s / 1e9
            hbm = {"achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                   "bytes_per_sweep": rec["bytes_per_sweep"],
                   "recorded_launch_sweeps": rec["launch_sweeps"]}
        roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                    "traffic_unit": "HBM bytes per launch (recorded per-sweep counters x sweeps per launch)",
                    "issue_rate": {"peak": VALU_ISSUE_TOPS, "unit": "T VALU op/s (one per lane per clock)",
                                   "frac": achieved / VALU_ISSUE_TOPS},
                    "hbm": hbm,
                    "valu_busy": rec.get("valu_busy") if rec else None,
                    "valu_utilization": rec.get("valu_utilization") if rec else None,
                    "waves_per_simd": rec.get("waves_per_simd") if rec else None,
                    "ops_per_move": opm, "ops_counted": "every + - * / sqrt rint min max compare, one each",
                    "kernel": "k_batch" if h["launches"] else "k_update",
                    "avg_launch_ms": launch_s * 1e3, "events_per_move": ev_per_move,
                    "events_counted_sweeps": n_count}
    line = {
        "metric": "trial moves/sec on 1 MI355X (4096 pentagons), mixed-prec+batched vs plain FP64",
        "value": h["value"],
        "unit": "trial moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "run": head, "replicas": h["replicas"],
                   "path": h["path"], "sweeps_per_step": 1, "seed": args.seed,
                   "queue": args.queue},
        "speedup_vs_fp64_single": (h["value"] / results["fp64_single"]["value"]
                                   if "fp64_single" in results else None),
        "runs": results,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host": platform.node(),
        "device": _device_info(),
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""NPT check against the paper's hard-disk state point (Sec. 4, Table 1):
at beta P sigma^2 = 9.1707 the NVT runs of the paper sit at packing fraction
0.698, so an NPT chain at that pressure must average to it.

Independent replicas start from the triangular lattice at packing fraction
0.698, run cycles of sweeps and one volume move each (``npt.npt_cycles``),
equilibrate, then average the packing fraction N v0 / V; the replicas give
the mean and two standard errors.

    python -m paper_1509_04692_amd.validate_npt [--N 16384] [--replicas 4]
        [--equil 100000] [--cycles 50000] [--sweeps 10] [--delta-v 20]

Prints one progress line per block and a JSON summary at the end.
"""
import argparse
import json
import math
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--N", type=int, default=16384)
    ap.add_argument("--pstar", type=float, default=9.1707, help="beta P sigma^2")
    ap.add_argument("--phi0", type=float, default=0.698, help="starting packing fraction")
    ap.add_argument("--replicas", type=int, default=4)
    ap.add_argument("--equil", type=int, default=100000, help="cycles before averaging")
    ap.add_argument("--cycles", type=int, default=50000, help="cycles averaged")
    ap.add_argument("--sweeps", type=int, default=10, help="sweeps per cycle")
    ap.add_argument("--delta-v", type=float, default=20.0, help="volume move half-width")
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args(argv)

    from . import inputs, npt
    from .system import System

    sp = inputs.disk_species(d=0.1)
    N, R = args.N, args.replicas
    L = inputs.box_length(N, sp["volume"], args.phi0, 2)
    pos, _ = inputs.disk_triangular_lattice(sp, N, L)
    system = System([sp] * R, [N] * R, [L] * R, [pos] * R, [None] * R, path="grid",
                    L_max=[1.05 * L] * R)
    u = inputs.box_move_uniforms((args.equil + args.cycles) * R, seed=2029).reshape(-1, R, 2)
    print(f"# {R} replicas of {N} disks, P*={args.pstar}, start phi={args.phi0}, L={L:.4f}",
          flush=True)
    t0 = time.time()
    sums, acc = np.zeros(R), np.zeros(R, dtype=np.int64)
    block = max(1, (args.equil + args.cycles) // 20)
    for c in range(args.equil + args.cycles):
        system.sweep(args.sweeps, args.seed)
        for r in range(R):
            acc[r] += npt.npt_cycles(system, r, args.seed, u[c, r:r + 1], 0, args.pstar,
                                     args.delta_v)
        if c >= args.equil:
            sums += np.array([N * sp["volume"] / system.L[r] ** 2 for r in range(R)])
        if (c + 1) % block == 0:
            phis = [N * sp["volume"] / system.L[r] ** 2 for r in range(R)]
            print(f"# cycle {c + 1}, phi " + " ".join(f"{x:.5f}" for x in phis)
                  + f", acceptance {acc.sum() / ((c + 1) * R):.3f}, {time.time() - t0:.1f} s",
                  flush=True)
    phi = sums / args.cycles
    sem = float(phi.std(ddof=1) / math.sqrt(R)) if R > 1 else float("nan")
    out = {"N": N, "pstar": args.pstar, "replicas": R, "equil_cycles": args.equil,
           "cycles": args.cycles, "sweeps_per_cycle": args.sweeps, "delta_v": args.delta_v,
           "phi": phi.tolist(), "phi_mean": float(phi.mean()), "two_sem": 2 * sem,
           "reference_phi": 0.698, "volume_acceptance": float(acc.sum() / ((args.equil + args.cycles) * R)),
           "overlaps": [int(x) for x in system.count_overlaps()], "seconds": time.time() - t0}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

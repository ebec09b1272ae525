"""NVT pressure of hard disks or hard spheres from the contact value of g(r)
-- the paper's validation of correct sampling (Sec. 4, Table 1): 65536 disks
at packing fraction 0.698, P* = beta P sigma^2 = 9.1707(2); 131072 spheres
at packing fraction 0.60 (FCC solid), P* = beta P v0 = 9.3135(4) (serial
run; v0 the sphere volume).

Independent replicas (own random streams) start from a triangular lattice
with random vacancies (disks) or the FCC lattice (spheres, one-vertex
spheropolyhedra), equilibrate, then sample the pair-separation histogram
just outside contact every few sweeps; each replica's shell averages are
extrapolated to contact and converted to a pressure, and the replicas give
the mean and two standard errors.

    python -m paper_1509_04692_amd.validate_pressure [--shape disk|sphere]
        [--N ...] [--phi ...] [--replicas 4] [--equil 20000] [--samples 400]
        [--every 50]

Prints one progress line per sampling block and a JSON summary at the end.
"""
import argparse
import json
import math
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--shape", choices=["disk", "sphere", "trunc_oct"], default="disk")
    ap.add_argument("--route", choices=["contact", "scale"], default=None,
                    help="contact value of g(r) (default for disks and spheres) or volume "
                         "perturbation (default, and the only route, for truncated octahedra)")
    ap.add_argument("--N", type=int, default=None, help="default 65536 disks / 131072 spheres")
    ap.add_argument("--phi", type=float, default=None, help="default 0.698 disks / 0.60 spheres")
    ap.add_argument("--replicas", type=int, default=4)
    ap.add_argument("--equil", type=int, default=20000, help="sweeps before sampling")
    ap.add_argument("--samples", type=int, default=400, help="histograms per replica")
    ap.add_argument("--every", type=int, default=50, help="sweeps between histograms")
    ap.add_argument("--d", type=float, default=None,
                    help="translation half-width (default 0.1 disks / 0.04 spheres)")
    ap.add_argument("--window", type=float, default=0.03, help="fit window beyond contact, in sigma")
    ap.add_argument("--bin", type=float, default=0.002, help="shell width, in sigma")
    ap.add_argument("--fits", default="0.02:2,0.03:2,0.05:3",
                    help="extra (window:degree) extrapolations reported from the same counts")
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args(argv)

    from . import inputs, pressure
    from .system import System

    sphere = args.shape == "sphere"
    if args.shape == "trunc_oct":
        return _scale_route_trunc_oct(args)
    if args.route == "scale":
        return _scale_route_trunc_oct(args)
    dim = 3 if sphere else 2
    N = args.N or (131072 if sphere else 65536)
    phi = args.phi or (0.60 if sphere else 0.698)
    d = args.d or (0.04 if sphere else 0.1)
    if sphere:
        sp = inputs.sphere_species(1.0, d=d)
        L, pos, orient = inputs.initial_state(sp, N, phi)
        reference = 9.3135

        def to_pstar(g):  # beta P v0 with v0 = pi sigma^3 / 6
            return pressure.sphere_pressure(N, L, 1.0, g) * math.pi / 6.0
    else:
        sp = inputs.disk_species(d=d)
        L = inputs.box_length(N, sp["volume"], phi, 2)
        pos, orient = inputs.disk_triangular_lattice(sp, N, L)
        reference = 9.1707

        def to_pstar(g):  # beta P sigma^2
            return pressure.disk_pressure(N, L, 1.0, g)
    args.phi = phi
    R = args.replicas
    system = System([sp] * R, [N] * R, [L] * R, [pos] * R, [orient] * R, path="grid")
    n = system.replica_info(0)["n"]
    w = L / n
    fits = [(float(a), int(b)) for a, b in (f.split(":") for f in args.fits.split(",") if f)]
    widest = max([args.window] + [f[0] for f in fits])
    nb = int(round(widest / args.bin))
    if nb > 64 or 1.0 + nb * args.bin >= 2.0 * w:
        raise SystemExit("too many shells, or shells beyond two cell widths")
    edges2 = (1.0 + args.bin * np.arange(nb + 1)) ** 2
    main_bins = int(round(args.window / args.bin))
    print(f"# {R} replicas of {N} {args.shape}s, phi={phi}, L={L:.4f}, n={n}, w={w:.5f}, d={d}",
          flush=True)
    t0 = time.time()
    done = 0
    while done < args.equil:
        step = min(5000, args.equil - done)
        system.sweep(step, args.seed)
        done += step
        system.synchronize()
        print(f"# equilibration {done}/{args.equil} sweeps, {time.time() - t0:.1f} s", flush=True)
    sums = np.zeros((R, nb))
    block = max(1, args.samples // 10)
    for s in range(args.samples):
        system.sweep(args.every, args.seed)
        for r in range(R):
            sums[r] += system.pair_histogram(edges2, r)
        if (s + 1) % block == 0:
            g0 = [pressure.contact_value(edges2[:main_bins + 1], sums[r, :main_bins] / (s + 1), N, L,
                                         1.0, dim=dim)[0] for r in range(R)]
            p = [to_pstar(g) for g in g0]
            print(f"# {s + 1}/{args.samples} samples, P* per replica "
                  + " ".join(f"{x:.4f}" for x in p) + f", {time.time() - t0:.1f} s", flush=True)
    def estimate(window, degree):
        k = int(round(window / args.bin))
        g = np.array([pressure.contact_value(edges2[:k + 1], sums[r, :k] / args.samples, N, L, 1.0,
                                             dim=dim, degree=degree, n_samples=args.samples)[0]
                      for r in range(R)])
        p = np.array([to_pstar(x) for x in g])
        sem = float(p.std(ddof=1) / math.sqrt(R)) if R > 1 else float("nan")
        return g, p, sem

    g0, p, sem = estimate(args.window, 2)
    others = {}
    for window, degree in fits:
        _, pf, sf = estimate(window, degree)
        others[f"{window}:{degree}"] = [float(pf.mean()), 2 * sf]
    st = system.stats()
    out = {"shape": args.shape, "N": N, "phi": phi, "L": L, "replicas": R,
           "equil_sweeps": args.equil,
           "samples": args.samples, "every": args.every, "window": args.window,
           "g_contact": g0.tolist(), "P_star": p.tolist(), "P_star_mean": float(p.mean()),
           "two_sem": 2 * sem, "reference": reference, "fits": others,
           "acceptance": sum(x["accept"] for x in st) / max(1, sum(x["attempted"] for x in st)),
           "overlaps": [int(x) for x in system.count_overlaps()],
           "seconds": time.time() - t0}
    print(json.dumps(out), flush=True)
    return 0


def _scale_route_trunc_oct(args):
    """Volume-perturbation route (Sec. 4): mean counts C(s) of pairs that
    overlap after shrinking the box by 1 - s, C'(0) from a polynomial fit of
    C(s) / s, beta P / rho = 1 + C'(0) / (dim N), P* = beta P v0 = phi beta P / rho.
    Truncated octahedra: 16000 on the BCC solid at packing fraction 0.7
    (reference 13.8975(17), serial); spheres and disks as cross-checks."""
    from . import inputs, pressure
    from .system import System

    if args.shape == "trunc_oct":
        N = args.N or 16000
        phi = args.phi or 0.70
        sp, N, L, pos, orient = inputs.workload_truncated_octahedra_solid(N, phi)
        if args.d:
            sp["d"] = args.d
        dim, reference = 3, 13.8975
    elif args.shape == "sphere":
        N = args.N or 131072
        phi = args.phi or 0.60
        sp = inputs.sphere_species(1.0, d=args.d or 0.04)
        L, pos, orient = inputs.initial_state(sp, N, phi)
        dim, reference = 3, 9.3135
    else:
        N = args.N or 65536
        phi = args.phi or 0.698
        sp = inputs.disk_species(d=args.d or 0.1)
        L = inputs.box_length(N, sp["volume"], phi, 2)
        pos, orient = inputs.disk_triangular_lattice(sp, N, L)
        dim, reference = 2, 9.1707

    def to_pstar(beta_p_over_rho):
        if args.shape == "disk":  # beta P sigma^2 = (beta P / rho) rho sigma^2
            return beta_p_over_rho * N / L ** 2
        return beta_p_over_rho * phi  # beta P v0 = (beta P / rho) phi

    R = args.replicas
    system = System([sp] * R, [N] * R, [L] * R, [pos] * R, [orient] * R, path="grid")
    fits = [(float(a), int(b)) for a, b in (f.split(":") for f in args.fits.split(",") if f)]
    widest = max([args.window] + [f[0] for f in fits])
    ns = int(round(widest / args.bin))
    if ns > 64:
        raise SystemExit("too many scale factors (at most 64)")
    scales = args.bin * np.arange(1, ns + 1)
    print(f"# {R} replicas of {N} {args.shape}s, phi={phi}, L={L:.4f}, "
          f"n={system.replica_info(0)['n']}, d={sp['d']}, a={sp['a']}, scales up to {scales[-1]}",
          flush=True)
    t0 = time.time()
    done = 0
    while done < args.equil:
        step = min(5000, args.equil - done)
        system.sweep(step, args.seed)
        done += step
        system.synchronize()
        print(f"# equilibration {done}/{args.equil} sweeps, {time.time() - t0:.1f} s", flush=True)
    sums = np.zeros((R, ns))
    block = max(1, args.samples // 10)

    def estimate(window, degree, n_done):
        k = int(round(window / args.bin))
        p = np.array([to_pstar(pressure.scale_pressure(N, dim, scales[:k], sums[r, :k] / n_done,
                                                       degree=degree, n_samples=n_done))
                      for r in range(R)])
        sem = float(p.std(ddof=1) / math.sqrt(R)) if R > 1 else float("nan")
        return p, sem

    for s in range(args.samples):
        system.sweep(args.every, args.seed)
        for r in range(R):
            sums[r] += system.scale_counts(scales, r)
        if (s + 1) % block == 0:
            p, _ = estimate(args.window, 1, s + 1)
            print(f"# {s + 1}/{args.samples} samples, P* per replica "
                  + " ".join(f"{x:.4f}" for x in p) + f", {time.time() - t0:.1f} s", flush=True)
    p, sem = estimate(args.window, 1, args.samples)
    others = {}
    for window, degree in fits:
        pf, sf = estimate(window, degree, args.samples)
        others[f"{window}:{degree}"] = [float(pf.mean()), 2 * sf]
    st = system.stats()
    out = {"shape": args.shape, "route": "scale", "N": N, "phi": phi, "L": L, "replicas": R,
           "equil_sweeps": args.equil, "samples": args.samples, "every": args.every,
           "window": args.window, "P_star": p.tolist(), "P_star_mean": float(p.mean()),
           "two_sem": 2 * sem, "reference": reference, "fits": others,
           "mean_counts_first": (sums[:, 0] / args.samples).tolist(),
           "acceptance": sum(x["accept"] for x in st) / max(1, sum(x["attempted"] for x in st)),
           "overlaps": [int(x) for x in system.count_overlaps()],
           "seconds": time.time() - t0}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

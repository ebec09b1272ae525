"""Isothermal-isobaric (NPT) runs: checkerboard sweeps interleaved with
isotropic volume moves (the paper runs NVT and NPT ensembles, Sec. 1).

Each cycle runs ``sweeps_per_cycle`` sweeps of every replica, then one volume
move of replica r: V -> V + delta_v (2 u1 - 1) with the cycle's uniforms
(u1, u2).  The move is rejected when V' <= 0, when L' = V'^(1/dim) exceeds
the replica's L_max or leaves fewer than 4 cells per side, or, for a
compression, when the scaled state has an overlapping pair; otherwise it is
accepted when u2 < exp(-beta_p dV + N ln(V'/V)).  The box change and the
overlap count run in the library's kernels (``System.scale_box``); this
module holds only the host-side acceptance arithmetic.
"""
import math

from ._lib import HpmcError


def npt_cycles(system, r, seed, uniforms, sweeps_per_cycle, beta_p, delta_v):
    """Run len(uniforms) cycles on replica r; returns accepted volume moves."""
    dim = system.species[r]["dim"]
    N = system.N[r]
    accepted = 0
    for u1, u2 in uniforms:
        if sweeps_per_cycle:
            system.sweep(sweeps_per_cycle, seed)
        L = system.L[r]
        V = L ** dim
        dV = delta_v * (2.0 * u1 - 1.0)
        V2 = V + dV
        if not V2 > 0.0:
            continue
        L2 = V2 ** (1.0 / dim)
        if L2 > system.L_max[r]:
            continue
        try:
            overlaps = system.scale_box(r, L2)
        except HpmcError as e:
            if e.code == -2:  # fewer than 4 cells per side: not a valid box
                continue
            raise
        if (dV < 0.0 and overlaps > 0) or not u2 < math.exp(-beta_p * dV + N * math.log(V2 / V)):
            system.restore_box(r)
            continue
        accepted += 1
    return accepted

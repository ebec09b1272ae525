"""Isothermal-isobaric (NPT) runs: checkerboard sweeps interleaved with
isotropic volume moves (the paper runs NVT and NPT ensembles, Sec. 1).

Each cycle runs ``sweeps_per_cycle`` sweeps of every replica, then one volume
move of replica r with the cycle's uniforms (u1, u2).  The library proposes,
scales, counts overlaps and decides the move (``hpmc_volume_move``); this
module only loops over the cycles.
"""


def npt_cycles(system, r, seed, uniforms, sweeps_per_cycle, beta_p, delta_v):
    """Run len(uniforms) cycles on replica r; returns accepted volume moves."""
    accepted = 0
    for u1, u2 in uniforms:
        if sweeps_per_cycle:
            system.sweep(sweeps_per_cycle, seed)
        accepted += int(system.volume_move(r, u1, u2, beta_p, delta_v))
    return accepted

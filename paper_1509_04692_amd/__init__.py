"""MI355X (gfx950) checkerboard hard-shape Metropolis Monte Carlo.

The hot path of HPMC (Anderson, Irrgang, Glotzer): a checkerboard-parallel
Metropolis sweep of hard disks, convex polygons and convex polyhedra, written
as HIP kernels behind the C ABI of include/hpmc.h.  ``System`` is the Python
front end; ``inputs`` writes down synthetic workloads.
"""


def __getattr__(name):
    if name == "System":
        from .system import System
        return System
    if name == "HpmcError":
        from ._lib import HpmcError
        return HpmcError
    raise AttributeError(name)

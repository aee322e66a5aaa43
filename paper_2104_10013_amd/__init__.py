"""MI355X (gfx950) training step of domain-decomposed PINNs (cPINN / XPINN).

The compute path is libddpinn.so (HIP kernels + C ABI, include/ddpinn.h);
this package holds its ctypes binding, the in-tree build script and the
seeded workload generator.
"""
from . import workloads  # noqa: F401


def problem(*args, **kw):
    from .ddpinn import Problem
    return Problem(*args, **kw)

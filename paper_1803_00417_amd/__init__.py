"""MI355X (gfx950) HIP implementation of one semi-implicit time step of the
Papanastasiou-regularised Herschel-Bulkley incompressible flow solver
(Sverdrup, Nikiforakis & Almgren, arXiv 1803.00417).

The compute path is the C-ABI library ``libhb.so`` (include/hb.h); ``hb`` is
its Python binding and ``inputs`` holds the seeded synthetic workloads.
"""
from . import inputs  # noqa: F401

__all__ = ["hb", "inputs"]

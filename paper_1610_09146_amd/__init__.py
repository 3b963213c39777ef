"""MI355X (gfx950) library for the explicit finite-difference compressible
Navier-Stokes residual and low-storage RK3 update of Jammy, Jacobs &
Sandham (arXiv 1610.09146), with the paper's derivative-storage algorithms.

The compute path is the HIP shared library ``libnsf.so`` (C ABI in
``include/nsf.h``); ``paper_1610_09146_amd.nsf`` is its Python binding.
Importing this package loads nothing; ``paper_1610_09146_amd.nsf`` loads
torch and the library on first use.
"""

__all__ = ["nsf", "workloads", "build"]

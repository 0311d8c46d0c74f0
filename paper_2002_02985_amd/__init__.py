"""Orbital-free DFT energy/potential engine for one AMD MI355X (gfx950).

The compute path is the C-ABI library ``libofdft.so`` (hand-written HIP
kernels); ``paper_2002_02985_amd.ofdft`` is its ctypes binding and
``paper_2002_02985_amd.workloads`` the seeded input generators.  Importing the
package does not load the library; ``ofdft.load()`` does, and raises if the
library has not been built.
"""
__all__ = ["ofdft", "workloads"]

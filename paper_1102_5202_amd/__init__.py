"""MI355X-native GRMHD substep (arXiv:1102.5202): HIP kernels behind a C ABI.

The compute path is ``libgrmhd.so`` (hand-written HIP for gfx950), reached
through the ctypes binding in :mod:`paper_1102_5202_amd.grmhd`.  Importing the
package does not load the library; :func:`paper_1102_5202_amd.grmhd.load`
does, and fails loudly when it is missing.
"""

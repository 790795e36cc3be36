"""MI355X-native multigrid solver for the axisymmetric 2D drift-diffusion
fluid equations of Ristivojevic & Petrovic (arXiv:0811.4446).

The compute path is the C-ABI library ``libmgfluid.so`` (hand-written HIP
kernels for gfx950); ``paper_0811_4446_amd.mgfluid`` is its thin Python
binding.  Importing the package itself loads nothing.
"""
__all__ = ["inputs", "mgfluid"]

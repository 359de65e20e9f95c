"""MI355X (gfx950) differentiable SG-splatting renderer (MEGS^2, arXiv 2509.07021).

The renderer lives in libmegs.so (C ABI in include/megs.h, HIP kernels in csrc/);
`render` exposes it to PyTorch. Importing the package loads nothing; the library is
loaded on first use and its absence is an error.
"""
__all__ = ["render", "scenes"]

"""chasm-advect: MI355X-native characteristic (spatial-advection) step of the CHASM
scheme for the 6-D Wigner equation (Xiong, Zhang, Shao, arXiv:2205.02380).

The compute path is the C-ABI library ``libchasm.so`` (hand-written gfx950 HIP
kernels plus a C++ host planner); ``paper_2205_02380_amd.chasm`` is its Python
binding.  Importing this package loads nothing: the library is loaded on first use
and its absence is an error, never a fallback.
"""
__all__ = ["inputs", "chasm"]

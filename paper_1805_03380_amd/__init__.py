"""MI355X-native sparse assembly and CSC SpMM (Sanderson & Curtin, arXiv:1805.03380).

COO -> CSC bulk assembly (sort by (col,row), sum duplicates in input order, drop exact zeros,
scan column pointers) and the CSC sparse x dense product with its adjoint, as hand-written HIP
kernels for gfx950 behind the C ABI declared in ``include/spm.h``.  Python here only marshals
arguments: importing the package does not load the native library; the first call does, and it
raises if the library is missing or no GPU is present.
"""
__all__ = ["ops", "synth"]
__version__ = "0.1.0"

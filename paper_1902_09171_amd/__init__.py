"""MI355X-native batched r-cell molecular dynamics (hierarchical FE-MD coupling of
arXiv:1902.09171) behind the C ABI of include/rcell.h.

Submodules: ``rcell`` (binding of the MD library), ``build`` (hipcc build of librcell.so).
Importing the package loads nothing; the binding raises if the library is not built.
"""
__all__ = ["rcell", "build"]

"""MI355X-native engine for sparse ragged-row spiking networks with e-prop,
DEEP R and topographic-map rewiring (arXiv 2510.19764).

The compute path is the HIP library ``libragsnn.so`` behind the C-ABI in
``include/ragsnn.h``; ``paper_2510_19764_amd.binding`` is its thin ctypes
binding.  Importing this package loads nothing; the library is loaded on first
use and a missing build is an error, never a fallback.
"""
__all__ = ["binding", "workload"]

"""Balanced-tree FMM evaluation pass for MI355X (gfx950).

The computation lives in the HIP library `libfmm.so` (C ABI: include/fmm.h);
`paper_2002_04894_amd.fmm` is its ctypes binding with the same function names.
"""
__all__ = ["fmm", "workloads"]

"""MI355X-native batched subsequence DTW for raw nanopore signal alignment
(RawAlign, arXiv 2310.05037, Sec. 2.2-2.4).

The compute path lives in the HIP library ``librawalign.so`` behind a C ABI
(``include/rawalign.h``); ``paper_2310_05037_amd.lib`` is a thin ctypes
binding with the same entry-point names.  ``workloads`` generates seeded
synthetic inputs.
"""
__all__ = ["lib", "workloads"]

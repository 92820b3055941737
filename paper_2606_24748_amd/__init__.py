"""Natively blocked smoothed-aggregation AMG solve phase for AMD MI355X (gfx950).

The compute lives in libblkamg.so (hand-written HIP kernels behind a C ABI, see
include/blkamg.h); `blkamg` is its ctypes binding and `roofline` the byte/flop models
used to report achieved bandwidth.  Import `paper_2606_24748_amd.blkamg` explicitly:
it raises if the library has not been built.
"""
__all__ = ["blkamg", "roofline", "build"]

"""MI355X-native full-polarisation A x W-projection gridding and degridding.

The compute path is the HIP library libpolgrid.so (C ABI: include/polgrid.h);
`paper_2206_15117_amd.polgrid` is its thin Python binding, which imports torch
lazily so the package loads without a GPU.
"""

"""MI355X GCAMPS hot path: HIP kernels behind a C ABI (include/gcamps.h).

``gcamps``   ctypes binding of libgcamps.so (fails loudly if the library is missing)
``workload`` seeded synthetic circuits and candidate sets (data only)
``build``    builds libgcamps.so for gfx950 in-tree
"""

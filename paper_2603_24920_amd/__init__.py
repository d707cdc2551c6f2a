"""DET-LSH hot path for AMD Instinct MI355X (gfx950).

The native library ``libpdet.so`` (HIP kernels behind a C ABI, see
``include/pdet.h``) does all the work; :mod:`paper_2603_24920_amd.pdet` is the
thin ctypes binding. :mod:`paper_2603_24920_amd.workloads` draws the seeded
synthetic inputs.
"""

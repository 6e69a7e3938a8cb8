"""qdmf: multifrontal LDL^T factorise + solve of regularised LP interior-point Newton
systems (arXiv 2508.04370, Sections 3-4) on one AMD Instinct MI355X.

Modules: ``qdmf`` (ctypes binding of libqdmf.so, the C ABI in include/qdmf.h),
``build`` (compiles libqdmf.so for gfx950), ``workloads`` (seeded synthetic inputs).
"""

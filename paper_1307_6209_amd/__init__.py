"""SELL-C-sigma sparse matrix-vector multiplication for AMD Instinct MI355X.

Implements the storage format and kernel of Kreutzer, Hager, Wellein,
Fehske, Bishop, "A unified sparse matrix data format for efficient general
sparse matrix-vector multiply on modern processors with wide SIMD units"
(arXiv:1307.6209) as hand-written HIP kernels for gfx950 behind a C ABI
(include/sellcs.h). ``sellcs`` is the Python binding; ``model`` holds the
paper's code-balance performance model.
"""
from .sellcs import (SellBatch, SellError, SellMatrix, sell_autotune, sell_batch_autotune,  # noqa: F401
                     sell_batch_create, sell_batch_create_persistent, sell_batch_destroy, sell_batch_spmv, sell_build,
                     sell_crs_spmv, sell_destroy, sell_export, sell_info, sell_permute, sell_probe_bandwidth,
                     sell_spmmv, sell_spmv, sell_unpermute)

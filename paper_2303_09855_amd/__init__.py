"""MI355X-native ADSampling-IVF (Gao & Long, SIGMOD 2023).

The compute path is the HIP library ``_lib/libads.so`` (sources in ``csrc/``,
C ABI in ``include/ads.h``); this package is its ctypes binding.  PyTorch is
used for device memory and streams only.
"""

from ._binding import (  # noqa: F401
    ADSAMPLING, BF16, EXPORTED, F16, F32, FDSCANNING, NSTATS, PDSCANNING, STAT_BYTES, STAT_DCOS,
    STAT_DIMS, STAT_POSITIVES, AdsError, Index, dco_batch, ivf_build, last_error, load,
    make_rotation, profile_collect, profile_enable, rotate, search, search_noalloc, search_workspace_size, version,
    PHASES, METRIC_COSINE, METRIC_L2, NOALLOC_SCRATCH_BYTES, Plan, dco_batch_ip, get_tuning, set_tuning,
    build_ivf, kmeans, HNSW_PLAIN, HNSW_PLUS, HNSW_PP, HnswIndex, hnsw_create, hnsw_search,
    hnsw_workspace_size,
)

"""MI355X (gfx950) Cluster-BFS: Python binding of libcbfs.so.

Argument marshalling only: every step runs in the C/HIP library declared in
``include/cbfs.h``.  PyTorch supplies device memory and the stream.  Importing
works without a GPU; calling a device entry point needs the built library
(``python -m paper_2410_17226_amd.build``) and a GPU, and raises otherwise.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    CBFS_OK, CBFS_E_RADIUS, CBFS_MODE_AUTO, CBFS_MODE_HOST_LOOP, CBFS_MODE_PERSISTENT,
    CBFS_CSR_ALL, CBFS_ENCODE_CENTER, CBFS_ENCODE_MIN, UNREACHED, CbfsError, LIB_PATH, load, exported_symbols,
    planes_of,
    build_csr, top_degree, select_clusters, select_landmarks,
    Tuning, run_batch_workspace_size, run_batch, autotune, run_batch_static, STATIC_SCRATCH_BYTES,
    labels_pack, query_batch, labels_pack_compact, query_batch_compact, query_local, LOCAL_TAU_MAX, pll_build, pll_query, PLL_LABEL_CAP_MAX,
    status_string,
    last_run_stats, profile_enable, profile_read, KERNEL_KINDS, release,
)

"""ctypes binding of libcbfs.so (names follow ``include/cbfs.h``)."""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcbfs.so")

CBFS_OK = 0
CBFS_E_RADIUS = -5
CBFS_MODE_AUTO = 0
CBFS_MODE_HOST_LOOP = 1
CBFS_MODE_PERSISTENT = 2
CBFS_CSR_ALL = 15
CBFS_ENCODE_CENTER = 0
CBFS_ENCODE_MIN = 1
UNREACHED = 0xFFFFFFFF

SYMBOLS = [
    "cbfs_status_string", "cbfs_last_error", "cbfs_build_csr", "cbfs_top_degree",
    "cbfs_select_clusters", "cbfs_run_batch_workspace_size", "cbfs_run_batch",
    "cbfs_last_run_stats", "cbfs_profile_enable", "cbfs_profile_read",
    "cbfs_labels_pack", "cbfs_query_batch", "cbfs_autotune_workspace_size", "cbfs_autotune",
    "cbfs_release", "cbfs_run_batch_static", "cbfs_select_landmarks", "cbfs_query_local",
    "cbfs_pll_workspace_size", "cbfs_pll_build", "cbfs_pll_query", "cbfs_labels_pack_compact",
    "cbfs_query_batch_compact",
]
KERNEL_KINDS = ["tiles", "init", "seed", "push", "pull", "finalize", "persistent", "labels", "query", "local", "pll"]

_lib = None


class CbfsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})" + (f": {detail}" if detail else ""))


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class _Batch(ctypes.Structure):
    _fields_ = [("num_clusters", ctypes.c_int32), ("cluster_ptr", ctypes.c_void_p),
                ("sources", ctypes.c_void_p), ("radius", ctypes.c_int32), ("encoding", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("group_words", ctypes.c_int32),
                ("concurrent_groups", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("alpha", ctypes.c_float), ("beta", ctypes.c_float),
                ("force_pull", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("gamma", ctypes.c_float), ("hub_arcs", ctypes.c_int32),
                ("field_bits", ctypes.c_int32)]


class _Trial(ctypes.Structure):
    _fields_ = [("tuning", _Tuning), ("ms", ctypes.c_float), ("mode", ctypes.c_int32)]


class _RunStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "groups", "group_words", "slots", "mode", "rounds", "push_rounds", "pull_rounds",
        "frontier_vertices", "frontier_arcs", "device_error", "persistent_blocks", "pull_frontier_vertices")]


class _CompactLabels(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("num_clusters", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("w", ctypes.c_int32), ("dist8", ctypes.c_void_p), ("masks", ctypes.c_void_p)]


class _Labels(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("num_clusters", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("dist_vm", ctypes.c_void_p), ("mask_vm", ctypes.c_void_p)]


@dataclass
class Tuning:
    """Mirror of ``cbfs_tuning``; zero fields mean the library default."""
    mode: int = 0
    group_words: int = 0
    concurrent_groups: int = 0
    block_size: int = 0
    alpha: float = 0.0
    beta: float = 0.0
    force_pull: int = 0
    blocks_per_cu: int = 0
    schedule: int = 0
    gamma: float = 0.0
    hub_arcs: int = 0
    field_bits: int = 0

    @classmethod
    def _from_c(cls, t: _Tuning) -> "Tuning":
        return cls(t.mode, t.group_words, t.concurrent_groups, t.block_size, t.alpha, t.beta, t.force_pull,
                   t.blocks_per_cu, t.schedule, t.gamma, t.hub_arcs, t.field_bits)

    def _c(self) -> _Tuning:
        return _Tuning(self.mode, self.group_words, self.concurrent_groups, self.block_size,
                       self.alpha, self.beta, self.force_pull, self.blocks_per_cu, self.schedule, self.gamma,
                       self.hub_arcs, self.field_bits)


def load():
    """Load libcbfs.so; raises if it was not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_17226_amd.build`")
    # One HIP runtime per process: torch brings its own libamdhip64 (same
    # soname); loading it first makes libcbfs bind to that copy instead of a
    # second runtime that would not see the device torch already opened.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    lib.cbfs_status_string.argtypes = [i32]
    lib.cbfs_status_string.restype = ctypes.c_char_p
    lib.cbfs_last_error.argtypes = []
    lib.cbfs_last_error.restype = ctypes.c_char_p
    lib.cbfs_build_csr.argtypes = [i64, i64, P, P, u32, P, P, i64, P, P, P]
    lib.cbfs_build_csr.restype = i32
    lib.cbfs_top_degree.argtypes = [i64, P, i32, P]
    lib.cbfs_top_degree.restype = i32
    lib.cbfs_select_clusters.argtypes = [i64, P, P, i32, P, i32, i32, P, P, i64]
    lib.cbfs_select_clusters.restype = i32
    lib.cbfs_select_landmarks.argtypes = [i64, P, P, i32, i32, i32, P, P, i64, P]
    lib.cbfs_select_landmarks.restype = i32
    lib.cbfs_run_batch_workspace_size.argtypes = [P, P, P]
    lib.cbfs_run_batch_workspace_size.restype = sz
    lib.cbfs_run_batch.argtypes = [P, P, P, P, P, P, P, sz, P]
    lib.cbfs_run_batch.restype = i32
    lib.cbfs_last_run_stats.argtypes = [P]
    lib.cbfs_last_run_stats.restype = i32
    lib.cbfs_profile_enable.argtypes = [i32]
    lib.cbfs_profile_enable.restype = i32
    lib.cbfs_profile_read.argtypes = [P, P]
    lib.cbfs_profile_read.restype = i32
    lib.cbfs_labels_pack.argtypes = [P, P, i32, i64, i32, P, P, P]
    lib.cbfs_labels_pack.restype = i32
    lib.cbfs_query_batch.argtypes = [P, i64, P, P, P, P]
    lib.cbfs_query_batch.restype = i32
    lib.cbfs_labels_pack_compact.argtypes = [P, P, i32, i64, i32, i32, P, P, P]
    lib.cbfs_labels_pack_compact.restype = i32
    lib.cbfs_query_batch_compact.argtypes = [P, i64, P, P, P, P]
    lib.cbfs_query_batch_compact.restype = i32
    lib.cbfs_pll_workspace_size.argtypes = [i64, P]
    lib.cbfs_pll_workspace_size.restype = sz
    lib.cbfs_pll_build.argtypes = [P, P, P, i64, P, i32, P, P, P, sz, P]
    lib.cbfs_pll_build.restype = i32
    lib.cbfs_pll_query.argtypes = [P, i64, i32, P, P, i64, P, P, P, P]
    lib.cbfs_pll_query.restype = i32
    lib.cbfs_query_local.argtypes = [P, i64, P, P, i32, P, P]
    lib.cbfs_query_local.restype = i32
    lib.cbfs_autotune_workspace_size.argtypes = [P, P, i32]
    lib.cbfs_autotune_workspace_size.restype = sz
    lib.cbfs_autotune.argtypes = [P, P, P, i32, P, P, P, P, sz, P, P, P, i32, P]
    lib.cbfs_autotune.restype = i32
    lib.cbfs_run_batch_static.argtypes = [P, P, P, P, P, P, P]
    lib.cbfs_run_batch_static.restype = i32
    lib.cbfs_release.argtypes = []
    lib.cbfs_release.restype = i32
    _lib = lib
    # the library's pinned buffers and events go back while the HIP runtime is
    # still up (this handler runs before torch's own exit handlers)
    atexit.register(_release_at_exit)
    return lib


def _release_at_exit():
    if _lib is not None:
        _lib.cbfs_release()


def release():
    """``cbfs_release``: free the library's pinned host buffers and events now."""
    _check(load().cbfs_release(), "cbfs_release")


def exported_symbols():
    """Names from ``include/cbfs.h`` that the loaded library resolves."""
    lib = load()
    return [s for s in SYMBOLS if hasattr(lib, s)]


def status_string(status: int) -> str:
    try:
        return load().cbfs_status_string(int(status)).decode()
    except Exception:
        return str(status)


def _check(rc: int, where: str):
    if rc != CBFS_OK:
        raise CbfsError(rc, where, load().cbfs_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------- host entry points
def build_csr(n_in: int, src, dst, flags: int = CBFS_CSR_ALL):
    """``cbfs_build_csr``: returns (row_ptr int32[n+1], col int32[m], old_to_new int64[n_in])."""
    src = np.ascontiguousarray(src, dtype=np.int64)
    dst = np.ascontiguousarray(dst, dtype=np.int64)
    cap = 2 * src.size
    row_ptr = np.empty(int(n_in) + 1, dtype=np.int32)
    col = np.empty(max(1, cap), dtype=np.int32)
    old_to_new = np.empty(int(n_in), dtype=np.int64)
    n_out, m_out = ctypes.c_int64(), ctypes.c_int64()
    _check(load().cbfs_build_csr(int(n_in), src.size, _np_ptr(src), _np_ptr(dst), int(flags),
                                 _np_ptr(row_ptr), _np_ptr(col), cap, ctypes.byref(n_out),
                                 ctypes.byref(m_out), _np_ptr(old_to_new)), "cbfs_build_csr")
    n, m = n_out.value, m_out.value
    return row_ptr[: n + 1].copy(), col[:m].copy(), old_to_new


def top_degree(row_ptr, count: int) -> np.ndarray:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    out = np.empty(int(count), dtype=np.int32)
    _check(load().cbfs_top_degree(row_ptr.size - 1, _np_ptr(row_ptr), int(count), _np_ptr(out)),
           "cbfs_top_degree")
    return out


def select_clusters(row_ptr, col, centers, k_max: int, hops: int):
    """``cbfs_select_clusters``: returns (cluster_ptr int32[C+1], sources int32[...])."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    centers = np.ascontiguousarray(centers, dtype=np.int32)
    cptr = np.empty(centers.size + 1, dtype=np.int32)
    cap = max(1, centers.size * int(k_max))
    src = np.empty(cap, dtype=np.int32)
    _check(load().cbfs_select_clusters(row_ptr.size - 1, _np_ptr(row_ptr), _np_ptr(col), centers.size,
                                       _np_ptr(centers), int(k_max), int(hops), _np_ptr(cptr),
                                       _np_ptr(src), cap), "cbfs_select_clusters")
    return cptr, src[: cptr[-1]].copy()


def select_landmarks(row_ptr, col, num_clusters: int, k: int, diameter: int):
    """``cbfs_select_landmarks``: the paper's degree-prioritised clusters with
    marking; returns (cluster_ptr int32[C+1], sources int32[...]), C <= num_clusters."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    cptr = np.empty(int(num_clusters) + 1, dtype=np.int32)
    cap = max(1, int(num_clusters) * int(k))
    src = np.empty(cap, dtype=np.int32)
    made = ctypes.c_int32(0)
    _check(load().cbfs_select_landmarks(row_ptr.size - 1, _np_ptr(row_ptr), _np_ptr(col), int(num_clusters), int(k),
                                        int(diameter), _np_ptr(cptr), _np_ptr(src), cap, ctypes.byref(made)),
           "cbfs_select_landmarks")
    C = made.value
    return cptr[: C + 1].copy(), src[: cptr[C]].copy()


# --------------------------------------------------------------------------- device entry points
def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def planes_of(R: int, encoding: int = CBFS_ENCODE_CENTER) -> int:
    return R + 1 if encoding == CBFS_ENCODE_MIN else 2 * R + 1


def _batch_structs(row_ptr_d, col_d, cluster_ptr, sources, R, tuning, encoding=CBFS_ENCODE_CENTER):
    cluster_ptr = np.ascontiguousarray(cluster_ptr, dtype=np.int32)
    sources = np.ascontiguousarray(sources, dtype=np.int32)
    if cluster_ptr.size >= 1 and int(cluster_ptr[-1]) > sources.size:
        raise ValueError("cluster_ptr[-1] exceeds the number of sources")
    g = _Csr(row_ptr_d.numel() - 1, col_d.numel(), row_ptr_d.data_ptr(), col_d.data_ptr())
    b = _Batch(cluster_ptr.size - 1, _np_ptr(cluster_ptr), _np_ptr(sources), int(R), int(encoding))
    t = tuning._c() if tuning is not None else None
    return g, b, t, cluster_ptr, sources


def run_batch_workspace_size(row_ptr_d, col_d, cluster_ptr, sources, R: int, tuning: Tuning | None = None,
                             encoding: int = CBFS_ENCODE_CENTER) -> int:
    g, b, t, _keep1, _keep2 = _batch_structs(row_ptr_d, col_d, cluster_ptr, sources, R, tuning, encoding)
    return int(load().cbfs_run_batch_workspace_size(ctypes.byref(g), ctypes.byref(b),
                                                    ctypes.byref(t) if t is not None else None))


def words_for(cluster_ptr) -> int:
    k = np.diff(np.asarray(cluster_ptr, dtype=np.int64))
    return int((int(k.max()) + 63) // 64)


def run_batch(row_ptr_d, col_d, cluster_ptr, sources, R: int, tuning: Tuning | None = None,
              out=None, workspace=None, stream=None, encoding: int = CBFS_ENCODE_CENTER):
    """``cbfs_run_batch`` on device CSR tensors (int32).

    Returns ``(dist, masks, status)`` as torch tensors on the graph's device:
    dist int32[C][n] (bit pattern of uint32), masks int64[C][P][n][W] (bit
    pattern of uint64; P = 2R+1, or R+1 with encoding CBFS_ENCODE_MIN where R
    is the cluster diameter), status int32[C].  ``out`` may pass preallocated
    tensors of those shapes, ``workspace`` a uint8 tensor of at least the
    required size.
    """
    torch = _torch()
    lib = load()
    g, b, t, cptr, srcs = _batch_structs(row_ptr_d, col_d, cluster_ptr, sources, R, tuning, encoding)
    C = cptr.size - 1
    n = row_ptr_d.numel() - 1
    W = words_for(cptr)
    dev = row_ptr_d.device
    if out is None:
        dist = torch.empty((C, n), dtype=torch.int32, device=dev)
        masks = torch.empty((C, planes_of(R, encoding), n, W), dtype=torch.int64, device=dev)
        status = torch.empty(C, dtype=torch.int32, device=dev)
    else:
        dist, masks, status = out
    need = int(lib.cbfs_run_batch_workspace_size(ctypes.byref(g), ctypes.byref(b),
                                                 ctypes.byref(t) if t is not None else None))
    if need == 0:
        # let the library report the argument error
        need = 1
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    rc = lib.cbfs_run_batch(ctypes.byref(g), ctypes.byref(b), ctypes.byref(t) if t is not None else None,
                            _dptr(dist), _dptr(masks), _dptr(status), _dptr(workspace),
                            workspace.numel(), _stream_ptr(stream))
    _check(rc, "cbfs_run_batch")
    return dist, masks, status


STATIC_SCRATCH_BYTES = 64 << 20


def run_batch_static(row_ptr_d, col_d, cluster_ptr, sources, R: int, tuning: Tuning | None = None,
                     out=None, stream=None, encoding: int = CBFS_ENCODE_CENTER):
    """``cbfs_run_batch_static``: ``run_batch`` with the library's own device
    scratch array as the workspace (no allocation by the library).  ``out``
    may pass preallocated output tensors; otherwise they are created here."""
    torch = _torch()
    lib = load()
    g, b, t, cptr, srcs = _batch_structs(row_ptr_d, col_d, cluster_ptr, sources, R, tuning, encoding)
    C = cptr.size - 1
    n = row_ptr_d.numel() - 1
    if out is None:
        W = words_for(cptr)
        dev = row_ptr_d.device
        out = (torch.empty((C, n), dtype=torch.int32, device=dev),
               torch.empty((C, planes_of(R, encoding), n, W), dtype=torch.int64, device=dev),
               torch.empty(C, dtype=torch.int32, device=dev))
    dist, masks, status = out
    rc = lib.cbfs_run_batch_static(ctypes.byref(g), ctypes.byref(b), ctypes.byref(t) if t is not None else None,
                                   _dptr(dist), _dptr(masks), _dptr(status), _stream_ptr(stream))
    _check(rc, "cbfs_run_batch_static")
    return dist, masks, status


def autotune(row_ptr_d, col_d, cluster_ptr, sources, R: int, start: Tuning | None = None,
             sample_clusters: int = 0, stream=None, max_trials: int = 64):
    """``cbfs_autotune``: returns (best Tuning, [(Tuning, ms, mode) for every trial])."""
    torch = _torch()
    lib = load()
    g, b, t, cptr, srcs = _batch_structs(row_ptr_d, col_d, cluster_ptr, sources, R, start)
    C = cptr.size - 1
    S = min(C, sample_clusters if sample_clusters > 0 else 16)
    n = row_ptr_d.numel() - 1
    dev = row_ptr_d.device
    W = words_for(cptr[: S + 1]) if S >= 1 else 1
    dist = torch.empty((max(S, 1), n), dtype=torch.int32, device=dev)
    masks = torch.empty((max(S, 1), 2 * R + 1, n, W), dtype=torch.int64, device=dev)
    status = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    need = max(1, int(lib.cbfs_autotune_workspace_size(ctypes.byref(g), ctypes.byref(b), int(sample_clusters))))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    best = _Tuning()
    trials = (_Trial * max_trials)()
    count = ctypes.c_int32(0)
    rc = lib.cbfs_autotune(ctypes.byref(g), ctypes.byref(b), ctypes.byref(t) if t is not None else None,
                           int(sample_clusters), _dptr(dist), _dptr(masks), _dptr(status), _dptr(ws), ws.numel(),
                           _stream_ptr(stream), ctypes.byref(best), trials, max_trials, ctypes.byref(count))
    _check(rc, "cbfs_autotune")
    out = [(Tuning._from_c(trials[i].tuning), float(trials[i].ms), int(trials[i].mode))
           for i in range(min(count.value, max_trials))]
    return Tuning._from_c(best), out


def labels_pack(dist, masks, R: int, stream=None):
    """``cbfs_labels_pack``: vertex-major labels (dist_vm int32[n][C], mask_vm int64[n][C][2R],
    planes -R .. R-1)."""
    torch = _torch()
    C, P, n, W = masks.shape
    if W != 1:
        raise ValueError("labels need one mask word per cluster")
    dist_vm = torch.empty((n, C), dtype=torch.int32, device=masks.device)
    mask_vm = torch.empty((n, C, 2 * R), dtype=torch.int64, device=masks.device)
    _check(load().cbfs_labels_pack(_dptr(dist), _dptr(masks), C, n, int(R), _dptr(dist_vm), _dptr(mask_vm),
                                   _stream_ptr(stream)), "cbfs_labels_pack")
    return dist_vm, mask_vm


LOCAL_TAU_MAX = 2048
_MASK_DTYPES = {8: "uint8", 16: "int16", 32: "int32", 64: "int64"}


def labels_pack_compact(dist, masks, R: int, w: int, stream=None):
    """``cbfs_labels_pack_compact``: (dist8 uint8[n][C], masks [n][C][2R] of w-bit words) on the device."""
    torch = _torch()
    C, Pl, n, W = masks.shape
    if W != 1:
        raise ValueError("labels need one mask word per cluster")
    if w not in _MASK_DTYPES:
        raise ValueError("w must be 8, 16, 32 or 64")
    dist8 = torch.empty((n, C), dtype=torch.uint8, device=masks.device)
    mc = torch.empty((n, C, max(1, 2 * R)), dtype=getattr(torch, _MASK_DTYPES[w]), device=masks.device)
    _check(load().cbfs_labels_pack_compact(_dptr(dist), _dptr(masks), C, n, int(R), int(w), _dptr(dist8), _dptr(mc),
                                           _stream_ptr(stream)), "cbfs_labels_pack_compact")
    return dist8, mc


def query_batch_compact(dist8, masks_c, R: int, w: int, s, t, out=None, stream=None):
    """``cbfs_query_batch_compact`` for device int32 tensors s, t; int32 answers (uint32 bits)."""
    torch = _torch()
    n, C = dist8.shape
    q = s.numel()
    ans = out if out is not None else torch.empty(q, dtype=torch.int32, device=s.device)
    L = _CompactLabels(n, C, int(R), int(w), dist8.data_ptr(), masks_c.data_ptr())
    _check(load().cbfs_query_batch_compact(ctypes.byref(L), q, _dptr(s), _dptr(t), _dptr(ans), _stream_ptr(stream)),
           "cbfs_query_batch_compact")
    return ans
PLL_LABEL_CAP_MAX = 4096


class _PllParams(ctypes.Structure):
    _fields_ = [("first", ctypes.c_int32), ("growth", ctypes.c_float), ("max_batch", ctypes.c_int32),
                ("slots", ctypes.c_int32)]


def pll_build(row_ptr, col, order, bp=None, label_cap: int = 256, first: int = 0, growth: float = 0.0,
              max_batch: int = 0, slots: int = 0, stream=None):
    """``cbfs_pll_build`` on device CSR tensors; ``order`` a device int32 tensor
    of roots by rank; ``bp`` = (dist_vm, mask_vm, R) phase-1 labels or None.
    Returns (lab_cnt int32[n], labels int64[n][label_cap]) on the device."""
    torch = _torch()
    n = row_ptr.numel() - 1
    params = _PllParams(int(first), float(growth), int(max_batch), int(slots))
    ws_bytes = load().cbfs_pll_workspace_size(n, ctypes.byref(params))
    if ws_bytes == 0:
        raise CbfsError(-1, "cbfs_pll_workspace_size", "bad batch parameters")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=row_ptr.device)
    cnt = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    labels = torch.empty((n, int(label_cap)), dtype=torch.int64, device=row_ptr.device)
    g = _Csr(n, col.numel(), row_ptr.data_ptr(), col.data_ptr())
    L = None
    if bp is not None:
        dist_vm, mask_vm, R = bp
        L = _Labels(n, dist_vm.shape[1], int(R), dist_vm.data_ptr(), mask_vm.data_ptr())
    _check(load().cbfs_pll_build(ctypes.byref(g), ctypes.byref(L) if L is not None else None, _dptr(order),
                                 order.numel(), ctypes.byref(params), int(label_cap), _dptr(cnt), _dptr(labels),
                                 _dptr(ws), ws_bytes, _stream_ptr(stream)), "cbfs_pll_build")
    return cnt, labels


def pll_query(cnt, labels, s, t, bp=None, out=None, stream=None):
    """``cbfs_pll_query`` for device int32 tensors s, t; int32 answers (uint32 bits)."""
    torch = _torch()
    n, cap = labels.shape
    q = s.numel()
    ans = out if out is not None else torch.empty(q, dtype=torch.int32, device=s.device)
    L = None
    if bp is not None:
        dist_vm, mask_vm, R = bp
        L = _Labels(n, dist_vm.shape[1], int(R), dist_vm.data_ptr(), mask_vm.data_ptr())
    _check(load().cbfs_pll_query(ctypes.byref(L) if L is not None else None, n, cap, _dptr(cnt), _dptr(labels), q,
                                 _dptr(s), _dptr(t), _dptr(ans), _stream_ptr(stream)), "cbfs_pll_query")
    return ans


def query_local(row_ptr, col, s, t, tau: int, out=None, stream=None):
    """``cbfs_query_local``: ans = min(ans, local search answer) for device int32
    tensors s, t; without ``out`` the local answer alone (int32 tensor, uint32 bits)."""
    torch = _torch()
    q = s.numel()
    if out is None:
        out = torch.full((q,), -1, dtype=torch.int32, device=s.device)
    g = _Csr(row_ptr.numel() - 1, col.numel(), row_ptr.data_ptr(), col.data_ptr())
    _check(load().cbfs_query_local(ctypes.byref(g), q, _dptr(s), _dptr(t), int(tau), _dptr(out),
                                   _stream_ptr(stream)), "cbfs_query_local")
    return out


def query_batch(dist_vm, mask_vm, R: int, s, t, out=None, stream=None):
    """``cbfs_query_batch`` for device int32 tensors s, t; returns int32 answers (uint32 bits)."""
    torch = _torch()
    n, C = dist_vm.shape
    q = s.numel()
    ans = out if out is not None else torch.empty(q, dtype=torch.int32, device=s.device)
    L = _Labels(n, C, int(R), dist_vm.data_ptr(), mask_vm.data_ptr())
    _check(load().cbfs_query_batch(ctypes.byref(L), q, _dptr(s), _dptr(t), _dptr(ans), _stream_ptr(stream)),
           "cbfs_query_batch")
    return ans


def last_run_stats() -> dict:
    """``cbfs_last_run_stats`` of this thread's last run_batch (waits for it)."""
    r = _RunStats()
    _check(load().cbfs_last_run_stats(ctypes.byref(r)), "cbfs_last_run_stats")
    return {name: int(getattr(r, name)) for name, _t in _RunStats._fields_}


def profile_enable(on: bool = True):
    """``cbfs_profile_enable``: time every kernel launch of this thread with HIP events."""
    _check(load().cbfs_profile_enable(1 if on else 0), "cbfs_profile_enable")


def profile_read() -> dict:
    """``cbfs_profile_read``: {kernel kind: (launches, total ms)} for the recorded launches."""
    n = len(KERNEL_KINDS)
    launches = (ctypes.c_int64 * n)()
    ms = (ctypes.c_double * n)()
    _check(load().cbfs_profile_read(launches, ms), "cbfs_profile_read")
    return {KERNEL_KINDS[k]: (int(launches[k]), float(ms[k])) for k in range(n)}

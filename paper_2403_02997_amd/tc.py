"""Thin ctypes binding of libtc.so (include/tc.h): argument marshalling only.

Every step of the counting path runs in the library's gfx950 kernels.  PyTorch supplies
device memory and streams: tensors are passed by ``data_ptr()`` and the stream by its
HIP handle.  There is no CPU fallback: if the library is missing or cannot be loaded,
every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK = 0
STATUS = {
    0: "TC_OK",
    -1: "TC_ERR_INVALID_ARG",
    -2: "TC_ERR_OUT_OF_MEMORY",
    -3: "TC_ERR_HIP",
    -4: "TC_ERR_INVALID_GRAPH",
    -5: "TC_ERR_TOO_LARGE",
    -6: "TC_ERR_INTERNAL",
}

# Every symbol include/tc.h declares.
EXPORTS = (
    "tc_count",
    "tc_count_ex",
    "tc_count_split",
    "tc_count_per_vertex",
    "tc_local_clustering",
    "tc_count_batch",
    "tc_count_batch_workspace_size",
    "tc_count_batch_noalloc",
    "tc_serve_create",
    "tc_serve_submit",
    "tc_serve_poll",
    "tc_serve_get_stats",
    "tc_serve_footprint",
    "tc_serve_destroy",
    "tc_validate_csr",
    "tc_set_isect_params",
    "tc_get_isect_params",
    "tc_set_hub_params",
    "tc_get_hub_params",
    "tc_last_call_info",
    "tc_set_forward_threshold",
    "tc_get_forward_threshold",
    "tc_profile_enable",
    "tc_profile_read",
    "tc_profile_step_name",
    "tc_status_string",
    "tc_version",
)


class TCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status_string(status)})")


class _Stats(ctypes.Structure):
    _fields_ = [
        ("triangles", ctypes.c_uint64),
        ("c1", ctypes.c_uint64),
        ("c2", ctypes.c_uint64),
        ("cover_edges", ctypes.c_uint64),
        ("probes", ctypes.c_uint64),
        ("depth", ctypes.c_uint32),
        ("num_roots", ctypes.c_uint32),
        ("bfs_levels_bottom_up", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("class_streamed", ctypes.c_uint64 * 3),
        ("class_staged", ctypes.c_uint64 * 3),
    ]


@dataclass
class Stats:
    triangles: int
    c1: int
    c2: int
    cover_edges: int
    probes: int
    depth: int
    num_roots: int
    bfs_levels_bottom_up: int
    class_streamed: tuple = (0, 0, 0)
    class_staged: tuple = (0, 0, 0)


class _CallInfo(ctypes.Structure):
    _fields_ = [
        ("cover_edges", ctypes.c_uint64),
        ("lane_vertices", ctypes.c_uint32),
        ("wave_vertices", ctypes.c_uint32),
        ("block_vertices", ctypes.c_uint32),
        ("block_items", ctypes.c_uint32),
        ("hubs", ctypes.c_uint32),
        ("hub_items", ctypes.c_uint32),
        ("side_stream", ctypes.c_uint32),
        ("forward", ctypes.c_uint32),
    ]


class _ServeConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("small_max_entries", ctypes.c_uint64),
        ("batch_max_graphs", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("batch_max_entries", ctypes.c_uint64),
        ("large_min_entries", ctypes.c_uint64),
    ]


class _ServeResult(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("triangles", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("path", ctypes.c_uint32),
        ("input_edges", ctypes.c_uint64),
        ("submit_s", ctypes.c_double),
        ("admit_s", ctypes.c_double),
        ("count_s", ctypes.c_double),
        ("done_s", ctypes.c_double),
    ]


class _ServeStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "submitted", "completed", "rejected", "batches", "singles", "queued", "in_flight",
        "hbm_in_use", "hbm_peak", "hbm_budget")] + [("busy_s", ctypes.c_double * 3),
                                                    ("device_s", ctypes.c_double * 3)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libtc.so (built by ``paper_2403_02997_amd.build``).  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2403_02997_amd.build` "
            "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    i = ctypes.c_int
    lib.tc_count.argtypes = [vp, vp, u32, u64, vp, ctypes.POINTER(u64)]
    lib.tc_count.restype = i
    lib.tc_count_split.argtypes = [vp, vp, u32, u64, vp, ctypes.POINTER(u64)]
    lib.tc_count_split.restype = i
    lib.tc_count_ex.argtypes = [vp, vp, u32, u64, vp, ctypes.POINTER(u64), vp,
                                ctypes.POINTER(_Stats)]
    lib.tc_count_ex.restype = i
    lib.tc_count_per_vertex.argtypes = [vp, vp, u32, u64, vp, vp]
    lib.tc_count_per_vertex.restype = i
    lib.tc_local_clustering.argtypes = [vp, vp, u32, vp, vp]
    lib.tc_local_clustering.restype = i
    lib.tc_count_batch.argtypes = [vp, vp, vp, vp, u32, u64, u64, vp, sz, vp, vp]
    lib.tc_count_batch.restype = i
    lib.tc_count_batch_workspace_size.argtypes = [u32, u64, u64]
    lib.tc_count_batch_workspace_size.restype = sz
    lib.tc_count_batch_noalloc.argtypes = [vp, vp, vp, vp, u32, u64, u64, vp, vp]
    lib.tc_count_batch_noalloc.restype = i
    P = ctypes.POINTER
    lib.tc_serve_create.argtypes = [P(_ServeConfig), P(vp)]
    lib.tc_serve_create.restype = i
    lib.tc_serve_submit.argtypes = [vp, vp, vp, u32, u64, P(u64)]
    lib.tc_serve_submit.restype = i
    lib.tc_serve_poll.argtypes = [vp, P(_ServeResult), u32, P(u32), ctypes.c_int32]
    lib.tc_serve_poll.restype = i
    lib.tc_serve_footprint.argtypes = [vp, u32, u64, P(u64)]
    lib.tc_serve_footprint.restype = i
    lib.tc_serve_get_stats.argtypes = [vp, P(_ServeStats)]
    lib.tc_serve_get_stats.restype = i
    lib.tc_serve_destroy.argtypes = [vp]
    lib.tc_serve_destroy.restype = i
    lib.tc_validate_csr.argtypes = [vp, vp, u32, u64, vp]
    lib.tc_validate_csr.restype = i
    lib.tc_set_isect_params.argtypes = [u32, u32, u32, u32]
    lib.tc_set_isect_params.restype = i
    lib.tc_get_isect_params.argtypes = [ctypes.POINTER(u32)]
    lib.tc_get_isect_params.restype = i
    lib.tc_last_call_info.argtypes = [ctypes.POINTER(_CallInfo)]
    lib.tc_last_call_info.restype = i
    lib.tc_set_forward_threshold.argtypes = [ctypes.c_double]
    lib.tc_set_forward_threshold.restype = i
    lib.tc_get_forward_threshold.argtypes = []
    lib.tc_get_forward_threshold.restype = ctypes.c_double
    lib.tc_set_hub_params.argtypes = [u32, u32]
    lib.tc_set_hub_params.restype = i
    lib.tc_get_hub_params.argtypes = [ctypes.POINTER(u32)]
    lib.tc_get_hub_params.restype = i
    lib.tc_profile_enable.argtypes = [i]
    lib.tc_profile_enable.restype = i
    lib.tc_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), u32, ctypes.POINTER(u64), i]
    lib.tc_profile_read.restype = i
    lib.tc_profile_step_name.argtypes = [i]
    lib.tc_profile_step_name.restype = ctypes.c_char_p
    lib.tc_status_string.argtypes = [i]
    lib.tc_status_string.restype = ctypes.c_char_p
    lib.tc_version.argtypes = []
    lib.tc_version.restype = i
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().tc_status_string(int(status)).decode()
    except Exception:  # noqa: BLE001 - only used while formatting another error
        return "?"


def _check(rc: int, where: str) -> None:
    if rc != TC_OK:
        raise TCError(rc, where)


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> int:
    if t is None:
        return 0
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr() if t.numel() else 0


def _n_m(rowptr: torch.Tensor, colidx: torch.Tensor):
    if rowptr.element_size() != 4 or colidx.element_size() != 4:
        raise TypeError("rowptr / colidx must hold 4-byte integers (uint32 bit patterns)")
    n = rowptr.numel() - 1
    if n < 0:
        raise ValueError("rowptr needs n + 1 >= 1 entries")
    return n, colidx.numel()


# --------------------------------------------------------------------------------------
# marshalling helpers
# --------------------------------------------------------------------------------------

def to_device(rowptr: np.ndarray, colidx: np.ndarray, device="cuda"):
    """Upload a uint32 CSR as int32 tensors holding the same bit patterns."""
    r = torch.from_numpy(np.ascontiguousarray(rowptr, dtype=np.uint32).view(np.int32))
    c = torch.from_numpy(np.ascontiguousarray(colidx, dtype=np.uint32).view(np.int32))
    return r.to(device), c.to(device)


# --------------------------------------------------------------------------------------
# entry points (same names as the C ABI)
# --------------------------------------------------------------------------------------

def tc_count(rowptr: torch.Tensor, colidx: torch.Tensor, stream=None) -> int:
    """T for one graph (blocking)."""
    lib = load()
    n, m = _n_m(rowptr, colidx)
    out = ctypes.c_uint64(0)
    rc = lib.tc_count(_ptr(rowptr), _ptr(colidx), n, m, _stream_handle(stream),
                      ctypes.byref(out))
    _check(rc, "tc_count")
    return int(out.value)


def tc_count_split(rowptr: torch.Tensor, colidx: torch.Tensor, stream=None) -> tuple:
    """(t0, t1) of the split form CETC-Seq-S from the pruned pass of tc_count: t0 = the
    triangles inside the subgraph of horizontal edges, t1 = the others (blocking)."""
    lib = load()
    n, m = _n_m(rowptr, colidx)
    out = (ctypes.c_uint64 * 2)()
    rc = lib.tc_count_split(_ptr(rowptr), _ptr(colidx), n, m, _stream_handle(stream), out)
    _check(rc, "tc_count_split")
    return int(out[0]), int(out[1])


def tc_count_ex(rowptr: torch.Tensor, colidx: torch.Tensor, want_levels: bool = False,
                stream=None):
    """(Stats, levels tensor or None)."""
    lib = load()
    n, m = _n_m(rowptr, colidx)
    level = torch.empty(n, dtype=torch.int32, device=rowptr.device) if want_levels else None
    st = _Stats()
    cnt = ctypes.c_uint64(0)
    rc = lib.tc_count_ex(_ptr(rowptr), _ptr(colidx), n, m, _stream_handle(stream),
                         ctypes.byref(cnt), _ptr(level) if level is not None else None,
                         ctypes.byref(st))
    _check(rc, "tc_count_ex")
    stats = Stats(int(st.triangles), int(st.c1), int(st.c2), int(st.cover_edges),
                  int(st.probes), int(st.depth), int(st.num_roots),
                  int(st.bfs_levels_bottom_up), tuple(int(v) for v in st.class_streamed),
                  tuple(int(v) for v in st.class_staged))
    return stats, level


def tc_count_per_vertex(rowptr: torch.Tensor, colidx: torch.Tensor, stream=None) -> torch.Tensor:
    """int64 tensor (uint64 bit patterns) of t(v), the triangles through each vertex."""
    lib = load()
    n, m = _n_m(rowptr, colidx)
    out = torch.empty(max(n, 0), dtype=torch.int64, device=rowptr.device)
    rc = lib.tc_count_per_vertex(_ptr(rowptr), _ptr(colidx), n, m, _stream_handle(stream),
                                 _ptr(out) if n else None)
    _check(rc, "tc_count_per_vertex")
    return out


def tc_local_clustering(rowptr: torch.Tensor, tri: torch.Tensor, stream=None) -> torch.Tensor:
    """float64 tensor of C(v) = 2 t(v) / (d(v) (d(v) - 1)) (0 for d(v) < 2), from the
    per-vertex counts `tri` that tc_count_per_vertex returned for the same graph.
    Stream-ordered: no synchronisation."""
    lib = load()
    n = int(rowptr.numel()) - 1
    if rowptr.element_size() != 4 or tri.element_size() != 8 or tri.is_floating_point():
        raise TypeError("rowptr must hold 4-byte and tri 8-byte integers")
    if n < 0 or tri.numel() != n:
        raise ValueError(f"tri has {tri.numel()} entries for {max(n, 0)} vertices")
    out = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    rc = lib.tc_local_clustering(_ptr(rowptr), _ptr(tri) if n else None, max(n, 0),
                                 _stream_handle(stream), _ptr(out) if n else None)
    _check(rc, "tc_local_clustering")
    return out


def tc_count_batch_workspace_size(num_graphs: int, total_rows: int, total_cols: int) -> int:
    return int(load().tc_count_batch_workspace_size(int(num_graphs), int(total_rows),
                                                    int(total_cols)))


def tc_count_batch(rowptr_cat: torch.Tensor, colidx_cat: torch.Tensor, row_off: torch.Tensor,
                   col_off: torch.Tensor, total_rows: int | None = None,
                   workspace: torch.Tensor | None = None, counts: torch.Tensor | None = None,
                   stream=None, total_cols: int | None = None) -> torch.Tensor:
    """Per-graph counts (int64 tensor of uint64 bit patterns) of a concatenated batch.
    row_off / col_off are int64 device tensors of num_graphs + 1 offsets; total_rows and
    total_cols default to the lengths of rowptr_cat and colidx_cat.  With a caller
    workspace the call is asynchronous and capturable."""
    lib = load()
    if row_off.dtype != torch.int64 or col_off.dtype != torch.int64:
        raise TypeError("row_off / col_off must be int64")
    G = row_off.numel() - 1
    if total_rows is None:
        total_rows = rowptr_cat.numel()
    if total_cols is None:
        total_cols = colidx_cat.numel()
    if counts is None:
        counts = torch.empty(max(G, 0), dtype=torch.int64, device=rowptr_cat.device)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    rc = lib.tc_count_batch(_ptr(rowptr_cat), _ptr(colidx_cat) or None, _ptr(row_off),
                            _ptr(col_off), G, int(total_rows), int(total_cols),
                            _ptr(workspace) if workspace is not None else None, ws_bytes,
                            _stream_handle(stream), _ptr(counts) if G else None)
    _check(rc, "tc_count_batch")
    return counts


NOALLOC_SCRATCH_BYTES = 64 << 20  # TC_NOALLOC_SCRATCH_BYTES


def tc_count_batch_noalloc(rowptr_cat: torch.Tensor, colidx_cat: torch.Tensor,
                           row_off: torch.Tensor, col_off: torch.Tensor, counts: torch.Tensor,
                           total_rows: int | None = None, total_cols: int | None = None,
                           stream=None) -> torch.Tensor:
    """tc_count_batch with the library's fixed per-device scratch array as its workspace:
    nothing is allocated, so `counts` (int64 device tensor of num_graphs entries) is
    required.  Calls that overlap on one device race (the caller serialises them)."""
    lib = load()
    if row_off.dtype != torch.int64 or col_off.dtype != torch.int64:
        raise TypeError("row_off / col_off must be int64")
    G = row_off.numel() - 1
    if G > 0 and (counts is None or counts.numel() < G or counts.dtype != torch.int64):
        raise ValueError("counts must be an int64 device tensor of num_graphs entries")
    if total_rows is None:
        total_rows = rowptr_cat.numel()
    if total_cols is None:
        total_cols = colidx_cat.numel()
    rc = lib.tc_count_batch_noalloc(_ptr(rowptr_cat), _ptr(colidx_cat) or None, _ptr(row_off),
                                    _ptr(col_off), G, int(total_rows), int(total_cols),
                                    _stream_handle(stream), _ptr(counts) if G else None)
    _check(rc, "tc_count_batch_noalloc")
    return counts


def tc_validate_csr(rowptr: torch.Tensor, colidx: torch.Tensor, stream=None) -> int:
    """Status of the device-side format check (TC_OK or TC_ERR_INVALID_GRAPH)."""
    lib = load()
    n, m = _n_m(rowptr, colidx)
    return int(lib.tc_validate_csr(_ptr(rowptr), _ptr(colidx) or None, n, m,
                                   _stream_handle(stream)))


def tc_set_isect_params(lane_max: int, wave_max: int, chunk: int, seg: int) -> None:
    _check(load().tc_set_isect_params(lane_max, wave_max, chunk, seg), "tc_set_isect_params")


def tc_get_isect_params():
    arr = (ctypes.c_uint32 * 4)()
    _check(load().tc_get_isect_params(arr), "tc_get_isect_params")
    return tuple(int(v) for v in arr)


def tc_last_call_info() -> dict:
    """How this thread's last single-graph call divided its work (tc_last_call_info)."""
    info = _CallInfo()
    _check(load().tc_last_call_info(ctypes.byref(info)), "tc_last_call_info")
    return {name: int(getattr(info, name)) for name, _ in _CallInfo._fields_}


def tc_set_forward_threshold(threshold: float) -> None:
    """CETC-Seq-FE's covering-ratio threshold (default 0.7; > 1 never switches)."""
    _check(load().tc_set_forward_threshold(float(threshold)), "tc_set_forward_threshold")


def tc_get_forward_threshold() -> float:
    return float(load().tc_get_forward_threshold())


def tc_set_hub_params(max_hubs: int, min_degree: int) -> None:
    _check(load().tc_set_hub_params(max_hubs, min_degree), "tc_set_hub_params")


def tc_get_hub_params():
    arr = (ctypes.c_uint32 * 2)()
    _check(load().tc_get_hub_params(arr), "tc_get_hub_params")
    return tuple(int(v) for v in arr)


def tc_profile_enable(on: bool = True) -> None:
    load().tc_profile_enable(1 if on else 0)


def tc_profile_read(reset: bool = False):
    """({step name: total ms}, number of profiled calls)."""
    lib = load()
    ms = (ctypes.c_double * 16)()
    calls = ctypes.c_uint64(0)
    k = lib.tc_profile_read(ms, 16, ctypes.byref(calls), 1 if reset else 0)
    names = [lib.tc_profile_step_name(i).decode() for i in range(k)]
    return {names[i]: float(ms[i]) for i in range(k)}, int(calls.value)


def tc_profile_step_name(step: int) -> str:
    return load().tc_profile_step_name(int(step)).decode()


def tc_version() -> int:
    return int(load().tc_version())


# --------------------------------------------------------------------------------------
# continuous-batching server
# --------------------------------------------------------------------------------------

@dataclass
class ServeResult:
    ticket: int
    triangles: int
    status: int
    path: int  # 0 batched, 1 single-graph medium, 3 single-graph large, 2 rejected
    input_edges: int
    submit_s: float
    admit_s: float  # job started: device memory reserved, upload begins
    count_s: float  # the count took the device
    done_s: float

    @property
    def latency_s(self) -> float:
        return self.done_s - self.submit_s


class Server:
    """tc_serve_* on the current device.  submit() takes HOST CSR arrays (numpy arrays or
    CPU torch tensors, e.g. pinned ones) and keeps references to them until their result
    has been polled (the C ABI's lifetime rule)."""

    def __init__(self, hbm_budget_bytes: int = 0, small_max_entries: int = 0,
                 batch_max_graphs: int = 0, batch_max_entries: int = 0,
                 large_min_entries: int = 0):
        lib = load()
        cfg = _ServeConfig(int(hbm_budget_bytes), int(small_max_entries),
                           int(batch_max_graphs), 0, int(batch_max_entries),
                           int(large_min_entries))
        h = ctypes.c_void_p()
        _check(lib.tc_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "tc_serve_create")
        self._h = h
        self._held = {}

    @staticmethod
    def _host(a):
        if isinstance(a, torch.Tensor):
            if a.is_cuda or a.element_size() != 4 or not a.is_contiguous():
                raise ValueError("host CSR tensors must be contiguous 4-byte CPU tensors")
            return a, a.data_ptr() if a.numel() else None, a.numel()
        arr = np.ascontiguousarray(a, dtype=np.uint32)
        return arr, arr.ctypes.data if arr.size else None, arr.shape[0]

    def submit(self, rowptr, colidx) -> int:
        rp, rp_ptr, rp_len = self._host(rowptr)
        ci, ci_ptr, m = self._host(colidx)
        n = rp_len - 1
        if n < 0:
            raise ValueError("rowptr needs n + 1 >= 1 entries")
        t = ctypes.c_uint64(0)
        rc = load().tc_serve_submit(self._h, rp_ptr, ci_ptr, n, m, ctypes.byref(t))
        _check(rc, "tc_serve_submit")
        self._held[int(t.value)] = (rp, ci)
        return int(t.value)

    def poll(self, cap: int = 256, timeout_ms: int = 0):
        arr = (_ServeResult * cap)()
        got = ctypes.c_uint32(0)
        _check(load().tc_serve_poll(self._h, arr, cap, ctypes.byref(got), int(timeout_ms)),
               "tc_serve_poll")
        out = []
        for k in range(got.value):
            r = arr[k]
            self._held.pop(int(r.ticket), None)
            out.append(ServeResult(int(r.ticket), int(r.triangles), int(r.status), int(r.path),
                                   int(r.input_edges), float(r.submit_s), float(r.admit_s),
                                   float(r.count_s), float(r.done_s)))
        return out

    def footprint(self, n: int, m: int) -> int:
        """Device bytes a request of n vertices and m stored entries needs alone."""
        b = ctypes.c_uint64(0)
        _check(load().tc_serve_footprint(self._h, int(n), int(m), ctypes.byref(b)),
               "tc_serve_footprint")
        return int(b.value)

    def stats(self) -> dict:
        st = _ServeStats()
        _check(load().tc_serve_get_stats(self._h, ctypes.byref(st)), "tc_serve_get_stats")
        out = {k: int(getattr(st, k)) for k, _ in _ServeStats._fields_[:-2]}
        for k in ("busy_s", "device_s"):
            a = getattr(st, k)
            out[k] = {"batched": float(a[0]), "medium": float(a[1]), "large": float(a[2])}
        return out

    def close(self) -> None:
        if self._h:
            _check(load().tc_serve_destroy(self._h), "tc_serve_destroy")
            self._h = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def as_u64(t: torch.Tensor) -> np.ndarray:
    """Host numpy uint64 view of an int64 tensor of uint64 bit patterns."""
    return t.cpu().numpy().view(np.uint64)

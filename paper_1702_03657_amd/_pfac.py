"""ctypes binding of ``libpfac.so`` (the C ABI declared in ``include/pfac.h``).

Argument marshalling only: every step of a scan runs in the library's HIP
kernels.  Functions keep the C names; device buffers are passed as torch CUDA
tensors (their ``data_ptr()``), streams as ``torch.cuda.Stream`` objects.
Importing this module does not touch the GPU; loading the library fails
loudly when it has not been built.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfac.so")

PFAC_OK = 0
PFAC_EINVAL = -1
PFAC_EEMPTY = -2
PFAC_ENOMEM = -3
PFAC_EDEVICE = -4
PFAC_ETRUNC = -5
PFAC_ENODEV = -6
PFAC_EBUSY = -7
PFAC_BUILD_HOST_ONLY = 1

MATCH_DTYPE = np.dtype([("pos", "<u8"), ("pattern_id", "<u4"), ("text_id", "<u4")])


class pfac_match(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_uint64), ("pattern_id", ctypes.c_uint32),
                ("text_id", ctypes.c_uint32)]


class pfac_stats(ctypes.Structure):
    _fields_ = [
        ("nodes", ctypes.c_uint64), ("edges", ctypes.c_uint64),
        ("n_patterns", ctypes.c_uint64), ("min_len", ctypes.c_uint64),
        ("max_len", ctypes.c_uint64), ("depth", ctypes.c_uint64),
        ("bytes_crs", ctypes.c_uint64), ("crs_elements", ctypes.c_uint64),
        ("bytes_dense256", ctypes.c_uint64), ("bytes_bitmap36", ctypes.c_uint64),
        ("bytes_device", ctypes.c_uint64),
        ("alphabet_size", ctypes.c_uint32), ("symbol_bits", ctypes.c_uint32),
        ("index_depth", ctypes.c_uint32), ("lds_bytes", ctypes.c_uint32),
        ("scan_kernel", ctypes.c_uint32), ("scan_waves", ctypes.c_uint32),
        ("stage1", ctypes.c_uint32), ("stage2", ctypes.c_uint32),
        ("build_seconds", ctypes.c_double), ("upload_seconds", ctypes.c_double),
        ("bytes_bitmap_narrow", ctypes.c_uint64), ("bytes_level_index", ctypes.c_uint64),
        ("bytes_top_nodes", ctypes.c_uint64), ("trunc_depth", ctypes.c_uint64),
        ("bytes_nodes", ctypes.c_uint64), ("bytes_tails", ctypes.c_uint64),
        ("dag_nodes", ctypes.c_uint64), ("dag_edges", ctypes.c_uint64),
        ("bytes_dag_crs", ctypes.c_uint64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class pfac_tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_uint32), ("bytes_per_lane", ctypes.c_uint32),
                ("index_bits", ctypes.c_uint32), ("fold_bits", ctypes.c_uint32),
                ("wg_per_cu", ctypes.c_uint32), ("waves_per_wg", ctypes.c_uint32),
                ("chunks_per_unit", ctypes.c_uint32), ("child_check", ctypes.c_uint32),
                ("top_nodes", ctypes.c_uint32), ("trunc_depth", ctypes.c_uint32),
                ("dag", ctypes.c_uint32)]


class PfacError(RuntimeError):
    def __init__(self, fn: str, code: int, hip: int = 0):
        self.code = code
        super().__init__(f"{fn} failed: {strerror(code)} (code {code}, hip error {hip})")


_lib = None
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i64 = ctypes.c_int64
_p = ctypes.POINTER

# (name, restype, argtypes) for every entry point of include/pfac.h
SIGNATURES = [
    ("pfac_last_hip_error", ctypes.c_int, []),
    ("pfac_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("pfac_build", ctypes.c_int, [_p(_vp), _p(_u64), _u32, _u32, _p(_vp)]),
    ("pfac_build_packed", ctypes.c_int, [_vp, _p(_u64), _u32, _u32, _p(_vp)]),
    ("pfac_trie_stats", ctypes.c_int, [_vp, _p(pfac_stats)]),
    ("pfac_trie_export", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    ("pfac_trie_free", None, [_vp]),
    ("pfac_trie_get_tuning", ctypes.c_int, [_vp, _p(pfac_tuning)]),
    ("pfac_trie_launch_kernel", ctypes.c_int, [_vp, ctypes.c_uint64, _p(ctypes.c_uint32), _p(pfac_tuning)]),
    ("pfac_trie_set_tuning", ctypes.c_int, [_vp, _p(pfac_tuning)]),
    ("pfac_workspace_create", ctypes.c_int, [_p(_vp)]),
    ("pfac_workspace_free", None, [_vp]),
    ("pfac_workspace_reserve", ctypes.c_int, [_vp, _u64, _u32, _u64]),
    ("pfac_workspace_set_timing", ctypes.c_int, [_vp, _vp, _vp]),
    ("pfac_scan", ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _u64, _vp, _vp, _vp]),
    ("pfac_scan_sync", ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _u64, _p(_u64), _vp, _vp]),
    ("pfac_scan_noalloc", ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp, _vp]),
    ("pfac_scan_batch", ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _u64, _vp, _u64, _vp, _vp]),
    ("pfac_scan_batch_plain", ctypes.c_int, [_vp, _vp, _vp, _p(_u64), _u32, _vp, _u64, _vp, _vp]),
    ("pfac_graph_create_batch", ctypes.c_int,
     [_vp, _vp, _vp, _vp, _u32, _u64, _vp, _u64, _vp, _vp, _p(_vp)]),
    ("pfac_graph_launch", ctypes.c_int, [_vp, _vp]),
    ("pfac_graph_set_timing", ctypes.c_int, [_vp, _vp, _vp]),
    ("pfac_graph_free", None, [_vp]),
    ("pfac_autotune", ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _p(pfac_tuning)]),
    ("pfac_autotune_batch", ctypes.c_int,
     [_vp, _vp, _vp, _vp, _u32, _u64, _vp, _p(pfac_tuning)]),
    ("pfac_server_create", ctypes.c_int, [_vp, _vp, _u64, _u64, _u32, _vp, _vp, _p(_vp)]),
    ("pfac_server_submit", ctypes.c_int, [_vp, _vp, _u64, _p(_u64)]),
    ("pfac_server_wait", ctypes.c_int,
     [_vp, _u64, _i64, _vp, _u64, _p(_u64), _p(ctypes.c_double)]),
    ("pfac_server_cancel", ctypes.c_int, [_vp, _u64]),
    ("pfac_server_stats", ctypes.c_int, [_vp, _p(_u64), _p(_u64), _p(_u64), _p(_u64)]),
    ("pfac_server_free", None, [_vp]),
]


def load(path: Optional[str] = None):
    """Load ``libpfac.so``; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
            " (the scanner has no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return load().pfac_strerror(code).decode()
    except Exception:  # library missing: still describe the code
        return str(code)


def check(fn: str, rc: int) -> int:
    if rc != PFAC_OK:
        raise PfacError(fn, rc, load().pfac_last_hip_error())
    return rc


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _dptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return int(t.data_ptr())


def _packed(patterns) -> tuple:
    if hasattr(patterns, "data") and hasattr(patterns, "offsets"):
        data = np.ascontiguousarray(patterns.data, dtype=np.uint8)
        offs = np.ascontiguousarray(patterns.offsets, dtype=np.uint64)
    else:
        pats = [bytes(p) for p in patterns]
        offs = np.zeros(len(pats) + 1, dtype=np.uint64)
        if pats:
            offs[1:] = np.cumsum([len(p) for p in pats])
        data = np.frombuffer(b"".join(pats) or b"\0", dtype=np.uint8).copy()
    if data.size == 0:
        data = np.zeros(1, dtype=np.uint8)
    return data, offs


# ------------------------------------------------------------------ objects


class Trie:
    """A built trie (``pfac_build_packed``) and its device image."""

    def __init__(self, patterns, host_only: bool = False):
        lib = load()
        data, offs = _packed(patterns)
        h = _vp()
        rc = lib.pfac_build_packed(data.ctypes.data, offs.ctypes.data_as(_p(_u64)),
                                   len(offs) - 1, PFAC_BUILD_HOST_ONLY if host_only else 0,
                                   ctypes.byref(h))
        check("pfac_build_packed", rc)
        self.handle = h.value
        self.n_patterns = len(offs) - 1

    def close(self):
        if getattr(self, "handle", None):
            load().pfac_trie_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        s = pfac_stats()
        check("pfac_trie_stats", load().pfac_trie_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def export(self) -> dict:
        st = self.stats()
        N, E, k = int(st["nodes"]), int(st["edges"]), int(st["n_patterns"])
        out = {
            "row_ptr": np.zeros(N + 1, dtype=np.uint32),
            "labels": np.zeros(max(E, 1), dtype=np.uint8),
            "child": np.zeros(max(E, 1), dtype=np.uint32),
            "term_ptr": np.zeros(N + 1, dtype=np.uint32),
            "term_ids": np.zeros(max(k, 1), dtype=np.uint32),
        }
        check("pfac_trie_export", load().pfac_trie_export(
            self.handle, out["row_ptr"].ctypes.data, out["labels"].ctypes.data,
            out["child"].ctypes.data, out["term_ptr"].ctypes.data, out["term_ids"].ctypes.data))
        out["labels"] = out["labels"][:E]
        out["child"] = out["child"][:E]
        out["term_ids"] = out["term_ids"][:k]
        return out

    def tuning(self) -> dict:
        t = pfac_tuning()
        check("pfac_trie_get_tuning", load().pfac_trie_get_tuning(self.handle, ctypes.byref(t)))
        return {n: getattr(t, n) for n, _ in t._fields_}

    def launch_kernel(self, total_bytes: int):
        """(kernel, tuning) of a launch over total_bytes: 0 = tile kernel,
        1 = fused wave kernel, 2 = split filter + walk kernels."""
        k = ctypes.c_uint32()
        t = pfac_tuning()
        check("pfac_trie_launch_kernel", load().pfac_trie_launch_kernel(
            self.handle, int(total_bytes), ctypes.byref(k), ctypes.byref(t)))
        return int(k.value), {n: getattr(t, n) for n, _ in t._fields_}

    def set_tuning(self, **fields):
        """Change the named fields of the launch tuning (pfac_tuning); the
        others keep their current values."""
        cur = self.tuning()
        unknown = set(fields) - set(cur)
        if unknown:
            raise TypeError(f"unknown tuning fields {sorted(unknown)}")
        cur.update(fields)
        t = pfac_tuning(*(int(cur[name]) for name, _ in pfac_tuning._fields_))
        check("pfac_trie_set_tuning", load().pfac_trie_set_tuning(self.handle, ctypes.byref(t)))


class Workspace:
    def __init__(self):
        h = _vp()
        check("pfac_workspace_create", load().pfac_workspace_create(ctypes.byref(h)))
        self.handle = h.value

    def reserve(self, max_bytes: int, max_texts: int, max_matches: int):
        check("pfac_workspace_reserve",
              load().pfac_workspace_reserve(self.handle, max_bytes, max_texts, max_matches))

    def set_timing(self, start_event=None, stop_event=None):
        """Record torch.cuda.Events around the main scan kernel of later scans."""
        s = int(start_event.cuda_event) if start_event is not None else None
        e = int(stop_event.cuda_event) if stop_event is not None else None
        check("pfac_workspace_set_timing", load().pfac_workspace_set_timing(self.handle, s, e))

    def close(self):
        if getattr(self, "handle", None):
            load().pfac_workspace_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ scans


def pfac_scan(trie: Trie, ws: Workspace, text_dev, n: int, out_dev, capacity: int,
              n_matches_dev, counts_dev=None, stream=None) -> int:
    return check("pfac_scan", load().pfac_scan(
        trie.handle, ws.handle, _dptr(text_dev), n, _dptr(out_dev), capacity,
        _dptr(n_matches_dev), _dptr(counts_dev), _stream_ptr(stream)))


def pfac_scan_noalloc(trie: Trie, text_dev, n: int, out_dev, capacity: int, n_matches_dev,
                      counts_dev=None, stream=None) -> int:
    return check("pfac_scan_noalloc", load().pfac_scan_noalloc(
        trie.handle, _dptr(text_dev), n, _dptr(out_dev), capacity, _dptr(n_matches_dev),
        _dptr(counts_dev), _stream_ptr(stream)))


def pfac_scan_sync(trie: Trie, ws: Workspace, text_dev, n: int, out_dev, capacity: int,
                   counts_dev=None, stream=None) -> tuple:
    """Returns (rc, n_matches); rc is PFAC_OK or PFAC_ETRUNC."""
    cnt = _u64(0)
    rc = load().pfac_scan_sync(trie.handle, ws.handle, _dptr(text_dev), n, _dptr(out_dev),
                               capacity, ctypes.byref(cnt), _dptr(counts_dev),
                               _stream_ptr(stream))
    if rc not in (PFAC_OK, PFAC_ETRUNC):
        check("pfac_scan_sync", rc)
    return rc, int(cnt.value)


def pfac_scan_batch(trie: Trie, ws: Workspace, texts_dev, offsets_dev, n_texts: int,
                    total_bytes: int, out_dev, capacity: int, n_matches_dev, stream=None) -> int:
    return check("pfac_scan_batch", load().pfac_scan_batch(
        trie.handle, ws.handle, _dptr(texts_dev), _dptr(offsets_dev), n_texts, total_bytes,
        _dptr(out_dev), capacity, _dptr(n_matches_dev), _stream_ptr(stream)))


def pfac_scan_batch_plain(trie: Trie, ws: Workspace, texts_dev, offsets_host: np.ndarray,
                          n_texts: int, out_dev, capacity: int, n_matches_dev,
                          stream=None) -> int:
    offs = np.ascontiguousarray(offsets_host, dtype=np.uint64)
    return check("pfac_scan_batch_plain", load().pfac_scan_batch_plain(
        trie.handle, ws.handle, _dptr(texts_dev), offs.ctypes.data_as(_p(_u64)), n_texts,
        _dptr(out_dev), capacity, _dptr(n_matches_dev), _stream_ptr(stream)))


class Graph:
    """``pfac_graph_create_batch``: a captured batched scan, replayed by ``launch``."""

    def __init__(self, trie: Trie, ws, texts_dev, offsets_dev, n_texts: int,
                 total_bytes: int, out_dev, capacity: int, n_matches_dev, stream=None):
        """The graph owns its scratch (``ws`` is not used and may be None) and
        pins the trie's device image until it is closed."""
        h = _vp()
        check("pfac_graph_create_batch", load().pfac_graph_create_batch(
            trie.handle, ws.handle if ws is not None else None, _dptr(texts_dev),
            _dptr(offsets_dev), n_texts, total_bytes, _dptr(out_dev), capacity,
            _dptr(n_matches_dev), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h.value
        self._trie = trie  # the trie must outlive the graph

    def launch(self, stream=None):
        check("pfac_graph_launch", load().pfac_graph_launch(self.handle, _stream_ptr(stream)))

    def set_timing(self, start_event, stop_event):
        """Later replays record these events around the main scan kernel (the
        graph must have been captured from a workspace with timing events)."""
        check("pfac_graph_set_timing", load().pfac_graph_set_timing(
            self.handle, int(start_event.cuda_event), int(stop_event.cuda_event)))

    def close(self):
        if getattr(self, "handle", None):
            load().pfac_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pfac_autotune(trie: Trie, ws: Workspace, text_dev, n: int, stream=None) -> dict:
    t = pfac_tuning()
    check("pfac_autotune", load().pfac_autotune(trie.handle, ws.handle, _dptr(text_dev), n,
                                                _stream_ptr(stream), ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in t._fields_}


def pfac_autotune_batch(trie: Trie, ws: Workspace, texts_dev, offsets_dev, n_texts: int,
                        total_bytes: int, stream=None) -> dict:
    t = pfac_tuning()
    check("pfac_autotune_batch", load().pfac_autotune_batch(
        trie.handle, ws.handle, _dptr(texts_dev), _dptr(offsets_dev), n_texts, total_bytes,
        _stream_ptr(stream), ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in t._fields_}


class Server:
    """``pfac_server_*``: continuous-batching scans into a caller-owned device arena."""

    def __init__(self, trie: Trie, arena_dev, budget_bytes: int, max_batch: int,
                 compute_stream, copy_stream):
        h = _vp()
        check("pfac_server_create", load().pfac_server_create(
            trie.handle, _dptr(arena_dev), arena_dev.numel() * arena_dev.element_size(),
            budget_bytes, max_batch, _stream_ptr(compute_stream), _stream_ptr(copy_stream),
            ctypes.byref(h)))
        self.handle = h.value
        self._keep = {}
        # the worker thread uses these until close(): keep them alive
        self._trie, self._arena = trie, arena_dev
        self._streams = (compute_stream, copy_stream)

    def submit(self, text_host: np.ndarray) -> int:
        """Queue a scan of a host uint8 array (kept alive until waited for)."""
        arr = np.ascontiguousarray(text_host, dtype=np.uint8)
        rid = _u64(0)
        check("pfac_server_submit", load().pfac_server_submit(
            self.handle, arr.ctypes.data if arr.size else None, arr.size, ctypes.byref(rid)))
        self._keep[rid.value] = arr
        return rid.value

    def submit_ptr(self, host_ptr: int, n: int, keep=None) -> int:
        rid = _u64(0)
        check("pfac_server_submit", load().pfac_server_submit(self.handle, host_ptr, n,
                                                             ctypes.byref(rid)))
        if keep is not None:
            self._keep[rid.value] = keep
        return rid.value

    def wait(self, request_id: int, capacity: int = 1 << 20, timeout_ms: int = -1):
        """Returns (matches as a structured array, latency seconds)."""
        out = np.zeros(max(capacity, 1), dtype=MATCH_DTYPE)
        n = _u64(0)
        lat = ctypes.c_double(0)
        rc = load().pfac_server_wait(self.handle, request_id, timeout_ms, out.ctypes.data,
                                     capacity, ctypes.byref(n), ctypes.byref(lat))
        if rc != PFAC_EBUSY:  # on a timeout the text is still read
            self._keep.pop(request_id, None)
        if rc == PFAC_ETRUNC:
            raise PfacError("pfac_server_wait", rc)
        check("pfac_server_wait", rc)
        return out[:int(n.value)].copy(), float(lat.value)

    def cancel(self, request_id: int) -> None:
        """Withdraw a request: its text is no longer read and its matches are dropped."""
        check("pfac_server_cancel", load().pfac_server_cancel(self.handle, request_id))
        self._keep.pop(request_id, None)

    def stats(self) -> dict:
        r, b, y, d = _u64(0), _u64(0), _u64(0), _u64(0)
        check("pfac_server_stats", load().pfac_server_stats(
            self.handle, ctypes.byref(r), ctypes.byref(b), ctypes.byref(y), ctypes.byref(d)))
        return {"requests": r.value, "batches": b.value, "bytes": y.value,
                "device_bytes": d.value}

    def close(self):
        if getattr(self, "handle", None):
            load().pfac_server_free(self.handle)
            self.handle = None
        self._keep = {}
        self._trie = self._arena = self._streams = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ conveniences


def matches_to_numpy(out_dev, n: int) -> np.ndarray:
    """Copy the first n records of a device uint8 tensor of pfac_match to the host."""
    import torch
    raw = out_dev.view(torch.uint8)[: n * 16].cpu().numpy()
    return raw.view(MATCH_DTYPE)[:n].copy()


def scan_host(trie: Trie, text: np.ndarray, ws: Optional[Workspace] = None,
              counts: bool = False, capacity: Optional[int] = None):
    """Copy a host text to the device, scan it, grow the output until it fits.

    Returns (matches structured array, counts array or None).
    """
    import torch
    ws = ws or Workspace()
    t = torch.from_numpy(np.ascontiguousarray(text, dtype=np.uint8)).to("cuda")
    n = t.numel()
    cap = capacity if capacity is not None else max(1024, n // 64)
    cdev = torch.empty(max(n, 1), dtype=torch.int32, device="cuda") if counts else None
    while True:
        out = torch.empty(max(cap, 1) * 16, dtype=torch.uint8, device="cuda")
        rc, cnt = pfac_scan_sync(trie, ws, t if n else None, n, out, cap,
                                 cdev[:n] if counts and n else None)
        if rc == PFAC_OK:
            break
        cap = cnt
    m = matches_to_numpy(out, cnt)
    c = cdev[:n].cpu().numpy().view(np.uint32) if counts else None
    return m, c

"""Thin ctypes binding of libhc (include/hc.h).

Argument marshalling only: every step of the searching phase runs in libhc's
HIP kernels. Device buffers are torch tensors (torch provides device memory
and streams); host buffers are bytes / numpy arrays. Each function has the
name of the C entry point it calls. When libhc.so is missing, loading raises:
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhc.so")

HC_OK, HC_EINVAL, HC_ENOMEM, HC_EOVERFLOW, HC_EAGAIN, HC_EHIP = 0, -1, -2, -3, -4, -5
HC_SCHED_AUTO, HC_SCHED_SEGMENT, HC_SCHED_WAVE, HC_SCHED_DENSE = 0, 1, 2, 3
HC_VARIANT_AUTO, HC_VARIANT_HC, HC_VARIANT_SENTINEL, HC_VARIANT_SPARSE = 0, 1, 2, 3

# every symbol declared in include/hc.h
EXPORTED = (
    "hc_preprocess", "hc_pattern_info", "hc_pattern_free", "hc_search", "hc_search_async",
    "hc_search_batched", "hc_batch_plan_create", "hc_batch_plan_run", "hc_batch_plan_free",
    "hc_serve_create", "hc_serve_submit", "hc_serve_poll", "hc_serve_next_done",
    "hc_serve_stats", "hc_serve_destroy", "hc_strerror", "hc_autotune", "hc_autotune_reset",
    "hc_preprocess_many", "hc_search_async_noalloc", "hc_batch_autotune",
)


class HCError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


class hc_params(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("alpha", ctypes.c_int32), ("w", ctypes.c_int32)]


class hc_launch(ctypes.Structure):
    _fields_ = [("segment", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32)]


class hc_tuning(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("params", hc_params), ("launch", hc_launch),
                ("gbps", ctypes.c_double)]


class hc_batch_tuning(ctypes.Structure):
    _fields_ = [("params", hc_params), ("segment", ctypes.c_int32), ("group", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("gbps", ctypes.c_double)]


class hc_batch(ctypes.Structure):
    _fields_ = [
        ("d_text", ctypes.c_void_p), ("text_off", ctypes.c_void_p), ("n_texts", ctypes.c_int32),
        ("pat", ctypes.c_void_p), ("pat_off", ctypes.c_void_p), ("n_pats", ctypes.c_int32),
        ("pair_pat", ctypes.c_void_p), ("pair_text", ctypes.c_void_p), ("n_pairs", ctypes.c_int64),
    ]


_lib = None


def lib():
    """Load libhc.so (built in-tree by __graft_entry__.build()); raises when absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libhc.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, u32, u64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    P = ctypes.POINTER
    sig = {
        "hc_preprocess": (i32, [p, i64, p, P(p)]),
        "hc_pattern_info": (i32, [p, P(hc_params), P(i32), P(u32), P(u32), P(p), P(i64), P(i64)]),
        "hc_pattern_free": (None, [p]),
        "hc_search": (i32, [p, p, i64, p, i64, P(i64), p]),
        "hc_search_async": (i32, [p, p, i64, p, i64, p, p, p]),
        "hc_search_batched": (i32, [P(hc_batch), p, p, i64, p, P(i64), p]),
        "hc_batch_plan_create": (i32, [P(hc_batch), p, P(p)]),
        "hc_batch_plan_run": (i32, [p, p, i64, p, P(i64), p]),
        "hc_batch_plan_free": (None, [p]),
        "hc_serve_create": (i32, [p, p, i32, i64, p, P(p)]),
        "hc_serve_submit": (i32, [p, i32, p, i64, P(u64)]),
        "hc_serve_poll": (i32, [p, u64, p, i64, P(i64), i32]),
        "hc_serve_next_done": (i32, [p, P(u64), i32]),
        "hc_serve_stats": (i32, [p, P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double), P(i64)]),
        "hc_serve_destroy": (i32, [p]),
        "hc_strerror": (ctypes.c_char_p, [i32]),
        "hc_autotune": (i32, [p, i64, P(i64), i32, i32, p, p]),
        "hc_autotune_reset": (None, []),
        "hc_preprocess_many": (i32, [p, p, i32, p, p, i64, p, p, p]),
        "hc_search_async_noalloc": (i32, [p, p, i64, p, i64, p, p, p]),
        "hc_batch_autotune": (i32, [P(hc_batch), i64, P(hc_batch_tuning), p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().hc_strerror(int(status)).decode()


def _check(status: int, what: str, ok=(HC_OK,)):
    if status not in ok:
        raise HCError(status, what)
    return status


def _stream_ptr(stream) -> Optional[int]:
    """hipStream_t of a torch stream (None = torch's current stream); an int is
    taken as a raw stream handle (0 = the default stream)."""
    import torch

    if isinstance(stream, int):
        return stream or None
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


def _params(params) -> Optional[hc_params]:
    if params is None:
        return None
    if isinstance(params, hc_params):
        return params
    q, alpha, w = (tuple(params) + (0, 0, 0))[:3]
    return hc_params(int(q), int(alpha), int(w))


def _launch(launch) -> Optional[hc_launch]:
    if launch is None or isinstance(launch, hc_launch):
        return launch
    if isinstance(launch, dict):
        return hc_launch(int(launch.get("segment", 0)), int(launch.get("schedule", 0)),
                         int(launch.get("variant", 0)), int(launch.get("wg_per_cu", 0)))
    seg, sched, var, wg = (tuple(launch) + (0, 0, 0, 0))[:4]
    return hc_launch(int(seg), int(sched), int(var), int(wg))


def _u8_host(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    a = np.ascontiguousarray(a)
    assert a.dtype == np.uint8
    return a


def _dev_ptr(t, dtype_name: str) -> int:
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device buffers are torch tensors on a GPU")
    if str(t.dtype) != dtype_name or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype_name} tensor")
    return t.data_ptr()


class Pattern:
    """Owner of an hc_pattern handle (hc_preprocess / hc_pattern_free)."""

    def __init__(self, handle: int, m: int):
        self.handle = ctypes.c_void_p(handle)
        self.m = m

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.hc_pattern_free(h)
            self.handle = None


def hc_preprocess(x, params=None) -> Pattern:
    xa = _u8_host(x)
    out = ctypes.c_void_p()
    pr = _params(params)
    st = lib().hc_preprocess(xa.ctypes.data if xa.size else None, int(xa.size),
                             ctypes.byref(pr) if pr is not None else None, ctypes.byref(out))
    _check(st, "hc_preprocess")
    return Pattern(out.value, int(xa.size))


def hc_pattern_info(p: Pattern) -> dict:
    used, s, mask, hv = hc_params(), ctypes.c_int32(), ctypes.c_uint32(), ctypes.c_uint32()
    Fp, Fw, m = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().hc_pattern_info(p.handle, ctypes.byref(used), ctypes.byref(s), ctypes.byref(mask),
                                 ctypes.byref(hv), ctypes.byref(Fp), ctypes.byref(Fw), ctypes.byref(m)),
           "hc_pattern_info")
    F = np.ctypeslib.as_array(ctypes.cast(Fp, ctypes.POINTER(ctypes.c_uint64)), shape=(Fw.value,)).copy()
    return {"q": used.q, "alpha": used.alpha, "w": used.w, "s": s.value, "mask": mask.value,
            "hv": hv.value, "F": F, "m": m.value}


def hc_search(p: Pattern, y, out, stream=None):
    """Returns (status, count); status is HC_OK or HC_EOVERFLOW."""
    cnt = ctypes.c_int64()
    cap = int(out.numel()) if out is not None else 0
    st = lib().hc_search(p.handle, _dev_ptr(y, "torch.uint8") if y.numel() else None, int(y.numel()),
                         _dev_ptr(out, "torch.int64") if cap else None, cap, ctypes.byref(cnt),
                         _stream_ptr(stream))
    _check(st, "hc_search", ok=(HC_OK, HC_EOVERFLOW))
    return st, cnt.value


def hc_search_async(p: Pattern, y, out, d_count, launch=None, stream=None, n=None, y_ptr=None):
    """Stream-ordered search; the total lands in d_count[0] (torch int64)."""
    cap = int(out.numel()) if out is not None else 0
    lc = _launch(launch)
    if y_ptr is None:
        y_ptr = _dev_ptr(y, "torch.uint8") if y.numel() else None
        n = int(y.numel()) if n is None else n
    if out is not None and out.numel() == 0:
        cap = 0
    st = lib().hc_search_async(p.handle, y_ptr, int(n),
                               _dev_ptr(out, "torch.int64") if cap else None, cap,
                               _dev_ptr(d_count, "torch.int64"),
                               ctypes.byref(lc) if lc is not None else None, _stream_ptr(stream))
    return _check(st, "hc_search_async")


def hc_search_async_noalloc(p: Pattern, y, out, d_count, launch=None, stream=None):
    """hc_search_async without allocations (fixed device scratch); returns the
    status (HC_EINVAL when the pattern is not resident on the device yet or
    the text needs more scratch than the fixed array holds)."""
    cap = int(out.numel()) if out is not None else 0
    lc = _launch(launch)
    return lib().hc_search_async_noalloc(p.handle, _dev_ptr(y, "torch.uint8") if y.numel() else None,
                                         int(y.numel()), _dev_ptr(out, "torch.int64") if cap else None, cap,
                                         _dev_ptr(d_count, "torch.int64"),
                                         ctypes.byref(lc) if lc is not None else None, _stream_ptr(stream))


def find_all(p: Pattern, y, cap: int = 1 << 16, stream=None):
    """All occurrences as a torch int64 tensor on y's device (grows cap on overflow)."""
    import torch

    while True:
        out = torch.empty(max(cap, 1), dtype=torch.int64, device=y.device)
        st, cnt = hc_search(p, y, out, stream)
        if st == HC_OK:
            return out[:cnt]
        cap = cnt


def _make_batch(d_text, text_off, patterns, pair_pat, pair_text):
    to = np.ascontiguousarray(text_off, dtype=np.int64)
    pat_bytes = b"".join(patterns)
    po = np.zeros(len(patterns) + 1, dtype=np.int64)
    po[1:] = np.cumsum([len(x) for x in patterns])
    pb = np.frombuffer(pat_bytes, dtype=np.uint8) if pat_bytes else np.zeros(1, np.uint8)
    pp = np.ascontiguousarray(pair_pat, dtype=np.int32)
    pt = np.ascontiguousarray(pair_text, dtype=np.int32)
    b = hc_batch(_dev_ptr(d_text, "torch.uint8") if d_text.numel() else None, to.ctypes.data,
                 len(to) - 1, pb.ctypes.data, po.ctypes.data, len(patterns),
                 pp.ctypes.data, pt.ctypes.data, len(pp))
    return b, (to, po, pb, pp, pt)   # keep the host arrays alive with the struct


def hc_search_batched(d_text, text_off: Sequence[int], patterns: Sequence[bytes],
                      pair_pat, pair_text, d_pos, d_pair_off, params=None, stream=None):
    """Returns (status, total). text_off has n_texts + 1 entries."""
    b, _keep = _make_batch(d_text, text_off, patterns, pair_pat, pair_text)
    total = ctypes.c_int64()
    pr = _params(params)
    cap = int(d_pos.numel()) if d_pos is not None else 0
    st = lib().hc_search_batched(ctypes.byref(b), ctypes.byref(pr) if pr is not None else None,
                                 _dev_ptr(d_pos, "torch.int64") if cap else None, cap,
                                 _dev_ptr(d_pair_off, "torch.int64"), ctypes.byref(total),
                                 _stream_ptr(stream))
    _check(st, "hc_search_batched", ok=(HC_OK, HC_EOVERFLOW))
    return st, total.value


def hc_batch_autotune(d_text, text_off, patterns, pair_pat, pair_text, max_pairs: int = 1 << 20,
                      stream=None) -> dict:
    """Tunes the batched kernel's table shape and launch shape on this batch
    and installs the choice for plans created afterwards with params None."""
    b, _keep = _make_batch(d_text, text_off, patterns, pair_pat, pair_text)
    out = hc_batch_tuning()
    _check(lib().hc_batch_autotune(ctypes.byref(b), int(max_pairs), ctypes.byref(out), _stream_ptr(stream)),
           "hc_batch_autotune")
    return {"alpha": out.params.alpha, "w": out.params.w, "segment": out.segment, "group": out.group,
            "wg_per_cu": out.wg_per_cu, "gbps": out.gbps}


class BatchPlan:
    """hc_batch_plan_create / hc_batch_plan_run / hc_batch_plan_free."""

    def __init__(self, d_text, text_off, patterns, pair_pat, pair_text, params=None):
        self._text = d_text
        b, keep = _make_batch(d_text, text_off, patterns, pair_pat, pair_text)
        out = ctypes.c_void_p()
        pr = _params(params)
        _check(lib().hc_batch_plan_create(ctypes.byref(b), ctypes.byref(pr) if pr is not None else None,
                                          ctypes.byref(out)), "hc_batch_plan_create")
        self.handle = out
        self.n_pairs = len(keep[3])

    def run(self, d_pos, d_pair_off, stream=None):
        """Returns (status, total)."""
        total = ctypes.c_int64()
        cap = int(d_pos.numel()) if d_pos is not None else 0
        st = lib().hc_batch_plan_run(self.handle, _dev_ptr(d_pos, "torch.int64") if cap else None, cap,
                                     _dev_ptr(d_pair_off, "torch.int64"), ctypes.byref(total),
                                     _stream_ptr(stream))
        _check(st, "hc_batch_plan_run", ok=(HC_OK, HC_EOVERFLOW))
        return st, total.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.hc_batch_plan_free(h)
            self.handle = None


class Server:
    """hc_serve_* over resident device texts (torch uint8 tensors)."""

    def __init__(self, texts, device_mem_budget: int, params=None):
        self._texts = list(texts)   # keep the tensors alive
        ptrs = (ctypes.c_void_p * len(texts))(*[_dev_ptr(t, "torch.uint8") for t in texts])
        ns = (ctypes.c_int64 * len(texts))(*[int(t.numel()) for t in texts])
        out = ctypes.c_void_p()
        pr = _params(params)
        _check(lib().hc_serve_create(ptrs, ns, len(texts), int(device_mem_budget),
                                     ctypes.byref(pr) if pr is not None else None, ctypes.byref(out)),
               "hc_serve_create")
        self.handle = out

    def submit(self, text_id: int, x) -> int:
        xa = _u8_host(x)
        rid = ctypes.c_uint64()
        _check(lib().hc_serve_submit(self.handle, int(text_id), xa.ctypes.data, int(xa.size),
                                     ctypes.byref(rid)), "hc_serve_submit")
        return rid.value

    def poll(self, req_id: int, cap: int = 1 << 16, timeout_us: int = 0):
        """None while running; else (status, positions as numpy int64, count).
        HC_EOVERFLOW leaves the request in place (poll again with cap >= count)."""
        out = np.empty(max(cap, 1), dtype=np.int64)
        cnt = ctypes.c_int64()
        st = lib().hc_serve_poll(self.handle, ctypes.c_uint64(req_id), out.ctypes.data, int(cap),
                                 ctypes.byref(cnt), int(timeout_us))
        if st == HC_EAGAIN:
            return None
        _check(st, "hc_serve_poll", ok=(HC_OK, HC_EOVERFLOW))
        return st, out[:min(cnt.value, cap)].copy(), cnt.value

    def result(self, req_id: int, timeout_s: float = 60.0) -> np.ndarray:
        """Waits for a request and returns all of its positions."""
        import time

        end = time.monotonic() + timeout_s
        cap = 1 << 12
        while True:
            r = self.poll(req_id, cap=cap, timeout_us=100_000)
            if r is not None:
                st, pos, cnt = r
                if st == HC_OK:
                    return pos
                cap = cnt   # overflow: the request is kept
                continue
            if time.monotonic() > end:
                raise TimeoutError(f"request {req_id} not done after {timeout_s} s")

    def next_done(self, timeout_us: int = 0):
        """Id of a request that completed and was not reported yet, or None."""
        rid = ctypes.c_uint64()
        st = lib().hc_serve_next_done(self.handle, ctypes.byref(rid), int(timeout_us))
        if st == HC_EAGAIN:
            return None
        _check(st, "hc_serve_next_done")
        return rid.value

    def stats(self) -> dict:
        p50, p99, gbps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        done = ctypes.c_int64()
        _check(lib().hc_serve_stats(self.handle, ctypes.byref(p50), ctypes.byref(p99),
                                    ctypes.byref(gbps), ctypes.byref(done)), "hc_serve_stats")
        return {"p50_us": p50.value, "p99_us": p99.value, "agg_gbps": gbps.value, "done": done.value}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(lib().hc_serve_destroy(self.handle), "hc_serve_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hc_autotune(y_dev, lengths, patterns: int = 5, stream=None) -> list:
    """Tunes q, alpha, w, schedule and segment per pattern length on a device
    text and installs the choices as defaults; returns them as dicts."""
    ms = (ctypes.c_int64 * len(lengths))(*[int(m) for m in lengths])
    out = (hc_tuning * len(lengths))()
    _check(lib().hc_autotune(_dev_ptr(y_dev, "torch.uint8"), int(y_dev.numel()), ms, len(lengths),
                             int(patterns), out, _stream_ptr(stream)), "hc_autotune")
    return [{"m": t.m, "params": (t.params.q, t.params.alpha, t.params.w),
             "launch": (t.launch.segment, t.launch.schedule, t.launch.variant, t.launch.wg_per_cu),
             "gbps": t.gbps} for t in out]


def hc_autotune_reset() -> None:
    lib().hc_autotune_reset()


def hc_preprocess_many(patterns: Sequence[bytes], d_F, table_stride: int, params=None, stream=None):
    """Device preprocessing of many patterns into d_F (torch uint8, n * stride
    bytes). Returns (used params per pattern, (s, mask, hv) per pattern)."""
    n = len(patterns)
    if int(d_F.numel()) < n * int(table_stride):
        raise ValueError("d_F holds fewer than n * table_stride bytes")
    po = np.zeros(n + 1, dtype=np.int64)
    po[1:] = np.cumsum([len(x) for x in patterns])
    pb = np.frombuffer(b"".join(patterns), dtype=np.uint8) if n else np.zeros(1, np.uint8)
    used = (hc_params * max(n, 1))()
    info = np.zeros(3 * max(n, 1), dtype=np.uint32)
    pr = _params(params)
    _check(lib().hc_preprocess_many(pb.ctypes.data, po.ctypes.data, n, ctypes.byref(pr) if pr is not None else None,
                                    _dev_ptr(d_F, "torch.uint8"), int(table_stride), used, info.ctypes.data,
                                    _stream_ptr(stream)), "hc_preprocess_many")
    return ([(u.q, u.alpha, u.w) for u in used[:n]],
            [tuple(int(v) for v in info[3 * i:3 * i + 3]) for i in range(n)])

"""Thin ctypes binding of ``libmemshield.so`` (include/memshield.h).

Every function here only marshals arguments: the cipher, the batching, the
scheduling and the key store all run inside the native library.  The module
fails loudly when the library has not been built; there is no fallback.

Two layers:
  * ``ms_*`` functions with the C names and C argument order (pointers are
    Python ints, status codes are returned as ints);
  * ``Engine`` - a small convenience wrapper that takes torch tensors for
    device buffers and torch streams, and raises ``MemShieldError`` on a
    non-zero status.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
import weakref

import numpy as np

import torch  # loaded first so that the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmemshield.so")

PAGE_SIZE = 4096
KEY_BYTES = 32
NONCE_BYTES = 12

MS_OK = 0
MS_EINVAL = -1
MS_ENOKEY = -2
MS_ENOMEM = -3
MS_EAGAIN = -4
MS_EBUSY = -5
MS_EDEVICE = -6
MS_ECLOSED = -7
MS_ETIMEDOUT = -8
MS_ENOTSUP = -9
MS_ECANCELED = -10

MS_ENCRYPT = 0
MS_DECRYPT = 1
MS_NONCE_ARRAY = 0
MS_NONCE_LINEAR = 1
# ms_host_mode (include/memshield_host.h)
MS_HOST_AUTO = 0
MS_HOST_MAPPED = 1
MS_HOST_DMA = 2
MS_HOST_DMA_IN = 3


class ms_nonce(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tag", ctypes.c_uint32),
                ("array", ctypes.c_void_p), ("base", ctypes.c_uint64),
                ("stride", ctypes.c_uint64)]


class ms_request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("client", ctypes.c_uint32),
                ("key", ctypes.c_uint64), ("src", ctypes.c_void_p),
                ("dst", ctypes.c_void_p), ("n_pages", ctypes.c_uint64),
                ("nonce", ms_nonce), ("priority", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class ms_config(ctypes.Structure):
    _fields_ = [("max_keys", ctypes.c_uint32), ("rounds", ctypes.c_uint32),
                ("queue_depth", ctypes.c_uint32),
                ("max_batch_requests", ctypes.c_uint32),
                ("admission_cap_bytes", ctypes.c_uint64),
                ("inflight_batches", ctypes.c_uint32),
                ("prefetch_depth", ctypes.c_uint32),
                ("validate_pointers", ctypes.c_uint32),
                ("use_graphs", ctypes.c_uint32),
                ("host_chunk_pages", ctypes.c_uint32),
                ("host_stage_slots", ctypes.c_uint32),
                ("host_mapped_waves", ctypes.c_uint32),
                ("serve_spin_us", ctypes.c_uint32),
                ("cipher", ctypes.c_uint32),
                ("serve_stage", ctypes.c_uint32)]


MS_CIPHER_CHACHA = 0
MS_CIPHER_SALSA = 1
MS_SERVE_STAGE_AUTO = 0
MS_SERVE_STAGE_LAUNCH = 1
MS_SERVE_STAGE_RING = 2


class ms_resident_config(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_uint32), ("ring_depth", ctypes.c_uint32),
                ("desc_pages", ctypes.c_uint32),
                ("idle_limit_ms", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 4)]


class ms_tuning(ctypes.Structure):
    _fields_ = [("pages_per_wave", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32),
                ("waves_per_cu", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32),
                ("us_per_launch", ctypes.c_double)]


class ms_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "completed", "rejected_eagain", "batches", "pages",
        "prefetch_issued", "prefetch_dropped", "cancelled", "inflight_bytes",
        "max_inflight_bytes", "max_batch_requests", "max_inflight_batches",
        "ring_direct", "ring_queued", "ring_max_queued", "ring_reap_ns")]


MS_SERVE_BATCHED = 0
MS_SERVE_PLAIN = 1
MS_SERVE_RESIDENT = 2


class ms_serve_trace(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("arrival_s", ctypes.c_void_p),
                ("client", ctypes.c_void_p), ("op", ctypes.c_void_p),
                ("n_pages", ctypes.c_void_p), ("src_page", ctypes.c_void_p),
                ("dst_page", ctypes.c_void_p), ("va", ctypes.c_void_p),
                ("pid", ctypes.c_void_p)]


class ms_serve_result(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "wall_s", "data_gbps", "mean_us", "p50_us", "p90_us", "p99_us",
        "p999_us", "max_us", "late_submit_us_max")] + \
        [(n, ctypes.c_uint64) for n in ("completed", "eagain_retries",
                                        "failed", "first_failed")] + \
        [("first_failed_state", ctypes.c_int64),
         ("submit_call_p50_us", ctypes.c_double),
         ("submit_call_p99_us", ctypes.c_double)]


class ms_launch_info(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 96)] + [
        (n, ctypes.c_uint32) for n in (
            "launches", "grid_blocks", "block_threads", "waves_per_cu",
            "cipher", "rounds", "unroll", "nonce_kind")]


class ms_mlp_shape(ctypes.Structure):
    _fields_ = [("vocab", ctypes.c_int32), ("context", ctypes.c_int32),
                ("embed", ctypes.c_int32), ("hidden", ctypes.c_int32)]


_lib = None
_lib_lock = threading.Lock()

_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32
_I32 = ctypes.c_int32
_SIGS = {
    "ms_config_default": ([ctypes.POINTER(ms_config)], None),
    "ms_status_str": ([_I32], ctypes.c_char_p),
    "ms_init": ([ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ms_config)],
                _I32),
    "ms_shutdown": ([_P], _I32),
    "ms_key_load": ([_P, ctypes.c_char_p, ctypes.POINTER(_U64)], _I32),
    "ms_key_generate": ([_P, ctypes.POINTER(_U64)], _I32),
    "ms_key_destroy": ([_P, _U64], _I32),
    "ms_encrypt_pages": ([_P, _U64, _P, _P, _U64, ctypes.POINTER(ms_nonce), _P],
                         _I32),
    "ms_decrypt_pages": ([_P, _U64, _P, _P, _U64, ctypes.POINTER(ms_nonce), _P],
                         _I32),
    "ms_process_batch": ([_P, ctypes.POINTER(ms_request), ctypes.c_size_t, _P],
                         _I32),
    "ms_plain_launch_info": ([_P, _U64, _I32, ctypes.POINTER(ms_launch_info)],
                             _I32),
    "ms_process_batch_static": ([_P, ctypes.POINTER(ms_request),
                                 ctypes.c_size_t, _P], _I32),
    "ms_submit": ([_P, ctypes.POINTER(ms_request), ctypes.c_size_t,
                   ctypes.POINTER(_U64)], _I32),
    "ms_poll": ([_P, ctypes.POINTER(_U64), ctypes.c_size_t,
                 ctypes.POINTER(_I32), _U64], _I32),
    "ms_prefetch_hint": ([_P, ctypes.POINTER(ms_request), ctypes.c_size_t,
                          ctypes.POINTER(_U64)], _I32),
    "ms_cancel_client": ([_P, _U32, ctypes.POINTER(_U64)], _I32),
    "ms_drain": ([_P, _U64], _I32),
    "ms_autotune": ([_P, _U64, ctypes.POINTER(ms_tuning)], _I32),
    "ms_get_tuning": ([_P, _U64, ctypes.POINTER(ms_tuning)], _I32),
    "ms_set_tuning": ([_P, ctypes.POINTER(ms_tuning)], _I32),
    "ms_get_stats": ([_P, ctypes.POINTER(ms_stats)], _I32),
    "ms_debug_staging_is_zero": ([_P], ctypes.c_int),
    "ms_probe_copy": ([_P, _P, _P, _U64, _U32, _P], _I32),
    "ms_probe_valu": ([_P, _P, _U32, _U32, _P, ctypes.POINTER(_U64)], _I32),
    "ms_device_cu_count": ([_P], ctypes.c_int),
    "ms_probe_link": ([_P, _P, _P, _U64, _I32, _P], _I32),
    "ms_resident_config_default": ([ctypes.POINTER(ms_resident_config)],
                                   None),
    "ms_resident_start": ([_P, ctypes.POINTER(ms_resident_config),
                           ctypes.c_char_p, ctypes.POINTER(_P)], _I32),
    "ms_resident_start_keys": ([_P, ctypes.POINTER(ms_resident_config),
                                ctypes.POINTER(_U64), _U32,
                                ctypes.POINTER(_P)], _I32),
    "ms_resident_submit": ([_P, _P, _P, _U64, ctypes.POINTER(ms_nonce),
                            ctypes.POINTER(_U64)], _I32),
    "ms_resident_submit_keyed": ([_P, _U32, _P, _P, _U64,
                                  ctypes.POINTER(ms_nonce),
                                  ctypes.POINTER(_U64)], _I32),
    "ms_resident_poll": ([_P, ctypes.POINTER(_U64), ctypes.c_size_t,
                          ctypes.POINTER(_I32), _U64], _I32),
    "ms_resident_alive": ([_P], ctypes.c_int),
    "ms_resident_stop": ([_P], _I32),
    "ms_resident_debug_key_wiped": ([_P], ctypes.c_int),
    "ms_host_alloc": ([_P, _U64, ctypes.POINTER(_P)], _I32),
    "ms_host_free": ([_P, _P], _I32),
    "ms_encrypt_host_pages": ([_P, _U64, _P, _P, _U64,
                               ctypes.POINTER(ms_nonce), _I32, _P], _I32),
    "ms_decrypt_host_pages": ([_P, _U64, _P, _P, _U64,
                               ctypes.POINTER(ms_nonce), _I32, _P], _I32),
    "ms_mlp_offsets": ([ctypes.POINTER(ms_mlp_shape), ctypes.POINTER(_U64)],
                       _U64),
    "ms_mlp_workspace_bytes": ([ctypes.POINTER(ms_mlp_shape), _I32], _U64),
    "ms_mlp_forward": ([ctypes.POINTER(ms_mlp_shape), _P, _P, _I32, _P, _P,
                        _U64, _P], _I32),
    "ms_mlp_backward": ([ctypes.POINTER(ms_mlp_shape), _P, _P, _P, _I32, _P,
                         _P, _P, _U64, _P], _I32),
    "ms_mlp_adam": ([ctypes.POINTER(ms_mlp_shape), _P, _P, _P, _P, _P,
                     ctypes.c_float, ctypes.c_float, ctypes.c_float,
                     ctypes.c_float, _I32, _P], _I32),
    "ms_mlp_to_bf16": ([_P, _P, _U64, _P], _I32),
    "ms_mlp_topk": ([_P, _I32, _I32, _I32, _I32, _P, _P, _P], _I32),
    "ms_serve_run": ([_P, ctypes.POINTER(ms_serve_trace),
                      ctypes.POINTER(_U64), _U32, _P, _U64, _P, _U64, _I32,
                      _U32, _P, ctypes.POINTER(ms_serve_result)], _I32),
}


def load_library(path: str | None = None):
    """Load the native library (once).  Raises if it is not built."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(
                "libmemshield.so is not built (%s); run "
                "`python -m paper_2004_09252_amd.build`" % p)
        lib = ctypes.CDLL(p)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def exported_symbols() -> list:
    return list(_SIGS)


def _L():
    return _lib if _lib is not None else load_library()


# ---- C-named functions (argument marshalling only) ----

def ms_config_default() -> ms_config:
    c = ms_config()
    _L().ms_config_default(ctypes.byref(c))
    return c


def ms_status_str(st: int) -> str:
    return _L().ms_status_str(st).decode()


def ms_init(device: int = 0, config: ms_config | None = None):
    ctx = ctypes.c_void_p()
    st = _L().ms_init(ctypes.byref(ctx), device,
                      ctypes.byref(config) if config is not None else None)
    return st, ctx


def ms_shutdown(ctx) -> int:
    return _L().ms_shutdown(ctx)


def ms_key_load(ctx, key: bytes):
    h = ctypes.c_uint64()
    st = _L().ms_key_load(ctx, bytes(key), ctypes.byref(h))
    return st, h.value


def ms_key_generate(ctx):
    h = ctypes.c_uint64()
    st = _L().ms_key_generate(ctx, ctypes.byref(h))
    return st, h.value


def ms_key_destroy(ctx, key: int) -> int:
    return _L().ms_key_destroy(ctx, key)


def ms_encrypt_pages(ctx, key, src, dst, n_pages, nonce: ms_nonce,
                     stream=None) -> int:
    return _L().ms_encrypt_pages(ctx, key, src, dst, n_pages,
                                 ctypes.byref(nonce), stream)


def ms_decrypt_pages(ctx, key, src, dst, n_pages, nonce: ms_nonce,
                     stream=None) -> int:
    return _L().ms_decrypt_pages(ctx, key, src, dst, n_pages,
                                 ctypes.byref(nonce), stream)


def _req_array(reqs):
    if isinstance(reqs, ctypes.Array):
        return reqs, len(reqs)
    arr = (ms_request * len(reqs))(*reqs)
    return arr, len(reqs)


def ms_plain_launch_info(ctx, n_pages: int, nonce_kind: int):
    info = ms_launch_info()
    st = _L().ms_plain_launch_info(ctx, n_pages, nonce_kind,
                                   ctypes.byref(info))
    return st, info


def ms_process_batch(ctx, reqs, stream=None) -> int:
    arr, n = _req_array(reqs)
    return _L().ms_process_batch(ctx, arr, n, stream)


MS_STATIC_BATCH_MAX_REQUESTS = 4096


def ms_process_batch_static(ctx, reqs, stream=None) -> int:
    arr, n = _req_array(reqs)
    return _L().ms_process_batch_static(ctx, arr, n, stream)


def ms_submit(ctx, reqs):
    arr, n = _req_array(reqs)
    t = (ctypes.c_uint64 * max(n, 1))()
    st = _L().ms_submit(ctx, arr, n, t)
    return st, list(t)[:n]


def ms_poll(ctx, tickets, timeout_ns: int = 0):
    n = len(tickets)
    t = (ctypes.c_uint64 * max(n, 1))(*tickets)
    d = (ctypes.c_int32 * max(n, 1))()
    st = _L().ms_poll(ctx, t, n, d, timeout_ns)
    return st, list(d)[:n]


def ms_prefetch_hint(ctx, reqs):
    arr, n = _req_array(reqs)
    t = (ctypes.c_uint64 * max(n, 1))()
    st = _L().ms_prefetch_hint(ctx, arr, n, t)
    return st, list(t)[:n]


def ms_cancel_client(ctx, client: int):
    n = ctypes.c_uint64()
    st = _L().ms_cancel_client(ctx, client, ctypes.byref(n))
    return st, n.value


def ms_drain(ctx, timeout_ns: int = 60 * 10**9) -> int:
    return _L().ms_drain(ctx, timeout_ns)


def ms_autotune(ctx, n_pages: int):
    t = ms_tuning()
    st = _L().ms_autotune(ctx, n_pages, ctypes.byref(t))
    return st, t


def ms_get_tuning(ctx, n_pages: int):
    t = ms_tuning()
    st = _L().ms_get_tuning(ctx, n_pages, ctypes.byref(t))
    return st, t


def ms_set_tuning(ctx, tuning: ms_tuning | None) -> int:
    return _L().ms_set_tuning(ctx, ctypes.byref(tuning)
                              if tuning is not None else None)


def ms_get_stats(ctx):
    s = ms_stats()
    st = _L().ms_get_stats(ctx, ctypes.byref(s))
    return st, s


def ms_debug_staging_is_zero(ctx) -> int:
    return _L().ms_debug_staging_is_zero(ctx)


def ms_probe_copy(ctx, src, dst, nbytes, grid_blocks=0, stream=None) -> int:
    return _L().ms_probe_copy(ctx, src, dst, nbytes, grid_blocks, stream)


def ms_probe_valu(ctx, out, iters, grid_blocks=0, stream=None):
    ops = ctypes.c_uint64()
    st = _L().ms_probe_valu(ctx, out, iters, grid_blocks, stream,
                            ctypes.byref(ops))
    return st, ops.value


def ms_device_cu_count(ctx) -> int:
    return _L().ms_device_cu_count(ctx)


def ms_probe_link(ctx, src, dst, nbytes, engine, stream=None) -> int:
    return _L().ms_probe_link(ctx, src, dst, nbytes, engine, stream)


def ms_resident_config_default() -> ms_resident_config:
    c = ms_resident_config()
    _L().ms_resident_config_default(ctypes.byref(c))
    return c


def ms_resident_start(ctx, config: ms_resident_config | None = None,
                      key: bytes | None = None):
    r = ctypes.c_void_p()
    st = _L().ms_resident_start(ctx, ctypes.byref(config)
                                if config is not None else None,
                                bytes(key) if key is not None else None,
                                ctypes.byref(r))
    return st, r.value


def ms_resident_start_keys(ctx, config: ms_resident_config | None, keys):
    r = ctypes.c_void_p()
    k = (_U64 * max(len(keys), 1))(*keys)
    st = _L().ms_resident_start_keys(ctx, ctypes.byref(config)
                                     if config is not None else None,
                                     k, len(keys), ctypes.byref(r))
    return st, r.value


def ms_resident_submit(r, src, dst, n_pages, nonce: ms_nonce):
    t = ctypes.c_uint64()
    st = _L().ms_resident_submit(r, src, dst, n_pages, ctypes.byref(nonce),
                                 ctypes.byref(t))
    return st, t.value


def ms_resident_submit_keyed(r, key_index, src, dst, n_pages,
                             nonce: ms_nonce):
    t = ctypes.c_uint64()
    st = _L().ms_resident_submit_keyed(r, key_index, src, dst, n_pages,
                                       ctypes.byref(nonce), ctypes.byref(t))
    return st, t.value


def ms_resident_poll(r, tickets, timeout_ns: int = 0):
    n = len(tickets)
    t = (ctypes.c_uint64 * max(n, 1))(*tickets)
    d = (ctypes.c_int32 * max(n, 1))()
    st = _L().ms_resident_poll(r, t, n, d, timeout_ns)
    return st, list(d)[:n]


def ms_resident_alive(r) -> int:
    return _L().ms_resident_alive(r)


def ms_resident_stop(r) -> int:
    return _L().ms_resident_stop(r)


def ms_resident_debug_key_wiped(r) -> int:
    return _L().ms_resident_debug_key_wiped(r)


def ms_host_alloc(ctx, nbytes: int):
    p = ctypes.c_void_p()
    st = _L().ms_host_alloc(ctx, nbytes, ctypes.byref(p))
    return st, p.value


def ms_host_free(ctx, ptr) -> int:
    return _L().ms_host_free(ctx, ptr)


def ms_encrypt_host_pages(ctx, key, src, dst, n_pages, nonce: ms_nonce,
                          mode=MS_HOST_AUTO, stream=None) -> int:
    return _L().ms_encrypt_host_pages(ctx, key, src, dst, n_pages,
                                      ctypes.byref(nonce), mode, stream)


def ms_decrypt_host_pages(ctx, key, src, dst, n_pages, nonce: ms_nonce,
                          mode=MS_HOST_AUTO, stream=None) -> int:
    return _L().ms_decrypt_host_pages(ctx, key, src, dst, n_pages,
                                      ctypes.byref(nonce), mode, stream)


def ms_serve_run(ctx, trace: ms_serve_trace, keys, src_pool, src_pages,
                 dst_pool, dst_pages, mode, submit_threads, latency_out=None):
    """latency_out: optional float64 numpy array of trace.n entries."""
    k = (ctypes.c_uint64 * max(len(keys), 1))(*keys)
    res = ms_serve_result()
    lat = latency_out.ctypes.data if latency_out is not None else None
    st = _L().ms_serve_run(ctx, ctypes.byref(trace), k, len(keys), src_pool,
                           src_pages, dst_pool, dst_pages, mode,
                           submit_threads, lat, ctypes.byref(res))
    return st, res


def ms_mlp_offsets(shape: ms_mlp_shape):
    off = (ctypes.c_uint64 * 7)()
    total = _L().ms_mlp_offsets(ctypes.byref(shape), off)
    return total, list(off)


def ms_mlp_workspace_bytes(shape: ms_mlp_shape, max_batch: int) -> int:
    return _L().ms_mlp_workspace_bytes(ctypes.byref(shape), max_batch)


def ms_mlp_forward(shape, params, ids, batch, logits, ws, ws_bytes,
                   stream=None) -> int:
    return _L().ms_mlp_forward(ctypes.byref(shape), params, ids, batch, logits,
                               ws, ws_bytes, stream)


def ms_mlp_backward(shape, params, ids, targets, batch, grads, loss, ws,
                    ws_bytes, stream=None) -> int:
    return _L().ms_mlp_backward(ctypes.byref(shape), params, ids, targets,
                                batch, grads, loss, ws, ws_bytes, stream)


def ms_mlp_adam(shape, master, m, v, grads, params, lr, beta1, beta2, eps,
                step, stream=None) -> int:
    return _L().ms_mlp_adam(ctypes.byref(shape), master, m, v, grads, params,
                            lr, beta1, beta2, eps, step, stream)


def ms_mlp_to_bf16(src, dst, n, stream=None) -> int:
    return _L().ms_mlp_to_bf16(src, dst, n, stream)


def ms_mlp_topk(logits, batch, vocab, k, exclude, out_ids, out_prob=None,
                stream=None) -> int:
    return _L().ms_mlp_topk(logits, batch, vocab, k, exclude, out_ids,
                            out_prob, stream)


# ---- convenience wrapper over torch tensors ----

class MemShieldError(RuntimeError):
    def __init__(self, st: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, ms_status_str(st), st))
        self.status = st


def _check(st: int, what: str):
    if st != MS_OK:
        raise MemShieldError(st, what)


def linear_nonce(base: int, stride: int, tag: int) -> ms_nonce:
    return ms_nonce(MS_NONCE_LINEAR, tag & 0xFFFFFFFF, None,
                    base % (1 << 64), stride % (1 << 64))


def array_nonce(t: torch.Tensor) -> ms_nonce:
    n = ms_nonce(MS_NONCE_ARRAY, 0, t.data_ptr(), 0, 0)
    n._keep = t   # the tensor outlives the nonce that points into it
    return n


def _stream_handle(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def request(key: int, src: torch.Tensor, dst: torch.Tensor, n_pages: int,
            nonce: ms_nonce, op: int = MS_ENCRYPT, client: int = 0,
            src_offset_pages: int = 0, dst_offset_pages: int = 0) -> ms_request:
    """A request over tensors; it holds them (and the nonce, which may hold
    an array tensor), so that an Engine can keep them alive while the
    request is in flight."""
    r = ms_request(op, client, key,
                   src.data_ptr() + src_offset_pages * PAGE_SIZE,
                   dst.data_ptr() + dst_offset_pages * PAGE_SIZE,
                   n_pages, nonce, 0, 0)
    r._keep = (src, dst, nonce)
    return r


def _hold(pending: dict, tickets, keeps) -> None:
    """Remember what each submitted ticket's buffers are (see _release)."""
    for t, k in zip(tickets, keeps):
        if t and k is not None:
            pending[t] = k


def _release(pending: dict, tickets, done) -> None:
    """Forget the buffers of tickets that poll reported finished."""
    if pending:
        for t, d in zip(tickets, done):
            if d != 0:
                pending.pop(t, None)


class HostBuffer:
    """Pinned, GPU-mapped host memory from ms_host_alloc; ``array`` is a
    numpy uint8 view of it.  Freed (after being zeroed) by ``free`` or when
    the owning engine closes."""

    def __init__(self, engine, ptr: int, nbytes: int):
        self.engine, self.ptr, self.nbytes = engine, ptr, nbytes
        self.array = np.ctypeslib.as_array(
            (ctypes.c_uint8 * nbytes).from_address(ptr))

    def data_ptr(self) -> int:
        return self.ptr

    def free(self):
        if self.ptr and self.engine.ctx:
            self.array = None
            _check(ms_host_free(self.engine.ctx, self.ptr), "ms_host_free")
        self.array = None
        self.ptr = 0

    def _invalidate(self):
        # the engine's shutdown freed (and zeroed) the memory
        self.array = None
        self.ptr = 0


def _addr(buf) -> int:
    return buf.data_ptr()


def _nbytes(buf) -> int:
    return buf.nbytes if isinstance(buf, HostBuffer) else \
        buf.numel() * buf.element_size()


class Resident:
    """A resident-key engine (include/memshield_resident.h) of an Engine.
    Pages are HostBuffers (pinned, coherent host memory) or device tensors;
    nonces are linear or an array; `key_index` picks one of the engine's
    keys."""

    def __init__(self, engine, handle: int):
        self.engine, self.handle = engine, handle
        # ticket -> the buffers it reads and writes, held until poll reports
        # it finished (or stop): the caching allocator must not hand them to
        # another tensor while the kernel still uses them
        self._pending = {}

    def submit(self, src, dst, nonce, n_pages=None, key_index=0) -> int:
        if n_pages is None:
            n_pages = _nbytes(src) // PAGE_SIZE
        st, t = ms_resident_submit_keyed(self.handle, key_index, _addr(src),
                                         _addr(dst), n_pages, nonce)
        _check(st, "ms_resident_submit_keyed")
        _hold(self._pending, [t], [(src, dst, nonce)])
        return t

    def poll(self, tickets, timeout_s: float = 0.0):
        st, done = ms_resident_poll(self.handle, tickets, int(timeout_s * 1e9))
        if st == MS_OK or st == MS_ETIMEDOUT:
            _release(self._pending, tickets, done)
        return st, done

    def wait(self, tickets, timeout_s: float = 30.0):
        st, done = self.poll(tickets, timeout_s)
        _check(st, "ms_resident_poll")
        if any(d != 1 for d in done):
            raise MemShieldError(MS_ECANCELED, "ms_resident_poll")

    def alive(self) -> bool:
        return bool(self.handle) and ms_resident_alive(self.handle) == 1

    def key_wiped(self) -> int:
        return ms_resident_debug_key_wiped(self.handle)

    def stop(self):
        if self.handle:
            st = MS_OK
            if self.engine.ctx:
                st = ms_resident_stop(self.handle)
            self.handle = 0
            if st != MS_OK:
                # the kernel did not stop, and the library keeps every buffer
                # it could still touch: keep the tensors alive with them
                _never_freed.append(self._pending)
            self._pending = {}
            if self in self.engine._residents:
                self.engine._residents.remove(self)
            _check(st, "ms_resident_stop")


# tensors of engines whose kernel would not stop (kept for the process)
_never_freed = []

_live_engines = weakref.WeakSet()


@atexit.register
def _close_live_engines():
    # a resident-key kernel must not outlive its process's last Python frame
    for e in list(_live_engines):
        try:
            e.close()
        except Exception:
            pass


class Engine:
    """One engine context on a GPU; buffers are torch uint8 tensors."""

    def __init__(self, device: int = 0, **config):
        cfg = ms_config_default()
        for k, v in config.items():
            if not hasattr(cfg, k):
                raise TypeError("unknown config field %r" % k)
            setattr(cfg, k, v)
        self.device = device
        self._pending = {}   # ticket -> buffers held while it is in flight
        self._residents = []
        self._host_buffers = weakref.WeakSet()
        st, self.ctx = ms_init(device, cfg)
        _check(st, "ms_init")
        _live_engines.add(self)

    def close(self):
        if self.ctx:
            for r in list(self._residents):
                r.stop()
            ms_shutdown(self.ctx)   # drains: nothing is in flight after it
            self.ctx = None
            self._pending.clear()
            for b in list(self._host_buffers):
                b._invalidate()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def key_load(self, key: bytes) -> int:
        st, h = ms_key_load(self.ctx, key)
        _check(st, "ms_key_load")
        return h

    def key_generate(self) -> int:
        st, h = ms_key_generate(self.ctx)
        _check(st, "ms_key_generate")
        return h

    def key_destroy(self, h: int):
        _check(ms_key_destroy(self.ctx, h), "ms_key_destroy")

    def _pages(self, fn, name, key, src, dst, nonce, n_pages, stream):
        if n_pages is None:
            n_pages = src.numel() // PAGE_SIZE
        _check(fn(self.ctx, key, src.data_ptr(), dst.data_ptr(), n_pages,
                  nonce, _stream_handle(stream)), name)

    def encrypt_pages(self, key, src, dst, nonce, n_pages=None, stream=None):
        self._pages(ms_encrypt_pages, "ms_encrypt_pages", key, src, dst, nonce,
                    n_pages, stream)

    def decrypt_pages(self, key, src, dst, nonce, n_pages=None, stream=None):
        self._pages(ms_decrypt_pages, "ms_decrypt_pages", key, src, dst, nonce,
                    n_pages, stream)

    def resident(self, key: bytes | None = None, keys=None,
                 **config) -> Resident:
        """Start a resident-key engine with one key (`key` bytes, or a fresh
        random key) or with `keys`, a list of this engine's key handles."""
        cfg = ms_resident_config_default()
        for k, v in config.items():
            if not hasattr(cfg, k):
                raise TypeError("unknown resident config field %r" % k)
            setattr(cfg, k, v)
        if keys is not None:
            if key is not None:
                raise TypeError("give key bytes or key handles, not both")
            st, h = ms_resident_start_keys(self.ctx, cfg, list(keys))
            _check(st, "ms_resident_start_keys")
        else:
            st, h = ms_resident_start(self.ctx, cfg, key)
            _check(st, "ms_resident_start")
        r = Resident(self, h)
        self._residents.append(r)
        return r

    def host_alloc(self, nbytes: int) -> HostBuffer:
        st, p = ms_host_alloc(self.ctx, nbytes)
        _check(st, "ms_host_alloc")
        b = HostBuffer(self, p, nbytes)
        self._host_buffers.add(b)
        return b

    def _host_pages(self, fn, name, key, src, dst, nonce, n_pages, mode,
                    stream):
        if n_pages is None:
            n_pages = _nbytes(src) // PAGE_SIZE
        _check(fn(self.ctx, key, _addr(src), _addr(dst), n_pages, nonce, mode,
                  _stream_handle(stream)), name)

    def encrypt_host_pages(self, key, src, dst, nonce, n_pages=None,
                           mode=MS_HOST_AUTO, stream=None):
        """src/dst: HostBuffer, pinned CPU tensor or CUDA tensor."""
        self._host_pages(ms_encrypt_host_pages, "ms_encrypt_host_pages", key,
                         src, dst, nonce, n_pages, mode, stream)

    def decrypt_host_pages(self, key, src, dst, nonce, n_pages=None,
                           mode=MS_HOST_AUTO, stream=None):
        self._host_pages(ms_decrypt_host_pages, "ms_decrypt_host_pages", key,
                         src, dst, nonce, n_pages, mode, stream)

    def process_batch(self, reqs, stream=None):
        _check(ms_process_batch(self.ctx, reqs, _stream_handle(stream)),
               "ms_process_batch")

    def process_batch_static(self, reqs, stream=None):
        """ms_process_batch without any allocation (descriptors in the
        library's fixed device array); at most MS_STATIC_BATCH_MAX_REQUESTS
        requests, and calls must not overlap on the device."""
        _check(ms_process_batch_static(self.ctx, reqs,
                                       _stream_handle(stream)),
               "ms_process_batch_static")

    def submit(self, reqs) -> list:
        """Queue requests; those built by `request` keep their tensors alive
        until poll reports them finished, or drain or close."""
        st, t = ms_submit(self.ctx, reqs)
        _check(st, "ms_submit")
        _hold(self._pending, t, [getattr(r, "_keep", None) for r in reqs])
        return t

    def poll(self, tickets, timeout_s: float = 0.0):
        st, done = ms_poll(self.ctx, tickets, int(timeout_s * 1e9))
        if st == MS_OK or st == MS_ETIMEDOUT:
            _release(self._pending, tickets, done)
        return st, done

    def prefetch_hint(self, reqs) -> list:
        st, t = ms_prefetch_hint(self.ctx, reqs)
        _check(st, "ms_prefetch_hint")
        _hold(self._pending, t, [getattr(r, "_keep", None) for r in reqs])
        return t

    def drain(self, timeout_s: float = 60.0):
        _check(ms_drain(self.ctx, int(timeout_s * 1e9)), "ms_drain")
        self._pending.clear()

    def autotune(self, n_pages: int) -> ms_tuning:
        st, t = ms_autotune(self.ctx, n_pages)
        _check(st, "ms_autotune")
        return t

    def stats(self) -> ms_stats:
        st, s = ms_get_stats(self.ctx)
        _check(st, "ms_get_stats")
        return s

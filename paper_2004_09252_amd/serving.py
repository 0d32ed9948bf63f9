"""Serving workload driver: device pools, trace layout, and runs of the native
load generator (``ms_serve_run``) in continuous-batching and plain modes.

The work itself (admission, batching, cipher, completion tracking and the
timing of every request) happens in the native library; this module only
lays out buffers and arrays and reduces the results.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import memshield as ms
from . import workloads

PAGE = 4096


def fill_pool(t: torch.Tensor, seed: int, chunk_pages: int = 65536) -> None:
    """Fill a device uint8 tensor with seeded uniform bytes, chunk by chunk
    (numpy PCG64 on the host, then copied)."""
    rng = np.random.default_rng(seed)
    n = t.numel()
    step = chunk_pages * PAGE
    for off in range(0, n, step):
        m = min(step, n - off)
        host = np.frombuffer(rng.bytes(m), dtype=np.uint8)
        t[off:off + m].copy_(torch.from_numpy(host.copy()))


@dataclasses.dataclass
class Layout:
    trace: ms.ms_serve_trace
    arrays: dict          # keeps the numpy arrays alive
    dst_pages: int        # size of the destination buffer in pages
    sample: np.ndarray    # indices of requests with dedicated output slots


def layout(w: workloads.Serving, ring_pages: int, sample_every: int = 100,
           limit: int | None = None) -> Layout:
    """Requests write into a ring of `ring_pages` output pages, except every
    `sample_every`-th request, which gets its own slot after the ring so its
    output survives the run for checking."""
    n = w.arrival_s.size if limit is None else min(limit, w.arrival_s.size)
    pages = w.n_pages[:n].astype(np.uint64)
    dst = np.empty(n, dtype=np.uint64)
    sample = np.arange(0, n, sample_every) if sample_every else \
        np.zeros(0, np.int64)
    is_sample = np.zeros(n, bool)
    is_sample[sample] = True
    cur = 0
    extra = ring_pages
    for i in range(n):
        p = int(pages[i])
        if is_sample[i]:
            dst[i] = extra
            extra += p
            continue
        if cur + p > ring_pages:
            cur = 0
        dst[i] = cur
        cur += p
    arrays = {
        "arrival_s": np.ascontiguousarray(w.arrival_s[:n], dtype=np.float64),
        "client": np.ascontiguousarray(w.clients[:n], dtype=np.uint32),
        "op": np.ascontiguousarray(w.ops[:n], dtype=np.int32),
        "n_pages": np.ascontiguousarray(pages),
        "src_page": np.ascontiguousarray(w.src_page[:n], dtype=np.uint64),
        "dst_page": dst,
        "va": np.ascontiguousarray(w.va[:n], dtype=np.uint64),
        "pid": np.ascontiguousarray(w.pid[:n], dtype=np.uint32),
    }
    tr = ms.ms_serve_trace(n, *(arrays[k].ctypes.data for k in (
        "arrival_s", "client", "op", "n_pages", "src_page", "dst_page", "va",
        "pid")))
    return Layout(tr, arrays, int(extra), sample)


def run(eng: ms.Engine, lay: Layout, keys, src: torch.Tensor,
        dst: torch.Tensor, mode: int, submit_threads: int = 4):
    """Run the trace; returns (result struct, latencies in us)."""
    n = lay.trace.n
    lat = np.zeros(n, dtype=np.float64)
    torch.cuda.synchronize()   # the engine's streams do not wait for torch
    st, res = ms.ms_serve_run(eng.ctx, lay.trace, keys, src.data_ptr(),
                              src.numel() // PAGE, dst.data_ptr(),
                              dst.numel() // PAGE, mode, submit_threads, lat)
    if st != ms.MS_OK:
        raise ms.MemShieldError(st, "ms_serve_run")
    return res, lat


def summarize(res) -> dict:
    return {"GBps": round(res.data_gbps, 3),
            "p50_us": round(res.p50_us, 1), "p90_us": round(res.p90_us, 1),
            "p99_us": round(res.p99_us, 1), "p999_us": round(res.p999_us, 1),
            "max_us": round(res.max_us, 1), "mean_us": round(res.mean_us, 1),
            "requests": int(res.completed), "wall_s": round(res.wall_s, 3),
            "eagain_retries": int(res.eagain_retries),
            "failed": int(res.failed),
            "late_submit_us_max": round(res.late_submit_us_max, 1),
            "submit_call_p50_us": round(res.submit_call_p50_us, 2),
            "submit_call_p99_us": round(res.submit_call_p99_us, 2)}


def sampled_outputs(lay: Layout, src: torch.Tensor, dst: torch.Tensor):
    """Yield (index, input bytes, output bytes) of the sampled requests."""
    a = lay.arrays
    for i in lay.sample:
        p = int(a["n_pages"][i])
        s0 = int(a["src_page"][i]) * PAGE
        d0 = int(a["dst_page"][i]) * PAGE
        yield (int(i), src[s0:s0 + p * PAGE].cpu().numpy(),
               dst[d0:d0 + p * PAGE].cpu().numpy())

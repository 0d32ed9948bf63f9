"""Seeded synthetic inputs for the page-cipher workloads.

This module only draws random numbers and lays them out; it holds none of
the cipher's arithmetic, so the engine's tests and the CPU oracle can both
take their inputs from here.  Everything is drawn from numpy's PCG64
(``default_rng(seed)``), so a workload is a pure function of its seed.

Workloads (sizes follow the paper's unit of work, one 4096-byte page,
section 4.4, and the page counts of the engine's benchmark configurations):
  * ``tiny``    - 64 random pages, one key, 64 distinct random nonces;
  * ``bulk``    - 262144 random pages (1 GiB), one key, nonce of page i =
                  LE64(i) || LE32(0) (a linear run: base 0, stride 1, tag 0);
  * ``batched`` - 512 requests from 32 clients, each client its own key, page
                  counts log-uniform in [1, 4096], encrypt/decrypt 50/50,
                  nonces from the page's virtual address and the client PID;
  * ``serving`` - Poisson arrivals, sizes log-uniform in [1, 256] pages.
"""
from __future__ import annotations

import dataclasses

import numpy as np

PAGE = 4096
VA_BASE = 0x7F0000000000


def random_pages(rng: np.random.Generator, n_pages: int) -> np.ndarray:
    """(n_pages, 4096) uniform uint8."""
    return rng.integers(0, 256, size=(n_pages, PAGE), dtype=np.uint8)


def random_key(rng: np.random.Generator) -> bytes:
    return rng.bytes(32)


@dataclasses.dataclass
class Tiny:
    key: bytes
    nonces: np.ndarray      # (64, 12) uint8, all distinct
    data: np.ndarray        # (64, 4096) uint8


def tiny(seed: int = 1, n_pages: int = 64) -> Tiny:
    rng = np.random.default_rng(seed)
    key = random_key(rng)
    nonces = np.frombuffer(b"".join(rng.bytes(12) for _ in range(n_pages)),
                           dtype=np.uint8).reshape(n_pages, 12).copy()
    assert len({bytes(r) for r in nonces}) == n_pages, "nonces must differ"
    data = random_pages(rng, n_pages)
    return Tiny(key, nonces, data)


@dataclasses.dataclass
class Bulk:
    key: bytes
    data: np.ndarray        # (n_pages, 4096) uint8
    nonce_base: int = 0
    nonce_stride: int = 1
    nonce_tag: int = 0


def bulk(seed: int = 2, n_pages: int = 262144) -> Bulk:
    rng = np.random.default_rng(seed)
    key = random_key(rng)
    data = random_pages(rng, n_pages)
    return Bulk(key, data)


@dataclasses.dataclass
class Request:
    client: int
    op: int                 # 0 = encrypt, 1 = decrypt
    n_pages: int
    va: int                 # virtual address of the first page
    pid: int                # nonce tag


@dataclasses.dataclass
class Batched:
    keys: list              # one 32-byte key per client
    requests: list          # list[Request]
    plain: list             # per request (n_pages, 4096) uint8 plaintext

    @property
    def total_pages(self) -> int:
        return sum(r.n_pages for r in self.requests)


def log_uniform_pages(rng: np.random.Generator, hi: int, size=None):
    """floor(exp(U(0, ln(hi+1)))) clipped to [1, hi]."""
    v = np.floor(np.exp(rng.uniform(0.0, np.log(hi + 1), size=size)))
    return np.clip(v, 1, hi).astype(np.int64)


def batched(seed: int = 3, n_requests: int = 512, n_clients: int = 32,
            max_pages: int = 4096, with_data: bool = True) -> Batched:
    rng = np.random.default_rng(seed)
    keys = [random_key(rng) for _ in range(n_clients)]
    clients = rng.integers(0, n_clients, size=n_requests)
    pages = log_uniform_pages(rng, max_pages, size=n_requests)
    ops = rng.integers(0, 2, size=n_requests)
    vas = VA_BASE + PAGE * rng.integers(0, 1 << 24, size=n_requests,
                                        endpoint=True)
    reqs = [Request(int(c), int(o), int(p), int(v), 1000 + int(c))
            for c, o, p, v in zip(clients, ops, pages, vas)]
    plain = [random_pages(rng, r.n_pages) for r in reqs] if with_data else []
    return Batched(keys, reqs, plain)


@dataclasses.dataclass
class Serving:
    keys: list              # one key per client
    arrival_s: np.ndarray   # float64 arrival times (seconds from start)
    clients: np.ndarray     # int32
    ops: np.ndarray         # int32 0/1
    n_pages: np.ndarray     # int64
    src_page: np.ndarray    # int64 first page of the input slice in the pool
    pid: np.ndarray         # int64 nonce tag per request
    va: np.ndarray          # int64 VA of the first page


def serving(seed: int = 4, rate_hz: float = 20000.0, duration_s: float = 10.0,
            n_clients: int = 64, max_pages: int = 256,
            pool_pages: int = 2097152) -> Serving:
    rng = np.random.default_rng(seed)
    keys = [random_key(rng) for _ in range(n_clients)]
    n_est = int(rate_hz * duration_s * 1.2) + 64
    gaps = rng.exponential(1.0 / rate_hz, size=n_est)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    n = t.size
    clients = rng.integers(0, n_clients, size=n).astype(np.int32)
    ops = rng.integers(0, 2, size=n).astype(np.int32)
    pages = log_uniform_pages(rng, max_pages, size=n)
    src = rng.integers(0, pool_pages - max_pages, size=n).astype(np.int64)
    va = (VA_BASE + PAGE * rng.integers(0, 1 << 24, size=n)).astype(np.int64)
    pid = (1000 + clients).astype(np.int64)
    return Serving(keys, t, clients, ops, pages, src, pid, va)


@dataclasses.dataclass
class AccessTrace:
    """Page accesses of several clients.  Client c owns pages
    [0, pages_per_client) of its own address space (virtual address
    VA_BASE + 4096*page, PID 1000 + c).  Access t of client c touches
    page[c][t]; when value[c][t] != 0 it is a write that XORs the 64-bit
    value into 8-byte word word[c][t] of the page."""
    pages_per_client: int
    page: np.ndarray      # (clients, steps) int32
    word: np.ndarray      # (clients, steps) int16
    value: np.ndarray     # (clients, steps) uint64, 0 = read
    kind: np.ndarray      # (clients, steps) int8: 0 scan1, 1 scank, 2 zipf, 3 loop

    @property
    def clients(self) -> int:
        return self.page.shape[0]

    @property
    def steps(self) -> int:
        return self.page.shape[1]


def _segment(rng, kind, length, n, perm, zipf_p):
    if kind == 0:        # stride-1 scan
        s = rng.integers(0, n)
        return (s + np.arange(length)) % n
    if kind == 1:        # stride-k scan
        k = int(rng.choice([2, 4, 8, 16, 64]))
        s = rng.integers(0, n)
        return (s + k * np.arange(length)) % n
    if kind == 2:        # Zipf(1.1) over a fixed permutation of the pages
        ranks = rng.choice(n, size=length, p=zipf_p)
        return perm[ranks]
    loop_len = min(512, n)  # a 512-page sequence repeated
    s = rng.integers(0, n)
    seq = (s + np.arange(loop_len)) % n
    return np.resize(seq, length)


def access_trace(seed: int = 5, total_pages: int = 65536,
                 accesses: int = 2_000_000, clients: int = 64,
                 mean_segment: int = 2048, write_fraction: float = 0.25,
                 zipf_alpha: float = 1.1) -> AccessTrace:
    """Segments of geometric length (mean `mean_segment`), each one of: a
    stride-1 scan, a stride-k scan (k in {2, 4, 8, 16, 64}), Zipf(alpha)
    random accesses over a fixed random permutation of the client's pages,
    or a 512-page loop; chosen uniformly."""
    rng = np.random.default_rng(seed)
    n = total_pages // clients
    steps = accesses // clients
    ranks = np.arange(1, n + 1, dtype=np.float64)
    zipf_p = ranks ** (-zipf_alpha)
    zipf_p /= zipf_p.sum()
    page = np.empty((clients, steps), dtype=np.int32)
    kind = np.empty((clients, steps), dtype=np.int8)
    for c in range(clients):
        perm = rng.permutation(n)
        t = 0
        while t < steps:
            length = min(int(rng.geometric(1.0 / mean_segment)), steps - t)
            k = int(rng.integers(0, 4))
            page[c, t:t + length] = _segment(rng, k, length, n, perm, zipf_p)
            kind[c, t:t + length] = k
            t += length
    word = rng.integers(0, 512, size=(clients, steps)).astype(np.int16)
    is_write = rng.random((clients, steps)) < write_fraction
    value = rng.integers(1, 2**63, size=(clients, steps), dtype=np.uint64)
    value[~is_write] = 0
    return AccessTrace(n, page, word, value, kind)

"""Decrypt-on-fault sliding-window simulation with learned pre-decryption.

The paper's server (sections 4.2, 4.3) keeps, per client, a sliding window
of at most W pages in clear; an access to any other page faults; the page is
decrypted on the GPU (or zero-filled on first touch) and enters the window,
whose oldest page is then encrypted on the GPU and stored.  This module
replays synthetic access traces of many clients through that policy with
the page data really living on the GPU: a ciphertext store per client and a
pool of clear page slots, all bytes moved by the engine's fused batched
launch (ms_process_batch).

Extension (not in the paper): a predictor looks at the last C fault deltas
of a client each time it faults and names the k most likely next deltas;
those pages are pre-decrypted into a per-client prefetch buffer of P slots.
A later fault on a pre-decrypted page is served without a decrypt (the page
moves into the window); decrypt-on-fault remains the fallback for every
other fault.  Prefetched pages count against the clear-page budget: the
baseline to beat uses a window of W + P.

Fault events (window misses) are what the server observes, with or without
prefetching, so the predictor's input sequence is the same in training and
in use.

Pre-decryptions go either into the same fused launches as the demand work,
in program order, or (``hints=True``) to the engine as prefetch hints
(ms_prefetch_hint): low-priority, droppable requests that run on the
engine's own streams beside the demand launches, which never wait for them.
A hint the engine drops is simply not a prefetch.  Before it hands a page
over, the simulation makes sure the work that last wrote the page's stored
ciphertext and the slot it fills has finished; a later use of the slot (a
prefetch hit, or reuse after the page was pushed out unused) first waits for
the hint's ticket.

Background pre-encryption (the paper's conclusions suggest it as future
work): after each window miss, while a client's reclaimable slots (free
slots plus "clean" pages, whose current contents a background encryption
has already stored) are fewer than `bg_threshold`, its oldest page that is
not clean is encrypted in the background and stays in the window.  A clean
page is evicted without an encryption on the fault path; a write makes it
dirty again.

GPU work is queued and flushed in fused launches; a flush happens before any
operation that would conflict with one already queued (a page read and
written in one launch, a slot reused, a write that must follow a fill or
precede an encryption), so the result is byte-identical to running every
operation in program order.
"""
from __future__ import annotations

import dataclasses
from collections import Counter, OrderedDict, deque

import numpy as np
import torch

from . import memshield as ms
from .workloads import VA_BASE

PAGE = 4096


class DeltaVocab:
    """The V-1 most frequent fault deltas get ids 0..V-2; id V-1 is the
    out-of-vocabulary id (also used to pad short histories)."""

    def __init__(self, deltas, size: int = 1024):
        common = [d for d, _ in Counter(deltas).most_common(size - 1)]
        self.size = size
        self.oov = size - 1
        self.delta_of = np.array(common + [0] * (size - 1 - len(common)),
                                 dtype=np.int64)
        self.n_known = len(common)
        self.id_of = {d: i for i, d in enumerate(common)}

    def ids(self, deltas) -> np.ndarray:
        get = self.id_of.get
        return np.fromiter((get(int(d), self.oov) for d in deltas),
                           dtype=np.int32, count=len(deltas))


class PagedMemory:
    """Ciphertext stores and clear slots of all clients on the GPU, with
    queued, conflict-checked, fused cipher launches."""

    def __init__(self, eng: ms.Engine, keys, n_pages: int, slots: int,
                 max_batch: int = 1024):
        self.eng = eng
        self.keys = keys
        self.n_clients = len(keys)
        self.n_pages = n_pages
        self.slots = slots
        self.max_batch = max_batch
        self.store = torch.zeros(self.n_clients * n_pages * PAGE,
                                 dtype=torch.uint8, device="cuda")
        self.clear = torch.zeros(self.n_clients * slots * PAGE,
                                 dtype=torch.uint8, device="cuda")
        self.free = [deque(range(slots)) for _ in range(self.n_clients)]
        self.launches = 0
        self.pages_moved = 0
        # hand-over to prefetch hints (module doc)
        self.flushes = 0            # fused launches issued so far
        self.done_flushes = 0       # ... known finished on the device
        self.wrote_in = {}          # (client, page) -> flush of last encrypt
        self.slot_used_in = {}      # (client, slot) -> flush of last use
        self.hint_ticket = {}       # (client, slot) -> unfinished hint
        self.hints_issued = 0
        self.hints_dropped = 0
        self.hint_waits = 0
        # (start, end) events around each ms_process_batch call: the
        # interval includes the call's host-side preparation
        self.flush_events = []
        self.time_flushes = False
        self._reset_queue()

    def _reset_queue(self):
        self.reqs = []
        self.store_read = set()     # (client, page) read by a queued decrypt
        self.store_write = set()    # (client, page) written by an encrypt
        self.slot_busy = set()      # (client, slot) with any queued op
        self.slot_fill = set()      # (client, slot) filled by decrypt/zero
        self.slot_written = set()   # (client, slot) with queued writes
        self.zero = []
        self.writes = {}            # (global slot, word) -> xor value

    def _nonce(self, c: int, p: int) -> ms.ms_nonce:
        return ms.linear_nonce(VA_BASE + PAGE * p, PAGE, 1000 + c)

    def _gslot(self, c, s):
        return c * self.slots + s

    def alloc(self, c: int) -> int:
        s = self.free[c].popleft()
        self.wait_hint(c, s)
        if (c, s) in self.slot_busy:
            self.flush()
        return s

    def wait_hint(self, c: int, s: int) -> None:
        """Wait until the prefetch hint that fills slot s (if any) is done."""
        t = self.hint_ticket.pop((c, s), None)
        if t is None:
            return
        st, done = self.eng.poll([t], timeout_s=30.0)
        if st != ms.MS_OK or done[0] != 1:
            raise RuntimeError("prefetch hint did not finish: status %d, "
                               "state %d" % (st, done[0]))
        self.hint_waits += 1

    def hint(self, items) -> list:
        """Pre-decrypt (client, page, slot) items as prefetch hints; returns
        for each whether the engine took it (a dropped hint fills nothing).
        The hints read the stored ciphertext and write the slots from the
        engine's streams, which do not wait for this stream: queued work on
        those pages or slots is launched first, and the stream is
        synchronized if such work may still run."""
        if not items:
            return []
        if any((c, p) in self.store_write or (c, s) in self.slot_busy
               for c, p, s in items):
            self.flush()
        last = max(max(self.wrote_in.get((c, p), 0),
                       self.slot_used_in.get((c, s), 0))
                   for c, p, s in items)
        if last > self.done_flushes:
            torch.cuda.current_stream().synchronize()
            self.done_flushes = self.flushes
        reqs = [ms.request(self.keys[c], self.store, self.clear, 1,
                           self._nonce(c, p), op=ms.MS_DECRYPT, client=c,
                           src_offset_pages=c * self.n_pages + p,
                           dst_offset_pages=self._gslot(c, s))
                for c, p, s in items]
        tickets = self.eng.prefetch_hint(reqs)
        took = []
        for (c, p, s), t in zip(items, tickets):
            if t:
                self.hint_ticket[(c, s)] = t
                self.hints_issued += 1
            else:
                self.hints_dropped += 1
            took.append(bool(t))
        return took

    def wait_all_hints(self) -> None:
        for c, s in list(self.hint_ticket):
            self.wait_hint(c, s)

    def release(self, c: int, s: int) -> None:
        self.free[c].append(s)

    def decrypt(self, c: int, p: int, s: int) -> None:
        if (c, p) in self.store_write or (c, s) in self.slot_busy:
            self.flush()
        self.reqs.append(ms.request(
            self.keys[c], self.store, self.clear, 1, self._nonce(c, p),
            op=ms.MS_DECRYPT, client=c,
            src_offset_pages=c * self.n_pages + p,
            dst_offset_pages=self._gslot(c, s)))
        self.store_read.add((c, p))
        self.slot_busy.add((c, s))
        self.slot_fill.add((c, s))
        self._maybe_flush()

    def zero_fill(self, c: int, s: int) -> None:
        if (c, s) in self.slot_busy:
            self.flush()
        self.zero.append(self._gslot(c, s))
        self.slot_busy.add((c, s))
        self.slot_fill.add((c, s))

    def write(self, c: int, s: int, word: int, value: int) -> None:
        key = (self._gslot(c, s), int(word))
        self.writes[key] = self.writes.get(key, 0) ^ int(value)
        self.slot_busy.add((c, s))
        self.slot_written.add((c, s))

    def encrypt(self, c: int, s: int, p: int) -> None:
        if ((c, s) in self.slot_fill or (c, s) in self.slot_written or
                (c, p) in self.store_read or (c, p) in self.store_write):
            self.flush()
        self.reqs.append(ms.request(
            self.keys[c], self.clear, self.store, 1, self._nonce(c, p),
            op=ms.MS_ENCRYPT, client=c,
            src_offset_pages=self._gslot(c, s),
            dst_offset_pages=c * self.n_pages + p))
        self.store_write.add((c, p))
        self.slot_busy.add((c, s))
        self._maybe_flush()

    def _maybe_flush(self):
        if len(self.reqs) >= self.max_batch:
            self.flush()

    def flush(self) -> None:
        if self.reqs:
            arr = (ms.ms_request * len(self.reqs))(*self.reqs)
            if self.time_flushes:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                self.eng.process_batch(arr)
                e1.record()
                self.flush_events.append((e0, e1))
            else:
                self.eng.process_batch(arr)
            self.launches += 1
            self.pages_moved += len(self.reqs)
        self.flushes += 1
        for cp in self.store_write:
            self.wrote_in[cp] = self.flushes
        for cs in self.slot_busy:
            self.slot_used_in[cs] = self.flushes
        if self.zero:
            idx = torch.tensor(self.zero, dtype=torch.int64, device="cuda")
            self.clear.view(-1, PAGE).index_fill_(0, idx, 0)
        if self.writes:
            keys = np.array(list(self.writes.keys()), dtype=np.int64)
            vals = np.array(list(self.writes.values()), dtype=np.uint64)
            flat = keys[:, 0] * 512 + keys[:, 1]
            words = self.clear.view(torch.int64)
            it = torch.from_numpy(flat).to("cuda")
            vt = torch.from_numpy(vals.view(np.int64)).to("cuda")
            words[it] = torch.bitwise_xor(words[it], vt)
        self._reset_queue()

    def page_bytes(self, c: int, p: int) -> torch.Tensor:
        o = (c * self.n_pages + p) * PAGE
        return self.store[o:o + PAGE]

    def slot_bytes(self, c: int, s: int) -> torch.Tensor:
        o = self._gslot(c, s) * PAGE
        return self.clear[o:o + PAGE]


@dataclasses.dataclass
class Client:
    win: OrderedDict          # page -> slot, oldest first
    pf: OrderedDict           # prefetched unused page -> slot
    touched: bytearray
    events: deque             # recent fault-event pages
    clean: set = dataclasses.field(default_factory=set)  # window pages
    # whose current contents a background encryption has stored


def new_counters():
    return {"accesses": 0, "faults": 0, "first_touch": 0, "decrypts": 0,
            "encrypts": 0, "prefetch_issued": 0, "prefetch_hits": 0,
            "prefetch_wasted": 0, "events": 0, "encrypts_bg": 0,
            "bg_wasted": 0, "evict_clean": 0, "prefetch_dropped": 0}


def run(trace, window: int, mem: PagedMemory | None = None,
        prefetch_slots: int = 0, predictor=None, vocab: DeltaVocab | None = None,
        k: int = 8, predict_from: int = 0, stop: int | None = None,
        count_from: int = 0, record_events: bool = False,
        min_prob: float | None = None, bg_threshold: int = 0,
        hints: bool = False):
    """Replay `trace` (workloads.AccessTrace) for steps [0, stop) with all
    clients in lockstep.  Prediction is active for steps >= predict_from,
    counters cover steps >= count_from.  Returns (counters, events, decisions)
    where events[c] is the list of fault-event pages of client c (if
    recorded) and decisions maps (c, t) to the pages pre-decrypted after
    step t.  Of the predictor's top-k deltas only those with a softmax
    probability of at least `min_prob` (default: the predictor's own
    min_prob) are pre-decrypted.  `hints` sends the pre-decryptions to the
    engine as prefetch hints instead of the fused launches (module doc).
    `bg_threshold` > 0 turns on background pre-encryption (module doc)."""
    if min_prob is None:
        min_prob = predictor.min_prob if predictor is not None else 0.0
    if hints and mem is None:
        raise ValueError("hints need the page data on the GPU (mem)")
    C = trace.clients
    n = trace.pages_per_client
    stop = trace.steps if stop is None else stop
    ctx = predictor.context if predictor is not None else 0
    clients = [Client(OrderedDict(), OrderedDict(), bytearray(n),
                      deque(maxlen=ctx + 1)) for _ in range(C)]
    cnt = new_counters()
    events = [[] for _ in range(C)] if record_events else None
    decisions = {}
    page, word, value = trace.page, trace.word, trace.value

    def admit(c, cl, p, s, counting):
        cl.win[p] = s
        if len(cl.win) > window:
            q, sq = cl.win.popitem(last=False)
            clean = q in cl.clean
            cl.clean.discard(q)
            if mem is not None:
                if not clean:
                    mem.encrypt(c, sq, q)
                mem.release(c, sq)
            if counting:
                cnt["evict_clean" if clean else "encrypts"] += 1

    def background(c, cl, counting):
        reclaimable = window - len(cl.win) + len(cl.clean)
        for q, sq in cl.win.items():
            if reclaimable >= bg_threshold:
                break
            if q not in cl.clean:
                cl.clean.add(q)
                if mem is not None:
                    mem.encrypt(c, sq, q)
                reclaimable += 1
                if counting:
                    cnt["encrypts_bg"] += 1

    for t in range(stop):
        counting = t >= count_from
        want = []          # clients to predict for at this step
        for c in range(C):
            cl = clients[c]
            p = int(page[c, t])
            if counting:
                cnt["accesses"] += 1
            s = cl.win.get(p)
            miss = s is None
            if miss:
                # fault event: the server sees it
                if counting:
                    cnt["events"] += 1
                if record_events:
                    events[c].append(p)
                if predictor is not None:
                    cl.events.append(p)
                if p in cl.pf:
                    s = cl.pf.pop(p)
                    if hints:
                        mem.wait_hint(c, s)
                    if counting:
                        cnt["prefetch_hits"] += 1
                elif cl.touched[p]:
                    s = mem.alloc(c) if mem is not None else 0
                    if mem is not None:
                        mem.decrypt(c, p, s)
                    if counting:
                        cnt["faults"] += 1
                        cnt["decrypts"] += 1
                else:
                    cl.touched[p] = 1
                    s = mem.alloc(c) if mem is not None else 0
                    if mem is not None:
                        mem.zero_fill(c, s)
                    if counting:
                        cnt["first_touch"] += 1
                admit(c, cl, p, s, counting)
                if predictor is not None and t >= predict_from and \
                        len(cl.events) == ctx + 1:
                    want.append(c)
            v = int(value[c, t])
            if v:
                if mem is not None:
                    mem.write(c, s, int(word[c, t]), v)
                if p in cl.clean:
                    cl.clean.discard(p)
                    if counting:
                        cnt["bg_wasted"] += 1
            if bg_threshold > 0 and miss:
                background(c, cl, counting)
        if want:
            hist = np.array([list(clients[c].events) for c in want],
                            dtype=np.int64)
            ids = vocab.ids(np.diff(hist, axis=1).reshape(-1)).reshape(
                len(want), ctx)
            top, prob = predictor.predict(ids, k, vocab.oov, with_prob=True)
            top = top.cpu().numpy()
            prob = prob.cpu().numpy()
            picks = []     # (client, page) in decision order
            for row, c in enumerate(want):
                cl = clients[c]
                last = int(clients[c].events[-1])
                chosen = set()
                for tid, pr in zip(top[row], prob[row]):
                    if int(tid) >= vocab.n_known or pr < min_prob:
                        continue
                    q = last + int(vocab.delta_of[int(tid)])
                    if not (0 <= q < n) or q in cl.win or q in cl.pf or \
                            not cl.touched[q] or q in chosen:
                        continue
                    chosen.add(q)
                    picks.append((c, q))
            if hints:
                # slots first, then one hint call for the whole step
                slots = [mem.alloc(c) for c, _ in picks]
                took = mem.hint([(c, q, s) for (c, q), s in
                                 zip(picks, slots)])
                for (c, _), s, ok in zip(picks, slots, took):
                    if not ok:
                        mem.release(c, s)
                        if counting:
                            cnt["prefetch_dropped"] += 1
            else:
                slots = [None] * len(picks)
                took = [True] * len(picks)
            for (c, q), s, ok in zip(picks, slots, took):
                if not ok:
                    continue
                cl = clients[c]
                if not hints:
                    s = mem.alloc(c) if mem is not None else 0
                    if mem is not None:
                        mem.decrypt(c, q, s)
                cl.pf[q] = s
                decisions.setdefault((c, t), []).append(q)
                if counting:
                    cnt["prefetch_issued"] += 1
                    cnt["decrypts"] += 1
                if len(cl.pf) > prefetch_slots:
                    _, sd = cl.pf.popitem(last=False)
                    if mem is not None:
                        mem.release(c, sd)
                    if counting:
                        cnt["prefetch_wasted"] += 1
    if mem is not None:
        mem.flush()
    return cnt, events, decisions, clients


def finish(mem: PagedMemory, clients) -> None:
    """Encrypt every page still in a window back into the store (the end of
    the run) unless a background encryption already stored it; unused
    prefetched pages are dropped."""
    mem.wait_all_hints()
    for c, cl in enumerate(clients):
        for p, s in cl.win.items():
            if p not in cl.clean:  # clean pages are already stored
                mem.encrypt(c, s, p)
        cl.win.clear()
        cl.pf.clear()
        cl.clean.clear()
    mem.flush()


def training_examples(events, vocab: DeltaVocab, context: int):
    """From each client's fault-event pages: inputs = ids of `context`
    consecutive deltas, target = id of the next delta."""
    xs, ys = [], []
    for ev in events:
        if len(ev) < context + 2:
            continue
        d = vocab.ids(np.diff(np.asarray(ev, dtype=np.int64)))
        win = np.lib.stride_tricks.sliding_window_view(d, context + 1)
        xs.append(win[:, :context])
        ys.append(win[:, context])
    return np.concatenate(xs).astype(np.int32), \
        np.concatenate(ys).astype(np.int32)


def train(predictor, xs, ys, steps: int, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0, log_every: int = 0):
    """Adam on random minibatches; returns the loss history (per step)."""
    rng = np.random.default_rng(seed)
    x_dev = torch.from_numpy(xs).to("cuda")
    y_dev = torch.from_numpy(ys).to("cuda")
    losses = torch.zeros(steps, dtype=torch.float32, device="cuda")
    for i in range(steps):
        idx = torch.from_numpy(rng.integers(0, xs.shape[0], size=batch)).to(
            "cuda")
        loss = predictor.train_step(x_dev[idx], y_dev[idx], lr=lr)
        losses[i:i + 1].copy_(loss)
    return losses.cpu().numpy()

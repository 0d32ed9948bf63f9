"""Reference model of MemShield's decrypt-on-fault sliding window.  TEST
INFRASTRUCTURE ONLY.

What it follows (paper sections 4.2 and 4.3):
  * every client has a sliding window: a list of its pages that are in clear,
    with a configurable maximum size;
  * an access to a page not in the window is a page fault; if the page was
    never touched before it is resolved with a page of zeros and nothing is
    decrypted (first touch); otherwise its ciphertext is decrypted (the GPU
    work) and the page becomes clear;
  * the faulting page is appended to the window; when the window exceeds its
    maximum, its oldest page is removed, encrypted (the GPU work) and stored
    as ciphertext.
Readings added here (the paper has no prefetcher): a prefetcher may
pre-decrypt pages into a separate FIFO of `prefetch_slots` clear pages; an
access that finds its page there is not a fault and moves the page into the
window (which may evict the window's oldest page); a prefetched page that is
pushed out of the prefetch FIFO unused is dropped without re-encryption (it
was never modified).  Writes: an access may XOR a 64-bit value into one
8-byte word of its page.

Background pre-encryption (the paper's conclusions, section 7, suggest
encrypting window pages in the background once the free slots of the window
fall below a threshold).  Reading: a window page is "clean" when a
background encryption has stored its current contents; a clean page can be
evicted without encrypting it on the fault path.  The reclaimable slots of a
window are its free slots plus its clean pages.  After each window miss,
while the reclaimable slots are fewer than `bg_threshold`, the oldest page
that is not clean is encrypted in the background and becomes clean (it
stays in the window, in clear).  A write to a clean page makes it dirty
again (that background encryption was wasted).  An evicted dirty page is
encrypted on the fault path as without the mechanism.

``simulate`` counts faults, first touches, decrypts and encrypts for a trace
and a given sequence of prefetch decisions; ``final_plaintext`` computes the
page contents every write sequence leads to, independent of the window.
"""
from __future__ import annotations

from collections import OrderedDict, deque

import numpy as np


def simulate(pages, window: int, prefetch=None, prefetch_slots: int = 0,
             start: int = 0, stop: int | None = None, writes=None,
             bg_threshold: int = 0):
    """One client's accesses `pages` (sequence of page ids).

    `prefetch`: optional dict {access index t: list of page ids} of pages the
    prefetcher asks for right after access t is served (already-clear pages
    are ignored).  `writes`: optional sequence, true where access t writes
    its page.  `bg_threshold`: background pre-encryption threshold (0 = no
    background encryption).  Counters are taken over accesses [start, stop).
    Returns a dict of counters and the ordered list of fault events
    (t, page) in [start, stop) that needed a decrypt.  "encrypts" counts
    encryptions on the fault path (evictions of pages that are not clean),
    "encrypts_bg" background encryptions, "bg_wasted" clean pages written
    again, "evict_clean" evictions that needed no encryption.
    """
    stop = len(pages) if stop is None else stop
    win = OrderedDict()          # page -> clean (bool), oldest first
    pf = OrderedDict()           # prefetched, unused pages
    touched = set()
    cnt = {"accesses": 0, "faults": 0, "first_touch": 0, "decrypts": 0,
           "encrypts": 0, "prefetch_issued": 0, "prefetch_hits": 0,
           "prefetch_wasted": 0, "encrypts_bg": 0, "bg_wasted": 0,
           "evict_clean": 0}
    fault_log = []

    def admit(p, counting):
        win[p] = False
        if len(win) > window:
            old, clean = win.popitem(last=False)
            if counting:
                cnt["evict_clean" if clean else "encrypts"] += 1

    def background(counting):
        reclaimable = window - len(win) + sum(1 for c in win.values() if c)
        for q in win:
            if reclaimable >= bg_threshold:
                break
            if not win[q]:
                win[q] = True
                reclaimable += 1
                if counting:
                    cnt["encrypts_bg"] += 1

    for t in range(stop):
        p = int(pages[t])
        counting = t >= start
        if counting:
            cnt["accesses"] += 1
        miss = p not in win
        if not miss:
            pass
        elif p in pf:
            del pf[p]
            if counting:
                cnt["prefetch_hits"] += 1
            admit(p, counting)
        else:
            if p in touched:
                if counting:
                    cnt["faults"] += 1
                    cnt["decrypts"] += 1
                    fault_log.append((t, p))
            else:
                touched.add(p)
                if counting:
                    cnt["first_touch"] += 1
            admit(p, counting)
        if writes is not None and writes[t] and win[p]:
            win[p] = False
            if counting:
                cnt["bg_wasted"] += 1
        if bg_threshold > 0 and miss:
            background(counting)
        if prefetch and t in prefetch:
            for q in prefetch[t]:
                q = int(q)
                if q in win or q in pf or q not in touched:
                    continue
                pf[q] = None
                if counting:
                    cnt["prefetch_issued"] += 1
                    cnt["decrypts"] += 1
                if len(pf) > prefetch_slots:
                    pf.popitem(last=False)
                    if counting:
                        cnt["prefetch_wasted"] += 1
    return cnt, fault_log


def final_plaintext(n_pages: int, pages, words, values) -> np.ndarray:
    """(n_pages, 4096) uint8: every page starts as zeros (first touch) and
    each access with a non-zero value XORs it into 8-byte word `words[t]`."""
    mem = np.zeros((n_pages, 512), dtype=np.uint64)
    np.bitwise_xor.at(mem, (np.asarray(pages, dtype=np.int64),
                            np.asarray(words, dtype=np.int64)),
                      np.asarray(values, dtype=np.uint64))
    return mem.astype("<u8").view(np.uint8).reshape(n_pages, 4096)


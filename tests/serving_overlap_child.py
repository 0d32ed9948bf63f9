"""Child process of test_gpu_serving.test_batches_overlap_on_device (not a
test module): a large request is submitted with a narrow forced tiling, then
six small requests one after another; prints one JSON line saying how many
small requests completed while the large one was still running, and whether
their outputs match the CPU oracle."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_09252_amd import memshield as ms  # noqa: E402
from paper_2004_09252_amd import workloads  # noqa: E402


def main():
    import torch
    # the process's first streams are the engine's; the launch stage
    eng = ms.Engine(0, serve_stage=ms.MS_SERVE_STAGE_LAUNCH)
    rng = np.random.default_rng(42)
    kb = [rng.bytes(32) for _ in range(2)]
    keys = [eng.key_load(k) for k in kb]
    n_small = 6
    small = workloads.random_pages(rng, n_small * 2)
    src = torch.from_numpy(small.reshape(-1).copy()).to("cuda")
    dst = torch.zeros_like(src)
    big_pages = 65536
    big = torch.zeros(big_pages * 4096, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    def small_req(i):
        return ms.request(keys[1], src, dst, 2, ms.linear_nonce(4096 * i, 1, 7),
                          src_offset_pages=2 * i, dst_offset_pages=2 * i)

    # warm up: kernels loaded, streams used once
    t = eng.submit([small_req(0)])
    assert eng.poll(t, timeout_s=30)[0] == 0
    # a narrow grid for the large request leaves room on the chip
    assert ms.ms_set_tuning(eng.ctx, ms.ms_tuning(64, 1, 2, 0, 0.0)) == 0
    before = eng.stats().batches
    tb = eng.submit([ms.request(keys[0], big, big, big_pages,
                                ms.linear_nonce(0, 1, 0))])
    t0 = time.time()
    while eng.stats().batches == before and time.time() - t0 < 10:
        pass
    overlapped = 0
    for i in range(n_small):
        ts = eng.submit([small_req(i)])
        st, d_small = eng.poll(ts, timeout_s=30)
        assert st == 0 and d_small == [1]
        overlapped += eng.poll(tb, timeout_s=0)[1] == [0]
    stats = eng.stats()
    assert eng.poll(tb, timeout_s=30)[0] == 0
    ms.ms_set_tuning(eng.ctx, None)
    got = dst.cpu().numpy().reshape(n_small * 2, 4096)
    exact = True
    for i in range(n_small):
        want = oracle.cipher_pages(kb[1], oracle.nonces_linear(2, 4096 * i, 1, 7),
                                   small[2 * i:2 * i + 2])
        exact = exact and np.array_equal(got[2 * i:2 * i + 2], want)
    for k in keys:
        eng.key_destroy(k)
    eng.close()
    print(json.dumps({"overlapped": int(overlapped),
                      "max_inflight_batches": int(stats.max_inflight_batches),
                      "small_exact": bool(exact)}), flush=True)


if __name__ == "__main__":
    main()

"""Write ``page_cipher_digests.txt``: SHA-256 digests of the oracle's output
on the seeded page workloads.  Calls only the CPU oracle and the seeded input
generators.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(
    os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_09252_amd import workloads  # noqa: E402


def main():
    lines = ["# ChaCha20 page cipher (paper section 4.4): SHA-256 of the",
             "# oracle's ciphertext for the seeded workloads.",
             "# workload seed n_pages sha256(ciphertext)"]
    t = workloads.tiny(seed=1)
    enc = oracle.cipher_pages(t.key, t.nonces, t.data)
    lines.append("tiny 1 64 %s" % hashlib.sha256(enc.tobytes()).hexdigest())
    b = workloads.bulk(seed=2)
    n = oracle.nonces_linear(b.data.shape[0], b.nonce_base, b.nonce_stride,
                             b.nonce_tag)
    threads = len(os.sched_getaffinity(0))
    enc = oracle.cipher_pages(b.key, n, b.data, threads=threads)
    lines.append("bulk 2 %d %s" % (b.data.shape[0],
                                   hashlib.sha256(enc.tobytes()).hexdigest()))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "page_cipher_digests.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(open(path).read())


if __name__ == "__main__":
    main()

"""Write the exact prime lists of large workloads as per-block digests.

Calls only ``oracle/`` (the definitional enumerator: the Lemma of Sec. 4.1,
MergeAll for M, then the O formula read with OR) and the input generator.
For a workload of n variables the cubes are split into the 81 blocks of their
top four ternary digits (block b holds b * 3^(n-4) <= rho < (b+1) * 3^(n-4)).
For each block the file records the number of primes and the SHA-256 of the
block's sorted prime indices as little-endian uint64 bytes.  The whole M is
held once (n = 24: 35.3 GB of host memory); O is evaluated one block at a
time and never held whole.

Usage: python tests/golden/make_block_digests.py CONFIG [CONFIG ...]
writes tests/golden/blocks_CONFIG.txt for each named workload of
``paper_2302_10083_amd.inputs.CONFIGS``.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2302_10083_amd import inputs  # noqa: E402

TOP = 4  # top ternary digits that name a block


def block_digests(n: int, M: np.ndarray, top: int = TOP, threads: int = 0):
    """[(count, sha256 hex)] per block of the top ``top`` digits, from M."""
    top = min(top, n)
    bs = 3 ** (n - top)
    out = []
    for b in range(3**top):
        lst = oracle.primes_range(n, M, b * bs, (b + 1) * bs, threads)
        out.append((int(lst.size), hashlib.sha256(lst.astype("<u8").tobytes()).hexdigest()))
    return out


def digests_of_list(n: int, lst: np.ndarray, top: int = TOP):
    """The same digests from a whole sorted prime list (for comparisons)."""
    top = min(top, n)
    bs = 3 ** (n - top)
    lst = np.asarray(lst, dtype=np.uint64)
    edges = np.searchsorted(lst, np.arange(3**top + 1, dtype=np.uint64) * np.uint64(bs))
    out = []
    for b in range(3**top):
        part = lst[edges[b]:edges[b + 1]]
        out.append((int(part.size), hashlib.sha256(part.astype("<u8").tobytes()).hexdigest()))
    return out


def path_for(config: str) -> str:
    return os.path.join(HERE, "blocks_%s.txt" % config)


def read(config: str):
    """(n, top, total, [(count, sha256)]) from a digest file."""
    n = top = total = None
    rows = []
    with open(path_for(config)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            if k == "n":
                n = int(v[0])
            elif k == "top":
                top = int(v[0])
            elif k == "total":
                total = int(v[0])
            elif k == "block":
                rows.append((int(v[1]), v[2]))
    return n, top, total, rows


def write(config: str, threads: int = 0) -> str:
    spec = inputs.CONFIGS[config]
    n = spec["n"]
    tt = inputs.make(spec)
    t0 = time.time()
    M = oracle.enum_M(n, tt, threads)
    t1 = time.time()
    rows = block_digests(n, M, TOP, threads)
    t2 = time.time()
    del M
    total = sum(c for c, _ in rows)
    with open(path_for(config), "w") as f:
        f.write("# Exact prime implicants of workload %s (%r),\n" % (config, spec))
        f.write("# from the CPU oracle only: M by the Lemma of Sec. 4.1 (MergeAll), O by its\n")
        f.write("# formula read with OR, evaluated per block of the top %d ternary digits.\n" % TOP)
        f.write("# Block b covers b * 3^(n-%d) <= rho < (b+1) * 3^(n-%d); each line gives the\n" % (TOP, TOP))
        f.write("# block's prime count and the SHA-256 of its sorted rho as little-endian uint64.\n")
        f.write("# Written by: python tests/golden/make_block_digests.py %s\n" % config)
        f.write("# (oracle time: M %.0f s, O %.0f s)\n" % (t1 - t0, t2 - t1))
        f.write("n %d\ntop %d\ntotal %d\n" % (n, TOP, total))
        for b, (c, h) in enumerate(rows):
            f.write("block %d %d %s\n" % (b, c, h))
    return path_for(config)


if __name__ == "__main__":
    for name in sys.argv[1:]:
        t = time.time()
        print("%s -> %s (%.0f s)" % (name, write(name), time.time() - t), flush=True)

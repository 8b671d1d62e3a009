"""CPU oracle for dense Quine-McCluskey prime implicants.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and the library never calls it.

Everything is computed from the paper's definitions (Udovenko, "DenseQMC",
arXiv 2302.10083):

* ``is_implicant`` / ``is_prime`` / ``is_prime_all_divisors``: Sec. 2,
  definitions of implicant and prime implicant, per cube.
* ``bruteforce``: those per-cube definitions over all 3^n cubes.
* ``enum_M`` / ``enum_O``: the Lemma of Sec. 4.1 (MergeAll, ReduceAll),
  cube by cube in increasing rho; the O formula is read with OR (see
  ``dqmc_oracle.c``).
* ``enum_O_range`` / ``primes_range``: the same O formula on one range of
  rho only, reading the whole M ("streaming": the O bitmap of the whole
  function is never held, so n = 24 fits next to its 35.3 GB M).
* ``extract``: set bits in increasing rho (Alg. 4, output step).

Cube index rho(s) = sum 3^(i-1) rho(s_i), with 0, 1, * -> 0, 1, 2 (Sec. 4.2).
Bitmaps are little-endian uint64 arrays with bit rho = membership.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dqmc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (host only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
            lib.orc_pow3.restype = u64
            lib.orc_pow3.argtypes = [i32]
            for name in ("orc_is_implicant", "orc_is_prime", "orc_is_prime_all_divisors"):
                f = getattr(lib, name)
                f.restype = i32
                f.argtypes = [i32, vp, u64]
            lib.orc_bruteforce.restype = None
            lib.orc_bruteforce.argtypes = [i32, vp, vp, vp, i32, i32]
            lib.orc_enum_M.restype = None
            lib.orc_enum_M.argtypes = [i32, vp, vp, i32]
            lib.orc_enum_O.restype = None
            lib.orc_enum_O.argtypes = [i32, vp, vp, i32]
            lib.orc_enum_O_range.restype = None
            lib.orc_enum_O_range.argtypes = [i32, vp, u64, u64, vp, i32]
            lib.orc_extract.restype = u64
            lib.orc_extract.argtypes = [i32, vp, vp, u64]
            lib.orc_extract_bits.restype = u64
            lib.orc_extract_bits.argtypes = [u64, vp, vp, u64, u64]
            lib.orc_sample.restype = i32
            lib.orc_sample.argtypes = [i32, vp, vp, u64, vp, i32, i32]
            _lib = lib
    return _lib


def num_cubes(n: int) -> int:
    return 3**n


def bitmap_words(n: int) -> int:
    return (3**n + 63) // 64


def _tt(tt) -> np.ndarray:
    a = np.ascontiguousarray(tt, dtype=np.uint32)
    return a


def is_implicant(n: int, tt, rho: int) -> bool:
    a = _tt(tt)
    return bool(_load().orc_is_implicant(n, a.ctypes.data, rho))


def is_prime(n: int, tt, rho: int) -> bool:
    a = _tt(tt)
    return bool(_load().orc_is_prime(n, a.ctypes.data, rho))


def is_prime_all_divisors(n: int, tt, rho: int) -> bool:
    a = _tt(tt)
    return bool(_load().orc_is_prime_all_divisors(n, a.ctypes.data, rho))


def bruteforce(n: int, tt, all_divisors: bool = False, threads: int = 0):
    """(M, O) bitmaps from the per-cube definitions over all 3^n cubes."""
    a = _tt(tt)
    M = np.zeros(bitmap_words(n), dtype=np.uint64)
    O = np.zeros(bitmap_words(n), dtype=np.uint64)
    _load().orc_bruteforce(n, a.ctypes.data, M.ctypes.data, O.ctypes.data, int(all_divisors), threads)
    return M, O


def enum_M(n: int, tt, threads: int = 0) -> np.ndarray:
    a = _tt(tt)
    M = np.zeros(bitmap_words(n), dtype=np.uint64)
    _load().orc_enum_M(n, a.ctypes.data, M.ctypes.data, threads)
    return M


def enum_O(n: int, M: np.ndarray, threads: int = 0) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.uint64)
    O = np.zeros(bitmap_words(n), dtype=np.uint64)
    _load().orc_enum_O(n, M.ctypes.data, O.ctypes.data, threads)
    return O


def enum_O_range(n: int, M: np.ndarray, r0: int, r1: int, threads: int = 0) -> np.ndarray:
    """O on the cubes r0 <= rho < r1 only: a bitmap whose bit k is cube
    r0 + k (ceil((r1 - r0) / 64) words)."""
    assert 0 <= r0 <= r1 <= 3**n
    M = np.ascontiguousarray(M, dtype=np.uint64)
    assert M.size >= bitmap_words(n)
    out = np.zeros(max(1, (r1 - r0 + 63) // 64), dtype=np.uint64)
    _load().orc_enum_O_range(n, M.ctypes.data, r0, r1, out.ctypes.data, threads)
    return out


def extract_bits(nbits: int, bm: np.ndarray, base: int = 0) -> np.ndarray:
    """Set bits of a bitmap whose bit k is cube base + k, ascending."""
    bm = np.ascontiguousarray(bm, dtype=np.uint64)
    lib = _load()
    cnt = int(lib.orc_extract_bits(nbits, bm.ctypes.data, None, 0, base))
    out = np.zeros(max(cnt, 1), dtype=np.uint64)
    lib.orc_extract_bits(nbits, bm.ctypes.data, out.ctypes.data, cnt, base)
    return out[:cnt]


def primes_range(n: int, M: np.ndarray, r0: int, r1: int, threads: int = 0) -> np.ndarray:
    """Sorted primes with r0 <= rho < r1, from the whole implicant bitmap M."""
    return extract_bits(r1 - r0, enum_O_range(n, M, r0, r1, threads), r0)


def extract(n: int, O: np.ndarray, cap: int | None = None):
    """(list of rho ascending, total count)."""
    O = np.ascontiguousarray(O, dtype=np.uint64)
    lib = _load()
    cnt = int(lib.orc_extract(n, O.ctypes.data, None, 0))
    k = cnt if cap is None else min(cap, cnt)
    out = np.zeros(max(k, 1), dtype=np.uint64)
    lib.orc_extract(n, O.ctypes.data, out.ctypes.data, k)
    return out[:k], cnt


def sample(n: int, tt, rhos, what: str = "prime", threads: int = 0):
    """Per-cube definitions on an array of cube indices: returns (bool array,
    threads used)."""
    a = _tt(tt)
    r = np.ascontiguousarray(rhos, dtype=np.uint64)
    out = np.zeros(max(1, r.size), dtype=np.uint8)
    used = _load().orc_sample(n, a.ctypes.data, r.ctypes.data, r.size, out.ctypes.data,
                              1 if what == "prime" else 0, threads)
    return out[: r.size].astype(bool), int(used)


def primes(n: int, tt, threads: int = 0):
    """(M, O, sorted prime list) by the definitional enumerator."""
    M = enum_M(n, tt, threads)
    O = enum_O(n, M, threads)
    lst, _ = extract(n, O)
    return M, O, lst


# ----------------------------------------------------------------------------
# string helpers (Sec. 2 notation; s_1 printed leftmost as in the paper)

def rho_of(s: str) -> int:
    """Index of a cube string s_1 s_2 ... s_n over {0, 1, *}."""
    val = {"0": 0, "1": 1, "*": 2}
    return sum(val[c] * 3**i for i, c in enumerate(s))


def string_of(n: int, rho: int) -> str:
    out = []
    for _ in range(n):
        out.append("01*"[rho % 3])
        rho //= 3
    return "".join(out)


def bitmap_to_set(n: int, bm: np.ndarray) -> set:
    lst, _ = extract(n, bm)
    return set(int(x) for x in lst)


def set_to_bitmap(n: int, rhos) -> np.ndarray:
    bm = np.zeros(bitmap_words(n), dtype=np.uint64)
    for r in rhos:
        bm[r >> 6] |= np.uint64(1) << np.uint64(r & 63)
    return bm

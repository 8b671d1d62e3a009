"""Seeded synthetic truth tables.

This module produces inputs only; it contains no part of the prime-implicant
method.  Both the GPU library's tests/benchmark and the CPU oracle take their
truth tables from here.

Truth-table format: a little-endian ``uint32`` array of ``max(1, 2**(n-5))``
words; bit ``x`` is ``f(x)`` and variable ``x_i`` is bit ``i-1`` of ``x``.
Random numbers come from counter-based SplitMix64 (see ``gen.c``).

The workloads follow the paper's experiments, which use random functions of a
given density (Sec. 6, Table 1); the configurations below fix the densities,
DNF shapes and seeds that the paper leaves open.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libdqmc_inputs.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (host code only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            u64, i32, f64, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
            lib.gen_u64.restype = u64
            lib.gen_u64.argtypes = [u64, u64]
            lib.gen_uniform.restype = f64
            lib.gen_uniform.argtypes = [u64, u64]
            lib.gen_u64_array.restype = None
            lib.gen_u64_array.argtypes = [u64, u64, u64, vp]
            lib.gen_bernoulli.restype = None
            lib.gen_bernoulli.argtypes = [i32, f64, u64, i32, vp]
            lib.gen_dnf.restype = None
            lib.gen_dnf.argtypes = [i32, ctypes.c_uint32, i32, i32, u64, i32, vp]
            lib.gen_terms.restype = None
            lib.gen_terms.argtypes = [i32, ctypes.c_uint32, vp, vp, i32, vp]
            _lib = lib
    return _lib


# ----------------------------------------------------------------------------
# sizes and raw random numbers

def tt_words(n: int) -> int:
    return 1 if n <= 5 else 1 << (n - 5)


def u64(seed: int, i: int) -> int:
    return int(_load().gen_u64(seed & (2**64 - 1), i))


def u64_array(seed: int, count: int, start: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gen_u64_array(seed & (2**64 - 1), start, count, out.ctypes.data)
    return out


def uniform(seed: int, i: int) -> float:
    return float(_load().gen_uniform(seed & (2**64 - 1), i))


def subseed(seed: int, tag: int) -> int:
    """Independent derived seed for a second stream of one input."""
    return u64(seed ^ 0x5EED5EED5EED5EED, tag)


# ----------------------------------------------------------------------------
# random families

def bernoulli(n: int, p: float, seed: int) -> np.ndarray:
    """Each truth-table bit i.i.d. Bernoulli(p)."""
    tt = np.zeros(tt_words(n), dtype=np.uint32)
    _load().gen_bernoulli(n, float(p), seed & (2**64 - 1), 0, tt.ctypes.data)
    return tt


def or_bernoulli(tt: np.ndarray, n: int, p: float, seed: int) -> np.ndarray:
    """OR Bernoulli(p) noise minterms into ``tt`` (in place) and return it."""
    _load().gen_bernoulli(n, float(p), seed & (2**64 - 1), 1, tt.ctypes.data)
    return tt


def dnf(n: int, terms: int, wlo: int, whi: int, seed: int) -> np.ndarray:
    """OR of ``terms`` random products, width uniform in [wlo, whi], random
    variables and random polarity."""
    tt = np.zeros(tt_words(n), dtype=np.uint32)
    _load().gen_dnf(n, int(terms), int(wlo), int(whi), seed & (2**64 - 1), 0, tt.ctypes.data)
    return tt


def from_terms(n: int, terms) -> np.ndarray:
    """OR of explicit products, each given as ``(care_mask, value_bits)``."""
    tt = np.zeros(tt_words(n), dtype=np.uint32)
    if len(terms) == 0:
        return tt
    care = np.array([t[0] for t in terms], dtype=np.uint64)
    val = np.array([t[1] for t in terms], dtype=np.uint64)
    _load().gen_terms(n, len(terms), care.ctypes.data, val.ctypes.data, 0, tt.ctypes.data)
    return tt


# ----------------------------------------------------------------------------
# structured families (used by closed-form checks)

def from_bits(n: int, bits: np.ndarray) -> np.ndarray:
    """Pack a boolean vector of length 2**n into the truth-table format."""
    bits = np.asarray(bits, dtype=np.uint8).reshape(-1)
    assert bits.size == 1 << n
    nbytes = tt_words(n) * 4
    packed = np.packbits(bits, bitorder="little")
    buf = np.zeros(nbytes, dtype=np.uint8)
    buf[: packed.size] = packed
    if n < 3:  # packbits pads the last byte with zeros already
        pass
    return buf.view(np.uint32).copy()


def to_bits(n: int, tt: np.ndarray) -> np.ndarray:
    """Unpack a truth table into a boolean vector of length 2**n."""
    b = np.unpackbits(np.asarray(tt, dtype=np.uint32).view(np.uint8), bitorder="little")
    return b[: 1 << n].astype(bool)


def _popcounts(n: int) -> np.ndarray:
    x = np.arange(1 << n, dtype=np.uint64)
    return np.bitwise_count(x).astype(np.int64)


def constant(n: int, value: int) -> np.ndarray:
    return from_bits(n, np.full(1 << n, bool(value)))


def parity(n: int) -> np.ndarray:
    """f(x) = x_1 xor ... xor x_n."""
    return from_bits(n, (_popcounts(n) & 1).astype(bool))


def interval(n: int, a: int, b: int) -> np.ndarray:
    """Symmetric function f(x) = [a <= popcount(x) <= b]."""
    pc = _popcounts(n)
    return from_bits(n, (pc >= a) & (pc <= b))


def unate_terms(n: int, terms: int, wlo: int, whi: int, seed: int):
    """Random product terms in which every variable has one fixed polarity
    (a unate DNF).  Returns the list of ``(care, value)`` pairs."""
    r = u64_array(seed, 1 + terms * (n + 2))
    pol = int(r[0]) & ((1 << n) - 1)
    out, k = [], 1
    for _ in range(terms):
        w = wlo + int(r[k]) % (whi - wlo + 1)
        k += 1
        w = max(0, min(n, w))
        perm = list(range(n))
        for j in range(w):
            jj = j + int(r[k]) % (n - j)
            k += 1
            perm[j], perm[jj] = perm[jj], perm[j]
        care = 0
        for j in range(w):
            care |= 1 << perm[j]
        k += n - w  # keep the stream position independent of w
        out.append((care, pol & care))
    return out


# ----------------------------------------------------------------------------
# named workloads

CONFIGS = {
    "c1_n12_bern05": dict(n=12, kind="bernoulli", p=0.5, seed=12),
    "c2a_n20_bern09": dict(n=20, kind="bernoulli", p=0.9, seed=2001),
    "c2b_n20_dnf200": dict(n=20, kind="dnf", terms=200, wlo=4, whi=10, seed=2002),
    "c3_n24_dnf2000_noise": dict(n=24, kind="dnf+noise", terms=2000, wlo=6, whi=14, p=0.02, seed=24),
    # the same recipe at n = 21..23 (exact block digests next to n = 24), at
    # n = 25 (the largest single state) and at n = 26, 27, past one state in
    # HBM (the sliced path)
    "c3x_n21_dnf2000_noise": dict(n=21, kind="dnf+noise", terms=2000, wlo=6, whi=14, p=0.02, seed=21),
    "c3x_n22_dnf2000_noise": dict(n=22, kind="dnf+noise", terms=2000, wlo=6, whi=14, p=0.02, seed=22),
    "c3x_n23_dnf2000_noise": dict(n=23, kind="dnf+noise", terms=2000, wlo=6, whi=14, p=0.02, seed=23),
    "c3x_n25_dnf2000_noise": dict(n=25, kind="dnf+noise", terms=2000, wlo=6, whi=14, p=0.02, seed=25),
    "c3x_n26_dnf2000_noise": dict(n=26, kind="dnf+noise", terms=2000, wlo=6, whi=14, p=0.02, seed=26),
    "c3x_n27_dnf2000_noise": dict(n=27, kind="dnf+noise", terms=2000, wlo=6, whi=14, p=0.02, seed=27),
}


def make(spec: dict) -> np.ndarray:
    """Truth table for a workload description (see ``CONFIGS``)."""
    n, kind, seed = spec["n"], spec["kind"], spec["seed"]
    if kind == "bernoulli":
        return bernoulli(n, spec["p"], seed)
    if kind == "dnf":
        return dnf(n, spec["terms"], spec["wlo"], spec["whi"], seed)
    if kind == "dnf+noise":
        tt = dnf(n, spec["terms"], spec["wlo"], spec["whi"], subseed(seed, 0))
        return or_bernoulli(tt, n, spec["p"], subseed(seed, 1))
    raise ValueError("unknown input kind %r" % kind)


def config(name: str) -> np.ndarray:
    return make(CONFIGS[name])


def dnf_width_for_density(d: float, terms: int, n: int) -> int:
    """Term width whose random DNF of ``terms`` terms has expected density
    about ``d``: 1 - (1 - 2^-w)^T = d."""
    q = 1.0 - (1.0 - d) ** (1.0 / terms)
    w = int(round(-math.log2(q))) if q > 0 else n
    return max(1, min(n, w))


def batch_specs(count: int = 8192, seed: int = 8192, nlo: int = 6, nhi: int = 16):
    """Mixed batch: n uniform in [nlo, nhi], density uniform in (0.1, 0.95);
    even jobs Bernoulli(d), odd jobs a random DNF of 10..100 terms whose width
    targets density d."""
    specs = []
    for j in range(count):
        r = u64_array(seed, 4, start=4 * j)
        n = nlo + int(r[0]) % (nhi - nlo + 1)
        d = 0.1 + 0.85 * (float(int(r[1]) >> 11) * 2.0**-53)
        s = int(r[3])
        if j % 2 == 0:
            specs.append(dict(n=n, kind="bernoulli", p=d, seed=s))
        else:
            T = 10 + int(r[2]) % 91
            w = dnf_width_for_density(d, T, n)
            specs.append(dict(n=n, kind="dnf", terms=T, wlo=w, whi=w, seed=s))
    return specs


SERVE_NS = (10, 14, 18, 22, 25)
SERVE_WEIGHTS = (0.4, 0.3, 0.15, 0.1, 0.05)


def serving_specs(count: int, seed: int = 25, ns=SERVE_NS, weights=SERVE_WEIGHTS):
    """Serving mix: n drawn from ``ns`` with ``weights``; half Bernoulli with
    p uniform in (0.5, 0.95), half random DNF as in ``batch_specs``."""
    cum = np.cumsum(np.asarray(weights, dtype=np.float64))
    cum /= cum[-1]
    specs = []
    for j in range(count):
        r = u64_array(seed, 5, start=5 * j)
        u = float(int(r[0]) >> 11) * 2.0**-53
        n = int(ns[int(np.searchsorted(cum, u, side="right"))])
        s = int(r[4])
        if int(r[1]) & 1 == 0:
            p = 0.5 + 0.45 * (float(int(r[2]) >> 11) * 2.0**-53)
            specs.append(dict(n=n, kind="bernoulli", p=p, seed=s))
        else:
            d = 0.5 + 0.45 * (float(int(r[2]) >> 11) * 2.0**-53)
            T = 10 + int(r[3]) % 91
            w = dnf_width_for_density(d, T, n)
            specs.append(dict(n=n, kind="dnf", terms=T, wlo=w, whi=w, seed=s))
    return specs

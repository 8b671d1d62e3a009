"""Shared helpers for the GPU tests (test code, not product code)."""
import functools
import sys

import numpy as np

import oracle
from paper_2302_10083_amd import inputs


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def context():
    from paper_2302_10083_amd import dqmc

    return dqmc.Context(0)


TILE_WORDS = 8 * 3**7  # digits 1..12: 2187 blocks of 8 words
SLOT_WORDS = TILE_WORDS + 8  # a tile and its 8 zero words, n > 12


def state_words(n):
    """Words of a state: 8 * 3^(n-5) up to n = 12, then 3^(n-12) slots."""
    return SLOT_WORDS * 3 ** (n - 12) if n > 12 else 8 * 3 ** max(n - 5, 0)


def h5_to_dense(n, state_u32):
    """Host conversion of a block state (uint32 words; cube rho at bit
    rho % 243 of the 256-bit block rho // 243; for n > 12 the blocks of digits
    13..n lie in slots of SLOT_WORDS words) into the exact 3^n-bit bitmap
    (uint64 words), written independently of the library's repack.  Checks
    that every padding bit and word is 0."""
    N = 3**n
    w = np.ascontiguousarray(state_u32, dtype=np.uint32)
    assert w.size == state_words(n)
    if n > 12:
        w = w.reshape(-1, SLOT_WORDS)
        if np.any(w[:, TILE_WORDS:]):
            raise AssertionError("slot padding words set")
        w = np.ascontiguousarray(w[:, :TILE_WORDS]).reshape(-1)
    assert w.size % 8 == 0
    bits = np.unpackbits(w.view(np.uint8), bitorder="little").reshape(-1, 256)
    if np.any(bits[:, 243:]):
        raise AssertionError("padding bits 243..255 set in a block")
    bits = bits[:, :243].reshape(-1)
    if np.any(bits[N:]):
        raise AssertionError("bits past 3^n set")
    bits = bits[:N]
    nbytes = ((N + 63) // 64) * 8
    packed = np.packbits(bits, bitorder="little")
    buf = np.zeros(nbytes, dtype=np.uint8)
    buf[: packed.size] = packed
    return buf.view(np.uint64)


def word_and_bit(rho, n):
    """State word and bit of cube rho in a state of n variables (numpy or
    torch integer arrays)."""
    blk, p = rho // 243, rho % 243
    w = 8 * blk + p // 32
    if n > 12:
        w = (w // TILE_WORDS) * SLOT_WORDS + w % TILE_WORDS
    return w, p % 32


def dev_to_u32(t):
    return t.cpu().numpy().view(np.uint32)


def dev_to_u64(t):
    return t.cpu().numpy().view(np.uint64)


def run_primes(n, tt, list_cap=None):
    """GPU prime computation; returns (state_dev, list_np, count)."""
    import torch

    ctx = context()
    ttd = ctx.tt_to_device(tt)
    if list_cap is None:
        list_cap = 3**n
    state, lst, count = ctx.primes(n, ttd, list_cap=min(list_cap, 3**n))
    torch.cuda.synchronize()
    c = int(count.item())
    k = min(c, list_cap)
    return state, dev_to_u64(lst[:k]) if k > 0 else np.zeros(0, dtype=np.uint64), c


def run_implicants(n, tt):
    import torch

    ctx = context()
    state = ctx.implicants(n, ctx.tt_to_device(tt))
    torch.cuda.synchronize()
    return state


def dense_of(n, state):
    import torch

    d = context().to_dense(n, state)
    torch.cuda.synchronize()
    return dev_to_u64(d)


@functools.lru_cache(maxsize=64)
def _oracle_cached(n, key):
    tt = _TT_STORE[key]
    return oracle.primes(n, tt)


_TT_STORE = {}


def oracle_primes(n, tt):
    key = (n, tt.tobytes())
    _TT_STORE[key] = tt
    return _oracle_cached(n, key)


def rho_of_binary(n, x):
    return sum(((x >> i) & 1) * 3**i for i in range(n))


def make_tt(n, kind, seed):
    if kind == "const0":
        return inputs.constant(n, 0)
    if kind == "const1":
        return inputs.constant(n, 1)
    if kind == "parity":
        return inputs.parity(n)
    if kind.startswith("bern"):
        return inputs.bernoulli(n, float(kind[4:]), seed)
    if kind.startswith("dnf"):
        T = int(kind[3:])
        return inputs.dnf(n, T, max(1, n // 4), max(2, n // 2), seed)
    raise ValueError(kind)


def relabel_tt(n, tt, sigma, c):
    """Truth table of g(y) = f(x) with x_i = y_sigma(i) XOR c_i."""
    bits = inputs.to_bits(n, tt)
    y = np.arange(1 << n, dtype=np.int64)
    x = np.zeros_like(y)
    for i in range(n):
        x |= (((y >> int(sigma[i])) & 1) ^ int(c[i])) << i
    return inputs.from_bits(n, bits[x])


def relabel_cubes(n, lst, sigma, c):
    """Sorted images of the cubes in the device tensor ``lst`` (cube indices of
    f) as cubes of g = relabel_tt(f): digit i moves to position sigma(i), and a
    binary digit is XORed with c_i.  Relabelling is an automorphism of the cube
    lattice, so it maps the primes of f onto the primes of g."""
    import torch

    out = torch.zeros_like(lst)
    p = 1
    for i in range(n):
        d = torch.div(lst, p, rounding_mode="floor") % 3
        out += torch.where(d == 2, d, d ^ int(c[i])) * (3 ** int(sigma[i]))
        p *= 3
        del d
    return torch.sort(out)[0]

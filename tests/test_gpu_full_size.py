"""Parity at the full benchmark sizes (n = 24, 25), where the oracle cannot
build whole bitmaps: sampled cubes are checked one by one with the oracle's
per-cube definitions, and closed-form families are checked exactly.  The
launch sequence is the one bench.py times (dqmc_primes with the default
plan)."""
import math

import numpy as np
import pytest

import oracle
from paper_2302_10083_amd import inputs

from _gpu_common import context, log, relabel_cubes, relabel_tt, word_and_bit

pytestmark = pytest.mark.gpu


def _bits_at(state, n, rhos):
    """State bits at the given cube indices (gathered on the device)."""
    import torch

    r = torch.from_numpy(np.asarray(rhos, dtype=np.int64)).to(state.device)
    w, b = word_and_bit(r, n)
    return ((state[w].to(torch.int64) >> b) & 1).cpu().numpy().astype(bool)


def _popcount_state(state):
    import torch

    total = 0
    chunk = 1 << 28
    for i in range(0, state.numel(), chunk):
        part = state[i:i + chunk]
        x = part.to(torch.int64) & 0xFFFFFFFF
        # SWAR popcount on int64 lanes holding 32-bit words
        x = x - ((x >> 1) & 0x5555555555555555)
        x = (x & 0x3333333333333333) + ((x >> 2) & 0x3333333333333333)
        x = (x + (x >> 4)) & 0x0F0F0F0F0F0F0F0F
        x = (x * 0x0101010101010101) >> 56
        total += int((x & 0xFF).sum().item())
        del part, x
    return total


def _run(n, tt, list_cap=None):
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    ttd = ctx.tt_to_device(tt)
    state = ctx.new_state(n)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    dqmc.dqmc_primes(ctx.ctx, n, ttd, state, None, 0, count)
    torch.cuda.synchronize()
    c = int(count.item())
    lst = None
    if list_cap is not None:
        # the same call bench.py times: bitmap and list in one dqmc_primes
        k = min(c, list_cap)
        lst = torch.empty(max(k, 1), dtype=torch.int64, device=ctx.torch_device)
        dqmc.dqmc_primes(ctx.ctx, n, ttd, state, lst, k, count)
        torch.cuda.synchronize()
        assert int(count.item()) == c
        lst = lst[:k]
    return state, lst, c


def test_config_c3_n24_sampled():
    import torch

    n = 24
    tt = inputs.config("c3_n24_dnf2000_noise")
    log("c3 n=24: primes")
    state, lst, c = _run(n, tt, list_cap=1 << 62)
    # the bitmap agrees with the per-cube definition on random cubes
    rng = np.random.default_rng(24)
    rhos = rng.integers(0, 3**n, size=400_000, dtype=np.int64)
    got = _bits_at(state, n, rhos)
    ref, _ = oracle.sample(n, tt, rhos.astype(np.uint64), "prime", 16)
    assert np.array_equal(got, ref), "%d mismatches" % int(np.count_nonzero(got != ref))
    # the list: strictly increasing, every entry set in the bitmap, count =
    # number of set bits, and sampled entries are primes by definition
    lh = lst.cpu().numpy()
    assert len(lh) == c
    assert np.all(np.diff(lh) > 0) and lh[0] >= 0 and lh[-1] < 3**n
    assert _bits_at(state, n, lh[:: max(1, len(lh) // 200_000)]).all()
    assert _popcount_state(state) == c
    pick = lh[:: max(1, len(lh) // 3000)]
    pr, _ = oracle.sample(n, tt, pick.astype(np.uint64), "prime", 16)
    assert pr.all()
    del state, lst
    torch.cuda.empty_cache()


def test_config_c3_n24_implicants_sampled():
    import torch

    n = 24
    tt = inputs.config("c3_n24_dnf2000_noise")
    ctx = context()
    state = ctx.implicants(n, ctx.tt_to_device(tt))
    torch.cuda.synchronize()
    rng = np.random.default_rng(2424)
    # bias towards low-weight cubes so that implicants are well represented
    d = rng.choice(3, size=(200_000, n), p=[0.4, 0.4, 0.2])
    rhos = (d * (3 ** np.arange(n, dtype=np.int64))[None, :]).sum(axis=1)
    got = _bits_at(state, n, rhos)
    ref, _ = oracle.sample(n, tt, rhos.astype(np.uint64), "implicant", 16)
    assert ref.any() and not ref.all()
    assert np.array_equal(got, ref)
    del state
    torch.cuda.empty_cache()


def _term_string(n, care, val):
    return "".join(("1" if (val >> i) & 1 else "0") if (care >> i) & 1 else "*" for i in range(n))


@pytest.mark.parametrize("n", [24, 25])
def test_constants_full_size(n):
    import torch

    state, lst, c = _run(n, inputs.constant(n, 1), list_cap=16)
    assert c == 1 and lst.cpu().numpy().tolist() == [3**n - 1]
    del state
    state, lst, c = _run(n, inputs.constant(n, 0), list_cap=16)
    assert c == 0
    del state
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [24, 25])
def test_unate_dnf_exact_full_size(n):
    """Unate DNF: the primes are exactly the terms left after absorption."""
    import torch

    terms = inputs.unate_terms(n, 300, 6, 14, 7000 + n)
    tt = inputs.from_terms(n, terms)
    ts = sorted(set(terms))
    keep = [t for t in ts if not any(u != t and (u[0] & t[0]) == u[0] for u in ts)]
    expected = sorted(oracle.rho_of(_term_string(n, c_, v_)) for c_, v_ in keep)
    log("unate n=%d: %d primes expected" % (n, len(expected)))
    state, lst, c = _run(n, tt, list_cap=len(expected) + 8)
    assert c == len(expected)
    assert lst.cpu().numpy().tolist() == expected
    del state
    torch.cuda.empty_cache()


def test_parity_n24():
    import torch

    n = 24
    state, lst, c = _run(n, inputs.parity(n), list_cap=1 << 24)
    assert c == 1 << (n - 1)
    lh = lst.cpu().numpy()
    assert np.all(np.diff(lh) > 0)
    # every listed cube is a minterm (no *) with an odd number of ones
    lh = lh[:: 37]
    digs = (lh[:, None] // (3 ** np.arange(n, dtype=np.int64))[None, :]) % 3
    assert not (digs == 2).any()
    assert np.all(digs.sum(axis=1) % 2 == 1)
    del state
    torch.cuda.empty_cache()


def test_interval_symmetric_n24_count_and_sample():
    """f = [a <= |x| <= b]: the primes are the cubes with a ones and b-a stars."""
    import torch

    n, a, b = 24, 9, 13
    state, _, c = _run(n, inputs.interval(n, a, b))
    assert c == math.comb(n, a) * math.comb(n - a, b - a)
    rng = np.random.default_rng(5)
    d = rng.choice(3, size=(300_000, n), p=[0.4, 0.4, 0.2])
    rhos = (d * (3 ** np.arange(n, dtype=np.int64))[None, :]).sum(axis=1)
    ones, stars = (d == 1).sum(axis=1), (d == 2).sum(axis=1)
    expect = (ones == a) & (ones + stars == b)
    assert expect.any()
    assert np.array_equal(_bits_at(state, n, rhos), expect)
    del state
    torch.cuda.empty_cache()


def test_n25_split_equals_whole_state_passes():
    """n = 25 runs the top-digit split by default; the whole-state passes
    (plan [5, 4, 4]) give the same bitmap, list and count."""
    import torch

    from paper_2302_10083_amd import dqmc

    n = 25
    ctx = context()
    tt = inputs.make(dict(n=25, kind="dnf+noise", terms=2000, wlo=6, whi=14, p=0.02, seed=25))
    ttd = ctx.tt_to_device(tt)
    state = ctx.new_state(n)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    h = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    results = []
    try:
        for mode in (1, 0):
            dqmc.dqmc_set_split(ctx.ctx, n, mode)
            dqmc.dqmc_primes(ctx.ctx, n, ttd, state, None, 0, count)
            torch.cuda.synchronize()
            c = int(count.item())
            lst = torch.empty(max(c, 1), dtype=torch.int64, device=ctx.torch_device)
            dqmc.dqmc_primes(ctx.ctx, n, ttd, state, lst, c, count)
            dqmc.dqmc_hash_words(ctx.ctx, state, state.numel(), h)
            lh = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
            dqmc.dqmc_hash_words(ctx.ctx, lst, 2 * c, lh)
            torch.cuda.synchronize()
            log("n=25 split=%d: %d primes" % (mode, c))
            results.append((c, int(h.item()), int(lh.item())))
            del lst
    finally:
        dqmc.dqmc_set_split(ctx.ctx, n, -1)
    assert results[0] == results[1]
    # and sampled cubes agree with the per-cube definition
    rng = np.random.default_rng(2525)
    rhos = rng.integers(0, 3**n, size=100_000, dtype=np.int64)
    ref, _ = oracle.sample(n, tt, rhos.astype(np.uint64), "prime", 16)
    assert np.array_equal(_bits_at(state, n, rhos), ref)
    del state
    torch.cuda.empty_cache()


def _all_primes(ctx, n, ttd, state, flags=0):
    """Count, then the whole sorted list, reusing one state buffer."""
    import torch

    from paper_2302_10083_amd import dqmc

    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    dqmc.dqmc_primes_ex(ctx.ctx, n, ttd, flags, state, None, 0, count)
    torch.cuda.synchronize()
    c = int(count.item())
    lst = torch.empty(max(c, 1), dtype=torch.int64, device=ctx.torch_device)
    dqmc.dqmc_primes_ex(ctx.ctx, n, ttd, flags, state, lst, c, count)
    torch.cuda.synchronize()
    assert int(count.item()) == c
    return lst[:c]


@pytest.mark.parametrize("n,flags", [(24, 0), (25, 0), (24, 1)])
def test_relabel_equivariance_full_list(n, flags):
    """Exact check of the whole prime list at the full sizes, GPU against GPU.
    Relabelling and negating variables is an automorphism of the cube lattice:
    if g(y) = f(x) with x_i = y_sigma(i) XOR c_i, then s is a prime of f iff
    the cube t with t_sigma(i) = s_i XOR c_i (and * kept) is a prime of g.
    The relabelling moves digits between the low tile, the column groups and
    (at n = 25) the split top digit, so an error tied to one pass or digit
    position breaks the equality.  flags = 1 (DQMC_NEGATE) checks the prime
    clauses the same way: NOT g is NOT f relabelled."""
    import torch

    ctx = context()
    spec = dict(inputs.CONFIGS["c3_n24_dnf2000_noise"])
    spec.update(n=n, seed=n)
    tt = inputs.make(spec)
    rng = np.random.default_rng(9000 + n)
    sigma = rng.permutation(n)
    c = rng.integers(0, 2, n)
    log("n=%d relabel sigma=%s c=%s" % (n, sigma.tolist(), c.tolist()))
    state = ctx.new_state(n)
    try:
        lf = _all_primes(ctx, n, ctx.tt_to_device(tt), state, flags)
        lg = _all_primes(ctx, n, ctx.tt_to_device(relabel_tt(n, tt, sigma, c)), state, flags)
        log("n=%d flags=%d: %d primes" % (n, flags, lf.numel()))
        assert lf.numel() == lg.numel() and lf.numel() > 0
        assert torch.equal(relabel_cubes(n, lf, sigma, c), lg)
    finally:
        del state
        torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", ["bern0.5", "bern0.9", "dnf300"])
def test_row_flags_equal_flag_free_plan_n24(kind):
    """At n = 24 the default plan [6, 6] passes row flags from the top group's
    pass to the reduce of digits 13..18 and chunk flags to the final reduce;
    the plan [4, 4, 4] runs without them.  Both give the same bitmap, count
    and list, on functions of three densities."""
    import torch

    from paper_2302_10083_amd import dqmc

    n = 24
    ctx = context()
    rng_seed = {"bern0.5": 2401, "bern0.9": 2402, "dnf300": 2403}[kind]
    if kind.startswith("bern"):
        tt = inputs.bernoulli(n, float(kind[4:]), rng_seed)
    else:
        tt = inputs.make({"n": n, "kind": "dnf", "terms": 300, "wlo": 4, "whi": 12, "seed": rng_seed})
    ttd = ctx.tt_to_device(tt)
    state = ctx.new_state(n)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    h = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    results = []
    try:
        for plan in ([], [4, 4, 4]):
            dqmc.dqmc_set_plan(ctx.ctx, n, plan)
            assert dqmc.dqmc_get_plan(ctx.ctx, n) == (plan or [6, 6])
            dqmc.dqmc_primes(ctx.ctx, n, ttd, state, None, 0, count)
            dqmc.dqmc_hash_words(ctx.ctx, state, state.numel(), h)
            torch.cuda.synchronize()
            c = int(count.item())
            lst = torch.empty(max(c, 1), dtype=torch.int64, device=ctx.torch_device)
            dqmc.dqmc_extract(ctx.ctx, n, state, lst, c, count)
            hl = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
            dqmc.dqmc_hash_words(ctx.ctx, lst, 2 * c, hl)
            torch.cuda.synchronize()
            results.append((c, int(h.item()), int(hl.item())))
            log("n=24 %s plan %s: %d primes" % (kind, plan or "[6, 6]", c))
            del lst
            state.fill_(0x7F7F7F7F)  # the second plan must overwrite everything it reads
    finally:
        dqmc.dqmc_set_plan(ctx.ctx, n, [])
    assert results[0] == results[1]
    del state
    torch.cuda.empty_cache()


def test_flag_units_bound_the_flagged_passes():
    """dqmc_flag_units after the flagged n = 24 call (c3 recipe): every figure
    is a whole number of rows, runs or chunks within its dense bound; the
    chunks the final bitmap holds a bit in (counted from the state) are within
    both the final reduce's store bound and the rows the reduce of digits
    13..18 was given (a chunk of a tile is a row segment of that pass); a
    flag-free plan reports nothing."""
    import torch

    from paper_2302_10083_amd import dqmc

    n, tiles, stride = 24, 3**12, 17504
    ctx = context()
    ttd = ctx.tt_to_device(inputs.config("c3_n24_dnf2000_noise"))
    state = ctx.new_state(n)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    try:
        dqmc.dqmc_primes(ctx.ctx, n, ttd, state, None, 0, count)
        torch.cuda.synchronize()
        u = dqmc.dqmc_flag_units(ctx.ctx)
        assert u["used"]
        rows, runs, stores = u["reduce13_rows_bytes"], u["final_runs_bytes"], u["final_store_bytes"]
        assert rows % 128 == 0 and 0 < rows <= 729 * 729 * (273 * 256 + 128)
        assert runs % 96 == 0 and 0 < runs <= tiles * 729 * 96
        assert stores % 32 == 0 and 0 < stores <= tiles * (273 * 256 + 96)
        # chunks of the final bitmap with a set bit: 273 of 64 words and one of 24 per tile
        S = state.view(tiles, stride)
        full = last = 0
        for t0 in range(0, tiles, 1 << 15):
            blk = S[t0:t0 + (1 << 15)]
            full += int(blk[:, :273 * 64].reshape(-1, 273, 64).ne(0).any(dim=2).sum())
            last += int(blk[:, 273 * 64:17496].ne(0).any(dim=1).sum())
        log("flag units: rows %.2f GB, runs %.2f GB, store bound %.2f GB; %d + %d non-zero chunks"
            % (rows / 1e9, runs / 1e9, stores / 1e9, full, last))
        assert full + last > 0
        assert 256 * full + 96 * last <= stores
        assert 256 * full + 128 * last <= rows
        dqmc.dqmc_set_plan(ctx.ctx, n, [4, 4, 4])
        dqmc.dqmc_primes(ctx.ctx, n, ttd, state, None, 0, count)
        torch.cuda.synchronize()
        u = dqmc.dqmc_flag_units(ctx.ctx)
        assert not u["used"] and u["reduce13_rows_bytes"] == u["final_runs_bytes"] == u["final_store_bytes"] == 0
    finally:
        dqmc.dqmc_set_plan(ctx.ctx, n, [])
        del state
        torch.cuda.empty_cache()

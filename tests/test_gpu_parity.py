"""Parity of the HIP path against the CPU oracle, element by element.

Every comparison is bit-exact: the prime set is unique (Sec. 2, definition of
prime implicant), so the bitmap, the sorted list and the count must all equal
the oracle's.
"""
import math
import random

import numpy as np
import pytest

import oracle
from paper_2302_10083_amd import inputs

from _gpu_common import (dense_of, dev_to_u32, log, make_tt, oracle_primes, rho_of_binary, run_implicants,
                         run_primes, h5_to_dense, context)

pytestmark = pytest.mark.gpu


def check_against_oracle(n, tt, what=""):
    log("parity n=%d %s" % (n, what))
    M, O, lst = oracle_primes(n, tt)
    state, glist, cnt = run_primes(n, tt)
    assert cnt == len(lst), "count %d vs oracle %d" % (cnt, len(lst))
    assert np.array_equal(glist, lst), "prime list differs"
    dense = dense_of(n, state)
    assert np.array_equal(dense, O), "prime bitmap differs"
    if n <= 16:
        assert np.array_equal(h5_to_dense(n, dev_to_u32(state)), O), "block state differs"
    mstate = run_implicants(n, tt)
    assert np.array_equal(dense_of(n, mstate), M), "implicant bitmap differs"
    return state


@pytest.mark.parametrize("n", list(range(0, 13)))
def test_single_tile_all_n(n):
    kinds = ["const0", "const1", "parity", "bern0.3", "bern0.7", "bern0.95", "dnf6"]
    for k, kind in enumerate(kinds):
        if n == 0 and kind.startswith("dnf"):
            continue
        check_against_oracle(n, make_tt(n, kind, 1000 + 17 * n + k), kind)


@pytest.mark.parametrize("n,kind,seed", [(4, "bern0.5", s) for s in range(20)] + [(7, "bern0.8", s) for s in range(10)])
def test_small_many_seeds(n, kind, seed):
    check_against_oracle(n, make_tt(n, kind, seed), kind)


@pytest.mark.parametrize("n", [13, 14, 15, 16, 17, 18])
def test_multi_pass_group_shapes(n):
    # n=13..16: one high group held in registers; 17, 18: one or two digits
    # across wavefronts
    for kind in ("bern0.9", "dnf40"):
        check_against_oracle(n, make_tt(n, kind, 3000 + n), kind)


def test_multi_pass_constants_and_parity_n15():
    for kind in ("const0", "const1", "parity", "bern0.5"):
        check_against_oracle(15, make_tt(15, kind, 15), kind)


@pytest.mark.parametrize("n", [19])
def test_two_high_groups(n):
    check_against_oracle(n, make_tt(n, "bern0.93", 19), "bern0.93")


def test_config_c1_n12():
    tt = inputs.config("c1_n12_bern05")
    check_against_oracle(12, tt, "c1")


def test_to_dense_matches_host_conversion():
    for n in (0, 1, 2, 3, 5, 9, 13):
        tt = make_tt(n, "bern0.8", 77 + n)
        state, _, _ = run_primes(n, tt)
        assert np.array_equal(dense_of(n, state), h5_to_dense(n, dev_to_u32(state)))


def test_capacity_overflow_keeps_smallest():
    n = 14
    tt = make_tt(n, "bern0.9", 5)
    _, _, lst = oracle_primes(n, tt)
    cap = len(lst) // 3
    _, glist, cnt = run_primes(n, tt, list_cap=cap)
    assert cnt == len(lst)
    assert np.array_equal(glist, lst[:cap])


def test_count_only_and_extract():
    import torch

    from paper_2302_10083_amd import dqmc

    n = 16
    tt = make_tt(n, "bern0.92", 6)
    _, _, lst = oracle_primes(n, tt)
    ctx = context()
    ttd = ctx.tt_to_device(tt)
    state = ctx.new_state(n)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    dqmc.dqmc_primes(ctx.ctx, n, ttd, state, None, 0, count)
    torch.cuda.synchronize()
    assert int(count.item()) == len(lst)
    glist, c2 = ctx.extract(n, state, len(lst) + 10)
    torch.cuda.synchronize()
    assert int(c2.item()) == len(lst)
    assert np.array_equal(glist[: len(lst)].cpu().numpy().view(np.uint64), lst)


def test_deterministic_repeat():
    n = 17
    tt = make_tt(n, "bern0.9", 8)
    s1, l1, c1 = run_primes(n, tt)
    d1 = dense_of(n, s1)
    s2, l2, c2 = run_primes(n, tt)
    assert c1 == c2 and np.array_equal(l1, l2) and np.array_equal(d1, dense_of(n, s2))


def test_bad_arguments_raise():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    tt = ctx.tt_to_device(make_tt(5, "bern0.5", 1))
    state = ctx.new_state(5)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    lib = dqmc.load()
    import ctypes

    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.dqmc_primes(ctx.ctx, 26, ctypes.c_void_p(tt.data_ptr()), ctypes.c_void_p(state.data_ptr()), None, 0,
                         ctypes.c_void_p(count.data_ptr()), st)
    assert rc == dqmc.DQMC_EINVAL and "outside" in dqmc.dqmc_last_error(ctx.ctx)
    rc = lib.dqmc_primes(ctx.ctx, 5, None, ctypes.c_void_p(state.data_ptr()), None, 0,
                         ctypes.c_void_p(count.data_ptr()), st)
    assert rc == dqmc.DQMC_EINVAL
    rc = lib.dqmc_primes(ctx.ctx, 5, ctypes.c_void_p(tt.data_ptr() + 2), ctypes.c_void_p(state.data_ptr()), None, 0,
                         ctypes.c_void_p(count.data_ptr()), st)
    assert rc == dqmc.DQMC_EINVAL


# ----------------------------------------------------------------------------
# metamorphic checks (GPU against GPU)


def test_variable_permutation_equivariance_n16():
    n = 16
    rng = random.Random(16)
    tt = make_tt(n, "bern0.9", 161)
    perm = list(range(n))
    rng.shuffle(perm)
    bits = inputs.to_bits(n, tt)
    x = np.arange(1 << n, dtype=np.int64)
    y = np.zeros_like(x)
    for i in range(n):
        y |= ((x >> i) & 1) << perm[i]
    ttp = inputs.from_bits(n, bits[y])
    _, l0, c0 = run_primes(n, tt)
    _, l1, c1 = run_primes(n, ttp)
    assert c0 == c1
    # map each prime of f through the permutation of digits
    p3 = np.array([3**i for i in range(n)], dtype=np.int64)
    digs = (l0.astype(np.int64)[:, None] // p3[None, :]) % 3
    mapped = (digs[:, perm] * p3[None, :]).sum(axis=1)
    assert np.array_equal(np.sort(mapped), l1.astype(np.int64))


# ----------------------------------------------------------------------------
# every plan gives the same primes; forcing plans exercises every column-pass
# shape (registers x wavefronts) in every mode at sizes the oracle handles


PLANS = [
    (16, [2, 2]), (16, [1, 3]), (16, [3, 1]), (17, [1, 1, 1, 1, 1]), (17, [5]),
    (18, [5, 1]), (18, [2, 2, 2]), (18, [1, 5]), (18, [6]),
    (19, [6, 1]), (19, [1, 6]), (19, [3, 4]), (19, [4, 3]), (19, [5, 2]),
]


@pytest.mark.parametrize("n,sizes", PLANS)
def test_forced_plans(n, sizes):
    from paper_2302_10083_amd import dqmc

    ctx = context()
    dqmc.dqmc_set_plan(ctx.ctx, n, sizes)
    try:
        assert dqmc.dqmc_get_plan(ctx.ctx, n) == sizes
        check_against_oracle(n, make_tt(n, "bern0.92", 500 + n + len(sizes)), "plan %s" % sizes)
    finally:
        dqmc.dqmc_set_plan(ctx.ctx, n, [])


def test_plan_validation():
    from paper_2302_10083_amd import dqmc

    ctx = context()
    for n, sizes in ((12, [1]), (16, [2, 1]), (16, [7, -3]), (20, [7, 1]), (26, [14])):
        with pytest.raises(dqmc.DqmcError):
            dqmc.dqmc_set_plan(ctx.ctx, n, sizes)
    assert dqmc.dqmc_get_plan(ctx.ctx, 24) == [6, 6]
    assert dqmc.dqmc_get_plan(ctx.ctx, 25) == [5, 4, 4]
    assert dqmc.dqmc_get_plan(ctx.ctx, 12) == []


@pytest.mark.parametrize("name", ["c2a_n20_bern09", "c2b_n20_dnf200"])
def test_config_n20_full_parity(name):
    tt = inputs.config(name)
    check_against_oracle(20, tt, name)


# the top-digit split of dqmc_primes: three (n-1)-variable slices in the
# thirds of the state, against the oracle at sizes it handles
@pytest.mark.parametrize("n", [13, 14, 15, 16, 17, 18, 19])
def test_top_digit_split_vs_oracle(n):
    from paper_2302_10083_amd import dqmc

    ctx = context()
    dqmc.dqmc_set_split(ctx.ctx, n, 1)
    try:
        assert dqmc.dqmc_get_split(ctx.ctx, n)
        kinds = ("bern0.9", "dnf40", "const1", "const0", "parity") if n <= 15 else ("bern0.93", "dnf60")
        for k, kind in enumerate(kinds):
            check_against_oracle(n, make_tt(n, kind, 9500 + 13 * n + k), "split " + kind)
    finally:
        dqmc.dqmc_set_split(ctx.ctx, n, -1)


@pytest.mark.parametrize("n", [13, 15, 17])
def test_top_digit_split_negate_vs_oracle(n):
    """The complement mode through the split: the primes of NOT f."""
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    tt = make_tt(n, "bern0.15", 9800 + n)
    _, _, ref = oracle_primes(n, ~tt)
    dqmc.dqmc_set_split(ctx.ctx, n, 1)
    try:
        _, lst, cnt = ctx.primes(n, ctx.tt_to_device(tt), flags=dqmc.DQMC_NEGATE)
        torch.cuda.synchronize()
        assert int(cnt.item()) == len(ref)
        assert np.array_equal(lst.cpu().numpy(), ref)
    finally:
        dqmc.dqmc_set_split(ctx.ctx, n, -1)


def test_top_digit_split_capacity_and_extract():
    """The split's list obeys the capacity rule, and its bitmap re-extracts."""
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    n = 15
    tt = make_tt(n, "bern0.9", 9660)
    _, _, ref = oracle_primes(n, tt)
    dqmc.dqmc_set_split(ctx.ctx, n, 1)
    try:
        cap = len(ref) // 3
        _, glist, cnt = run_primes(n, tt, list_cap=cap)
        assert cnt == len(ref)
        assert np.array_equal(glist, ref[:cap])
        state, _, _ = ctx.primes(n, ctx.tt_to_device(tt), list_cap=0)
        lst, c2 = ctx.extract(n, state, len(ref))
        torch.cuda.synchronize()
        assert int(c2.item()) == len(ref)
        assert np.array_equal(lst[: len(ref)].cpu().numpy(), ref)
    finally:
        dqmc.dqmc_set_split(ctx.ctx, n, -1)


def test_top_digit_split_is_one_level():
    """With the split on for n and n - 1, the thirds of n are not split again."""
    from paper_2302_10083_amd import dqmc

    ctx = context()
    dqmc.dqmc_set_split(ctx.ctx, 16, 1)
    dqmc.dqmc_set_split(ctx.ctx, 15, 1)
    try:
        check_against_oracle(16, make_tt(16, "bern0.9", 9611), "split 16 and 15")
    finally:
        dqmc.dqmc_set_split(ctx.ctx, 16, -1)
        dqmc.dqmc_set_split(ctx.ctx, 15, -1)


def test_top_digit_split_settings():
    from paper_2302_10083_amd import dqmc

    ctx = context()
    assert dqmc.dqmc_get_split(ctx.ctx, 25) and not dqmc.dqmc_get_split(ctx.ctx, 24)
    for n, mode in ((12, 1), (26, 1), (20, 2), (20, -2)):
        with pytest.raises(dqmc.DqmcError):
            dqmc.dqmc_set_split(ctx.ctx, n, mode)
    dqmc.dqmc_set_split(ctx.ctx, 25, 0)
    assert not dqmc.dqmc_get_split(ctx.ctx, 25)
    dqmc.dqmc_set_split(ctx.ctx, 25, -1)
    assert dqmc.dqmc_get_split(ctx.ctx, 25)

"""Sliced path (functions cut along their top t variables): the same prime
list and count as the oracle for every slice shape at small n, the same as
the single-state path at n = 24, and at n = 26 (a state of 377 GB, beyond one
GPU) exact closed forms plus per-cube definitions on sampled cubes."""
import ctypes
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2302_10083_amd import inputs

from _gpu_common import context, log, make_tt, oracle_primes, relabel_cubes, relabel_tt

pytestmark = pytest.mark.gpu


def _sliced(n, t, tt, list_cap=None, flags=0):
    import torch

    ctx = context()
    lst, count = ctx.sliced_primes(n, t, ctx.tt_to_device(tt), list_cap=list_cap, flags=flags)
    torch.cuda.synchronize()
    return lst, int(count.item())


# (n, t): slices with m = n - t of 0 (one cube), < 3 (one word), < 5 (one
# truth-table word), <= 12 (one tile), 13.. (column passes), two high groups,
# and the largest t
SHAPES = [(1, 1), (2, 1), (3, 2), (4, 3), (5, 5), (6, 2), (7, 3), (8, 3), (9, 1), (12, 4), (13, 1), (14, 1),
          (15, 2), (16, 3), (17, 4), (16, 1), (18, 2), (20, 5), (14, 8)]


@pytest.mark.parametrize("n,t", SHAPES)
def test_sliced_vs_oracle(n, t):
    kinds = ["bern0.5", "bern0.9", "const1", "const0", "parity"] + (["dnf30"] if n >= 4 else [])
    for k, kind in enumerate(kinds):
        tt = make_tt(n, kind, 8100 + 31 * n + 7 * t + k)
        log("sliced n=%d t=%d %s" % (n, t, kind))
        _, _, ref = oracle_primes(n, tt)
        lst, c = _sliced(n, t, tt)
        assert c == len(ref), "count %d vs oracle %d" % (c, len(ref))
        assert np.array_equal(lst.cpu().numpy(), ref), "prime list differs"


@pytest.mark.parametrize("n,t", [(5, 2), (11, 3), (15, 1), (17, 3)])
def test_sliced_negate_vs_oracle(n, t):
    tt = make_tt(n, "bern0.2", 8200 + n)
    _, _, ref = oracle_primes(n, ~tt)
    from paper_2302_10083_amd import dqmc

    lst, c = _sliced(n, t, tt, flags=dqmc.DQMC_NEGATE)
    assert c == len(ref)
    assert np.array_equal(lst.cpu().numpy(), ref)


def test_sliced_two_shapes_n19_agree_with_oracle():
    n = 19
    tt = inputs.dnf(n, 120, 3, 9, 8300)
    _, _, ref = oracle_primes(n, tt)
    for t in (1, 2, 6):
        lst, c = _sliced(n, t, tt)
        assert c == len(ref)
        assert np.array_equal(lst.cpu().numpy(), ref)


def test_sliced_capacity_and_count_only():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    n, t = 15, 2
    tt = make_tt(n, "bern0.8", 8400)
    _, _, ref = oracle_primes(n, tt)
    ttd = ctx.tt_to_device(tt)
    o, m = ctx.new_state(n - t), ctx.new_state(n - t)
    count = torch.full((1,), -5, dtype=torch.int64, device=ctx.torch_device)
    dqmc.dqmc_primes_sliced(ctx.ctx, n, t, ttd, 0, o, m, None, 0, count)
    torch.cuda.synchronize()
    assert int(count.item()) == len(ref)
    # a list shorter than the count keeps the smallest indices, over all slices
    for k in (0, 1, len(ref) // 7, len(ref) - 1):
        lst = torch.full((k + 4,), -1, dtype=torch.int64, device=ctx.torch_device)
        dqmc.dqmc_primes_sliced(ctx.ctx, n, t, ttd, 0, o, m, lst, k, count)
        torch.cuda.synchronize()
        assert int(count.item()) == len(ref)
        got = lst.cpu().numpy()
        assert np.array_equal(got[:k], ref[:k])
        assert (got[k:] == -1).all()  # nothing past the capacity


def test_sliced_bad_arguments():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    tt = ctx.tt_to_device(make_tt(12, "bern0.5", 1))
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    o, m = ctx.new_state(10), ctx.new_state(10)
    for n, t in ((12, 0), (12, 9), (12, 13), (31, 6), (27, 1)):
        with pytest.raises(dqmc.DqmcError):
            dqmc.dqmc_primes_sliced(ctx.ctx, n, t, tt, 0, o, m, None, 0, count)
    with pytest.raises(dqmc.DqmcError):
        dqmc.dqmc_primes_sliced(ctx.ctx, 12, 2, tt, 2, o, m, None, 0, count)  # unknown flag
    with pytest.raises(dqmc.DqmcError):
        dqmc.dqmc_primes_sliced(ctx.ctx, 12, 2, tt, 0, o, o, None, 0, count)  # overlapping states
    lib = dqmc.load()
    assert lib.dqmc_primes_sliced(ctx.ctx, 12, 2, None, 0, None, None, None, 0, None, None) == dqmc.DQMC_EINVAL
    # the context still works afterwards
    lst, c = _sliced(12, 2, make_tt(12, "bern0.5", 1))
    assert c == len(oracle_primes(12, make_tt(12, "bern0.5", 1))[2])


def test_sliced_matches_single_state_n24():
    """At n = 24 both paths fit: the sliced list equals dqmc_primes's."""
    import torch

    ctx = context()
    n = 24
    tt = inputs.config("c3_n24_dnf2000_noise")
    ttd = ctx.tt_to_device(tt)
    state, dl, dc = ctx.primes(n, ttd)
    torch.cuda.synchronize()
    del state
    torch.cuda.empty_cache()
    for t in (1, 3):
        log("sliced n=24 t=%d" % t)
        lst, c = _sliced(n, t, tt, list_cap=int(dc.item()) + 16)
        assert c == int(dc.item())
        assert torch.equal(lst[:c], dl)
        del lst
        torch.cuda.empty_cache()
    del dl


def _prime_from_minterm(n, tt, x, order):
    """Grow the minterm x into a prime: star digits one by one (in the given
    order) while the cube stays an implicant (per-cube definition).  No digit
    can be starred afterwards, since a digit refused earlier is refused on
    every larger cube."""
    d = [(x >> i) & 1 for i in range(n)]
    for i in order:
        keep = d[i]
        d[i] = 2
        rho = sum(v * 3**k for k, v in enumerate(d))
        ok, _ = oracle.sample(n, tt, np.array([rho], dtype=np.uint64), "implicant", 1)
        if not ok[0]:
            d[i] = keep
    return sum(v * 3**k for k, v in enumerate(d))


def test_sliced_n26_c3_recipe_sampled():
    """n = 26 with the n = 24 workload's recipe: sampled listed cubes are
    primes by definition; primes grown from random true minterms are listed;
    random cubes are listed exactly when they are prime."""
    import torch

    n, t = 26, 2
    tt = inputs.config("c3x_n26_dnf2000_noise")
    lst, c = _sliced(n, t, tt, list_cap=None)
    log("sliced n=26: %d primes" % c)
    assert c == lst.numel() and c > 0
    assert bool((lst[1:] > lst[:-1]).all()) and int(lst[0]) >= 0 and int(lst[-1]) < 3**n
    rng = np.random.default_rng(26)
    pick = lst[torch.from_numpy(rng.integers(0, c, size=2000)).to(lst.device)].cpu().numpy()
    ok, _ = oracle.sample(n, tt, pick.astype(np.uint64), "prime", 16)
    assert ok.all()

    def listed(rhos):
        r = torch.from_numpy(np.asarray(rhos, dtype=np.int64)).to(lst.device)
        i = torch.searchsorted(lst, r).clamp(max=c - 1)
        return (lst[i] == r).cpu().numpy()

    bits = np.unpackbits(tt.view(np.uint8), bitorder="little")
    ones = np.flatnonzero(bits)
    grown = []
    for x in rng.choice(ones, size=40, replace=False):
        grown.append(_prime_from_minterm(n, tt, int(x), rng.permutation(n).tolist()))
    assert listed(grown).all()
    d = rng.choice(3, size=(200_000, n), p=[0.4, 0.4, 0.2])
    rhos = (d * (3 ** np.arange(n, dtype=np.int64))[None, :]).sum(axis=1)
    ref, _ = oracle.sample(n, tt, rhos.astype(np.uint64), "prime", 16)
    assert np.array_equal(listed(rhos), ref)
    del lst
    torch.cuda.empty_cache()


def test_sliced_n26_relabel_equivariance_full_list():
    """The whole n = 26 prime list, exactly, GPU against GPU: a random
    relabelling and negation of the variables (g(y) = f(x) with
    x_i = y_sigma(i) XOR c_i) maps the primes of f onto those of g.  f runs
    with two slice variables, g with three, so the relabelling also moves
    variables into and out of the slice digits."""
    import torch

    n = 26
    tt = inputs.config("c3x_n26_dnf2000_noise")
    rng = np.random.default_rng(9026)
    sigma = rng.permutation(n)
    c = rng.integers(0, 2, n)
    log("sliced n=26 relabel sigma=%s c=%s" % (sigma.tolist(), c.tolist()))
    lf, cf = _sliced(n, 2, tt)
    lg, cg = _sliced(n, 3, relabel_tt(n, tt, sigma, c))
    log("sliced n=26: %d / %d primes" % (cf, cg))
    assert cf == cg == lf.numel() == lg.numel() and cf > 0
    assert torch.equal(relabel_cubes(n, lf, sigma, c), lg)
    del lf, lg
    torch.cuda.empty_cache()

@pytest.mark.parametrize("t", [1, 2])
def test_sliced_n26_interval_exact(t):
    """f = [a <= |x| <= b]: the primes are the cubes with a ones and b-a
    stars (exact list for a small family, count for a large one)."""
    import torch

    n = 26
    torch.cuda.empty_cache()
    try:
        lst, c = _sliced(n, t, inputs.interval(n, 24, 26), list_cap=400)
    except torch.cuda.OutOfMemoryError:
        if t == 1:  # two n = 25 slice states: 251 GB
            torch.cuda.empty_cache()
            pytest.skip("two n = 25 slice states do not fit in free device memory")
        raise
    expect = []
    for stars in itertools.combinations(range(n), 2):
        expect.append(sum((2 if i in stars else 1) * 3**i for i in range(n)))
    assert c == len(expect) == 325
    assert lst[:c].cpu().numpy().tolist() == sorted(expect)
    if t == 2:
        _, c = _sliced(n, t, inputs.interval(n, 10, 20), list_cap=0)
        assert c == math.comb(26, 10) * math.comb(16, 10)
    torch.cuda.empty_cache()


def test_sliced_n26_unate_exact():
    """Unate DNF: the primes are exactly the terms left after absorption."""
    import torch

    n = 26
    terms = inputs.unate_terms(n, 400, 6, 15, 8600)
    ts = sorted(set(terms))
    keep = [u for u in ts if not any(v != u and (v[0] & u[0]) == v[0] for v in ts)]
    expected = sorted(sum(((v_ >> i) & 1 if (c_ >> i) & 1 else 2) * 3**i for i in range(n)) for c_, v_ in keep)
    lst, c = _sliced(n, 3, inputs.from_terms(n, terms), list_cap=len(expected) + 8)
    assert c == len(expected)
    assert lst[:c].cpu().numpy().tolist() == expected
    torch.cuda.empty_cache()


def test_sliced_with_split_slices_vs_oracle():
    """Slices whose size has the top-digit split switched on are computed as
    three thirds (one level: the thirds themselves are not split again)."""
    from paper_2302_10083_amd import dqmc

    ctx = context()
    for m in (13, 14, 15):
        dqmc.dqmc_set_split(ctx.ctx, m, 1)
    try:
        for n, t, kind in ((15, 1, "bern0.9"), (16, 2, "dnf40"), (16, 1, "bern0.85"), (17, 3, "bern0.95")):
            tt = make_tt(n, kind, 9700 + n + t)
            log("sliced n=%d t=%d with split slices" % (n, t))
            _, _, ref = oracle_primes(n, tt)
            lst, c = _sliced(n, t, tt)
            assert c == len(ref)
            assert np.array_equal(lst.cpu().numpy(), ref)
    finally:
        for m in (13, 14, 15):
            dqmc.dqmc_set_split(ctx.ctx, m, -1)


def test_sliced_n27_interval_exact():
    """n = 27 (the paper's largest dense run) as 27 slices of 24 variables:
    f = [25 <= |x| <= 27] has exactly the 351 primes with 25 ones and 2 stars."""
    import torch

    n = 27
    lst, c = _sliced(n, 3, inputs.interval(n, 25, 27), list_cap=400)
    log("sliced n=27: %d primes" % c)
    expect = sorted(sum((2 if i in st else 1) * 3**i for i in range(n)) for st in itertools.combinations(range(n), 2))
    assert c == len(expect) == 351
    assert lst[:c].cpu().numpy().tolist() == expect
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,t,nm", [(12, 3, 2), (14, 4, 3), (16, 3, 4), (13, 2, 2), (15, 5, 6)])
def test_sliced_multi_states_vs_oracle(n, t, nm):
    """Several implicant states: fewer recomputed bitmaps, the same primes."""
    ctx = context()
    tt = make_tt(n, "bern0.9", 10100 + 7 * n + t + nm)
    _, _, ref = oracle_primes(n, tt)
    lst, count = ctx.sliced_primes(n, t, ctx.tt_to_device(tt), n_m=nm)
    import torch

    torch.cuda.synchronize()
    assert int(count.item()) == len(ref)
    assert np.array_equal(lst.cpu().numpy(), ref)


def test_sliced_multi_bad_arguments():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    n, t = 12, 2
    tt = ctx.tt_to_device(make_tt(n, "bern0.5", 3))
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    o = ctx.new_state(n - t)
    ms = [ctx.new_state(n - t) for _ in range(17)]
    with pytest.raises(dqmc.DqmcError):
        dqmc.dqmc_primes_sliced_multi(ctx.ctx, n, t, tt, 0, o, [], None, 0, count)  # no state
    with pytest.raises(dqmc.DqmcError):
        dqmc.dqmc_primes_sliced_multi(ctx.ctx, n, t, tt, 0, o, ms, None, 0, count)  # too many
    with pytest.raises(dqmc.DqmcError):
        dqmc.dqmc_primes_sliced_multi(ctx.ctx, n, t, tt, 0, o, [ms[0], ms[0]], None, 0, count)  # overlap
    with pytest.raises(dqmc.DqmcError):
        dqmc.dqmc_primes_sliced_multi(ctx.ctx, n, t, tt, 0, o, [ms[0], o], None, 0, count)  # overlap with o
    lib = dqmc.load()
    arr = (ctypes.c_void_p * 2)(ctypes.c_void_p(ms[0].data_ptr()).value, None)
    assert lib.dqmc_primes_sliced_multi(ctx.ctx, n, t, ctypes.c_void_p(tt.data_ptr()), 0,
                                        ctypes.c_void_p(o.data_ptr()), arr, 2, None, 0,
                                        ctypes.c_void_p(count.data_ptr()), None) == dqmc.DQMC_EINVAL
    # the context still works afterwards
    dqmc.dqmc_primes_sliced_multi(ctx.ctx, n, t, tt, 0, o, ms[:3], None, 0, count)
    torch.cuda.synchronize()
    assert int(count.item()) == len(oracle_primes(n, make_tt(n, "bern0.5", 3))[2])

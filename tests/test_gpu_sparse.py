"""Sparse path (level-by-level QMC with hash sets): the same prime list and
count as the oracle and as the dense path, workspace handling, and sizes past
the dense path's range (n = 26..31) checked against closed forms and the
per-cube definitions."""
import numpy as np
import pytest

import oracle
from paper_2302_10083_amd import inputs

from _gpu_common import context, log

pytestmark = pytest.mark.gpu


def _sparse(n, tt):
    ctx = context()
    lst, count = ctx.sparse_primes(n, ctx.tt_to_device(tt))
    return lst.cpu().numpy(), int(count.item())


CASES = [(0, 0.7), (1, 0.5), (2, 0.5), (3, 0.6), (4, 0.3), (5, 0.5), (6, 0.1), (8, 0.3), (9, 0.95), (10, 0.5),
         (11, 0.25), (12, 0.6), (13, 0.05), (14, 0.4)]


@pytest.mark.parametrize("n,p", CASES)
def test_sparse_vs_oracle_bernoulli(n, p):
    tt = inputs.bernoulli(n, p, 5100 + n)
    got, c = _sparse(n, tt)
    _, _, ref = oracle.primes(n, tt)
    assert c == len(ref)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,terms,wlo,whi", [(9, 12, 2, 6), (12, 40, 3, 8), (15, 60, 5, 12)])
def test_sparse_vs_oracle_dnf(n, terms, wlo, whi):
    tt = inputs.dnf(n, terms, wlo, whi, 5200 + n)
    got, c = _sparse(n, tt)
    _, _, ref = oracle.primes(n, tt)
    assert c == len(ref)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,p", [(18, 0.25), (20, 0.5), (20, 0.1)])
def test_sparse_vs_dense(n, p):
    import torch

    ctx = context()
    tt = inputs.bernoulli(n, p, 5300 + n)
    got, c = _sparse(n, tt)
    _, dl, dc = ctx.primes(n, ctx.tt_to_device(tt))
    torch.cuda.synchronize()
    assert c == int(dc.item())
    assert np.array_equal(got, dl.cpu().numpy())


def test_sparse_workspace_too_small_then_enough():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    n = 16
    tt = inputs.bernoulli(n, 0.4, 5400)
    ttd = ctx.tt_to_device(tt)
    count = torch.full((1,), -7, dtype=torch.int64, device=ctx.torch_device)
    small = torch.empty(64 << 10, dtype=torch.uint8, device=ctx.torch_device)
    rc, lv, npr = dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, None, 0, count, small)
    assert rc == dqmc.DQMC_ENOMEM and lv > 0
    torch.cuda.synchronize()
    assert int(count.item()) == -7  # nothing written on failure
    # grow until the reported sizes are complete, then the sized workspace works
    for _ in range(4):
        work = torch.empty(dqmc.dqmc_sparse_workspace_bytes(n, max(lv, 1), max(npr, 1)), dtype=torch.uint8,
                           device=ctx.torch_device)
        rc, lv2, npr2 = dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, None, 0, count, work)
        if rc == dqmc.DQMC_OK:
            break
        lv, npr = max(lv, lv2) * 2, max(npr, npr2) * 2
    assert rc == dqmc.DQMC_OK
    _, _, ref = oracle.primes(n, tt)
    assert int(count.item()) == len(ref)
    # and the exact sizes it reports are enough on their own
    exact = torch.empty(dqmc.dqmc_sparse_workspace_bytes(n, lv2, npr2), dtype=torch.uint8, device=ctx.torch_device)
    lst = torch.empty(len(ref), dtype=torch.int64, device=ctx.torch_device)
    rc, _, _ = dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, lst, len(ref), count, exact)
    assert rc == dqmc.DQMC_OK
    assert np.array_equal(lst.cpu().numpy(), ref)


def test_sparse_capacity_and_bad_args():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    n = 12
    tt = inputs.bernoulli(n, 0.5, 5500)
    ttd = ctx.tt_to_device(tt)
    _, _, ref = oracle.primes(n, tt)
    work = torch.empty(64 << 20, dtype=torch.uint8, device=ctx.torch_device)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    k = len(ref) // 3
    lst = torch.empty(k, dtype=torch.int64, device=ctx.torch_device)
    rc, _, _ = dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, lst, k, count, work)
    assert rc == dqmc.DQMC_OK
    assert int(count.item()) == len(ref)
    assert np.array_equal(lst.cpu().numpy(), ref[:k])
    with pytest.raises(dqmc.DqmcError):
        dqmc.dqmc_sparse_primes(ctx.ctx, 32, ttd, None, 0, count, work)
    with pytest.raises(dqmc.DqmcError):
        dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, None, 0, count, work[1:])  # misaligned workspace


def _term_rho(n, care, val):
    r = 0
    for i in reversed(range(n)):
        r = 3 * r + (((val >> i) & 1) if (care >> i) & 1 else 2)
    return r


@pytest.mark.parametrize("n,terms,wlo,whi", [(27, 400, 19, 25), (31, 300, 24, 29)])
def test_sparse_unate_beyond_dense_range(n, terms, wlo, whi):
    """Unate DNF: the primes are exactly the terms left after absorption."""
    ts = sorted(set(inputs.unate_terms(n, terms, wlo, whi, 5600 + n)))
    keep = [t for t in ts if not any(u != t and (u[0] & t[0]) == u[0] for u in ts)]
    expected = sorted(_term_rho(n, c_, v_) for c_, v_ in keep)
    log("sparse unate n=%d: %d primes expected" % (n, len(expected)))
    got, c = _sparse(n, inputs.from_terms(n, ts))
    assert c == len(expected)
    assert got.tolist() == expected


def test_sparse_n26_bernoulli_definitions():
    """n = 26 at density 0.002: every listed cube satisfies the per-cube
    prime definition, and sampled true minterms are covered by the list."""
    n = 26
    tt = inputs.bernoulli(n, 0.002, 5700)
    got, c = _sparse(n, tt)
    log("sparse n=26: %d primes" % c)
    assert c == len(got) and np.all(np.diff(got) > 0)
    rng = np.random.default_rng(26)
    pick = got[rng.integers(0, c, size=min(c, 3000))]
    ok, _ = oracle.sample(n, tt, pick.astype(np.uint64), "prime")
    assert ok.all()
    # coverage: random true minterms lie in some listed prime
    digs = (got[:, None] // (3 ** np.arange(n, dtype=np.int64))[None, :]) % 3
    care = ((digs != 2) * (1 << np.arange(n, dtype=np.int64))).sum(axis=1)
    val = ((digs == 1) * (1 << np.arange(n, dtype=np.int64))).sum(axis=1)
    bits = np.unpackbits(tt.view(np.uint8), bitorder="little")
    ones = np.flatnonzero(bits)
    for x in rng.choice(ones, size=300, replace=False):
        assert np.any((x & care) == val)

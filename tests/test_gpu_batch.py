"""Batched prime implicants (device-resident job array, planned on the
device): every job's result equals what dqmc_primes gives for it
alone and the oracle's, malformed jobs fail alone with their status set on
the device, and a captured graph of the batch replays correctly."""
import numpy as np
import pytest

import oracle
from paper_2302_10083_amd import inputs

from _gpu_common import context, log

pytestmark = pytest.mark.gpu


def _alloc_job(ctx, n, tt, cap=None):
    import torch

    from paper_2302_10083_amd import dqmc

    cap = 3**n if cap is None else cap
    return dict(n=n, tt=ctx.tt_to_device(tt), state=ctx.new_state(n),
                list=torch.empty(max(cap, 1), dtype=torch.int64, device=ctx.torch_device), list_cap=cap,
                count=torch.full((1,), -1, dtype=torch.int64, device=ctx.torch_device))


def _single(ctx, n, tt):
    import torch

    state, lst, count = ctx.primes(n, ctx.tt_to_device(tt), list_cap=3**n)
    torch.cuda.synchronize()
    c = int(count.item())
    return state, lst[:c].cpu().numpy(), c


def _job_result(j):
    c = int(j["count"].item())
    k = min(c, j["list_cap"])
    return j["state"], j["list"][:k].cpu().numpy(), c


def _mixed_specs(count, seed, nlo=0, nhi=16):
    specs = inputs.batch_specs(count, seed=seed, nlo=max(nlo, 6), nhi=nhi)
    # also the degenerate sizes
    for n in range(0, 6):
        specs.append(dict(n=n, kind="bernoulli", p=0.7, seed=seed + n))
    return specs


def test_batch_matches_single_and_oracle():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    specs = _mixed_specs(120, 77)
    specs += [dict(n=13, kind="dnf", terms=30, wlo=3, whi=6, seed=13)]
    tts = [inputs.make(s) for s in specs]
    jobs = [_alloc_job(ctx, s["n"], tt) for s, tt in zip(specs, tts)]
    status = dqmc.dqmc_primes_batch(ctx.ctx, jobs)
    assert status == [0] * len(jobs)
    for s, tt, j in zip(specs, tts, jobs):
        n = s["n"]
        bstate, blist, bc = _job_result(j)
        sstate, slist, sc = _single(ctx, n, tt)
        assert bc == sc, (n, bc, sc)
        assert np.array_equal(blist, slist)
        assert torch.equal(bstate, sstate)
        if n <= 16:
            _, _, ref = oracle.primes(n, tt)
            assert np.array_equal(blist, ref), n


def test_batch_malformed_jobs_fail_alone():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    good = [dict(n=n, kind="bernoulli", p=0.8, seed=900 + n) for n in (8, 14, 11)]
    tts = [inputs.make(s) for s in good]
    jobs = [_alloc_job(ctx, s["n"], tt) for s, tt in zip(good, tts)]
    bad_n = dict(jobs[0])
    bad_n["n"] = 26
    big_n = dict(jobs[0])
    big_n["n"] = 17  # batches take n <= 16
    bad_state = dict(n=14, tt=jobs[1]["tt"], state=None, list=None, list_cap=0, count=jobs[1]["count"])
    allj = [jobs[0], bad_n, jobs[1], bad_state, big_n, jobs[2]]
    status = dqmc.dqmc_primes_batch(ctx.ctx, allj)
    assert status == [0, dqmc.DQMC_EINVAL, 0, dqmc.DQMC_EINVAL, dqmc.DQMC_EINVAL, 0]
    for s, tt, j in zip(good, tts, jobs):
        _, blist, bc = _job_result(j)
        _, _, lst = oracle.primes(s["n"], tt)
        assert bc == len(lst) and np.array_equal(blist, lst)


def test_batch_capacity_and_count_only():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    n = 14
    tt = inputs.bernoulli(n, 0.9, 4242)
    _, _, ref = oracle.primes(n, tt)
    j1 = _alloc_job(ctx, n, tt, cap=len(ref) // 2)
    j2 = dict(_alloc_job(ctx, n, tt), list=None, list_cap=0)
    status = dqmc.dqmc_primes_batch(ctx.ctx, [j1, j2])
    assert status == [0, 0]
    _, l1, c1 = _job_result(j1)
    assert c1 == len(ref) and np.array_equal(l1, ref[: len(ref) // 2])
    assert int(j2["count"].item()) == len(ref)


def test_batch_plan_graph_replay():
    """Capture dqmc_batch_run in a graph and replay it several times with
    eager work in between; every replay must reproduce the eager results."""
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    specs = _mixed_specs(60, 99)
    tts = [inputs.make(s) for s in specs]
    jobs = [_alloc_job(ctx, s["n"], tt) for s, tt in zip(specs, tts)]
    plan = dqmc.Batch(ctx.ctx, jobs)
    plan.run()
    torch.cuda.synchronize()
    assert plan.status == [0] * len(jobs)
    eager = [(j["state"].clone(), j["list"][: int(j["count"].item())].clone(), int(j["count"].item())) for j in jobs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.run()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for j in jobs:
            j["state"].fill_(0x5A5A5A5)
            j["count"].fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (es, el, ec), j in zip(eager, jobs):
            assert int(j["count"].item()) == ec, rep
            assert torch.equal(j["state"], es), rep
            assert torch.equal(j["list"][:ec], el), rep
        # eager work between replays
        x = torch.arange(1 << 20, device=ctx.torch_device).sum()
        torch.cuda.synchronize()
    del g
    plan.close()


def test_batch_plan_rejects_changed_sizes():
    """A plan's launches are sized for the jobs' n at creation: a run after a
    job's n changed must do nothing but reject every job; restoring the n
    restores the results."""
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    specs = [dict(n=n, kind="bernoulli", p=0.8, seed=700 + n) for n in (9, 13, 15, 10)]
    tts = [inputs.make(s) for s in specs]
    jobs = [_alloc_job(ctx, s["n"], tt) for s, tt in zip(specs, tts)]
    plan = dqmc.Batch(ctx.ctx, jobs)
    words = plan.table.view(torch.int32)  # dqmc_job: 12 int32 words, n first
    per = words.numel() // len(jobs)
    words[0] = 8  # job 0: n = 9 -> 8 (its buffers are large enough)
    for j in jobs:
        j["count"].fill_(-7)
    plan.run()
    assert plan.status == [dqmc.DQMC_EINVAL] * len(jobs)
    assert all(int(j["count"].item()) == -7 for j in jobs)
    words[0] = 9
    plan.run()
    assert plan.status == [0] * len(jobs)
    for s, tt, j in zip(specs, tts, jobs):
        _, blist, bc = _job_result(j)
        _, _, ref = oracle.primes(s["n"], tt)
        assert bc == len(ref) and np.array_equal(blist, ref)
    assert per == 12
    plan.close()


@pytest.mark.parametrize("col_cap,order", [(0, 0), (0, 1), (1, 0), (3, 1)])
def test_batch_configs_same_results(col_cap, order):
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    specs = _mixed_specs(40, 31 + col_cap + order)
    tts = [inputs.make(s) for s in specs]
    jobs = [_alloc_job(ctx, s["n"], tt) for s, tt in zip(specs, tts)]
    plan = dqmc.Batch(ctx.ctx, jobs)
    plan.config(col_cap, order)
    plan.run()
    torch.cuda.synchronize()
    for s, tt, j in zip(specs, tts, jobs):
        _, blist, bc = _job_result(j)
        _, slist, sc = _single(ctx, s["n"], tt)
        assert bc == sc and np.array_equal(blist, slist)
    plan.close()


def test_config_c4_batch_8192_vs_single():
    """The 8192-function batch workload: every job equal to its single call,
    and a sample of jobs equal to the oracle."""
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    specs = inputs.batch_specs(8192, seed=8192)
    log("c4: generating %d truth tables" % len(specs))
    tts = [inputs.make(s) for s in specs]
    jobs = [_alloc_job(ctx, s["n"], tt, cap=min(3**s["n"], 1 << 22)) for s, tt in zip(specs, tts)]
    log("c4: batch run")
    status = dqmc.dqmc_primes_batch(ctx.ctx, jobs)
    assert status == [0] * len(jobs)
    log("c4: single calls")
    for i, (s, tt, j) in enumerate(zip(specs, tts, jobs)):
        n = s["n"]
        st = ctx.new_state(n)
        cnt = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
        lst = torch.empty(j["list_cap"], dtype=torch.int64, device=ctx.torch_device)
        dqmc.dqmc_primes(ctx.ctx, n, j["tt"], st, lst, j["list_cap"], cnt)
        assert torch.equal(st, j["state"]), i
        c = int(cnt.item())
        assert c == int(j["count"].item()), i
        k = min(c, j["list_cap"])
        assert torch.equal(lst[:k], j["list"][:k]), i
    rng = np.random.default_rng(4)
    pick = list(rng.choice(len(specs), size=40, replace=False))
    # and some of the largest jobs (n = 15, 16: the tile-parallel path)
    pick += [i for i, s in enumerate(specs) if s["n"] >= 15][:12]
    for i in pick:
        n = specs[i]["n"]
        _, _, ref = oracle.primes(n, tts[i])
        _, blist, bc = _job_result(jobs[i])
        assert bc == len(ref) and np.array_equal(blist, ref[: len(blist)])

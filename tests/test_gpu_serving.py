"""Serving loop: every request's result is identical alone and in the mix
(count, prime bitmap and list, compared through device hashes), every served
list with n <= 18 equals the oracle's, admission
never exceeds the memory budget, and bad requests fail alone."""
import time

import numpy as np
import pytest

import oracle
from paper_2302_10083_amd import inputs

from _gpu_common import context, log, state_words

pytestmark = pytest.mark.gpu


def list_reserve(n):
    return min(3**n, max(1 << 18, 3 ** max(n - 3, 0) // 16))


def footprint(n):
    tt = 1 if n <= 5 else 1 << (n - 5)
    a = lambda x: (x + 255) // 256 * 256
    return a(4 * state_words(n)) + a(8 * list_reserve(n)) + a(4 * tt) + 256


def _hash(ctx, addr, nwords):
    import torch

    from paper_2302_10083_amd import dqmc

    out = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    dqmc.dqmc_hash_words(ctx.ctx, addr, nwords, out)
    torch.cuda.synchronize()
    return int(out.item())


def _alone(n, tt):
    """(count, state hash, list hash) of dqmc_primes alone, with the same list
    capacity the server reserves."""
    import torch

    ctx = context()
    cap = list_reserve(n)
    state, lst, count = ctx.primes(n, ctx.tt_to_device(tt), list_cap=cap)
    torch.cuda.synchronize()
    c = int(count.item())
    k = min(c, cap)
    res = (c, _hash(ctx, state, state.numel()), _hash(ctx, lst, 2 * k))
    del state, lst
    torch.cuda.empty_cache()
    return res


def _served(srv, jid):
    ctx = context()
    r = srv.wait(jid)
    assert r["status"] == 0
    n = r["n"]
    sw = state_words(n)
    return r, (r["count"], _hash(ctx, r["state"], sw), _hash(ctx, r["list"], 2 * r["listed"]))


def test_alone_equals_mix():
    from paper_2302_10083_amd import dqmc

    specs = inputs.serving_specs(48, seed=2525)
    # at most two of the largest requests keep the test short
    big = [i for i, s in enumerate(specs) if s["n"] == 25]
    for i in big[2:]:
        specs[i] = dict(specs[i], n=22)
    tts = [inputs.make(s) for s in specs]
    rng = np.random.default_rng(3)
    with dqmc.Server(0) as srv:
        ids = []
        for s, tt in zip(specs, tts):
            ids.append(srv.submit(s["n"], tt))
            time.sleep(float(rng.exponential(0.002)))
        served = []
        for jid, s, tt in zip(ids, specs, tts):
            r, key = _served(srv, jid)
            if s["n"] <= 18:
                lst = srv.read(jid, r["listed"])
                _, _, ref = oracle.primes(s["n"], tt)
                assert r["count"] == len(ref) and np.array_equal(lst, ref[: len(lst)])
            srv.release(jid)
            served.append(key)
    log("served %d requests; checking alone" % len(ids))
    for i, (s, tt, key) in enumerate(zip(specs, tts, served)):
        if i % 8 == 0:
            log("alone check %d/%d (n=%d)" % (i, len(specs), s["n"]))
        assert _alone(s["n"], tt) == key, s


def test_admission_respects_budget():
    from paper_2302_10083_amd import dqmc

    budget = 2 * footprint(22) + 40 * footprint(10)
    specs = [dict(n=22, kind="bernoulli", p=0.9, seed=220 + i) for i in range(5)]
    specs += [dict(n=10, kind="bernoulli", p=0.7, seed=100 + i) for i in range(30)]
    tts = [inputs.make(s) for s in specs]
    with dqmc.Server(0, budget=budget, slots=4) as srv:
        ids = [srv.submit(s["n"], tt) for s, tt in zip(specs, tts)]
        res = []
        for j in ids:  # results hold their memory until released
            res.append(srv.wait(j))
            srv.release(j)
        keys = [(r["count"],) for r in res]
    # at every admission instant the admitted-and-unfinished footprints fit
    events = sorted([(r["t_admit"], footprint(r["n"])) for r in res] + [(r["t_done"], -footprint(r["n"])) for r in res],
                    key=lambda e: (e[0], e[1]))
    used = peak = 0
    for _, d in events:
        used += d
        peak = max(peak, used)
    assert peak <= budget
    for s, tt, k in zip(specs, tts, keys):
        assert _alone(s["n"], tt)[0] == k[0]


def test_wait_reports_blocked_job():
    """A job that cannot be admitted while unreleased results hold the budget
    is reported to the waiter, and runs once a result is released."""
    from paper_2302_10083_amd import dqmc

    with dqmc.Server(0, budget=footprint(18) + footprint(16)) as srv:
        a = srv.submit(18, inputs.bernoulli(18, 0.9, 1))
        b = srv.submit(18, inputs.bernoulli(18, 0.9, 2))
        srv.wait(a)
        with pytest.raises(dqmc.DqmcError) as e:
            srv.wait(b)
        assert e.value.code == dqmc.DQMC_ENOMEM
        srv.release(a)
        rb = srv.wait(b)
        assert rb["status"] == 0
        srv.release(b)


def test_bad_requests_fail_alone():
    from paper_2302_10083_amd import dqmc

    with dqmc.Server(0, budget=footprint(16) * 4) as srv:
        with pytest.raises(dqmc.DqmcError):
            srv.submit(26, np.zeros(1 << 21, dtype=np.uint32))
        with pytest.raises(dqmc.DqmcError) as e:
            srv.submit(20, np.zeros(1 << 15, dtype=np.uint32))  # larger than the whole budget
        assert e.value.code == dqmc.DQMC_ENOMEM
        tt = inputs.bernoulli(12, 0.8, 12)
        jid = srv.submit(12, tt)
        r = srv.wait(jid)
        _, _, ref = oracle.primes(12, tt)
        assert r["count"] == len(ref)
        assert np.array_equal(srv.read(jid, r["listed"]), ref)
        srv.release(jid)
        with pytest.raises(dqmc.DqmcError):
            srv.release(jid)
        with pytest.raises(dqmc.DqmcError):
            srv.poll(123456)


def test_destroy_with_blocked_queue():
    """Closing a server whose queue cannot move (its budget is held by an
    unreleased result) returns, dropping the queued job."""
    import time as _time

    from paper_2302_10083_amd import dqmc

    srv = dqmc.Server(0, budget=footprint(18) + footprint(16))
    a = srv.submit(18, inputs.bernoulli(18, 0.9, 11))
    srv.submit(18, inputs.bernoulli(18, 0.9, 12))
    srv.wait(a)
    t0 = _time.perf_counter()
    srv.close()
    assert _time.perf_counter() - t0 < 5.0

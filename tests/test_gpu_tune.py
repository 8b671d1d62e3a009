"""Autotuning: the tuners time every candidate they promise, keep the fastest,
and leave results exactly as the untuned calls produce them."""
import numpy as np
import pytest

import oracle
from paper_2302_10083_amd import inputs

from _gpu_common import context, log

pytestmark = pytest.mark.gpu


def _splits(h, k):
    """Ordered splits of h digits into k groups of 1..6 (lexicographic)."""
    if k == 0:
        return [[]] if h == 0 else []
    out = []
    for s in range(1, min(6, h) + 1):
        if h - s > 6 * (k - 1):
            continue
        out += [[s] + rest for rest in _splits(h - s, k - 1)]
    return out


def _hash(ctx, t):
    import torch

    from paper_2302_10083_amd import dqmc

    out = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    dqmc.dqmc_hash_words(ctx.ctx, t, t.numel(), out)
    torch.cuda.synchronize()
    return int(out.item())


@pytest.mark.parametrize("n,extra", [(18, 1), (20, 0), (20, 1)])
def test_plan_autotune(n, extra):
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    tt = inputs.bernoulli(n, 0.9, 7000 + n)
    ttd = ctx.tt_to_device(tt)
    ref_state, _, ref_count = ctx.primes(n, ttd, list_cap=0)
    torch.cuda.synchronize()
    ref = (_hash(ctx, ref_state), int(ref_count.item()))
    state = ctx.new_state(n)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    try:
        trials = dqmc.dqmc_plan_autotune(ctx.ctx, n, ttd, state, count, extra_groups=extra, reps=1)
        h = n - 12
        kmin = (h + 5) // 6
        want = [s for k in range(kmin, min(h, kmin + extra) + 1) for s in _splits(h, k)][:64]
        # the group plans, then the top-digit split
        assert [t["sizes"] for t in trials[:-1]] == want
        assert not any(t["split"] for t in trials[:-1]) and trials[-1]["split"] and trials[-1]["sizes"] == []
        assert all(t["ms"] > 0 for t in trials)
        best = min(trials[:-1], key=lambda t: t["ms"])
        assert dqmc.dqmc_get_plan(ctx.ctx, n) == best["sizes"]
        assert dqmc.dqmc_get_split(ctx.ctx, n) == (trials[-1]["ms"] < best["ms"])
        log("n=%d extra=%d: %d plans, best %s %.3f ms, split %.3f ms" % (n, extra, len(trials) - 1, best["sizes"],
                                                                       best["ms"], trials[-1]["ms"]))
        # the tuner's own output and a fresh call under the chosen plan
        assert (_hash(ctx, state), int(count.item())) == ref
        s2, _, c2 = ctx.primes(n, ttd, list_cap=0)
        torch.cuda.synchronize()
        assert (_hash(ctx, s2), int(c2.item())) == ref
    finally:
        dqmc.dqmc_set_plan(ctx.ctx, n, [])
        dqmc.dqmc_set_split(ctx.ctx, n, -1)


def test_plan_autotune_rejects_small_n():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    tt = inputs.bernoulli(12, 0.8, 12)
    ttd = ctx.tt_to_device(tt)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    with pytest.raises(dqmc.DqmcError) as e:
        dqmc.dqmc_plan_autotune(ctx.ctx, 12, ttd, ctx.new_state(12), count)
    assert e.value.code == dqmc.DQMC_EINVAL


def test_batch_autotune_keeps_results():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    specs = inputs.batch_specs(300, seed=4141)
    tts = [inputs.make(s) for s in specs]
    jobs = []
    for s, tt in zip(specs, tts):
        n = s["n"]
        jobs.append(dict(n=n, tt=ctx.tt_to_device(tt), state=ctx.new_state(n),
                         list=torch.empty(3**n, dtype=torch.int64, device=ctx.torch_device), list_cap=3**n,
                         count=torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)))
    plan = dqmc.Batch(ctx.ctx, jobs)
    plan.run()
    torch.cuda.synchronize()
    eager = [(j["state"].clone(), int(j["count"].item())) for j in jobs]
    trials = plan.autotune(reps=2)
    assert [(t["col_cap"], t["order"]) for t in trials] == [(c, o) for o in (0, 1) for c in (0, 1, 2, 3)]
    best = min(trials, key=lambda t: t["ms"])
    log("batch trials: %s" % ", ".join("%d/%d %.2f ms" % (t["col_cap"], t["order"], t["ms"]) for t in trials))
    for j in jobs:
        j["count"].fill_(-1)
        j["state"].fill_(0x5A5A5A5)
    plan.run()
    torch.cuda.synchronize()
    for (es, ec), j, s, tt in zip(eager, jobs, specs, tts):
        assert int(j["count"].item()) == ec
        assert torch.equal(j["state"], es)
    # a sample against the oracle
    for i in range(0, len(specs), 37):
        if specs[i]["n"] <= 16:
            _, _, ref = oracle.primes(specs[i]["n"], tts[i])
            c = int(jobs[i]["count"].item())
            assert c == len(ref)
            assert np.array_equal(jobs[i]["list"][:c].cpu().numpy(), ref)
    assert best["ms"] > 0
    plan.close()


def test_set_plan_rejects_group_starting_above_digit_24():
    """A group's lanes address its rows with 32-bit offsets: a group starting
    at digit 25 (rows 8 * 3^19 words apart) is refused, at n = 25 with the
    plan [6, 6, 1]; other plans of 25 digits are accepted."""
    from paper_2302_10083_amd import dqmc

    ctx = context()
    try:
        with pytest.raises(dqmc.DqmcError) as e:
            dqmc.dqmc_set_plan(ctx.ctx, 25, [6, 6, 1])
        assert e.value.code == dqmc.DQMC_EINVAL
        with pytest.raises(dqmc.DqmcError):
            dqmc.dqmc_set_plan(ctx.ctx, 25, [1, 6, 5, 1])
        dqmc.dqmc_set_plan(ctx.ctx, 25, [6, 6, 1][::-1])  # [1, 6, 6]: top group starts at digit 20
        assert dqmc.dqmc_get_plan(ctx.ctx, 25) == [1, 6, 6]
    finally:
        dqmc.dqmc_set_plan(ctx.ctx, 25, [])


def test_tune_cache_round_trip(tmp_path):
    """dqmc_tune_save writes the non-default settings keyed by architecture
    and n; dqmc_tune_load applies a file of this architecture all or nothing
    and ignores one of another architecture."""
    import json

    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    c = ctx.ctx
    path = str(tmp_path / "tune.json")
    want = {19: ([], 1), 20: ([1, 1, 6], -1), 22: ([6, 4], 0)}

    def reset():
        for n in range(13, 26):
            dqmc.dqmc_set_plan(c, n, [])
            dqmc.dqmc_set_split(c, n, -1)

    def state():
        return {n: (dqmc.dqmc_get_plan(c, n), dqmc.dqmc_get_split(c, n)) for n in range(13, 26)}

    try:
        reset()
        default = state()
        assert default[20][0] != [1, 1, 6] and default[22][0] != [6, 4]
        for n, (g, sp) in want.items():
            dqmc.dqmc_set_plan(c, n, g)
            dqmc.dqmc_set_split(c, n, sp)
        tuned = state()
        dqmc.dqmc_tune_save(c, path)
        doc = json.load(open(path))
        assert doc["format"] == "dqmc-tune-1"
        assert doc["arch"] == torch.cuda.get_device_properties(0).gcnArchName
        assert {e["n"]: (e["groups"], e["split"]) for e in doc["plans"]} == {n: (g, sp) for n, (g, sp) in want.items()}
        reset()
        assert dqmc.dqmc_tune_load(c, path) == 3
        assert state() == tuned
        # another architecture: nothing applied
        reset()
        other = dict(doc, arch="gfx000")
        json.dump(other, open(path, "w"))
        assert dqmc.dqmc_tune_load(c, path) == 0
        assert state() == default
        # an invalid entry after a valid one: nothing applied
        bad = dict(doc, plans=[{"n": 20, "groups": [2, 6], "split": 0}, {"n": 21, "groups": [4, 4], "split": 0}])
        json.dump(bad, open(path, "w"))
        with pytest.raises(dqmc.DqmcError) as e:
            dqmc.dqmc_tune_load(c, path)
        assert e.value.code == dqmc.DQMC_EINVAL
        assert state() == default
        # malformed JSON, an unknown key, a missing file
        for text in ('{"format": "dqmc-tune-1", "arch": "x", "plans": [', '{"format": "dqmc-tune-1", "plans": [], "z": 1}'):
            open(path, "w").write(text)
            with pytest.raises(dqmc.DqmcError) as e:
                dqmc.dqmc_tune_load(c, path)
            assert e.value.code == dqmc.DQMC_EINVAL
        with pytest.raises(dqmc.DqmcError) as e:
            dqmc.dqmc_tune_load(c, str(tmp_path / "missing.json"))
        assert e.value.code == dqmc.DQMC_EIO
        assert state() == default
    finally:
        reset()

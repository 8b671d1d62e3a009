"""The single-function entry points only enqueue kernels on the caller's
stream, so they can be captured in a HIP graph.  Each captured call is
replayed several times, with eager work and a clobbered output in between,
and every replay must reproduce the eager result."""
import numpy as np
import pytest

from _gpu_common import context, log, make_tt, oracle_primes

pytestmark = pytest.mark.gpu


def _replay_and_check(capture, outputs, expect, reps=3):
    import torch

    ctx = context()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            capture()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(reps):
        for t in outputs:
            t.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        expect(rep)
        torch.arange(1 << 20, device=ctx.torch_device).sum()  # eager work between replays
        torch.cuda.synchronize()
    del g


@pytest.mark.parametrize("n,split", [(18, 0), (17, 1), (12, 0)])
def test_primes_graph_replay(n, split):
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    tt = make_tt(n, "bern0.9", 9900 + n)
    _, O, ref = oracle_primes(n, tt)
    ttd = ctx.tt_to_device(tt)
    state = ctx.new_state(n)
    lst = torch.empty(len(ref) + 4, dtype=torch.int64, device=ctx.torch_device)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    if n > 12:
        dqmc.dqmc_set_split(ctx.ctx, n, split)
    try:
        log("graph: dqmc_primes n=%d split=%d" % (n, split))

        def expect(rep):
            assert int(count.item()) == len(ref), rep
            assert np.array_equal(lst[: len(ref)].cpu().numpy(), ref), rep
            assert np.array_equal(ctx.to_dense(n, state).cpu().numpy().view(np.uint64), O), rep

        _replay_and_check(lambda: dqmc.dqmc_primes(ctx.ctx, n, ttd, state, lst, len(ref), count),
                          [state, lst, count], expect)
    finally:
        if n > 12:
            dqmc.dqmc_set_split(ctx.ctx, n, -1)


def test_sliced_graph_replay():
    import torch

    from paper_2302_10083_amd import dqmc

    ctx = context()
    n, t = 16, 2
    tt = make_tt(n, "bern0.9", 9950)
    _, _, ref = oracle_primes(n, tt)
    ttd = ctx.tt_to_device(tt)
    o, m = ctx.new_state(n - t), ctx.new_state(n - t)
    lst = torch.empty(len(ref) + 4, dtype=torch.int64, device=ctx.torch_device)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    log("graph: dqmc_primes_sliced n=%d t=%d" % (n, t))

    def expect(rep):
        assert int(count.item()) == len(ref), rep
        assert np.array_equal(lst[: len(ref)].cpu().numpy(), ref), rep

    _replay_and_check(lambda: dqmc.dqmc_primes_sliced(ctx.ctx, n, t, ttd, 0, o, m, lst, len(ref), count),
                      [o, m, lst, count], expect)

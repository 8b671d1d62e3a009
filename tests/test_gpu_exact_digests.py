"""Exact parity of the large recipe (DNF of 2000 terms of width 6..14 OR
Bernoulli(0.02) noise) at n = 21..24 against the CPU oracle.

The oracle's prime lists at these sizes are stored as per-block digests
(``tests/golden/blocks_*.txt``, written by ``make_block_digests.py`` from
``oracle/`` alone): for each of the 81 blocks of the top four ternary digits,
the prime count and the SHA-256 of the block's sorted cube indices.  The GPU
list, from the same ``dqmc_primes`` call that bench.py times (bitmap and list
in one call, default plan), is cut into the same blocks and hashed the same
way; a mismatch names its block.  The count is also checked against the
bitmap's set bits."""
import os
import sys

import numpy as np
import pytest

from paper_2302_10083_amd import inputs

from _gpu_common import context, log

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_block_digests as mbd  # noqa: E402

CONFIGS = ["c3x_n21_dnf2000_noise", "c3x_n22_dnf2000_noise", "c3x_n23_dnf2000_noise", "c3_n24_dnf2000_noise"]


def _have(config):
    return os.path.exists(mbd.path_for(config))


@pytest.mark.parametrize("config", CONFIGS)
def test_block_digests_match_oracle(config):
    import torch

    from paper_2302_10083_amd import dqmc

    if not _have(config):
        pytest.skip("no oracle digest file for %s" % config)
    n, top, total, rows = mbd.read(config)
    spec = inputs.CONFIGS[config]
    assert spec["n"] == n
    tt = inputs.make(spec)
    ctx = context()
    log("%s: dqmc_primes (bitmap + list), %d primes expected" % (config, total))
    ttd = ctx.tt_to_device(tt)
    state = ctx.new_state(n)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    lst = torch.empty(total + 1, dtype=torch.int64, device=ctx.torch_device)
    dqmc.dqmc_primes(ctx.ctx, n, ttd, state, lst, total + 1, count)
    torch.cuda.synchronize()
    c = int(count.item())
    assert c == total, "prime count %d, oracle %d" % (c, total)
    got = lst[:c].cpu().numpy().view(np.uint64)
    del lst, state
    torch.cuda.empty_cache()
    log("%s: hashing %d blocks" % (config, len(rows)))
    mine = mbd.digests_of_list(n, got, top)
    bad = [(b, mine[b], rows[b]) for b in range(len(rows)) if mine[b] != rows[b]]
    assert not bad, "blocks differing from the oracle (block, gpu, oracle): %r" % bad[:5]

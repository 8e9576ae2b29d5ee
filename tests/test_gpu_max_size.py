"""Item counts past 2^31: every index, address and block count of the
Black-Scholes entry points is 64-bit where it must be.

n = 2^31 + 2^20 + 7 options (five 8.6 GB input columns, two output
columns: 60 GB of the device's memory); item i is pool tuple i mod 2^20, so
the oracle prices the 2^20 pool once and sampled outputs -- around 2^31,
at both ends and at random -- are checked against it.  Exact: within the
FP32 tolerance of the parity tests.  Perforation (dense and counted): a
dropped item keeps its fill value, a kept one equals the exact output bit
for bit.  iACT and TAF at threshold 0 compute every item: bit-identical to
the exact kernel.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, SENTINEL, say
from paper_2308_16877_amd import hpac, inputs

pytestmark = pytest.mark.gpu

POOL = 1 << 20
N = (1 << 31) + POOL + 7


@pytest.fixture(scope="module")
def big():
    assert torch.cuda.is_available()
    hpac.lib()
    pool = inputs.portfolio(POOL, 1024)
    reps = -(-N // POOL)
    say("max size: building %d items" % N)
    cols = [torch.from_numpy(c).to(DEV).repeat(reps)[:N] for c in pool]
    outs = [torch.empty(N, dtype=torch.float32, device=DEV) for _ in range(2)]
    g = np.random.default_rng(7)
    idx = np.unique(np.concatenate([
        [0, 1, 63, 64, (1 << 31) - 2, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, (1 << 31) + 64, N - 2, N - 1],
        g.integers(0, N, 400)]))
    C, P, sC, sP = oracle.bs_price(*pool)
    yield cols, outs, idx, np.stack([C, P]), np.stack([sC, sP])
    del cols, outs
    torch.cuda.empty_cache()


def sample(outs, idx):
    t = torch.from_numpy(idx).to(DEV)
    return np.stack([o.index_select(0, t).cpu().numpy().astype(np.float64) for o in outs])


def test_exact_past_2_31_items(big):
    cols, outs, idx, ref, scale = big
    for o in outs:
        o.fill_(SENTINEL)
    hpac.hpac_exact(cols, outs, items_per_lane=1)
    torch.cuda.synchronize()
    y = sample(outs, idx)
    r, s = ref[:, idx % POOL], scale[:, idx % POOL]
    assert np.all(np.abs(y - r) <= 1e-5 * s + 1e-30)


def test_techniques_past_2_31_items(big):
    cols, outs, idx, _, _ = big
    hpac.hpac_exact(cols, outs, items_per_lane=1)
    torch.cuda.synchronize()
    exact = sample(outs, idx)
    for name, call in (("iact", lambda: hpac.hpac_iact(cols, outs, 8, 0.0, items_per_lane=16)),
                       ("taf", lambda: hpac.hpac_taf(cols, outs, 4, 4, 0.0, items_per_lane=16))):
        for o in outs:
            o.fill_(SENTINEL)
        call()
        torch.cuda.synchronize()
        say("max size: %s" % name)
        assert np.array_equal(sample(outs, idx), exact), name
    ipt, M = 20, 10
    L = 64 * (((N + ipt - 1) // ipt + 63) // 64)  # lanes of the grid-stride mapping
    dropped = (idx // L) % M == M - 1
    for counted in (False, True):
        for o in outs:
            o.fill_(SENTINEL)
        cnt = torch.zeros(hpac.NUM_COUNTERS, dtype=torch.int64, device=DEV) if counted else None
        hpac.hpac_perfo(cols, outs, "small", M, items_per_lane=ipt, counters=cnt)
        torch.cuda.synchronize()
        say("max size: perforation, counted=%s" % counted)
        y = sample(outs, idx)
        assert np.all(y[:, dropped] == SENTINEL)
        assert np.array_equal(y[:, ~dropped], exact[:, ~dropped])
        if counted:
            c = cnt.cpu().numpy()
            steps = -(-N // L)
            kept_items = sum(min(L, N - k * L) for k in range(steps) if k % M != M - 1)
            assert c[0] == N and c[1] == N - kept_items

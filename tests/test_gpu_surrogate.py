"""GPU parity for the MLP surrogate: training gradients and the Adam step
against the FP64 oracle, BF16 MFMA inference against the oracle's forward
with the same BF16 rounding points, box routing with the exact fallback, and
what training buys.

Inference bound (Higham-style, u = 2^-8 at each BF16 rounding of a layer
input): the GPU and the oracle round the same quantities, but an FP32 and an
FP64 pre-activation may round to neighbouring BF16 values, so per output
|dy| <= u (|W3||h2| + g |W3||W2||h1| + g^2 |W3||W2||W1||xh|) * out_scale,
g = 1.13 the largest slope of GELU, plus FP32 accumulation.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, run, say
from paper_2308_16877_amd import hpac, inputs, surrogate

pytestmark = pytest.mark.gpu
P = hpac.MLP_NUM_PARAMS


def norm_for(labels, shift=0.0):
    lo, hi = inputs.BOX_LO, inputs.BOX_HI
    c = (lo + hi) / 2
    h = (hi - lo) / 2
    s = np.where(h > 0, 1.0 / np.where(h > 0, h, 1.0), 0.0)
    lab = np.log(labels + shift) if shift > 0 else labels
    return dict(in_center=c, in_scale=s, out_mean=lab.mean(axis=1), out_scale=lab.std(axis=1),
                out_shift=np.array([shift, shift]))


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    hpac.lib()


def dev_cols(a):
    return [torch.from_numpy(np.ascontiguousarray(c, np.float32)).to(DEV) for c in a]


@pytest.mark.parametrize("shift", [0.0, surrogate.PRICE_SHIFT])
@pytest.mark.parametrize("n", [4096, 4099])
def test_training_gradient_matches_oracle(shift, n):
    """Loss and gradient of the GPU's training kernel against the oracle's
    FP64 ones, on price targets and on log(price + shift) targets; n = 4099
    ends in a workgroup of three items whose other 61 lanes contribute
    nothing."""
    x = inputs.uniform_box(n, seed=51).astype(np.float32)
    C, Pp, _, _ = oracle.bs_price(*x)
    t = np.stack([C, Pp]).astype(np.float32)
    nm = norm_for(t.astype(np.float64), shift)
    # norm values as the GPU sees them (FP32)
    nm32 = {k: f32(v) for k, v in nm.items()}
    w = f32(surrogate.init_params(3))
    nb = hpac.hpac_mlp_grad_blocks(n)
    gp = torch.empty(nb * P, dtype=torch.float32, device=DEV)
    lp = torch.empty(nb, dtype=torch.float32, device=DEV)
    hpac.hpac_mlp_grad(dev_cols(x), dev_cols(t), torch.from_numpy(w.astype(np.float32)).to(DEV),
                       hpac.make_norm(**nm), n, gp, lp)
    torch.cuda.synchronize()
    g = gp.view(nb, P).double().sum(0).cpu().numpy()
    loss = float(lp.double().sum()) / (2 * n)
    loss_ref, g_ref = oracle.mlp_loss_grad(x, t, w, nm32)
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    say("gradient relative error %.2e, loss %.6f vs %.6f" % (err, loss, loss_ref))
    assert err <= 1e-4
    assert np.max(np.abs(g - g_ref)) <= 1e-4 * np.max(np.abs(g_ref))


def test_adam_step():
    nb = 3
    rng = np.random.default_rng(2)
    parts = rng.standard_normal((nb, P)).astype(np.float32)
    w0 = rng.standard_normal(P).astype(np.float32)
    m0 = (rng.standard_normal(P) * 0.1).astype(np.float32)
    v0 = (rng.random(P) * 0.1).astype(np.float32)
    w, m, v = (torch.from_numpy(a.copy()).to(DEV) for a in (w0, m0, v0))
    hpac.hpac_mlp_adam(torch.from_numpy(parts.ravel()).to(DEV), nb, w, m, v, 1e-3, 0.9, 0.999, 1e-8, 5)
    torch.cuda.synchronize()
    # the oracle's FP64 Adam step at the FP32 hyper-parameters the kernel receives
    f = lambda q: float(np.float32(q))
    wr, mr, vr = oracle.adam(parts, w0, m0, v0, f(1e-3), f(0.9), f(0.999), f(1e-8), 5)
    assert np.allclose(m.cpu().numpy(), mr, rtol=1e-6, atol=1e-7)
    assert np.allclose(v.cpu().numpy(), vr, rtol=1e-6, atol=1e-9)
    assert np.allclose(w.cpu().numpy(), wr, rtol=1e-6, atol=1e-6)


def inference_bound(x, w, nm):
    W1 = np.abs(oracle.bf16(w[:320])).reshape(64, 5)
    W2 = np.abs(oracle.bf16(w[384:4480])).reshape(64, 64)
    W3 = np.abs(oracle.bf16(w[4544:4672])).reshape(2, 64)
    xh = np.abs((np.asarray(x, np.float64) - nm["in_center"][:, None]) * nm["in_scale"][:, None])
    h1 = np.abs(W1 @ xh) + np.abs(w[320:384])[:, None]  # |h1| <= |z1| for GELU up to a constant
    h1 = 1.13 * h1
    h2 = 1.13 * (W2 @ h1 + np.abs(w[4480:4544])[:, None])
    u = 2.0 ** -8
    b = u * (W3 @ h2 + 1.13 * W3 @ (W2 @ h1) + 1.13 ** 2 * W3 @ (W2 @ (W1 @ xh))) + 1e-5 * (W3 @ h2)
    return b * nm["out_scale"][:, None]


@pytest.mark.parametrize("n", [1 << 16, (1 << 20) + 37])
@pytest.mark.parametrize("shift", [0.0, surrogate.PRICE_SHIFT])
def test_mfma_inference_matches_oracle_forward(shift, n):
    """With log outputs (shift > 0) the bound on v = yh * scale + mean maps
    through exp: |dy| <= (y + shift) (exp(b) - 1) plus FP32 expf rounding.
    n = 2^20 + 37 ends in a 37-item chunk and gives every wave of the
    persistent grid five or six chunks, each loaded while the previous one
    computes."""
    x = inputs.uniform_box(n, seed=53).astype(np.float32)
    w = f32(surrogate.init_params(4))
    labels = np.stack(oracle.bs_price(*x)[:2])
    nm = {k: f32(v) for k, v in norm_for(labels, shift).items()}
    s = surrogate.Surrogate(w, nm)
    out = [torch.zeros(n, dtype=torch.float32, device=DEV) for _ in range(2)]
    s(dev_cols(x), out)
    torch.cuda.synchronize()
    y = np.stack([o.cpu().numpy().astype(np.float64) for o in out])
    ref = oracle.mlp_forward(x, w, nm, round_act=True)
    bound = inference_bound(x, w, nm)
    if shift > 0:
        e = np.abs(ref) + nm["out_shift"][:, None]
        bound = e * np.expm1(bound) + 4 * 2.0 ** -24 * e
    err = np.abs(y - ref)
    say("inference |err| median %.2e max %.2e; max err/bound %.3f" % (np.median(err), err.max(), (err / bound).max()))
    assert np.all(err <= bound)
    # most results agree to FP32 accumulation accuracy
    assert np.median(err / (np.abs(ref) + 1e-3)) < 1e-4


def test_box_routing_and_exact_fallback():
    n = 200003
    x0 = inputs.uniform_box(n, seed=55).astype(np.float32)
    x, moved = inputs.with_out_of_box(x0, 0.05)
    w = f32(surrogate.init_params(5))
    labels = np.stack(oracle.bs_price(*x0)[:2])
    s = surrogate.Surrogate(w, {k: f32(v) for k, v in norm_for(labels).items()})
    out = [torch.zeros(n, dtype=torch.float32, device=DEV) for _ in range(2)]
    s(dev_cols(x), out)
    torch.cuda.synchronize()
    cnt = int(s.count.item())
    q = np.sort(s.queue[:cnt].cpu().numpy())
    assert np.array_equal(q, moved)
    y = np.stack([o.cpu().numpy().astype(np.float64) for o in out])
    C, Pp, sC, sP = oracle.bs_price(*x[:, moved])
    assert np.all(np.abs(y[:, moved] - np.stack([C, Pp])) <= 1e-5 * np.stack([sC, sP]) + 1e-30)


def test_training_reduces_error_and_what_it_buys():
    """Train on 2^20 exact-labelled box samples (log(price + 0.01) targets).
    What training buys: the same network and routing with the initial
    weights is useless (relative L2 error of order 1); the trained one prices
    every in-box option to a fraction of a percent in relative L2, and to
    about 1% MAPE (floored at 0.01; on price targets it was 0.4, from
    near-worthless options), with no locality in the inputs.  On
    the same unstructured inputs the techniques without a model gain nothing
    at that accuracy: iACT finds no input within its threshold, and 10%
    perforation loses about 30% in relative L2."""
    xs, ys = surrogate.make_training_set(1 << 20)
    s_trained, hist = surrogate.train(xs, ys, log=say)
    assert hist[-1] < 0.01 * hist[0]
    n = 1 << 16
    x = inputs.uniform_box(n, seed=57).astype(np.float32)
    C, Pp, _, _ = oracle.bs_price(*x)
    exact = np.stack([C, Pp])
    l2 = lambda a: float(np.linalg.norm(a - exact) / np.linalg.norm(exact))
    out = [torch.zeros(n, dtype=torch.float32, device=DEV) for _ in range(2)]
    s_trained(dev_cols(x), out)
    torch.cuda.synchronize()
    y = np.stack([o.cpu().numpy().astype(np.float64) for o in out])
    s_untrained = surrogate.Surrogate(surrogate.init_params(), s_trained.norm_dict)
    s_untrained(dev_cols(x), out)
    torch.cuda.synchronize()
    yu = np.stack([o.cpu().numpy().astype(np.float64) for o in out])
    ya, _, cnt = run("iact", dev_cols(x), 2, 16, counters=True, table_size=8, threshold=0.05)
    yp, _, _ = run("perfo", dev_cols(x), 2, 20, fill=0.0, kind="small", param=10)
    say("relative L2: trained %.4f, untrained %.4f, perforation-10%% %.4f; iACT approximated %d of %d; "
        "MAPE trained %.4f" % (l2(y), l2(yu), l2(yp), cnt[1], n, oracle.mape(exact, y)[0]))
    assert l2(y) < 0.01 and l2(yu) > 0.5
    assert oracle.mape(exact, y)[0] < 0.02
    assert cnt[1] <= 0.01 * n and l2(ya) < 1e-5
    assert l2(yp) > 10 * l2(y)

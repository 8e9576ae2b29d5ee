"""Pins for the oracle's MLP surrogate (forward, loss gradient, BF16
rounding, GELU), independent of its own code paths: scipy's normal CDF for
GELU, finite differences for the gradient, numpy matrix products for the
identity-activation network, and closed cases (zero weights)."""
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2308_16877_amd import inputs

P = 64 * 5 + 64 + 64 * 64 + 64 + 2 * 64 + 2


def norm():
    lo, hi = inputs.BOX_LO, inputs.BOX_HI
    c = (lo + hi) / 2
    h = (hi - lo) / 2
    s = np.where(h > 0, 1.0 / np.where(h > 0, h, 1.0), 0.0)
    return dict(in_center=c, in_scale=s, out_mean=np.array([3.0, 40.0]), out_scale=np.array([4.0, 25.0]))


def random_params(seed, scale=0.3):
    g = np.random.default_rng(seed)
    return g.standard_normal(P) * scale


def split(w):
    W1 = w[:320].reshape(64, 5)
    b1 = w[320:384]
    W2 = w[384:4480].reshape(64, 64)
    b2 = w[4480:4544]
    W3 = w[4544:4672].reshape(2, 64)
    b3 = w[4672:4674]
    return W1, b1, W2, b2, W3, b3


def test_param_count():
    assert oracle.mlp_num_params() == P


def test_bf16_rounding():
    assert oracle.bf16(1.0 + 2.0 ** -8) == 1.0  # tie to even (down)
    assert oracle.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie to even (up)
    assert oracle.bf16(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    assert oracle.bf16(-3.14159) == -3.140625
    assert oracle.bf16(0.0) == 0.0
    v = np.random.default_rng(1).standard_normal(1000) * 10
    r = oracle.bf16(v)

    # 8 significant bits: relative error at most 2^-8
    assert np.all(np.abs(r - v) <= 2.0 ** -8 * np.abs(v))


def test_gelu_tanh_form_against_normal_cdf():
    x = np.linspace(-8, 8, 3201)
    g = oracle.gelu(x)
    exact = x * stats.norm.cdf(x)
    # the tanh form approximates x Phi(x) to within about 5e-4 everywhere
    assert np.max(np.abs(g - exact)) < 5e-4
    assert oracle.gelu([0.0])[0] == 0.0
    assert abs(oracle.gelu([30.0])[0] - 30.0) < 1e-12 and abs(oracle.gelu([-30.0])[0]) < 1e-12


def test_zero_weights_output_the_bias():
    w = np.zeros(P)
    w[4672:] = [0.5, -0.25]
    x = inputs.uniform_box(100, seed=3)
    n = norm()
    y = oracle.mlp_forward(x, w, n)
    assert np.allclose(y[0], 0.5 * 4.0 + 3.0) and np.allclose(y[1], -0.25 * 25.0 + 40.0)


def test_zero_weights_with_log_outputs():
    """With out_shift > 0 a zero-weight network outputs exp(bias * scale +
    mean) - shift, and the loss of constant targets t is zero exactly when the
    bias is (log(t + shift) - mean) / scale: the forward map and the
    training target's transform are inverse to each other."""
    x = inputs.uniform_box(50, seed=11)
    n = dict(norm(), out_shift=np.array([0.01, 0.5]))
    t = np.array([1e-6, 12.5])  # a near-worthless call and an ordinary put
    w = np.zeros(P)
    w[4672:] = (np.log(t + n["out_shift"]) - n["out_mean"]) / n["out_scale"]
    y = oracle.mlp_forward(x, w, n, round_act=False)
    assert np.allclose(y, t[:, None], rtol=1e-12, atol=1e-15)
    loss, g = oracle.mlp_loss_grad(x, np.repeat(t[:, None], 50, axis=1), w, n)
    assert loss < 1e-28 and np.max(np.abs(g)) < 1e-12
    # without the shift the same bias is far from the targets
    loss0, _ = oracle.mlp_loss_grad(x, np.repeat(t[:, None], 50, axis=1), w, norm())
    assert loss0 > 0.1
    w[4672:] = [0.5, -0.25]
    y = oracle.mlp_forward(x, w, n, round_act=False)
    assert np.allclose(y[0], np.exp(0.5 * 4.0 + 3.0) - 0.01) and np.allclose(y[1], np.exp(-0.25 * 25.0 + 40.0) - 0.5)


def test_identity_activation_is_plain_matrix_products():
    w = random_params(5)
    x = inputs.uniform_box(300, seed=4)
    n = norm()
    y = oracle.mlp_forward(x, w, n, round_act=False, act=False)
    W1, b1, W2, b2, W3, b3 = (oracle.bf16(a) if i % 2 == 0 else a for i, a in enumerate(split(w)))
    xh = (x - n["in_center"][:, None]) * n["in_scale"][:, None]
    yh = W3 @ (W2 @ (W1 @ xh + b1[:, None]) + b2[:, None]) + b3[:, None]
    ref = yh * n["out_scale"][:, None] + n["out_mean"][:, None]
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("act,shift", [(True, 0.0), (False, 0.0), (True, 0.01)])
def test_loss_gradient_matches_finite_differences(act, shift):
    # perturb biases and a sample of weights whose BF16 rounding is the
    # identity for the step used (exact BF16 values with spare bits)
    w = oracle.bf16(random_params(7, 0.2))
    x = inputs.uniform_box(64, seed=8)
    C, Pp, _, _ = oracle.bs_price(*x)
    n = norm()
    if shift:
        # log targets: their own mean and deviation
        lt = np.log(np.stack([C, Pp]) + shift)
        n = dict(n, out_mean=lt.mean(axis=1), out_scale=lt.std(axis=1), out_shift=np.array([shift, shift]))
    loss, g = oracle.mlp_loss_grad(x, np.stack([C, Pp]), w, n, act=act)
    rng = np.random.default_rng(9)
    idx = list(range(320, 384)) + list(range(4480, 4544)) + [4672, 4673]
    idx += list(rng.choice(320, 10, replace=False)) + list(384 + rng.choice(4096, 20, replace=False))
    idx += list(4544 + rng.choice(128, 10, replace=False))
    for p in idx:
        if p in range(320, 384) or p in range(4480, 4544) or p >= 4672:
            h = 1e-6
            wp, wm = w.copy(), w.copy()
            wp[p] += h
            wm[p] -= h
        else:
            # move the weight by one BF16 ulp either side so the rounding is exact
            ulp = 2.0 ** (np.floor(np.log2(abs(w[p]))) - 7)
            h = ulp
            wp, wm = w.copy(), w.copy()
            wp[p] += h
            wm[p] -= h
        lp, _ = oracle.mlp_loss_grad(x, np.stack([C, Pp]), wp, n, act=act)
        lm, _ = oracle.mlp_loss_grad(x, np.stack([C, Pp]), wm, n, act=act)
        fd = (lp - lm) / (2 * h)
        tol = 2e-6 * abs(g[p]) + 1e-9 + (1e-4 * abs(g[p]) + 1e-8 if h > 1e-6 else 0)
        assert abs(fd - g[p]) <= tol, (p, fd, g[p])

"""Pins of the fill-network oracle: layers against direct loops written from
their definitions, gradients against central finite differences, bfloat16
rounding against torch's conversion, Adam against its first-step closed
form."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import unet as U


def test_bf16_round_ties_and_library():
    assert U.bf16_round(1.0) == 1.0
    assert U.bf16_round(1.0 + 2 ** -8) == 1.0                 # tie -> even
    assert U.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6   # tie -> even
    assert U.bf16_round(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    import torch
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 100
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16_round(x), ref)


def test_conv3_matches_direct_loop():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 4, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = U.conv3(x, w, b)
    N, H, W, C = x.shape
    for n in range(N):
        for y in range(H):
            for xx in range(W):
                for co in range(4):
                    s = b[co]
                    for ky in range(3):
                        for kx in range(3):
                            yy, xs = y + ky - 1, xx + kx - 1
                            if 0 <= yy < H and 0 <= xs < W:
                                s += sum(w[co, ky, kx, ci] * x[n, yy, xs, ci] for ci in range(C))
                    assert abs(out[n, y, xx, co] - s) < 1e-12


def test_convT2_and_maxpool_match_direct_loops():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 3, 2, 4))
    w = rng.standard_normal((2, 2, 5, 4))
    b = rng.standard_normal(5)
    out = U.convT2(x, w, b)
    assert out.shape == (1, 6, 4, 5)
    for y in range(6):
        for xx in range(4):
            for co in range(5):
                s = b[co] + sum(w[y % 2, xx % 2, co, ci] * x[0, y // 2, xx // 2, ci] for ci in range(4))
                assert abs(out[0, y, xx, co] - s) < 1e-12
    z = rng.standard_normal((1, 4, 6, 2))
    p, arg = U.maxpool2(z)
    for y in range(2):
        for xx in range(3):
            for c in range(2):
                blk = [z[0, 2 * y + a, 2 * xx + bb, c] for a in range(2) for bb in range(2)]
                assert p[0, y, xx, c] == max(blk) and arg[0, y, xx, c] == int(np.argmax(blk))


def _small_problem(seed=3, levels=2, base=4, H=8, W=8):
    rng = np.random.default_rng(seed)
    theta = U.init_params(seed, levels, base)
    theta = theta + 0.05 * rng.standard_normal(theta.size)   # non-zero head
    x = rng.random((1, H, W, U.IN_CH))
    rgb = rng.integers(0, 256, (1, H, W, 3)).astype(np.float64)
    tgt = rng.integers(0, 256, (1, H, W, 3)).astype(np.float64)
    return theta, x, rgb, tgt


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_network_gradient_central_differences(levels):
    """Central differences (h = 1e-6, fp64) on a small net agree with the
    analytic gradient for a random subset of parameters."""
    theta, x, rgb, tgt = _small_problem(levels=levels, H=8, W=8)
    loss, g, _ = U.loss_and_grad(theta, x, rgb, tgt, levels, 4)
    rng = np.random.default_rng(4)
    idx = rng.choice(theta.size, size=min(150, theta.size), replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (U.loss_and_grad(tp, x, rgb, tgt, levels, 4)[0] - U.loss_and_grad(tm, x, rgb, tgt, levels, 4)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, g[i])


def test_input_gradient_through_pool_and_concat():
    """Gradient w.r.t. the network input (via a zero-padding identity layer
    trick: perturb the input) matches central differences."""
    theta, x, rgb, tgt = _small_problem(levels=3, H=8, W=8)
    P = U.unpack(theta, 3, 4)
    out, acts = U.forward(theta, x, 3, 4)
    dout = np.random.default_rng(5).standard_normal(out.shape)
    # d/dx sum(dout * f(x)) through the first conv's input gradient
    rng = np.random.default_rng(6)
    for _ in range(40):
        n, y, xx, c = 0, rng.integers(8), rng.integers(8), rng.integers(U.IN_CH)
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[n, y, xx, c] += h
        xm[n, y, xx, c] -= h
        fd = ((U.forward(theta, xp, 3, 4)[0] - U.forward(theta, xm, 3, 4)[0]) * dout).sum() / (2 * h)
        # analytic: one backward step through the whole net, then conv3 input grad
        g = _input_grad(theta, acts, dout)
        assert abs(fd - g[n, y, xx, c]) <= 1e-6 + 1e-4 * abs(fd)


def _input_grad(theta, acts, dout):
    # the flat-parameter backward does not return the input gradient; get it
    # by differentiating w.r.t. a prepended identity: perturbation of the
    # first conv's bias equals the sum of its output gradient, so instead
    # reuse conv3_bwd on the recorded first-layer gradient
    levels, base = 3, 4
    P = U.unpack(theta, levels, base)
    # recompute the gradient at the first conv output by a backward pass
    # with the first layer's input gradient exposed
    grads = {}

    def conv3_bwd_spy(x, w, dz, _orig=U.conv3_bwd):
        r = _orig(x, w, dz)
        if x is acts["x"]:
            grads["x"] = r[0]
        return r
    orig = U.conv3_bwd
    U.conv3_bwd = conv3_bwd_spy
    try:
        U.backward(theta, acts, dout, levels, base)
    finally:
        U.conv3_bwd = orig
    return grads["x"]


def test_adam_first_step_closed_form():
    """After one step from m = v = 0 the bias-corrected update is
    -lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = U.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)


def test_untrained_network_returns_splat():
    theta = U.init_params(0, 2, 4)
    rgba = np.random.default_rng(7).integers(0, 2 ** 32, (1, 8, 8), dtype=np.uint64).astype(np.uint32)
    depth = np.ones((1, 8, 8), np.float32) * 1.5
    cov = np.ones((1, 8, 8), np.uint8)
    out, _ = U.forward(theta, U.unpack_input(rgba, depth, cov), 2, 4)
    assert np.all(out == 0)
    img = U.fill_image(rgba, out)
    assert np.array_equal(img & 0xFFFFFF, rgba & 0xFFFFFF)


def test_parameter_count_of_the_full_network():
    # by hand: encoder 1760 + 9248 + 18496 + 36928 + 73856 + 147584 + 295168
    # + 590080; decoder 131200 + 295040 + 147584, 32832 + 73792 + 36928,
    # 8224 + 18464 + 9248; head 99
    assert U.n_params(4, 32) == 1_926_531


def test_absolute_term_sums_bound_the_gradient():
    """The absolute term sums bound every gradient element (triangle
    inequality) and equal it when every factor is non-negative: then no
    term cancels another."""
    rng = np.random.default_rng(3)
    levels = 2
    th = U.init_params(2, levels) + 0.05 * rng.standard_normal(U.n_params(levels))
    x = rng.random((1, 8, 8, U.IN_CH))
    out, acts = U.forward(th, x, levels)
    g, t = U.backward(th, acts, rng.standard_normal(out.shape), levels, abs_terms=True)
    assert np.all(np.abs(g) <= t * (1 + 1e-12))
    # one level, non-negative weights, inputs and output gradient
    th1 = np.abs(U.init_params(4, 1)) + 0.01
    x1 = rng.random((1, 6, 6, U.IN_CH))
    out1, acts1 = U.forward(th1, x1, 1)
    g1, t1 = U.backward(th1, acts1, rng.random(out1.shape), 1, abs_terms=True)
    assert np.allclose(g1, t1, rtol=1e-12, atol=0)

"""Learned fill on the GPU (through the C ABI) against the fp64 oracle.

Two oracle runs on the same bfloat16 weights and input: `exact` keeps every
activation in fp64; `emulated` rounds every stored activation (and
activation gradient) to bfloat16 where the GPU stores one. The GPU differs
from `emulated` only by fp32 accumulation order, which now and then lands a
value on the other side of a bfloat16 rounding boundary; such a one-ulp
flip (2^-8 relative) moves the next layer's inputs and can flip further
roundings, so GPU and `emulated` are not element-wise equal. Both carry the
same kind of error with respect to `exact`: bfloat16 storage. The bounds:
  forward residual  RMS(gpu - exact) <= 1.5 RMS(emulated - exact) + 1e-6,
                    max |gpu - exact| <= 2^-5 max |exact|
  gradients         per layer ||gpu - exact|| <= 1.5 ||emulated - exact||
                    + 2^-10 ||exact||
and every kernel of the training step is checked element by element on the
tensors it actually read in tests/test_gpu_fill_trace.py.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import unet as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    return fhv


def splat_batch(seed, N, H, W, hole=0.3):
    rng = np.random.default_rng(seed)
    cov = (rng.random((N, H, W)) > hole).astype(np.uint8)
    rgba = (rng.integers(0, 2 ** 24, (N, H, W)).astype(np.uint32) | np.uint32(0xFF000000)) * cov
    depth = np.where(cov > 0, 1.0 + rng.random((N, H, W)), 0.0).astype(np.float32)
    tgt = (rng.integers(0, 2 ** 24, (N, H, W)).astype(np.uint32) | np.uint32(0xFF000000))
    return rgba.astype(np.uint32), depth, cov, tgt


def gpu_theta_view(theta, levels):
    """Parameters as the GPU uses them: conv and transposed-conv weights
    rounded to bfloat16; biases and the head in fp32."""
    t = theta.copy()
    o = 0
    for (kind, ci, co), (ws, bs) in zip(U.layer_specs(levels), U.param_shapes(levels)):
        nw = int(np.prod(ws))
        if kind != "h1":
            t[o:o + nw] = U.bf16_round(t[o:o + nw])
        o += nw + int(np.prod(bs))
    return t


def to_t(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def params_for(seed, levels):
    rng = np.random.default_rng(seed + 100)
    th = U.init_params(seed, levels)
    th = th + 0.02 * rng.standard_normal(th.size)       # non-zero biases and head
    return th.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("levels,N,H,W", [(1, 1, 8, 16), (2, 2, 16, 24), (3, 1, 24, 40), (4, 2, 16, 24),
                                          (4, 1, 8, 8),
                                          # ragged tiles: rows not a multiple of 4, several
                                          # 64-pixel column tiles with a partial last one
                                          (1, 1, 13, 70), (2, 1, 18, 130), (3, 2, 20, 132),
                                          # more 8-row x 62-pixel tiles than the persistent
                                          # kernels have workgroups (256), so that workgroups
                                          # go on to further tiles: full-size layers, then
                                          # also the 64-channel layers of the second level
                                          # (widths that 62-pixel tiles cover with little
                                          # waste, as those kernels are used only there;
                                          # the last tile of a row partial)
                                          (1, 4, 64, 600), (2, 4, 144, 960)])
def test_forward_parity(F, levels, N, H, W):
    th = params_for(levels, levels)
    rgba, depth, cov, _ = splat_batch(levels, N, H, W)
    img, res = F.fill(to_t(th.astype(np.float32)), to_t(rgba), to_t(depth), to_t(cov), levels, residual=True)
    res = res.cpu().numpy().astype(np.float64)
    x = U.bf16_round(U.unpack_input(rgba, depth, cov))
    thg = gpu_theta_view(th, levels)
    emu, _ = U.forward(thg, x, levels, round_acts=True)
    exact, _ = U.forward(thg, x, levels, round_acts=False)
    rms = lambda a: float(np.sqrt((a ** 2).mean()))
    assert rms(res - exact) <= 1.5 * rms(emu - exact) + 1e-6, (rms(res - exact), rms(emu - exact))
    assert np.abs(res - exact).max() <= 2 ** -5 * np.abs(exact).max()
    want = U.fill_image(rgba, res)       # rounding of the GPU's own residual
    got = img.cpu().numpy().view(np.uint32)
    d = np.abs(got.view(np.uint8).astype(int) - want.view(np.uint8).astype(int))
    assert d.max() <= 1 and (d > 0).mean() < 1e-3


@pytest.mark.parametrize("levels,N,H,W", [(1, 1, 8, 16), (2, 2, 16, 24), (4, 2, 16, 16), (2, 1, 18, 130)])
def test_gradient_parity(F, levels, N, H, W):
    import torch
    th = params_for(7 + levels, levels)
    rgba, depth, cov, tgt = splat_batch(11 + levels, N, H, W)
    n = U.n_params(levels)
    assert F.unet_param_count(levels) == n
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    pt = to_t(th.astype(np.float32))
    F.fill_train_step(pt, None, None, 0, 0.0, to_t(rgba), to_t(depth), to_t(cov), to_t(tgt), levels,
                      loss=loss, grad=grad)
    torch.cuda.synchronize()
    assert np.array_equal(pt.cpu().numpy(), th.astype(np.float32))    # step 0: no update
    g = grad.cpu().numpy().astype(np.float64)
    x = U.bf16_round(U.unpack_input(rgba, depth, cov))
    rgb = np.stack([(rgba >> (8 * k)) & 0xFF for k in range(3)], -1).astype(np.float64)
    trgb = np.stack([(tgt >> (8 * k)) & 0xFF for k in range(3)], -1).astype(np.float64)
    thg = gpu_theta_view(th, levels)
    grads = {}
    for name, rnd in (("emu", True), ("exact", False)):
        out, acts = U.forward(thg, x, levels, round_acts=rnd)
        diff = rgb / 255 + out - trgb / 255
        grads[name] = U.backward(thg, acts, 2 * diff / diff.size, levels, round_grads=rnd)
        if rnd:
            emu_loss = (diff ** 2).mean()
    assert abs(loss.item() - emu_loss) <= 1e-3 * emu_loss
    o = 0
    nrm = np.linalg.norm
    for (kind, ci, co), (ws, bs) in zip(U.layer_specs(levels), U.param_shapes(levels)):
        for part, nn in (("w", int(np.prod(ws))), ("b", int(np.prod(bs)))):
            a, e, r = g[o:o + nn], grads["emu"][o:o + nn], grads["exact"][o:o + nn]
            assert nrm(a - r) <= 1.5 * nrm(e - r) + 2 ** -10 * nrm(r) + 1e-12, (
                kind, ci, co, part, nrm(a - r), nrm(e - r), nrm(r))
            o += nn


def test_adam_first_step(F):
    import torch
    levels = 2
    th = params_for(3, levels)
    rgba, depth, cov, tgt = splat_batch(5, 1, 16, 16)
    n = U.n_params(levels)
    pt = to_t(th.astype(np.float32))
    m = torch.zeros(n, dtype=torch.float32, device="cuda")
    v = torch.zeros(n, dtype=torch.float32, device="cuda")
    F.fill_train_step(pt, m, v, 1, 1e-3, to_t(rgba), to_t(depth), to_t(cov), to_t(tgt), levels)
    torch.cuda.synchronize()
    x = U.bf16_round(U.unpack_input(rgba, depth, cov))
    rgb = np.stack([(rgba >> (8 * k)) & 0xFF for k in range(3)], -1).astype(np.float64)
    trgb = np.stack([(tgt >> (8 * k)) & 0xFF for k in range(3)], -1).astype(np.float64)
    thg = gpu_theta_view(th, levels)
    out, acts = U.forward(thg, x, levels)
    diff = rgb / 255 + out - trgb / 255
    g = U.backward(thg, acts, 2 * diff / diff.size, levels)
    want, _, _ = U.adam(th, np.zeros(n), np.zeros(n), g, 1, 1e-3)
    got = pt.cpu().numpy().astype(np.float64)
    big = np.abs(g) > 1e-2 * np.abs(g).max()       # away from sign ambiguity
    assert np.allclose(got[big], want[big], atol=2e-5)
    assert np.abs(got - th).max() <= 1e-3 * 1.0001


def test_training_reduces_loss(F):
    import torch
    levels = 2
    th = U.init_params(1, levels)
    rgba, depth, cov, tgt = splat_batch(9, 2, 32, 32)
    # target: the splat with holes filled by a constant colour (learnable)
    tgt = np.where(cov > 0, rgba, np.uint32(0xFF4080C0)).astype(np.uint32)
    n = U.n_params(levels)
    pt = to_t(th.astype(np.float32))
    m = torch.zeros(n, dtype=torch.float32, device="cuda")
    v = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = None
    losses = []
    args = [to_t(a) for a in (rgba, depth, cov, tgt)]
    for step in range(1, 61):
        ws = F.fill_train_step(pt, m, v, step, 2e-3, *args, levels, loss=loss, ws=ws)
        losses.append(loss.item())
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0], losses[::10]


def test_fill_rejects_bad_sizes(F):
    import ctypes as C
    L = F.lib()
    assert L.fhv_fill_workspace(4, 1, 12, 16, 0) == 0        # 12 not a multiple of 8
    assert L.fhv_fill_workspace(5, 1, 16, 16, 0) == 0
    assert L.fhv_unet_param_count(4) == U.n_params(4)
    assert L.fhv_fill(F.ctx(), 4, None, None, None, None, 1, 8, 8, None, None, None, 0, None) == -1

"""Every kernel of the fill's training step, element by element, on the
tensors it actually read (fhv_fill_train_step_traced keeps every activation
and activation gradient of the step; fhv_fill_trace_tensors locates them).

Whole-network outputs cannot be compared element-wise with an independent
summation order: a one-ulp bfloat16 rounding difference early in the
network reaches every later layer, and deep layers amplify it far beyond
any bound on the element's own terms. Each layer is therefore checked on
its own: the oracle (fp64) recomputes the layer from the GPU's stored
inputs (bfloat16 values, exact in fp64) and the GPU's result must lie
within the rounding bound of that computation:

  a bfloat16 store of an fp32 sum S of n terms (products of two bfloat16
  values, exact in fp32) computed in any order:
      |stored - exact| <= 2^-8 |exact| + (1 + 2^-8) g_K sum|terms|
  an fp32 result (weight and bias gradients): |gpu - exact| <= g_K sum|terms|

with g_K = 2 K 2^-24 for a summation tree of depth K (K additions along the
longest chain; twice the first-order bound K u, which also covers an
accumulator that truncates). K is the number of terms for the convolutions
(any order), and the depth of the pixel-split tree for the weight and bias
gradients. ReLU gradients and the max pool are compared bit for bit.
Shapes: the training batch (8 x 256 x 256, four levels: weight gradients
split over 1,024 pixel ranges per wave tile and summed in several groups,
every channel width of the network), and small ragged ones."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import unet as U
from tests.test_gpu_fill import gpu_theta_view, params_for, splat_batch, to_t

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    return fhv


def g_k(K):
    return 2.0 * K * U24


def bf16_bits_to_f64(a16: np.ndarray) -> np.ndarray:
    return (a16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def tensor(ws: np.ndarray, e) -> np.ndarray:
    """Entry e of the trace table as fp64 [n, h, w, channels]."""
    n, h, w = e["shape"]
    cnt = n * h * w * e["stride"]
    raw = ws[e["offset"]:e["offset"] + 2 * cnt].view(np.uint16).reshape(n, h, w, e["stride"])
    return bf16_bits_to_f64(raw[..., :e["channels"]])


def check_store(got, exact, terms, K, what):
    """bfloat16 store of an fp32 sum: see the module docstring."""
    bound = 2.0 ** -8 * np.abs(exact) + (1 + 2.0 ** -8) * g_k(K) * terms
    bad = np.abs(got - exact) > bound
    assert not bad.any(), (what, int(bad.sum()), float((np.abs(got - exact) / (bound + 1e-300)).max()))


def check_sum(got, exact, terms, K, what):
    bound = g_k(K) * terms
    bad = np.abs(got - exact) > bound
    assert not bad.any(), (what, int(bad.sum()), float((np.abs(got - exact) / (bound + 1e-300)).max()))


def wgrad_depth(P, cin, cout):
    """Depth of the weight-gradient summation tree: per wave, `per` 32-pixel
    chunks (one 32-term matrix product each), four waves added in order,
    then the partial rows in 16 ordered groups and the group sums in order
    (the split rule of the library's weight-gradient launch)."""
    tiles = (cout // 32) * ((cin + 31) // 32)
    chunks = (P + 31) // 32
    s = min(max((1024 + tiles - 1) // tiles, 1), chunks)
    per = (chunks + s - 1) // s
    splits = (chunks + per - 1) // per
    groups = (splits + 3) // 4
    return 33 * per + 4 + (groups + 15) // 16 + 16


def bgrad_depth(P):
    splits = min((P + 255) // 256, 512)
    per = (P + splits - 1) // splits
    return per + splits + 256


def patches_t(x):
    """[N,H,W,C] -> 3x3 patches [N*H*W, 9*C] (zero padding)."""
    N, H, W, C = x.shape
    return U.patches3(x).reshape(N * H * W, 9 * C)


def run_traced(F, levels, N, H, W, seed):
    import torch
    th = params_for(seed, levels)
    rgba, depth, cov, tgt = splat_batch(seed + 10, N, H, W)
    n = U.n_params(levels)
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    pt = to_t(th.astype(np.float32))
    ws = F.fill_train_step_traced(pt, to_t(rgba), to_t(depth), to_t(cov), to_t(tgt), levels, loss=loss, grad=grad)
    # the untraced step computes the same gradient, bit for bit
    grad2 = torch.zeros(n, dtype=torch.float32, device="cuda")
    F.fill_train_step(pt, None, None, 0, 0.0, to_t(rgba), to_t(depth), to_t(cov), to_t(tgt), levels, grad=grad2)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)
    table = F.fill_trace_tensors(levels, N, H, W)
    return th, (rgba, depth, cov, tgt), ws.cpu().numpy(), table, grad.cpu().numpy().astype(np.float64), loss.item()


@pytest.mark.parametrize("levels,N,H,W", [(1, 1, 8, 16), (2, 1, 18, 130), (3, 2, 20, 132), (4, 2, 16, 24),
                                          # the training batch
                                          pytest.param(4, 8, 256, 256, marks=pytest.mark.slow),
                                          # 1080p-like widths: 62-pixel tiles, more tiles than the
                                          # persistent kernels have workgroups at every level
                                          pytest.param(4, 2, 512, 992, marks=pytest.mark.slow)])
def test_every_layer_of_a_training_step(F, levels, N, H, W):
    print(f"traced training step levels={levels} {N}x{H}x{W}", flush=True)
    th, (rgba, depth, cov, tgt), ws, T, grad, loss = run_traced(F, levels, N, H, W, 60 + levels)
    thg = gpu_theta_view(th, levels)
    P = U.unpack(thg, levels)
    specs = U.layer_specs(levels)
    offs = np.cumsum([0] + [int(np.prod(a)) + int(np.prod(b)) for a, b in U.param_shapes(levels)])
    ent = lambda i, k: T[5 * i + k]
    get = lambda i, k: tensor(ws, ent(i, k))

    # input packing: the first layer's input is the rounded network input
    x0 = get(0, 0)
    assert np.array_equal(x0[..., :6], U.bf16_round(U.unpack_input(rgba, depth, cov)))
    assert not x0[..., 6:].any()

    for i, (kind, ci, co) in enumerate(specs):
        w, b = P[i]
        gw = grad[offs[i]:offs[i] + w.size].reshape(w.shape)
        gb = grad[offs[i] + w.size:offs[i + 1]]
        if kind == "c3":
            x = get(i, 0)[..., :ci]
            y = get(i, 1)
            Nn, Hl, Wl, _ = x.shape
            Pl = Nn * Hl * Wl
            # forward: y = bf16(relu(conv3(x)))
            z = U.conv3(x, w, b)
            tz = U.conv3(np.abs(x), np.abs(w), np.abs(b))
            check_store(y, np.maximum(z, 0.0), tz, 9 * ci + 1, (i, kind, "forward"))
            # max pool of an encoder output feeds the next level
            if kind == "c3" and i % 2 == 1 and i < 2 * levels - 1:
                pooled, _ = U.maxpool2(y)
                assert np.array_equal(get(i + 1, 0), pooled), (i, "max pool")
            # ReLU gradient, bit for bit
            g = get(i, 2)
            dz = get(i, 3)
            assert np.array_equal(dz, g * (y > 0)), (i, kind, "relu gradient")
            # weight and bias gradients (fp32) from the stored dz and x
            d = dz.reshape(Pl, co)
            Px = patches_t(x)
            ew = (d.T @ Px).reshape(w.shape)
            tw = (np.abs(d).T @ np.abs(Px)).reshape(w.shape)
            check_sum(gw, ew, tw, wgrad_depth(Pl, ((ci + 7) // 8) * 8, co), (i, kind, "weight gradient"))
            check_sum(gb, d.sum(0), np.abs(d).sum(0), bgrad_depth(Pl), (i, kind, "bias gradient"))
            # input gradient: bf16(conv3 transposed of dz)
            if ent(i, 4) is not None:
                gin = get(i, 4)
                dx, _, _ = U.conv3_bwd(x, w, dz)
                adx, _, _ = U.conv3_bwd(np.abs(x), np.abs(w), np.abs(dz))
                check_store(gin, dx, adx, 9 * co, (i, kind, "input gradient"))
        elif kind == "t2":
            x = get(i, 0)
            u = get(i, 1)
            Nn, Hu, Wu, _ = x.shape
            # forward: u = bf16(convT2(x)) (no activation)
            check_store(u, U.convT2(x, w, b), U.convT2(np.abs(x), np.abs(w), np.abs(b)), ci + 1, (i, kind, "forward"))
            g = get(i, 2)
            dx, ew, eb = U.convT2_bwd(x, w, g)
            adx, aw, ab = U.convT2_bwd(np.abs(x), np.abs(w), np.abs(g))
            check_store(get(i, 4), dx, adx, 4 * co, (i, kind, "input gradient"))
            check_sum(gw, ew, aw, wgrad_depth(Nn * Hu * Wu, ci, co), (i, kind, "weight gradient"))
            check_sum(gb, eb, ab, bgrad_depth(g.shape[0] * g.shape[1] * g.shape[2]), (i, kind, "bias gradient"))
        else:   # head: residual, loss and gradients, fp32 on the GPU
            h = get(i, 0)
            gh = get(i, 4)
            rgb = np.stack([(rgba >> (8 * k)) & 0xFF for k in range(3)], -1).astype(np.float64)
            trgb = np.stack([(tgt >> (8 * k)) & 0xFF for k in range(3)], -1).astype(np.float64)
            out = U.head(h, w, b)
            n_el = out.size
            diff = rgb / 255 + out - trgb / 255
            # error of the GPU's fp32 difference: the 33-term head sum (fp32
            # weights times bfloat16 activations), the two colour quotients
            # and the two additions around it
            tout = np.abs(h) @ np.abs(w).T + np.abs(b)
            ediff = g_k(40) * (tout + rgb / 255 + trgb / 255 + np.abs(out))
            dout = 2 * diff / n_el
            edout = 2 * ediff / n_el + g_k(3) * np.abs(dout)
            # per-pixel values summed by a wave butterfly, the waves in order,
            # then the block partials (a sequential pass and a tree)
            Ph = h.shape[0] * h.shape[1] * h.shape[2]
            K = 64 + (Ph + 65535) // 65536
            lref = (diff ** 2).mean()
            assert abs(loss - lref) <= g_k(K) * lref + 2 * np.mean(np.abs(diff) * ediff) + ediff.max() ** 2
            eg = dout @ w
            tg = np.abs(dout) @ np.abs(w)
            bound = 2.0 ** -8 * np.abs(eg) + (1 + 2.0 ** -8) * (g_k(8) * tg + edout @ np.abs(w))
            assert np.all(np.abs(gh - eg) <= bound), ("head input gradient",
                                                       float((np.abs(gh - eg) / (bound + 1e-300)).max()))
            hw = h.reshape(Ph, -1)
            do = dout.reshape(Ph, 3)
            ed = edout.reshape(Ph, 3)
            bw = g_k(K) * (np.abs(do).T @ np.abs(hw)) + ed.T @ np.abs(hw)
            assert np.all(np.abs(gw - do.T @ hw) <= bw), "head weight gradient"
            bb = g_k(K) * np.abs(do).sum(0) + ed.sum(0)
            assert np.all(np.abs(gb - do.sum(0)) <= bb), "head bias gradient"

    # gradients received: what each layer's backward pass was handed is
    # what the layer above produced (plus the skip gradient at a max pool)
    for l in range(levels - 1):
        e2 = 2 * l + 1
        pooled_grad = get(e2 + 1, 4) if levels > 1 else None
        # the skip half of the concat gradient of decoder level l
        dec_c1 = 2 * levels + 3 * (levels - 2 - l) + 1
        skip = get(dec_c1, 4)[..., skip_lo(specs, dec_c1):]
        y = get(e2, 1)
        routed = maxpool_route(y, pooled_grad)
        exact = routed + skip
        check_store(get(e2, 2), exact, np.abs(routed) + np.abs(skip), 2, (e2, "max pool gradient"))
    print(f"  every layer within its rounding bound; loss {loss:.6g}", flush=True)


@pytest.mark.parametrize("levels,N,H,W", [(4, 2, 16, 24), (2, 4, 144, 960),
                                          pytest.param(4, 2, 512, 992, marks=pytest.mark.slow)])
def test_inference_equals_the_traced_forward(F, levels, N, H, W):
    """Inference runs the same convolutions as the training forward (the
    last one with the 1x1 head fused into its epilogue): its residual is
    the head applied to the traced step's last activation, within the fp32
    rounding of the 33-term head sum, and its image the rounding of that."""
    print(f"inference vs traced forward levels={levels} {N}x{H}x{W}", flush=True)
    th, (rgba, depth, cov, _), ws, T, _, _ = run_traced(F, levels, N, H, W, 80 + levels)
    img, res = F.fill(to_t(th.astype(np.float32)), to_t(rgba), to_t(depth), to_t(cov), levels, residual=True)
    res = res.cpu().numpy().astype(np.float64)
    i = len(U.layer_specs(levels)) - 1
    h = tensor(ws, T[5 * i])
    w, b = U.unpack(gpu_theta_view(th, levels), levels)[-1]
    exact = U.head(h, w, b)
    bound = g_k(33) * (np.abs(h) @ np.abs(w).T + np.abs(b))
    assert np.all(np.abs(res - exact) <= bound), float((np.abs(res - exact) / (bound + 1e-300)).max())
    # the image: the rounding of the GPU's own residual, up to one step
    # where the fp32 sum splat/255 + residual lands next to a rounding
    # boundary (fp32 against the fp64 of the check)
    got = img.cpu().numpy().view(np.uint32)
    want = U.fill_image(rgba, res)
    rgb = np.stack([(rgba >> (8 * k)) & 0xFF for k in range(3)], -1).astype(np.float64) / 255.0
    v = np.clip(rgb + res, 0.0, 1.0) * 255.0 + 0.5
    near = np.abs(v - np.round(v)) < 2e-4                   # next to an integer: a rounding boundary
    d = np.abs(got.view(np.uint8).reshape(*got.shape, 4)[..., :3].astype(int) -
               want.view(np.uint8).reshape(*want.shape, 4)[..., :3].astype(int))
    assert d.max() <= 1 and not (d > 0)[~near].any(), (int((d > 0).sum()), int(near.sum()))
    assert np.array_equal(got >> 24, want >> 24)


def skip_lo(specs, i):
    """First channel of the skip half in the concat input of layer i."""
    return specs[i][1] // 2


def maxpool_route(y, gp):
    """Gradient of a 2x2 max pool (first maximum in (0,0), (0,1), (1,0),
    (1,1) order) routed back to its window."""
    _, arg = U.maxpool2(y)
    return U.maxpool2_bwd(arg, gp, y.shape)


def test_traced_step_rejects_small_workspace(F):
    import torch
    levels, N, H, W = 2, 1, 16, 16
    need = F.fill_workspace(levels, N, H, W, F.FHV_FILL_TRACE)
    assert need > F.fill_workspace(levels, N, H, W, F.FHV_FILL_TRAIN)
    assert F.fill_workspace(levels, N, H, W, 3) == 0
    th = params_for(1, levels)
    rgba, depth, cov, tgt = splat_batch(2, N, H, W)
    ws = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    L = F.lib()
    import ctypes as C
    st = L.fhv_fill_train_step_traced(F.ctx(), levels, F._ptr(to_t(th.astype(np.float32))), None, None, 0, 0.0,
                                      F._ptr(to_t(rgba)), F._ptr(to_t(depth)), F._ptr(to_t(cov)), F._ptr(to_t(tgt)),
                                      N, H, W, None, None, F._ptr(ws), ws.numel(), F._stream())
    assert st == -2
    assert math.isfinite(float(need))
    del C

"""CPU oracle for the learned hole-fill network.

TEST INFRASTRUCTURE ONLY (tests, smoke, CPU baseline). Not in the paper: the
fill network is this project's addition. Everything here is plain fp64
numpy; a convolution is written as the explicit patch matrix times the
weight matrix (one library matmul), transposed convolution and pooling as
index arithmetic.

Network: a U-Net of `levels` levels with channels base * 2^l. Per level two
3x3 convolutions (padding 1) with ReLU; 2x2 max pooling going down; a 2x2
stride-2 transposed convolution going up, concatenated (up first, skip
second) with the level's encoder output; a 1x1 head with 3 outputs giving a
residual added to the splat colour.

Tensors are NHWC. Parameters live in one flat vector, layer after layer:
  3x3 convolution     W[co][ky][kx][ci], then bias[co]
  2x2 transposed conv W[dy][dx][co][ci], then bias[co]
  1x1 head            W[k][c] (k < 3),   then bias[k]
Input channels: R, G, B, A / 255, depth - 1 where covered (0 elsewhere),
coverage (0 or 1).
"""
from __future__ import annotations

import numpy as np

IN_CH = 6


# ------------------------------------------------------------ precision

def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    NaN stays NaN; the inputs here are finite."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ------------------------------------------------------------ layout

def layer_specs(levels: int = 4, base: int = 32, in_ch: int = IN_CH):
    """[(kind, cin, cout)] in parameter order."""
    ch = [base * 2 ** l for l in range(levels)]
    s = []
    cin = in_ch
    for l in range(levels):
        s += [("c3", cin, ch[l]), ("c3", ch[l], ch[l])]
        cin = ch[l]
    for l in reversed(range(levels - 1)):
        s += [("t2", ch[l + 1], ch[l]), ("c3", 2 * ch[l], ch[l]), ("c3", ch[l], ch[l])]
    s += [("h1", ch[0], 3)]
    return s


def param_shapes(levels: int = 4, base: int = 32):
    out = []
    for kind, ci, co in layer_specs(levels, base):
        if kind == "c3":
            out.append(((co, 3, 3, ci), (co,)))
        elif kind == "t2":
            out.append(((2, 2, co, ci), (co,)))
        else:
            out.append(((co, ci), (co,)))
    return out


def n_params(levels: int = 4, base: int = 32) -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes(levels, base))


def unpack(theta: np.ndarray, levels: int = 4, base: int = 32):
    """Flat parameter vector -> [(W, b)] views in layer order."""
    out, o = [], 0
    for ws, bs in param_shapes(levels, base):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb]))
        o += nw + nb
    assert o == theta.size
    return out


def init_params(seed: int, levels: int = 4, base: int = 32) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the head starts
    at zero so the untrained network returns the splat unchanged."""
    rng = np.random.default_rng(seed)
    parts = []
    for (kind, ci, co), (ws, bs) in zip(layer_specs(levels, base), param_shapes(levels, base)):
        fan = ci * (9 if kind == "c3" else 4 if kind == "t2" else 1)
        w = rng.standard_normal(ws) * np.sqrt(2.0 / fan) if kind != "h1" else np.zeros(ws)
        parts += [w.reshape(-1), np.zeros(bs)]
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


# ------------------------------------------------------------ layers

def patches3(x: np.ndarray) -> np.ndarray:
    """3x3 patches with zero padding: [N,H,W,C] -> [N,H,W,3,3,C]."""
    N, H, W, C = x.shape
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    P = np.empty((N, H, W, 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            P[:, :, :, ky, kx] = xp[:, ky:ky + H, kx:kx + W]
    return P


def conv3(x, w, b):
    """out[n,y,x,co] = b[co] + sum w[co,ky,kx,ci] x[n,y+ky-1,x+kx-1,ci]."""
    N, H, W, C = x.shape
    P = patches3(x).reshape(N * H * W, 9 * C)
    return (P @ w.reshape(w.shape[0], -1).T + b).reshape(N, H, W, -1)


def conv3_bwd(x, w, dz):
    """Gradients of conv3 w.r.t. input, weights, bias."""
    N, H, W, C = x.shape
    co = w.shape[0]
    d = dz.reshape(-1, co)
    P = patches3(x).reshape(N * H * W, 9 * C)
    dw = (d.T @ P).reshape(w.shape)
    db = d.sum(0)
    dP = (d @ w.reshape(co, -1)).reshape(N, H, W, 3, 3, C)
    dxp = np.zeros((N, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + H, kx:kx + W] += dP[:, :, :, ky, kx]
    return dxp[:, 1:-1, 1:-1], dw, db


def convT2(x, w, b):
    """out[n,2y+dy,2x+dx,co] = b[co] + sum_ci w[dy,dx,co,ci] x[n,y,x,ci]."""
    N, H, W, C = x.shape
    co = w.shape[2]
    out = np.empty((N, 2 * H, 2 * W, co))
    for dy in range(2):
        for dx in range(2):
            out[:, dy::2, dx::2] = x @ w[dy, dx].T + b
    return out


def convT2_bwd(x, w, dz):
    dx_ = np.zeros_like(x)
    dw = np.zeros_like(w)
    for dy in range(2):
        for dx in range(2):
            g = dz[:, dy::2, dx::2]
            dx_ += g @ w[dy, dx]
            dw[dy, dx] = g.reshape(-1, g.shape[-1]).T @ x.reshape(-1, x.shape[-1])
    return dx_, dw, dz.sum((0, 1, 2))


def maxpool2(x):
    """2x2 max pooling; the argmax is the first maximum in the order
    (0,0), (0,1), (1,0), (1,1)."""
    N, H, W, C = x.shape
    v = np.stack([x[:, 0::2, 0::2], x[:, 0::2, 1::2], x[:, 1::2, 0::2], x[:, 1::2, 1::2]])
    return v.max(0), v.argmax(0)


def maxpool2_bwd(arg, dy, shape):
    dx = np.zeros(shape)
    for k, (oy, ox) in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        dx[:, oy::2, ox::2] = dy * (arg == k)
    return dx


def head(x, w, b):
    return x @ w.T + b


# ------------------------------------------------------------ network

def unpack_input(rgba: np.ndarray, depth: np.ndarray, cov: np.ndarray) -> np.ndarray:
    """[N,H,W] splat images -> [N,H,W,6] network input (fp64)."""
    c = np.stack([(rgba >> (8 * k)) & 0xFF for k in range(4)], -1).astype(np.float64) / 255.0
    d = np.where(cov > 0, depth.astype(np.float64) - 1.0, 0.0)[..., None]
    return np.concatenate([c, d, (cov > 0).astype(np.float64)[..., None]], -1)


def forward(theta, x, levels: int = 4, base: int = 32, round_acts: bool = False):
    """Network output (3-channel residual) and the saved activations.

    round_acts=True rounds every stored activation to bfloat16 as the GPU
    stores them (inputs and weights are the caller's to round)."""
    rnd = bf16_round if round_acts else (lambda a: a)
    P = unpack(theta, levels, base)
    acts = {"x": x}
    h = x
    i = 0
    skips = []
    for l in range(levels):
        for s in range(2):
            z = conv3(h, *P[i])
            h = rnd(np.maximum(z, 0.0))
            acts[f"e{l}_{s}"] = h
            i += 1
        if l < levels - 1:
            skips.append(h)
            h, arg = maxpool2(h)
            acts[f"p{l}"] = (h, arg)
    for l in reversed(range(levels - 1)):
        u = rnd(convT2(h, *P[i]))
        i += 1
        h = np.concatenate([u, skips[l]], -1)
        acts[f"cat{l}"] = h
        for s in range(2):
            z = conv3(h, *P[i])
            h = rnd(np.maximum(z, 0.0))
            acts[f"d{l}_{s}"] = h
            i += 1
    out = head(h, *P[i])
    return out, acts


def backward(theta, acts, dout, levels: int = 4, base: int = 32, round_grads: bool = False,
             abs_terms: bool = False):
    """Gradient of sum(dout * output) w.r.t. the flat parameter vector, by
    the chain rule through the layers in reverse order. round_grads=True
    rounds every stored activation gradient to bfloat16 as the GPU does.

    abs_terms=True also returns, per parameter, the sum of the absolute
    values of the terms its gradient adds up (|dz|^T |x| for a weight,
    sum |dz| for a bias, with the same dz and x): the scale of the rounding
    error any order of summation can make in it."""
    rnd = bf16_round if round_grads else (lambda a: a)
    P = unpack(theta, levels, base)
    nl = len(P)
    grads = [None] * nl
    absg = [None] * nl
    # layer indices
    enc = [(2 * l, 2 * l + 1) for l in range(levels)]
    dec = {}
    i = 2 * levels
    for l in reversed(range(levels - 1)):
        dec[l] = (i, i + 1, i + 2)   # t2, c3, c3
        i += 3
    hidx = i
    hlast = acts["d0_1"] if levels > 1 else acts[f"e{levels - 1}_1"]
    grads[hidx] = (dout.reshape(-1, 3).T @ hlast.reshape(-1, hlast.shape[-1]), dout.sum((0, 1, 2)))
    if abs_terms:
        absg[hidx] = (np.abs(dout.reshape(-1, 3)).T @ np.abs(hlast.reshape(-1, hlast.shape[-1])),
                      np.abs(dout).sum((0, 1, 2)))
    g = rnd(dout @ P[hidx][0])
    skip_g = {}
    for l in range(levels - 1):             # decoder, top level first
        it, i1, i2 = dec[l]
        for s, li in ((1, i2), (0, i1)):
            y = acts[f"d{l}_{s}"]
            xin = acts[f"cat{l}"] if s == 0 else acts[f"d{l}_0"]
            gx, dw, db = conv3_bwd(xin, P[li][0], g * (y > 0))
            grads[li] = (dw, db)
            if abs_terms:
                absg[li] = conv3_abs_terms(xin, np.abs(g * (y > 0)), P[li][0].shape)
            g = rnd(gx)
        cu = P[it][0].shape[2]
        g_up, skip_g[l] = g[..., :cu], g[..., cu:]
        hin = acts[f"e{levels - 1}_1"] if l == levels - 2 else acts[f"d{l + 1}_1"]
        gx, dw, db = convT2_bwd(hin, P[it][0], g_up)
        grads[it] = (dw, db)
        if abs_terms:
            _, aw, ab = convT2_bwd(np.abs(hin), np.abs(P[it][0]), np.abs(g_up))
            absg[it] = (aw, ab)
        g = rnd(gx)
    for l in reversed(range(levels)):       # encoder, deepest level first
        if l < levels - 1:
            g = rnd(maxpool2_bwd(acts[f"p{l}"][1], g, acts[f"e{l}_1"].shape) + skip_g[l])
        i0, i1 = enc[l]
        for s, li in ((1, i1), (0, i0)):
            y = acts[f"e{l}_{s}"]
            xin = (acts["x"] if l == 0 else acts[f"p{l - 1}"][0]) if s == 0 else acts[f"e{l}_0"]
            gx, dw, db = conv3_bwd(xin, P[li][0], g * (y > 0))
            grads[li] = (dw, db)
            if abs_terms:
                absg[li] = conv3_abs_terms(xin, np.abs(g * (y > 0)), P[li][0].shape)
            g = rnd(gx)
    flat = lambda gs: np.concatenate([np.concatenate([dw.reshape(-1), db.reshape(-1)]) for dw, db in gs])
    return (flat(grads), flat(absg)) if abs_terms else flat(grads)


def conv3_abs_terms(x, adz, wshape):
    """|dz|^T |patches| and sum |dz|: the absolute term sums of a 3x3
    convolution's weight and bias gradients."""
    N, H, W, C = x.shape
    co = wshape[0]
    d = adz.reshape(-1, co)
    P = np.abs(patches3(x)).reshape(N * H * W, 9 * C)
    return (d.T @ P).reshape(wshape), d.sum(0)


def loss_and_grad(theta, x, rgb_splat, rgb_target, levels: int = 4, base: int = 32,
                  round_acts: bool = False):
    """MSE over the R, G, B values of (splat/255 + residual) vs target/255,
    and its gradient w.r.t. the parameters."""
    out, acts = forward(theta, x, levels, base, round_acts)
    pred = rgb_splat / 255.0 + out
    diff = pred - rgb_target / 255.0
    n = diff.size
    loss = float((diff ** 2).sum() / n)
    dout = 2.0 * diff / n
    return loss, backward(theta, acts, dout, levels, base, round_acts), out


def adam(theta, m, v, g, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; step >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def fill_image(rgba, out_residual) -> np.ndarray:
    """RGBA8 of clamp(splat/255 + residual) (rounded half up), alpha 255."""
    rgb = np.stack([(rgba >> (8 * k)) & 0xFF for k in range(3)], -1).astype(np.float64) / 255.0
    v = np.clip(rgb + out_residual, 0.0, 1.0)
    q = np.floor(v * 255.0 + 0.5).astype(np.uint32)
    return q[..., 0] | (q[..., 1] << 8) | (q[..., 2] << 16) | np.uint32(0xFF000000)

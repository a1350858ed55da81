"""Training and running the learned hole fill on splat images.

Everything numeric runs in libfhv (fhv_capture, fhv_compact, fhv_splat,
fhv_fill, fhv_fill_train_step); this module holds the orchestration: render
splat images for a scene and views, cut random training crops, keep the
parameters and Adam state on the device, and step the optimizer. Training
targets (reference images of the same views) are the caller's: any renderer
of the triangles with a depth test will do.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import fhv, scenes


@dataclass
class SplatImages:
    rgba: torch.Tensor     # int32 [V, H, W]
    depth: torch.Tensor    # float32 [V, H, W]
    cov: torch.Tensor      # uint8 [V, H, W]


def render_splats(mesh, levels: int, views, capacity: int | None = None) -> tuple[SplatImages, int]:
    """Capture `mesh` into per-octant lists at octree depth `levels`, compact
    and splat every view (all of one size). Returns the images and the
    fragment count."""
    d = fhv.desc(fhv.FHV_POFL, levels=levels)
    dm = fhv.to_device(mesh)
    cap = capacity or (1 << 22)
    while True:
        lists = fhv.alloc_lists(d, cap)
        fhv.capture(dm, d, lists)
        F = int(lists.counter.item())
        if F <= cap:
            break
        cap = F               # re-allocate and capture again (overflow rule)
    pofa = fhv.alloc_pofa(cap)
    fhv.compact(lists, d, pofa)
    img = fhv.splat(pofa, d, views)
    return SplatImages(img.rgba, img.depth, img.cov), F


def crop_origins(target: torch.Tensor, n: int, size: int, rng: np.random.Generator, min_cover: float = 0.3,
                 oversample: int = 4) -> np.ndarray:
    """n crop origins (view, y, x) of size x size drawn uniformly, keeping
    only crops with at least min_cover of their pixels covered in the target
    (alpha > 0); the coverage of every candidate comes from a summed-area
    table of the targets (one pass on the host). Origins are distinct."""
    V, H, W = target.shape
    cov = (((target.view(torch.int32) >> 24) & 0xFF) > 0).cpu().numpy()
    sat = np.zeros((V, H + 1, W + 1), np.int64)
    sat[:, 1:, 1:] = cov.cumsum(1).cumsum(2)
    chosen: list[tuple[int, int, int]] = []
    seen = set()
    for _round in range(64):
        if len(chosen) == n:
            break
        m = oversample * (n - len(chosen))
        v = rng.integers(0, V, m)
        y = rng.integers(0, H - size + 1, m)
        x = rng.integers(0, W - size + 1, m)
        c = sat[v, y + size, x + size] - sat[v, y, x + size] - sat[v, y + size, x] + sat[v, y, x]
        for vi, yi, xi, ci in zip(v.tolist(), y.tolist(), x.tolist(), c.tolist()):
            if ci >= min_cover * size * size and (vi, yi, xi) not in seen:
                seen.add((vi, yi, xi))
                chosen.append((vi, yi, xi))
                if len(chosen) == n:
                    break
    if len(chosen) < n:
        raise ValueError(f"only {len(chosen)} of {n} crops reach the coverage {min_cover}")
    return np.array(chosen, np.int64)


def cut_crops(src: SplatImages, target: torch.Tensor, origins: np.ndarray, size: int):
    """The crops at `origins` (rows of view, y, x): device gathers only."""
    dev = target.device
    o = torch.from_numpy(np.ascontiguousarray(origins)).to(dev)
    ar = torch.arange(size, device=dev)
    vv = o[:, 0].view(-1, 1, 1)
    yy = (o[:, 1].view(-1, 1) + ar).view(-1, size, 1)
    xx = (o[:, 2].view(-1, 1) + ar).view(-1, 1, size)
    g = lambda t: t[vv, yy, xx].contiguous()
    return g(src.rgba), g(src.depth), g(src.cov), g(target)


@dataclass
class TrainingSet:
    src: SplatImages          # splats of the training views
    target: torch.Tensor      # reference images of the same views, int32 RGBA8
    views: list               # (scene seed, octree depth, theta) per view


def training_set(reference, seeds, levels_list, views_per_scene: int, rng: np.random.Generator,
                 width: int = 1920, height: int = 1080) -> TrainingSet:
    """Splats and reference images of random orbit views (theta uniform in
    [0, 90) degrees) of the benchmark's scene family (scenes.pofl_scene) at
    each octree depth of levels_list. reference(mesh, levels, view) returns
    the reference RGBA8 image [H, W] of a view (int32 device tensor)."""
    srcs, tgts, meta = [], [], []
    for seed in seeds:
        mesh = scenes.pofl_scene(seed)
        for L in levels_list:
            thetas = [float(t) for t in rng.uniform(0.0, 90.0, views_per_scene)]
            views = [scenes.cube_view(t, L, width, height) for t in thetas]
            img, _ = render_splats(mesh, L, views)
            srcs.append(img)
            tgts.append(torch.stack([reference(mesh, L, v) for v in views]))
            meta += [(seed, L, t) for t in thetas]
    cat = lambda f: torch.cat([getattr(i, f) for i in srcs])
    return TrainingSet(SplatImages(cat("rgba"), cat("depth"), cat("cov")), torch.cat(tgts), meta)


def train(model: "FillModel", ts: TrainingSet, n_crops: int, batch: int, size: int, rng: np.random.Generator,
          lr0: float = 1e-3, lr1: float = 5e-5) -> int:
    """Adam steps over n_crops distinct random crops (n_crops / batch steps,
    cosine learning-rate decay); crops are cut on the device, so the loop
    waits for nothing. Returns the number of steps."""
    origins = crop_origins(ts.target, n_crops, size, rng)
    steps = n_crops // batch
    for st in range(steps):
        rgba, depth, cov, tgt = cut_crops(ts.src, ts.target, origins[st * batch:(st + 1) * batch], size)
        model.train_step(rgba, depth, cov, tgt, lr_at(st + 1, steps, lr0, lr1))
    return steps


def evaluate(model: "FillModel", reference, seeds, levels: int, thetas=(30.0, 60.0), width: int = 1920,
             height: int = 1080) -> list[dict]:
    """PSNR over RGB of the plain splat and of the filled splat against the
    reference image, per (held-out scene, view)."""
    out = []
    for seed in seeds:
        mesh = scenes.pofl_scene(seed)
        for th in thetas:
            v = scenes.cube_view(th, levels, width, height)
            img, _ = render_splats(mesh, levels, [v])
            ref = reference(mesh, levels, v)
            out.append({"seed": seed, "levels": levels, "theta": th,
                        "psnr_splat_db": psnr_rgb(img.rgba[0], ref), "psnr_fill_db": psnr_rgb(model.fill(img)[0], ref)})
    return out


class FillModel:
    """Parameters (fp32) and Adam moments on the device."""

    def __init__(self, levels: int = 4, seed: int = 0, device="cuda"):
        self.levels = levels
        n = fhv.unet_param_count(levels)
        self.params = torch.from_numpy(init_params(seed, levels)).to(device)
        assert self.params.numel() == n
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self._ws = None

    def train_step(self, rgba, depth, cov, target, lr: float) -> torch.Tensor:
        self.step += 1
        self._ws = fhv.fill_train_step(self.params, self.m, self.v, self.step, lr, rgba, depth, cov,
                                       target, self.levels, loss=self.loss, ws=self._ws)
        return self.loss

    def fill(self, img: SplatImages) -> torch.Tensor:
        out, _ = fhv.fill(self.params, img.rgba, img.depth, img.cov, self.levels)
        return out

    def state(self) -> dict:
        return {"params": self.params.cpu().numpy(), "m": self.m.cpu().numpy(),
                "v": self.v.cpu().numpy(), "step": self.step, "levels": self.levels}


def init_params(seed: int, levels: int = 4) -> np.ndarray:
    """He-normal convolution weights, zero biases, zero head (the untrained
    network returns the splat), in the parameter layout of fhv_fill."""
    rng = np.random.default_rng(seed)
    ch = [32 << l for l in range(levels)]
    parts = []

    def conv(ci, co, taps, shape):
        parts.append(rng.standard_normal(shape).reshape(-1) * math.sqrt(2.0 / (ci * taps)))
        parts.append(np.zeros(co))
    cin = 6
    for l in range(levels):
        conv(cin, ch[l], 9, (ch[l], 3, 3, cin))
        conv(ch[l], ch[l], 9, (ch[l], 3, 3, ch[l]))
        cin = ch[l]
    for l in reversed(range(levels - 1)):
        conv(ch[l + 1], ch[l], 4, (2, 2, ch[l], ch[l + 1]))
        conv(2 * ch[l], ch[l], 9, (ch[l], 3, 3, 2 * ch[l]))
        conv(ch[l], ch[l], 9, (ch[l], 3, 3, ch[l]))
    parts += [np.zeros(3 * ch[0]), np.zeros(3)]
    return np.concatenate(parts).astype(np.float32)


def lr_at(step: int, total: int, lr0: float, lr1: float) -> float:
    """Cosine decay from lr0 to lr1 over `total` steps."""
    t = min(max(step / max(total, 1), 0.0), 1.0)
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * t))


def training_scene(seed: int, n_tri: int = 200_000) -> "scenes.Mesh":
    """Many small objects (the large-scene regime): subdivided icospheres and
    boxes of about 100 triangles at scales 0.02-0.1 over a ground grid."""
    return scenes.cube_scene(n_tri, seed, scale_range=(0.02, 0.1), n_objects=n_tri // 100)


def psnr_rgb(a: torch.Tensor, b: torch.Tensor) -> float:
    """PSNR over the R, G, B bytes of two RGBA8 images (MAX = 255)."""
    ai = a.view(torch.int32)
    bi = b.view(torch.int32)
    se = 0.0
    for k in range(3):
        d = ((ai >> (8 * k)) & 0xFF).double() - ((bi >> (8 * k)) & 0xFF).double()
        se += float((d * d).sum())
    mse = se / (3.0 * ai.numel())
    return float("inf") if mse == 0 else 10.0 * math.log10(255.0 ** 2 / mse)


def gpu_reference(mesh, levels: int, view) -> torch.Tensor:
    """reference_render's image as [H, W]."""
    return reference_render(mesh, levels, view)[0]


def reference_render(mesh, levels: int, view) -> torch.Tensor:
    """Depth-tested rendering of the triangles themselves into `view`, on the
    GPU through the per-pixel capture: the vertices (grid units) are taken to
    the view's screen space on the host (fp64, stored fp32), captured per
    pixel at the output size, and the nearest fragment of every pixel kept
    (Sec. 3.3: a splat of per-pixel lists back into the capture view selects
    each list's nearest fragment). Returns RGBA8 [1, H, W] (0 where empty)."""
    W, H = view.width, view.height
    G = float(2 ** (levels + 8))
    m = view.m.astype(np.float64)
    p = mesh.pos.astype(np.float64) * G
    s = p @ m[:, :3].T + m[:, 3]
    clip = np.empty_like(s)
    clip[:, 0] = s[:, 0] / W * 2.0 - 1.0
    clip[:, 1] = s[:, 1] / H * 2.0 - 1.0
    clip[:, 2] = (s[:, 2] - 1.0) * 2.0 - 1.0
    cm = scenes.Mesh(clip.astype(np.float32), mesh.rgba, mesh.tri, None)
    d = fhv.desc(fhv.FHV_PPFL, W, H)
    dm = fhv.to_device(cm)
    cap = 1 << 22
    while True:
        lists = fhv.alloc_lists(d, cap)
        fhv.capture(dm, d, lists)
        F = int(lists.counter.item())
        if F <= cap:
            break
        cap = F
    pofa = fhv.alloc_pofa(cap)
    fhv.compact(lists, d, pofa)
    return fhv.splat(pofa, d, [scenes.ppfl_view(0.0, W, H)]).rgba

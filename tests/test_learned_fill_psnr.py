"""The trained fill beats the plain splat at the benchmark's configuration.

Training pairs: splats of per-octant arrays of the benchmark's scene family
(200k triangles, seeds 100-115), two random orbit views each in [0, 90)
degrees at octree depths 9 and 8, 1920x1080, standard footprint, against
the oracle's direct rasterization of the same views; 20,000 distinct random
256x256 crops in batches of 8, trained on the GPU by the library's own
forward and backward kernels. Evaluation on held-out scenes (seeds 0-9) at
30 and 60 degrees, at depth 9 (the benchmark's step) and depth 8: PSNR over
RGB of the filled image and of the plain splat, both against the oracle's
direct raster. Stated margin: at least 1.0 dB on every evaluated view."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

MARGIN_DB = 1.0
W, H = 1920, 1080


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2211_15460_amd import fhv, learned_fill, scenes
    fhv.lib()
    return torch, oracle, learned_fill, scenes


def oracle_reference(torch, O):
    def ref(mesh, levels, view):
        img = O.direct_raster(1, mesh, view, levels=levels)[0]
        return torch.from_numpy(np.ascontiguousarray(img).view(np.int32)).cuda()
    return ref


def test_fill_beats_plain_splat(env):
    torch, O, LF, S = env
    ref = oracle_reference(torch, O)
    rng = np.random.default_rng(0)
    ts = LF.training_set(ref, range(100, 116), (9, 8), 2, rng, W, H)
    model = LF.FillModel(4, 0)
    steps = LF.train(model, ts, 20000, 8, 256, rng)
    assert steps == 2500 and np.isfinite(model.loss.item())
    del ts
    for L in (9, 8):
        ev = LF.evaluate(model, ref, range(10), L, width=W, height=H)
        for e in ev:
            print(f"depth {L} seed {e['seed']} theta {e['theta']}: splat {e['psnr_splat_db']:.2f} dB, "
                  f"fill {e['psnr_fill_db']:.2f} dB", flush=True)
        gains = [e["psnr_fill_db"] - e["psnr_splat_db"] for e in ev]
        assert min(gains) >= MARGIN_DB, (L, gains)


def test_gpu_reference_render_matches_direct_raster(env):
    """The GPU reference renderer the benchmark uses for its PSNR agrees with
    the oracle's direct raster at the benchmark's configuration: the same
    coverage up to a few edge pixels, and colours that differ only where
    depth ties or fp32-stored vertices move a sample across an edge."""
    torch, O, LF, S = env
    for seed, L in ((3, 9), (4, 8)):
        mesh = S.pofl_scene(seed)
        for th in (30.0, 60.0):
            v = S.cube_view(th, L, W, H)
            got = LF.gpu_reference(mesh, L, v).cpu().numpy().view(np.uint32)
            ref, _, cov = O.direct_raster(1, mesh, v, levels=L)
            mism = ((got != 0) != (cov == 1)).mean()
            p = O.psnr_rgb(got, ref)
            print(f"seed {seed} depth {L} theta {th}: coverage mismatch {mism:.2e}, PSNR {p:.1f} dB", flush=True)
            assert mism < 1e-3
            assert p > 35.0

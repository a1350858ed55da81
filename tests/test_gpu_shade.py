"""Shading of splat winners (fhv_shade, Sec. 5 Blinn-Phong from the packed
normals) against the oracle bit for bit, on the oracle's own splat of its own
arrays; a stereo pair (two views from one FHV in one splat call) shaded the
same way; argument errors."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S
from tests.gpu_util import run_capture, run_compact, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    return fhv


def arrays_of(F, orc, mesh, L, cap=1 << 21):
    d = F.desc(F.FHV_POFL, levels=L)
    _, _, _, cnt, lists = run_capture(F, mesh, d, cap)
    g, pofa = run_compact(F, lists, d)
    oh, op, oc = orc.capture_pofl(mesh, L, cap)
    o = orc.compact(oh, op, oc)
    for f in ("key", "off", "cnt", "frag"):
        assert np.array_equal(g[f], o[f]), f
    return d, o, pofa


@pytest.mark.parametrize("L,W,H", [(6, 160, 96), (9, 1920, 1080)])
def test_shade_matches_oracle(F, orc, L, W, H):
    import torch
    mesh = S.cube_scene(4000 if L == 6 else 60_000, 71, scale_range=(0.05, 0.3), ground=8)
    d, o, pofa = arrays_of(F, orc, mesh, L, cap=1 << 22)
    views = S.stereo_views(30.0, L, W, H, splat_px=1) + [S.cube_view(t, L, W, H, splat_px=1) for t in (0.0, 75.0)]
    lights = np.stack([F.light_vectors(v, (0.3, 1.0, -0.5), 0.15, 0.7, 0.35, s)
                       for v, s in zip(views, (0, 3, 5, 8))])
    img = F.splat(pofa, d, views)
    out = F.shade(pofa, img, lights)
    torch.cuda.synchronize()
    _, _, ocov, ozb = orc.splat(1, o["key"], o["frag"], views, levels=L, return_zbuf=True)
    assert np.array_equal(u64(img.zbuf), ozb)
    want = orc.shade(o["frag"], ozb, lights)
    got = out.cpu().numpy()
    print(f"L={L} {W}x{H}: {int(ocov.sum())} shaded pixels", flush=True)
    assert np.array_equal(got, want)
    assert np.all(got[..., 3] == ocov.astype(np.float32))


def test_stereo_pair_is_two_views_of_one_fhv(F, orc):
    import torch
    L = 6
    mesh = S.cube_scene(3000, 72, scale_range=(0.05, 0.3), ground=8)
    d, o, pofa = arrays_of(F, orc, mesh, L)
    pair = S.stereo_views(20.0, L, 128, 80, eye_deg=6.0, splat_px=1)
    both = F.splat(pofa, d, pair)
    torch.cuda.synchronize()
    zb = u64(both.zbuf)
    for e, v in enumerate(pair):
        one = F.splat(pofa, d, [v])
        torch.cuda.synchronize()
        assert np.array_equal(u64(one.zbuf)[0], zb[e])
    assert not np.array_equal(zb[0], zb[1])     # the eyes see different images


def test_shade_rejects_bad_arguments(F):
    import torch
    Lb = F.lib()
    pofa = F.alloc_pofa(16)
    zb = torch.full((1, 4, 4), -1, dtype=torch.int64, device="cuda")
    out = torch.empty((1, 4, 4, 4), dtype=torch.float32, device="cuda")
    lt = (F.Light_ * 1)()
    lt[0].shine = 17
    ps = pofa.struct()
    call = lambda n, w, h: Lb.fhv_shade(F.ctx(), C.byref(ps), C.c_void_p(zb.data_ptr()), n, w, h, lt,
                                        C.c_void_p(out.data_ptr()), None)
    assert call(1, 4, 4) == -1
    lt[0].shine = 3
    assert call(0, 4, 4) == -3 and call(1, 0, 4) == -3
    assert call(1, 4, 4) == 0
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out).item()) == 0

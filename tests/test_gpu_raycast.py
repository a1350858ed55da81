"""Ray casting (fhv_raycast) against the oracle, bit for bit: the nearest
fragment ("R") equals the splat in every pixel, and front-to-back
transparency ("R/T") equals the oracle's fp32 compositing for several
thresholds, for pixels met by more fragments than one walk keeps (repeated
walks), for the Fig. 2 example, at octree depths 1 and 10, on empty arrays,
and at the benchmark's full size (200k triangles, depth 9, three 1080p
views). Argument errors are rejected before any launch."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S
from tests.gpu_util import run_capture, run_compact, run_splat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    return fhv


def with_alpha(mesh, seed):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 256, mesh.rgba.size, dtype=np.uint32)
    return S.Mesh(mesh.pos, (mesh.rgba & 0x00FFFFFF) | (a << 24), mesh.tri, mesh.obj)


def arrays_of(F, orc, mesh, L, cap=1 << 21):
    """The GPU's arrays (for the GPU's ray casting) and the oracle's own
    arrays (for the oracle's), checked equal on the way."""
    d = F.desc(F.FHV_POFL, levels=L)
    _, _, _, cnt, lists = run_capture(F, mesh, d, cap)
    assert cnt <= cap
    g, pofa = run_compact(F, lists, d)
    oh, op, oc = orc.capture_pofl(mesh, L, cap)
    o = orc.compact(oh, op, oc)
    for f in ("key", "off", "cnt", "frag"):
        assert np.array_equal(g[f], o[f]), f
    return d, o, pofa


def cast(F, pofa, d, views, mode, tau=0.0):
    import torch
    out = F.raycast(pofa, d, views, mode=mode, tau=tau)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_nearest_is_the_splat(F, orc):
    L = 6
    mesh = with_alpha(S.cube_scene(4000, 11, scale_range=(0.05, 0.3), ground=8), 1)
    d, g, pofa = arrays_of(F, orc, mesh, L)
    views = [S.cube_view(t, L, 160, 96, splat_px=1) for t in (0.0, 30.0, 75.0)]
    out = cast(F, pofa, d, views, F.FHV_RAY_NEAREST)
    rgba, _, cov = run_splat(F, pofa, d, views)
    assert np.array_equal(out[..., 3], cov.astype(np.float32))
    for k in range(3):
        want = ((rgba >> (8 * k)) & 0xFF).astype(np.float32) / np.float32(255)
        assert np.array_equal(out[..., k], np.where(cov == 1, want, np.float32(0)))
    o, _ = orc.raycast(g["key"], g["frag"], views, L, mode=0)
    assert np.array_equal(out, o)


@pytest.mark.parametrize("tau", [0.0, 1.0 / 256, 0.5, 1.0])
def test_blend_matches_oracle(F, orc, tau):
    L = 6
    mesh = with_alpha(S.cube_scene(4000, 12, scale_range=(0.05, 0.3), ground=8), 2)
    d, g, pofa = arrays_of(F, orc, mesh, L)
    views = [S.cube_view(t, L, 160, 96, splat_px=1) for t in (0.0, 40.0, 90.0, 200.0)]
    out = cast(F, pofa, d, views, F.FHV_RAY_BLEND, tau)
    o, deepest = orc.raycast(g["key"], g["frag"], views, L, mode=1, tau=tau)
    print(f"tau={tau} deepest pixel {deepest} fragments", flush=True)
    assert np.array_equal(out, o)


def stacked_planes(n, alpha, seed):
    """n parallel squares at z = 0.1 + 0.8 i / n, each in one colour with the
    given alpha: every pixel behind the square is met n times."""
    rng = np.random.default_rng(seed)
    pos, col = [], []
    for i in range(n):
        z = 0.1 + 0.8 * i / n
        c = int(rng.integers(0, 1 << 24)) | (alpha << 24)
        for tri in (((0.2, 0.2, z), (0.8, 0.2, z), (0.8, 0.8, z)), ((0.2, 0.2, z), (0.8, 0.8, z), (0.2, 0.8, z))):
            pos.extend(tri)
            col.extend([c] * 3)
    pos = np.asarray(pos, np.float32)
    return S.Mesh(pos, np.asarray(col, np.uint32), np.arange(pos.shape[0], dtype=np.uint32).reshape(-1, 3),
                  np.zeros(pos.shape[0] // 3, np.uint8))


@pytest.mark.parametrize("tau", [0.0, 1.0 / 256])
def test_deep_pixels_take_several_walks(F, orc, tau):
    L = 5
    mesh = stacked_planes(40, 12, 3)
    d, g, pofa = arrays_of(F, orc, mesh, L)
    views = [S.cube_view(t, L, 64, 40, splat_px=1) for t in (0.0, 20.0)]
    out = cast(F, pofa, d, views, F.FHV_RAY_BLEND, tau)
    o, deepest = orc.raycast(g["key"], g["frag"], views, L, mode=1, tau=tau)
    print(f"deepest pixel {deepest} fragments", flush=True)
    assert deepest > 2 * 16
    assert np.array_equal(out, o)


def test_fig2_weights(F, orc):
    """Three quads of alpha 1/3, red in front of green in front of blue."""
    L = 4
    quads = []
    for z, c in ((0.3, 0x550000FF), (0.5, 0x5500FF00), (0.7, 0x55FF0000)):
        quads.append((z, c))
    pos, col = [], []
    for z, c in quads[::-1]:      # insertion order differs from depth order
        for tri in (((0.3, 0.3, z), (0.7, 0.3, z), (0.7, 0.7, z)), ((0.3, 0.3, z), (0.7, 0.7, z), (0.3, 0.7, z))):
            pos.extend(tri)
            col.extend([c] * 3)
    pos = np.asarray(pos, np.float32)
    mesh = S.Mesh(pos, np.asarray(col, np.uint32), np.arange(pos.shape[0], dtype=np.uint32).reshape(-1, 3),
                  np.zeros(pos.shape[0] // 3, np.uint8))
    d, g, pofa = arrays_of(F, orc, mesh, L)
    views = [S.cube_view(0.0, L, 64, 40, splat_px=1)]
    out = cast(F, pofa, d, views, F.FHV_RAY_BLEND)
    o, _ = orc.raycast(g["key"], g["frag"], views, L, mode=1)
    assert np.array_equal(out, o)
    centre = out[0, 20, 32]
    assert np.allclose(centre, [1 / 3, 2 / 9, 4 / 27, 19 / 27], atol=1e-6)


@pytest.mark.parametrize("L", [1, 10])
def test_depth_extremes(F, orc, L):
    # small objects and no ground at depth 10 (2^11 samples per cube side)
    mesh = with_alpha(S.cube_scene(300 if L == 10 else 600, 13, scale_range=(0.02, 0.05) if L == 10 else (0.1, 0.4),
                                   ground=0 if L == 10 else 4), 4)
    d, g, pofa = arrays_of(F, orc, mesh, L, cap=1 << 20)
    views = [S.cube_view(t, L, 640, 400, splat_px=1) for t in (10.0, 50.0)]
    print(f"L={L} fragments {g['frag'].shape[0]}", flush=True)
    for mode in (F.FHV_RAY_NEAREST, F.FHV_RAY_BLEND):
        out = cast(F, pofa, d, views, mode, 1.0 / 256)
        o, _ = orc.raycast(g["key"], g["frag"], views, L, mode=mode, tau=1.0 / 256)
        assert np.array_equal(out, o)


def test_empty_arrays(F):
    import torch
    L = 6
    d = F.desc(F.FHV_POFL, levels=L)
    pofa = F.alloc_pofa(1024)
    pofa.n_occ.zero_()
    pofa.n_frag.zero_()
    views = [S.cube_view(0.0, L, 32, 24, splat_px=1)]
    out = F.raycast(pofa, d, views, mode=F.FHV_RAY_BLEND)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out).item()) == 0


def test_rejects_bad_arguments(F):
    import torch
    Lb = F.lib()
    L = 6
    d = F.desc(F.FHV_POFL, levels=L)
    pofa = F.alloc_pofa(1024)
    pofa.n_occ.zero_()
    ps = pofa.struct()
    out = torch.empty((1, 24, 32, 4), dtype=torch.float32, device="cuda")
    need = F.raycast_workspace(d)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    good = F.views_struct([S.cube_view(0.0, L, 32, 24, splat_px=1)])
    call = lambda dd, vs, mode=1, tau=0.0, nbytes=need: Lb.fhv_raycast(
        F.ctx(), C.byref(ps), C.byref(dd), vs, 1, mode, tau, C.c_void_p(out.data_ptr()),
        C.c_void_p(ws.data_ptr()), nbytes, None)
    assert call(d, good) == 0
    torch.cuda.synchronize()
    assert call(F.desc(F.FHV_PPFL, 32, 24), good) == -1
    assert call(d, F.views_struct([S.cube_view(0.0, L, 32, 24, splat_px=2)])) == -1
    assert call(d, good, mode=2) == -1
    assert call(d, good, tau=float("nan")) == -1
    assert call(d, good, nbytes=need - 1) == -2
    assert Lb.fhv_raycast_workspace(C.byref(F.desc(F.FHV_POFL, levels=11))) == 0
    assert call(F.desc(F.FHV_POFL, levels=11), good) == -3


def test_full_size_benchmark_scene(F, orc):
    """The benchmark's arrays (200k triangles, depth 9) cast into its three
    1080p views, both modes, against the oracle."""
    L = 9
    mesh = with_alpha(S.pofl_scene(0, 200_000), 5)
    d, g, pofa = arrays_of(F, orc, mesh, L, cap=6 << 20)
    views = [S.cube_view(t, L, 1920, 1080, splat_px=1) for t in (0.0, 30.0, 60.0)]
    print(f"full size: {g['frag'].shape[0]} fragments", flush=True)
    for mode, tau in ((F.FHV_RAY_NEAREST, 0.0), (F.FHV_RAY_BLEND, 1.0 / 256)):
        out = cast(F, pofa, d, views, mode, tau)
        o, deepest = orc.raycast(g["key"], g["frag"], views, L, mode=mode, tau=tau)
        print(f"mode {mode}: deepest pixel {deepest}", flush=True)
        assert np.array_equal(out, o)

"""The splat's screen tiles against the oracle, bit for bit, where the tile
walk has cases of its own: footprints up to the largest side (a chunk's box
then reaches many tiles), one view per footprint side in one call, views of
one pixel, ragged tile edges, views with part of the scene behind the viewer
or entirely off screen, matrices that are not finite, a truncated octant
table, 32 views in one call, and tiles that so many chunk groups reach that
they are split into 2 to 16 sub-tiles drawn by separate workgroups."""
from __future__ import annotations

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


@pytest.fixture(scope="module")
def scene(F, orc):
    mesh = S.cube_scene(20000, 31)
    L = 7
    d = F.desc(F.FHV_POFL, levels=L)
    _, _, _, cnt, lists = run_capture(F, mesh, d, 1 << 22)
    g, pofa = run_compact(F, lists, d)
    print(f"tile scene F={cnt} n_occ={g['n_occ']}", flush=True)
    return mesh, L, d, g, pofa


def check(F, orc, scene, views, keys=None, pofa=None):
    _, L, d, g, pf = scene
    pofa = pf if pofa is None else pofa
    keys = g["key"] if keys is None else keys
    gr, gd, gc = run_splat(F, pofa, d, views)
    orr, od, oc = orc.splat(1, keys, g["frag"], views, levels=L)
    assert np.array_equal(gc, oc)
    assert np.array_equal(gr, orr)
    assert np.array_equal(gd.view(np.uint32), od.view(np.uint32))
    return oc


def test_large_footprints(F, orc, scene):
    _, L, _, _, _ = scene
    for k in (17, 64):
        cov = check(F, orc, scene, [S.cube_view(40.0, L, 300, 200, splat_px=k)])
        assert cov.mean() > 0.1   # the footprints cover a good part of the view


def test_per_view_footprints_in_one_call(F, orc, scene):
    _, L, _, _, _ = scene
    views = [S.cube_view(15.0 * i, L, 257, 129, splat_px=k) for i, k in enumerate((1, 2, 3, 5, 8))]
    check(F, orc, scene, views)


@pytest.mark.parametrize("W,H", [(1, 1), (65, 1), (1, 65), (129, 63), (64, 64), (200, 331)])
def test_ragged_and_tiny_views(F, orc, scene, W, H):
    _, L, _, _, _ = scene
    check(F, orc, scene, [S.cube_view(25.0, L, W, H), S.cube_view(70.0, L, W, H, splat_px=2)])


def test_views_behind_and_off_screen(F, orc, scene):
    _, L, _, _, _ = scene
    behind = S.cube_view(30.0, L, 160, 120)
    m = behind.m.copy()
    m[2, 3] -= np.float32(1.5)          # depth < 0 for about half of the scene
    behind = S.View(m, 160, 120, 1)
    off = S.cube_view(30.0, L, 160, 120)
    m = off.m.copy()
    m[0, 3] += np.float32(5000.0)       # everything far to the right
    off = S.View(m, 160, 120, 1)
    cov = check(F, orc, scene, [behind, off])
    assert cov[0].sum() > 0 and cov[1].sum() == 0


def test_non_finite_matrices_draw_nothing(F, orc, scene):
    _, L, _, _, _ = scene
    views = []
    for bad in (np.nan, np.inf, -np.inf):
        v = S.cube_view(30.0, L, 96, 80)
        m = v.m.copy()
        m[0, 1] = np.float32(bad)
        views.append(S.View(m, 96, 80, 1))
    cov = check(F, orc, scene, views)
    assert cov.sum() == 0


def test_truncated_table(F, orc, scene):
    """Fragments whose octant row was not stored are not drawn."""
    _, L, d, g, _ = scene
    import torch
    pofa = F.alloc_pofa(g["frag"].shape[0], 500)
    pofa.frag[: g["frag"].shape[0]] = torch.from_numpy(g["frag"].view(np.int32)).cuda()
    pofa.oct_key[:500] = torch.from_numpy(g["key"][:500].view(np.int64)).cuda()
    pofa.n_frag[0] = g["frag"].shape[0]
    pofa.n_occ[0] = g["n_occ"]
    cov = check(F, orc, scene, [S.cube_view(10.0, L, 200, 150)], keys=g["key"][:500], pofa=pofa)
    assert 0 < cov.sum()


def test_thirty_two_views(F, orc, scene):
    _, L, _, _, _ = scene
    views = [S.cube_view(360.0 * i / 32, L, 120, 90, splat_px=1 + i % 3) for i in range(32)]
    check(F, orc, scene, views)


def test_empty_arrays(F, orc):
    """No fragments: every pixel empty."""
    d = F.desc(F.FHV_POFL, levels=5)
    mesh = S.Mesh(np.zeros((3, 3), np.float32), np.zeros(3, np.uint32), np.zeros((0, 3), np.uint32), None)
    _, _, _, cnt, lists = run_capture(F, mesh, d, 64)
    _, pofa = run_compact(F, lists, d)
    gr, gd, gc = run_splat(F, pofa, d, [S.cube_view(30.0, 5, 70, 70)])
    assert cnt == 0 and gc.sum() == 0 and np.all(gr == 0) and np.all(gd == 0)


@pytest.fixture(scope="module")
def dense_scene(F, orc):
    # 2.7 M fragments, about 660 groups of 64 chunks: a view that holds the
    # whole scene in one 64 x 64 tile splits that tile into 16 sub-tiles,
    # larger views into fewer pieces per tile (at 100 x 100 some of them
    # partly outside the image); with four one-tile views the
    # launch's budget of extra workgroups (16) runs out after the first
    # split, so the other tiles are drawn whole
    mesh = S.cube_scene(80000, 3)
    L = 9
    d = F.desc(F.FHV_POFL, levels=L)
    _, _, _, cnt, lists = run_capture(F, mesh, d, 1 << 22)
    assert cnt <= 1 << 22
    g, pofa = run_compact(F, lists, d)
    print(f"dense scene F={cnt} n_occ={g['n_occ']}", flush=True)
    return mesh, L, d, g, pofa


@pytest.mark.parametrize("size,views", [(64, ((0.0, 1), (25.0, 3), (50.0, 1), (75.0, 2))),
                                        (128, ((10.0, 1), (40.0, 2))),
                                        (192, ((60.0, 3),)),
                                        (100, ((15.0, 1), (35.0, 2)))])
def test_split_tiles(F, orc, dense_scene, size, views):
    _, L, _, _, _ = dense_scene
    vs = [S.cube_view(th, L, size, size, vertical_extent=1.7, splat_px=k) for th, k in views]
    print(f"split tiles: {len(vs)} views of {size}x{size}", flush=True)
    cov = check(F, orc, dense_scene, vs)
    assert cov.reshape(len(vs), -1).sum(axis=1).min() > 0

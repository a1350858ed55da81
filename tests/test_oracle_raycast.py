"""Pins of the oracle's ray casting (Sec. 3.3, evaluation by ray casting)
against facts that do not come from its code: the compositing weights of
the Fig. 2 example (three quads of alpha 1/3: 1/3, 2/9 and 4/27), the
nearest-fragment mode against the oracle's independent splat, the
closed-form product of transmittances in fp64, the threshold's effect and
independence from the order of the fragment array."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S


def _view(m, W, H):
    return S.View(np.asarray(m, np.float32).reshape(3, 4), W, H, 1)


def _pofa(orc, L, recs):
    """Per-octant arrays from (leaf x, y, z, sub x, y, z, rgba) records:
    table keys ascending, records grouped by key, w3 = octant rank."""
    rows = sorted(recs, key=lambda r: orc.morton3(r[0], r[1], r[2], L))
    keys = sorted({orc.morton3(r[0], r[1], r[2], L) for r in rows})
    frag = []
    for r in rows:
        k = orc.morton3(r[0], r[1], r[2], L)
        frag.append([r[3] | (r[4] << 8) | (r[5] << 16), r[6], 0, keys.index(k)])
    return np.array(keys, np.uint64), np.array(frag, np.uint32).reshape(-1, 4)


def test_fig2_three_quads_weights(orc):
    """Fig. 2: red nearest, then green, then blue along the view, each with
    alpha 1/3; the pixel is red/3 + green 2/9 + blue 4/27, opacity 19/27."""
    L = 2                                    # 1024 grid units per side
    m = [[1 / 256, 0, 0, 0], [0, 1 / 256, 0, 0], [0, 0, 1 / 1024, 1.0]]
    red, green, blue = 0x550000FF, 0x5500FF00, 0x55FF0000      # alpha 85 = 255/3
    keys, frag = _pofa(orc, L, [(1, 2, 3, 9, 9, 9, blue), (1, 2, 0, 9, 9, 9, red),
                                (1, 2, 1, 9, 9, 9, green)])
    out, deepest = orc.raycast(keys, frag, [_view(m, 4, 4)], L, mode=1)
    assert deepest == 3
    px = out[0, 2, 1]
    assert abs(px[0] - 1 / 3) < 1e-6 and abs(px[1] - 2 / 9) < 1e-6 and abs(px[2] - 4 / 27) < 1e-6
    assert abs(px[3] - 19 / 27) < 1e-6
    others = np.ones((4, 4), bool)
    others[2, 1] = False
    assert np.all(out[0][others] == 0)
    # simple ray casting keeps the nearest alone, opaque
    out, _ = orc.raycast(keys, frag, [_view(m, 4, 4)], L, mode=0)
    assert np.array_equal(out[0, 2, 1], np.array([1, 0, 0, 1], np.float32))


def _scene(seed, L):
    rng = np.random.default_rng(seed)
    mesh = S.cube_scene(2500, seed, scale_range=(0.05, 0.3), ground=8)
    # random alpha per vertex (the generator's colours keep their RGB)
    mesh = S.Mesh(mesh.pos, (mesh.rgba & 0x00FFFFFF) | (rng.integers(0, 256, mesh.rgba.size, dtype=np.uint32) << 24),
                  mesh.tri, mesh.obj)
    return mesh


@pytest.fixture(scope="module")
def arrays(orc):
    L = 6
    mesh = _scene(3, L)
    head, pool, cnt = orc.capture_pofl(mesh, L, 1 << 21)
    o = orc.compact(head, pool, cnt)
    views = [S.cube_view(t, L, 96, 64, splat_px=1) for t in (0.0, 35.0, 80.0)]
    return L, o, views


def test_nearest_mode_is_the_splat(orc, arrays):
    """Simple ray casting ("R") and the one-pixel splat pick the same fragment
    in every pixel (both order by depth, then index)."""
    L, o, views = arrays
    out, deepest = orc.raycast(o["key"], o["frag"], views, L, mode=0)
    rgba, _, cov = orc.splat(1, o["key"], o["frag"], views, levels=L)
    assert deepest > 3
    assert np.array_equal(out[..., 3], cov.astype(np.float32))
    for k in range(3):
        want = ((rgba >> (8 * k)) & 0xFF).astype(np.float32) / np.float32(255)
        assert np.array_equal(out[..., k], np.where(cov == 1, want, 0))


def _fragment_lists(orc, o, view, L):
    """(pixel, depth, rgba) of every fragment, from the geometry of the
    Morton grid (not the oracle's code)."""
    keys, frag = o["key"], o["frag"]
    k = keys[frag[:, 3]].astype(np.int64)
    xyz = np.zeros((k.size, 3), np.int64)
    for b in range(L):
        for a in range(3):
            xyz[:, a] |= ((k >> (3 * b + 2 - a)) & 1) << b
    sub = np.stack([frag[:, 0] & 0xFF, (frag[:, 0] >> 8) & 0xFF, (frag[:, 0] >> 16) & 0xFF], 1).astype(np.int64)
    p = ((xyz << 8) | sub).astype(np.float32) + np.float32(0.5)
    m = view.m.astype(np.float32)
    s = [((m[r, 0] * p[:, 0] + m[r, 1] * p[:, 1]) + m[r, 2] * p[:, 2]) + m[r, 3] for r in range(3)]
    fx, fy = np.floor(s[0]), np.floor(s[1])
    ok = (s[2] > 0) & (fx >= 0) & (fx < view.width) & (fy >= 0) & (fy < view.height)
    pix = np.where(ok, fy * view.width + fx, -1).astype(np.int64)
    return pix, s[2], frag[:, 1]


def test_product_form_in_fp64(orc, arrays):
    """Each pixel equals sum_i a_i c_i prod_{j<i} (1 - a_j) over the
    fragments it meets sorted by depth (fp64, product form), within fp32
    accumulation error; with tau = 0 every fragment counts."""
    L, o, views = arrays
    out, _ = orc.raycast(o["key"], o["frag"], views, L, mode=1, tau=0.0)
    for v, view in enumerate(views):
        pix, dep, rgba = _fragment_lists(orc, o, view, L)
        idx = np.nonzero(pix >= 0)[0]
        order = idx[np.lexsort((idx, dep[idx].view(np.uint32), pix[idx]))]
        want = np.zeros((view.height * view.width, 4))
        for p in np.unique(pix[order]):
            seq = order[pix[order] == p]
            a = ((rgba[seq] >> 24) & 0xFF) / 255.0
            trans = np.concatenate([[1.0], np.cumprod(1.0 - a)[:-1]])
            for c in range(3):
                want[p, c] = np.sum(a * trans * (((rgba[seq] >> (8 * c)) & 0xFF) / 255.0))
            want[p, 3] = 1.0 - np.prod(1.0 - a)
        got = out[v].reshape(-1, 4).astype(np.float64)
        assert np.abs(got - want).max() < 1e-5


def test_threshold_one_keeps_the_first_fragment(orc, arrays):
    """With tau = 1 the accumulation stops after the first fragment that has
    any opacity: each pixel is a_1 c_1 with opacity a_1 (a zero alpha leaves
    T = 1 and the next fragment is taken)."""
    L, o, views = arrays
    out, _ = orc.raycast(o["key"], o["frag"], views[:1], L, mode=1, tau=1.0)
    pix, dep, rgba = _fragment_lists(orc, o, views[0], L)
    idx = np.nonzero(pix >= 0)[0]
    order = idx[np.lexsort((idx, dep[idx].view(np.uint32), pix[idx]))]
    got = out[0].reshape(-1, 4)
    for p in np.unique(pix[order])[:500]:
        seq = [i for i in order[pix[order] == p] if (rgba[i] >> 24) != 0]
        if not seq:
            assert got[p, 3] == 0
            continue
        i = seq[0]
        a = np.float32((rgba[i] >> 24) & 0xFF) / np.float32(255)
        assert got[p, 3] == np.float32(1) - (np.float32(1) - a)
        assert abs(got[p, 0] - a * ((rgba[i] & 0xFF) / 255.0)) < 1e-6


def test_independent_of_array_order(orc, arrays):
    """Reordering fragments inside their octants changes only indices: with
    no two fragments of a pixel at one depth the image is unchanged."""
    L, o, views = arrays
    frag = o["frag"].copy()
    rng = np.random.default_rng(1)
    off, cnt = o["off"].astype(np.int64), o["cnt"].astype(np.int64)
    for b, n in zip(off, cnt):
        if n > 1:
            frag[b:b + n] = frag[b + rng.permutation(n)]
    a, _ = orc.raycast(o["key"], o["frag"], views, L, mode=1)
    b2, _ = orc.raycast(o["key"], frag, views, L, mode=1)
    for v, view in enumerate(views):
        pix, dep, _ = _fragment_lists(orc, o, view, L)
        sel = pix >= 0
        pairs = np.stack([pix[sel], dep[sel].view(np.uint32)], 1)
        ties = np.unique(pairs, axis=0).shape[0] < pairs.shape[0]
        if not ties:
            assert np.array_equal(a[v], b2[v])

"""The batch at its configured shape: 64 procedural scenes with triangle
counts log-uniform in [1e3, 5e5] (5.46 M triangles), octree depth 9 (a key
space of 64 * 8^9 = 2^33 keys: 64-bit keys), 8 views each at 1280 x 720, in
one fhv_batch_run call (recorded graph, as the benchmark replays it).

Every scene is checked against the invariants of per-octant arrays (table
keys ascending and grouped by scene in scene order, offsets the exclusive
sums of the counts, every record's rank its row, record totals equal to the
counter) and every view against the z-buffer's own winners (colour, depth
and coverage of the winning record, the winner from the view's scene); the
smallest, the largest and the median scene are compared with the oracle run
on that scene alone, table, records and all 8 images bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S
from tests.gpu_util import u32, u64

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

L, V, W, H = 9, 8, 1280, 720


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    fhv.set_tuning()
    yield fhv
    fhv.set_tuning()


def test_batch_of_64_scenes_at_depth_9(F, orc):
    import torch
    meshes = S.batched_scenes(0, 64)
    n_tri = [m.n_tri for m in meshes]
    views = [[S.cube_view(45.0 * v, L, W, H) for v in range(V)] for _ in meshes]
    k = views[0][0].splat_px
    b = F.to_device_batch(meshes, L)
    vm = F.batch_view_matrices(views)
    cap = 170 << 20
    lists = F.alloc_batch_lists(b, cap)
    pofa = F.alloc_pofa(cap)
    img = F.alloc_images(64 * V, W, H)
    print(f"batch64: {sum(n_tri)} triangles, graph run", flush=True)
    F.batch_run(b, vm, W, H, k, lists, pofa, img, flags=F.FHV_BATCH_GRAPH)
    torch.cuda.synchronize()
    Fn = int(lists.counter.item())
    n_occ = int(pofa.n_occ.item())
    print(f"batch64: {Fn} fragments, {n_occ} occupied octants", flush=True)
    assert Fn <= cap and int(pofa.n_frag.item()) == Fn
    key = u64(pofa.oct_key)[:n_occ]
    off = u32(pofa.oct_off)[:n_occ].astype(np.int64)
    cnt = u32(pofa.oct_cnt)[:n_occ].astype(np.int64)
    frag = u32(pofa.frag)[:Fn]
    # table: keys strictly ascending, scene = key / 8^L ascending, counts
    # positive and summing to the counter, offsets their exclusive sums
    span = np.uint64(8 ** L)
    assert np.all(np.diff(key.astype(np.float64)) > 0) and np.all(key[1:] > key[:-1])
    scene_of_row = (key // span).astype(np.int64)
    assert scene_of_row.min() >= 0 and scene_of_row.max() < 64
    assert np.all(cnt > 0) and int(cnt.sum()) == Fn
    assert off[0] == 0 and np.array_equal(off[1:], np.cumsum(cnt)[:-1])
    # every record's w3 is its row
    assert np.array_equal(frag[:, 3].astype(np.int64), np.repeat(np.arange(n_occ), cnt))
    del lists
    # images: per view, each covered pixel shows its z-buffer winner, a
    # record of the view's own scene; empty pixels are zero
    zb = u64(img.zbuf).reshape(64, V, H * W)
    rgba = u32(img.rgba).reshape(64, V, H * W)
    depth = img.depth.cpu().numpy().view(np.uint32).reshape(64, V, H * W)
    cov = img.cov.cpu().numpy().reshape(64, V, H * W)
    rec_scene = np.repeat(scene_of_row, cnt)
    covered = np.zeros(64, np.int64)
    for s in range(64):
        z = zb[s]
        empty = z == np.uint64(~np.uint64(0))
        assert np.array_equal(cov[s] == 0, empty), s
        assert np.all(rgba[s][empty] == 0) and np.all(depth[s][empty] == 0), s
        idx = (z[~empty] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        assert np.all(idx < Fn), s
        assert np.all(rec_scene[idx] == s), s
        assert np.array_equal(rgba[s][~empty], frag[idx, 1]), s
        assert np.array_equal(depth[s][~empty], (z[~empty] >> np.uint64(32)).astype(np.uint32)), s
        covered[s] = int((~empty).sum())
    # per-scene record totals, then three scenes against the oracle
    rows_of = np.bincount(scene_of_row, minlength=64)
    frags_of = np.bincount(scene_of_row, weights=cnt, minlength=64).astype(np.int64)
    first_row = np.concatenate([[0], np.cumsum(rows_of)[:-1]])
    first_frag = np.concatenate([[0], np.cumsum(frags_of)[:-1]])
    order = np.argsort(n_tri, kind="stable")
    for s in (int(order[0]), int(order[32]), int(order[-1])):
        print(f"batch64: oracle scene {s} ({n_tri[s]} triangles)", flush=True)
        oh, op, oc = orc.capture_pofl(meshes[s], L, 40 << 20)
        o = orc.compact(oh, op, oc)
        del oh, op
        assert frags_of[s] == oc and rows_of[s] == o["key"].size, s
        r0, f0 = int(first_row[s]), int(first_frag[s])
        sel = slice(r0, r0 + rows_of[s])
        assert np.array_equal(key[sel] - np.uint64(s) * span, o["key"]), s
        assert np.array_equal(cnt[sel], o["cnt"].astype(np.int64)), s
        assert np.array_equal(off[sel] - f0, o["off"].astype(np.int64)), s
        seg = frag[f0:f0 + oc]
        assert np.array_equal(seg[:, :3], o["frag"][:, :3]), s
        assert np.array_equal(seg[:, 3].astype(np.int64), o["frag"][:, 3].astype(np.int64) + r0), s
        orgba, odepth, ocov, ozb = orc.splat(1, o["key"], o["frag"], views[s], levels=L, return_zbuf=True)
        # the batch's winners carry global record indices: the scene's first
        # record f0 plus the oracle's index within the scene
        for v in range(V):
            assert np.array_equal(cov[s, v], ocov[v].reshape(-1)), (s, v)
            assert np.array_equal(rgba[s, v], orgba[v].reshape(-1)), (s, v)
            assert np.array_equal(depth[s, v], odepth[v].reshape(-1).view(np.uint32)), (s, v)
            hit = cov[s, v] > 0
            gi = (zb[s, v][hit] & np.uint64(0xFFFFFFFF)).astype(np.int64) - f0
            oi = (ozb[v].reshape(-1)[hit] & np.uint64(0xFFFFFFFF)).astype(np.int64)
            assert np.array_equal(gi, oi), (s, v)
    assert covered.min() > 0

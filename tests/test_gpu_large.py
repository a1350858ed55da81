"""Octree depth 11 (2048^3 leaves, 2^33 keys, 64-bit key sidecar).

The dense oracle cannot hold 2^33 list heads, so parity is taken per key
range: the oracle captures only the keys of two level-3 sub-cubes (2^24 keys
each) chosen from the scene geometry, and the GPU's lists, arrays and table
rows restricted to those keys must equal the oracle's bit for bit. The whole
GPU result is checked against the invariants that hold at any size (every
pool slot in exactly one list, counts summing to the fragment count, offsets
the exclusive sums of counts, keys ascending, ranks = table rows)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S
from tests.gpu_util import u32, u64
from tests.listutil import canonical, expected_arrays

pytestmark = pytest.mark.gpu

NIL = 0xFFFFFFFF


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    return fhv


def walk_from(head_slice, key_lo, pool, F):
    """Walk the lists whose heads are given (keys key_lo + i)."""
    keys, recs = [], []
    for i in np.nonzero(head_slice != NIL)[0]:
        j, steps = int(head_slice[i]), 0
        while j != NIL:
            assert j < F
            keys.append(key_lo + int(i))
            recs.append(pool[j])
            j = int(pool[j, 3])
            steps += 1
            assert steps <= F
    if not keys:
        return np.zeros(0, np.uint64), np.zeros((0, 4), np.uint32)
    return np.array(keys, np.uint64), np.stack(recs)


def subcube_ranges(orc, mesh, levels, picks):
    """Key ranges of the level-3 sub-cubes that contain the given vertices."""
    G = 2 ** (levels + 8)
    out = []
    for v in picks:
        P = np.minimum(np.floor(mesh.pos[v].astype(np.float64) * G), G - 1).astype(np.int64)
        top = P >> (levels + 8 - 3)
        sub = orc.morton3(int(top[0]), int(top[1]), int(top[2]), 3)
        span = 8 ** (levels - 3)
        out.append((sub * span, (sub + 1) * span))
    return sorted(set(out))


def test_depth11_lists_and_arrays_by_key_range(F, orc):
    import torch
    L = 11
    mesh = S.cube_scene(20000, 21, scale_range=(0.005, 0.03), ground=0)
    d = F.desc(F.FHV_POFL, levels=L)
    cap = 16 << 20
    lists = F.alloc_lists(d, cap)
    assert lists.keys.dtype == torch.int64
    F.capture(F.to_device(mesh), d, lists)
    pofa = F.alloc_pofa(cap)
    F.compact(lists, d, pofa)
    torch.cuda.synchronize()
    Fn = int(lists.counter.item())
    print(f"depth 11: {Fn} fragments", flush=True)
    assert 0 < Fn <= cap
    pool = u32(lists.pool)[:Fn]
    keys = lists.keys[:Fn].cpu().numpy().view(np.uint64)
    n_occ = int(pofa.n_occ.item())
    tk = u64(pofa.oct_key)[:n_occ]
    to = u32(pofa.oct_off)[:n_occ]
    tc = u32(pofa.oct_cnt)[:n_occ]
    fr = u32(pofa.frag)[:Fn]
    # invariants of the whole result
    assert int(tc.sum()) == Fn and np.all(np.diff(tk.astype(np.int64)) > 0) and tk[-1] < 8 ** L
    assert np.array_equal(to, np.concatenate([[0], np.cumsum(tc)[:-1]]).astype(np.uint32))
    assert np.array_equal(fr[:, 3], np.repeat(np.arange(n_occ, dtype=np.uint32), tc))
    assert np.array_equal(np.repeat(tk, tc), np.sort(keys))
    ranges = subcube_ranges(orc, mesh, L, [0, mesh.n_vert // 2, mesh.n_vert - 1])
    for lo, hi in ranges:
        oh, op, oF = orc.capture_pofl_range(mesh, L, lo, hi, 1 << 22)
        ok, orecs = walk_from(oh, lo, op, oF)
        gh = lists.head[lo:hi].cpu().numpy().view(np.uint32)
        gk, grecs = walk_from(gh, lo, pool, Fn)
        print(f"range [{lo}, {hi}): oracle {oF} fragments, GPU {gk.size}", flush=True)
        assert oF > 0 and gk.size == oF
        assert np.array_equal(canonical(gk, grecs), canonical(ok, orecs))
        # arrays restricted to the range
        ek, eo, ec, ef = expected_arrays(ok, orecs)
        sel = (tk >= lo) & (tk < hi)
        assert np.array_equal(tk[sel], ek) and np.array_equal(tc[sel], ec)
        rows = np.nonzero(sel)[0]
        seg = np.concatenate([fr[to[r]:to[r] + tc[r], :3] for r in rows])
        assert np.array_equal(seg, ef[:, :3])


def test_splat_decodes_keys_above_32_bits(F, orc):
    """Fragments whose Morton keys use bits 32 and up land where the oracle
    puts them."""
    import torch
    L = 11
    rng = np.random.default_rng(4)
    pts = rng.integers(0, 2 ** 11, (40, 3))
    pts[:, 0] |= 1 << 10                      # x bit 10 -> key bit 32
    kk = np.array(sorted({orc.morton3(int(x), int(y), int(z), L) for x, y, z in pts}), np.uint64)
    assert kk.max() >= 2 ** 32
    n = kk.size
    frag = np.zeros((n, 4), np.uint32)
    frag[:, 0] = rng.integers(0, 2 ** 24, n)
    frag[:, 1] = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    frag[:, 3] = np.arange(n)
    views = [S.cube_view(th, L, 320, 180, splat_px=2) for th in (0.0, 40.0)]
    pofa = F.Pofa(torch.from_numpy(kk.view(np.int64)).cuda(),
                  torch.from_numpy(np.arange(n, dtype=np.uint32).view(np.int32)).cuda(),
                  torch.ones(n, dtype=torch.int32, device="cuda"),
                  torch.from_numpy(frag.view(np.int32)).cuda(),
                  torch.tensor([n], dtype=torch.int64, device="cuda"),
                  torch.tensor([n], dtype=torch.int64, device="cuda"), n, n)
    img = F.splat(pofa, F.desc(F.FHV_POFL, levels=L), views)
    torch.cuda.synchronize()
    orgba, odepth, ocov = orc.splat(1, kk, frag, views, levels=L)
    assert ocov.sum() > 0
    assert np.array_equal(img.cov.cpu().numpy(), ocov)
    assert np.array_equal(u32(img.rgba), orgba)


def subcube_triangles(mesh, levels, top):
    """Triangles whose snapped bounding box meets level-3 sub-cube `top`
    (integer xyz): no other triangle can put a fragment there, since
    interpolated positions stay within the vertices' range per axis."""
    G = 2 ** (levels + 8)
    sh = levels + 8 - 3
    g = np.minimum(np.floor(mesh.pos.astype(np.float64) * G), G - 1).astype(np.int64)
    tg = g[mesh.tri]
    lo, hi = tg.min(axis=1) >> sh, tg.max(axis=1) >> sh
    sel = np.all((lo <= top) & (hi >= top), axis=1)
    return S.Mesh(mesh.pos, mesh.rgba, mesh.tri[sel], mesh.obj[sel]), g


@pytest.mark.slow
def test_large_scene_full_size(F, orc):
    """The 5M-triangle depth-11 workload at full size (about 0.9e9
    fragments): invariants over the whole result on the device, records and
    table rows of two level-3 sub-cubes bit for bit against the oracle, and
    two of the 16 4K views checked against the oracle's splat of those
    sub-cubes' fragments (a pixel they cover is covered, never farther than
    their nearest fragment, and identical where the winner is one of
    them)."""
    import torch
    L = 11
    mesh = S.large_scene(0)
    d = F.desc(F.FHV_POFL, levels=L)
    dm = F.to_device(mesh)
    head = torch.empty(8 ** L, dtype=torch.int32, device="cuda")
    mk = lambda cap: F.Lists(head, torch.empty((max(cap, 1), 4), dtype=torch.int32, device="cuda"),
                             torch.empty(max(cap, 1), dtype=torch.int64, device="cuda"),
                             torch.zeros(1, dtype=torch.int64, device="cuda"), cap)
    probe = mk(1 << 16)
    F.capture(dm, d, probe)
    torch.cuda.synchronize()
    Fn = int(probe.counter.item())
    del probe
    print(f"large scene: {mesh.n_tri} triangles, {Fn} fragments", flush=True)
    assert 5e8 < Fn < 2 ** 32 - 1
    lists = mk(Fn)
    F.capture(dm, d, lists)
    pofa = F.alloc_pofa(Fn)
    F.compact(lists, d, pofa)
    views = [S.cube_view(22.5 * v, L, 3840, 2160) for v in range(16)]
    img = F.splat(pofa, d, views)
    torch.cuda.synchronize()
    assert int(lists.counter.item()) == Fn
    n_occ = int(pofa.n_occ.item())
    tk = pofa.oct_key[:n_occ]
    tc = pofa.oct_cnt[:n_occ].to(torch.int64) & 0xFFFFFFFF
    to = pofa.oct_off[:n_occ].to(torch.int64) & 0xFFFFFFFF
    assert int(tc.sum()) == Fn and int(pofa.n_frag.item()) == Fn
    assert bool((tk[1:] > tk[:-1]).all()) and int(tk[0]) >= 0 and int(tk[-1]) < 8 ** L
    assert torch.equal(to, torch.cumsum(tc, 0) - tc)
    rank = torch.repeat_interleave(torch.arange(n_occ, device="cuda"), tc)
    assert torch.equal(pofa.frag[:Fn, 3].to(torch.int64) & 0xFFFFFFFF, rank)
    del rank
    keys = lists.keys[:Fn]
    assert int(keys.sum()) == int((tk * tc).sum())
    assert int((keys * keys).sum()) == int((tk * tk * tc).sum())     # both wrap mod 2^64
    print("invariants hold", flush=True)

    span = 8 ** (L - 3)
    zb = img.zbuf.cpu().numpy().view(np.uint64)
    n_mine = 0
    for v in (0, mesh.n_vert // 2):
        g0 = np.minimum(np.floor(mesh.pos[v].astype(np.float64) * 2 ** (L + 8)), 2 ** (L + 8) - 1).astype(np.int64)
        top = g0 >> (L + 8 - 3)
        sub, _ = subcube_triangles(mesh, L, top)
        lo = orc.morton3(int(top[0]), int(top[1]), int(top[2]), 3) * span
        oh, op, oF = orc.capture_pofl_range(sub, L, lo, lo + span, 1 << 24)
        assert 0 < oF <= 1 << 24
        o = orc.compact(oh, op, oF)
        rows = torch.nonzero((tk >= lo) & (tk < lo + span)).flatten()
        r0 = int(rows[0])
        assert rows.numel() == o["key"].size and int(rows[-1]) == r0 + rows.numel() - 1
        assert np.array_equal(u64(tk[rows]) - np.uint64(lo), o["key"])
        assert np.array_equal(tc[rows].cpu().numpy().astype(np.uint32), o["cnt"])
        f0 = int(to[r0])
        seg = u32(pofa.frag[f0:f0 + oF])
        assert np.array_equal(seg[:, :3], o["frag"][:, :3])
        assert np.array_equal(seg[:, 3], o["frag"][:, 3] + np.uint32(r0))
        print(f"sub-cube {top.tolist()}: {oF} fragments from {sub.tri.shape[0]} triangles match", flush=True)
        for vi in (0, 5):
            orgba, odepth, ocov = orc.splat(1, o["key"] + np.uint64(lo), o["frag"], [views[vi]], levels=L)
            cov = ocov[0] > 0
            gz = zb[vi]
            assert np.all(img.cov[vi].cpu().numpy()[cov] == 1)
            gd = (gz >> np.uint64(32)).astype(np.uint32).view(np.float32)
            assert np.all(gd[cov] <= odepth[0][cov])
            gid = (gz & np.uint64(0xFFFFFFFF)).astype(np.int64)
            mine = cov & (gid >= f0) & (gid < f0 + oF)
            n_mine += int(mine.sum())
            assert np.array_equal(gd[mine].view(np.uint32), odepth[0][mine].view(np.uint32))
            assert np.array_equal(u32(img.rgba[vi])[mine], orgba[0][mine])
    assert n_mine > 0      # some checked pixel is won by a sub-cube fragment

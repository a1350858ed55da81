"""Per-octant arrays straight from the triangles (fhv_capture_arrays: count
pass, scan, insert pass; no lists) against the oracle's compaction of its
lists, bit for bit, for every capture variant, at depths 6, 9 and 11 (a key
range at 11), with the overflow report and argument errors."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S
from tests.gpu_util import u32, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    return fhv


def arrays(F, mesh, d, cap):
    import torch
    out = F.alloc_pofa(cap)
    F.capture_arrays(F.to_device(mesh), d, out)
    torch.cuda.synchronize()
    n_occ, n_frag = int(out.n_occ.item()), int(out.n_frag.item())
    n = min(n_occ, out.cap_occ)
    return {"key": u64(out.oct_key)[:n], "off": u32(out.oct_off)[:n], "cnt": u32(out.oct_cnt)[:n],
            "frag": u32(out.frag)[:n_frag], "n_occ": n_occ, "n_frag": n_frag}, out


@pytest.mark.parametrize("proj", [0, 1, 2, 3])
@pytest.mark.parametrize("L", [6, 9])
def test_arrays_match_oracle(F, orc, proj, L):
    mesh = S.cube_scene(3000, 51 + L, scale_range=(0.05, 0.3), ground=8)
    cap = 1 << 22
    d = F.desc(F.FHV_POFL, levels=L, projection=proj)
    g, _ = arrays(F, mesh, d, cap)
    oh, op, oc = orc.capture_pofl(mesh, L, cap, projection=proj)
    o = orc.compact(oh, op, oc)
    print(f"L={L} projection={proj}: {g['n_frag']} fragments, {g['n_occ']} octants", flush=True)
    assert g["n_frag"] == oc and g["n_occ"] == o["n_occ"]
    for f in ("key", "off", "cnt", "frag"):
        assert np.array_equal(g[f], o[f]), f


def test_arrays_depth11_key_range(F, orc):
    L = 11
    mesh = S.cube_scene(800, 60, scale_range=(0.02, 0.08), ground=0)
    d = F.desc(F.FHV_POFL, levels=L)
    g, _ = arrays(F, mesh, d, 1 << 23)
    span = 8 ** 8
    top = int(g["key"][g["key"].size // 2]) // span          # a level-3 sub-cube that has fragments
    lo = top * span
    oh, op, oc = orc.capture_pofl_range(mesh, L, lo, lo + span, 1 << 22)
    o = orc.compact(oh, op, oc)
    rows = np.nonzero((g["key"] >= lo) & (g["key"] < lo + span))[0]
    print(f"depth 11: {g['n_frag']} fragments; sub-cube {top}: {oc}", flush=True)
    assert rows.size == o["key"].size and oc > 0
    assert np.array_equal(g["key"][rows] - np.uint64(lo), o["key"])
    assert np.array_equal(g["cnt"][rows], o["cnt"])
    f0 = int(g["off"][rows[0]])
    seg = g["frag"][f0:f0 + oc]
    assert np.array_equal(seg[:, :3], o["frag"][:, :3])
    assert np.array_equal(seg[:, 3], o["frag"][:, 3] + np.uint32(rows[0]))


def test_arrays_too_small_report_the_count(F, orc):
    import torch
    L = 6
    mesh = S.cube_scene(2000, 61, scale_range=(0.05, 0.3), ground=8)
    _, _, oc = orc.capture_pofl(mesh, L, 1 << 22)
    d = F.desc(F.FHV_POFL, levels=L)
    out = F.alloc_pofa(oc // 2)
    out.frag.fill_(0x5A5A5A5A)
    out.oct_key.fill_(7)
    F.capture_arrays(F.to_device(mesh), d, out)
    torch.cuda.synchronize()
    assert int(out.n_frag.item()) == oc and int(out.n_occ.item()) == 0
    assert bool((out.frag == 0x5A5A5A5A).all()) and bool((out.oct_key == 7).all())
    # and with room, the same call fills them
    g, _ = arrays(F, mesh, d, oc)
    assert g["n_frag"] == oc


def test_arrays_of_an_empty_mesh(F):
    L = 5
    mesh = S.Mesh(np.zeros((3, 3), np.float32), np.zeros(3, np.uint32), np.zeros((0, 3), np.uint32),
                  np.zeros(0, np.uint8))
    g, _ = arrays(F, mesh, F.desc(F.FHV_POFL, levels=L), 1024)
    assert g["n_frag"] == 0 and g["n_occ"] == 0


def test_arrays_reject_bad_arguments(F):
    Lb = F.lib()
    assert Lb.fhv_capture_arrays_workspace(C.byref(F.desc(F.FHV_PPFL, 64, 64)), 10, 100) == 0
    assert Lb.fhv_capture_arrays_workspace(C.byref(F.desc(F.FHV_POFL, levels=6)), 10, 0) == 0
    assert Lb.fhv_capture_arrays(None, None, None, None, None, 0, None) == -1

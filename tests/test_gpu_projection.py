"""The capture variants of Table 2 (Sec. 3.2) on the GPU against the oracle:
per-octant lists (as canonical multisets per key) and the compacted arrays
bit for bit, for 1-Pass/Normal, 1-Pass/View, 3-Pass/1-Way and 1-Pass/3-Way,
plus the overflow rule across the three passes of 3-Pass/1-Way."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S
from tests.gpu_util import run_capture, run_compact
from tests.listutil import canonical, walk_lists

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    return fhv


@pytest.mark.parametrize("proj", [0, 1, 2, 3])
@pytest.mark.parametrize("L", [6, 9])
def test_projection_matches_oracle(F, orc, proj, L):
    mesh = S.cube_scene(3000, 31 + L, scale_range=(0.05, 0.3), ground=8)
    cap = 1 << 22
    d = F.desc(F.FHV_POFL, levels=L, projection=proj)
    head, pool, keys, cnt, lists = run_capture(F, mesh, d, cap)
    oh, op, oc = orc.capture_pofl(mesh, L, cap, projection=proj)
    print(f"L={L} projection={proj}: {cnt} fragments", flush=True)
    assert cnt == oc
    k, recs = walk_lists(head, pool, cnt)
    ok, orecs = walk_lists(oh, op, oc)
    assert np.array_equal(canonical(k, recs), canonical(ok, orecs))
    g, _ = run_compact(F, lists, d)
    o = orc.compact(oh, op, oc)
    for f in ("key", "off", "cnt", "frag"):
        assert np.array_equal(g[f], o[f]), f


def test_three_passes_keep_the_overflow_rule(F, orc):
    L = 6
    mesh = S.cube_scene(3000, 40, scale_range=(0.05, 0.3), ground=8)
    d = F.desc(F.FHV_POFL, levels=L, projection=F.FHV_PROJ_AXES_3PASS)
    _, _, full = orc.capture_pofl(mesh, L, 1 << 22, projection=2)
    cap = full // 2            # overflows during the second pass or later
    head, pool, keys, cnt, lists = run_capture(F, mesh, d, cap)
    assert cnt == full
    k, recs = walk_lists(head, pool, cap)     # every slot below the capacity on exactly one list
    assert k.size == cap


def test_projection_rejected_for_pixel_lists(F):
    import ctypes as C
    Lb = F.lib()
    d = F.desc(F.FHV_PPFL, 64, 64, projection=1)
    assert Lb.fhv_capture_workspace(C.byref(d), 10) == 0
    d = F.desc(F.FHV_POFL, levels=6, projection=4)
    assert Lb.fhv_capture_workspace(C.byref(d), 10) == 0

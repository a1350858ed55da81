"""Pins of the capture variants of Table 2 (Sec. 3.2, Figs. 7 and 8) in the
oracle: which plane a triangle is rasterized in.

* A square in an axis plane has the same lattice points whether it is
  rasterized in its own plane (1-Pass/Normal) or in the matching axis plane
  (the two other axis planes see it edge-on; 1-Pass/View, the x-y plane,
  captures it only when it faces z). Facing z, the frames coincide and the
  fragments are identical; facing x, the tangent frame is mirrored with
  respect to the axis plane's, so the fill rule keeps other boundary edges:
  the counts agree and the fragments strictly inside the square agree.
* On a sphere the projected area in a plane is the area times |n . axis|,
  so the fragment counts follow the mean of |n_z| (1/2) and of
  |n_x| + |n_y| + |n_z| (3/2) relative to 1-Pass/Normal.
* 3-Pass/1-Way and 1-Pass/3-Way capture the same fragments."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S
from tests.listutil import canonical, walk_lists
from tests.test_oracle_pins import _plane_grid, mesh_from


def _x_plane(n, c, lo, hi):
    """The +z square rotated into the plane x = c (normal +x)."""
    tris = _plane_grid(n, c, lo, hi, 5, "+z")
    return [(p[2], p[0], p[1]) for p in tris]     # (x, y, z) <- (z, x, y): +z -> +x


def _canon(orc, mesh, L, proj, cap=1 << 21):
    head, pool, cnt = orc.capture_pofl(mesh, L, cap, projection=proj)
    k, recs = walk_lists(head, pool, cnt)
    return cnt, canonical(k, recs)


def _positions(orc, mesh, L, proj):
    """Grid position -> (colour, normal) of every captured fragment."""
    head, pool, cnt = orc.capture_pofl(mesh, L, 1 << 21, projection=proj)
    k, recs = walk_lists(head, pool, cnt)
    out = {}
    for key, r in zip(k, recs):
        key = int(key)
        xyz = [0, 0, 0]
        for b in range(L):
            for a in range(3):
                xyz[a] |= ((key >> (3 * b + 2 - a)) & 1) << b
        p = tuple((xyz[a] << 8) | ((int(r[0]) >> (8 * a)) & 0xFF) for a in range(3))
        assert p not in out
        out[p] = (int(r[1]), int(r[2]))
    return cnt, out


@pytest.mark.parametrize("facing", ["z", "x"])
def test_axis_plane_square_in_every_variant(orc, facing):
    L = 5
    G = 2 ** (L + 8)
    lo, hi, c = 0.1171875, 0.8359375, 0.40625
    tris = _plane_grid(6, c, lo, hi, L, "+z") if facing == "z" else _x_plane(6, c, lo, hi)
    # one colour: a sample on an edge shared inside the square then looks the
    # same whichever of the two triangles the fill rule gives it to
    mesh = mesh_from(tris, colors=np.full(len(tris), 0xFF336699, np.uint32))
    n_norm, c_norm = _canon(orc, mesh, L, 0)
    assert n_norm > 1000
    n_view, c_view = _canon(orc, mesh, L, 1)
    if facing == "z":
        assert n_view == n_norm and np.array_equal(c_view, c_norm)
        for proj in (2, 3):
            n, cc = _canon(orc, mesh, L, proj)
            assert n == n_norm and np.array_equal(cc, c_norm), proj
        return
    assert n_view == 0
    _, p_norm = _positions(orc, mesh, L, 0)
    inside = lambda p: all(lo * G < p[a] < hi * G for a in (1, 2))
    for proj in (2, 3):
        n, p_ax = _positions(orc, mesh, L, proj)
        assert n == n_norm
        a = {p: v for p, v in p_norm.items() if inside(p)}
        b = {p: v for p, v in p_ax.items() if inside(p)}
        assert len(a) > 0.9 * n and a == b


def test_sphere_counts_follow_projected_area(orc):
    L = 7
    p0, f0 = S.icosphere(5)
    pos = (0.5 + 0.35 * p0).astype(np.float32)
    rgba = np.full(pos.shape[0], 0xFF808080, np.uint32)
    mesh = S.Mesh(pos, rgba, f0.astype(np.uint32), np.zeros(f0.shape[0], np.uint8))
    counts = {}
    for proj in range(4):
        _, _, counts[proj] = orc.capture_pofl(mesh, L, 1 << 23, projection=proj)
    print(counts)
    normal = counts[0]
    assert abs(counts[1] / normal - 0.5) < 0.02
    assert abs(counts[2] / normal - 1.5) < 0.03
    assert counts[2] == counts[3]


def test_three_axis_capture_contains_the_view_capture(orc):
    """The three-axis variants rasterize every triangle in the y-z, z-x and
    x-y planes; their fragments include, as a multiset, every fragment of the
    x-y plane alone (1-Pass/View), and the rest come from the other two
    planes (a triangle parallel to z is edge-on in x-y)."""
    mesh = S.cube_scene(1500, 21, scale_range=(0.05, 0.3), ground=4)
    n1, c1 = _canon(orc, mesh, 6, 1)
    n2, c2 = _canon(orc, mesh, 6, 2)
    assert n2 > n1 > 0
    a = {}
    for row in map(tuple, c2.tolist()):
        a[row] = a.get(row, 0) + 1
    for row in map(tuple, c1.tolist()):
        assert a.get(row, 0) > 0, row
        a[row] -= 1

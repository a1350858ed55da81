"""Pins of the oracle's record contents and of its reference image, against
facts computed here without the oracle's code:

* every captured record's normal word (Sec. 3.1 record content: the
  fragment's normal) equals an independent floating-point octahedral
  encoding (Cigolle et al. 2014) of its own triangle's face normal, the
  cross product of the snapped vertices in the authored order;
* every per-octant fragment lies on its triangle: on the triangle's plane
  and inside its edges within the rounding of the integer interpolation, and
  on the tangent-plane sample lattice of 2^7 grid units (Sec. 3.2, Fig. 8);
* the direct rasterization that judges a novel view (the reference image)
  equals a brute force over every (pixel, triangle) pair with exact rational
  projection, coverage (the sample moved by (eps, -eps^2)) and
  interpolation, the nearest (depth, triangle) winning per pixel.

Each triangle of these scenes carries its own object byte, so the record's
aux byte names the triangle that produced it."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2211_15460_amd import scenes as S
from tests.listutil import walk_lists

SQRT3 = math.sqrt(3.0)


def _soup(tris, cols=None):
    pos = np.asarray(tris, np.float32).reshape(-1, 3)
    nt = pos.shape[0] // 3
    assert nt <= 256
    if cols is None:
        cols = (np.arange(pos.shape[0], dtype=np.uint64) * 0x9E3779B1 & 0xFFFFFFFF).astype(np.uint32)
    tri = np.arange(pos.shape[0], dtype=np.uint32).reshape(nt, 3)
    return S.Mesh(pos, np.asarray(cols, np.uint32), tri, np.arange(nt, dtype=np.uint8))


def _float_oct(n):
    """Octahedral encoding of a normal in floating point: n / |n|_1, folded
    into the upper square when n_z < 0 (sign of 0 taken as +), components
    times 32767 rounded to nearest. Returns (qx, qy, tie) where tie flags a
    product within 1e-6 of a half-integer (either rounding is then
    acceptable)."""
    n = np.asarray(n, np.float64)
    l1 = np.abs(n).sum()
    if l1 == 0:
        return 0, 0, False
    p = n / l1
    if n[2] < 0:
        sx = 1.0 if p[0] >= 0 else -1.0
        sy = 1.0 if p[1] >= 0 else -1.0
        p = np.array([(1 - abs(p[1])) * sx, (1 - abs(p[0])) * sy])
    v = p[:2] * 32767.0
    q = np.sign(v) * np.floor(np.abs(v) + 0.5)
    tie = bool(np.any(np.abs(np.abs(v) - np.floor(np.abs(v)) - 0.5) < 1e-6))
    return int(q[0]), int(q[1]), tie


def _unpack(w2):
    return int(np.uint16(w2 & 0xFFFF).view(np.int16)), int(np.uint16(w2 >> 16).view(np.int16))


def _check_normals(recs, normals):
    """Every record's w2 against the float encoding of its triangle's normal
    (exact, or within one unit at a rounding tie)."""
    assert recs.shape[0] > 0
    for t in np.unique(recs[:, 0] >> 24):
        ws = np.unique(recs[(recs[:, 0] >> 24) == t, 2])
        assert ws.size == 1, f"triangle {t}: several normal words {ws}"
        qx, qy = _unpack(int(ws[0]))
        ex, ey, tie = _float_oct(normals[int(t)])
        tol = 1 if tie else 0
        assert abs(qx - ex) <= tol and abs(qy - ey) <= tol, (int(t), (qx, qy), (ex, ey))


def _random_tris(rng, n, lo=0.1, hi=0.9):
    return (lo + (hi - lo) * rng.random((n, 3, 3))).reshape(-1, 3).tolist()


def _grid_pos(mesh, L):
    G = float(2 ** (L + 8))
    return np.clip(np.floor(mesh.pos.astype(np.float64) * G), 0, G - 1).astype(np.int64)


def _decode_keys(keys, L):
    keys = np.asarray(keys, np.uint64).astype(np.int64)
    x = np.zeros_like(keys)
    y = np.zeros_like(keys)
    z = np.zeros_like(keys)
    for b in range(L):
        x |= ((keys >> (3 * b + 2)) & 1) << b
        y |= ((keys >> (3 * b + 1)) & 1) << b
        z |= ((keys >> (3 * b)) & 1) << b
    return x, y, z


# ------------------------------------------------------------ normal word

@pytest.mark.parametrize("seed", range(4))
def test_pofl_record_normal_is_its_triangles_face_normal(orc, seed):
    rng = np.random.default_rng(100 + seed)
    L = 5
    m = _soup(_random_tris(rng, 60))
    head, pool, cnt = orc.capture_pofl(m, L, 1 << 20)
    _, recs = walk_lists(head, pool, cnt)
    P = _grid_pos(m, L).reshape(-1, 3, 3)
    normals = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    _check_normals(recs, normals)


@pytest.mark.parametrize("seed", range(3))
def test_ppfl_record_normal_is_its_triangles_face_normal(orc, seed):
    """Per-pixel capture: the face normal of the vertices snapped to the
    2^-20 lattice of clip space (the capture's reading of a flat normal)."""
    rng = np.random.default_rng(200 + seed)
    m = _soup((rng.random((40, 3, 3)) * 1.6 - 0.8).reshape(-1, 3).tolist())
    head, pool, cnt = orc.capture_ppfl(m, 64, 64, 1 << 18)
    _, recs = walk_lists(head, pool, cnt)
    q = np.rint(m.pos.astype(np.float64) * 2.0 ** 20).astype(np.int64).reshape(-1, 3, 3)
    normals = np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0])
    _check_normals(recs, normals)


def test_axis_square_normal_codes(orc):
    """Squares in axis planes pack to exact codes: +z is (0, 0), +y is
    (0, 32767), -y is (0, -32767), +x is (32767, 0), and -z folds to
    (32767, 32767)."""
    L = 5
    lo, hi, c = 0.25, 0.75, 0.5
    sq = {
        "+z": [(lo, lo, c), (hi, lo, c), (hi, hi, c), (lo, lo, c), (hi, hi, c), (lo, hi, c)],
        "+y": [(lo, c, lo), (lo, c, hi), (hi, c, hi), (lo, c, lo), (hi, c, hi), (hi, c, lo)],
        "+x": [(c, lo, lo), (c, hi, lo), (c, hi, hi), (c, lo, lo), (c, hi, hi), (c, lo, hi)],
    }
    sq["-y"] = [sq["+y"][i] for i in (0, 2, 1, 3, 5, 4)]
    sq["-z"] = [sq["+z"][i] for i in (0, 2, 1, 3, 5, 4)]
    want = {"+z": (0, 0), "+y": (0, 32767), "-y": (0, -32767), "+x": (32767, 0), "-z": (32767, 32767)}
    for name, tris in sq.items():
        head, pool, cnt = orc.capture_pofl(_soup(tris), L, 1 << 16)
        assert cnt > 0, name
        _, recs = walk_lists(head, pool, cnt)
        got = {_unpack(int(w)) for w in np.unique(recs[:, 2])}
        assert got == {want[name]}, (name, got)


# ------------------------------------------------------------ positions

@pytest.mark.parametrize("seed", range(3))
def test_pofl_fragments_lie_on_their_triangle(orc, seed):
    """A fragment's grid position is the interpolation Q = sum_k lambda_k P_k
    at a lattice sample (lambda >= 0, Q in the triangle) rounded per axis, so
    |P - Q|_inf <= 1/2:
      * distance to the triangle's plane <= |n|_1 / 2 (n the unit normal);
      * barycentric coordinates of P's projection >= -(sqrt(3)/2) / h_k with
        h_k the altitude from vertex k;
      * in the tangent frame of the packed normal, 2 P.t and 2 P.b (16.8
        sample units) lie within 1/2 + |t|_1 (resp. |b|_1) of a lattice point
        256 i + 128 (the snapped vertices move the lattice by at most 1/2)."""
    rng = np.random.default_rng(300 + seed)
    L = 5
    m = _soup(_random_tris(rng, 40, 0.15, 0.85))
    head, pool, cnt = orc.capture_pofl(m, L, 1 << 20)
    keys, recs = walk_lists(head, pool, cnt)
    kx, ky, kz = _decode_keys(keys, L)
    pos = np.stack([(kx << 8) | (recs[:, 0] & 0xFF), (ky << 8) | ((recs[:, 0] >> 8) & 0xFF),
                    (kz << 8) | ((recs[:, 0] >> 16) & 0xFF)], 1).astype(np.float64)
    tid = (recs[:, 0] >> 24).astype(np.int64)
    P = _grid_pos(m, L).reshape(-1, 3, 3).astype(np.float64)
    per_tri = np.bincount(tid, minlength=P.shape[0])
    for t in range(P.shape[0]):
        sel = tid == t
        if not sel.any():
            continue
        p0, p1, p2 = P[t]
        n = np.cross(p1 - p0, p2 - p0)
        area2 = np.linalg.norm(n)
        nu = n / area2
        d = pos[sel] - p0
        assert np.all(np.abs(d @ nu) <= 0.5 * np.abs(nu).sum() + 1e-9), t
        # barycentric coordinates of the projection onto the plane
        e1, e2 = p1 - p0, p2 - p0
        g = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
        ab = np.linalg.solve(g, np.stack([d @ e1, d @ e2]))
        lam = np.stack([1 - ab[0] - ab[1], ab[0], ab[1]])
        edges = [p2 - p1, p0 - p2, p1 - p0]
        for k in range(3):
            h = area2 / np.linalg.norm(edges[k])
            assert np.all(lam[k] >= -0.5 * SQRT3 / h - 1e-9), (t, k, lam[k].min())
        # on the sample lattice of the packed normal's tangent frame
        w2 = int(recs[sel][0, 2])
        tt, bb = orc.tangent_frame(w2)
        for axis, bound in ((tt, 0.5 + np.abs(tt).sum()), (bb, 0.5 + np.abs(bb).sum())):
            s = 2.0 * pos[sel] @ axis
            r = np.mod(s - 128.0, 256.0)
            r = np.minimum(r, 256.0 - r)
            assert np.all(r <= bound + 1e-6), (t, r.max(), bound)
        # distinct samples of one triangle give distinct positions
        assert len({tuple(v) for v in pos[sel].astype(np.int64).tolist()}) == int(sel.sum())
    assert per_tri.sum() == cnt


# ------------------------------------------------------------ direct raster

def _rint(q: Fraction) -> int:
    """Round half to even, exactly."""
    f = math.floor(q)
    r = q - f
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and f % 2 == 1):
        return f + 1
    return f


def brute_direct(mesh, m, W, H, L):
    """Reference image of per-octant scene coordinates: vertices scaled to
    grid units (2^(L+8) per side), the view's fp32 3x4 matrix applied with
    exact rationals, screen x, y snapped to 16.8, depth row mapped to depth24
    = rint((d - 1)(2^24 - 1)) clamped; per pixel every covering triangle
    (sample moved by (eps, -eps^2) strictly inside), depth and colour
    interpolated exactly and rounded half up; the smallest (depth24,
    triangle) wins. Returns (rgba, depth24 or -1) as [H, W] arrays."""
    G = 2 ** (L + 8)
    M = [[Fraction(float(v)) for v in row] for row in np.asarray(m, np.float32).reshape(3, 4)]
    best = {}
    for t in range(mesh.n_tri):
        X, Y, Z, C = [], [], [], []
        for k in range(3):
            p = [Fraction(float(c)) * G for c in mesh.pos[mesh.tri[t, k]]]
            s = [M[r][0] * p[0] + M[r][1] * p[1] + M[r][2] * p[2] + M[r][3] for r in range(3)]
            X.append(Fraction(_rint(s[0] * 256)))
            Y.append(Fraction(_rint(s[1] * 256)))
            Z.append(min(max(_rint((s[2] - 1) * (2 ** 24 - 1)), 0), 2 ** 24 - 1))
            C.append(int(mesh.rgba[mesh.tri[t, k]]))
        det = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0])
        if det == 0:
            continue
        for py in range(H):
            for px in range(W):
                sx, sy = Fraction(256 * px + 128), Fraction(256 * py + 128)
                lam = []
                for k in range(3):
                    i, j = (k + 1) % 3, (k + 2) % 3
                    c0 = ((X[i] - sx) * (Y[j] - sy) - (X[j] - sx) * (Y[i] - sy)) / det
                    c1 = (Y[i] - Y[j]) / det
                    c2 = (X[i] - X[j]) / det
                    if next((c for c in (c0, c1, c2) if c != 0), 0) <= 0:
                        break
                    lam.append(c0)
                if len(lam) < 3:
                    continue
                z = math.floor(sum(lam[k] * Z[k] for k in range(3)) + Fraction(1, 2))
                rgba = 0
                for ch in range(4):
                    v = sum(lam[k] * ((C[k] >> (8 * ch)) & 0xFF) for k in range(3))
                    rgba |= math.floor(v + Fraction(1, 2)) << (8 * ch)
                cur = best.get((px, py))
                if cur is None or (z, t) < cur[:2]:
                    best[(px, py)] = (z, t, rgba)
    rgba = np.zeros((H, W), np.uint32)
    d24 = np.full((H, W), -1, np.int64)
    for (px, py), (z, _, c) in best.items():
        rgba[py, px] = c
        d24[py, px] = z
    return rgba, d24


def _dyadic_view(L, W, H, a, b):
    """An affine view of grid units with dyadic entries (every fp64 step of
    the oracle exact): screen x mixes x and z (a shear standing in for the
    orbit's rotation), screen y is y, the depth row mixes z and x into
    [1, 2)."""
    G = 2.0 ** (L + 8)
    s = W / G
    m = np.array([[s * a, 0.0, s * b, 0.5],
                  [0.0, H / G, 0.0, 0.25],
                  [-0.25 / G, 0.0, 0.5 / G, 1.25]], np.float32)
    return S.View(m, W, H, 1)


def _compare_direct(orc, mesh, view, L):
    rgba, depth, cov = orc.direct_raster(1, mesh, view, levels=L)
    brgba, bd = brute_direct(mesh, view.m, view.width, view.height, L)
    assert np.array_equal(cov == 1, bd >= 0)
    assert np.array_equal(rgba, brgba)
    want = np.where(bd >= 0, (1.0 + bd / (2 ** 24 - 1)).astype(np.float32), np.float32(0))
    assert np.array_equal(depth, want)
    return cov


def test_direct_raster_two_squares_nearer_wins(orc):
    """Two overlapping squares at different depths, seen through a sheared
    view: the pixels of each square are known in closed form, and where they
    overlap the nearer square's colour wins."""
    L = 3
    G = 2 ** (L + 8)
    W = H = 16
    # square A at z = 0.25 (nearer: depth grows with z), B at z = 0.75;
    # x, y spans chosen on pixel boundaries of this view
    def square(x0, x1, y0, y1, z):
        a, b, c, d = (x0, y0, z), (x1, y0, z), (x1, y1, z), (x0, y1, z)
        return [a, b, c, a, c, d]
    ta = square(0.125, 0.625, 0.125, 0.625, 0.25)
    tb = square(0.375, 0.875, 0.375, 0.875, 0.75)
    red, blue = 0xFF0000FF, 0xFFFF0000
    mesh = _soup(ta + tb, [red] * 6 + [blue] * 6)
    view = _dyadic_view(L, W, H, 1.0, 0.0)
    cov = _compare_direct(orc, mesh, view, L)
    rgba, _, _ = orc.direct_raster(1, mesh, view, levels=L)
    # pixel px covers screen x in [px, px+1); the sample px + 1/2 lies in
    # [16 x0, 16 x1) horizontally and (16 y0 + 1/4, 16 y1 + 1/4] vertically
    def pix(x0, x1, y0, y1):
        xs = [p for p in range(W) if 16 * x0 <= p + 0.5 < 16 * x1]
        ys = [p for p in range(H) if 16 * y0 + 0.25 < p + 0.5 <= 16 * y1 + 0.25]
        return {(x, y) for x in xs for y in ys}
    pa, pb = pix(0.125, 0.625, 0.125, 0.625), pix(0.375, 0.875, 0.375, 0.875)
    assert pa & pb
    for y in range(H):
        for x in range(W):
            want = red if (x, y) in pa else (blue if (x, y) in pb else 0)
            assert rgba[y, x] == want, (x, y)
    assert int(cov.sum()) == len(pa | pb)
    # the far square drawn first changes nothing (depth decides, not order)
    mesh2 = _soup(tb + ta, [blue] * 6 + [red] * 6)
    rgba2, _, _ = orc.direct_raster(1, mesh2, view, levels=L)
    assert np.array_equal(rgba2, rgba)


@pytest.mark.parametrize("seed", range(4))
def test_direct_raster_brute_force(orc, seed):
    """Random tiny scenes on a dyadic grid under sheared views."""
    rng = np.random.default_rng(400 + seed)
    L = 3
    W, H = (12, 10) if seed % 2 else (10, 12)
    tris = (rng.integers(8, 120, (7, 3, 3)) / 128.0).reshape(-1, 3).tolist()
    cols = rng.integers(0, 2 ** 32, 21, dtype=np.uint64).astype(np.uint32)
    mesh = _soup(tris, cols)
    a, b = [(1.0, 0.0), (0.75, 0.5), (0.5, -0.75), (0.875, 0.25)][seed]
    cov = _compare_direct(orc, mesh, _dyadic_view(L, W, H, a, b), L)
    assert cov.sum() > 0

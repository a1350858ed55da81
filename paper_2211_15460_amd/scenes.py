"""Seeded synthetic inputs for the fragment-history-volume path.

This module only makes inputs: triangle soups, per-vertex colours, object ids
and orthographic orbit cameras. It holds none of the method's arithmetic
(no rasterization, no list building, no compaction, no splatting), so both the
GPU path and the CPU oracle can be fed from it without sharing method code.

The paper's benchmark scenes (a 1,532-triangle "simple" scene and a
23.5M-triangle "complex" scene, Sec. 4 / Fig. 10) are not available; the
procedural scenes here stand in for them by reproducing their two regimes:
few large triangles with many fragments each, and many small triangles.

Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014),
evaluated counter-style: draw n of stream s is mix(s + (n+1)*GAMMA).
Uniform floats take the top 24 bits, so every value is exact in fp32.
Random rotations follow Shoemake, "Uniform random rotations" (Graphics Gems
III, 1992).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
ONE_MINUS_ULP = np.float32(1.0 - 2.0 ** -24)


class SplitMix64:
    """Counter-based SplitMix64 stream; ``next(n)`` returns n uint64 draws."""

    def __init__(self, seed: int):
        self.state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.n = 0

    def next(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            k = np.arange(self.n + 1, self.n + 1 + n, dtype=np.uint64)
            z = self.state + k * GAMMA
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        self.n += n
        return z

    def unit(self, n: int) -> np.ndarray:
        """n floats uniform on [0, 1) with 24 random bits (exact in fp32)."""
        return ((self.next(n) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24)

    def u32(self, n: int) -> np.ndarray:
        return (self.next(n) >> np.uint64(32)).astype(np.uint32)


@dataclass
class Mesh:
    """Indexed triangle soup in host memory.

    pos  float32 [nv, 3]   PPFL: clip-space xyz; POFL: scene cube [0,1)^3
    rgba uint32  [nv]      R in the low byte
    tri  uint32  [nt, 3]   vertex indices, authored winding
    obj  uint8   [nt]      low 8 bits of the object id
    """
    pos: np.ndarray
    rgba: np.ndarray
    tri: np.ndarray
    obj: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_vert(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])


# ---------------------------------------------------------------- PPFL soup

def clip_soup(n_tri: int, seed: int) -> Mesh:
    """n_tri independent triangles, vertices uniform in [-1,1]^3 clip space,
    per-vertex random RGBA8, random object byte per triangle."""
    rng = SplitMix64(seed)
    nv = 3 * n_tri
    pos = (2.0 * rng.unit(3 * nv) - 1.0).astype(np.float32).reshape(nv, 3)
    rgba = rng.u32(nv)
    tri = np.arange(nv, dtype=np.uint32).reshape(n_tri, 3)
    obj = (rng.next(n_tri) >> np.uint64(56)).astype(np.uint8)
    return Mesh(pos, rgba, tri, obj, {"kind": "clip_soup", "seed": seed})


# ------------------------------------------------------------ primitives

_ICO_CACHE: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere after `level` 4:1 subdivisions: 20*4^level triangles,
    outward counter-clockwise winding."""
    if level in _ICO_CACHE:
        return _ICO_CACHE[level]
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / math.sqrt(1 + t * t) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid: dict[tuple[int, int], int] = {}

        def midpoint(a: int, b: int) -> int:
            k = (a, b) if a < b else (b, a)
            if k not in mid:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                mid[k] = len(verts) - 1
            return mid[k]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    out = (np.array(verts), np.array(faces, dtype=np.int64))
    _ICO_CACHE[level] = out
    return out


def box(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Cube [-1,1]^3 with each face split into n x n quads (12 n^2 triangles),
    outward counter-clockwise winding; faces do not share vertices."""
    g = np.linspace(-1.0, 1.0, n + 1)
    uu, vv = np.meshgrid(g, g, indexing="ij")
    uu, vv = uu.ravel(), vv.ravel()
    one = np.ones_like(uu)
    # (u-axis, v-axis, normal) per face with u x v = normal
    frames = [((0, 1, 0), (0, 0, 1), (1, 0, 0)), ((0, 0, 1), (0, 1, 0), (-1, 0, 0)),
              ((0, 0, 1), (1, 0, 0), (0, 1, 0)), ((1, 0, 0), (0, 0, 1), (0, -1, 0)),
              ((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((0, 1, 0), (1, 0, 0), (0, 0, -1))]
    verts, faces = [], []
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    quads = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    for f, (eu, ev, en) in enumerate(frames):
        p = (np.outer(uu, eu) + np.outer(vv, ev) + np.outer(one, en))
        verts.append(p)
        faces.append(quads + f * (n + 1) * (n + 1))
    return np.concatenate(verts), np.concatenate(faces)


def shoemake_rotation(u: np.ndarray) -> np.ndarray:
    """Rotation matrix from three uniforms (Shoemake 1992)."""
    u1, u2, u3 = u
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def ground_grid(n: int, height: float) -> tuple[np.ndarray, np.ndarray]:
    """n x n quads (2 n^2 triangles) covering the cube's x,z extent at y=height,
    winding with normal +y."""
    g = np.linspace(0.0, 1.0, n + 1)
    xx, zz = np.meshgrid(g, g, indexing="ij")
    p = np.stack([xx.ravel(), np.full(xx.size, height), zz.ravel()], 1)
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    a, b = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel()
    c, d = idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    # (x, z) grid: normal +y needs order a, d, c (z then x)
    f = np.concatenate([np.stack([a, d, c], 1), np.stack([a, c, b], 1)])
    return p, f


def cube_scene(n_tri: int, seed: int, scale_range=(0.02, 0.2), n_objects: int | None = None,
               ground: int = 32) -> Mesh:
    """Procedural scene in the unit cube [0,1)^3 with exactly n_tri triangles.

    A ground grid (ground x ground quads at y = 0.05) plus objects:
    subdivided icospheres and boxes under a uniform random rotation, a
    log-uniform scale in scale_range and a uniform position; vertices are
    clamped into [0, 1-2^-24]. Object mesh sizes are drawn so that the count
    comes out near n_tri (n_objects, when given, fixes the number of
    objects instead); the last object is truncated to hit n_tri exactly.
    Colours: per-object base colour with per-vertex jitter, alpha 255.
    """
    rng = SplitMix64(seed)
    pos_parts, tri_parts, rgba_parts, obj_parts = [], [], [], []
    nv = 0
    nt = 0
    oid = 0

    def add(p: np.ndarray, f: np.ndarray, base: np.ndarray):
        nonlocal nv, nt, oid
        take = min(f.shape[0], n_tri - nt)
        if take <= 0:
            return
        f = f[:take]
        p = np.clip(p, 0.0, float(ONE_MINUS_ULP)).astype(np.float32)
        jit = (rng.unit(3 * p.shape[0]).reshape(-1, 3) * 64.0 - 32.0)
        col = np.clip(base[None, :] + jit, 0, 255).astype(np.uint32)
        rgba = col[:, 0] | (col[:, 1] << 8) | (col[:, 2] << 16) | np.uint32(255 << 24)
        pos_parts.append(p)
        rgba_parts.append(rgba.astype(np.uint32))
        tri_parts.append((f + nv).astype(np.uint32))
        obj_parts.append(np.full(take, oid & 0xFF, dtype=np.uint8))
        nv += p.shape[0]
        nt += take
        oid += 1

    if ground > 0:
        gp, gf = ground_grid(ground, 0.05)
        add(gp, gf, np.array([96.0, 140.0, 80.0]))
    lo, hi = math.log(scale_range[0]), math.log(scale_range[1])
    if n_objects:
        per_obj = max(1, (n_tri - nt) // n_objects)
    while nt < n_tri:
        r = rng.unit(8)
        if n_objects:
            # pick the primitive whose size is closest to the per-object budget
            if r[0] < 0.5:
                lvl = int(np.clip(round(math.log(max(per_obj, 20) / 20.0, 4)), 0, 6))
                p0, f0 = icosphere(lvl)
            else:
                n = max(1, int(round(math.sqrt(per_obj / 12.0))))
                p0, f0 = box(n)
        elif r[0] < 0.5:
            p0, f0 = icosphere(3 if r[1] < 0.6 else 4)
        else:
            p0, f0 = box(4 + int(r[1] * 13))
        s = math.exp(lo + (hi - lo) * r[2])
        R = shoemake_rotation(r[3:6])
        c = rng.unit(3)
        p = c[None, :] + 0.5 * s * (p0 @ R.T)
        base = 40.0 + 175.0 * rng.unit(3)
        add(p, f0, base)
    return Mesh(np.concatenate(pos_parts), np.concatenate(rgba_parts),
                np.concatenate(tri_parts), np.concatenate(obj_parts),
                {"kind": "cube_scene", "seed": seed, "objects": oid})


# ------------------------------------------------------------ cameras

@dataclass
class View:
    """Orthographic orbit camera as a row-major fp32 3x4 matrix.

    Row 0 maps a fragment position to the screen x in pixels, row 1 to the
    screen y in pixels (y up, row 0 of the image is the bottom), row 2 to a
    depth value in [1, 2) that grows away from the viewer.
    splat_px is the side of the square footprint each fragment covers.
    """
    m: np.ndarray
    width: int
    height: int
    splat_px: int


def _orbit(theta_deg: float) -> np.ndarray:
    t = math.radians(theta_deg)
    c, s = math.cos(t), math.sin(t)
    # rotation about +y; theta = 0 looks along +z with x right and y up
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def ppfl_view(theta_deg: float, width: int, height: int, out_w: int | None = None,
              out_h: int | None = None, splat_px: int = 1) -> View:
    """Orbit view for a per-pixel capture of width x height.

    PPFL fragment positions are given in capture units
    (px + 0.5, py + 0.5, depth24); the matrix maps them to clip space
    [-1,1]^3, rotates about +y by theta and maps to the output window and to
    a depth in [1, 2). theta = 0 reproduces the capture window.
    """
    out_w = out_w or width
    out_h = out_h or height
    s_in = np.array([[2.0 / width, 0, 0, -1.0], [0, 2.0 / height, 0, -1.0],
                     [0, 0, 2.0 / (2 ** 24 - 1), -1.0], [0, 0, 0, 1.0]])
    rot = np.eye(4)
    rot[:3, :3] = _orbit(theta_deg)
    rad = math.sqrt(3.0)
    s_out = np.array([[out_w / 2.0, 0, 0, out_w / 2.0], [0, out_h / 2.0, 0, out_h / 2.0],
                      [0, 0, 0.49 / rad, 1.5], [0, 0, 0, 1.0]])
    m = (s_out @ rot @ s_in)[:3, :]
    return View(m.astype(np.float32), out_w, out_h, splat_px)


def cube_view(theta_deg: float, levels: int, width: int, height: int,
              vertical_extent: float = 1.25, splat_px: int | None = None) -> View:
    """Orbit view for a per-octant capture of the unit cube at octree depth
    `levels`. Fragment positions are in grid units (2^(levels+8) per cube
    side). The vertical extent covers vertical_extent cube sides; the
    orbit is about the vertical axis through the cube centre."""
    g = float(2 ** (levels + 8))
    ppu = height / (vertical_extent * g)          # pixels per grid unit
    cen = np.eye(4)
    cen[:3, 3] = -0.5 * g
    rot = np.eye(4)
    rot[:3, :3] = _orbit(theta_deg)
    rad = math.sqrt(3.0) * 0.5 * g
    s_out = np.array([[ppu, 0, 0, width / 2.0], [0, ppu, 0, height / 2.0],
                      [0, 0, 0.49 / rad, 1.5], [0, 0, 0, 1.0]])
    m = (s_out @ rot @ cen)[:3, :]
    if splat_px is None:
        spacing_px = 128.0 * ppu          # sample spacing is 2^7 grid units
        splat_px = max(1, math.ceil(spacing_px - 1e-9))
    return View(m.astype(np.float32), width, height, splat_px)


# ------------------------------------------------------------ named workloads

def stereo_views(theta_deg: float, levels: int, width: int, height: int, eye_deg: float = 4.0,
                 splat_px: int | None = None) -> list[View]:
    """Left and right eye of a stereo pair (Sec. 5: several novel views from
    one FHV): two orbit views eye_deg apart around theta_deg (toe-in)."""
    return [cube_view(theta_deg - 0.5 * eye_deg, levels, width, height, splat_px=splat_px),
            cube_view(theta_deg + 0.5 * eye_deg, levels, width, height, splat_px=splat_px)]


def ppfl_plain(seed: int = 0) -> Mesh:
    """64 triangles, vertices uniform in [-1,1]^3 clip space (128x128 capture)."""
    return clip_soup(64, seed)


def pofl_scene(seed: int = 0, n_tri: int = 200_000) -> Mesh:
    """~600-object procedural scene, exactly n_tri triangles (octree depth 9)."""
    return cube_scene(n_tri, seed)


def large_scene(seed: int = 0) -> Mesh:
    """5M triangles in 20,000 objects (octree depth 11): object scales
    log-uniform in [0.012, 0.046] give about 0.9e9 fragments."""
    return cube_scene(5_000_000, seed, scale_range=(0.012, 0.046), n_objects=20_000)


def batched_scenes(seed: int = 0, n_scenes: int = 64) -> list[Mesh]:
    """n_scenes procedural scenes with triangle counts log-uniform in [1e3, 5e5]."""
    rng = SplitMix64(seed ^ 0x5CE7E5)
    u = rng.unit(n_scenes)
    counts = np.round(np.exp(math.log(1e3) + u * (math.log(5e5) - math.log(1e3)))).astype(int)
    return [cube_scene(int(n), seed * 1000 + i) for i, n in enumerate(counts)]

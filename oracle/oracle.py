"""ctypes front end of the C oracle (fhv_oracle.c).

TEST INFRASTRUCTURE ONLY. Array marshalling around the plain C reference;
every function here states which part of the paper the C routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fhv_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
NIL = 0xFFFFFFFF

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        L = _lib
        L.orc_oct_encode.argtypes = [C.c_int64] * 3
        L.orc_oct_encode.restype = C.c_uint32
        L.orc_oct_decode.argtypes = [C.c_uint32, f64p]
        L.orc_tangent_frame.argtypes = [C.c_uint32, f64p, f64p]
        L.orc_morton3.argtypes = [C.c_uint32] * 4
        L.orc_morton3.restype = C.c_uint64
        L.orc_capture_ppfl.argtypes = [f32p, u32p, u32p, C.c_void_p, C.c_uint32, C.c_uint32,
                                       C.c_uint32, u32p, u32p, C.c_uint64]
        L.orc_capture_ppfl.restype = C.c_uint64
        L.orc_capture_pofl.argtypes = [f32p, u32p, u32p, C.c_void_p, C.c_uint32, C.c_uint32,
                                       u32p, u32p, C.c_uint64]
        L.orc_capture_pofl.restype = C.c_uint64
        L.orc_capture_pofl_range.argtypes = [f32p, u32p, u32p, C.c_void_p, C.c_uint32, C.c_uint32,
                                             C.c_uint64, C.c_uint64, u32p, u32p, C.c_uint64]
        L.orc_capture_pofl_range.restype = C.c_uint64
        L.orc_compact.argtypes = [u32p, C.c_uint64, u32p, C.c_uint64, C.c_uint64, u64p, u32p,
                                  u32p, C.c_uint64, u32p]
        L.orc_compact.restype = C.c_uint64
        L.orc_splat.argtypes = [C.c_int, C.c_uint32, C.c_uint32, u64p, C.c_uint64, u32p, C.c_uint64, f32p,
                                u32p, C.c_uint32, u64p, u32p, f32p, u8p]
        L.orc_direct_raster.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, f32p, u32p,
                                        u32p, C.c_uint32, f32p, C.c_uint32, C.c_uint32, u64p, u32p,
                                        f32p, u8p]
        L.orc_psnr_rgb.argtypes = [u32p, u32p, C.c_uint64]
        L.orc_capture_pofl_proj.argtypes = [f32p, u32p, u32p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32,
                                            C.c_uint64, C.c_uint64, u32p, u32p, C.c_uint64]
        L.orc_capture_pofl_proj.restype = C.c_uint64
        L.orc_shade.argtypes = [u32p, u64p, C.c_uint64, C.c_uint32, f32p, f32p]
        L.orc_raycast.argtypes = [C.c_uint32, u64p, u32p, C.c_uint64, f32p, C.c_uint32, C.c_uint32, C.c_int,
                                  C.c_float, f32p]
        L.orc_raycast.restype = C.c_uint64
        L.orc_psnr_rgb.restype = C.c_double
    return _lib


def _obj_ptr(obj):
    return None if obj is None else obj.ctypes.data_as(C.c_void_p)


def _mesh_arrays(mesh):
    pos = np.ascontiguousarray(mesh.pos, dtype=np.float32).reshape(-1)
    rgba = np.ascontiguousarray(mesh.rgba, dtype=np.uint32)
    tri = np.ascontiguousarray(mesh.tri, dtype=np.uint32).reshape(-1)
    obj = None if mesh.obj is None else np.ascontiguousarray(mesh.obj, dtype=np.uint8)
    return pos, rgba, tri, obj


# ----------------------------------------------------------- small pieces

def oct_encode(nx: int, ny: int, nz: int) -> int:
    """Exact octahedral packing of an integer normal (x low 16, y high 16)."""
    return int(lib().orc_oct_encode(nx, ny, nz))


def oct_decode(nrm: int) -> np.ndarray:
    out = np.zeros(3, np.float64)
    lib().orc_oct_decode(nrm, out)
    return out


def tangent_frame(nrm: int) -> tuple[np.ndarray, np.ndarray]:
    """(t, b) of the Duff et al. basis for the decoded packed normal."""
    t = np.zeros(3, np.float64)
    b = np.zeros(3, np.float64)
    lib().orc_tangent_frame(nrm, t, b)
    return t, b


def morton3(x: int, y: int, z: int, levels: int) -> int:
    return int(lib().orc_morton3(x, y, z, levels))


# ----------------------------------------------------------- capture

def capture_ppfl(mesh, width: int, height: int, cap: int):
    """Per-pixel fragment lists (Sec. 3.1 simple layout, Sec. 3.2 FHV_PPFL).

    Returns (head uint32[H*W], pool uint32[cap, 4], counter)."""
    pos, rgba, tri, obj = _mesh_arrays(mesh)
    head = np.full(width * height, NIL, np.uint32)
    pool = np.zeros(4 * max(cap, 1), np.uint32)
    cnt = lib().orc_capture_ppfl(pos, rgba, tri, _obj_ptr(obj), mesh.tri.shape[0], width, height,
                                 head, pool, cap)
    return head, pool.reshape(-1, 4)[:cap], int(cnt)


def capture_pofl(mesh, levels: int, cap: int, projection: int = 0):
    """Per-octant fragment lists with tangent-space rasterization
    (Sec. 3.1 octree layout, Sec. 3.2 FHV_POFL, Fig. 8), or with the
    rasterization plane of another capture variant (Table 2): 1 the x-y plane
    ("1-Pass/View"), 2 or 3 all three axis planes ("3-Pass/1-Way",
    "1-Pass/3-Way").

    Returns (head uint32[8^L], pool uint32[cap, 4], counter)."""
    pos, rgba, tri, obj = _mesh_arrays(mesh)
    head = np.full(8 ** levels, NIL, np.uint32)
    pool = np.zeros(4 * max(cap, 1), np.uint32)
    cnt = lib().orc_capture_pofl_proj(pos, rgba, tri, _obj_ptr(obj), mesh.tri.shape[0], levels, projection,
                                      0, 8 ** levels, head, pool, cap)
    return head, pool.reshape(-1, 4)[:cap], int(cnt)


def capture_pofl_range(mesh, levels: int, key_lo: int, key_hi: int, cap: int):
    """Per-octant lists of only the keys in [key_lo, key_hi) (head index key
    - key_lo); the counter counts those fragments only."""
    pos, rgba, tri, obj = _mesh_arrays(mesh)
    head = np.full(key_hi - key_lo, NIL, np.uint32)
    pool = np.zeros(4 * max(cap, 1), np.uint32)
    cnt = lib().orc_capture_pofl_range(pos, rgba, tri, _obj_ptr(obj), mesh.tri.shape[0], levels,
                                       key_lo, key_hi, head, pool, cap)
    return head, pool.reshape(-1, 4)[:cap], int(cnt)


# ----------------------------------------------------------- compaction

def compact(head: np.ndarray, pool: np.ndarray, counter: int, cap_occ: int | None = None):
    """Per-octant arrays (Sec. 3.1/3.2 FHV_POFA) from lists.

    Returns dict(key uint64[n_occ], off uint32, cnt uint32, frag uint32[F,4],
    n_occ)."""
    cap = pool.shape[0]
    F = min(counter, cap)
    if cap_occ is None:
        cap_occ = max(F, 1)
    keys = np.zeros(max(cap_occ, 1), np.uint64)
    off = np.zeros(max(cap_occ, 1), np.uint32)
    cnt = np.zeros(max(cap_occ, 1), np.uint32)
    frag = np.zeros(4 * max(F, 1), np.uint32)
    poolc = np.ascontiguousarray(pool, dtype=np.uint32).reshape(-1)
    if poolc.size == 0:
        poolc = np.zeros(4, np.uint32)
    n_occ = lib().orc_compact(np.ascontiguousarray(head), head.size, poolc, counter, cap,
                              keys, off, cnt, cap_occ, frag)
    if n_occ == 2 ** 64 - 1:
        raise ValueError("malformed fragment lists")
    n = min(int(n_occ), cap_occ)
    return {"key": keys[:n], "off": off[:n], "cnt": cnt[:n],
            "frag": frag.reshape(-1, 4)[:F], "n_occ": int(n_occ)}


# ----------------------------------------------------------- splat / raster

def _views_arrays(views):
    m = np.ascontiguousarray(np.stack([v.m.astype(np.float32).reshape(12) for v in views]))
    whk = np.array([[v.width, v.height, v.splat_px] for v in views], np.uint32).reshape(-1)
    return m.reshape(-1), whk


def splat(mode: int, keys: np.ndarray, frag: np.ndarray, views, width_cap: int = 0,
          levels: int = 0, return_zbuf: bool = False):
    """Point splat with nearest-fragment resolve (Sec. 3.3). Fragments whose
    octant rank has no row in `keys` (a truncated table) are not drawn.

    Returns (rgba uint32[V,H,W], depth float32[V,H,W], cov uint8[V,H,W]),
    and the z-buffer of winners (uint64 [V,H,W]) when return_zbuf; all
    views must share one size."""
    W, H = views[0].width, views[0].height
    assert all(v.width == W and v.height == H for v in views)
    m, whk = _views_arrays(views)
    V = len(views)
    z = np.zeros(V * H * W, np.uint64)
    rgba = np.zeros(V * H * W, np.uint32)
    depth = np.zeros(V * H * W, np.float32)
    cov = np.zeros(V * H * W, np.uint8)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    n_keys = keys.size
    if keys.size == 0:
        keys = np.zeros(1, np.uint64)
    fr = np.ascontiguousarray(frag, dtype=np.uint32).reshape(-1)
    if fr.size == 0:
        fr = np.zeros(4, np.uint32)
    lib().orc_splat(mode, width_cap, levels, keys, n_keys, fr, frag.shape[0], m, whk, V, z, rgba, depth, cov)
    if return_zbuf:
        return rgba.reshape(V, H, W), depth.reshape(V, H, W), cov.reshape(V, H, W), z.reshape(V, H, W)
    return rgba.reshape(V, H, W), depth.reshape(V, H, W), cov.reshape(V, H, W)


def raycast(keys: np.ndarray, frag: np.ndarray, views, levels: int, mode: int = 1, tau: float = 0.0):
    """Ray casting of per-octant arrays (Sec. 3.3): per pixel, the fragments
    its ray meets, nearest first, composited front to back with their alpha
    (mode 1, "R/T") or the nearest alone (mode 0, "R"), stopping once the
    transmittance falls below tau. Returns (float32 [V,H,W,4] premultiplied
    RGB and coverage, largest number of fragments met by one pixel)."""
    W, H = views[0].width, views[0].height
    assert all(v.width == W and v.height == H for v in views)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    if keys.size == 0:
        keys = np.zeros(1, np.uint64)
    fr = np.ascontiguousarray(frag, dtype=np.uint32).reshape(-1)
    n = fr.size // 4
    if fr.size == 0:
        fr = np.zeros(4, np.uint32)
    out = np.zeros((len(views), H, W, 4), np.float32)
    deepest = 0
    for v, view in enumerate(views):
        o = np.zeros((H, W, 4), np.float32)
        d = lib().orc_raycast(levels, keys, fr, n, np.ascontiguousarray(view.m.astype(np.float32).reshape(12)),
                              W, H, mode, float(tau), o)
        out[v] = o
        deepest = max(deepest, int(d))
    return out, deepest


def shade(frag: np.ndarray, zbuf: np.ndarray, lights: np.ndarray) -> np.ndarray:
    """Blinn-Phong shading of a splat's winners (Sec. 5). zbuf: uint64
    [V, H, W] splat keys; lights: float32 [V, 13] = L, V, H (unit vectors),
    ka, kd, ks, shine (exponent 2^shine). Returns float32 [V, H, W, 4]."""
    zb = np.ascontiguousarray(zbuf, dtype=np.uint64)
    V = zb.shape[0]
    npix = zb.size // V
    fr = np.ascontiguousarray(frag, dtype=np.uint32).reshape(-1)
    if fr.size == 0:
        fr = np.zeros(4, np.uint32)
    out = np.zeros(zb.shape + (4,), np.float32)
    lib().orc_shade(fr, zb.reshape(-1), npix, V, np.ascontiguousarray(lights, np.float32).reshape(-1),
                    out.reshape(-1))
    return out


def direct_raster(mode: int, mesh, view, width_cap: int = 0, height_cap: int = 0, levels: int = 0):
    """Depth-tested rasterization of the triangles into one view: the
    reference image for a novel-view reconstruction. Returns (rgba, depth,
    cov) with shape [H, W]."""
    pos, rgba, tri, _ = _mesh_arrays(mesh)
    W, H = view.width, view.height
    z = np.zeros(W * H, np.uint64)
    col = np.zeros(W * H, np.uint32)
    depth = np.zeros(W * H, np.float32)
    cov = np.zeros(W * H, np.uint8)
    lib().orc_direct_raster(mode, width_cap, height_cap, levels, pos, rgba, tri, mesh.tri.shape[0],
                            np.ascontiguousarray(view.m.astype(np.float32).reshape(12)), W, H, z, col,
                            depth, cov)
    return col.reshape(H, W), depth.reshape(H, W), cov.reshape(H, W)


def psnr_rgb(a: np.ndarray, b: np.ndarray) -> float:
    """PSNR over the R, G, B bytes of two RGBA8 images (MAX = 255)."""
    a = np.ascontiguousarray(a, dtype=np.uint32).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.uint32).reshape(-1)
    assert a.size == b.size
    return float(lib().orc_psnr_rgb(a, b, a.size))


__all__ = ["NIL", "build", "lib", "oct_encode", "oct_decode", "tangent_frame", "morton3",
           "capture_ppfl", "capture_pofl", "capture_pofl_range", "compact", "splat", "raycast", "shade", "direct_raster",
           "psnr_rgb"]

"""Python binding of libfhv (include/fhv.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; this module only
allocates device tensors with torch, fills the C structs and passes torch's
current HIP stream. It raises if the native library is missing: there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch  # loads the HIP runtime the library binds to

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfhv.so")

FHV_PPFL, FHV_POFL = 0, 1
NIL = 0xFFFFFFFF


class FhvError(RuntimeError):
    pass


class Mesh_(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("rgba", C.c_void_p), ("tri", C.c_void_p),
                ("obj", C.c_void_p), ("n_vert", C.c_uint32), ("n_tri", C.c_uint32)]


class Desc_(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("width", C.c_uint32), ("height", C.c_uint32),
                ("levels", C.c_uint32), ("projection", C.c_uint32)]


class Light_(C.Structure):
    _fields_ = [("l", C.c_float * 3), ("v", C.c_float * 3), ("h", C.c_float * 3), ("ka", C.c_float),
                ("kd", C.c_float), ("ks", C.c_float), ("shine", C.c_uint32)]


class Lists_(C.Structure):
    _fields_ = [("head", C.c_void_p), ("n_head", C.c_uint64), ("pool", C.c_void_p),
                ("capacity", C.c_uint64), ("keys", C.c_void_p), ("counter", C.c_void_p)]


class Pofa_(C.Structure):
    _fields_ = [("oct_key", C.c_void_p), ("oct_off", C.c_void_p), ("oct_cnt", C.c_void_p),
                ("cap_occ", C.c_uint64), ("frag", C.c_void_p), ("cap_frag", C.c_uint64),
                ("n_occ", C.c_void_p), ("n_frag", C.c_void_p)]


class View_(C.Structure):
    _fields_ = [("m", C.c_float * 12), ("width", C.c_uint32), ("height", C.c_uint32),
                ("splat_px", C.c_uint32)]


class BatchMesh_(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("rgba", C.c_void_p), ("tri", C.c_void_p),
                ("obj", C.c_void_p), ("scene_tri", C.c_void_p), ("n_vert", C.c_uint32),
                ("n_tri", C.c_uint32), ("n_scenes", C.c_uint32), ("levels", C.c_uint32)]


class BatchViews_(C.Structure):
    _fields_ = [("m", C.c_void_p), ("n_views", C.c_uint32), ("width", C.c_uint32),
                ("height", C.c_uint32), ("splat_px", C.c_uint32)]


class FillTensor_(C.Structure):
    _fields_ = [("offset", C.c_uint64), ("stride", C.c_uint32), ("channels", C.c_uint32), ("n", C.c_uint32),
                ("height", C.c_uint32), ("width", C.c_uint32)]


class Tuning_(C.Structure):
    _fields_ = [("tile_w", C.c_uint32), ("raster_wg", C.c_uint32), ("splat_wg", C.c_uint32)]


FHV_BATCH_GRAPH, FHV_BATCH_TUNE = 1, 2


class KernelStat_(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_uint64), ("total_ms", C.c_double)]


EXPORTS = ["fhv_create", "fhv_destroy", "fhv_status_str", "fhv_capture_workspace", "fhv_capture",
           "fhv_compact_workspace", "fhv_compact", "fhv_splat_workspace", "fhv_splat", "fhv_profile_begin",
           "fhv_profile_end", "fhv_unet_param_count", "fhv_fill_workspace", "fhv_fill",
           "fhv_fill_train_step", "fhv_get_tuning", "fhv_set_tuning", "fhv_batch_workspace",
           "fhv_batch_run", "fhv_probe", "fhv_raycast_workspace", "fhv_raycast", "fhv_capture_arrays_workspace",
           "fhv_capture_arrays", "fhv_shade", "fhv_splat_static", "fhv_fill_trace_tensors",
           "fhv_fill_train_step_traced"]

_lib = None
_ctx: dict[int, C.c_void_p] = {}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FhvError(f"native library {LIB_PATH} is not built "
                           "(run python -m paper_2211_15460_amd.build)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.fhv_create.argtypes = [C.POINTER(P), C.c_int]
        L.fhv_destroy.argtypes = [P]
        L.fhv_status_str.argtypes = [C.c_int32]
        L.fhv_status_str.restype = C.c_char_p
        L.fhv_capture_workspace.argtypes = [C.POINTER(Desc_), C.c_uint32]
        L.fhv_capture_workspace.restype = C.c_size_t
        L.fhv_capture.argtypes = [P, C.POINTER(Mesh_), C.POINTER(Desc_), C.POINTER(Lists_), P,
                                  C.c_size_t, P]
        L.fhv_compact_workspace.argtypes = [C.POINTER(Desc_), C.c_uint64]
        L.fhv_compact_workspace.restype = C.c_size_t
        L.fhv_compact.argtypes = [P, C.POINTER(Lists_), C.POINTER(Desc_), C.POINTER(Pofa_), P,
                                  C.c_size_t, P]
        L.fhv_splat_workspace.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.fhv_splat_workspace.restype = C.c_size_t
        L.fhv_splat.argtypes = [P, C.POINTER(Pofa_), C.POINTER(Desc_), C.POINTER(View_), C.c_uint32,
                                P, P, P, P, P, C.c_size_t, P]
        L.fhv_splat_static.argtypes = [P, C.POINTER(Pofa_), C.POINTER(Desc_), C.POINTER(View_), C.c_uint32,
                                       P, P, P, P, P]
        L.fhv_unet_param_count.argtypes = [C.c_uint32]
        L.fhv_unet_param_count.restype = C.c_uint64
        L.fhv_fill_workspace.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int]
        L.fhv_fill_workspace.restype = C.c_size_t
        L.fhv_fill.argtypes = [P, C.c_uint32, P, P, P, P, C.c_uint32, C.c_uint32, C.c_uint32, P, P, P,
                               C.c_size_t, P]
        L.fhv_fill_train_step.argtypes = [P, C.c_uint32, P, P, P, C.c_uint32, C.c_float, P, P, P, P,
                                          C.c_uint32, C.c_uint32, C.c_uint32, P, P, P, C.c_size_t, P]
        L.fhv_fill_train_step_traced.argtypes = L.fhv_fill_train_step.argtypes
        L.fhv_fill_trace_tensors.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                             C.POINTER(FillTensor_), C.c_uint32]
        L.fhv_fill_trace_tensors.restype = C.c_uint32
        L.fhv_get_tuning.argtypes = [P, C.POINTER(Tuning_)]
        L.fhv_set_tuning.argtypes = [P, C.POINTER(Tuning_)]
        L.fhv_batch_workspace.argtypes = [C.POINTER(BatchMesh_), C.POINTER(BatchViews_), C.c_uint64]
        L.fhv_batch_workspace.restype = C.c_size_t
        L.fhv_batch_run.argtypes = [P, C.POINTER(BatchMesh_), C.POINTER(BatchViews_), C.POINTER(Lists_),
                                    C.POINTER(Pofa_), P, P, P, P, P, C.c_size_t, C.c_uint32, P]
        L.fhv_probe.argtypes = [P, C.c_uint32, P, C.c_uint64, C.c_uint32, C.c_uint32, P]
        L.fhv_capture_arrays_workspace.argtypes = [C.POINTER(Desc_), C.c_uint32, C.c_uint64]
        L.fhv_capture_arrays_workspace.restype = C.c_size_t
        L.fhv_capture_arrays.argtypes = [P, C.POINTER(Mesh_), C.POINTER(Desc_), C.POINTER(Pofa_), P, C.c_size_t, P]
        L.fhv_shade.argtypes = [P, C.POINTER(Pofa_), P, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(Light_),
                                P, P]
        L.fhv_raycast_workspace.argtypes = [C.POINTER(Desc_)]
        L.fhv_raycast_workspace.restype = C.c_size_t
        L.fhv_raycast.argtypes = [P, C.POINTER(Pofa_), C.POINTER(Desc_), C.POINTER(View_), C.c_uint32, C.c_uint32,
                                  C.c_float, P, P, C.c_size_t, P]
        L.fhv_profile_begin.argtypes = [P]
        L.fhv_profile_end.argtypes = [P, C.POINTER(KernelStat_), C.c_uint32, C.POINTER(C.c_uint32)]
        for f in ("fhv_create", "fhv_destroy", "fhv_capture", "fhv_compact", "fhv_splat",
                  "fhv_profile_begin", "fhv_profile_end", "fhv_fill", "fhv_fill_train_step",
                  "fhv_get_tuning", "fhv_set_tuning", "fhv_batch_run", "fhv_probe", "fhv_raycast", "fhv_capture_arrays",
                  "fhv_shade", "fhv_splat_static", "fhv_fill_train_step_traced"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _check(st: int, what: str):
    if st != 0:
        raise FhvError(f"{what}: {lib().fhv_status_str(st).decode()} (status {st})")


def ctx(device: int | None = None) -> C.c_void_p:
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _ctx:
        h = C.c_void_p()
        _check(lib().fhv_create(C.byref(h), dev), "fhv_create")
        _ctx[dev] = h
    return _ctx[dev]


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ inputs

@dataclass
class DeviceMesh:
    pos: torch.Tensor      # float32 [nv, 3]
    rgba: torch.Tensor     # int32 view of uint32 [nv]
    tri: torch.Tensor      # int32 view of uint32 [nt, 3]
    obj: torch.Tensor | None   # uint8 [nt]

    @property
    def n_vert(self):
        return int(self.pos.shape[0])

    @property
    def n_tri(self):
        return int(self.tri.shape[0])


def to_device(mesh, device="cuda") -> DeviceMesh:
    """Copy a host mesh (scenes.Mesh) into device tensors."""
    pos = torch.from_numpy(np.ascontiguousarray(mesh.pos, np.float32)).to(device)
    rgba = torch.from_numpy(np.ascontiguousarray(mesh.rgba, np.uint32).view(np.int32)).to(device)
    tri = torch.from_numpy(np.ascontiguousarray(mesh.tri, np.uint32).view(np.int32)).to(device)
    obj = None if mesh.obj is None else torch.from_numpy(np.ascontiguousarray(mesh.obj, np.uint8)).to(device)
    return DeviceMesh(pos, rgba, tri, obj)


FHV_PROJ_NORMAL, FHV_PROJ_VIEW, FHV_PROJ_AXES_3PASS, FHV_PROJ_AXES_1PASS = 0, 1, 2, 3


def desc(mode: int, width: int = 0, height: int = 0, levels: int = 0, projection: int = 0) -> Desc_:
    return Desc_(mode, width, height, levels, projection)


def n_head(d: Desc_) -> int:
    return d.width * d.height if d.mode == FHV_PPFL else 8 ** d.levels


# ------------------------------------------------------------------ capture

@dataclass
class Lists:
    head: torch.Tensor | None   # int32 [n_head] (uint32 bits); None: no lists (batches)
    pool: torch.Tensor      # int32 [cap, 4]
    keys: torch.Tensor      # int32 [cap], or int64 [cap] when n_head > 2^32
    counter: torch.Tensor   # int64 [1]
    capacity: int
    key_space: int = 0      # n_head when head is None

    def struct(self) -> Lists_:
        nh = self.head.numel() if self.head is not None else self.key_space
        return Lists_(_ptr(self.head), nh,
                      self.pool.data_ptr() if self.capacity else None, self.capacity,
                      self.keys.data_ptr(), self.counter.data_ptr())


def alloc_lists(d: Desc_, capacity: int, device="cuda", n_head_override: int | None = None) -> Lists:
    nh = n_head(d) if n_head_override is None else n_head_override
    kt = torch.int64 if nh > 2 ** 32 else torch.int32
    return Lists(torch.empty(nh, dtype=torch.int32, device=device),
                 torch.empty((max(capacity, 1), 4), dtype=torch.int32, device=device),
                 torch.empty(max(capacity, 1), dtype=kt, device=device),
                 torch.zeros(1, dtype=torch.int64, device=device), capacity)


def capture_workspace(d: Desc_, n_tri: int) -> int:
    return int(lib().fhv_capture_workspace(C.byref(d), n_tri))


def capture(m: DeviceMesh, d: Desc_, lists: Lists, ws: torch.Tensor | None = None) -> Lists:
    """fhv_capture into pre-allocated lists; returns them (counter on device)."""
    need = capture_workspace(d, m.n_tri)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=m.pos.device)
    mesh = Mesh_(m.pos.data_ptr(), m.rgba.data_ptr(), m.tri.data_ptr(),
                 None if m.obj is None else m.obj.data_ptr(), m.n_vert, m.n_tri)
    ls = lists.struct()
    _check(lib().fhv_capture(ctx(), C.byref(mesh), C.byref(d), C.byref(ls), _ptr(ws), ws.numel(),
                             _stream()), "fhv_capture")
    return lists


# ------------------------------------------------------------------ compact

@dataclass
class Pofa:
    oct_key: torch.Tensor   # int64 [cap_occ]
    oct_off: torch.Tensor   # int32 [cap_occ]
    oct_cnt: torch.Tensor   # int32 [cap_occ]
    frag: torch.Tensor      # int32 [cap_frag, 4]
    n_occ: torch.Tensor     # int64 [1]
    n_frag: torch.Tensor    # int64 [1]
    cap_occ: int
    cap_frag: int

    def struct(self) -> Pofa_:
        return Pofa_(self.oct_key.data_ptr(), self.oct_off.data_ptr(), self.oct_cnt.data_ptr(),
                     self.cap_occ, self.frag.data_ptr(), self.cap_frag, self.n_occ.data_ptr(),
                     self.n_frag.data_ptr())


def alloc_pofa(cap_frag: int, cap_occ: int | None = None, device="cuda") -> Pofa:
    cap_occ = cap_frag if cap_occ is None else cap_occ
    return Pofa(torch.empty(max(cap_occ, 1), dtype=torch.int64, device=device),
                torch.empty(max(cap_occ, 1), dtype=torch.int32, device=device),
                torch.empty(max(cap_occ, 1), dtype=torch.int32, device=device),
                torch.empty((max(cap_frag, 1), 4), dtype=torch.int32, device=device),
                torch.zeros(1, dtype=torch.int64, device=device),
                torch.zeros(1, dtype=torch.int64, device=device), cap_occ, cap_frag)


def capture_arrays_workspace(d: Desc_, n_tri: int, capacity: int) -> int:
    return int(lib().fhv_capture_arrays_workspace(C.byref(d), n_tri, capacity))


def capture_arrays(m: DeviceMesh, d: Desc_, out: Pofa, ws: torch.Tensor | None = None) -> Pofa:
    """fhv_capture_arrays: per-octant arrays straight from the triangles
    (two rasterization passes, no lists); returns `out`."""
    need = capture_arrays_workspace(d, m.n_tri, out.cap_frag)
    if need == 0:
        raise FhvError("fhv_capture_arrays_workspace: unsupported arguments")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=m.pos.device)
    mesh = Mesh_(m.pos.data_ptr(), m.rgba.data_ptr(), m.tri.data_ptr(),
                 None if m.obj is None else m.obj.data_ptr(), m.n_vert, m.n_tri)
    ps = out.struct()
    _check(lib().fhv_capture_arrays(ctx(), C.byref(mesh), C.byref(d), C.byref(ps), _ptr(ws), ws.numel(),
                                    _stream()), "fhv_capture_arrays")
    return out


def compact_workspace(d: Desc_, capacity: int) -> int:
    return int(lib().fhv_compact_workspace(C.byref(d), capacity))


def compact(lists: Lists, d: Desc_, out: Pofa, ws: torch.Tensor | None = None) -> Pofa:
    need = compact_workspace(d, lists.capacity)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=lists.head.device)
    ls = lists.struct()
    ps = out.struct()
    _check(lib().fhv_compact(ctx(), C.byref(ls), C.byref(d), C.byref(ps), _ptr(ws), ws.numel(),
                             _stream()), "fhv_compact")
    return out


# ------------------------------------------------------------------ splat

@dataclass
class Images:
    zbuf: torch.Tensor    # int64 [V, H, W]
    rgba: torch.Tensor    # int32 [V, H, W]
    depth: torch.Tensor   # float32 [V, H, W]
    cov: torch.Tensor     # uint8 [V, H, W]


def alloc_images(n_views: int, width: int, height: int, device="cuda") -> Images:
    shp = (n_views, height, width)
    return Images(torch.empty(shp, dtype=torch.int64, device=device),
                  torch.empty(shp, dtype=torch.int32, device=device),
                  torch.empty(shp, dtype=torch.float32, device=device),
                  torch.empty(shp, dtype=torch.uint8, device=device))


def views_struct(views) -> C.Array:
    arr = (View_ * len(views))()
    for i, v in enumerate(views):
        arr[i].m[:] = [float(x) for x in np.asarray(v.m, np.float32).reshape(12)]
        arr[i].width, arr[i].height, arr[i].splat_px = v.width, v.height, v.splat_px
    return arr


def splat_workspace(cap_frag: int, n_views: int, width: int, height: int) -> int:
    return int(lib().fhv_splat_workspace(cap_frag, n_views, width, height))


def splat(arrays: Pofa, d: Desc_, views, out: Images | None = None, vstruct=None,
          ws: torch.Tensor | None = None) -> Images:
    """fhv_splat of all views (at most 32 per call; more are split)."""
    W, H = views[0].width, views[0].height
    if out is None:
        out = alloc_images(len(views), W, H, device=arrays.frag.device)
    need = splat_workspace(arrays.cap_frag, min(len(views), 32), W, H)
    if need == 0:
        raise FhvError("fhv_splat_workspace: sizes out of range")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=arrays.frag.device)
    ps = arrays.struct()
    for v0 in range(0, len(views), 32):
        vs = views[v0:v0 + 32]
        arr = vstruct if (vstruct is not None and len(views) <= 32) else views_struct(vs)
        _check(lib().fhv_splat(ctx(), C.byref(ps), C.byref(d), arr, len(vs),
                               _ptr(out.zbuf[v0:]), _ptr(out.rgba[v0:]), _ptr(out.depth[v0:]),
                               _ptr(out.cov[v0:]), _ptr(ws), ws.numel(), _stream()), "fhv_splat")
    return out


SPLAT_STATIC_BYTES = 64 << 20   # FHV_SPLAT_STATIC_BYTES


def splat_static(arrays: Pofa, d: Desc_, views, out: Images, vstruct=None) -> Images:
    """fhv_splat_static of up to 32 views into the caller's images: the
    library's static scratch instead of a workspace; nothing is allocated."""
    if len(views) > 32:
        raise FhvError("fhv_splat_static: at most 32 views per call")
    arr = vstruct if vstruct is not None else views_struct(views)
    ps = arrays.struct()
    _check(lib().fhv_splat_static(ctx(), C.byref(ps), C.byref(d), arr, len(views), _ptr(out.zbuf),
                                  _ptr(out.rgba), _ptr(out.depth), _ptr(out.cov), _stream()),
           "fhv_splat_static")
    return out


def light_vectors(view, light_dir, ka: float = 0.2, kd: float = 0.7, ks: float = 0.3, shine: int = 5):
    """[13] float32 light record for a view: unit light direction (towards
    the light), unit viewer direction (towards the viewer: minus the view's
    depth axis), their half vector, ka, kd, ks, shine (exponent 2^shine)."""
    m = np.asarray(view.m, np.float64).reshape(3, 4)
    vv = -m[2, :3] / np.linalg.norm(m[2, :3])
    ll = np.asarray(light_dir, np.float64)
    ll = ll / np.linalg.norm(ll)
    hh = (ll + vv) / np.linalg.norm(ll + vv)
    return np.concatenate([ll, vv, hh, [ka, kd, ks, float(shine)]]).astype(np.float32)


def shade(arrays: Pofa, images: Images, lights) -> torch.Tensor:
    """fhv_shade of a splat's z-buffers (images from fhv.splat with the same
    arrays); lights: [V, 13] records (light_vectors). Returns float32
    [V, H, W, 4]."""
    V, H, W = images.zbuf.shape
    lights = np.asarray(lights, np.float32).reshape(V, 13)
    arr = (Light_ * V)()
    for i in range(V):
        arr[i].l[:] = [float(x) for x in lights[i, 0:3]]
        arr[i].v[:] = [float(x) for x in lights[i, 3:6]]
        arr[i].h[:] = [float(x) for x in lights[i, 6:9]]
        arr[i].ka, arr[i].kd, arr[i].ks = float(lights[i, 9]), float(lights[i, 10]), float(lights[i, 11])
        arr[i].shine = int(lights[i, 12])
    out = torch.empty((V, H, W, 4), dtype=torch.float32, device=images.zbuf.device)
    ps = arrays.struct()
    _check(lib().fhv_shade(ctx(), C.byref(ps), _ptr(images.zbuf), V, W, H, arr, _ptr(out), _stream()), "fhv_shade")
    return out


FHV_RAY_NEAREST, FHV_RAY_BLEND = 0, 1


def raycast_workspace(d: Desc_) -> int:
    return int(lib().fhv_raycast_workspace(C.byref(d)))


def raycast(arrays: Pofa, d: Desc_, views, mode: int = FHV_RAY_BLEND, tau: float = 0.0,
            out: torch.Tensor | None = None, ws: torch.Tensor | None = None, vstruct=None) -> torch.Tensor:
    """fhv_raycast of all views (at most 32 per call; more are split).
    Returns float32 [V, H, W, 4]: premultiplied R, G, B and 1 - T."""
    W, H = views[0].width, views[0].height
    dev = arrays.frag.device
    if out is None:
        out = torch.empty((len(views), H, W, 4), dtype=torch.float32, device=dev)
    need = raycast_workspace(d)
    if need == 0:
        raise FhvError("fhv_raycast_workspace: unsupported descriptor")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ps = arrays.struct()
    for v0 in range(0, len(views), 32):
        vs = views[v0:v0 + 32]
        arr = vstruct if (vstruct is not None and len(views) <= 32) else views_struct(vs)
        _check(lib().fhv_raycast(ctx(), C.byref(ps), C.byref(d), arr, len(vs), mode, float(tau),
                                 _ptr(out[v0:]), _ptr(ws), ws.numel(), _stream()), "fhv_raycast")
    return out


# ------------------------------------------------------------------ timing

def profile_begin():
    """Start bracketing every library kernel with HIP events."""
    _check(lib().fhv_profile_begin(ctx()), "fhv_profile_begin")


def profile_end() -> dict[str, tuple[int, float]]:
    """Stop; returns {kernel scope name: (launches, summed ms)}."""
    arr = (KernelStat_ * 64)()
    n = C.c_uint32()
    _check(lib().fhv_profile_end(ctx(), arr, 64, C.byref(n)), "fhv_profile_end")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms))
            for i in range(min(n.value, 64))}


FHV_PROBE_COPY, FHV_PROBE_ADD_U32, FHV_PROBE_EXCH_U32, FHV_PROBE_MIN_U64 = 0, 1, 2, 3
FHV_PROBE_READ, FHV_PROBE_WRITE = 4, 5
FHV_PROBE_COPY_CACHED, FHV_PROBE_READ_CACHED, FHV_PROBE_WRITE_CACHED = 6, 7, 8


def probe(kind: int, buf: torch.Tensor, line: int = 128, passes: int = 1):
    """One ceiling probe over `buf` (device tensor, any dtype) on torch's
    current stream: a copy of its first half onto its second, a read or a
    write of every byte, or one atomic per `line`-byte line and pass."""
    nbytes = buf.numel() * buf.element_size()
    _check(lib().fhv_probe(ctx(), kind, _ptr(buf), nbytes, line, passes, _stream()), "fhv_probe")


# ------------------------------------------------------------------ learned fill

def unet_param_count(levels: int = 4) -> int:
    return int(lib().fhv_unet_param_count(levels))


FHV_FILL_INFER, FHV_FILL_TRAIN, FHV_FILL_TRACE = 0, 1, 2


def fill_workspace(levels: int, n_img: int, height: int, width: int, training: bool | int) -> int:
    mode = training if isinstance(training, int) and not isinstance(training, bool) else (1 if training else 0)
    return int(lib().fhv_fill_workspace(levels, n_img, height, width, mode))


def _ws(t: torch.Tensor | None, need: int, device) -> torch.Tensor:
    if t is None or t.numel() < need:
        t = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    return t


def fill(params: torch.Tensor, rgba: torch.Tensor, depth: torch.Tensor, cov: torch.Tensor,
         levels: int = 4, residual: bool = False, ws: torch.Tensor | None = None):
    """fhv_fill on [N, H, W] splat images; returns (rgba int32 [N,H,W],
    residual float32 [N,H,W,3] or None)."""
    N, H, W = rgba.shape
    ws = _ws(ws, fill_workspace(levels, N, H, W, False), rgba.device)
    out = torch.empty((N, H, W), dtype=torch.int32, device=rgba.device)
    res = torch.empty((N, H, W, 3), dtype=torch.float32, device=rgba.device) if residual else None
    _check(lib().fhv_fill(ctx(), levels, _ptr(params), _ptr(rgba), _ptr(depth), _ptr(cov), N, H, W,
                          _ptr(out), _ptr(res), _ptr(ws), ws.numel(), _stream()), "fhv_fill")
    return out, res


def fill_train_step(params: torch.Tensor, m: torch.Tensor | None, v: torch.Tensor | None, step: int,
                    lr: float, rgba: torch.Tensor, depth: torch.Tensor, cov: torch.Tensor,
                    target: torch.Tensor, levels: int = 4, loss: torch.Tensor | None = None,
                    grad: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """fhv_fill_train_step; params, m, v updated in place (step >= 1)."""
    N, H, W = rgba.shape
    ws = _ws(ws, fill_workspace(levels, N, H, W, True), rgba.device)
    _check(lib().fhv_fill_train_step(ctx(), levels, _ptr(params), _ptr(m), _ptr(v), step, lr,
                                     _ptr(rgba), _ptr(depth), _ptr(cov), _ptr(target), N, H, W,
                                     _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(), _stream()),
           "fhv_fill_train_step")
    return ws


def fill_trace_tensors(levels: int, n_img: int, height: int, width: int) -> list[dict]:
    """fhv_fill_trace_tensors: five entries per parameter layer (input,
    output, gradient received, masked gradient, input gradient); None where
    a layer has no such tensor."""
    n = int(lib().fhv_fill_trace_tensors(levels, n_img, height, width, None, 0))
    if n == 0:
        raise FhvError("fhv_fill_trace_tensors: sizes out of range")
    arr = (FillTensor_ * n)()
    lib().fhv_fill_trace_tensors(levels, n_img, height, width, arr, n)
    return [None if t.channels == 0 else {"offset": int(t.offset), "stride": int(t.stride),
                                          "channels": int(t.channels), "shape": (t.n, t.height, t.width)}
            for t in arr]


def fill_train_step_traced(params: torch.Tensor, rgba: torch.Tensor, depth: torch.Tensor, cov: torch.Tensor,
                           target: torch.Tensor, levels: int = 4, loss: torch.Tensor | None = None,
                           grad: torch.Tensor | None = None) -> torch.Tensor:
    """fhv_fill_train_step_traced with step 0 (gradients only); returns the
    workspace, whose tensors fill_trace_tensors locates."""
    N, H, W = rgba.shape
    ws = _ws(None, fill_workspace(levels, N, H, W, FHV_FILL_TRACE), rgba.device)
    _check(lib().fhv_fill_train_step_traced(ctx(), levels, _ptr(params), None, None, 0, 0.0,
                                            _ptr(rgba), _ptr(depth), _ptr(cov), _ptr(target), N, H, W,
                                            _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(), _stream()),
           "fhv_fill_train_step_traced")
    return ws


# ------------------------------------------------------------------ tuning

def get_tuning() -> dict:
    t = Tuning_()
    _check(lib().fhv_get_tuning(ctx(), C.byref(t)), "fhv_get_tuning")
    return {"tile_w": t.tile_w, "raster_wg": t.raster_wg, "splat_wg": t.splat_wg}


def set_tuning(tile_w: int = 8, raster_wg: int = 16, splat_wg: int = 16):
    t = Tuning_(tile_w, raster_wg, splat_wg)
    _check(lib().fhv_set_tuning(ctx(), C.byref(t)), "fhv_set_tuning")


# ------------------------------------------------------------------ batches

@dataclass
class DeviceBatch:
    pos: torch.Tensor        # float32 [nv, 3], all scenes
    rgba: torch.Tensor       # int32 [nv]
    tri: torch.Tensor        # int32 [nt, 3], indices into the concatenated vertices
    obj: torch.Tensor | None
    scene_tri: torch.Tensor  # int32 [n_scenes + 1] triangle offsets
    n_scenes: int
    levels: int
    tri_off: np.ndarray      # host copy of scene_tri

    def struct(self) -> BatchMesh_:
        return BatchMesh_(self.pos.data_ptr(), self.rgba.data_ptr(), self.tri.data_ptr(),
                          _ptr(self.obj), self.scene_tri.data_ptr(), int(self.pos.shape[0]),
                          int(self.tri.shape[0]), self.n_scenes, self.levels)


def to_device_batch(meshes, levels: int, device="cuda") -> DeviceBatch:
    """Concatenate host meshes (scenes.Mesh) into one batch on the device."""
    pos, rgba, tri, obj = [], [], [], []
    nv = 0
    offs = [0]
    for m in meshes:
        pos.append(np.asarray(m.pos, np.float32))
        rgba.append(np.asarray(m.rgba, np.uint32))
        tri.append(np.asarray(m.tri, np.uint64) + nv)
        obj.append(np.zeros(m.tri.shape[0], np.uint8) if m.obj is None else np.asarray(m.obj, np.uint8))
        nv += m.pos.shape[0]
        offs.append(offs[-1] + m.tri.shape[0])
    assert nv < 2 ** 32 and offs[-1] < 2 ** 31
    cat = lambda xs, dt: np.ascontiguousarray(np.concatenate(xs).astype(dt))
    t = lambda a: torch.from_numpy(a).to(device)
    off = np.array(offs, np.uint32)
    return DeviceBatch(t(cat(pos, np.float32)), t(cat(rgba, np.uint32).view(np.int32)),
                       t(cat(tri, np.uint32).view(np.int32)), t(cat(obj, np.uint8)),
                       t(off.view(np.int32)), len(meshes), levels, off)


def batch_view_matrices(views_per_scene, device="cuda") -> torch.Tensor:
    """float32 [n_scenes, n_views, 12] device tensor of view matrices."""
    m = np.stack([np.stack([np.asarray(v.m, np.float32).reshape(12) for v in vs]) for vs in views_per_scene])
    return torch.from_numpy(np.ascontiguousarray(m)).to(device)


def alloc_batch_lists(b: DeviceBatch, capacity: int, link: bool = False, device="cuda") -> Lists:
    """Pool, keys and counter for a batch; head array only when link=True."""
    ks = b.n_scenes * 8 ** b.levels
    kt = torch.int64 if ks > 2 ** 32 else torch.int32
    head = torch.empty(ks, dtype=torch.int32, device=device) if link else None
    return Lists(head, torch.empty((max(capacity, 1), 4), dtype=torch.int32, device=device),
                 torch.empty(max(capacity, 1), dtype=kt, device=device),
                 torch.zeros(1, dtype=torch.int64, device=device), capacity, ks)


def batch_workspace(b: DeviceBatch, vstruct: BatchViews_, capacity: int) -> int:
    ms = b.struct()
    return int(lib().fhv_batch_workspace(C.byref(ms), C.byref(vstruct), capacity))


def batch_run(b: DeviceBatch, vm: torch.Tensor, width: int, height: int, splat_px: int, lists: Lists,
              out: Pofa, img: Images, ws: torch.Tensor | None = None, flags: int = 0) -> torch.Tensor:
    """fhv_batch_run; img tensors are [n_scenes * n_views, H, W]. Returns the
    workspace tensor for reuse."""
    n_views = int(vm.shape[1])
    vs = BatchViews_(vm.data_ptr(), n_views, width, height, splat_px)
    ms = b.struct()
    need = int(lib().fhv_batch_workspace(C.byref(ms), C.byref(vs), lists.capacity))
    if need == 0:
        raise FhvError("fhv_batch_workspace: invalid batch shape")
    ws = _ws(ws, need, b.pos.device)
    ls = lists.struct()
    ps = out.struct()
    _check(lib().fhv_batch_run(ctx(), C.byref(ms), C.byref(vs), C.byref(ls), C.byref(ps), _ptr(img.zbuf),
                               _ptr(img.rgba), _ptr(img.depth), _ptr(img.cov), _ptr(ws), ws.numel(), flags,
                               _stream()), "fhv_batch_run")
    return ws

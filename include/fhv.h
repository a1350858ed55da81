/*
 * fhv.h - C ABI of the MI355X (gfx950) fragment-history-volume library.
 *
 * Fragment-history volumes (Inacio and Springer, arXiv 2211.15460) record
 * every fragment a rasterizer produces for a scene, with no culling of any
 * kind, in pre-allocated storage (Sec. 3.1, Sec. 3.2), and reconstruct novel
 * views from that record (Sec. 3.3). This library implements the
 * data-parallel path:
 *
 *   fhv_capture  rasterize triangles into per-pixel (FHV_PPFL) or per-octant
 *                (FHV_POFL) linked fragment lists, Sec. 3.1 "Simple Layout"
 *                and "Octree Layout", Sec. 3.2 FHV_PPFL / FHV_POFL;
 *   fhv_compact  turn the lists into per-octant arrays (FHV_POFA): a count
 *                and an offset per occupied octant, offsets in Morton order,
 *                each octant's fragments contiguous, Sec. 3.1 and 3.2
 *                FHV_POFA;
 *   fhv_splat    point-splat the arrays into novel views, the nearest
 *                fragment per pixel winning, Sec. 3.3.
 *
 * Conventions shared by every call:
 *   - Every buffer pointer in a struct or argument is a DEVICE pointer owned
 *     by the caller, unless the comment says "host". The library allocates
 *     nothing on the device; scratch memory comes in through `ws` (except
 *     fhv_splat_static, whose scratch is a fixed array in the library).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the calls return without waiting for it. Results that are data
 *     dependent (fragment counts, occupied octants) stay on the device.
 *   - Host-side argument checks happen before anything is enqueued; a
 *     negative status means nothing was enqueued. A positive status
 *     FHV_EHIP + e reports HIP runtime error e from a launch.
 *   - Calls on different streams with disjoint buffers do not interact;
 *     calls sharing a workspace or output buffers must be ordered by the
 *     caller.
 *   - Records are 16 bytes, four little-endian uint32 words:
 *       w0  PPFL: depth24 | aux << 24
 *           POFL: sub-leaf x | y << 8 | z << 16 | aux << 24 (grid units)
 *       w1  RGBA8 interpolated from the vertices, R in the low byte
 *       w2  octahedral-packed face normal, int16 x | int16 y << 16
 *       w3  lists: index of the previous fragment of the same key, or
 *           0xFFFFFFFF; arrays: rank of the fragment's octant in the table
 *     aux is the low byte of the triangle's object id (0 without ids).
 *
 * Geometry conventions (the paper fixes none of them):
 *   - PPFL: orthographic capture of clip space [-1,1]^3 along +z into a
 *     width x height window, y up; screen positions in 16.8 fixed point,
 *     one sample at every pixel centre; depth24 = rint((z+1)/2 (2^24-1)).
 *     Triangles with a vertex coordinate beyond +-64 or not finite are
 *     skipped.
 *   - POFL: scene cube [0,1)^3 on a grid of 2^(L+8) units per side; each
 *     triangle is rasterized in the tangent plane of its own packed normal
 *     (Sec. 3.2, Fig. 8) on a lattice of 2^7 grid units (2^(L+1) samples
 *     per side) anchored at the grid origin; the fragment's leaf octant is
 *     the top L bits of its grid position per axis, keyed by the Morton
 *     code with x as the most significant bit of each level. Triangles with
 *     a non-finite coordinate or a zero integer normal are skipped.
 *   - Both: top-left fill rule for counter-clockwise triangles with y up;
 *     both windings are rasterized; attributes are interpolated with integer
 *     edge-function weights, (sum_k w_k a_k + floor(A/2)) / A.
 */
#ifndef FHV_H
#define FHV_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define FHV_API __attribute__((visibility("default")))
#else
#define FHV_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fhv_status;
#define FHV_OK 0
#define FHV_EINVAL (-1)     /* null pointer, bad mode, inconsistent sizes   */
#define FHV_EWORKSPACE (-2) /* ws_bytes below the workspace query's result  */
#define FHV_ERANGE (-3)     /* a size beyond what the kernels support       */
#define FHV_EHIP 1000       /* FHV_EHIP + hipError_t from the HIP runtime   */

enum { FHV_PPFL = 0, FHV_POFL = 1 };

typedef struct fhv_ctx fhv_ctx; /* opaque: device id and properties         */
typedef void* fhv_stream;       /* hipStream_t                              */

/* Context for HIP device `hip_device` (made current by every call).
 * *out receives a host object freed by fhv_destroy. */
FHV_API fhv_status fhv_create(fhv_ctx** out, int hip_device);
FHV_API fhv_status fhv_destroy(fhv_ctx* ctx);
/* Static string naming a status code (never NULL). */
FHV_API const char* fhv_status_str(fhv_status s);

/* Indexed triangle soup. pos: float [n_vert][3] (PPFL: clip space; POFL:
 * scene cube [0,1)); rgba: uint32 [n_vert]; tri: uint32 [n_tri][3] vertex
 * indices, every index < n_vert (not checked on the device); obj: uint8
 * [n_tri] object ids or NULL. */
typedef struct {
    const float* pos;
    const uint32_t* rgba;
    const uint32_t* tri;
    const uint8_t* obj;
    uint32_t n_vert;
    uint32_t n_tri;
} fhv_mesh;

/* What to capture. PPFL: width, height in [1, 16384]; POFL: levels in
 * [1, 11] (octree depth L). Unused fields are ignored.
 * projection (POFL only; PPFL requires 0): the plane each triangle is
 * rasterized in (Sec. 3.2, Fig. 7 and 8, Table 2). Every variant samples its
 * plane on a lattice of 2^7 grid units anchored at the projected grid origin
 * and interpolates the sample's 3D grid position, colour and flat normal:
 *   FHV_PROJ_NORMAL      the triangle's own plane (tangent frame of its packed
 *                        normal; "1-Pass/Normal", the default)
 *   FHV_PROJ_VIEW        the x-y plane (seen along z, the capture view;
 *                        "1-Pass/View")
 *   FHV_PROJ_AXES_3PASS  the y-z, z-x and x-y planes in three passes over the
 *                        triangles ("3-Pass/1-Way")
 *   FHV_PROJ_AXES_1PASS  the same three planes, three projected copies of
 *                        every triangle in one pass ("1-Pass/3-Way"; the same
 *                        fragments as 3-Pass/1-Way, in another order)
 * A triangle seen edge-on in a plane yields no fragments there. */
#define FHV_PROJ_NORMAL 0u
#define FHV_PROJ_VIEW 1u
#define FHV_PROJ_AXES_3PASS 2u
#define FHV_PROJ_AXES_1PASS 3u

typedef struct {
    uint32_t mode;
    uint32_t width;
    uint32_t height;
    uint32_t levels;
    uint32_t projection;
} fhv_capture_desc;

/* Fragment lists (Sec. 3.1, Fig. 3 and Fig. 5).
 * head: uint32 [n_head], n_head = width*height (PPFL) or 8^L (POFL); entry
 *       = index of the last fragment inserted for that pixel/octant, or
 *       0xFFFFFFFF. Reset by fhv_capture.
 * pool: uint32 [capacity][4] records, 16-byte aligned; capacity < 2^32 - 1.
 * keys: the pixel or octant key of every pool slot (a sidecar that lets
 *       fhv_compact read the pool linearly): uint32 [capacity] when n_head
 *       <= 2^32, else uint64 [capacity].
 * counter: one uint64; after the stream has run, the number of fragments
 *       produced. Reset by fhv_capture. If *counter > capacity the capture
 *       overflowed: the pool holds the first `capacity` fragments that
 *       claimed a slot, no head or link refers to an index >= capacity, and
 *       the caller re-allocates *counter slots and captures again (the
 *       paper's re-allocation for the next frame, Sec. 3.1). */
typedef struct {
    uint32_t* head;
    uint64_t n_head;
    uint32_t* pool;
    uint64_t capacity;
    void* keys;
    uint64_t* counter;
} fhv_lists;

/* Bytes of scratch memory fhv_capture needs for n_tri triangles; 0 for an
 * invalid desc. */
FHV_API size_t fhv_capture_workspace(const fhv_capture_desc* desc, uint32_t n_tri);

/* Capture every rasterized fragment of `mesh` (Sec. 3.2): resets head to
 * 0xFFFFFFFF and the counter to 0, then for every covered sample takes
 * idx = counter++; when idx < capacity it writes the record with w3 = the
 * key's previous head and makes idx the key's head (atomic exchange), and
 * writes keys[idx]. Fragment order in the pool and in each list is not
 * deterministic; the multiset of records per key is.
 * Errors: EINVAL (null ctx/desc/mesh arrays/lists arrays, bad mode, n_head
 * not matching desc), ERANGE (sizes out of range), EWORKSPACE. */
FHV_API fhv_status fhv_capture(fhv_ctx* ctx, const fhv_mesh* mesh, const fhv_capture_desc* desc,
                       const fhv_lists* lists, void* ws, size_t ws_bytes, fhv_stream stream);

/* Per-octant arrays (FHV_POFA, Sec. 3.1 Fig. 6, Sec. 3.2).
 * oct_key/oct_off/oct_cnt: [cap_occ] table of occupied keys ascending, the
 *       offset of the key's first fragment in frag and its fragment count.
 * frag: uint32 [cap_frag][4], 16-byte aligned; cap_frag >= the lists'
 *       capacity.
 * n_occ: one uint64, number of occupied keys (table rows at index >=
 *       cap_occ are not written); n_frag: one uint64, number of fragments
 *       in frag = min(counter, capacity). */
typedef struct {
    uint64_t* oct_key;
    uint32_t* oct_off;
    uint32_t* oct_cnt;
    uint64_t cap_occ;
    uint32_t* frag;
    uint64_t cap_frag;
    uint64_t* n_occ;
    uint64_t* n_frag;
} fhv_pofa;

/* Bytes of scratch memory fhv_compact needs for lists of `capacity` slots. */
FHV_API size_t fhv_compact_workspace(const fhv_capture_desc* desc, uint64_t capacity);

/* Compaction (Sec. 3.2 FHV_POFA): for every occupied key in ascending
 * order, count = its list length, offset = sum of the counts of all smaller
 * keys; its records are stored at frag[offset .. offset+count) ascending by
 * (w0, w1, w2) as unsigned words, with w3 = the key's rank in the table.
 * PPFL lists compact the same way with key = py*width + px (an S-buffer-like
 * per-pixel array). Reads the pool's first min(counter, capacity) slots and
 * their keys; the lists must come from fhv_capture with the same desc.
 * Errors: EINVAL, ERANGE, EWORKSPACE as for fhv_capture. */
FHV_API fhv_status fhv_compact(fhv_ctx* ctx, const fhv_lists* lists, const fhv_capture_desc* desc,
                       const fhv_pofa* out, void* ws, size_t ws_bytes, fhv_stream stream);

/* POFL per-octant arrays straight from the triangles, created the way the
 * paper creates FHV_POFA (Sec. 3.2): a first rasterization counts the
 * fragments of every octant, a prefix sum in Morton order turns the counts
 * into offsets, and a second rasterization stores every fragment at its
 * octant's next free slot; no lists and no pool. The result is the one
 * fhv_compact makes from fhv_capture's lists (the same table, offsets,
 * counts and records in the same canonical in-octant order), bit for bit.
 * out: as for fhv_compact; cap_frag must be >= 1 and < 2^32 - 1. If the
 * scene has more than cap_frag fragments, *n_frag is set to their number,
 * *n_occ to 0 and nothing else is written (allocate and call again, as
 * after an overflowed capture). ws: fhv_capture_arrays_workspace(desc,
 * n_tri, out->cap_frag) bytes, device, caller-owned.
 * Errors: EINVAL (null pointers, PPFL desc, misaligned frag), ERANGE,
 * EWORKSPACE. */
FHV_API size_t fhv_capture_arrays_workspace(const fhv_capture_desc* desc, uint32_t n_tri, uint64_t capacity);
FHV_API fhv_status fhv_capture_arrays(fhv_ctx* ctx, const fhv_mesh* mesh, const fhv_capture_desc* desc,
                                      const fhv_pofa* out, void* ws, size_t ws_bytes, fhv_stream stream);

/* One novel view (host struct, passed by value inside a host array).
 * m: row-major fp32 3x4 matrix taking a fragment position to (screen x,
 * screen y, depth) with screen units of pixels, y up, and depth > 0
 * growing away from the viewer; each row is evaluated in fp32 as
 * ((m0 x + m1 y) + m2 z) + m3 with no fused multiply-add. Fragment
 * positions: PPFL (px + 1/2, py + 1/2, depth24); POFL grid position + 1/2
 * per axis. splat_px: side k of the square footprint, >= 1. */
typedef struct {
    float m[12];
    uint32_t width;
    uint32_t height;
    uint32_t splat_px;
} fhv_view;

/* Point splat (Sec. 3.3): every array fragment i covers the k x k pixels
 * whose lower-left pixel is floor(s + 1/2 - k/2) per axis in every view;
 * per pixel the smallest (fp32 depth bits << 32 | i) wins (a 64-bit minimum
 * in an on-chip tile of the view); fragments with depth <= 0 or NaN are
 * skipped. Then each pixel resolves to the winner's w1 colour, its depth and
 * coverage 1, or to 0, 0.0 and 0 when nothing covers it.
 * Fragments whose rank has no stored table row (rank >= cap_occ) are not
 * drawn. The arrays must be in key order, as fhv_compact and
 * fhv_capture_arrays leave them.
 * views: host array of n_views in [1, 32] entries sharing width, height in
 * [1, 16384]. zbuf: uint64 [n_views][height][width] winning keys (the
 * input of fhv_shade), 16-byte aligned; rgba: uint32, depth: float, cov:
 * uint8, each [n_views][height][width]. ws: fhv_splat_workspace(
 * arrays->cap_frag, n_views, width, height) bytes, device, caller-owned;
 * 0 from the query means the sizes are out of range.
 * Errors: EINVAL (null pointers, views of different sizes, splat_px 0 or
 * above 64), ERANGE, EWORKSPACE. */
FHV_API size_t fhv_splat_workspace(uint64_t cap_frag, uint32_t n_views, uint32_t width, uint32_t height);
FHV_API fhv_status fhv_splat(fhv_ctx* ctx, const fhv_pofa* arrays, const fhv_capture_desc* desc,
                     const fhv_view* views, uint32_t n_views, uint64_t* zbuf, uint32_t* rgba,
                     float* depth, uint8_t* cov, void* ws, size_t ws_bytes, fhv_stream stream);

/* fhv_splat without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): same arguments (minus ws), same kernels, same
 * results. The scratch is a FHV_SPLAT_STATIC_BYTES array in the library's
 * device image, one per GPU, present from the library's load until the
 * process ends; fhv_create looks up its address on the context's device.
 * The call allocates nothing and calls no allocating routine.
 * Limit: fhv_splat_workspace(arrays->cap_frag, n_views, width, height) must
 * be at most FHV_SPLAT_STATIC_BYTES (cap_frag up to about 7.8 M records
 * for a few 1080p views, 7.5 M for 32 of them, 7.2 M for sixteen 4K views:
 * each 64 x 64 tile of the views takes about 170 bytes of it); larger calls
 * return EWORKSPACE before anything is enqueued. Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (each call clears what it counts in): calls on one
 * stream are ordered, but calls that can overlap on one GPU (different
 * streams, or different contexts on the same device) race on it and must be
 * ordered by the caller.
 * Errors: as fhv_splat, and EWORKSPACE for calls beyond the limit. */
#define FHV_SPLAT_STATIC_BYTES (64u << 20)
FHV_API fhv_status fhv_splat_static(fhv_ctx* ctx, const fhv_pofa* arrays, const fhv_capture_desc* desc,
                                    const fhv_view* views, uint32_t n_views, uint64_t* zbuf, uint32_t* rgba,
                                    float* depth, uint8_t* cov, fhv_stream stream);

/* Ray casting (Sec. 3.3, evaluation by ray casting) of POFL per-octant
 * arrays into orthographic views. The ray of pixel (x, y) meets array
 * fragment i when i projects into that pixel, floor(s) = (x, y) per axis,
 * with depth > 0 (the splat's one-pixel footprint). The fragments a ray
 * meets are ordered by (fp32 depth bits, i) and composited front to back in
 * fp32, each operation in this order and without fused multiply-adds:
 *   a = A/255 (FHV_RAY_BLEND) or 1 (FHV_RAY_NEAREST), w = T*a,
 *   C_c = C_c + w*(c/255) for c = R, G, B, T = T*(1 - a),
 * from C = 0, T = 1, stopping after the fragment that leaves T < tau or
 * T = 0. FHV_RAY_NEAREST is simple ray casting ("R": the nearest fragment,
 * opaque); FHV_RAY_BLEND resolves transparency ("R/T"). The walk descends
 * the octree from the root through occupied octants only, rebuilding every
 * level's occupancy from the table on each call (Sec. 3.1: coarser levels
 * store the occupancy of their children).
 * Fragments whose table row was not stored (rank >= cap_occ) are not met.
 * desc: FHV_POFL with levels in [1, 10] (ERANGE above). views: host array
 * of n_views in [1, 32] entries sharing width, height in [1, 16384], each
 * with splat_px = 1. rgba: float [n_views][height][width][4] (premultiplied
 * R, G, B and 1 - T; zero where no fragment is met), device, 16-byte
 * aligned. ws: fhv_raycast_workspace(desc) bytes, device, caller-owned.
 * Errors: EINVAL (null pointers, mode, NaN tau, views of different sizes,
 * splat_px other than 1, PPFL desc), ERANGE, EWORKSPACE. */
#define FHV_RAY_NEAREST 0u
#define FHV_RAY_BLEND 1u

FHV_API size_t fhv_raycast_workspace(const fhv_capture_desc* desc);
FHV_API fhv_status fhv_raycast(fhv_ctx* ctx, const fhv_pofa* arrays, const fhv_capture_desc* desc,
                               const fhv_view* views, uint32_t n_views, uint32_t mode, float tau,
                               float* rgba, void* ws, size_t ws_bytes, fhv_stream stream);

/* Shading of the splat's nearest fragments (Sec. 5: a local illumination
 * model per fragment, Phong 1975 / Blinn 1977). Per pixel of a splat's
 * z-buffer holding a fragment: n = its packed normal unfolded from the
 * octahedron, (int16 x, int16 y)/32767 with z = (1 - |x|) - |y| and, when
 * z < 0, (x, y) = ((1 - |y|) s(x), (1 - |x|) s(y)), s(0) = +1, normalised by
 * sqrt((x^2 + y^2) + z^2); flipped when n.v < 0 (no culling at capture);
 * d = max(n.l, 0), s = (n.l > 0 ? max(n.h, 0) : 0)^(2^shine) by repeated
 * squaring; out = albedo/255 * (ka + kd d) + ks s per channel, alpha 1; fp32,
 * dot products as (x0 y0 + x1 y1) + x2 y2, no fused multiply-adds. Pixels
 * without a fragment get 0.
 * l, v, h: unit light, viewer and half vectors (world), given per view.
 * zbuf: the uint64 [n_views][height][width] z-buffer of fhv_splat with the
 * same arrays; rgba: float [n_views][height][width][4], device, 16-byte
 * aligned. lights: host array of n_views in [1, 32]; shine <= 16.
 * Errors: EINVAL (null pointers, shine above 16), ERANGE. */
typedef struct {
    float l[3];
    float v[3];
    float h[3];
    float ka, kd, ks;
    uint32_t shine;
} fhv_light;

FHV_API fhv_status fhv_shade(fhv_ctx* ctx, const fhv_pofa* arrays, const uint64_t* zbuf, uint32_t n_views,
                             uint32_t width, uint32_t height, const fhv_light* lights, float* rgba,
                             fhv_stream stream);

/* Batches (not in the paper): many POFL scenes, each with several views,
 * through capture, compaction and splat in one call. The scenes share one
 * key space, key = scene * 8^L + Morton code of the leaf, so one launch per
 * stage covers every scene and each scene's arrays are one contiguous run
 * of the table and of frag, in scene order.
 *
 * Mesh: the scenes' triangle soups concatenated; tri holds indices into
 * the concatenated pos/rgba; scene_tri: DEVICE uint32 [n_scenes + 1],
 * non-decreasing, scene_tri[0] = 0, scene_tri[n_scenes] = n_tri: scene s
 * owns triangles [scene_tri[s], scene_tri[s+1]). Every scene uses the scene
 * cube [0,1)^3 and octree depth `levels` (1..11); the key space
 * n_scenes * 8^levels is at most 2^39. */
typedef struct {
    const float* pos;
    const uint32_t* rgba;
    const uint32_t* tri;
    const uint8_t* obj;
    const uint32_t* scene_tri;
    uint32_t n_vert;
    uint32_t n_tri;
    uint32_t n_scenes;
    uint32_t levels;
} fhv_batch_mesh;

/* Views of a batch: m is a DEVICE float array [n_scenes][n_views][12],
 * one fhv_view matrix per (scene, view), read when the splat runs (a graph
 * replay sees the values present at replay time). Every view has the same
 * width, height (1..16384) and splat_px (1..64); n_views in [1, 32]. */
typedef struct {
    const float* m;
    uint32_t n_views;
    uint32_t width;
    uint32_t height;
    uint32_t splat_px;
} fhv_batch_views;

/* Kernel launch choices, per context (used by every call on it):
 * tile_w: raster tile width in samples, 8, 16 or 32 (tiles hold 64 samples:
 *   8x8, 16x4 or 32x2); raster_wg, splat_wg: workgroups per compute unit of
 *   the rasterizer and of the splat, 1..64. Results do not depend on them. */
typedef struct {
    uint32_t tile_w;
    uint32_t raster_wg;
    uint32_t splat_wg;
} fhv_tuning;

FHV_API fhv_status fhv_get_tuning(fhv_ctx* ctx, fhv_tuning* out);
FHV_API fhv_status fhv_set_tuning(fhv_ctx* ctx, const fhv_tuning* t);

#define FHV_BATCH_GRAPH 1u /* record the call's launches in a HIP graph once
                              per distinct argument set, then replay it    */
#define FHV_BATCH_TUNE 2u  /* before running, time candidate fhv_tuning
                              values on these inputs (running the stages
                              many times and waiting for the stream) and
                              keep the fastest in the context             */

FHV_API size_t fhv_batch_workspace(const fhv_batch_mesh* mesh, const fhv_batch_views* views,
                                   uint64_t capacity);

/* Capture, compaction and splat of a batch (Sec. 3.2, Sec. 3.3 per scene).
 * lists: n_head = n_scenes * 8^L (the key space); head may be NULL, then no
 *   linked lists are built (records keep w3 = 0xFFFFFFFF) and only the
 *   pool, keys and counter are written; keys are uint64 when n_head > 2^32.
 *   Overflow as for fhv_capture: after the stream has run, *counter >
 *   capacity means the arrays and images are incomplete and the call must
 *   be repeated with capacity >= *counter.
 * out: arrays as fhv_compact makes them over the whole key space; scene s's
 *   rows are those with oct_key / 8^L == s.
 * zbuf, rgba, depth, cov: [n_scenes][n_views][height][width] as for
 *   fhv_splat; a fragment only reaches its own scene's views.
 * flags: FHV_BATCH_GRAPH, FHV_BATCH_TUNE. A graph is kept per context for
 *   each distinct set of pointers, sizes and tuning (at most 8; the oldest
 *   is dropped); it is recorded on a stream of the context and launched on
 *   `stream`. Profiling (fhv_profile_begin) does not see graph launches.
 * Errors: EINVAL (null pointers, sizes, flags), ERANGE, EWORKSPACE. */
FHV_API fhv_status fhv_batch_run(fhv_ctx* ctx, const fhv_batch_mesh* mesh, const fhv_batch_views* views,
                                 const fhv_lists* lists, const fhv_pofa* out, uint64_t* zbuf,
                                 uint32_t* rgba, float* depth, uint8_t* cov, void* ws, size_t ws_bytes,
                                 uint32_t flags, fhv_stream stream);

/* Learned hole fill (not in the paper; fills what the splat leaves
 * uncovered, where Sec. 3.3 suggests adapting quad sizes or deforming
 * geometry). A U-Net of `levels` (1..4) levels with 32 * 2^l channels on
 * level l: per level two 3x3 convolutions (padding 1) with ReLU, 2x2 max pool
 * going down, 2x2 stride-2 transposed convolution going up concatenated
 * (transposed first) with the level's encoder output, and a 1x1 head to 3
 * channels: an RGB residual added to splat RGB / 255. Input channels: R, G,
 * B, A / 255, depth - 1 where covered (0 elsewhere), coverage. Weights and
 * activations are rounded to bfloat16 (nearest even) for the matrix cores;
 * sums accumulate in fp32.
 * params: fp32 vector of fhv_unet_param_count(levels) values, layer after
 *   layer: 3x3 conv W[co][ky][kx][ci] then b[co]; transposed conv
 *   W[dy][dx][co][ci] then b[co]; head W[k][c] then b[k]. Layer order: for
 *   each encoder level two convs; for each decoder level from the deepest:
 *   transposed conv, two convs; the head.
 * Images: n_img x height x width, row-major, height and width multiples of
 *   2^(levels-1); n_img * height * width < 2^31. */
FHV_API uint64_t fhv_unet_param_count(uint32_t levels);
/* Workspace bytes of fhv_fill (training FHV_FILL_INFER), fhv_fill_train_step
 * (FHV_FILL_TRAIN) or fhv_fill_train_step_traced (FHV_FILL_TRACE); 0 for
 * sizes or a mode out of range. */
#define FHV_FILL_INFER 0
#define FHV_FILL_TRAIN 1
#define FHV_FILL_TRACE 2
FHV_API size_t fhv_fill_workspace(uint32_t levels, uint32_t n_img, uint32_t height, uint32_t width,
                                  int training);

/* Inference: out_rgba = clamp(splat RGB / 255 + residual, 0, 1) * 255
 * rounded half up, alpha 255 (in fp32, splat RGB times the fp32
 * reciprocal of 255, so a channel may differ by one step from the exact
 * quotient's where the sum lands next to a rounding boundary);
 * out_residual (nullable) receives the fp32 residual
 * [n_img][height][width][3].
 * Errors: EINVAL (null pointers, levels, sizes), ERANGE, EWORKSPACE. */
FHV_API fhv_status fhv_fill(fhv_ctx* ctx, uint32_t levels, const float* params, const uint32_t* rgba,
                            const float* depth, const uint8_t* cov, uint32_t n_img, uint32_t height,
                            uint32_t width, uint32_t* out_rgba, float* out_residual, void* ws,
                            size_t ws_bytes, fhv_stream stream);

/* One training step on a batch: loss = mean over n_img*height*width*3 of
 * (splat RGB / 255 + residual - target RGB / 255)^2, its gradient w.r.t.
 * params by backpropagation (written to grad_out when not null), then, when
 * step >= 1, an Adam update (beta 0.9 / 0.999, eps 1e-8, bias correction for
 * step `step`) of params, adam_m and adam_v in place. step 0 computes the
 * loss and gradient only. loss_out (device, nullable): one float. */
FHV_API fhv_status fhv_fill_train_step(fhv_ctx* ctx, uint32_t levels, float* params, float* adam_m,
                                       float* adam_v, uint32_t step, float lr, const uint32_t* rgba,
                                       const float* depth, const uint8_t* cov,
                                       const uint32_t* target_rgba, uint32_t n_img, uint32_t height,
                                       uint32_t width, float* loss_out, float* grad_out, void* ws,
                                       size_t ws_bytes, fhv_stream stream);

/* Layer-by-layer tracing of the training step, for checking every kernel
 * on the tensors it actually read: fhv_fill_train_step_traced does exactly
 * what fhv_fill_train_step does (same kernels, same results) but keeps every
 * activation gradient in a buffer of its own instead of reusing scratch
 * buffers; ws: fhv_fill_workspace(..., FHV_FILL_TRACE) bytes.
 * fhv_fill_trace_tensors describes where the tensors are afterwards: five
 * entries per parameter layer, in parameter order: [0] the layer's input
 * activation, [1] its output activation (after ReLU), [2] the gradient of
 * the loss w.r.t. that output as the layer's backward pass received it,
 * [3] that gradient after the ReLU mask (3x3 convolutions), [4] the
 * gradient w.r.t. the layer's input. The head (last layer) has [0] and [4].
 * A tensor is bfloat16 NHWC: element (i, y, x, c) at byte offset + 2 *
 * (((i * height + y) * width + x) * stride + c) of ws; channels 0 marks an
 * entry the layer does not have. out: host array of `cap` entries (NULL to
 * query the count). Returns the number of entries, 0 for bad sizes. */
typedef struct {
    uint64_t offset;
    uint32_t stride;
    uint32_t channels;
    uint32_t n;
    uint32_t height;
    uint32_t width;
} fhv_fill_tensor;
FHV_API uint32_t fhv_fill_trace_tensors(uint32_t levels, uint32_t n_img, uint32_t height, uint32_t width,
                                        fhv_fill_tensor* out, uint32_t cap);
FHV_API fhv_status fhv_fill_train_step_traced(fhv_ctx* ctx, uint32_t levels, float* params, float* adam_m,
                                              float* adam_v, uint32_t step, float lr, const uint32_t* rgba,
                                              const float* depth, const uint8_t* cov,
                                              const uint32_t* target_rgba, uint32_t n_img, uint32_t height,
                                              uint32_t width, float* loss_out, float* grad_out, void* ws,
                                              size_t ws_bytes, fhv_stream stream);

/* Kernel timing (tracing). Between fhv_profile_begin and fhv_profile_end
 * every kernel the library enqueues is bracketed by two HIP events on the
 * stream it runs on. fhv_profile_end waits for those events and reports,
 * per kernel name, the number of launches and their summed duration; it
 * writes at most `cap` entries to `out` (host array) and the number of
 * distinct kernels to *n_out. Names are static strings owned by the
 * library. Not for use while a caller captures the stream into a graph. */
typedef struct {
    const char* name;
    uint64_t launches;
    double total_ms;
} fhv_kernel_stat;

FHV_API fhv_status fhv_profile_begin(fhv_ctx* ctx);
FHV_API fhv_status fhv_profile_end(fhv_ctx* ctx, fhv_kernel_stat* out, uint32_t cap,
                                   uint32_t* n_out);

/* Measurement probes: the ceilings against which the capture, compaction
 * and splat kernels are measured (roofline of memory-side atomics and of
 * HBM copies). Not an operation of the method.
 *   FHV_PROBE_COPY      second half of buf <- first half, 16-byte vector
 *                       loads and stores (bytes a multiple of 32)
 *   FHV_PROBE_READ      every 16 bytes of buf loaded once (bytes a multiple
 *                       of 16; buf is left as it was when filled with 0xFF
 *                       bytes)
 *   FHV_PROBE_WRITE     every byte of buf set to 0xFF with 16-byte stores
 *                       (bytes a multiple of 16)
 *   The three streams above use non-temporal loads and stores (past the
 *   caches); FHV_PROBE_COPY_CACHED, FHV_PROBE_READ_CACHED and
 *   FHV_PROBE_WRITE_CACHED are the same streams with ordinary accesses, as
 *   the library's kernels make them.
 *   FHV_PROBE_ADD_U32   per line of `line` bytes and per pass: atomic add of
 *                       1 to the line's first u32, result unused
 *   FHV_PROBE_EXCH_U32  atomic exchange of the line's first u32 with
 *                       pass + 1, result used (each thread writes the sum of
 *                       what it received into the line's second u32)
 *   FHV_PROBE_MIN_U64   atomic minimum of the line's first u64 with
 *                       ((passes - pass) << 32 | line index), result unused
 * Lines are uncontended: one atomic per line per pass. `buf` is a device
 * pointer owned by the caller, 16-byte aligned; `line` is a power of two in
 * [8, 4096] (atomic probes), `passes` in [1, 1024]; FHV_EINVAL otherwise.
 * Launches on `stream`; timed by fhv_profile_begin/end as "probe.copy",
 * "probe.read", "probe.write", "probe.copy_cached", "probe.read_cached",
 * "probe.write_cached", "probe.add_u32", "probe.exch_u32", "probe.min_u64". */
#define FHV_PROBE_COPY 0u
#define FHV_PROBE_ADD_U32 1u
#define FHV_PROBE_EXCH_U32 2u
#define FHV_PROBE_MIN_U64 3u
#define FHV_PROBE_READ 4u
#define FHV_PROBE_WRITE 5u
#define FHV_PROBE_COPY_CACHED 6u
#define FHV_PROBE_READ_CACHED 7u
#define FHV_PROBE_WRITE_CACHED 8u

FHV_API fhv_status fhv_probe(fhv_ctx* ctx, uint32_t kind, void* buf, uint64_t bytes, uint32_t line,
                             uint32_t passes, fhv_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* FHV_H */

// C ABI entry points (include/fhv.h): host-side validation, workspace
// queries and dispatch to the kernels' launchers on the caller's stream.
#include <new>
#include <string.h>
#include <vector>

#include "fhv_common.h"

namespace fhv {

// Pairs of HIP events around kernel launches, resolved at the end of a
// profiling session into per-name launch counts and summed durations.
struct Profiler {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    hipError_t err = hipSuccess;

    hipEvent_t take()
    {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) err = r;
        return e;
    }
};

void prof_mark(Profiler* p, const char* name, hipStream_t s, bool start)
{
    hipEvent_t e = p->take();
    if (!e) return;
    hipError_t r = hipEventRecord(e, s);
    if (r != hipSuccess) p->err = r;
    if (start) {
        p->recs.push_back({name, e, nullptr});
    } else if (!p->recs.empty() && p->recs.back().b == nullptr) {
        p->recs.back().b = e;
    } else {
        p->spare.push_back(e);
    }
}

}  // namespace fhv

struct fhv_ctx {
    fhv::Device dev;
    fhv::Profiler prof;
    // recorded batch graphs, keyed by the bytes of every argument
    struct Graph {
        std::vector<unsigned char> key;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipStream_t rec_stream = nullptr;   // stream the graphs are recorded on
    // device address of the static splat scratch on this context's device
    void* scratch = nullptr;
};

// Scratch of fhv_splat_static: one array per GPU in the library's device
// image. Host code never uses this name as an address (on the host it is a
// stand-in, not device memory): fhv_create looks up the array's address on
// its device and keeps it in the context.
static __device__ __align__(256) unsigned char scratch[FHV_SPLAT_STATIC_BYTES];

namespace {

fhv_status hip_status(hipError_t e) { return e == hipSuccess ? FHV_OK : FHV_EHIP + (int)e; }

bool desc_ok(const fhv_capture_desc* d)
{
    if (!d) return false;
    if (d->mode == FHV_PPFL)
        return d->width >= 1 && d->width <= 16384 && d->height >= 1 && d->height <= 16384 && d->projection == 0;
    if (d->mode == FHV_POFL) return d->levels >= 1 && d->levels <= 11 && d->projection <= FHV_PROJ_AXES_1PASS;
    return false;
}

uint64_t n_head_of(const fhv_capture_desc* d)
{
    return d->mode == FHV_PPFL ? (uint64_t)d->width * d->height : 1ull << (3 * d->levels);
}

fhv_status check_lists(const fhv_lists* L, const fhv_capture_desc* d)
{
    if (!L || !L->head || !L->counter || !L->keys) return FHV_EINVAL;
    if (L->n_head != n_head_of(d)) return FHV_EINVAL;
    if (L->capacity >= 0xFFFFFFFFull) return FHV_ERANGE;
    if (L->capacity > 0 && !L->pool) return FHV_EINVAL;
    if ((uintptr_t)L->pool & 15) return FHV_EINVAL;  // 16-byte records
    return FHV_OK;
}

fhv_status set_device(fhv_ctx* ctx)
{
    return hip_status(hipSetDevice(ctx->dev.id));
}

// ---------------------------------------------------------------- batches

bool batch_shape_ok(const fhv_batch_mesh* m, const fhv_batch_views* v)
{
    if (!m || !v) return false;
    if (m->n_scenes < 1 || m->levels < 1 || m->levels > 11) return false;
    // key space n_scenes * 8^L up to 2^39 (bricks and bitmap of the
    // compaction grow with it; the splat packs a fragment's scene and grid
    // position into 63 bits)
    if (((uint64_t)m->n_scenes << (3 * m->levels)) > (1ull << 39)) return false;
    if (v->n_views < 1 || v->n_views > fhv::kMaxViews) return false;
    if (v->width < 1 || v->width > 16384 || v->height < 1 || v->height > 16384) return false;
    if (v->splat_px < 1 || v->splat_px > 64) return false;
    return (uint64_t)m->n_scenes * v->n_views * v->width * v->height < (1ull << 40);
}

fhv_capture_desc batch_desc(const fhv_batch_mesh* m)
{
    fhv_capture_desc d;
    d.mode = FHV_POFL;
    d.width = 0;
    d.height = 0;
    d.levels = m->levels;
    d.projection = FHV_PROJ_NORMAL;
    return d;
}

// Workspace: the capture's, the compaction's, then the splat's (each
// 256-byte aligned).
size_t batch_ws(const fhv_batch_mesh* m, const fhv_batch_views* v, uint64_t capacity, void* ws, void** cap_ws,
                void** cmp_ws, void** spl_ws)
{
    const fhv_capture_desc d = batch_desc(m);
    const size_t a = (fhv::capture_ws_bytes(&d, m->n_tri) + 255) & ~(size_t)255;
    const size_t b = (fhv::compact_ws_bytes(&d, (uint64_t)m->n_scenes << (3 * m->levels), capacity) + 255) &
                     ~(size_t)255;
    const size_t c = fhv::splat_ws_bytes(capacity, m->n_scenes, v->n_views, v->width, v->height);
    if (cap_ws) *cap_ws = ws;
    if (cmp_ws) *cmp_ws = ws ? (void*)((char*)ws + a) : nullptr;
    if (spl_ws) *spl_ws = ws ? (void*)((char*)ws + a + b) : nullptr;
    return a + b + c;
}

struct BatchCall {
    const fhv_batch_mesh* mesh;
    const fhv_batch_views* views;
    const fhv_lists* lists;
    const fhv_pofa* out;
    uint64_t* zbuf;
    uint32_t* rgba;
    float* depth;
    uint8_t* cov;
    void* ws;
};

hipError_t batch_capture(const fhv::Device& dev, const BatchCall& c, hipStream_t s)
{
    const fhv_capture_desc d = batch_desc(c.mesh);
    const fhv_mesh m{c.mesh->pos, c.mesh->rgba, c.mesh->tri, c.mesh->obj, c.mesh->n_vert, c.mesh->n_tri};
    const fhv::Scenes sc{c.mesh->scene_tri, c.mesh->n_scenes};
    void* cw = nullptr;
    batch_ws(c.mesh, c.views, c.lists->capacity, c.ws, &cw, nullptr, nullptr);
    return fhv::capture_launch(dev, &m, &d, c.lists, cw, s, &sc);
}

hipError_t batch_compact(const fhv::Device& dev, const BatchCall& c, hipStream_t s)
{
    const fhv_capture_desc d = batch_desc(c.mesh);
    void* mw = nullptr;
    batch_ws(c.mesh, c.views, c.lists->capacity, c.ws, nullptr, &mw, nullptr);
    return fhv::compact_launch(dev, c.lists, &d, c.out, mw, s);
}

hipError_t batch_splat(const fhv::Device& dev, const BatchCall& c, hipStream_t s)
{
    const fhv::BatchViews bv{c.views->m, c.mesh->n_scenes, c.views->n_views, c.views->width,
                             c.views->height, c.views->splat_px};
    void* sw = nullptr;
    batch_ws(c.mesh, c.views, c.lists->capacity, c.ws, nullptr, nullptr, &sw);
    // the arrays hold at most `capacity` records (the splat workspace's size)
    fhv_pofa a = *c.out;
    a.cap_frag = a.cap_frag < c.lists->capacity ? a.cap_frag : c.lists->capacity;
    return fhv::splat_batch_launch(dev, &a, c.mesh->levels, bv, c.zbuf, c.rgba, c.depth, c.cov, sw, s);
}

hipError_t batch_enqueue(const fhv::Device& dev, const BatchCall& c, hipStream_t s)
{
    hipError_t e = batch_capture(dev, c, s);
    if (e == hipSuccess) e = batch_compact(dev, c, s);
    if (e == hipSuccess) e = batch_splat(dev, c, s);
    return e;
}

// Milliseconds of the best of `reps` runs of fn on stream s.
template <class Fn>
hipError_t time_best(Fn fn, int reps, hipStream_t s, hipEvent_t a, hipEvent_t b, float* best)
{
    *best = 1e30f;
    for (int r = 0; r < reps; ++r) {
        hipError_t e = hipEventRecord(a, s);
        if (e == hipSuccess) e = fn();
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) return e;
        *best = ms < *best ? ms : *best;
    }
    return hipSuccess;
}

// Autotuner: on the call's own inputs, time the capture under every raster
// tile shape and raster grid size, then the splat under every splat grid
// size, and keep the fastest in the context. Blocks until done; the
// results do not depend on these choices.
hipError_t batch_tune(fhv_ctx* ctx, const BatchCall& c, hipStream_t s)
{
    fhv::Device d = ctx->dev;
    d.prof = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = batch_enqueue(d, c, s);   // warm-up
    const uint32_t tiles[3] = {8, 16, 32};
    const uint32_t grids[4] = {4, 8, 16, 32};
    fhv::Tuning best = d.tune;
    float best_ms = 1e30f;
    for (int ti = 0; ti < 3 && e == hipSuccess; ++ti)
        for (int gi = 0; gi < 4 && e == hipSuccess; ++gi) {
            d.tune.tile_w = tiles[ti];
            d.tune.raster_wg = grids[gi];
            float ms = 0.0f;
            e = time_best([&] { return batch_capture(d, c, s); }, 2, s, a, b, &ms);
            if (e == hipSuccess && ms < best_ms) {
                best_ms = ms;
                best.tile_w = tiles[ti];
                best.raster_wg = grids[gi];
            }
        }
    d.tune = best;
    if (e == hipSuccess) e = batch_capture(d, c, s);
    if (e == hipSuccess) e = batch_compact(d, c, s);
    best_ms = 1e30f;
    for (int gi = 0; gi < 4 && e == hipSuccess; ++gi) {
        d.tune.splat_wg = grids[gi];
        float ms = 0.0f;
        e = time_best([&] { return batch_splat(d, c, s); }, 2, s, a, b, &ms);
        if (e == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best.splat_wg = grids[gi];
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e == hipSuccess) ctx->dev.tune = best;
    return e;
}

}  // namespace

extern "C" {

fhv_status fhv_create(fhv_ctx** out, int hip_device)
{
    if (!out) return FHV_EINVAL;
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_status(e);
    if (hip_device < 0 || hip_device >= n) return FHV_EINVAL;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device);
    if (e != hipSuccess) return hip_status(e);
    // the static splat scratch's address on this device (each GPU holds its
    // own copy of the array), looked up with the device current
    int prev = 0;
    e = hipGetDevice(&prev);
    if (e != hipSuccess) return hip_status(e);
    e = hipSetDevice(hip_device);
    if (e != hipSuccess) return hip_status(e);
    void* sp = nullptr;
    e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    const hipError_t e2 = hipSetDevice(prev);
    if (e != hipSuccess) return hip_status(e);
    if (e2 != hipSuccess) return hip_status(e2);
    if (!sp) return FHV_EHIP + (int)hipErrorInvalidSymbol;
    fhv_ctx* c = new (std::nothrow) fhv_ctx;
    if (!c) return FHV_EINVAL;
    c->scratch = sp;
    c->dev.id = hip_device;
    c->dev.cus = cus > 0 ? cus : 256;
    c->dev.prof = nullptr;
    c->dev.tune = fhv::Tuning{};
    *out = c;
    return FHV_OK;
}

fhv_status fhv_destroy(fhv_ctx* ctx)
{
    if (!ctx) return FHV_OK;
    (void)hipSetDevice(ctx->dev.id);
    for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    if (ctx->rec_stream) (void)hipStreamDestroy(ctx->rec_stream);
    for (auto& r : ctx->prof.recs) {
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->prof.spare) (void)hipEventDestroy(e);
    delete ctx;
    return FHV_OK;
}

fhv_status fhv_profile_begin(fhv_ctx* ctx)
{
    if (!ctx) return FHV_EINVAL;
    for (auto& r : ctx->prof.recs) {
        ctx->prof.spare.push_back(r.a);
        if (r.b) ctx->prof.spare.push_back(r.b);
    }
    ctx->prof.recs.clear();
    ctx->prof.err = hipSuccess;
    ctx->dev.prof = &ctx->prof;
    return FHV_OK;
}

fhv_status fhv_profile_end(fhv_ctx* ctx, fhv_kernel_stat* out, uint32_t cap, uint32_t* n_out)
{
    if (!ctx || (cap > 0 && !out) || !n_out) return FHV_EINVAL;
    ctx->dev.prof = nullptr;
    fhv::Profiler& p = ctx->prof;
    std::vector<fhv_kernel_stat> acc;
    hipError_t err = p.err;
    for (auto& r : p.recs) {
        if (!r.b) continue;
        hipError_t e = hipEventSynchronize(r.b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) {
            err = e;
            continue;
        }
        size_t k = 0;
        while (k < acc.size() && strcmp(acc[k].name, r.name) != 0) ++k;
        if (k == acc.size()) acc.push_back({r.name, 0, 0.0});
        acc[k].launches += 1;
        acc[k].total_ms += ms;
    }
    for (size_t k = 0; k < acc.size() && k < cap; ++k) out[k] = acc[k];
    *n_out = (uint32_t)acc.size();
    return hip_status(err);
}

const char* fhv_status_str(fhv_status s)
{
    switch (s) {
    case FHV_OK: return "ok";
    case FHV_EINVAL: return "invalid argument";
    case FHV_EWORKSPACE: return "workspace too small";
    case FHV_ERANGE: return "size out of range";
    default: return s >= FHV_EHIP ? "HIP runtime error" : "unknown status";
    }
}

size_t fhv_capture_workspace(const fhv_capture_desc* desc, uint32_t n_tri)
{
    if (!desc_ok(desc)) return 0;
    return fhv::capture_ws_bytes(desc, n_tri);
}

fhv_status fhv_capture(fhv_ctx* ctx, const fhv_mesh* mesh, const fhv_capture_desc* desc,
                       const fhv_lists* lists, void* ws, size_t ws_bytes, fhv_stream stream)
{
    if (!ctx || !mesh || !desc_ok(desc)) return FHV_EINVAL;
    if (desc->mode == FHV_POFL && desc->projection == FHV_PROJ_AXES_1PASS && mesh->n_tri > 0x55555555u)
        return FHV_ERANGE;   // three setup records per triangle
    fhv_status st = check_lists(lists, desc);
    if (st != FHV_OK) return st;
    if (mesh->n_tri > 0 && (!mesh->pos || !mesh->rgba || !mesh->tri || mesh->n_vert == 0))
        return FHV_EINVAL;
    if (mesh->n_tri >= (1u << 31)) return FHV_ERANGE;
    if (ws_bytes < fhv::capture_ws_bytes(desc, mesh->n_tri)) return FHV_EWORKSPACE;
    if (mesh->n_tri > 0 && !ws) return FHV_EINVAL;
    if ((st = set_device(ctx)) != FHV_OK) return st;
    return hip_status(fhv::capture_launch(ctx->dev, mesh, desc, lists, ws, (hipStream_t)stream));
}

size_t fhv_compact_workspace(const fhv_capture_desc* desc, uint64_t capacity)
{
    if (!desc_ok(desc)) return 0;
    return fhv::compact_ws_bytes(desc, n_head_of(desc), capacity);
}

fhv_status fhv_compact(fhv_ctx* ctx, const fhv_lists* lists, const fhv_capture_desc* desc,
                       const fhv_pofa* out, void* ws, size_t ws_bytes, fhv_stream stream)
{
    if (!ctx || !desc_ok(desc) || !out) return FHV_EINVAL;
    fhv_status st = check_lists(lists, desc);
    if (st != FHV_OK) return st;
    if (!out->n_occ || !out->n_frag) return FHV_EINVAL;
    if (out->cap_frag < lists->capacity) return FHV_EINVAL;
    if (lists->capacity > 0 && !out->frag) return FHV_EINVAL;
    if ((uintptr_t)out->frag & 15) return FHV_EINVAL;
    if (out->cap_occ > 0 && (!out->oct_key || !out->oct_off || !out->oct_cnt)) return FHV_EINVAL;
    if (ws_bytes < fhv::compact_ws_bytes(desc, lists->n_head, lists->capacity)) return FHV_EWORKSPACE;
    if (!ws) return FHV_EINVAL;
    if ((st = set_device(ctx)) != FHV_OK) return st;
    return hip_status(fhv::compact_launch(ctx->dev, lists, desc, out, ws, (hipStream_t)stream));
}

size_t fhv_splat_workspace(uint64_t cap_frag, uint32_t n_views, uint32_t width, uint32_t height)
{
    if (n_views == 0 || n_views > fhv::kMaxViews || width < 1 || width > 16384 || height < 1 || height > 16384 ||
        cap_frag >= 0xFFFFFFFFull || !fhv::splat_fits(cap_frag, 1, n_views, width, height))
        return 0;
    return fhv::splat_ws_bytes(cap_frag, 1, n_views, width, height);
}

namespace {

// Host-side checks shared by fhv_splat and fhv_splat_static; fills the
// kernels' view arguments and the workspace the call needs.
fhv_status splat_check(fhv_ctx* ctx, const fhv_pofa* arrays, const fhv_capture_desc* desc, const fhv_view* views,
                       uint32_t n_views, uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov,
                       fhv::ViewArgs* out, size_t* need)
{
    if (!ctx || !arrays || !desc_ok(desc) || !views) return FHV_EINVAL;
    if (n_views == 0 || n_views > fhv::kMaxViews) return FHV_ERANGE;
    if (!zbuf || !rgba || !depth || !cov || !arrays->n_frag) return FHV_EINVAL;
    if (arrays->cap_frag > 0 && (!arrays->frag || !arrays->oct_key)) return FHV_EINVAL;
    if (arrays->cap_frag >= 0xFFFFFFFFull) return FHV_ERANGE;
    if (((uintptr_t)arrays->frag & 15) || ((uintptr_t)zbuf & 15)) return FHV_EINVAL;
    fhv::ViewArgs va;
    memset(&va, 0, sizeof(va));
    va.n_views = n_views;
    va.width = views[0].width;
    va.height = views[0].height;
    va.all_k1 = 1;
    if (va.width < 1 || va.width > 16384 || va.height < 1 || va.height > 16384) return FHV_ERANGE;
    for (uint32_t v = 0; v < n_views; ++v) {
        if (views[v].width != va.width || views[v].height != va.height) return FHV_EINVAL;
        if (views[v].splat_px < 1 || views[v].splat_px > 64) return FHV_EINVAL;
        memcpy(va.m[v], views[v].m, sizeof(va.m[v]));
        va.k[v] = views[v].splat_px;
        if (views[v].splat_px != 1) va.all_k1 = 0;
        va.c[v] = 0.5f - 0.5f * (float)views[v].splat_px;
    }
    if (!fhv::splat_fits(arrays->cap_frag, 1, n_views, va.width, va.height)) return FHV_ERANGE;
    *need = fhv::splat_ws_bytes(arrays->cap_frag, 1, n_views, va.width, va.height);
    *out = va;
    return FHV_OK;
}

}  // namespace

fhv_status fhv_splat(fhv_ctx* ctx, const fhv_pofa* arrays, const fhv_capture_desc* desc,
                     const fhv_view* views, uint32_t n_views, uint64_t* zbuf, uint32_t* rgba,
                     float* depth, uint8_t* cov, void* ws, size_t ws_bytes, fhv_stream stream)
{
    fhv::ViewArgs va;
    size_t need = 0;
    fhv_status st = splat_check(ctx, arrays, desc, views, n_views, zbuf, rgba, depth, cov, &va, &need);
    if (st != FHV_OK) return st;
    if (ws_bytes < need) return FHV_EWORKSPACE;
    if (!ws) return FHV_EINVAL;
    if ((st = set_device(ctx)) != FHV_OK) return st;
    return hip_status(fhv::splat_launch(ctx->dev, arrays, desc, va, zbuf, rgba, depth, cov, ws,
                                        (hipStream_t)stream));
}

fhv_status fhv_splat_static(fhv_ctx* ctx, const fhv_pofa* arrays, const fhv_capture_desc* desc,
                            const fhv_view* views, uint32_t n_views, uint64_t* zbuf, uint32_t* rgba,
                            float* depth, uint8_t* cov, fhv_stream stream)
{
    fhv::ViewArgs va;
    size_t need = 0;
    fhv_status st = splat_check(ctx, arrays, desc, views, n_views, zbuf, rgba, depth, cov, &va, &need);
    if (st != FHV_OK) return st;
    if (need > (size_t)FHV_SPLAT_STATIC_BYTES) return FHV_EWORKSPACE;
    if (!ctx->scratch) return FHV_EINVAL;
    if ((st = set_device(ctx)) != FHV_OK) return st;
    // the kernels get the array's device address, never its host-side name
    return hip_status(fhv::splat_launch(ctx->dev, arrays, desc, va, zbuf, rgba, depth, cov, ctx->scratch,
                                        (hipStream_t)stream));
}

fhv_status fhv_probe(fhv_ctx* ctx, uint32_t kind, void* buf, uint64_t bytes, uint32_t line,
                     uint32_t passes, fhv_stream stream)
{
    if (!ctx || !buf || ((uintptr_t)buf & 15) || kind > FHV_PROBE_WRITE_CACHED) return FHV_EINVAL;
    if (kind == FHV_PROBE_COPY || kind == FHV_PROBE_COPY_CACHED) {
        if (bytes < 32 || bytes % 32 != 0) return FHV_EINVAL;
    } else if (kind == FHV_PROBE_READ || kind == FHV_PROBE_WRITE || kind == FHV_PROBE_READ_CACHED ||
               kind == FHV_PROBE_WRITE_CACHED) {
        if (bytes < 16 || bytes % 16 != 0) return FHV_EINVAL;
    } else {
        if (line < 8 || line > 4096 || (line & (line - 1)) || bytes < line) return FHV_EINVAL;
        if (passes < 1 || passes > 1024) return FHV_EINVAL;
    }
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::probe_launch(ctx->dev, kind, buf, bytes, line, passes, (hipStream_t)stream));
}

size_t fhv_capture_arrays_workspace(const fhv_capture_desc* desc, uint32_t n_tri, uint64_t capacity)
{
    if (!desc_ok(desc) || desc->mode != FHV_POFL || capacity == 0 || capacity >= 0xFFFFFFFFull) return 0;
    if (desc->projection == FHV_PROJ_AXES_1PASS && n_tri > 0x55555555u) return 0;
    return fhv::capture_arrays_ws_bytes(desc, n_tri, capacity);
}

fhv_status fhv_capture_arrays(fhv_ctx* ctx, const fhv_mesh* mesh, const fhv_capture_desc* desc,
                              const fhv_pofa* out, void* ws, size_t ws_bytes, fhv_stream stream)
{
    if (!ctx || !mesh || !desc_ok(desc) || !out || !ws) return FHV_EINVAL;
    if (desc->mode != FHV_POFL) return FHV_EINVAL;
    if (mesh->n_tri > 0 && (!mesh->pos || !mesh->rgba || !mesh->tri)) return FHV_EINVAL;
    if (!out->n_occ || !out->n_frag || !out->frag || !out->oct_key || !out->oct_off || !out->oct_cnt)
        return FHV_EINVAL;
    if (out->cap_frag == 0 || out->cap_frag >= 0xFFFFFFFFull || out->cap_occ == 0) return FHV_ERANGE;
    if ((uintptr_t)out->frag & 15) return FHV_EINVAL;
    if (desc->projection == FHV_PROJ_AXES_1PASS && mesh->n_tri > 0x55555555u) return FHV_ERANGE;
    if (ws_bytes < fhv::capture_arrays_ws_bytes(desc, mesh->n_tri, out->cap_frag)) return FHV_EWORKSPACE;
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::capture_arrays_launch(ctx->dev, mesh, desc, out, ws, (hipStream_t)stream));
}

fhv_status fhv_shade(fhv_ctx* ctx, const fhv_pofa* arrays, const uint64_t* zbuf, uint32_t n_views,
                     uint32_t width, uint32_t height, const fhv_light* lights, float* rgba, fhv_stream stream)
{
    if (!ctx || !arrays || !zbuf || !lights || !rgba) return FHV_EINVAL;
    if (n_views == 0 || n_views > fhv::kMaxViews) return FHV_ERANGE;
    if (width < 1 || width > 16384 || height < 1 || height > 16384) return FHV_ERANGE;
    if (arrays->cap_frag > 0 && !arrays->frag) return FHV_EINVAL;
    if (((uintptr_t)rgba & 15) || ((uintptr_t)zbuf & 7)) return FHV_EINVAL;
    fhv::ShadeArgs a;
    memset(&a, 0, sizeof(a));
    for (uint32_t v = 0; v < n_views; ++v) {
        if (lights[v].shine > 16) return FHV_EINVAL;
        for (int k = 0; k < 3; ++k) {
            a.l[v][k] = lights[v].l[k];
            a.v[v][k] = lights[v].v[k];
            a.h[v][k] = lights[v].h[k];
        }
        a.ka[v] = lights[v].ka;
        a.kd[v] = lights[v].kd;
        a.ks[v] = lights[v].ks;
        a.shine[v] = lights[v].shine;
    }
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::shade_launch(ctx->dev, arrays, zbuf, n_views, (uint64_t)width * height, a, rgba,
                                        (hipStream_t)stream));
}

size_t fhv_raycast_workspace(const fhv_capture_desc* desc)
{
    if (!desc_ok(desc) || desc->mode != FHV_POFL) return 0;
    return fhv::raycast_ws_bytes(desc->levels);
}

fhv_status fhv_raycast(fhv_ctx* ctx, const fhv_pofa* arrays, const fhv_capture_desc* desc,
                       const fhv_view* views, uint32_t n_views, uint32_t mode, float tau, float* rgba,
                       void* ws, size_t ws_bytes, fhv_stream stream)
{
    if (!ctx || !arrays || !desc_ok(desc) || !views || !rgba || !ws) return FHV_EINVAL;
    if (desc->mode != FHV_POFL || mode > FHV_RAY_BLEND || tau != tau) return FHV_EINVAL;
    if (desc->levels > fhv::kMaxRayLevels) return FHV_ERANGE;
    if (n_views == 0 || n_views > fhv::kMaxViews) return FHV_ERANGE;
    if (!arrays->n_occ) return FHV_EINVAL;
    if (arrays->cap_occ > 0 && (!arrays->oct_key || !arrays->oct_off || !arrays->oct_cnt)) return FHV_EINVAL;
    if (arrays->cap_frag > 0 && !arrays->frag) return FHV_EINVAL;
    if (arrays->cap_frag >= 0xFFFFFFFFull) return FHV_ERANGE;
    if (((uintptr_t)arrays->frag & 15) || ((uintptr_t)rgba & 15)) return FHV_EINVAL;
    fhv::RayViews rv;
    rv.n_views = n_views;
    rv.width = views[0].width;
    rv.height = views[0].height;
    if (rv.width < 1 || rv.width > 16384 || rv.height < 1 || rv.height > 16384) return FHV_ERANGE;
    for (uint32_t v = 0; v < n_views; ++v) {
        if (views[v].width != rv.width || views[v].height != rv.height) return FHV_EINVAL;
        if (views[v].splat_px != 1) return FHV_EINVAL;
        memcpy(rv.m[v], views[v].m, sizeof(rv.m[v]));
    }
    if (ws_bytes < fhv::raycast_ws_bytes(desc->levels)) return FHV_EWORKSPACE;
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::raycast_launch(ctx->dev, arrays, desc->levels, rv, mode, tau, rgba, ws,
                                          (hipStream_t)stream));
}

static bool fill_dims_ok(uint32_t levels, uint32_t n, uint32_t h, uint32_t w)
{
    if (levels < 1 || levels > 4 || n == 0 || h == 0 || w == 0) return false;
    const uint32_t m = 1u << (levels - 1);
    return h % m == 0 && w % m == 0;
}

uint64_t fhv_unet_param_count(uint32_t levels)
{
    if (levels < 1 || levels > 4) return 0;
    return fhv::nn::param_count(levels);
}

size_t fhv_fill_workspace(uint32_t levels, uint32_t n_img, uint32_t height, uint32_t width, int training)
{
    if (!fill_dims_ok(levels, n_img, height, width)) return 0;
    if ((uint64_t)n_img * height * width >= (1ull << 31)) return 0;
    if (training < FHV_FILL_INFER || training > FHV_FILL_TRACE) return 0;
    return fhv::nn::fill_ws_bytes(levels, n_img, height, width, training != FHV_FILL_INFER,
                                  training == FHV_FILL_TRACE);
}

uint32_t fhv_fill_trace_tensors(uint32_t levels, uint32_t n_img, uint32_t height, uint32_t width,
                                fhv_fill_tensor* out, uint32_t cap)
{
    if (!fill_dims_ok(levels, n_img, height, width)) return 0;
    if ((uint64_t)n_img * height * width >= (1ull << 31)) return 0;
    return fhv::nn::trace_tensors(levels, n_img, height, width, out, cap);
}

fhv_status fhv_fill(fhv_ctx* ctx, uint32_t levels, const float* params, const uint32_t* rgba,
                    const float* depth, const uint8_t* cov, uint32_t n_img, uint32_t height,
                    uint32_t width, uint32_t* out_rgba, float* out_residual, void* ws, size_t ws_bytes,
                    fhv_stream stream)
{
    if (!ctx || !params || !rgba || !depth || !cov || !out_rgba || !ws) return FHV_EINVAL;
    if (!fill_dims_ok(levels, n_img, height, width)) return FHV_EINVAL;
    if ((uint64_t)n_img * height * width >= (1ull << 31)) return FHV_ERANGE;
    if (ws_bytes < fhv::nn::fill_ws_bytes(levels, n_img, height, width, false)) return FHV_EWORKSPACE;
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::nn::fill(ctx->dev, levels, params, rgba, depth, cov, n_img, height, width, out_rgba,
                                    out_residual, ws, (hipStream_t)stream));
}

namespace {

fhv_status train_call(fhv_ctx* ctx, uint32_t levels, float* params, float* adam_m, float* adam_v, uint32_t step,
                      float lr, const uint32_t* rgba, const float* depth, const uint8_t* cov,
                      const uint32_t* target_rgba, uint32_t n_img, uint32_t height, uint32_t width, float* loss_out,
                      float* grad_out, void* ws, size_t ws_bytes, fhv_stream stream, bool trace)
{
    if (!ctx || !params || !rgba || !depth || !cov || !target_rgba || !ws) return FHV_EINVAL;
    if (step > 0 && (!adam_m || !adam_v)) return FHV_EINVAL;
    if (!fill_dims_ok(levels, n_img, height, width)) return FHV_EINVAL;
    if ((uint64_t)n_img * height * width >= (1ull << 31)) return FHV_ERANGE;
    if (ws_bytes < fhv::nn::fill_ws_bytes(levels, n_img, height, width, true, trace)) return FHV_EWORKSPACE;
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    return hip_status(fhv::nn::train_step(ctx->dev, levels, params, adam_m, adam_v, step, lr, rgba, depth, cov,
                                          target_rgba, n_img, height, width, loss_out, grad_out, ws,
                                          (hipStream_t)stream, trace));
}

}  // namespace

fhv_status fhv_fill_train_step(fhv_ctx* ctx, uint32_t levels, float* params, float* adam_m,
                               float* adam_v, uint32_t step, float lr, const uint32_t* rgba,
                               const float* depth, const uint8_t* cov, const uint32_t* target_rgba,
                               uint32_t n_img, uint32_t height, uint32_t width, float* loss_out,
                               float* grad_out, void* ws, size_t ws_bytes, fhv_stream stream)
{
    return train_call(ctx, levels, params, adam_m, adam_v, step, lr, rgba, depth, cov, target_rgba, n_img, height,
                      width, loss_out, grad_out, ws, ws_bytes, stream, false);
}

fhv_status fhv_fill_train_step_traced(fhv_ctx* ctx, uint32_t levels, float* params, float* adam_m,
                                      float* adam_v, uint32_t step, float lr, const uint32_t* rgba,
                                      const float* depth, const uint8_t* cov, const uint32_t* target_rgba,
                                      uint32_t n_img, uint32_t height, uint32_t width, float* loss_out,
                                      float* grad_out, void* ws, size_t ws_bytes, fhv_stream stream)
{
    return train_call(ctx, levels, params, adam_m, adam_v, step, lr, rgba, depth, cov, target_rgba, n_img, height,
                      width, loss_out, grad_out, ws, ws_bytes, stream, true);
}

fhv_status fhv_get_tuning(fhv_ctx* ctx, fhv_tuning* out)
{
    if (!ctx || !out) return FHV_EINVAL;
    out->tile_w = ctx->dev.tune.tile_w;
    out->raster_wg = ctx->dev.tune.raster_wg;
    out->splat_wg = ctx->dev.tune.splat_wg;
    return FHV_OK;
}

fhv_status fhv_set_tuning(fhv_ctx* ctx, const fhv_tuning* t)
{
    if (!ctx || !t) return FHV_EINVAL;
    if (t->tile_w != 8 && t->tile_w != 16 && t->tile_w != 32) return FHV_EINVAL;
    if (t->raster_wg < 1 || t->raster_wg > 64 || t->splat_wg < 1 || t->splat_wg > 64) return FHV_EINVAL;
    ctx->dev.tune.tile_w = t->tile_w;
    ctx->dev.tune.raster_wg = t->raster_wg;
    ctx->dev.tune.splat_wg = t->splat_wg;
    return FHV_OK;
}

size_t fhv_batch_workspace(const fhv_batch_mesh* mesh, const fhv_batch_views* views, uint64_t capacity)
{
    if (!batch_shape_ok(mesh, views) || capacity >= 0xFFFFFFFFull) return 0;
    if (!fhv::splat_fits(capacity, mesh->n_scenes, views->n_views, views->width, views->height)) return 0;
    return batch_ws(mesh, views, capacity, nullptr, nullptr, nullptr, nullptr);
}

fhv_status fhv_batch_run(fhv_ctx* ctx, const fhv_batch_mesh* mesh, const fhv_batch_views* views,
                         const fhv_lists* lists, const fhv_pofa* out, uint64_t* zbuf, uint32_t* rgba,
                         float* depth, uint8_t* cov, void* ws, size_t ws_bytes, uint32_t flags,
                         fhv_stream stream)
{
    if (!ctx || !batch_shape_ok(mesh, views) || !lists || !out) return FHV_EINVAL;
    if (flags & ~(FHV_BATCH_GRAPH | FHV_BATCH_TUNE)) return FHV_EINVAL;
    if (mesh->n_tri >= (1u << 31)) return FHV_ERANGE;
    if (mesh->n_tri > 0 && (!mesh->pos || !mesh->rgba || !mesh->tri || mesh->n_vert == 0)) return FHV_EINVAL;
    if (!mesh->scene_tri || !views->m) return FHV_EINVAL;
    const uint64_t n_head = (uint64_t)mesh->n_scenes << (3 * mesh->levels);
    if (lists->n_head != n_head) return FHV_EINVAL;
    if (!lists->counter || !lists->keys) return FHV_EINVAL;
    if (lists->capacity >= 0xFFFFFFFFull) return FHV_ERANGE;
    if (lists->capacity > 0 && !lists->pool) return FHV_EINVAL;
    if ((uintptr_t)lists->pool & 15) return FHV_EINVAL;
    if (!out->n_occ || !out->n_frag || out->cap_frag < lists->capacity) return FHV_EINVAL;
    if (lists->capacity > 0 && !out->frag) return FHV_EINVAL;
    if ((uintptr_t)out->frag & 15) return FHV_EINVAL;
    if (out->cap_occ > 0 && (!out->oct_key || !out->oct_off || !out->oct_cnt)) return FHV_EINVAL;
    if (!zbuf || !rgba || !depth || !cov || ((uintptr_t)zbuf & 15)) return FHV_EINVAL;
    if (!fhv::splat_fits(lists->capacity, mesh->n_scenes, views->n_views, views->width, views->height))
        return FHV_ERANGE;
    if (ws_bytes < batch_ws(mesh, views, lists->capacity, nullptr, nullptr, nullptr, nullptr)) return FHV_EWORKSPACE;
    if (!ws) return FHV_EINVAL;
    fhv_status st = set_device(ctx);
    if (st != FHV_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    BatchCall call{mesh, views, lists, out, zbuf, rgba, depth, cov, ws};
    if (flags & FHV_BATCH_TUNE) {
        if ((st = hip_status(batch_tune(ctx, call, s))) != FHV_OK) return st;
    }
    if (!(flags & FHV_BATCH_GRAPH)) return hip_status(batch_enqueue(ctx->dev, call, s));

    // graph: look up by every argument byte and the launch choices
    std::vector<unsigned char> key;
    auto put = [&key](const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        key.insert(key.end(), b, b + n);
    };
    put(mesh, sizeof(*mesh));
    put(views, sizeof(*views));
    put(lists, sizeof(*lists));
    put(out, sizeof(*out));
    const void* ptrs[5] = {zbuf, rgba, depth, cov, ws};
    put(ptrs, sizeof(ptrs));
    put(&ws_bytes, sizeof(ws_bytes));
    put(&ctx->dev.tune, sizeof(ctx->dev.tune));
    hipGraphExec_t exec = nullptr;
    for (auto& g : ctx->graphs)
        if (g.key == key) exec = g.exec;
    if (!exec) {
        hipError_t e = hipSuccess;
        if (!ctx->rec_stream) e = hipStreamCreateWithFlags(&ctx->rec_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_status(e);
        fhv::Device d = ctx->dev;
        d.prof = nullptr;   // no event records inside the graph
        e = hipStreamBeginCapture(ctx->rec_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_status(e);
        const hipError_t el = batch_enqueue(d, call, ctx->rec_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->rec_stream, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_status(el != hipSuccess ? el : e);
        }
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_status(e);
        if (ctx->graphs.size() >= 8) {
            (void)hipGraphExecDestroy(ctx->graphs.front().exec);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back({key, exec});
    }
    return hip_status(hipGraphLaunch(exec, s));
}

}  // extern "C"

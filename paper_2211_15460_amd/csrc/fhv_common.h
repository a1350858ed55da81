// Device-side definitions shared by the HIP translation units of libfhv.
// gfx950 (CDNA4) only: wave64, 64-bit atomics on global memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fhv.h"

namespace fhv {

constexpr uint32_t kNil = 0xFFFFFFFFu;
constexpr int kBlock = 256;          // threads per workgroup (4 waves)
constexpr int kWave = 64;
constexpr int kBrickShift = 9;       // compaction bucket: 512 consecutive keys
constexpr uint32_t kBrickKeys = 1u << kBrickShift;
constexpr uint32_t kMaxViews = 32;

// Triangle after setup: oriented counter-clockwise in 16.8 fixed point, with
// its sample bounding box and per-vertex integer attributes. 128 bytes.
struct alignas(16) TriRec {
    int32_t x[3], y[3];      // 16.8 screen (PPFL) or tangent-plane (POFL)
    int32_t lo_i, lo_j;      // first sample column / row
    int32_t hi_i, hi_j;      // last sample column / row (inclusive)
    uint32_t tiles_x;        // tiles per bbox row
    uint32_t nrm;            // packed normal
    uint32_t aux;            // object byte
    uint32_t scene;          // scene of a batch (key space offset scene << 3L)
    uint32_t rgba[3];
    uint32_t pad1;
    int32_t a[3][3];         // PPFL: a[k][0] = depth24; POFL: grid xyz
    int32_t pad2;
    int64_t A;               // twice the area, > 0
    double rA;               // 1 / A, for the quotient estimate
};
static_assert(sizeof(TriRec) == 128, "TriRec layout");

struct ViewArgs {
    float m[kMaxViews][12];
    float c[kMaxViews];       // 1/2 - k/2
    uint32_t k[kMaxViews];
    uint32_t n_views;
    uint32_t width;
    uint32_t height;
    uint32_t all_k1;        // every view has a one-pixel footprint
};

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t uniform32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    return (1ull << __lane_id()) - 1ull;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v |= (uint32_t)__shfl_xor((int)v, d, kWave);
    return v;
}

// Every active lane adds 1 to ctr[b]; lanes of the wave with equal b share
// one atomic add. Returns, per active lane, the counter's value before the
// add plus the lane's rank among the lanes sharing b (a unique slot).
// Must be called by all lanes of the wave.
template <bool kWantSlot>
__device__ __forceinline__ uint32_t wave_count_add(uint32_t* ctr, uint32_t b, bool active)
{
    const int lane = __lane_id();
    uint64_t todo = __ballot(active);
    uint32_t slot = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const uint32_t lb = (uint32_t)__shfl((int)b, leader, kWave);
        const uint64_t m = __ballot(active && b == lb) & todo;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(ctr + lb, (uint32_t)__popcll(m));
        if (kWantSlot) {
            base = (uint32_t)__shfl((int)base, leader, kWave);
            if ((m >> lane) & 1ull) slot = base + (uint32_t)__popcll(m & lanemask_lt());
        }
        todo &= ~m;
    }
    return slot;
}

// Per-brick histogram of keys (compaction buckets of kBrickKeys keys):
// every active lane adds 1 to brick_cnt[key >> kBrickShift] and sets the
// key's bit in `bitmap`. Lanes with the same brick or bitmap word share one
// atomic; no atomic's result is waited for (the number of distinct keys of a
// brick is the popcount of its bitmap words, taken afterwards).
// Must be called by all lanes of the wave.
__device__ __forceinline__ void wave_hist(uint64_t key, bool act, uint32_t* brick_cnt, uint32_t* bitmap)
{
    const int lane = __lane_id();
    wave_count_add<false>(brick_cnt, (uint32_t)(key >> kBrickShift), act);
    const uint64_t word = key >> 5;
    uint64_t todo = __ballot(act);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const uint64_t lw = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(word >> 32), leader, kWave) << 32) |
                            (uint32_t)__shfl((int)(uint32_t)word, leader, kWave);
        const uint64_t m = __ballot(act && word == lw) & todo;
        const uint32_t bits = wave_or(((m >> lane) & 1ull) ? (1u << (key & 31)) : 0u);
        if (lane == leader) atomicOr(bitmap + lw, bits);
        todo &= ~m;
    }
}

// Spread the low 21 bits of v to every third bit (bit b -> bit 3b).
__device__ __forceinline__ uint64_t spread3(uint32_t v32)
{
    uint64_t v = v32 & 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Inverse of spread3: every third bit of v (bit 3b -> bit b).
__device__ __forceinline__ uint32_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v | (v >> 2)) & 0x10C30C30C30C30C3ull;
    v = (v | (v >> 4)) & 0x100F00F00F00F00Full;
    v = (v | (v >> 8)) & 0x1F0000FF0000FFull;
    v = (v | (v >> 16)) & 0x1F00000000FFFFull;
    v = (v | (v >> 32)) & 0x1FFFFFull;
    return (uint32_t)v;
}

}  // namespace fhv

// Launchers (host side), defined next to their kernels.
namespace fhv {

struct Profiler;  // kernel timing with HIP events, owned by the context

// Launch choices (fhv_tuning): raster tile width (8, 16 or 32 samples; a
// tile is 64 samples), workgroups per compute unit of the rasterizer and of
// the splat.
struct Tuning {
    uint32_t tile_w = 8;
    uint32_t raster_wg = 16;
    uint32_t splat_wg = 16;
};

struct Device {
    int id;
    int cus;
    Profiler* prof;  // non-null while profiling is on
    Tuning tune;
};

void prof_mark(Profiler* p, const char* name, hipStream_t s, bool start);

// Brackets the kernel launches of one scope with events when profiling.
struct ProfScope {
    Profiler* p;
    const char* name;
    hipStream_t s;
    ProfScope(const Device& d, const char* n, hipStream_t st) : p(d.prof), name(n), s(st)
    {
        if (p) prof_mark(p, name, s, true);
    }
    ~ProfScope()
    {
        if (p) prof_mark(p, name, s, false);
    }
};

hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);

// Exclusive (or inclusive) prefix sums of n values; `partial` needs
// scan_partials(n) elements; *total (device, may be null) gets the sum.
size_t scan_partials(uint64_t n);
hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, bool inclusive,
                    uint32_t* partial, uint64_t* total, hipStream_t s);
hipError_t scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, bool inclusive,
                    uint64_t* partial, uint64_t* total, hipStream_t s);

// Scenes of a batch: triangle t belongs to the scene s with
// scene_tri[s] <= t < scene_tri[s + 1]; its keys are offset by s << 3L.
struct Scenes {
    const uint32_t* scene_tri;
    uint32_t n_scenes;
};

size_t capture_ws_bytes(const fhv_capture_desc* d, uint32_t n_tri);
hipError_t capture_launch(const Device& dev, const fhv_mesh* m, const fhv_capture_desc* d,
                          const fhv_lists* L, void* ws, hipStream_t s, const Scenes* sc = nullptr);

size_t compact_ws_bytes(const fhv_capture_desc* d, uint64_t n_head, uint64_t capacity);
hipError_t compact_launch(const Device& dev, const fhv_lists* L, const fhv_capture_desc* d,
                          const fhv_pofa* out, void* ws, hipStream_t s);

// Splat workspace for arrays of cap_frag records into n_scenes x n_views
// views of width x height.
size_t splat_ws_bytes(uint64_t cap_frag, uint32_t n_scenes, uint32_t n_views, uint32_t width, uint32_t height);
// Whether the splat's bins of such a call fit its 32-bit offsets.
bool splat_fits(uint64_t cap_frag, uint32_t n_scenes, uint32_t n_views, uint32_t width, uint32_t height);
hipError_t splat_launch(const Device& dev, const fhv_pofa* a, const fhv_capture_desc* d,
                        const ViewArgs& va, uint64_t* zbuf, uint32_t* rgba, float* depth,
                        uint8_t* cov, void* ws, hipStream_t s);

// Views of a batch: matrices [n_scenes][n_views][12] in device memory.
struct BatchViews {
    const float* m;
    uint32_t n_scenes, n_views, width, height, k;
};

hipError_t splat_batch_launch(const Device& dev, const fhv_pofa* a, uint32_t levels, const BatchViews& bv,
                              uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov, void* ws,
                              hipStream_t s);

// Two-pass capture straight into per-octant arrays (fhv_capture_arrays):
// the rasterizer counts fragments per brick (kActCount) or stores each at its
// brick's next free staging slot (kActInsert) instead of appending to lists.
enum RasterAct { kActList = 0, kActCount = 1, kActInsert = 2 };
struct BrickSink {
    uint32_t *cnt, *bitmap;         // kActCount: per-brick counts, key bitmap
    const uint32_t* off;            // kActInsert: brick offsets in the staging array
    uint32_t* cur;                  //             per-brick slot cursors (zeroed)
    uint4* stage;                   //             staging records, w3 = key within the brick
    const uint32_t* skip;           //             non-zero: the arrays are too small, store nothing
};
hipError_t capture_bricks_launch(const Device& dev, const fhv_mesh* m, const fhv_capture_desc* d, void* ws,
                                 int act, const BrickSink& bs, hipStream_t s);
size_t capture_arrays_ws_bytes(const fhv_capture_desc* d, uint32_t n_tri, uint64_t capacity);
hipError_t capture_arrays_launch(const Device& dev, const fhv_mesh* m, const fhv_capture_desc* d,
                                 const fhv_pofa* out, void* ws, hipStream_t s);

// Shading of splat winners (fhv_shade): per view the light, viewer and half
// vectors and the material terms.
struct ShadeArgs {
    float l[kMaxViews][3], v[kMaxViews][3], h[kMaxViews][3];
    float ka[kMaxViews], kd[kMaxViews], ks[kMaxViews];
    uint32_t shine[kMaxViews];
};
hipError_t shade_launch(const Device& dev, const fhv_pofa* p, const uint64_t* zbuf, uint32_t n_views,
                        uint64_t n_pix, const ShadeArgs& a, float* out, hipStream_t s);

// Ray casting of per-octant arrays (fhv_raycast): octree depth up to
// kMaxRayLevels (Morton codes of octants fit 32 bits).
constexpr uint32_t kMaxRayLevels = 10;
struct RayViews {
    float m[kMaxViews][12];
    uint32_t n_views, width, height;
};
size_t raycast_ws_bytes(uint32_t levels);
hipError_t raycast_launch(const Device& dev, const fhv_pofa* p, uint32_t levels, const RayViews& rv,
                          uint32_t mode, float tau, float* out, void* ws, hipStream_t s);

// Measurement probes (fhv_probe): copy over the buffer's two halves, or
// one atomic per line and pass.
hipError_t probe_launch(const Device& dev, uint32_t kind, void* buf, uint64_t bytes, uint32_t line,
                        uint32_t passes, hipStream_t s);

namespace nn {
uint64_t param_count(uint32_t levels);
size_t fill_ws_bytes(uint32_t levels, uint32_t N, uint32_t H, uint32_t W, bool training, bool trace = false);
uint32_t trace_tensors(uint32_t levels, uint32_t N, uint32_t H, uint32_t W, fhv_fill_tensor* out, uint32_t cap);
hipError_t fill(const Device& dev, uint32_t levels, const float* th, const uint32_t* rgba, const float* depth,
                const uint8_t* cov, uint32_t N, uint32_t H, uint32_t W, uint32_t* out, float* residual,
                void* ws, hipStream_t s);
hipError_t train_step(const Device& dev, uint32_t levels, float* th, float* m, float* v, uint32_t step,
                      float lr, const uint32_t* rgba, const float* depth, const uint8_t* cov,
                      const uint32_t* tgt, uint32_t N, uint32_t H, uint32_t W, float* loss, float* grad_out,
                      void* ws, hipStream_t s, bool trace);
}  // namespace nn

// Workspace carving with 256-byte alignment.
struct Carver {
    char* base;
    size_t off;
    template <class T>
    T* take(uint64_t n)
    {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += (size_t)n * sizeof(T);
        return p;
    }
};

}  // namespace fhv

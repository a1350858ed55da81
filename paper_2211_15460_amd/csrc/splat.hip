// Point splatting of per-octant arrays into novel views (Sec. 3.3): every
// fragment is projected, covers a k x k pixel square (at least one pixel),
// and per pixel the nearest fragment wins, as in deferred shading.
//
// Screen-tile ownership: every view is cut into tiles of 64 x 64 pixels and
// one workgroup owns a tile, holding its depth test in LDS, so no z-buffer
// entry is touched by more than one workgroup and no global atomic decides a
// pixel. The arrays are cut into chunks of 64 consecutive fragments (one per
// lane); in Morton order a chunk is a compact piece of surface, and so is a
// run of 64 consecutive chunks, and of 64 such runs, and so on: the bounding
// boxes of those runs form a tree over the arrays that a tile's workgroup
// walks to find the few chunks that can reach it, with no binning pass and
// no atomic on global memory.
//
//   k_chunk_box   one wave per chunk: the bounding box of its fragment
//                 positions (and the range of scenes its keys belong to)
//   k_node_box    one wave per node of the next level up: the union of its
//                 64 children's boxes, up to a single root
//   k_tile_est    a workgroup of 4 waves per tile: the tree walked down to
//                 the groups of chunks that can reach the tile, which set
//                 how many workgroups draw it (a busy tile is split into up
//                 to 16 sub-tiles) and the order of the draw: items listed
//                 in 8 classes of their share of groups, busiest first
//   k_tile_splat  one workgroup of 16 waves per tile or sub-tile: z-tile of 64-bit keys
//                 (fp32 depth bits << 32 | fragment index) in LDS, cleared;
//                 the tree walked from the root, each node's 64 children
//                 tested at once (one per lane) by projecting the child's box
//                 into the view with a margin that covers the fp32 rounding
//                 of every fragment inside it; every chunk that can reach the
//                 tile projected fragment by fragment (fp32 3x4 transform
//                 without fused multiply-adds) with an LDS 64-bit minimum for
//                 each footprint pixel inside the (sub-)tile; then each pixel
//                 of it written once: key, winner's colour (w1), depth and
//                 coverage
//
// A batch (many scenes in one key space, key = scene << 3L | Morton code)
// runs the same kernels over (scene, view) slots; a fragment only draws into
// the views of its own scene, and the matrices are read from device memory.
#include <math.h>
#include <string.h>

#include "fhv_common.h"

namespace fhv {

namespace {

constexpr int kChunk = kWave;       // fragments per chunk, one per lane
constexpr int kTile = 64;           // tile side in pixels
constexpr int kTilePix = kTile * kTile;

// Position of array fragment r in the view's input space: PPFL
// (px + 1/2, py + 1/2, depth24), POFL grid position + 1/2.
template <int kMode>
__device__ __forceinline__ void frag_pos(const uint4& r, uint64_t key, uint32_t cap_w, float* x,
                                         float* y, float* z)
{
    if (kMode == FHV_PPFL) {
        const uint32_t px = (uint32_t)(key % cap_w), py = (uint32_t)(key / cap_w);
        *x = (float)px + 0.5f;
        *y = (float)py + 0.5f;
        *z = (float)(r.x & 0xFFFFFFu);
    } else {
        const uint32_t kx = compact3(key >> 2), ky = compact3(key >> 1), kz = compact3(key);
        *x = (float)((kx << 8) | (r.x & 0xFFu)) + 0.5f;
        *y = (float)((ky << 8) | ((r.x >> 8) & 0xFFu)) + 0.5f;
        *z = (float)((kz << 8) | ((r.x >> 16) & 0xFFu)) + 0.5f;
    }
}

// What every kernel needs to know about the call.
struct TileArgs {
    uint32_t n_scenes;     // 1 for fhv_splat
    uint32_t n_views;      // views per scene
    uint32_t width, height;
    uint32_t nx, ny;       // tiles per row and per column of a view
    uint32_t per_view;     // nx * ny
    uint32_t n_tiles;      // n_scenes * n_views * per_view
    uint32_t shift;        // batches: scene = key >> shift; else 64 (no scene bits)
    uint32_t cap_w;        // PPFL capture width (pixel keys)
    uint64_t cap_frag, cap_occ;
    // chunk tree: levels (level 0 = chunks, the last = the root), where each
    // level's boxes start (in nodes), nodes of all levels for cap_frag
    uint32_t levels;
    uint64_t lv_off[8];
    uint64_t n_nodes;
    uint32_t gbits;        // POFL: bits per grid coordinate (octree depth + 8)
};

// Matrix, footprint side and offset 1/2 - k/2 of view slot g (scene g / V,
// view g % V): from the kernel arguments (one scene) or, for a batch, from
// device memory [scene][view][12] with one footprint for all views.
template <bool kBatch>
struct ViewSrc {
    const ViewArgs& va;
    const float* vm;
    __device__ __forceinline__ const float* m(uint32_t g) const
    {
        return kBatch ? vm + 12ull * g : va.m[g];
    }
    __device__ __forceinline__ uint32_t k(uint32_t g) const { return kBatch ? va.k[0] : va.k[g]; }
    __device__ __forceinline__ float c(uint32_t g) const { return kBatch ? va.c[0] : va.c[g]; }
};

// Inclusive pixel rectangle; empty when x0 > x1.
struct PixRect {
    int32_t x0, y0, x1, y1;
};

// Pixels that the footprint of any fragment in the box [lo, hi] can reach
// in a view, in fp32. Each row of the matrix taken over the box has its
// smallest and largest values at m3 plus, per axis, the smaller and the
// larger of the products with the box's two bounds; B (per axis the larger
// absolute product, plus |m3|) bounds the sum of the absolute terms at any
// point of the box. A fragment's fp32 projection differs from the exact
// value at its position by less than 2^-21 B, the fp32 evaluation here
// (four products and sums) by less than 2^-22 B, and the rounding of the
// shifted bounds below by less than 2^-24 (B + |c| + 1): the margin
// 2^-20 (B + |c| + 1) covers all three. A matrix or box that is not finite
// reaches the whole view; a box whose depth is <= 0 everywhere reaches
// nothing (such fragments are not drawn).
__device__ PixRect chunk_rect(const float* M, float c, uint32_t k, uint32_t W, uint32_t H, float4 lo, float4 hi)
{
    PixRect r{1, 1, 0, 0};
    if (!(lo.x <= hi.x)) return r;   // no drawable fragment
    const float l3[3] = {lo.x, lo.y, lo.z}, h3[3] = {hi.x, hi.y, hi.z};
    float smin[3], smax[3], B[3];
#pragma unroll
    for (int row = 0; row < 3; ++row) {
        const float m3 = M[4 * row + 3];
        float mn = m3, mx = m3, b = fabsf(m3);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float m = M[4 * row + a];
            const float p = m * l3[a], q = m * h3[a];
            mn += fminf(p, q);
            mx += fmaxf(p, q);
            b += fmaxf(fabsf(p), fabsf(q));
        }
        smin[row] = mn;
        smax[row] = mx;
        B[row] = b;
    }
    const float eps = 0x1p-20f;
    bool finite = true;
#pragma unroll
    for (int row = 0; row < 3; ++row) finite = finite && isfinite(smin[row]) && isfinite(smax[row]) && isfinite(B[row]);
    if (!finite) return PixRect{0, 0, (int32_t)W - 1, (int32_t)H - 1};
    if (smax[2] + eps * (B[2] + 1.0f) <= 0.0f) return r;
    const float mx = eps * (B[0] + fabsf(c) + 1.0f), my = eps * (B[1] + fabsf(c) + 1.0f);
    const float fx0 = floorf(smin[0] - mx + c), fx1 = floorf(smax[0] + mx + c) + (float)(k - 1);
    const float fy0 = floorf(smin[1] - my + c), fy1 = floorf(smax[1] + my + c) + (float)(k - 1);
    if (!(fx1 >= 0.0f && fy1 >= 0.0f && fx0 <= (float)W - 1.0f && fy0 <= (float)H - 1.0f)) return r;
    r.x0 = fx0 < 0.0f ? 0 : (int32_t)fx0;
    r.y0 = fy0 < 0.0f ? 0 : (int32_t)fy0;
    r.x1 = fx1 > (float)W - 1.0f ? (int32_t)W - 1 : (int32_t)fx1;
    r.y1 = fy1 > (float)H - 1.0f ? (int32_t)H - 1 : (int32_t)fy1;
    return r;
}

__device__ __forceinline__ float wave_fmin(float v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v = fminf(v, __shfl_xor(v, d, kWave));
    return v;
}

__device__ __forceinline__ float wave_fmax(float v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v = fmaxf(v, __shfl_xor(v, d, kWave));
    return v;
}

__device__ __forceinline__ uint32_t wave_umin(uint32_t v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, d, kWave);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_umax(uint32_t v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, d, kWave);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t frag_total(const uint64_t* n_frag, uint64_t cap)
{
    const uint64_t nf = *n_frag;
    return nf < cap ? nf : cap;
}

// The chunk tree: level 0 holds the chunks' boxes, every node of level
// l + 1 the union of the boxes of its kFan children (nodes kFan n .. kFan n
// + kFan - 1 of level l), up to a single root. Boxes are pairs (low, high)
// of float4 with the scene range in w (as uint bits: lowest scene in the
// low corner, highest in the high one); an empty box has low > high.
constexpr int kFan = kWave;
constexpr int kMaxLevels = 8;

// Nodes of each level for F fragments, into n[0 .. levels).
__device__ __forceinline__ void level_counts(uint64_t F, uint32_t levels, uint32_t* n)
{
    uint64_t c = (F + kChunk - 1) / kChunk;
    for (uint32_t l = 0; l < levels; ++l) {
        n[l] = (uint32_t)c;
        c = (c + kFan - 1) / kFan;
    }
}

// Packed position of a fragment for the tile kernel: bit 63 set when the
// fragment is drawn at all; POFL: grid x, y, z (gbits each) and the scene
// above them; PPFL: pixel x, y (14 bits each) and depth24.
template <int kMode>
__device__ __forceinline__ uint64_t pack_pos(const uint4& r, uint64_t key, uint32_t scene, bool ok, const TileArgs& ta)
{
    if (!ok) return 0;
    if (kMode == FHV_PPFL) {
        const uint64_t px = key % ta.cap_w, py = key / ta.cap_w;
        return (1ull << 63) | px | (py << 14) | ((uint64_t)(r.x & 0xFFFFFFu) << 28);
    }
    const uint32_t S = ta.gbits;
    const uint64_t kx = compact3(key >> 2), ky = compact3(key >> 1), kz = compact3(key);
    const uint64_t gx = (kx << 8) | (r.x & 0xFFu), gy = (ky << 8) | ((r.x >> 8) & 0xFFu),
                   gz = (kz << 8) | ((r.x >> 16) & 0xFFu);
    return (1ull << 63) | gx | (gy << S) | (gz << (2 * S)) | ((uint64_t)scene << (3 * S));
}

template <int kMode, bool kBatch>
__global__ void __launch_bounds__(kBlock)
k_chunk_box(const uint4* __restrict__ frag, const uint64_t* __restrict__ oct_key, const uint64_t* __restrict__ n_frag,
            TileArgs ta, float4* __restrict__ box, uint64_t* __restrict__ pos, uint32_t* __restrict__ bucket)
{
    if (blockIdx.x == 0 && threadIdx.x < 9) bucket[threadIdx.x] = 0;   // the tile pass's item counters, anew
    if (ta.cap_occ == 0) return;   // no table rows: nothing to draw
    const uint64_t F = frag_total(n_frag, ta.cap_frag);
    const uint64_t nch = (F + kChunk - 1) / kChunk;
    const int lane = __lane_id();
    const uint64_t n_waves = (uint64_t)gridDim.x * (kBlock / kWave);
    const uint64_t kmask = ta.shift >= 64 ? ~0ull : (1ull << ta.shift) - 1ull;
    for (uint64_t ch = uniform64((uint64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave); ch < nch;
         ch += n_waves) {
        const uint64_t f = ch * kChunk + lane;
        bool ok = f < F;
        const uint4 r = ok ? frag[f] : make_uint4(0, 0, 0, 0);
        ok = ok && r.w < ta.cap_occ;
        const uint64_t key = oct_key[ok ? r.w : 0];
        const uint32_t scene = ta.shift >= 64 ? 0u : (uint32_t)(key >> ta.shift);
        ok = ok && scene < ta.n_scenes;
        float x, y, z;
        frag_pos<kMode>(r, key & kmask, ta.cap_w, &x, &y, &z);
        pos[f] = pack_pos<kMode>(r, key & kmask, scene, ok, ta);
        float4 lo, hi;
        lo.x = wave_fmin(ok ? x : INFINITY);
        lo.y = wave_fmin(ok ? y : INFINITY);
        lo.z = wave_fmin(ok ? z : INFINITY);
        hi.x = wave_fmax(ok ? x : -INFINITY);
        hi.y = wave_fmax(ok ? y : -INFINITY);
        hi.z = wave_fmax(ok ? z : -INFINITY);
        lo.w = __uint_as_float(wave_umin(ok ? scene : 0xFFFFFFFFu));
        hi.w = __uint_as_float(wave_umax(ok ? scene : 0u));
        if (lane == 0) {
            box[2 * ch] = lo;
            box[2 * ch + 1] = hi;
        }
    }
}

// Boxes of level l (its nodes' children are on level l - 1): one wave per
// node, one lane per child.
__global__ void __launch_bounds__(kBlock)
k_node_box(const uint64_t* __restrict__ n_frag, TileArgs ta, uint32_t l, float4* __restrict__ box)
{
    if (ta.cap_occ == 0) return;
    uint32_t n[kMaxLevels];
    level_counts(frag_total(n_frag, ta.cap_frag), ta.levels, n);
    const int lane = __lane_id();
    const uint64_t n_waves = (uint64_t)gridDim.x * (kBlock / kWave);
    const float4* src = box + 2 * ta.lv_off[l - 1];
    float4* dst = box + 2 * ta.lv_off[l];
    for (uint64_t node = uniform64((uint64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave); node < n[l];
         node += n_waves) {
        const uint64_t c = node * kFan + lane;
        const bool ok = c < n[l - 1];
        const float4 a = ok ? src[2 * c] : make_float4(INFINITY, INFINITY, INFINITY, __uint_as_float(0xFFFFFFFFu));
        const float4 b = ok ? src[2 * c + 1] : make_float4(-INFINITY, -INFINITY, -INFINITY, __uint_as_float(0u));
        float4 lo, hi;
        lo.x = wave_fmin(a.x);
        lo.y = wave_fmin(a.y);
        lo.z = wave_fmin(a.z);
        hi.x = wave_fmax(b.x);
        hi.y = wave_fmax(b.y);
        hi.z = wave_fmax(b.z);
        lo.w = __uint_as_float(wave_umin(__float_as_uint(a.w)));
        hi.w = __uint_as_float(wave_umax(__float_as_uint(b.w)));
        if (lane == 0) {
            dst[2 * node] = lo;
            dst[2 * node + 1] = hi;
        }
    }
}

// Workgroup order: consecutive workgroups go to the 8 accelerator dies in
// turn, so that the tiles of one die form one contiguous run of tile indices
// (neighbouring tiles share chunks, which then meet in that die's cache).
__device__ __forceinline__ uint32_t die_major(uint32_t b, uint32_t n)
{
    const uint32_t q = n / 8, r = n % 8, x = b % 8, j = b / 8;
    return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

constexpr int kTileWaves = 16;                 // waves per tile workgroup
constexpr int kTileThreads = kTileWaves * kWave;
constexpr uint32_t kFront = 2048;              // breadth-first frontier capacity (node ids)
// Ordering and splitting the tiles: a tile whose walk reaches n groups of
// chunks is drawn by P workgroups, ceil(n / kSplitGroups) rounded up to a
// power of two (at most kMaxParts), each on a sub-tile of 64 x 64 / P
// pixels (square or twice as wide as tall: fewer chunks straddle two
// sub-tiles than narrow column strips), with at most kMaxItems workgroups beyond one per tile per launch; the workgroups
// start in decreasing order of their share of groups (8 classes), the
// busiest first. Launches of 2^22 tiles or more keep one workgroup per tile
// in the plain order.
constexpr uint32_t kSplitGroups = 64, kMaxParts = 16, kMaxItems = 4096, kOrderTiles = 1u << 22;
constexpr int kEstWaves = 4;                   // waves per workgroup of the estimate pass
// A tile whose walk ends on at most kGroupList groups of chunks gets them
// listed by the estimate pass, and its workgroup in the tile pass starts
// from that list instead of walking the tree again.
constexpr uint32_t kGroupList = 32;

// What one tile's workgroup knows about its view.
struct TileView {
    float M[12];
    float c;
    int32_t k;
    uint32_t scene;
    int32_t X0, Y0;
    int32_t XS, XE;   // the sub-tile this workgroup draws: columns [XS, XE),
    int32_t YS, YE;   // rows [YS, YE), within the tile
};

// Workgroups beyond one per tile: up to kMaxItems; none when the tiles are
// not ordered.
__host__ __device__ __forceinline__ uint32_t split_items(uint32_t n_tiles)
{
    if (n_tiles >= kOrderTiles) return 0;
    const uint32_t m = 2 * ((n_tiles + 7) / 8 * 8);
    return m < kMaxItems ? m : kMaxItems;
}

// Which of the kFan children of node `node` (on level l, children on level
// l - 1) can reach the tile: a bit per lane.
template <bool kBatch>
__device__ __forceinline__ uint64_t test_children(const float4* __restrict__ box, const TileArgs& ta,
                                                  const uint32_t* nl, uint32_t l, uint32_t node, const TileView& tv)
{
    const uint64_t c = (uint64_t)node * kFan + __lane_id();
    bool ok = c < nl[l - 1];
    float4 lo = make_float4(1.f, 0.f, 0.f, 0.f), hi = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok) {
        const float4* b = box + 2 * (ta.lv_off[l - 1] + c);
        lo = b[0];
        hi = b[1];
    }
    if (kBatch) ok = ok && __float_as_uint(lo.w) <= tv.scene && tv.scene <= __float_as_uint(hi.w);
    if (ok) {
        const PixRect r = chunk_rect(tv.M, tv.c, (uint32_t)tv.k, ta.width, ta.height, lo, hi);
        ok = r.x0 <= r.x1 && r.y0 <= r.y1 && r.x1 >= tv.XS && r.x0 < tv.XE && r.y1 >= tv.YS && r.y0 < tv.YE;
    }
    return __ballot(ok);
}

// The lanes' fragments (packed position p, array index f) drawn into the
// z-tile.
template <int kMode, bool kBatch>
__device__ __forceinline__ void draw_pos(uint64_t p, uint64_t f, const TileArgs& ta, const TileView& tv,
                                         unsigned long long* zt)
{
    bool ok = (p >> 63) != 0;
    float x, y, z;
    if (kMode == FHV_PPFL) {
        x = (float)(uint32_t)(p & 0x3FFFu) + 0.5f;
        y = (float)(uint32_t)((p >> 14) & 0x3FFFu) + 0.5f;
        z = (float)(uint32_t)((p >> 28) & 0xFFFFFFu);
    } else {
        const uint32_t S = ta.gbits;
        const uint64_t gm = (1ull << S) - 1ull;
        x = (float)(uint32_t)(p & gm) + 0.5f;
        y = (float)(uint32_t)((p >> S) & gm) + 0.5f;
        z = (float)(uint32_t)((p >> (2 * S)) & gm) + 0.5f;
        if (kBatch) ok = ok && (uint32_t)((p & ~(1ull << 63)) >> (3 * S)) == tv.scene;
    }
    const float* M = tv.M;
    const float sx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
    const float sy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
    const float d = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
    if (!ok || !(d > 0.0f)) return;
    const float fx = floorf(sx + tv.c), fy = floorf(sy + tv.c);
    const unsigned long long zk = ((unsigned long long)__float_as_uint(d) << 32) | (unsigned long long)(uint32_t)f;
    const int32_t k = tv.k, X0 = tv.X0, Y0 = tv.Y0;
    if (k == 1) {
        if (fx >= 0.0f && fx < (float)ta.width && fy >= 0.0f && fy < (float)ta.height) {
            const int32_t px = (int32_t)fx - X0, py = (int32_t)fy - Y0;
            if ((uint32_t)((int32_t)fx - tv.XS) < (uint32_t)(tv.XE - tv.XS) &&
                (uint32_t)((int32_t)fy - tv.YS) < (uint32_t)(tv.YE - tv.YS))
                atomicMin(zt + py * kTile + px, zk);
        }
        return;
    }
    if (!(fx > -1073741824.0f && fx < 1073741824.0f)) return;
    if (!(fy > -1073741824.0f && fy < 1073741824.0f)) return;
    int32_t xa = (int32_t)fx, ya = (int32_t)fy;
    int32_t xb = xa + k, yb = ya + k;   // exclusive
    xa = xa < tv.XS ? tv.XS : xa;
    ya = ya < tv.YS ? tv.YS : ya;
    const int32_t xe = tv.XE < (int32_t)ta.width ? tv.XE : (int32_t)ta.width;
    const int32_t ye = tv.YE < (int32_t)ta.height ? tv.YE : (int32_t)ta.height;
    xb = xb > xe ? xe : xb;
    yb = yb > ye ? ye : yb;
    for (int32_t yy = ya; yy < yb; ++yy)
        for (int32_t xx = xa; xx < xb; ++xx) atomicMin(zt + (yy - Y0) * kTile + (xx - X0), zk);
}

// The chunks q[i] (or base + i when q is null), i = i0, i0 + step, ... < n,
// drawn in batches of kDrawBatch, the next batch's positions loading while
// the current batch is drawn (so that up to 2 kDrawBatch loads of a wave
// are in flight). Chunks beyond the arrays' end hold positions that are not
// drawn.
constexpr int kDrawBatch = 4;

template <int kMode, bool kBatch>
__device__ __forceinline__ void draw_queue(const uint32_t* q, uint64_t base, uint32_t i0, uint32_t step, uint32_t n,
                                           const uint64_t* __restrict__ pos, const TileArgs& ta, const TileView& tv,
                                           unsigned long long* zt)
{
    if (i0 >= n) return;
    const int lane = __lane_id();
    // chunk ids fit 32 bits (fewer than 2^32 chunks per launch)
    auto chunk = [&](uint32_t i) -> uint32_t { return q ? q[i] : (uint32_t)base + i; };
    uint32_t ca[kDrawBatch];
    uint64_t pa[kDrawBatch];
#pragma unroll
    for (int j = 0; j < kDrawBatch; ++j) {
        const uint32_t i = i0 + (uint32_t)j * step;
        ca[j] = i < n ? chunk(i) : 0;
        pa[j] = i < n ? pos[(uint64_t)ca[j] * kChunk + lane] : 0;
    }
    for (uint32_t ib = i0; ib < n; ib += kDrawBatch * step) {
        uint32_t cb[kDrawBatch];
        uint64_t pb[kDrawBatch];
#pragma unroll
        for (int j = 0; j < kDrawBatch; ++j) {
            const uint32_t i = ib + (uint32_t)(kDrawBatch + j) * step;
            cb[j] = i < n ? chunk(i) : 0;
            pb[j] = i < n ? pos[(uint64_t)cb[j] * kChunk + lane] : 0;
        }
#pragma unroll
        for (int j = 0; j < kDrawBatch; ++j)
            if (ib + (uint32_t)j * step < n)
                draw_pos<kMode, kBatch>(pa[j], (uint64_t)ca[j] * kChunk + lane, ta, tv, zt);
#pragma unroll
        for (int j = 0; j < kDrawBatch; ++j) {
            ca[j] = cb[j];
            pa[j] = pb[j];
        }
    }
}

// The view of tile `tile` (slot g = tile / per_view) for the walk and the draw.
template <bool kBatch>
__device__ __forceinline__ TileView tile_view(uint32_t tile, const TileArgs& ta, const ViewArgs& va, const float* vm,
                                              bool drawn, uint32_t part = 0, uint32_t n_parts = 1)
{
    const uint32_t g = tile / ta.per_view, t = tile % ta.per_view;
    TileView tv;
    tv.X0 = (int32_t)((t % ta.nx) * kTile);
    tv.Y0 = (int32_t)((t / ta.nx) * kTile);
    // n_parts (a power of two up to 16) square or 2:1 sub-tiles: 2 x 1,
    // 2 x 2, 4 x 2, 4 x 4 (columns x rows), numbered along the rows
    const uint32_t lg = 31u - (uint32_t)__builtin_clz(n_parts | 1u);
    const uint32_t cols = 1u << ((lg + 1) >> 1), rows = n_parts >> ((lg + 1) >> 1);
    tv.XS = tv.X0 + (int32_t)((part % cols) * (kTile / cols));
    tv.XE = tv.XS + (int32_t)(kTile / cols);
    tv.YS = tv.Y0 + (int32_t)((part / cols) * (kTile / rows));
    tv.YE = tv.YS + (int32_t)(kTile / rows);
    tv.scene = g / ta.n_views;
    if (drawn) {
        const ViewSrc<kBatch> vs{va, vm};
#pragma unroll
        for (int q = 0; q < 12; ++q) tv.M[q] = vs.m(g)[q];
        tv.c = vs.c(g);
        tv.k = (int32_t)vs.k(g);
    }
    return tv;
}

// Breadth-first walk of the chunk tree from the root (front[0][0]) by the
// workgroup's kWaves waves, children tested one per lane, down to the
// groups of chunks (level 1) that can reach the tile, or until a level's
// frontier does not fit kFront. Returns the level lv of the final frontier
// front[*cur] of *curn nodes (lv >= 2 when it stopped early).
template <bool kBatch, int kWaves>
__device__ __forceinline__ uint32_t walk_tree(const float4* __restrict__ box, const TileArgs& ta, const uint32_t* nl,
                                              const TileView& tv, uint32_t (*front)[kFront], uint32_t* sh_next,
                                              uint32_t* sh_over, uint32_t* cur, uint32_t* curn)
{
    const uint32_t wave = threadIdx.x / kWave;
    const int lane = __lane_id();
    uint32_t lv = ta.levels - 1, c = 0, n = 1;
    while (lv >= 2) {
        if (threadIdx.x == 0) {
            *sh_next = 0;
            *sh_over = 0;
        }
        __syncthreads();
        for (uint32_t e = wave; e < n; e += kWaves) {
            const uint32_t node = front[c][e];
            const uint64_t m = test_children<kBatch>(box, ta, nl, lv, node, tv);
            const uint32_t cnt = (uint32_t)__popcll(m);
            uint32_t base = 0;
            if (lane == 0 && cnt) base = atomicAdd(sh_next, cnt);
            base = uniform32((uint32_t)__shfl((int)base, 0, kWave));
            if ((m >> lane) & 1ull) {
                const uint32_t pos = base + (uint32_t)__popcll(m & lanemask_lt());
                if (pos < kFront) front[c ^ 1][pos] = node * kFan + (uint32_t)lane;
                else *sh_over = 1;
            }
        }
        __syncthreads();
        const uint32_t nn = *sh_next, over = *sh_over;
        __syncthreads();
        if (over) break;   // keep the current frontier; depth first from here
        c ^= 1;
        n = nn;
        --lv;
    }
    *cur = c;
    *curn = n;
    return lv;
}

// Estimate pass, one workgroup of kEstWaves waves per tile: the walk down to
// the groups of chunks that can reach the tile sets how many workgroups
// draw it (P, reserved from the launch's extra budget: counter[8]) and the
// class of their share of groups (0 for nothing to draw, then 1 + log2 of
// the share, at most 7). Its items (tile << 5 | part) go to its class's
// list, items[class * item_cap + rank ...] (counter[class] counts the
// class's items); parts[tile] = P | (1 + listed groups, or 0) << 8, the
// groups listed in glist[tile * kGroupList ...].
template <bool kBatch>
__global__ void __launch_bounds__(kEstWaves * kWave)
k_tile_est(const uint64_t* __restrict__ n_frag, TileArgs ta, ViewArgs va, const float* __restrict__ vm,
           const float4* __restrict__ box, uint32_t* __restrict__ items, uint32_t* __restrict__ parts,
           uint32_t* __restrict__ counter, uint32_t* __restrict__ glist)
{
    __shared__ uint32_t front[2][kFront];
    __shared__ uint32_t nl[kMaxLevels];
    __shared__ uint32_t sh_next, sh_over;
    const uint32_t tile = blockIdx.x;
    const uint64_t F = frag_total(n_frag, ta.cap_frag);
    const bool drawn = ta.cap_occ > 0 && F > 0;
    const TileView tv = tile_view<kBatch>(tile, ta, va, vm, drawn);
    if (threadIdx.x == 0) {
        uint32_t n[kMaxLevels];
        level_counts(F, ta.levels, n);
        for (uint32_t l = 0; l < ta.levels; ++l) nl[l] = n[l];
        front[0][0] = 0;
    }
    __syncthreads();
    uint32_t groups = 0;   // groups of chunks that can reach the tile (a large value when uncounted)
    uint32_t listed = 0;   // 1 + the number of groups listed for the tile, or 0: no list
    if (drawn) {
        uint32_t cur, curn;
        const uint32_t lv = walk_tree<kBatch, kEstWaves>(box, ta, nl, tv, front, &sh_next, &sh_over, &cur, &curn);
        groups = lv >= 2 ? 1u << 16 : (lv == 1 ? curn : 1);
        if (lv == 1 && curn <= kGroupList) {
            if (threadIdx.x < curn) glist[(size_t)tile * kGroupList + threadIdx.x] = front[cur][threadIdx.x];
            listed = curn + 1;
        }
    } else {
        listed = 1;   // nothing to draw: an empty list
    }
    if (threadIdx.x == 0) {
        const uint32_t q = (groups + kSplitGroups - 1) / kSplitGroups;
        uint32_t P = 1;
        while (P < q && P < kMaxParts) P *= 2;
        if (P > 1 && atomicAdd(counter + 8, P - 1) + (P - 1) > split_items(ta.n_tiles)) P = 1;
        const uint32_t share = (groups + P - 1) / P;
        const uint32_t cls = share == 0 ? 0u : (share >= 64 ? 7u : 32u - __builtin_clz(share));
        const uint32_t r = atomicAdd(counter + cls, P);
        uint32_t* it = items + (size_t)cls * (ta.n_tiles + split_items(ta.n_tiles)) + r;
        for (uint32_t i = 0; i < P; ++i) it[i] = (tile << 5) | i;
        parts[tile] = P | (listed << 8);
    }
}

// One workgroup per item: a 64 x 64 tile of one view slot, or a sub-tile
// of one (items in the estimate's order; one per tile, in the plain order,
// for launches of 2^22 tiles or more). The chunk tree is walked from the
// root breadth first (children tested one per lane) down to the groups of
// 64 chunks that can reach the workgroup's sub-tile; then, in rounds of one
// group per wave, the chunks of those groups that can reach it are queued
// in LDS and drawn by all waves in turn into the z-tile in LDS with 64-bit
// minima (fragments outside the sub-tile rejected). Should a level's
// frontier not fit in LDS, every chunk below the last frontier that did is
// drawn. Then each pixel of the sub-tile is written once.
template <int kMode, bool kBatch>
__global__ void __launch_bounds__(kTileThreads, 8)   // 8 waves per SIMD (two workgroups per compute unit): 64 registers
k_tile_splat(const uint4* __restrict__ frag, const uint64_t* __restrict__ pos, const uint64_t* __restrict__ n_frag,
             TileArgs ta, ViewArgs va, const float* __restrict__ vm, const float4* __restrict__ box,
             const uint32_t* __restrict__ parts, const uint32_t* __restrict__ items,
             const uint32_t* __restrict__ counter, const uint32_t* __restrict__ glist,
             unsigned long long* __restrict__ zbuf, uint32_t* __restrict__ rgba, float* __restrict__ depth,
             uint8_t* __restrict__ cov)
{
    __shared__ unsigned long long zt[kTilePix];
    __shared__ uint32_t front[2][kFront];
    __shared__ uint32_t queue[kTileWaves * kFan];
    __shared__ uint32_t nl[kMaxLevels];
    __shared__ uint32_t sh_next, sh_over, sh_q;
    uint32_t tile, part = 0, P = 1, listed = 0;
    if (ta.n_tiles < kOrderTiles) {
        // item blockIdx.x of the classes' lists taken from class 7 down
        uint32_t b = blockIdx.x, c = 8;
        for (;;) {
            if (c == 0) return;   // whole workgroup: past the last item
            --c;
            const uint32_t n = counter[c];
            if (b < n) break;
            b -= n;
        }
        const uint32_t it = items[(size_t)c * (ta.n_tiles + split_items(ta.n_tiles)) + b];
        tile = uniform32(it >> 5);
        part = uniform32(it & 31u);
        const uint32_t pw = uniform32(parts[tile]);
        P = pw & 0xFFu;
        listed = pw >> 8;
    } else {
        tile = uniform32(die_major(blockIdx.x, ta.n_tiles));
    }
    const uint64_t F = frag_total(n_frag, ta.cap_frag);
    const bool drawn = ta.cap_occ > 0 && F > 0;
    const TileView tv = tile_view<kBatch>(tile, ta, va, vm, drawn, part, P);
    for (int p = threadIdx.x; p < kTilePix; p += kTileThreads) zt[p] = ~0ull;
    if (threadIdx.x == 0) {
        uint32_t n[kMaxLevels];
        level_counts(F, ta.levels, n);
        for (uint32_t l = 0; l < ta.levels; ++l) nl[l] = n[l];
        front[0][0] = 0;   // the root
    }
    // the groups the estimate listed for the tile, as the walk's last frontier
    if (listed > 0 && threadIdx.x < listed - 1) front[0][threadIdx.x] = glist[(size_t)tile * kGroupList + threadIdx.x];
    __syncthreads();
    if (drawn) {
        const uint32_t wave = threadIdx.x / kWave;
        const int lane = __lane_id();
        uint32_t cur = 0, curn = listed > 0 ? listed - 1 : 0, lv = 1;
        if (listed == 0) lv = walk_tree<kBatch, kTileWaves>(box, ta, nl, tv, front, &sh_next, &sh_over, &cur, &curn);
        const uint32_t* fr = front[cur];
        if (lv <= 1) {
            // rounds: every wave tests one group's chunks and queues those
            // that can reach the tile (its sub-tile); all waves then
            // draw the queue
            for (uint32_t r0 = 0; r0 < curn; r0 += kTileWaves) {
                if (threadIdx.x == 0) sh_q = 0;
                __syncthreads();
                const uint32_t e = r0 + wave;
                if (e < curn) {
                    const uint32_t node = fr[e];
                    const uint64_t m = lv == 1 ? test_children<kBatch>(box, ta, nl, 1, node, tv) : 1ull;
                    const uint32_t cnt = (uint32_t)__popcll(m);
                    uint32_t base = 0;
                    if (lane == 0 && cnt) base = atomicAdd(&sh_q, cnt);
                    base = uniform32((uint32_t)__shfl((int)base, 0, kWave));
                    if ((m >> lane) & 1ull)
                        queue[base + (uint32_t)__popcll(m & lanemask_lt())] =
                            lv == 1 ? node * kFan + (uint32_t)lane : node;
                }
                __syncthreads();
                const uint32_t nq = sh_q;
                draw_queue<kMode, kBatch>(queue, 0, wave, kTileWaves, nq, pos, ta, tv, zt);
                __syncthreads();
            }
        } else {
            // a frontier too large for LDS (a tile that the whole scene
            // projects into): every chunk below each frontier node is drawn,
            // the fragments outside the tile rejected one by one
            for (uint32_t e = 0; e < curn; ++e) {
                uint64_t lo = fr[e];
                for (uint32_t l = 0; l < lv; ++l) lo *= kFan;
                const uint64_t span = lo + ((uint64_t)1 << (6 * lv)) < nl[0] ? (uint64_t)1 << (6 * lv) : nl[0] - lo;
                draw_queue<kMode, kBatch>(nullptr, lo, wave, kTileWaves, (uint32_t)span, pos, ta, tv, zt);
            }
        }
    }
    __syncthreads();
    const uint32_t g = tile / ta.per_view;
    const uint64_t plane = (uint64_t)ta.width * ta.height;
    const uint32_t* f32 = (const uint32_t*)frag;
    for (int p = threadIdx.x; p < kTilePix; p += kTileThreads) {
        const int32_t X = tv.X0 + (p % kTile), Y = tv.Y0 + (p / kTile);
        if (X < tv.XS || X >= tv.XE || Y < tv.YS || Y >= tv.YE || X >= (int32_t)ta.width || Y >= (int32_t)ta.height)
            continue;
        const uint64_t o = (uint64_t)g * plane + (uint64_t)Y * ta.width + (uint32_t)X;
        const unsigned long long zk = zt[p];
        zbuf[o] = zk;
        if (zk == ~0ull) {
            rgba[o] = 0u;
            depth[o] = 0.0f;
            cov[o] = 0;
        } else {
            rgba[o] = f32[4ull * (uint32_t)zk + 1];
            depth[o] = __uint_as_float((uint32_t)(zk >> 32));
            cov[o] = 1;
        }
    }
}

TileArgs tile_args(uint32_t n_scenes, uint32_t n_views, uint32_t W, uint32_t H, uint64_t cap_frag)
{
    TileArgs ta{};
    ta.n_scenes = n_scenes;
    ta.n_views = n_views;
    ta.width = W;
    ta.height = H;
    ta.nx = (W + kTile - 1) / kTile;
    ta.ny = (H + kTile - 1) / kTile;
    ta.per_view = ta.nx * ta.ny;
    ta.n_tiles = n_scenes * n_views * ta.per_view;
    ta.shift = 64;
    ta.cap_frag = cap_frag;
    // levels of the chunk tree for the largest fragment count, and where
    // each level's boxes start
    uint64_t c = (cap_frag + kChunk - 1) / kChunk, off = 0;
    if (c == 0) c = 1;
    ta.levels = 0;
    for (;;) {
        ta.lv_off[ta.levels++] = off;
        off += c;
        if (c == 1) break;
        c = (c + kFan - 1) / kFan;
    }
    ta.n_nodes = off;
    return ta;
}

// Workspace: the tree's boxes, then the packed positions (a whole number of
// chunks).
size_t tile_pos_off(const TileArgs& ta) { return ((size_t)ta.n_nodes * 2 * sizeof(float4) + 255) & ~(size_t)255; }

// Then, from tile_split_off: the parts of each tile, the items' lists of
// the 8 classes (each with room for all items), 9 counters, and for ordered
// launches kGroupList group ids per tile.
size_t tile_split_off(const TileArgs& ta)
{
    return (tile_pos_off(ta) + (size_t)((ta.cap_frag + kChunk - 1) / kChunk) * kChunk * sizeof(uint64_t) + 255) &
           ~(size_t)255;
}

size_t tile_ws_bytes(const TileArgs& ta)
{
    const size_t cap = ta.n_tiles < kOrderTiles ? (size_t)ta.n_tiles + split_items(ta.n_tiles) : 0;
    const size_t lists = cap ? (size_t)ta.n_tiles * kGroupList : 0;
    return tile_split_off(ta) + ((size_t)ta.n_tiles + 8 * cap + 9 + lists) * sizeof(uint32_t) + 256;
}

template <bool kBatch>
hipError_t tiles_launch(const Device& dev, const fhv_pofa* a, int mode, TileArgs ta, const ViewArgs& va,
                        const float* vm, void* ws, uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov,
                        hipStream_t s)
{
    char* base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    float4* box = (float4*)base;
    uint64_t* pos = (uint64_t*)(base + tile_pos_off(ta));
    uint32_t* parts = (uint32_t*)(base + tile_split_off(ta));
    uint32_t* items = parts + ta.n_tiles;
    const bool ordered = ta.n_tiles < kOrderTiles;
    uint32_t* bucket = items + (ordered ? 8 * ((size_t)ta.n_tiles + split_items(ta.n_tiles)) : 0);
    uint32_t* glist = bucket + 9;   // ordered launches only
    const uint64_t chunks = (a->cap_frag + kChunk - 1) / kChunk;
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    auto grid_for = [&](uint64_t waves) {
        uint64_t gb = (waves + (kBlock / kWave) - 1) / (kBlock / kWave);
        return (unsigned)(gb < 1 ? 1 : (gb > gmax ? gmax : gb));
    };
    hipError_t e;
    {
        ProfScope ps(dev, "splat.bin", s);
        if (mode == FHV_PPFL)
            k_chunk_box<FHV_PPFL, kBatch><<<dim3(grid_for(chunks)), dim3(kBlock), 0, s>>>(
                (const uint4*)a->frag, a->oct_key, a->n_frag, ta, box, pos, bucket);
        else
            k_chunk_box<FHV_POFL, kBatch><<<dim3(grid_for(chunks)), dim3(kBlock), 0, s>>>(
                (const uint4*)a->frag, a->oct_key, a->n_frag, ta, box, pos, bucket);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (uint32_t l = 1; l < ta.levels; ++l) {
            const uint64_t nodes = (l + 1 < ta.levels ? ta.lv_off[l + 1] : ta.n_nodes) - ta.lv_off[l];
            k_node_box<<<dim3(grid_for(nodes)), dim3(kBlock), 0, s>>>(a->n_frag, ta, l, box);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (ordered) {
        ProfScope ps(dev, "splat.est", s);
        k_tile_est<kBatch><<<dim3(ta.n_tiles), dim3(kEstWaves * kWave), 0, s>>>(a->n_frag, ta, va, vm, box, items,
                                                                                  parts, bucket, glist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    ProfScope ps(dev, "splat.splat", s);
    const dim3 grid(ta.n_tiles + split_items(ta.n_tiles));
    if (mode == FHV_PPFL)
        k_tile_splat<FHV_PPFL, kBatch><<<grid, dim3(kTileThreads), 0, s>>>(
            (const uint4*)a->frag, pos, a->n_frag, ta, va, vm, box, parts, items, bucket, glist,
            (unsigned long long*)zbuf, rgba, depth, cov);
    else
        k_tile_splat<FHV_POFL, kBatch><<<grid, dim3(kTileThreads), 0, s>>>(
            (const uint4*)a->frag, pos, a->n_frag, ta, va, vm, box, parts, items, bucket, glist,
            (unsigned long long*)zbuf, rgba, depth, cov);
    return hipGetLastError();
}

}  // namespace

bool splat_fits(uint64_t cap_frag, uint32_t n_scenes, uint32_t n_views, uint32_t width, uint32_t height)
{
    const uint64_t tiles = (uint64_t)n_scenes * n_views * ((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile);
    return tiles < (1ull << 31) && (cap_frag + kChunk - 1) / kChunk < (1ull << 32);
}

size_t splat_ws_bytes(uint64_t cap_frag, uint32_t n_scenes, uint32_t n_views, uint32_t width, uint32_t height)
{
    return tile_ws_bytes(tile_args(n_scenes, n_views, width, height, cap_frag));
}

hipError_t splat_launch(const Device& dev, const fhv_pofa* a, const fhv_capture_desc* d, const ViewArgs& va,
                        uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov, void* ws, hipStream_t s)
{
    TileArgs ta = tile_args(1, va.n_views, va.width, va.height, a->cap_frag);
    ta.cap_w = d->width;
    ta.cap_occ = a->cap_occ;
    ta.gbits = d->levels + 8;
    return tiles_launch<false>(dev, a, (int)d->mode, ta, va, nullptr, ws, zbuf, rgba, depth, cov, s);
}

hipError_t splat_batch_launch(const Device& dev, const fhv_pofa* a, uint32_t levels, const BatchViews& bv,
                              uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov, void* ws, hipStream_t s)
{
    TileArgs ta = tile_args(bv.n_scenes, bv.n_views, bv.width, bv.height, a->cap_frag);
    ta.shift = 3 * levels;
    ta.cap_occ = a->cap_occ;
    ta.gbits = levels + 8;
    ViewArgs va;
    memset(&va, 0, sizeof(va));
    va.n_views = bv.n_views;
    va.width = bv.width;
    va.height = bv.height;
    va.k[0] = bv.k;
    va.c[0] = 0.5f - 0.5f * (float)bv.k;
    return tiles_launch<true>(dev, a, FHV_POFL, ta, va, bv.m, ws, zbuf, rgba, depth, cov, s);
}

}  // namespace fhv

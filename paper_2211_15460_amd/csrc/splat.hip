// Point splatting of per-octant arrays into novel views (Sec. 3.3): every
// fragment is projected, covers a k x k pixel square (at least one pixel),
// and per pixel the nearest fragment wins, as in deferred shading.
//
// Screen-tile ownership: every view is cut into tiles of 64 x 64 pixels and
// one workgroup owns a tile, holding its depth test in LDS, so no z-buffer
// entry is touched by more than one workgroup and no global atomic decides a
// pixel. The arrays are cut into chunks of 64 consecutive fragments (one per
// lane); in Morton order a chunk is a compact piece of surface, and its
// positions' bounding box, projected into a view, names the few tiles the
// chunk can reach there.
//
//   k_tile_count  one wave per chunk: the bounding box of its fragment
//                 positions (and the range of scenes its keys belong to);
//                 per (scene, view) of the chunk, the pixel rectangle its
//                 footprints can reach (with a margin that covers the fp32
//                 rounding of every fragment inside the box); a rectangle
//                 over at most 4 tiles counts the chunk once in each tile's
//                 bin, a larger one once in the view's own bin
//   scan          bin offsets (bins: every tile, then every view)
//   k_tile_write  the same rectangles again; the chunk's index goes into
//                 each tile bin, or the chunk with its rectangle into the
//                 view bin
//   k_tile_splat  one workgroup per tile: z-tile of 64-bit keys (fp32 depth
//                 bits << 32 | fragment index) in LDS, cleared; every chunk of
//                 the tile's bin, and every chunk of the view's bin whose
//                 rectangle meets the tile, projected fragment by fragment
//                 (fp32 3x4 transform without fused multiply-adds) with an
//                 LDS 64-bit minimum for each footprint pixel inside the tile;
//                 then each pixel of the tile written once: key, winner's
//                 colour (w1), depth and coverage
//
// A batch (many scenes in one key space, key = scene << 3L | Morton code)
// runs the same kernels over (scene, view) slots; a fragment only draws into
// the views of its own scene, and the matrices are read from device memory.
#include <math.h>
#include <string.h>

#include "fhv_common.h"
#include "scan.h"

namespace fhv {

namespace {

constexpr int kChunk = kWave;       // fragments per chunk, one per lane
constexpr int kTile = 64;           // tile side in pixels
constexpr int kTilePix = kTile * kTile;
constexpr uint32_t kTileBinMax = 4; // larger rectangles go to the view's bin

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
    // capacities of the two lists; arrays in key order never reach them (a
    // write beyond is dropped, a read beyond is not made)
    uint32_t cap_t, cap_b;
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
// in a view. The box's corners are projected in fp64 (every product of two
// fp32 values is exact there); a fragment's fp32 projection differs from the
// exact value at its position by less than 2^-21 of the sum of the absolute
// terms, which is largest at a corner, so the margin 2^-20 (B + |c| + 1)
// covers it and the rounding of sx + c. A matrix or box that is not finite
// reaches the whole view; a box whose depth is <= 0 everywhere reaches
// nothing (such fragments are not drawn).
__device__ PixRect chunk_rect(const float* M, float c, uint32_t k, uint32_t W, uint32_t H, float4 lo, float4 hi)
{
    PixRect r{1, 1, 0, 0};
    if (!(lo.x <= hi.x)) return r;   // no drawable fragment
    double smin[3] = {INFINITY, INFINITY, INFINITY}, smax[3] = {-INFINITY, -INFINITY, -INFINITY};
    double B[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 8; ++q) {
        const double x = (q & 1) ? hi.x : lo.x, y = (q & 2) ? hi.y : lo.y, z = (q & 4) ? hi.z : lo.z;
        for (int row = 0; row < 3; ++row) {
            const double a0 = (double)M[4 * row] * x, a1 = (double)M[4 * row + 1] * y,
                         a2 = (double)M[4 * row + 2] * z, a3 = (double)M[4 * row + 3];
            const double sv = ((a0 + a1) + a2) + a3;
            const double b = ((fabs(a0) + fabs(a1)) + fabs(a2)) + fabs(a3);
            smin[row] = fmin(smin[row], sv);
            smax[row] = fmax(smax[row], sv);
            B[row] = fmax(B[row], b);
        }
    }
    const double eps = 0x1p-20;
    bool finite = true;
    for (int row = 0; row < 3; ++row) finite = finite && isfinite(smin[row]) && isfinite(smax[row]) && isfinite(B[row]);
    if (!finite) return PixRect{0, 0, (int32_t)W - 1, (int32_t)H - 1};
    if (smax[2] + eps * (B[2] + 1.0) <= 0.0) return r;
    const double cc = (double)c;
    const double mx = eps * (B[0] + fabs(cc) + 1.0), my = eps * (B[1] + fabs(cc) + 1.0);
    const double fx0 = floor(smin[0] - mx + cc), fx1 = floor(smax[0] + mx + cc) + (double)(k - 1);
    const double fy0 = floor(smin[1] - my + cc), fy1 = floor(smax[1] + my + cc) + (double)(k - 1);
    if (fx1 < 0.0 || fy1 < 0.0 || fx0 > (double)W - 1.0 || fy0 > (double)H - 1.0) return r;
    r.x0 = fx0 < 0.0 ? 0 : (int32_t)fx0;
    r.y0 = fy0 < 0.0 ? 0 : (int32_t)fy0;
    r.x1 = fx1 > (double)W - 1.0 ? (int32_t)W - 1 : (int32_t)fx1;
    r.y1 = fy1 > (double)H - 1.0 ? (int32_t)H - 1 : (int32_t)fy1;
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

// Binning of one chunk: `pass` 0 counts into cnt, pass 1 writes into the
// lists at the cursors. Lanes take the chunk's (scene, view) slots.
template <bool kBatch>
__device__ void bin_chunk(int pass, uint32_t ch, float4 lo, float4 hi, const TileArgs& ta, const ViewSrc<kBatch>& vs,
                          uint32_t* __restrict__ cnt, uint32_t* __restrict__ cur, uint32_t* __restrict__ list_t,
                          uint4* __restrict__ list_b, const uint32_t* __restrict__ off)
{
    if (!(lo.x <= hi.x)) return;
    const uint32_t s_lo = __float_as_uint(lo.w), s_hi = __float_as_uint(hi.w);
    const uint32_t n_pairs = (s_hi - s_lo + 1) * ta.n_views;
    for (uint32_t p = __lane_id(); p < n_pairs; p += kWave) {
        const uint32_t g = (s_lo + p / ta.n_views) * ta.n_views + p % ta.n_views;
        const PixRect r = chunk_rect(vs.m(g), vs.c(g), vs.k(g), ta.width, ta.height, lo, hi);
        if (r.x0 > r.x1 || r.y0 > r.y1) continue;
        const uint32_t tx0 = (uint32_t)r.x0 / kTile, tx1 = (uint32_t)r.x1 / kTile;
        const uint32_t ty0 = (uint32_t)r.y0 / kTile, ty1 = (uint32_t)r.y1 / kTile;
        const uint32_t n = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
        if (n <= kTileBinMax) {
            for (uint32_t ty = ty0; ty <= ty1; ++ty)
                for (uint32_t tx = tx0; tx <= tx1; ++tx) {
                    const uint32_t b = g * ta.per_view + ty * ta.nx + tx;
                    if (pass == 0) {
                        atomicAdd(cnt + b, 1u);
                    } else {
                        const uint32_t at = atomicAdd(cur + b, 1u);
                        if (at < ta.cap_t) list_t[at] = ch;
                    }
                }
        } else {
            const uint32_t b = ta.n_tiles + g;
            if (pass == 0) {
                atomicAdd(cnt + b, 1u);
            } else {
                const uint32_t at = atomicAdd(cur + b, 1u) - off[ta.n_tiles];
                if (at < ta.cap_b)
                    list_b[at] = make_uint4(ch, (uint32_t)r.x0 | ((uint32_t)r.y0 << 16),
                                            (uint32_t)r.x1 | ((uint32_t)r.y1 << 16), 0u);
            }
        }
    }
}

template <int kMode, bool kBatch>
__global__ void __launch_bounds__(kBlock)
k_tile_count(const uint4* __restrict__ frag, const uint64_t* __restrict__ oct_key, const uint64_t* __restrict__ n_frag,
             TileArgs ta, ViewArgs va, const float* __restrict__ vm, float4* __restrict__ box,
             uint32_t* __restrict__ cnt)
{
    if (ta.cap_occ == 0) return;   // no table rows: nothing to draw
    const uint64_t F = frag_total(n_frag, ta.cap_frag);
    const uint64_t nch = (F + kChunk - 1) / kChunk;
    const int lane = __lane_id();
    const uint64_t n_waves = (uint64_t)gridDim.x * (kBlock / kWave);
    const ViewSrc<kBatch> vs{va, vm};
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
        bin_chunk<kBatch>(0, (uint32_t)ch, lo, hi, ta, vs, cnt, nullptr, nullptr, nullptr, nullptr);
    }
}

template <bool kBatch>
__global__ void __launch_bounds__(kBlock)
k_tile_write(const uint64_t* __restrict__ n_frag, TileArgs ta, ViewArgs va, const float* __restrict__ vm,
             const float4* __restrict__ box, uint32_t* __restrict__ cur, const uint32_t* __restrict__ off,
             uint32_t* __restrict__ list_t, uint4* __restrict__ list_b)
{
    if (ta.cap_occ == 0) return;
    const uint64_t F = frag_total(n_frag, ta.cap_frag);
    const uint64_t nch = (F + kChunk - 1) / kChunk;
    const uint64_t n_waves = (uint64_t)gridDim.x * (kBlock / kWave);
    const ViewSrc<kBatch> vs{va, vm};
    for (uint64_t ch = uniform64((uint64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave); ch < nch;
         ch += n_waves)
        bin_chunk<kBatch>(1, (uint32_t)ch, box[2 * ch], box[2 * ch + 1], ta, vs, nullptr, cur, list_t, list_b, off);
}

// Bin offsets: off[b] = sum of the counts of bins before b; the write pass's
// cursors start there.
struct StoreBinOff {
    uint32_t* off;
    uint32_t* cur;
    __device__ void operator()(uint64_t i, uint32_t, uint32_t ex) const
    {
        off[i] = ex;
        cur[i] = ex;
    }
};

// Workgroup order: consecutive workgroups go to the 8 accelerator dies in
// turn, so that the tiles of one die form one contiguous run of tile indices
// (neighbouring tiles share chunks, which then meet in that die's cache).
__device__ __forceinline__ uint32_t die_major(uint32_t b, uint32_t n)
{
    const uint32_t q = n / 8, r = n % 8, x = b % 8, j = b / 8;
    return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// The lanes' fragments of chunk ch, drawn into the z-tile at (X0, Y0) of
// view slot g of scene `scene`.
template <int kMode, bool kBatch>
__device__ __forceinline__ void tile_chunk(uint32_t ch, uint64_t F, const uint4* __restrict__ frag,
                                           const uint64_t* __restrict__ oct_key, const TileArgs& ta, const float* M,
                                           float c, int32_t k, uint32_t scene, int32_t X0, int32_t Y0,
                                           unsigned long long* zt)
{
    const uint64_t kmask = ta.shift >= 64 ? ~0ull : (1ull << ta.shift) - 1ull;
    const uint64_t f = (uint64_t)ch * kChunk + __lane_id();
    bool ok = f < F;
    const uint4 r = ok ? frag[f] : make_uint4(0, 0, 0, 0);
    ok = ok && r.w < ta.cap_occ;
    const uint64_t key = oct_key[ok ? r.w : 0];
    if (kBatch) ok = ok && (uint32_t)(key >> ta.shift) == scene;
    float x, y, z;
    frag_pos<kMode>(r, key & kmask, ta.cap_w, &x, &y, &z);
    const float sx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
    const float sy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
    const float d = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
    if (!ok || !(d > 0.0f)) return;
    const float fx = floorf(sx + c), fy = floorf(sy + c);
    const unsigned long long zk = ((unsigned long long)__float_as_uint(d) << 32) | (unsigned long long)(uint32_t)f;
    if (k == 1) {
        if (fx >= 0.0f && fx < (float)ta.width && fy >= 0.0f && fy < (float)ta.height) {
            const int32_t px = (int32_t)fx - X0, py = (int32_t)fy - Y0;
            if ((uint32_t)px < (uint32_t)kTile && (uint32_t)py < (uint32_t)kTile)
                atomicMin(zt + py * kTile + px, zk);
        }
        return;
    }
    if (!(fx > -1073741824.0f && fx < 1073741824.0f)) return;
    if (!(fy > -1073741824.0f && fy < 1073741824.0f)) return;
    int32_t xa = (int32_t)fx, ya = (int32_t)fy;
    int32_t xb = xa + k, yb = ya + k;   // exclusive
    xa = xa < X0 ? X0 : xa;
    ya = ya < Y0 ? Y0 : ya;
    const int32_t xe = X0 + kTile < (int32_t)ta.width ? X0 + kTile : (int32_t)ta.width;
    const int32_t ye = Y0 + kTile < (int32_t)ta.height ? Y0 + kTile : (int32_t)ta.height;
    xb = xb > xe ? xe : xb;
    yb = yb > ye ? ye : yb;
    for (int32_t yy = ya; yy < yb; ++yy)
        for (int32_t xx = xa; xx < xb; ++xx) atomicMin(zt + (yy - Y0) * kTile + (xx - X0), zk);
}

template <int kMode, bool kBatch>
__global__ void __launch_bounds__(kBlock)
k_tile_splat(const uint4* __restrict__ frag, const uint64_t* __restrict__ oct_key, const uint64_t* __restrict__ n_frag,
             TileArgs ta, ViewArgs va, const float* __restrict__ vm, const uint32_t* __restrict__ off,
             const uint32_t* __restrict__ list_t, const uint4* __restrict__ list_b,
             unsigned long long* __restrict__ zbuf, uint32_t* __restrict__ rgba, float* __restrict__ depth,
             uint8_t* __restrict__ cov)
{
    __shared__ unsigned long long zt[kTilePix];
    const uint32_t tile = uniform32(die_major(blockIdx.x, gridDim.x));
    const uint32_t g = tile / ta.per_view, t = tile % ta.per_view;
    const int32_t X0 = (int32_t)((t % ta.nx) * kTile), Y0 = (int32_t)((t / ta.nx) * kTile);
    const uint32_t scene = g / ta.n_views;
    for (int p = threadIdx.x; p < kTilePix; p += kBlock) zt[p] = ~0ull;
    __syncthreads();
    if (ta.cap_occ > 0) {
        const uint64_t F = frag_total(n_frag, ta.cap_frag);
        const ViewSrc<kBatch> vs{va, vm};
        float M[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) M[q] = vs.m(g)[q];
        const float c = vs.c(g);
        const int32_t k = (int32_t)vs.k(g);
        const uint32_t wave = threadIdx.x / kWave;
        const uint32_t e0 = off[tile], e1 = off[tile + 1] < ta.cap_t ? off[tile + 1] : ta.cap_t;
        for (uint32_t e = e0 + wave; e < e1; e += kBlock / kWave)
            tile_chunk<kMode, kBatch>(uniform32(list_t[e]), F, frag, oct_key, ta, M, c, k, scene, X0, Y0, zt);
        const uint32_t base = off[ta.n_tiles];
        const uint32_t b0 = off[ta.n_tiles + g] - base;
        const uint32_t b1 = off[ta.n_tiles + g + 1] - base < ta.cap_b ? off[ta.n_tiles + g + 1] - base : ta.cap_b;
        for (uint32_t e = b0 + wave; e < b1; e += kBlock / kWave) {
            const uint4 be = list_b[e];
            const int32_t rx0 = (int32_t)(be.y & 0xFFFFu), ry0 = (int32_t)(be.y >> 16);
            const int32_t rx1 = (int32_t)(be.z & 0xFFFFu), ry1 = (int32_t)(be.z >> 16);
            if (rx1 < X0 || rx0 >= X0 + kTile || ry1 < Y0 || ry0 >= Y0 + kTile) continue;   // wave-uniform
            tile_chunk<kMode, kBatch>(uniform32(be.x), F, frag, oct_key, ta, M, c, k, scene, X0, Y0, zt);
        }
    }
    __syncthreads();
    const uint64_t plane = (uint64_t)ta.width * ta.height;
    const uint32_t* f32 = (const uint32_t*)frag;
    for (int p = threadIdx.x; p < kTilePix; p += kBlock) {
        const int32_t X = X0 + (p % kTile), Y = Y0 + (p / kTile);
        if (X >= (int32_t)ta.width || Y >= (int32_t)ta.height) continue;
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

// Workspace of the tiled splat.
struct TileWs {
    float4* box;       // [2 * chunks]: low and high corner, scene range in w
    uint32_t* cnt;     // [bins + 1] counts
    uint32_t* cur;     // [bins + 1] write cursors
    uint32_t* off;     // [bins + 1] exclusive offsets
    uint32_t* list_t;  // tile bins: chunk indices
    uint4* list_b;     // view bins: chunk, rectangle
    uint32_t* part;    // scan scratch
};

TileArgs tile_args(uint32_t n_scenes, uint32_t n_views, uint32_t W, uint32_t H)
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
    return ta;
}

// Bound on the (chunk, view slot) pairs: a chunk's slots are the views of
// the scenes its fragments belong to, and each scene boundary adds at most
// one scene to one chunk.
uint64_t pair_bound(uint64_t cap_frag, uint32_t n_scenes, uint32_t n_views)
{
    const uint64_t chunks = (cap_frag + kChunk - 1) / kChunk;
    return (chunks + n_scenes) * n_views;
}

TileWs carve_tiles(void* ws, uint64_t cap_frag, const TileArgs& ta, size_t* bytes)
{
    const uint64_t chunks = (cap_frag + kChunk - 1) / kChunk;
    const uint64_t bins = (uint64_t)ta.n_tiles + (uint64_t)ta.n_scenes * ta.n_views;
    const uint64_t pairs = pair_bound(cap_frag, ta.n_scenes, ta.n_views);
    Carver c{(char*)ws, 0};
    TileWs w;
    w.box = c.take<float4>(2 * chunks + 2);
    w.cnt = c.take<uint32_t>(bins + 1);
    w.cur = c.take<uint32_t>(bins + 1);
    w.off = c.take<uint32_t>(bins + 1);
    w.list_t = c.take<uint32_t>(kTileBinMax * pairs + 1);
    w.list_b = c.take<uint4>(pairs + 1);
    w.part = c.take<uint32_t>(scan_scratch(bins + 1));
    if (bytes) *bytes = c.off + 256;
    return w;
}

template <bool kBatch>
hipError_t tiles_launch(const Device& dev, const fhv_pofa* a, int mode, TileArgs ta, const ViewArgs& va,
                        const float* vm, void* ws, uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov,
                        hipStream_t s)
{
    const TileWs w = carve_tiles(ws, a->cap_frag, ta, nullptr);
    const uint64_t pairs = pair_bound(a->cap_frag, ta.n_scenes, ta.n_views);
    ta.cap_t = (uint32_t)(kTileBinMax * pairs);
    ta.cap_b = (uint32_t)pairs;
    const uint64_t bins = (uint64_t)ta.n_tiles + (uint64_t)ta.n_scenes * ta.n_views;
    const uint64_t chunks = (a->cap_frag + kChunk - 1) / kChunk;
    uint64_t gb = (chunks + (kBlock / kWave) - 1) / (kBlock / kWave);
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    gb = gb < 1 ? 1 : (gb > gmax ? gmax : gb);
    hipError_t e;
    {
        ProfScope ps(dev, "splat.bin", s);
        e = fill_u32(w.cnt, bins + 1, 0u, s);
        if (e != hipSuccess) return e;
        if (mode == FHV_PPFL)
            k_tile_count<FHV_PPFL, kBatch><<<dim3((unsigned)gb), dim3(kBlock), 0, s>>>(
                (const uint4*)a->frag, a->oct_key, a->n_frag, ta, va, vm, w.box, w.cnt);
        else
            k_tile_count<FHV_POFL, kBatch><<<dim3((unsigned)gb), dim3(kBlock), 0, s>>>(
                (const uint4*)a->frag, a->oct_key, a->n_frag, ta, va, vm, w.box, w.cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        e = scan<uint32_t>(LoadArray<uint32_t>{w.cnt}, StoreBinOff{w.off, w.cur}, bins + 1, w.part,
                           (uint32_t*)nullptr, s);
        if (e != hipSuccess) return e;
        k_tile_write<kBatch><<<dim3((unsigned)gb), dim3(kBlock), 0, s>>>(a->n_frag, ta, va, vm, w.box, w.cur, w.off,
                                                                       w.list_t, w.list_b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    ProfScope ps(dev, "splat.splat", s);
    if (mode == FHV_PPFL)
        k_tile_splat<FHV_PPFL, kBatch><<<dim3(ta.n_tiles), dim3(kBlock), 0, s>>>(
            (const uint4*)a->frag, a->oct_key, a->n_frag, ta, va, vm, w.off, w.list_t, w.list_b,
            (unsigned long long*)zbuf, rgba, depth, cov);
    else
        k_tile_splat<FHV_POFL, kBatch><<<dim3(ta.n_tiles), dim3(kBlock), 0, s>>>(
            (const uint4*)a->frag, a->oct_key, a->n_frag, ta, va, vm, w.off, w.list_t, w.list_b,
            (unsigned long long*)zbuf, rgba, depth, cov);
    return hipGetLastError();
}

}  // namespace

bool splat_fits(uint64_t cap_frag, uint32_t n_scenes, uint32_t n_views, uint32_t width, uint32_t height)
{
    const uint64_t tiles = (uint64_t)n_scenes * n_views * ((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile);
    const uint64_t bins = tiles + (uint64_t)n_scenes * n_views + 1;
    const uint64_t entries = (kTileBinMax + 1) * pair_bound(cap_frag, n_scenes, n_views);
    return tiles < (1ull << 31) && bins < (1ull << 31) && entries < (1ull << 32) &&
           (cap_frag + kChunk - 1) / kChunk < (1ull << 32);
}

size_t splat_ws_bytes(uint64_t cap_frag, uint32_t n_scenes, uint32_t n_views, uint32_t width, uint32_t height)
{
    size_t b = 0;
    carve_tiles(nullptr, cap_frag, tile_args(n_scenes, n_views, width, height), &b);
    return b;
}

hipError_t splat_launch(const Device& dev, const fhv_pofa* a, const fhv_capture_desc* d, const ViewArgs& va,
                        uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov, void* ws, hipStream_t s)
{
    TileArgs ta = tile_args(1, va.n_views, va.width, va.height);
    ta.cap_w = d->width;
    ta.cap_frag = a->cap_frag;
    ta.cap_occ = a->cap_occ;
    return tiles_launch<false>(dev, a, (int)d->mode, ta, va, nullptr, ws, zbuf, rgba, depth, cov, s);
}

hipError_t splat_batch_launch(const Device& dev, const fhv_pofa* a, uint32_t levels, const BatchViews& bv,
                              uint64_t* zbuf, uint32_t* rgba, float* depth, uint8_t* cov, void* ws, hipStream_t s)
{
    TileArgs ta = tile_args(bv.n_scenes, bv.n_views, bv.width, bv.height);
    ta.shift = 3 * levels;
    ta.cap_frag = a->cap_frag;
    ta.cap_occ = a->cap_occ;
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

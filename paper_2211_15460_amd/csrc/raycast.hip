// Ray casting of per-octant arrays (Sec. 3.3, evaluation by ray casting).
//
// The occupancy of every octree level is rebuilt from the table of occupied
// leaves (Sec. 3.1: coarser levels hold only the occupancy of their
// children, for empty-space skipping). Then one wave per 8 x 8 pixel tile
// walks the octree from the root (every decision of the walk is uniform
// across the wave), descending only into occupied children whose box can
// project into the tile, down to bricks of 4^3 or 8^3 leaves; a brick's
// fragments are one contiguous range of the arrays, tested one per lane and
// handed to the lane owning the pixel they land in. With an orthographic
// view the ray of a pixel meets a fragment when the fragment projects into
// that pixel (the one-pixel footprint of the splat).
//
// Children are visited nearest first (one order per view). Each lane keeps
// the fragments met for its pixel in a list ordered by (depth bits, index)
// and composites them front to back as soon as no unvisited octant can hold
// a nearer one; a lane is final when its transmittance falls below the
// threshold, and the walk ends when every lane of the tile is final. An
// octant is skipped when its depth range lies behind every compositing
// lane's list, or in front of what earlier walks composited; when a list
// overflows, the walk is repeated for the fragments behind the last one
// composited.
//
//   k_occ_build   one thread per table row: the row's leaf bit and, where
//                 the row is the first of its parent octant, the bits of its
//                 ancestors (rows are in Morton order, so a parent's first
//                 row sets it once)
//   k_raycast     one wave per 8 x 8 pixel tile, one lane per pixel
//
// Workspace: level l (1 <= l <= L) has a bitmap of 8^l bits in Morton order
// (the 8 children of octant n of level l-1 are byte n of level l's bitmap);
// the leaf level has, per 64-bit word, the number of set bits before it,
// which turns a leaf's Morton code into its table row.
#include "fhv_common.h"
#include "scan.h"

namespace fhv {

namespace {

constexpr int kCap = 16;   // fragments a lane keeps per walk

struct OccLayout {
    uint64_t word[kMaxRayLevels + 2];   // u32 offset of level l's bitmap, l = 1..L; [L+1] = end
    uint64_t n64;                       // 64-bit words of the leaf bitmap
};

OccLayout occ_layout(uint32_t L)
{
    OccLayout o{};
    uint64_t w = 0;
    for (uint32_t l = 1; l <= L; ++l) {
        o.word[l] = w;
        const uint64_t bits = 1ull << (3 * l);
        uint64_t words = (bits + 31) / 32;
        words = (words + 1) & ~1ull;   // 8-byte aligned levels
        w += words;
    }
    o.word[L + 1] = w;
    o.n64 = ((1ull << (3 * L)) + 63) / 64;
    return o;
}

__global__ void __launch_bounds__(kBlock)
k_occ_build(const uint64_t* __restrict__ oct_key, const uint64_t* __restrict__ n_occ, uint64_t cap_occ,
            uint32_t* __restrict__ occ, OccLayout lay, uint32_t L)
{
    const uint64_t n = *n_occ < cap_occ ? *n_occ : cap_occ;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += stride) {
        const uint64_t key = oct_key[r];
        const uint64_t prev = r > 0 ? oct_key[r - 1] : ~0ull;
        for (uint32_t l = L; l >= 1; --l) {
            const uint32_t sh = 3 * (L - l);
            const uint64_t b = key >> sh;
            if (l < L && r > 0 && (prev >> sh) == b) break;   // set by an earlier row
            atomicOr(occ + lay.word[l] + (b >> 5), 1u << (b & 31));
        }
    }
}

struct LoadPopc {
    const uint64_t* bits;
    __device__ uint32_t operator()(uint64_t i) const { return (uint32_t)__popcll(bits[i]); }
};

struct RayArgs {
    float m[kMaxViews][12];
    const uint4* frag;
    const uint64_t* oct_key;
    const uint32_t* oct_off;
    const uint32_t* oct_cnt;
    const uint32_t* occ;
    const uint32_t* rank;   // set leaf bits before each 64-bit word
    OccLayout lay;
    float4* out;            // [V][H][W]
    uint32_t order[kMaxViews];   // per view: child octants nearest first, 4 bits each
    uint32_t L, width, height, tiles_x, n_tiles;
    float tau;
};

__device__ __forceinline__ float proj(const float* M, int row, float x, float y, float z)
{
    return ((M[4 * row + 0] * x + M[4 * row + 1] * y) + M[4 * row + 2] * z) + M[4 * row + 3];
}

__device__ __forceinline__ float wave_max(float x)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x = fmaxf(x, __shfl_xor(x, d, kWave));
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x)));
}

__device__ __forceinline__ float wave_min(float x)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x = fminf(x, __shfl_xor(x, d, kWave));
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x)));
}

// One wave per 8 x 8 pixel tile: the wave walks the octree once for the
// tile (its window is the tile, so every decision of the walk is uniform),
// projects a leaf's fragments one per lane and hands each fragment that
// lands in the tile to the lane owning its pixel. Per lane: the pixel's
// kept fragments, compositing state and depth window; the walk skips an
// octant only when it is outside the window of every lane still compositing.
template <int kMode>
__global__ void __launch_bounds__(kBlock) k_raycast(RayArgs a)
{
    // per-lane fragment list, interleaved so that lanes hit distinct banks
    __shared__ uint64_t lst[(kMode == 0 ? 1 : kCap) * kBlock];
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    const uint32_t tile = blockIdx.x * (kBlock / kWave) + wv;
    if (tile >= a.n_tiles) return;   // whole wave
    const uint32_t x0 = (tile % a.tiles_x) * 8, y0 = (tile / a.tiles_x) * 8;
    const uint32_t px = x0 + (lane & 7), py = y0 + (lane >> 3);
    const bool mine = px < a.width && py < a.height;
    const uint32_t v = blockIdx.y;
    const float* M = a.m[v];
    const uint32_t L = a.L;
    const float tcx = (float)x0 + 4.0f, tcy = (float)y0 + 4.0f;
    constexpr float kWin = 4.0f + 0.0625f;     // half the tile, and room for rounding
    constexpr float kDepthSlack = 1e-5f;       // depth rounding, far below a leaf's depth extent
    const float ax = fabsf(M[0]) + fabsf(M[1]) + fabsf(M[2]), ay = fabsf(M[4]) + fabsf(M[5]) + fabsf(M[6]);
    const float az = fabsf(M[8]) + fabsf(M[9]) + fabsf(M[10]);
    const uint8_t* const occ8 = (const uint8_t*)a.occ;
    const uint64_t* const leaf64 = (const uint64_t*)(a.occ + a.lay.word[L]);
    uint64_t* const my = lst + threadIdx.x;
    const uint32_t order = a.order[v];
    const uint32_t my_c = (order >> (4 * (lane & 7))) & 7u;   // lanes 0..7 test child rank `lane`
    // the walk stops at bricks of 8^kBrick leaves (level B), whose fragments
    // are one contiguous range of the arrays: larger bricks trade fragment
    // tests, done 64 at a time, for fewer dependent loads along the walk
    // (measured best: 512 leaves for the nearest fragment, 64 with
    // transparency, where the walk stops earlier)
    constexpr uint32_t kBrick = kMode == 0 ? 3u : 2u;
    const uint32_t B = L > kBrick ? L - kBrick : 1;
    const uint64_t n_leaf = 1ull << (3 * L);
    // table rows of the leaves before Morton code k (k <= 8^L)
    auto rank_of = [&](uint64_t k) -> uint32_t {
        if (k >= n_leaf) return a.rank[a.lay.n64 - 1] + (uint32_t)__popcll(leaf64[a.lay.n64 - 1]);
        return a.rank[k >> 6] + (uint32_t)__popcll(leaf64[k >> 6] & ((1ull << (k & 63)) - 1ull));
    };

    // children of octant n (level l, origin o in leaves) that are occupied and
    // whose box can project into the tile; bit i stands for the i-th nearest
    // child of the view's order
    auto expand = [&](uint32_t l, uint32_t n, uint32_t ox, uint32_t oy, uint32_t oz) -> uint32_t {
        const uint32_t m = occ8[a.lay.word[l + 1] * 4 + n];
        const uint32_t hc = 1u << (L - l - 1);            // child side in leaves
        const float hw = (float)hc * 128.0f;              // half side in grid units
        const float X = (float)((ox + ((my_c >> 2) & 1u) * hc) * 256u) + hw;
        const float Y = (float)((oy + ((my_c >> 1) & 1u) * hc) * 256u) + hw;
        const float Z = (float)((oz + (my_c & 1u) * hc) * 256u) + hw;
        const float sx = proj(M, 0, X, Y, Z), sy = proj(M, 1, X, Y, Z);
        const bool ok = lane < 8 && ((m >> my_c) & 1u) && fabsf(sx - tcx) <= hw * ax + kWin &&
                        fabsf(sy - tcy) <= hw * ay + kWin;
        return (uint32_t)__ballot(ok) & 0xFFu;
    };

    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
    uint64_t after = 0;     // keys at or below this were composited
    bool walked = false;    // this lane composited in an earlier walk
    bool fin = !mine;       // this lane's pixel is final
    // composite one fragment (front to back); true when the pixel is final
    auto blend = [&](uint64_t key) -> bool {
        const uint32_t rgba = a.frag[(uint32_t)key].y;
        const float al = kMode == 0 ? 1.0f : (float)(rgba >> 24) / 255.0f;
        const float wgt = T * al;
        C0 = C0 + wgt * ((float)(rgba & 0xFFu) / 255.0f);
        C1 = C1 + wgt * ((float)((rgba >> 8) & 0xFFu) / 255.0f);
        C2 = C2 + wgt * ((float)((rgba >> 16) & 0xFFu) / 255.0f);
        T = T * (1.0f - al);
        after = key;
        walked = true;
        return T < a.tau || T == 0.0f;
    };
    for (;;) {
        // the lane's kept fragments are my[h .. n_in), ascending and below
        // `cut`: once a fragment is left out of a walk (list full, or its
        // octant skipped), no key at or above it may be kept in that walk,
        // so that what is composited stays in order. Depths beyond `far`
        // cannot enter the list; depths before `near` were composited.
        uint32_t h = 0, n_in = 0;
        bool over = false;
        uint64_t cut = ~0ull;
        float far = INFINITY;
        const float near = walked ? __uint_as_float((uint32_t)(after >> 32)) : -INFINITY;
        float wfar = wave_max(fin ? -INFINITY : far);
        const float wnear = wave_min(fin ? INFINITY : near);
        constexpr uint32_t cap = kMode == 0 ? 1u : (uint32_t)kCap;
        auto set_far = [&]() {
            float f = cut == ~0ull ? INFINITY : __uint_as_float((uint32_t)(cut >> 32));
            if (n_in - h == cap) f = fminf(f, __uint_as_float((uint32_t)(my[(n_in - 1) * kBlock] >> 32)));
            far = f;
        };
        auto take = [&](uint64_t key) {
            if (walked && key <= after) return;
            if (key >= cut) {
                over = true;
                return;
            }
            if (n_in == cap && h > 0) {   // reclaim the composited front
                for (uint32_t j = h; j < n_in; ++j) my[(j - h) * kBlock] = my[j * kBlock];
                n_in -= h;
                h = 0;
            }
            if (n_in == cap) {
                over = true;
                const uint64_t last = my[(cap - 1) * kBlock];
                if (key > last) {
                    cut = key;
                    set_far();
                    return;
                }
                cut = last;   // the farthest kept fragment makes room
                n_in = cap - 1;
            }
            uint32_t j = n_in;
            while (j > h && my[(j - 1) * kBlock] > key) {
                my[j * kBlock] = my[(j - 1) * kBlock];
                --j;
            }
            my[j * kBlock] = key;
            ++n_in;
            set_far();
        };
        // composite the kept fragments nearer than `front` (nothing still
        // unvisited can come before them)
        auto drain = [&](float front) {
            while (!fin && h < n_in) {
                const uint64_t key = my[h * kBlock];
                if (!(__uint_as_float((uint32_t)(key >> 32)) < front)) break;
                ++h;
                if (blend(key)) fin = true;
            }
        };
        // depth-first walk without a stack: per level the children still to
        // visit (8 bits each, levels 0..7 and 8..15 in two words)
        uint64_t mlo = 0, mhi = 0;
        auto get_m = [&](uint32_t l) -> uint32_t {
            return (uint32_t)(((l < 8 ? mlo : mhi) >> ((l & 7) * 8)) & 0xFFu);
        };
        auto set_m = [&](uint32_t l, uint32_t m) {
            const uint32_t sh = (l & 7) * 8;
            if (l < 8)
                mlo = (mlo & ~(0xFFull << sh)) | ((uint64_t)m << sh);
            else
                mhi = (mhi & ~(0xFFull << sh)) | ((uint64_t)m << sh);
        };
        uint32_t l = 0, n = 0, ox = 0, oy = 0, oz = 0;
        // nearest depth any unvisited octant of the walk can hold: the
        // nearest pending child on every level of the current path
        auto frontier = [&]() -> float {
            float f = INFINITY;
            for (uint32_t k = 0; k <= l; ++k) {
                const uint32_t m = get_m(k);
                if (m == 0) continue;
                const uint32_t c = (order >> (4 * (__ffs(m) - 1))) & 7u;
                const uint32_t side = 1u << (L - k), hc = side >> 1;
                const float hw = (float)hc * 128.0f;
                const float dc = proj(M, 2, (float)(((ox & ~(side - 1)) + ((c >> 2) & 1u) * hc) * 256u) + hw,
                                      (float)(((oy & ~(side - 1)) + ((c >> 1) & 1u) * hc) * 256u) + hw,
                                      (float)(((oz & ~(side - 1)) + (c & 1u) * hc) * 256u) + hw);
                f = fminf(f, dc - hw * az);
            }
            return f - kDepthSlack;
        };
        set_m(0, expand(0, 0, 0, 0, 0));
        for (;;) {
            const uint32_t m = get_m(l);
            if (m == 0) {
                if (l == 0) break;
                --l;
                n >>= 3;
                const uint32_t side = 1u << (L - l);
                ox &= ~(side - 1);
                oy &= ~(side - 1);
                oz &= ~(side - 1);
                continue;
            }
            const uint32_t c = (order >> (4 * (__ffs(m) - 1))) & 7u;
            set_m(l, m & (m - 1));
            const uint32_t hc = 1u << (L - l - 1);
            const uint32_t cx = ox + ((c >> 2) & 1u) * hc, cy = oy + ((c >> 1) & 1u) * hc,
                           cz = oz + (c & 1u) * hc;
            const uint32_t cn = n * 8 + c;
            {
                // the child's depth range against the lanes' windows
                const float hw = (float)hc * 128.0f;
                const float dc = proj(M, 2, (float)(cx * 256u) + hw, (float)(cy * 256u) + hw, (float)(cz * 256u) + hw);
                if (dc - hw * az > wfar + kDepthSlack) {
                    // behind every compositing lane's window: left out of
                    // this walk, with everything as deep or deeper
                    if (!fin) {
                        over = true;
                        const uint64_t c2 = (uint64_t)(__float_as_uint(wfar) + 1u) << 32;
                        if (c2 < cut) {
                            cut = c2;
                            set_far();
                        }
                    }
                    continue;
                }
                if (dc + hw * az < wnear - kDepthSlack) continue;
            }
            if (l + 1 < B) {
                ++l;
                n = cn;
                ox = cx;
                oy = cy;
                oz = cz;
                set_m(l, expand(l, n, ox, oy, oz));
                continue;
            }
            // brick cn: its leaves are consecutive Morton codes, so their
            // table rows and their fragments are consecutive too
            const uint32_t bs = 3 * (L - B);
            const uint32_t row_lo = rank_of((uint64_t)cn << bs);
            const uint32_t row_hi = rank_of((uint64_t)(cn + 1) << bs);
            const uint32_t off = row_hi > row_lo ? a.oct_off[row_lo] : 0u;
            const uint32_t cnt = row_hi > row_lo ? a.oct_off[row_hi - 1] + a.oct_cnt[row_hi - 1] - off : 0u;
            for (uint32_t b = 0; b < cnt; b += kWave) {
                bool hit = false;
                uint32_t t = 0;
                uint64_t key = 0;
                if (b + (uint32_t)lane < cnt) {
                    const uint32_t i = off + b + (uint32_t)lane;
                    const uint4 r = a.frag[i];
                    const uint64_t lk = a.oct_key[r.w];   // the fragment's leaf
                    const uint32_t lx = compact3(lk >> 2), ly = compact3(lk >> 1), lz = compact3(lk);
                    const float x = (float)((lx << 8) | (r.x & 0xFFu)) + 0.5f;
                    const float y = (float)((ly << 8) | ((r.x >> 8) & 0xFFu)) + 0.5f;
                    const float z = (float)((lz << 8) | ((r.x >> 16) & 0xFFu)) + 0.5f;
                    const float d = proj(M, 2, x, y, z);
                    const float fx = floorf(proj(M, 0, x, y, z)), fy = floorf(proj(M, 1, x, y, z));
                    if (d > 0.0f && fx >= (float)x0 && fx < (float)(x0 + 8) && fy >= (float)y0 &&
                        fy < (float)(y0 + 8)) {
                        hit = true;
                        t = ((uint32_t)fy - y0) * 8 + ((uint32_t)fx - x0);
                        key = ((uint64_t)__float_as_uint(d) << 32) | i;
                    }
                }
                // hand every hit to the lane that owns its pixel
                for (uint64_t bal = __ballot(hit); bal; bal &= bal - 1) {
                    const int s = __ffsll((unsigned long long)bal) - 1;
                    const uint32_t ts = (uint32_t)__shfl((int)t, s, kWave);
                    const uint64_t ks = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(key >> 32), s, kWave) << 32) |
                                        (uint32_t)__shfl((int)(uint32_t)key, s, kWave);
                    if ((uint32_t)lane == ts && !fin) take(ks);
                }
            }
            drain(frontier());
            if (__ballot(!fin) == 0) break;   // every pixel of the tile is final
            wfar = wave_max(fin ? -INFINITY : far);
        }
        // the walk is complete: everything kept can be composited
        drain(INFINITY);
        if (!fin && !over) fin = true;   // nothing was left out
        if (__ballot(!fin) == 0) break;
    }
    if (mine) a.out[((size_t)v * a.height + py) * a.width + px] = make_float4(C0, C1, C2, 1.0f - T);
}

}  // namespace

size_t raycast_ws_bytes(uint32_t levels)
{
    if (levels < 1 || levels > kMaxRayLevels) return 0;
    const OccLayout o = occ_layout(levels);
    const size_t occ_b = (size_t)o.word[levels + 1] * 4;
    const size_t rank_b = ((size_t)o.n64 * 4 + 255) & ~(size_t)255;
    const size_t part_b = (scan_partials(o.n64) * 4 + 255) & ~(size_t)255;
    return ((occ_b + 255) & ~(size_t)255) + rank_b + part_b;
}

hipError_t raycast_launch(const Device& dev, const fhv_pofa* p, uint32_t levels, const RayViews& rv,
                          uint32_t mode, float tau, float* out, void* ws, hipStream_t s)
{
    const OccLayout lay = occ_layout(levels);
    const size_t occ_b = (((size_t)lay.word[levels + 1] * 4) + 255) & ~(size_t)255;
    const size_t rank_b = ((size_t)lay.n64 * 4 + 255) & ~(size_t)255;
    uint32_t* occ = (uint32_t*)ws;
    uint32_t* rank = (uint32_t*)((char*)ws + occ_b);
    uint32_t* part = (uint32_t*)((char*)ws + occ_b + rank_b);
    hipError_t e;
    {
        ProfScope ps(dev, "ray.occupancy", s);
        e = fill_u32(occ, lay.word[levels + 1], 0u, s);
        if (e != hipSuccess) return e;
        if (p->cap_occ > 0) {
            uint64_t g = (p->cap_occ + kBlock - 1) / kBlock;
            const uint64_t gmax = (uint64_t)dev.cus * 8;
            g = g > gmax ? gmax : g;
            k_occ_build<<<dim3((unsigned)g), dim3(kBlock), 0, s>>>(p->oct_key, p->n_occ, p->cap_occ, occ, lay,
                                                                  levels);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        e = scan<uint32_t>(LoadPopc{(const uint64_t*)(occ + lay.word[levels])}, StoreExcl<uint32_t>{rank},
                           lay.n64, part, (uint32_t*)nullptr, s);
        if (e != hipSuccess) return e;
    }
    RayArgs a;
    for (uint32_t v = 0; v < rv.n_views; ++v) {
        for (int k = 0; k < 12; ++k) a.m[v][k] = rv.m[v][k];
        // children by the depth of their offset (x, y, z) in {0, 1}^3,
        // nearest first (Morton child index x << 2 | y << 1 | z)
        uint32_t idx[8];
        float dep[8];
        for (uint32_t c = 0; c < 8; ++c) {
            idx[c] = c;
            dep[c] = rv.m[v][8] * (float)((c >> 2) & 1u) + rv.m[v][9] * (float)((c >> 1) & 1u) +
                     rv.m[v][10] * (float)(c & 1u);
        }
        for (int i = 1; i < 8; ++i)
            for (int j = i; j > 0 && dep[idx[j]] < dep[idx[j - 1]]; --j) {
                const uint32_t t = idx[j];
                idx[j] = idx[j - 1];
                idx[j - 1] = t;
            }
        a.order[v] = 0;
        for (int i = 0; i < 8; ++i) a.order[v] |= idx[i] << (4 * i);
    }
    a.frag = (const uint4*)p->frag;
    a.oct_key = p->oct_key;
    a.oct_off = p->oct_off;
    a.oct_cnt = p->oct_cnt;
    a.occ = occ;
    a.rank = rank;
    a.lay = lay;
    a.out = (float4*)out;
    a.L = levels;
    a.width = rv.width;
    a.height = rv.height;
    a.tiles_x = (rv.width + 7) / 8;
    a.n_tiles = a.tiles_x * ((rv.height + 7) / 8);
    a.tau = tau;
    const dim3 grid((a.n_tiles + kBlock / kWave - 1) / (kBlock / kWave), rv.n_views);
    ProfScope ps(dev, "ray.cast", s);
    if (mode == FHV_RAY_NEAREST)
        k_raycast<0><<<grid, dim3(kBlock), 0, s>>>(a);
    else
        k_raycast<1><<<grid, dim3(kBlock), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace fhv

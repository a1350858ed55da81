// Compaction of fragment lists into per-octant arrays (FHV_POFA, Sec. 3.1
// Fig. 6 and Sec. 3.2): per occupied key a count and an offset, the offsets
// being sums of counts in ascending key (Morton) order, every key's records
// contiguous, ascending by (w0, w1, w2), w3 = the key's table rank.
//
// The paper counts per octant, scans, resets the counters and rasterizes a
// second time. Here the pool is read linearly instead, through the key
// sidecar the capture wrote, and keys are grouped in buckets ("bricks") of
// 512 consecutive keys so that every bucket fits a workgroup's LDS:
//   k_hist     per brick: fragment count (atomic add) and number of
//              distinct keys (atomic or into a key bitmap; the first setter
//              of a bit counts the key)
//   scan       exclusive sums of both per-brick counts: brick fragment
//              offsets and brick rank bases; totals = n_frag, n_occ
//   k_scatter  every pool record to its brick's range of a staging array
//              (slot within the brick from an atomic cursor), key in w3
//   k_brick    one workgroup per brick: counting sort of the brick's records
//              by key inside LDS (in place in the output when the brick is
//              larger than LDS), a per-key insertion sort into canonical
//              order, then the output records with w3 = rank and the
//              brick's table rows
#include "fhv_common.h"

namespace fhv {

namespace {

constexpr int kLdsRecs = 2048;   // records staged in LDS per brick (32 KiB)

__device__ __forceinline__ uint64_t frag_count(const uint64_t* counter, uint64_t cap)
{
    const uint64_t c = *counter;
    return c < cap ? c : cap;
}

__global__ void __launch_bounds__(kBlock)
k_hist(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ counter, uint64_t cap,
       uint32_t* __restrict__ brick_cnt, uint32_t* __restrict__ brick_occ,
       uint32_t* __restrict__ bitmap)
{
    const uint64_t F = frag_count(counter, cap);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < F; i += stride) {
        const uint32_t key = keys[i];
        const uint32_t b = key >> kBrickShift;
        atomicAdd(brick_cnt + b, 1u);
        const uint32_t bit = 1u << (key & 31);
        const uint32_t old = atomicOr(bitmap + (key >> 5), bit);
        if (!(old & bit)) atomicAdd(brick_occ + b, 1u);
    }
}

__global__ void __launch_bounds__(kBlock)
k_scatter(const uint4* __restrict__ pool, const uint32_t* __restrict__ keys,
          const uint64_t* __restrict__ counter, uint64_t cap, const uint32_t* __restrict__ brick_off,
          uint32_t* __restrict__ brick_cur, uint4* __restrict__ stage)
{
    const uint64_t F = frag_count(counter, cap);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < F; i += stride) {
        const uint32_t key = keys[i];
        const uint32_t b = key >> kBrickShift;
        const uint32_t slot = brick_off[b] + atomicAdd(brick_cur + b, 1u);
        uint4 r = pool[i];
        r.w = key;
        stage[slot] = r;
    }
}

__device__ __forceinline__ bool rec_less(const uint4& a, const uint4& b)
{
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.z < b.z;
}

// 512-entry exclusive scan in LDS by one 256-thread workgroup (2 per thread).
__device__ void scan512(uint32_t* v, uint32_t* tmp)
{
    const int t = threadIdx.x;
    // inclusive Hillis-Steele over 512 values in place
    for (int d = 1; d < 512; d <<= 1) {
        const uint32_t a0 = (2 * t >= d) ? v[2 * t - d] : 0u;
        const uint32_t a1 = (2 * t + 1 >= d) ? v[2 * t + 1 - d] : 0u;
        __syncthreads();
        v[2 * t] += a0;
        v[2 * t + 1] += a1;
        __syncthreads();
    }
    // to exclusive
    tmp[2 * t] = 2 * t ? v[2 * t - 1] : 0u;
    tmp[2 * t + 1] = v[2 * t];
    __syncthreads();
    v[2 * t] = tmp[2 * t];
    v[2 * t + 1] = tmp[2 * t + 1];
    __syncthreads();
}

template <bool kInLds>
__device__ void brick_sort(uint4* __restrict__ buf, const uint4* __restrict__ src, uint32_t n,
                           uint32_t* cnt, uint32_t* off, uint32_t* cur, uint32_t* rank,
                           uint32_t* tmp, uint32_t brick, uint32_t base_off, uint32_t base_rank,
                           uint4* __restrict__ out, uint64_t* __restrict__ oct_key,
                           uint32_t* __restrict__ oct_off, uint32_t* __restrict__ oct_cnt,
                           uint64_t cap_occ)
{
    const int t = threadIdx.x;
    cnt[2 * t] = cnt[2 * t + 1] = 0;
    __syncthreads();
    for (uint32_t i = t; i < n; i += kBlock) atomicAdd(cnt + (src[i].w & (kBrickKeys - 1)), 1u);
    __syncthreads();
    for (int k = 0; k < 2; ++k) {
        const uint32_t c = cnt[2 * t + k];
        off[2 * t + k] = c;
        rank[2 * t + k] = c ? 1u : 0u;
    }
    __syncthreads();
    scan512(off, tmp);
    scan512(rank, tmp);
    for (int k = 0; k < 2; ++k) cur[2 * t + k] = off[2 * t + k];
    __syncthreads();
    // counting sort by key into buf
    for (uint32_t i = t; i < n; i += kBlock) {
        const uint4 r = src[i];
        const uint32_t p = atomicAdd(cur + (r.w & (kBrickKeys - 1)), 1u);
        buf[p] = r;
    }
    __syncthreads();
    // canonical order inside every key, then table rows
    for (int k = 0; k < 2; ++k) {
        const uint32_t leaf = 2 * t + k;
        const uint32_t c = cnt[leaf], o = off[leaf];
        for (uint32_t a = 1; a < c; ++a) {
            const uint4 x = buf[o + a];
            uint32_t b = a;
            while (b > 0 && rec_less(x, buf[o + b - 1])) {
                buf[o + b] = buf[o + b - 1];
                --b;
            }
            buf[o + b] = x;
        }
        if (c) {
            const uint64_t rk = (uint64_t)base_rank + rank[leaf];
            if (rk < cap_occ) {
                oct_key[rk] = ((uint64_t)brick << kBrickShift) | leaf;
                oct_off[rk] = base_off + o;
                oct_cnt[rk] = c;
            }
        }
    }
    __syncthreads();
    // records out with w3 = rank
    for (uint32_t i = t; i < n; i += kBlock) {
        uint4 r = buf[i];
        r.w = base_rank + rank[r.w & (kBrickKeys - 1)];
        out[i] = r;
    }
}

__global__ void __launch_bounds__(kBlock)
k_brick(const uint4* __restrict__ stage, const uint32_t* __restrict__ brick_cnt,
        const uint32_t* __restrict__ brick_off, const uint32_t* __restrict__ brick_rank,
        uint32_t n_brick, uint4* __restrict__ frag, uint64_t* __restrict__ oct_key,
        uint32_t* __restrict__ oct_off, uint32_t* __restrict__ oct_cnt, uint64_t cap_occ)
{
    __shared__ uint4 lbuf[kLdsRecs];
    __shared__ uint32_t cnt[kBrickKeys], off[kBrickKeys], cur[kBrickKeys], rank[kBrickKeys],
        tmp[kBrickKeys];
    for (uint32_t b = blockIdx.x; b < n_brick; b += gridDim.x) {
        const uint32_t n = brick_cnt[b];
        if (n == 0) continue;
        const uint32_t o = brick_off[b];
        if (n <= (uint32_t)kLdsRecs)
            brick_sort<true>(lbuf, stage + o, n, cnt, off, cur, rank, tmp, b, o, brick_rank[b],
                             frag + o, oct_key, oct_off, oct_cnt, cap_occ);
        else
            brick_sort<false>(frag + o, stage + o, n, cnt, off, cur, rank, tmp, b, o,
                              brick_rank[b], frag + o, oct_key, oct_off, oct_cnt, cap_occ);
        __syncthreads();
    }
}

__global__ void k_totals(const uint64_t* __restrict__ counter, uint64_t cap,
                         uint64_t* __restrict__ n_frag)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_frag = frag_count(counter, cap);
}

}  // namespace

struct CompactWs {
    uint32_t *brick_cnt, *brick_occ, *brick_cur, *brick_off, *brick_rank, *bitmap, *part;
    uint4* stage;
};

static CompactWs carve_compact(void* ws, uint64_t n_head, uint64_t capacity, size_t* bytes)
{
    const uint64_t n_brick = (n_head + kBrickKeys - 1) / kBrickKeys;
    Carver c{(char*)ws, 0};
    CompactWs w;
    // the three zero-initialised arrays are adjacent so one fill clears them
    const uint64_t zlen = 3 * n_brick + (n_head + 31) / 32;
    uint32_t* z = c.take<uint32_t>(zlen);
    w.brick_cnt = z;
    w.brick_occ = z ? z + n_brick : nullptr;
    w.brick_cur = z ? z + 2 * n_brick : nullptr;
    w.bitmap = z ? z + 3 * n_brick : nullptr;
    w.brick_off = c.take<uint32_t>(n_brick);
    w.brick_rank = c.take<uint32_t>(n_brick);
    w.part = c.take<uint32_t>(scan_partials(n_brick));
    w.stage = c.take<uint4>(capacity);
    if (bytes) *bytes = c.off + 256;
    return w;
}

size_t compact_ws_bytes(const fhv_capture_desc* d, uint64_t n_head, uint64_t capacity)
{
    (void)d;
    size_t b = 0;
    carve_compact(nullptr, n_head, capacity, &b);
    return b;
}

hipError_t compact_launch(const Device& dev, const fhv_lists* L, const fhv_capture_desc* d,
                          const fhv_pofa* out, void* ws, hipStream_t s)
{
    (void)d;
    const uint64_t n_brick = (L->n_head + kBrickKeys - 1) / kBrickKeys;
    CompactWs w = carve_compact(ws, L->n_head, L->capacity, nullptr);
    hipError_t e;
    uint64_t gb = (L->capacity + kBlock - 1) / kBlock;
    const uint64_t gmax = (uint64_t)dev.cus * 16;
    const unsigned grid = (unsigned)(gb < 1 ? 1 : (gb > gmax ? gmax : gb));
    {
        ProfScope ps(dev, "compact.hist", s);
        e = fill_u32(w.brick_cnt, 3 * n_brick + (L->n_head + 31) / 32, 0u, s);
        if (e != hipSuccess) return e;
        k_totals<<<dim3(1), dim3(64), 0, s>>>(L->counter, L->capacity, out->n_frag);
        k_hist<<<dim3(grid), dim3(kBlock), 0, s>>>(L->keys, L->counter, L->capacity, w.brick_cnt,
                                                   w.brick_occ, w.bitmap);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    {
        ProfScope ps(dev, "compact.scan", s);
        e = scan_u32(w.brick_cnt, w.brick_off, n_brick, false, w.part, nullptr, s);
        if (e == hipSuccess) e = scan_u32(w.brick_occ, w.brick_rank, n_brick, false, w.part, out->n_occ, s);
    }
    if (e != hipSuccess) return e;
    {
        ProfScope ps(dev, "compact.scatter", s);
        k_scatter<<<dim3(grid), dim3(kBlock), 0, s>>>((const uint4*)L->pool, L->keys, L->counter,
                                                      L->capacity, w.brick_off, w.brick_cur, w.stage);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    const uint64_t bmax = (uint64_t)dev.cus * 32;
    const unsigned gbrick = (unsigned)(n_brick < bmax ? n_brick : bmax);
    ProfScope ps(dev, "compact.brick", s);
    k_brick<<<dim3(gbrick ? gbrick : 1), dim3(kBlock), 0, s>>>(
        w.stage, w.brick_cnt, w.brick_off, w.brick_rank, (uint32_t)n_brick, (uint4*)out->frag,
        out->oct_key, out->oct_off, out->oct_cnt, out->cap_occ);
    return hipGetLastError();
}

}  // namespace fhv

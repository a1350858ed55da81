// Prefix sums and fills.
//
// The scan is a three-pass reduce-then-scan over chunks of 2048 values
// (256 threads x 8 consecutive values): per-chunk sums, one workgroup that
// scans the chunk sums, then every chunk scanned again with its offset.
// Within a workgroup each thread sums its 8 values, the 64 thread sums of a
// wave are scanned with shuffles and the 4 wave totals through LDS.
#include "fhv_common.h"

namespace fhv {

namespace {

constexpr int kItems = 8;
constexpr int kChunk = kBlock * kItems;

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan of one value per thread across the workgroup; returns the
// thread's exclusive prefix and sets *total to the workgroup sum.
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T* total)
{
    __shared__ T wsum[kBlock / kWave];
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
    T inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    T base = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (w < wid) base += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return base + inc - v;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_reduce(const T* __restrict__ in, uint64_t n,
                                                   T* __restrict__ partial)
{
    const uint64_t base = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kItems;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) s += in[base + k];
    T tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the chunk sums in place, with carry.
template <class T>
__global__ void __launch_bounds__(kBlock) k_scan_partials(T* __restrict__ partial, uint64_t nb,
                                                          uint64_t* __restrict__ total)
{
    T carry = 0;
    for (uint64_t c0 = 0; c0 < nb; c0 += kChunk) {
        const uint64_t base = c0 + (uint64_t)threadIdx.x * kItems;
        T v[kItems];
        T s = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            v[k] = (base + k < nb) ? partial[base + k] : T(0);
            s += v[k];
        }
        T tot;
        T run = carry + block_excl_scan(s, &tot);
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (base + k < nb) partial[base + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = (uint64_t)carry;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_scan_final(const T* __restrict__ in, T* __restrict__ out,
                                                       uint64_t n, const T* __restrict__ partial,
                                                       int inclusive)
{
    const uint64_t base = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kItems;
    T v[kItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : T(0);
        s += v[k];
    }
    T tot;
    T run = partial[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (inclusive) run += v[k];
        if (base + k < n) out[base + k] = run;
        if (!inclusive) run += v[k];
    }
}

template <class T>
hipError_t scan_impl(const T* in, T* out, uint64_t n, bool inclusive, T* partial, uint64_t* total,
                     hipStream_t s)
{
    if (n == 0) {
        if (total) return fill_u64(total, 1, 0, s);
        return hipSuccess;
    }
    const uint64_t nb = (n + kChunk - 1) / kChunk;
    k_reduce<T><<<dim3((unsigned)nb), dim3(kBlock), 0, s>>>(in, n, partial);
    k_scan_partials<T><<<dim3(1), dim3(kBlock), 0, s>>>(partial, nb, total);
    k_scan_final<T><<<dim3((unsigned)nb), dim3(kBlock), 0, s>>>(in, out, n, partial, inclusive ? 1 : 0);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    // 16-byte stores over the aligned body, scalar head and tail
    const uint64_t mis = ((uintptr_t)p & 15) ? (16 - ((uintptr_t)p & 15)) / 4 : 0;
    const uint64_t head = mis < n ? mis : n;
    if (i < head) p[i] = v;
    uint4* q = (uint4*)(p + head);
    const uint64_t nq = (n - head) / 4;
    const uint4 vv = make_uint4(v, v, v, v);
    for (uint64_t j = i; j < nq; j += stride) q[j] = vv;
    const uint64_t t0 = head + nq * 4;
    if (t0 + i < n) p[t0 + i] = v;
}

__global__ void __launch_bounds__(kBlock) k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = v;
}

}  // namespace

size_t scan_partials(uint64_t n) { return (size_t)((n + kChunk - 1) / kChunk) + 1; }

hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, bool inclusive,
                    uint32_t* partial, uint64_t* total, hipStream_t s)
{
    return scan_impl<uint32_t>(in, out, n, inclusive, partial, total, s);
}

hipError_t scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, bool inclusive,
                    uint64_t* partial, uint64_t* total, hipStream_t s)
{
    return scan_impl<uint64_t>(in, out, n, inclusive, partial, total, s);
}

static unsigned grid_for(uint64_t n_threads)
{
    uint64_t b = (n_threads + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_fill_u32<<<dim3(grid_for(n / 4 + 4)), dim3(kBlock), 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_fill_u64<<<dim3(grid_for(n)), dim3(kBlock), 0, s>>>(p, n, v);
    return hipGetLastError();
}

}  // namespace fhv

// Prefix sums over n values with caller-defined load and store functors.
//
// Three passes over chunks of 2048 values (256 threads x 8 consecutive
// values): per-chunk sums, one workgroup that scans the chunk sums (with a
// carry across its own chunks), then every chunk scanned again with its
// offset and handed to the store functor. Up to 1024 chunks the second pass
// is folded into the third: each chunk's workgroup sums the chunk sums
// before it. Within a workgroup each thread sums
// its 8 values, the 64 thread sums of a wave are scanned with shuffles and the
// 4 wave totals through LDS.
//
//   Load:  T operator()(uint64_t i) const          value i (i < n)
//   Store: void operator()(uint64_t i, T v, T excl) value i and the sum of
//          all values before it
#pragma once

#include "fhv_common.h"

namespace fhv {
namespace scan_detail {

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

template <class T, class Load>
__global__ void __launch_bounds__(kBlock) k_reduce(Load ld, uint64_t n, T* __restrict__ partial)
{
    const uint64_t base = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kItems;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) s += ld(base + k);
    T tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the chunk sums in place, with carry.
template <class T>
__global__ void __launch_bounds__(kBlock) k_scan_partials(T* __restrict__ partial, uint64_t nb,
                                                          T* __restrict__ total)
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
    if (threadIdx.x == 0 && total) *total = carry;
}

template <class T, class Load, class Store>
__global__ void __launch_bounds__(kBlock) k_scan_final(Load ld, Store st, uint64_t n,
                                                       const T* __restrict__ partial)
{
    const uint64_t base = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kItems;
    T v[kItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = (base + k < n) ? ld(base + k) : T(0);
        s += v[k];
    }
    T tot;
    T run = partial[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) st(base + k, v[k], run);
        run += v[k];
    }
}

// k_scan_final without the separate pass over the chunk sums: each
// workgroup adds up the sums of the chunks before its own (at most
// kDirectChunks of them; integers, so in any order), and the last one
// writes the total.
constexpr uint64_t kDirectChunks = 1024;

template <class T, class Load, class Store>
__global__ void __launch_bounds__(kBlock) k_scan_direct(Load ld, Store st, uint64_t n, uint64_t nb,
                                                        const T* __restrict__ partial, T* __restrict__ total)
{
    T pre = 0;
    for (uint64_t c = threadIdx.x; c < blockIdx.x; c += kBlock) pre += partial[c];
    T off;
    block_excl_scan(pre, &off);
    const uint64_t base = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kItems;
    T v[kItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = (base + k < n) ? ld(base + k) : T(0);
        s += v[k];
    }
    T tot;
    T run = off + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) st(base + k, v[k], run);
        run += v[k];
    }
    if (total && threadIdx.x == 0 && blockIdx.x + 1 == nb) *total = off + tot;
}

}  // namespace scan_detail

// Number of T elements of scratch scan() needs for n values.
inline size_t scan_scratch(uint64_t n)
{
    return (size_t)((n + scan_detail::kChunk - 1) / scan_detail::kChunk) + 1;
}

// Enqueues the scan; *total (device, may be null) receives the sum of all n.
template <class T, class Load, class Store>
hipError_t scan(Load ld, Store st, uint64_t n, T* partial, T* total, hipStream_t s)
{
    using namespace scan_detail;
    if (n == 0) return hipSuccess;
    const uint64_t nb = (n + kChunk - 1) / kChunk;
    k_reduce<T, Load><<<dim3((unsigned)nb), dim3(kBlock), 0, s>>>(ld, n, partial);
    if (nb <= kDirectChunks) {
        k_scan_direct<T, Load, Store><<<dim3((unsigned)nb), dim3(kBlock), 0, s>>>(ld, st, n, nb, partial, total);
        return hipGetLastError();
    }
    k_scan_partials<T><<<dim3(1), dim3(kBlock), 0, s>>>(partial, nb, total);
    k_scan_final<T, Load, Store><<<dim3((unsigned)nb), dim3(kBlock), 0, s>>>(ld, st, n, partial);
    return hipGetLastError();
}

template <class T>
struct LoadArray {
    const T* p;
    __device__ T operator()(uint64_t i) const { return p[i]; }
};

template <class T>
struct StoreExcl {
    T* p;
    __device__ void operator()(uint64_t i, T, T excl) const { p[i] = excl; }
};

template <class T>
struct StoreIncl {
    T* p;
    __device__ void operator()(uint64_t i, T v, T excl) const { p[i] = excl + v; }
};

}  // namespace fhv

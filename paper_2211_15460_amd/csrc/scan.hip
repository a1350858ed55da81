// Plain array prefix sums and fills.
#include "scan.h"

namespace fhv {

namespace {

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

unsigned grid_for(uint64_t n_threads)
{
    uint64_t b = (n_threads + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

}  // namespace

size_t scan_partials(uint64_t n) { return scan_scratch(n); }

hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, bool inclusive,
                    uint32_t* partial, uint64_t* total, hipStream_t s)
{
    (void)total;
    if (inclusive) return scan<uint32_t>(LoadArray<uint32_t>{in}, StoreIncl<uint32_t>{out}, n, partial, (uint32_t*)nullptr, s);
    return scan<uint32_t>(LoadArray<uint32_t>{in}, StoreExcl<uint32_t>{out}, n, partial, (uint32_t*)nullptr, s);
}

hipError_t scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, bool inclusive,
                    uint64_t* partial, uint64_t* total, hipStream_t s)
{
    if (n == 0 && total) return fill_u64(total, 1, 0, s);
    if (inclusive) return scan<uint64_t>(LoadArray<uint64_t>{in}, StoreIncl<uint64_t>{out}, n, partial, total, s);
    return scan<uint64_t>(LoadArray<uint64_t>{in}, StoreExcl<uint64_t>{out}, n, partial, total, s);
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

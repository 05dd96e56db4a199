// KNN with ties kept (Algorithm 2's selection d <= d_k): the k nearest plus
// every further candidate at exactly the k-th FP32 length. The library runs
// its KNN search with TIES_K = 64 neighbours per source (so the 64 - k keys
// after the k-th are the tie candidates, in key order) and compacts, per
// source, the keys up to the last one whose length equals the k-th.
#include "mg_internal.h"

namespace mg {

__global__ __launch_bounds__(256) void k_ties_count(int64_t N, int k, const int32_t* __restrict__ dst,
                                                    const float* __restrict__ length, uint32_t* __restrict__ counts,
                                                    mg_report* __restrict__ rep) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool trunc = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const int64_t e0 = i * TIES_K;
        uint32_t c = 0;
        if (dst[e0] >= 0) {                       // a valid row (skipped sources hold dst = -1)
            const float lk = length[e0 + k - 1];
            c = (uint32_t)k;
            while (c < (uint32_t)TIES_K && length[e0 + c] <= lk) ++c;
            trunc |= c == (uint32_t)TIES_K && k < TIES_K;
        }
        counts[i] = c;
    }
    if (ballot(trunc) != 0 && lane_id() == 0) atomicOr(&rep->flags, (uint32_t)MG_FLAG_TIES);
}

__global__ __launch_bounds__(256) void k_ties_fill(int64_t N, const int32_t* __restrict__ src,
                                                   const int32_t* __restrict__ dst, const int32_t* __restrict__ image,
                                                   const float* __restrict__ length,
                                                   const uint32_t* __restrict__ counts,
                                                   const int64_t* __restrict__ offsets, int64_t capacity,
                                                   int32_t* __restrict__ osrc, int32_t* __restrict__ odst,
                                                   int32_t* __restrict__ oimg, float* __restrict__ olen) {
    const int64_t total = N * TIES_K;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t i = e / TIES_K;
        const uint32_t r = (uint32_t)(e - i * TIES_K);
        if (r >= counts[i]) continue;
        const int64_t o = offsets[i] + r;
        if (o >= capacity) continue;
        osrc[o] = src[e];
        odst[o] = dst[e];
        oimg[3 * o] = image[3 * e];
        oimg[3 * o + 1] = image[3 * e + 1];
        oimg[3 * o + 2] = image[3 * e + 2];
        olen[o] = length[e];
    }
}

hipError_t launch_ties(int64_t N, int k, const int32_t* src, const int32_t* dst, const int32_t* image,
                       const float* length, int64_t capacity, int32_t* osrc, int32_t* odst, int32_t* oimg,
                       float* olen, int64_t* offsets, uint32_t* counts, int64_t* bsum, mg_report* report,
                       hipStream_t s) {
    const int cu = device_cu_count();
    if (N > 0)
        hipLaunchKernelGGL(k_ties_count, dim3(cu * 4), dim3(256), 0, s, N, k, dst, length, counts, report);
    hipError_t e = launch_scan_counts(counts, N, offsets, bsum, capacity, report, s);
    if (e != hipSuccess || N == 0) return e;
    hipLaunchKernelGGL(k_ties_fill, dim3(cu * 16), dim3(256), 0, s, N, src, dst, image, length, counts, offsets,
                       capacity, osrc, odst, oimg, olen);
    return hipGetLastError();
}

}  // namespace mg

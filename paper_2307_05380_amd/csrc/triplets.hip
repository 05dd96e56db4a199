// Triplets Gamma_2 (Definition def6): every ordered pair (e1, e2) of two
// different edges with the same source, as edge indices into a graph whose
// edges are grouped by source (row_ptr). Optionally the angle between the two
// edge vectors.
//
// count (d (d - 1) per source) -> scan (offsets, total, capacity flag) ->
// fill. The fill gives each source to one wave (static cyclic assignment); the
// wave writes the source's pairs in (e1, e2) order with consecutive lanes on
// consecutive outputs, so the stores are fully coalesced. The pass is bound by
// the 8 bytes (12 with the angle) written per triplet.
#include "mg_internal.h"

namespace mg {

// Largest out-degree handled: d (d - 1) must fit the 32-bit per-source count.
constexpr int64_t TRIP_MAX_DEG = 65536;

__global__ __launch_bounds__(256) void k_trip_count(const int64_t* __restrict__ row_ptr, int64_t N, int64_t E,
                                                    uint32_t* __restrict__ counts, mg_report* __restrict__ rep) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const int64_t a = row_ptr[i], b = row_ptr[i + 1];
        const int64_t d = b - a;
        const bool ok = a >= 0 && d >= 0 && b <= E && d <= TRIP_MAX_DEG;
        bad |= !ok;
        counts[i] = ok ? (uint32_t)(d * (d - 1)) : 0u;
    }
    if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&rep->flags, (uint32_t)MG_FLAG_RANGE);
}

__global__ __launch_bounds__(256) void k_trip_fill(const int64_t* __restrict__ row_ptr, int64_t N,
                                                   const uint32_t* __restrict__ counts,
                                                   const int64_t* __restrict__ offsets, int64_t capacity,
                                                   const float* __restrict__ vec, int32_t* __restrict__ e1,
                                                   int32_t* __restrict__ e2, float* __restrict__ cosv) {
    // a row of at most 64 edges: its vectors and their norms staged once per
    // source (the per-triplet arithmetic is the same as from global memory)
    __shared__ float4 sv[4][WAVE];
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t i = grid_wave(); i < N; i += grid_waves()) {
        const uint32_t cnt = counts[i];
        if (cnt == 0) continue;
        const int64_t r0 = row_ptr[i];
        const uint32_t dm1 = (uint32_t)(row_ptr[i + 1] - r0) - 1u;   // d - 1 >= 1
        const int64_t o0 = offsets[i];
        const bool staged = cosv != nullptr && dm1 < (uint32_t)WAVE;
        if (staged) {
            if ((uint32_t)lane <= dm1) {
                const int64_t e = r0 + lane;
                const float x = vec[3 * e], y = vec[3 * e + 1], z = vec[3 * e + 2];
                sv[wv][lane] = make_float4(x, y, z, sqrtf(fmaf(z, z, fmaf(y, y, x * x))));
            }
            wave_lds_sync();
        }
        for (uint32_t p = (uint32_t)lane; p < cnt; p += WAVE) {
            const int64_t q = o0 + p;
            if (q >= capacity) break;
            const uint32_t a = p / dm1;
            uint32_t b = p - a * dm1;
            b += b >= a ? 1u : 0u;
            const int64_t ea = r0 + a, eb = r0 + b;
            e1[q] = (int32_t)ea;
            e2[q] = (int32_t)eb;
            if (staged) {
                const float4 va = sv[wv][a], vb = sv[wv][b];
                const float num = fmaf(va.z, vb.z, fmaf(va.y, vb.y, va.x * vb.x));
                const float den = va.w * vb.w;
                cosv[q] = den > 0.0f ? num / den : 0.0f;
            } else if (cosv) {
                const float ax = vec[3 * ea], ay = vec[3 * ea + 1], az = vec[3 * ea + 2];
                const float bx = vec[3 * eb], by = vec[3 * eb + 1], bz = vec[3 * eb + 2];
                const float num = fmaf(az, bz, fmaf(ay, by, ax * bx));
                const float den = sqrtf(fmaf(az, az, fmaf(ay, ay, ax * ax))) * sqrtf(fmaf(bz, bz, fmaf(by, by, bx * bx)));
                cosv[q] = den > 0.0f ? num / den : 0.0f;
            }
        }
        if (staged) wave_lds_sync();   // the next source overwrites the staged row
    }
}

hipError_t launch_triplets(const int64_t* row_ptr, int64_t N, int64_t E, const float* vec, int64_t capacity,
                           int32_t* e1, int32_t* e2, float* cosv, int64_t* offsets, uint32_t* counts,
                           int64_t* bsum, mg_report* report, hipStream_t s) {
    const int cu = device_cu_count();
    if (N > 0) {
        const int64_t g = (N + 255) / 256;
        hipLaunchKernelGGL(k_trip_count, dim3((unsigned)(g < cu * 8 ? g : cu * 8)), dim3(256), 0, s, row_ptr, N,
                           E, counts, report);
    }
    hipError_t e = launch_scan_counts(counts, N, offsets, bsum, capacity, report, s);
    if (e != hipSuccess || N == 0) return e;
    // up to four times the resident grid (the dispatcher refills)
    const int64_t gf = (N + 3) / 4;
    hipLaunchKernelGGL(k_trip_fill, dim3((unsigned)(gf < cu * 32 ? gf : cu * 32)), dim3(256), 0, s, row_ptr, N,
                       counts, offsets, capacity, vec,
                       e1, e2, cosv);
    return hipGetLastError();
}

}  // namespace mg

// Symmetric closure of a multigraph grouped by source: every edge (i, j, t)
// whose reverse (j, i, -t) is missing gives j the edge (j, i, -t) with the same
// length (the paper's symmetric-graph procedure, Sec. 2.2; each edge once).
//
// Output order: source by source, the source's own edges in input order, then
// the reverse edges it receives, in the order of the input edges they reverse.
//
// Passes: mark (reverse lookup in the destination's out-list; count the
// missing ones per receiving atom) -> two scans (received offsets, output
// offsets) -> bucket (each missing edge claims a slot of its receiver) ->
// fill (each receiver orders its bucket by input-edge index: a rank count,
// quadratic in the bucket size, which stays small for neighbour lists).
// The lookups scan out-lists of length d, so the pass suits graphs of modest
// degree (KNN); a cutoff graph is already symmetric. The per-source passes give
// each source 16 lanes (four sources per wave: a KNN row of k <= 16 fills its
// lanes, longer rows loop), and a lookup reads the out-list eight entries at a
// time, every load of a group issued before the first is compared.
#include "mg_internal.h"

namespace mg {

constexpr int SYM_LANES = 16;                  // lanes per source
constexpr int SYM_PER_WAVE = WAVE / SYM_LANES;  // sources per wave
constexpr int SYM_CHUNK = 8;                   // out-list entries read together by a lookup

__global__ __launch_bounds__(256) void k_sym_zero(uint32_t* __restrict__ a, uint32_t* __restrict__ b, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += stride) {
        a[q] = 0u;
        b[q] = 0u;
    }
}

// Edge range of source i clamped to [0, E] (a malformed row_ptr never makes
// the passes read outside the edge arrays); false if clamping was needed.
__device__ __forceinline__ bool row_range(const int64_t* __restrict__ row_ptr, int64_t i, int64_t E, int64_t& a,
                                          int64_t& b) {
    const int64_t ra = row_ptr[i], rb = row_ptr[i + 1];
    a = min(max(ra, (int64_t)0), E);
    b = min(max(rb, a), E);
    return a == ra && b == rb;
}

__device__ __forceinline__ bool has_edge(const int64_t* __restrict__ row_ptr, int64_t E,
                                         const int32_t* __restrict__ dst, const int32_t* __restrict__ image,
                                         int64_t j, int32_t i, int t0, int t1, int t2) {
    int64_t a, b;
    row_range(row_ptr, j, E, a, b);
    bool found = false;
    for (int64_t f = a; f < b && !found; f += SYM_CHUNK) {
        int32_t d[SYM_CHUNK], x0[SYM_CHUNK], x1[SYM_CHUNK], x2[SYM_CHUNK];
#pragma unroll
        for (int u = 0; u < SYM_CHUNK; ++u) {   // indices clamped into the row: no branch between loads
            const int64_t q = min(f + u, b - 1);
            d[u] = dst[q];
            x0[u] = image[3 * q];
            x1[u] = image[3 * q + 1];
            x2[u] = image[3 * q + 2];
        }
#pragma unroll
        for (int u = 0; u < SYM_CHUNK; ++u)
            found |= f + u < b && d[u] == i && x0[u] == t0 && x1[u] == t1 && x2[u] == t2;
    }
    return found;
}

// Sources four to a wave (static cyclic assignment), a lane per edge.
__global__ __launch_bounds__(256) void k_sym_mark(const int64_t* __restrict__ row_ptr, int64_t N, int64_t E,
                                                  const int32_t* __restrict__ dst, const int32_t* __restrict__ image,
                                                  uint8_t* __restrict__ miss, uint32_t* __restrict__ addcnt,
                                                  mg_report* __restrict__ rep) {
    const int lane = lane_id();
    const int sub = lane / SYM_LANES, sl = lane - sub * SYM_LANES;
    bool bad = false;
    for (int64_t i = grid_wave() * SYM_PER_WAVE + sub; i < N; i += grid_waves() * SYM_PER_WAVE) {
        int64_t a, b;
        bad |= !row_range(row_ptr, i, E, a, b);
        for (int64_t e = a + sl; e < b; e += SYM_LANES) {
            const int32_t j = dst[e];
            bool m = false;
            if (j < 0 || j >= N) {
                bad = true;
            } else {
                m = !has_edge(row_ptr, E, dst, image, j, (int32_t)i, -image[3 * e], -image[3 * e + 1],
                              -image[3 * e + 2]);
                if (m) atomicAdd(&addcnt[j], 1u);
            }
            miss[e] = m ? 1 : 0;
        }
    }
    if (ballot(bad) != 0 && lane == 0) atomicOr(&rep->flags, (uint32_t)MG_FLAG_RANGE);
}

__global__ __launch_bounds__(256) void k_sym_counts(const int64_t* __restrict__ row_ptr, int64_t N, int64_t E,
                                                    const uint32_t* __restrict__ addcnt,
                                                    uint32_t* __restrict__ total) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += stride) {
        int64_t a, b;
        row_range(row_ptr, q, E, a, b);
        total[q] = (uint32_t)(b - a) + addcnt[q];
    }
}

__global__ __launch_bounds__(256) void k_sym_bucket(const int64_t* __restrict__ row_ptr, int64_t N, int64_t E,
                                                    const int32_t* __restrict__ dst,
                                                    const uint8_t* __restrict__ miss,
                                                    const int64_t* __restrict__ aoff, uint32_t* __restrict__ cursor,
                                                    uint64_t* __restrict__ bucket) {
    const int lane = lane_id();
    const int sub = lane / SYM_LANES, sl = lane - sub * SYM_LANES;
    for (int64_t i = grid_wave() * SYM_PER_WAVE + sub; i < N; i += grid_waves() * SYM_PER_WAVE) {
        int64_t a, b;
        row_range(row_ptr, i, E, a, b);
        for (int64_t e = a + sl; e < b; e += SYM_LANES) {
            if (!miss[e]) continue;
            const int32_t j = dst[e];
            const uint32_t slot = atomicAdd(&cursor[j], 1u);
            bucket[aoff[j] + slot] = ((uint64_t)e << 32) | (uint64_t)(uint32_t)i;
        }
    }
}

__global__ __launch_bounds__(256) void k_sym_fill(const int64_t* __restrict__ row_ptr, int64_t N, int64_t E,
                                                  const int32_t* __restrict__ dst, const int32_t* __restrict__ image,
                                                  const float* __restrict__ length,
                                                  const uint32_t* __restrict__ addcnt,
                                                  const int64_t* __restrict__ aoff,
                                                  const uint64_t* __restrict__ bucket,
                                                  const int64_t* __restrict__ out_off, int64_t capacity,
                                                  int32_t* __restrict__ osrc, int32_t* __restrict__ odst,
                                                  int32_t* __restrict__ oimg, float* __restrict__ olen) {
    const int lane = lane_id();
    const int sub = lane / SYM_LANES, sl = lane - sub * SYM_LANES;
    for (int64_t i = grid_wave() * SYM_PER_WAVE + sub; i < N; i += grid_waves() * SYM_PER_WAVE) {
        int64_t a, b;
        row_range(row_ptr, i, E, a, b);
        const int64_t d = b - a;
        const int64_t o0 = out_off[i];
        for (int64_t q = sl; q < d; q += SYM_LANES) {
            const int64_t o = o0 + q, e = a + q;
            if (o >= capacity) break;
            osrc[o] = (int32_t)i;
            odst[o] = dst[e];
            oimg[3 * o] = image[3 * e];
            oimg[3 * o + 1] = image[3 * e + 1];
            oimg[3 * o + 2] = image[3 * e + 2];
            if (olen) olen[o] = length[e];
        }
        const uint32_t c = addcnt[i];
        const uint64_t* bk = bucket + aoff[i];
        for (uint32_t r = sl; r < c; r += SYM_LANES) {
            const uint64_t key = bk[r];
            uint32_t rank = 0;
            for (uint32_t s = 0; s < c; ++s) rank += bk[s] < key ? 1u : 0u;
            const int64_t o = o0 + d + rank;
            if (o >= capacity) continue;
            const int64_t e = (int64_t)(key >> 32);
            osrc[o] = (int32_t)i;
            odst[o] = (int32_t)(uint32_t)key;
            oimg[3 * o] = -image[3 * e];
            oimg[3 * o + 1] = -image[3 * e + 1];
            oimg[3 * o + 2] = -image[3 * e + 2];
            if (olen) olen[o] = length[e];
        }
    }
}

hipError_t launch_symmetrize(const int64_t* row_ptr, int64_t N, int64_t E, const int32_t* dst, const int32_t* image,
                             const float* length, int64_t capacity, int32_t* osrc, int32_t* odst, int32_t* oimg,
                             float* olen, int64_t* out_off, const SymWs& w, mg_report* report, hipStream_t s) {
    const int cu = device_cu_count();
    const int g = cu * 8;
    // the per-source passes: four sources per wave, grid up to four times what
    // stays resident (the hardware dispatcher refills)
    const int gs = (int)std::max<int64_t>(1, std::min<int64_t>((N + 4 * SYM_PER_WAVE - 1) / (4 * SYM_PER_WAVE),
                                                               (int64_t)cu * 32));
    if (N > 0) {
        hipLaunchKernelGGL(k_sym_zero, dim3(g), dim3(256), 0, s, w.addcnt, w.cursor, N);
        hipLaunchKernelGGL(k_sym_mark, dim3(gs), dim3(256), 0, s, row_ptr, N, E, dst, image, w.miss, w.addcnt, report);
        hipLaunchKernelGGL(k_sym_counts, dim3(g), dim3(256), 0, s, row_ptr, N, E, w.addcnt, w.total);
    }
    hipError_t e = launch_scan_counts(w.addcnt, N, w.aoff, w.bsum, INT64_MAX, nullptr, s);
    if (e != hipSuccess) return e;
    e = launch_scan_counts(w.total, N, out_off, w.bsum, capacity, report, s);
    if (e != hipSuccess || N == 0) return e;
    hipLaunchKernelGGL(k_sym_bucket, dim3(gs), dim3(256), 0, s, row_ptr, N, E, dst, w.miss, w.aoff, w.cursor, w.bucket);
    hipLaunchKernelGGL(k_sym_fill, dim3(gs), dim3(256), 0, s, row_ptr, N, E, dst, image, length, w.addcnt, w.aoff,
                       w.bucket, out_off, capacity, osrc, odst, oimg, olen);
    return hipGetLastError();
}

}  // namespace mg

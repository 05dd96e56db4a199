// Edge geometry and its backward pass.
//
// v_e = (x_dst - x_src + t_e) L and l_e = ||v_e|| are the quantities inside the
// norm of Definition def6. The backward pass (edge set held fixed) is what lets
// a generative model move the geometry and rebuild the graph inside its
// forward pass (abstract; Sec. 4):
//   g_e = g_v + g_l v / l (0 when l = 0),
//   grad_x[dst] += g L^T, grad_x[src] -= g L^T, grad_L[s] += f^T g.
// Both kernels are bound by HBM traffic on the per-edge arrays; the per-edge
// arithmetic is done in FP64 (full rate on CDNA) so that thin cells with large
// image offsets lose no accuracy, and results are stored in FP32.
#include "mg_internal.h"

namespace mg {

namespace {

__device__ inline int64_t edge_count(int64_t E, const int64_t* __restrict__ num_edges) {
    if (num_edges == nullptr) return E;
    const int64_t d = *num_edges;
    return d < E ? (d < 0 ? 0 : d) : E;
}

}  // namespace

__global__ __launch_bounds__(256) void k_geom_fwd(const float* __restrict__ lattices,
                                                  const float* __restrict__ frac,
                                                  const int32_t* __restrict__ atom_struct, int64_t N,
                                                  const int32_t* __restrict__ src,
                                                  const int32_t* __restrict__ dst,
                                                  const int32_t* __restrict__ image, int64_t E,
                                                  const int64_t* __restrict__ num_edges,
                                                  float* __restrict__ vec, float* __restrict__ length) {
    const int64_t Ee = edge_count(E, num_edges);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < Ee; e += stride) {
        const int32_t i = src[e], j = dst[e];
        double v0 = __builtin_nan(""), v1 = v0, v2 = v0;
        if (i >= 0 && j >= 0 && i < N && j < N) {
            const float* L = lattices + 9 * (int64_t)atom_struct[i];
            const double f0 = (double)frac[3 * (int64_t)j] - (double)frac[3 * (int64_t)i] + (double)image[3 * e];
            const double f1 = (double)frac[3 * (int64_t)j + 1] - (double)frac[3 * (int64_t)i + 1] + (double)image[3 * e + 1];
            const double f2 = (double)frac[3 * (int64_t)j + 2] - (double)frac[3 * (int64_t)i + 2] + (double)image[3 * e + 2];
            v0 = f0 * (double)L[0] + f1 * (double)L[3] + f2 * (double)L[6];
            v1 = f0 * (double)L[1] + f1 * (double)L[4] + f2 * (double)L[7];
            v2 = f0 * (double)L[2] + f1 * (double)L[5] + f2 * (double)L[8];
        }
        if (vec) {
            vec[3 * e] = (float)v0;
            vec[3 * e + 1] = (float)v1;
            vec[3 * e + 2] = (float)v2;
        }
        if (length) length[e] = (float)sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    }
}

__global__ __launch_bounds__(256) void k_zero_f32(float* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = 0.0f;
}

__global__ __launch_bounds__(256) void k_zero_f64(double* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = 0.0;
}

// Backward pass. Each workgroup takes a contiguous range of edges and walks it
// 256 edges at a time (64 per wave).
// - Destination side: coordinate gradients go to an LDS window of GB_WIN atoms
//   (FP32 LDS atomics) that follows the edges; when a step touches atoms
//   outside the window, the touched part is flushed to global memory with FP32
//   atomics and the window moves. A step spanning more atoms than the window
//   uses global atomics directly.
// - Source side and lattice: edges grouped by source give every wave long runs
//   of one source and one structure, so each lane keeps running sums in
//   registers for the wave's current source (3 FP32) and structure (9 FP64)
//   and the wave reduces and flushes them (global atomics) only when the run
//   ends; a step that mixes sources (or structures) flushes and falls back to
//   per-lane atomics for that step.
constexpr int GB_WIN = 2048;

__global__ __launch_bounds__(256) void k_geom_bwd(const float* __restrict__ lattices,
                                                  const float* __restrict__ frac,
                                                  const int32_t* __restrict__ atom_struct, int64_t N,
                                                  const int32_t* __restrict__ src,
                                                  const int32_t* __restrict__ dst,
                                                  const int32_t* __restrict__ image, int64_t E,
                                                  const int64_t* __restrict__ num_edges,
                                                  const float* __restrict__ gvec,
                                                  const float* __restrict__ glen,
                                                  float* __restrict__ grad_frac,
                                                  double* __restrict__ acc) {
    __shared__ float win[GB_WIN * 3];
    __shared__ int s_lo[4], s_hi[4];
    const int64_t Ee = edge_count(E, num_edges);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t per = ((Ee + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
    const int64_t e0 = (int64_t)blockIdx.x * per;
    const int64_t e1 = min(Ee, e0 + per);
    for (int q = tid; q < GB_WIN * 3; q += 256) win[q] = 0.0f;
    int64_t wb = -1;              // window base atom (block-uniform), -1: no window
    int tlo = GB_WIN, thi = -1;   // touched local range of the window
    int32_t src_cur = -1;         // wave's current source run (uniform), -1: none
    float sa0 = 0.f, sa1 = 0.f, sa2 = 0.f;
    int32_t st_cur = -1;          // wave's current structure run (uniform), -1: none
    double la[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) la[q] = 0.0;
    __syncthreads();
    auto flush_window = [&]() {
        __syncthreads();   // every LDS atomic of the previous steps is done
        if (wb >= 0 && thi >= tlo) {
            for (int q = tlo * 3 + tid; q < (thi + 1) * 3; q += 256) {
                const float v = win[q];
                if (v != 0.0f) unsafeAtomicAdd(&grad_frac[wb * 3 + q], v);
                win[q] = 0.0f;
            }
        }
        __syncthreads();
    };
    auto flush_src = [&]() {
        if (src_cur >= 0) {
            const float r0 = wave_sum_f32(sa0), r1 = wave_sum_f32(sa1), r2 = wave_sum_f32(sa2);
            if (lane == 0) {
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)src_cur], r0);
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)src_cur + 1], r1);
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)src_cur + 2], r2);
            }
        }
        sa0 = sa1 = sa2 = 0.f;
    };
    auto flush_lat = [&]() {
        if (st_cur >= 0) {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const double t = wave_sum_f64(la[q]);
                if (lane == 0) unsafeAtomicAdd(&acc[9 * (int64_t)st_cur + q], t);
            }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) la[q] = 0.0;
    };
    for (int64_t base = e0; base < e1; base += 256) {
        const int64_t e = base + tid;
        int32_t i = 0, j = 0, s = 0;
        bool act = e < e1;
        double f0 = 0, f1 = 0, f2 = 0, g0 = 0, g1 = 0, g2 = 0;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if (act) {
            i = src[e];
            j = dst[e];
            act = i >= 0 && j >= 0 && i < N && j < N;
        }
        if (act) {
            s = atom_struct[i];
            const float* L = lattices + 9 * (int64_t)s;
            f0 = (double)frac[3 * (int64_t)j] - (double)frac[3 * (int64_t)i] + (double)image[3 * e];
            f1 = (double)frac[3 * (int64_t)j + 1] - (double)frac[3 * (int64_t)i + 1] + (double)image[3 * e + 1];
            f2 = (double)frac[3 * (int64_t)j + 2] - (double)frac[3 * (int64_t)i + 2] + (double)image[3 * e + 2];
            const double v0 = f0 * (double)L[0] + f1 * (double)L[3] + f2 * (double)L[6];
            const double v1 = f0 * (double)L[1] + f1 * (double)L[4] + f2 * (double)L[7];
            const double v2 = f0 * (double)L[2] + f1 * (double)L[5] + f2 * (double)L[8];
            if (gvec) {
                g0 = gvec[3 * e];
                g1 = gvec[3 * e + 1];
                g2 = gvec[3 * e + 2];
            }
            if (glen) {
                const double l = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
                const double c = l > 0.0 ? (double)glen[e] / l : 0.0;
                g0 += c * v0;
                g1 += c * v1;
                g2 += c * v2;
            }
            // g L^T: component k is g . (row k of L)
            x0 = (float)(g0 * (double)L[0] + g1 * (double)L[1] + g2 * (double)L[2]);
            x1 = (float)(g0 * (double)L[3] + g1 * (double)L[4] + g2 * (double)L[5]);
            x2 = (float)(g0 * (double)L[6] + g1 * (double)L[7] + g2 * (double)L[8]);
        }
        if (grad_frac) {
            // ---- destination side: LDS window (block-uniform decisions)
            int lo = act ? j : INT32_MAX, hi = act ? j : -1;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                lo = min(lo, __shfl_xor(lo, d, WAVE));
                hi = max(hi, __shfl_xor(hi, d, WAVE));
            }
            if (lane == 0) {
                s_lo[wv] = lo;
                s_hi[wv] = hi;
            }
            __syncthreads();
            lo = min(min(s_lo[0], s_lo[1]), min(s_lo[2], s_lo[3]));
            hi = max(max(s_hi[0], s_hi[1]), max(s_hi[2], s_hi[3]));
            __syncthreads();
            if (hi >= 0) {
                if (hi - lo + 1 > GB_WIN) {
                    if (act) {
                        unsafeAtomicAdd(&grad_frac[3 * (int64_t)j], x0);
                        unsafeAtomicAdd(&grad_frac[3 * (int64_t)j + 1], x1);
                        unsafeAtomicAdd(&grad_frac[3 * (int64_t)j + 2], x2);
                    }
                } else {
                    if (wb < 0 || lo < wb || hi >= wb + GB_WIN) {
                        flush_window();
                        wb = lo;
                        tlo = GB_WIN;
                        thi = -1;
                    }
                    tlo = min(tlo, (int)(lo - wb));
                    thi = max(thi, (int)(hi - wb));
                    if (act) {
                        const int lj = 3 * (int)(j - wb);
                        unsafeAtomicAdd(&win[lj], x0);
                        unsafeAtomicAdd(&win[lj + 1], x1);
                        unsafeAtomicAdd(&win[lj + 2], x2);
                    }
                }
            }
            // ---- source side: per-lane running sums over the wave's source run
            const uint64_t am = ballot(act);
            const int fl = am ? __builtin_ctzll(am) : 0;
            const int32_t iu = am ? __builtin_amdgcn_readlane(i, fl) : -1;
            const bool uni = iu >= 0 && ballot(act && i != iu) == 0;
            if (!(uni && iu == src_cur)) {
                flush_src();
                src_cur = uni ? iu : -1;
            }
            if (src_cur >= 0) {
                sa0 -= x0;
                sa1 -= x1;
                sa2 -= x2;
            } else if (act) {
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)i], -x0);
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)i + 1], -x1);
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)i + 2], -x2);
            }
        }
        if (acc) {
            const double F[3] = {f0, f1, f2}, Gv[3] = {g0, g1, g2};
            const uint64_t am = ballot(act);
            const int fl = am ? __builtin_ctzll(am) : 0;
            const int32_t su = am ? __builtin_amdgcn_readlane(s, fl) : -1;
            const bool uni = su >= 0 && ballot(act && s != su) == 0;
            if (!(uni && su == st_cur)) {
                flush_lat();
                st_cur = uni ? su : -1;
            }
            if (st_cur >= 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) la[3 * a + b] += F[a] * Gv[b];
            } else if (act) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) unsafeAtomicAdd(&acc[9 * (int64_t)s + 3 * a + b], F[a] * Gv[b]);
            }
        }
    }
    if (grad_frac) {
        flush_src();
        flush_window();
    }
    if (acc) flush_lat();
}

__global__ __launch_bounds__(256) void k_finalize_lattice(const double* __restrict__ acc, int64_t n,
                                                          float* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = (float)acc[q];
}

static int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_geometry_fwd(const float* lattices, const float* frac, const int32_t* atom_struct,
                               int64_t N, const int32_t* src, const int32_t* dst,
                                 const int32_t* image, int64_t E, const int64_t* num_edges,
                                 float* vec, float* length, hipStream_t s) {
    if (E == 0) return hipSuccess;
    const int grid = grid_for(E, 256, device_cu_count() * 16);
    hipLaunchKernelGGL(k_geom_fwd, dim3(grid), dim3(256), 0, s, lattices, frac, atom_struct, N, src,
                       dst, image, E, num_edges, vec, length);
    return hipGetLastError();
}

hipError_t launch_geometry_bwd(const float* lattices, const float* frac, const int32_t* atom_struct,
                               int B, int64_t N, const int32_t* src, const int32_t* dst,
                               const int32_t* image, int64_t E, const int64_t* num_edges,
                               const float* grad_vec, const float* grad_length, float* grad_frac,
                               float* grad_lattice, double* acc, hipStream_t s) {
    const int cu = device_cu_count();
    if (grad_frac && N > 0)
        hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(3 * N, 256, cu * 4)), dim3(256), 0, s, grad_frac, 3 * N);
    if (grad_lattice && B > 0)
        hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(9 * (int64_t)B, 256, cu * 4)), dim3(256), 0, s, acc,
                           9 * (int64_t)B);
    if (E > 0 && (grad_frac || grad_lattice) && (grad_vec || grad_length)) {
        const int grid = grid_for(E, 256 * 8, cu * 8);
        hipLaunchKernelGGL(k_geom_bwd, dim3(grid), dim3(256), 0, s, lattices, frac, atom_struct, N, src,
                           dst, image, E, num_edges, grad_vec, grad_length, grad_frac,
                           grad_lattice ? acc : nullptr);
    }
    if (grad_lattice && B > 0)
        hipLaunchKernelGGL(k_finalize_lattice, dim3(grid_for(9 * (int64_t)B, 256, 1 << 30)), dim3(256), 0, s,
                           acc, 9 * (int64_t)B, grad_lattice);
    return hipGetLastError();
}

}  // namespace mg

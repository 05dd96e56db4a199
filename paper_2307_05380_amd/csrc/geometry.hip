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

// Waves stay converged over their edges (lanes past the end are inactive but
// take part in the reductions). Coordinate gradients use FP32 atomics, with the
// source side summed over the wave first when all its edges share one source
// (edges grouped by source); lattice gradients are summed over the wave in FP64
// and accumulated with FP64 atomics.
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
    const int64_t Ee = edge_count(E, num_edges);
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    for (int64_t base = w0 * WAVE; base < Ee; base += waves * WAVE) {
        const int64_t e = base + lane;
        int32_t i = 0, j = 0, s = 0;
        bool act = e < Ee;
        double f0 = 0, f1 = 0, f2 = 0, g0 = 0, g1 = 0, g2 = 0;
        double x0 = 0, x1 = 0, x2 = 0;
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
            x0 = g0 * (double)L[0] + g1 * (double)L[1] + g2 * (double)L[2];
            x1 = g0 * (double)L[3] + g1 * (double)L[4] + g2 * (double)L[5];
            x2 = g0 * (double)L[6] + g1 * (double)L[7] + g2 * (double)L[8];
        }
        if (grad_frac) {
            if (act) {
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)j], (float)x0);
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)j + 1], (float)x1);
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)j + 2], (float)x2);
            }
            const int32_t i0 = __builtin_amdgcn_readfirstlane(i);
            const bool same = ballot(!act || i == i0) == ~0ull;
            if (same) {
                const double s0 = wave_sum_f64(x0), s1 = wave_sum_f64(x1), s2 = wave_sum_f64(x2);
                if (lane == 0 && ballot(act) != 0) {
                    unsafeAtomicAdd(&grad_frac[3 * (int64_t)i0], (float)-s0);
                    unsafeAtomicAdd(&grad_frac[3 * (int64_t)i0 + 1], (float)-s1);
                    unsafeAtomicAdd(&grad_frac[3 * (int64_t)i0 + 2], (float)-s2);
                }
            } else if (act) {
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)i], (float)-x0);
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)i + 1], (float)-x1);
                unsafeAtomicAdd(&grad_frac[3 * (int64_t)i + 2], (float)-x2);
            }
        }
        if (acc) {
            const double F[3] = {f0, f1, f2}, Gv[3] = {g0, g1, g2};
            const int32_t s0 = __builtin_amdgcn_readfirstlane(s);
            const bool same = ballot(!act || s == s0) == ~0ull;
            const bool any = ballot(act) != 0;
            if (same) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const double t = wave_sum_f64(act ? F[a] * Gv[b] : 0.0);
                        if (lane == 0 && any) unsafeAtomicAdd(&acc[9 * (int64_t)s0 + 3 * a + b], t);
                    }
            } else if (act) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) unsafeAtomicAdd(&acc[9 * (int64_t)s + 3 * a + b], F[a] * Gv[b]);
            }
        }
    }
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
        const int grid = grid_for(E, 256, cu * 16);
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

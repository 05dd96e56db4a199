// Cell lists for large structures (the large-cell form of the paper's
// KD-tree-like search, Sec. 1 and Sec. 2.2).
//
// A structure whose lattice planes are far apart compared with the search
// radius R is cut into m_k >= 3 bins per lattice direction, each at least R
// thick, so every neighbour within R of an atom lies in the 27 bins around the
// atom's bin (with the periodic wrap giving the image offset). Atoms are
// counting-sorted into bins (histogram, scan, scatter, then each bin sorted by
// atom index so the order is deterministic) and stored as their position
// relative to their bin's origin, in FP32 from FP64: for a source i and a
// stencil bin nb with wrap u the displacement of any atom j of nb is
//     d = (xw_j - o_nb) L + (o_nb + u - xw_i) L,   xw = x - floor(x),
// where the second term is one FP64-derived offset per (source, bin), so the
// FP32 arithmetic only ever sees lengths of a few bin widths. The image of the
// edge is t = u - floor(x_j) + floor(x_i).
#include "mg_internal.h"

namespace mg {

namespace {

__device__ __forceinline__ int ufirst(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void decode_bin(int lb, const int* m, int& b0, int& b1, int& b2) {
    b2 = lb % m[2];
    const int r = lb / m[2];
    b1 = r % m[1];
    b0 = r / m[1];
}

}  // namespace

__global__ __launch_bounds__(256) void k_cl_clear(uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                                                  int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        a[q] = 0u;
        b[q] = 0u;
    }
}

// Bin of every atom of every cell-list structure, and the bin histogram.
__global__ __launch_bounds__(256) void k_cl_count(const StructInfo* __restrict__ info,
                                                  const float* __restrict__ frac,
                                                  int32_t* __restrict__ atom_bin,
                                                  int32_t* __restrict__ atom_shift,
                                                  int32_t* __restrict__ atom_struct,
                                                  uint32_t* __restrict__ bin_count) {
    const int b = blockIdx.x;
    const StructInfo* si = info + b;
    if (si->mode != 1) return;
    const int64_t a0 = si->atom0, a1 = a0 + si->n;
    const int m0 = si->m[0], m1 = si->m[1], m2 = si->m[2];
    for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        int bk[3], sk[3];
        const int mm[3] = {m0, m1, m2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double x = (double)frac[3 * a + k];
            const double f = floor(x);
            sk[k] = (int)f;
            const int q = (int)floor((x - f) * (double)mm[k]);
            bk[k] = min(max(q, 0), mm[k] - 1);
        }
        const int lb = (bk[0] * m1 + bk[1]) * m2 + bk[2];
        atom_bin[a] = lb;
        atom_shift[a] = pack_t(max(min(sk[0], TMAX), -TMAX), max(min(sk[1], TMAX), -TMAX),
                               max(min(sk[2], TMAX), -TMAX));
        atom_struct[a] = b;
        atomicAdd(&bin_count[si->bin_off + lb], 1u);
    }
}

__global__ __launch_bounds__(256) void k_cl_scatter(const StructInfo* __restrict__ info,
                                                    const int32_t* __restrict__ atom_bin,
                                                    const int64_t* __restrict__ bin_start,
                                                    uint32_t* __restrict__ bin_fill,
                                                    int32_t* __restrict__ slot_atom) {
    const int b = blockIdx.x;
    const StructInfo* si = info + b;
    if (si->mode != 1) return;
    const int64_t a0 = si->atom0, a1 = a0 + si->n;
    for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const int64_t q = si->bin_off + atom_bin[a];
        const int64_t pos = bin_start[q] + atomicAdd(&bin_fill[q], 1u);
        slot_atom[pos] = (int32_t)a;
    }
}

// Each bin's atoms in ascending atom order (insertion sort; bins are small).
__global__ __launch_bounds__(256) void k_cl_sortbins(const int64_t* __restrict__ bin_start,
                                                     const Counters* __restrict__ ctr,
                                                     int32_t* __restrict__ slot_atom) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ctr->total_bins) return;
    const int64_t s = bin_start[q], e = bin_start[q + 1];
    for (int64_t p = s + 1; p < e; ++p) {
        const int32_t v = slot_atom[p];
        int64_t r = p - 1;
        while (r >= s && slot_atom[r] > v) {
            slot_atom[r + 1] = slot_atom[r];
            --r;
        }
        slot_atom[r + 1] = v;
    }
}

// Position of every binned atom relative to its bin origin, FP64 -> FP32.
__global__ __launch_bounds__(256) void k_cl_prep(const StructInfo* __restrict__ info,
                                                 const float* __restrict__ frac,
                                                 const int32_t* __restrict__ atom_bin,
                                                 const int64_t* __restrict__ bin_start,
                                                 const int32_t* __restrict__ slot_atom,
                                                 float4* __restrict__ slot_pos) {
    const int b = blockIdx.x;
    const StructInfo* si = info + b;
    if (si->mode != 1) return;
    const int64_t p0 = bin_start[si->bin_off], p1 = bin_start[si->bin_off + si->nbins];
    double L[9];
    for (int r = 0; r < 9; ++r) L[r] = si->L[r];
    const int m[3] = {si->m[0], si->m[1], si->m[2]};
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int32_t a = slot_atom[p];
        int bk[3];
        decode_bin(atom_bin[a], m, bk[0], bk[1], bk[2]);
        double f[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double x = (double)frac[3 * (int64_t)a + k];
            f[k] = (x - floor(x)) - (double)bk[k] / (double)m[k];
        }
        slot_pos[p] = make_float4((float)(f[0] * L[0] + f[1] * L[3] + f[2] * L[6]),
                                  (float)(f[0] * L[1] + f[1] * L[4] + f[2] * L[7]),
                                  (float)(f[0] * L[2] + f[1] * L[5] + f[2] * L[8]), __int_as_float(a));
    }
}

// Exclusive scan of the bin histogram over the batch's bins (device count).
__global__ __launch_bounds__(256) void k_cl_scan_sums(const uint32_t* __restrict__ cnt,
                                                      const Counters* __restrict__ ctr,
                                                      int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[4];
    const int64_t n = ctr->total_bins;
    const int64_t base = (int64_t)blockIdx.x * 2048;
    int64_t s = 0;
    if (base < n) {
        for (int k = 0; k < 8; ++k) {
            const int64_t idx = base + k * 256 + threadIdx.x;
            if (idx < n) s += cnt[idx];
        }
    }
    s = wave_sum_i64(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(256) void k_cl_scan_final(const uint32_t* __restrict__ cnt,
                                                       const Counters* __restrict__ ctr,
                                                       const int64_t* __restrict__ bsum,
                                                       int64_t* __restrict__ start) {
    __shared__ int64_t sh[4], swave[4];
    const int64_t n = ctr->total_bins;
    const int64_t base0 = (int64_t)blockIdx.x * 2048;
    if (base0 > n) return;     // uniform per block
    int64_t p = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) p += bsum[b];
    p = wave_sum_i64(p);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = p;
    __syncthreads();
    p = sh[0] + sh[1] + sh[2] + sh[3];
    const int64_t base = base0 + (int64_t)threadIdx.x * 8;
    uint32_t v[8];
    int64_t tsum = 0;
    for (int k = 0; k < 8; ++k) {
        v[k] = (base + k < n) ? cnt[base + k] : 0u;
        tsum += v[k];
    }
    const int64_t inc = wave_incl_scan_i64(tsum);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) swave[w] = inc;
    __syncthreads();
    int64_t excl = p + inc - tsum;
    for (int q = 0; q < w; ++q) excl += swave[q];
    for (int k = 0; k < 8; ++k) {
        if (base + k <= n) start[base + k] = excl;   // start[n] = total
        excl += v[k];
    }
}

hipError_t launch_cl_build(int B, int64_t N, const float* frac, const int64_t* batch_ptr,
                           const StructInfo* info, const ClWs& w, hipStream_t s) {
    (void)batch_ptr;
    if (B == 0 || N == 0) return hipSuccess;
    const int cu = device_cu_count();
    const int64_t nb = (w.cap + 2047) / 2048;
    int g = (int)((w.cap + 255) / 256);
    hipLaunchKernelGGL(k_cl_clear, dim3(g < cu * 8 ? g : cu * 8), dim3(256), 0, s, w.bin_count, w.bin_fill, w.cap);
    hipLaunchKernelGGL(k_cl_count, dim3(B), dim3(256), 0, s, info, frac, w.atom_bin, w.atom_shift, w.atom_struct,
                       w.bin_count);
    Counters* ctr = w.ctr;
    hipLaunchKernelGGL(k_cl_scan_sums, dim3((unsigned)nb), dim3(256), 0, s, w.bin_count, ctr, w.bsum);
    hipLaunchKernelGGL(k_cl_scan_final, dim3((unsigned)nb), dim3(256), 0, s, w.bin_count, ctr, w.bsum, w.bin_start);
    hipLaunchKernelGGL(k_cl_scatter, dim3(B), dim3(256), 0, s, info, w.atom_bin, w.bin_start, w.bin_fill,
                       w.slot_atom);
    hipLaunchKernelGGL(k_cl_sortbins, dim3((unsigned)((w.cap + 255) / 256)), dim3(256), 0, s, w.bin_start, ctr,
                       w.slot_atom);
    hipLaunchKernelGGL(k_cl_prep, dim3(B), dim3(256), 0, s, info, frac, w.atom_bin, w.bin_start, w.slot_atom,
                       w.slot_pos);
    return hipGetLastError();
}

// ------------------------------------------------------- cutoff sweep (cells)

// One wave per source; the 27 stencil bins are visited as 9 rows of 3 bins along
// the third lattice direction. Without a wrap in that direction the three bins
// are contiguous in bin order, so one lane range covers them (each lane finds
// its bin from the two inner boundaries); at the cell boundary the three bins
// are visited one by one. Hits are ranked with ballot + mbcnt; the count and
// fill passes enumerate candidates in the same order.
template <int MODE>
__global__ __launch_bounds__(256) void k_cl_sweep(int B, const StructInfo* __restrict__ info, ClWs w,
                                                  const float* __restrict__ frac, float c2thr,
                                                  const float* __restrict__ thr,
                                                  uint32_t* __restrict__ counts,
                                                  const int64_t* __restrict__ offsets, int64_t capacity,
                                                  int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                  int32_t* __restrict__ image, float* __restrict__ length,
                                                  float* __restrict__ vec,
                                                  Counters* __restrict__ ctr, mg_report* __restrict__ rep,
                                                  int64_t* __restrict__ partials) {
    const int lane = lane_id();
    const int64_t total = w.cl_off[B];
    int64_t wave_cand = 0;
    for (int64_t q = grid_wave(); q < total; q += grid_waves()) {
        int lo = 0, hi = B;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (w.cl_off[mid] <= q) lo = mid;
            else hi = mid;
        }
        const StructInfo* si = info + lo;
        const int64_t i = si->atom0 + (q - w.cl_off[lo]);
        const float c2 = thr ? thr[i] : c2thr;   // the source's cutoff
        const int m[3] = {si->m[0], si->m[1], si->m[2]};
        double L[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) L[r] = si->L[r];
        int b0, b1, b2;
        decode_bin(ufirst(w.atom_bin[i]), m, b0, b1, b2);
        const int32_t shi = ufirst(w.atom_shift[i]);
        const int si0 = unpack_t0(shi), si1 = unpack_t1(shi), si2 = unpack_t2(shi);
        const double x0 = frac[3 * i], x1 = frac[3 * i + 1], x2 = frac[3 * i + 2];
        const double xw0 = x0 - floor(x0), xw1 = x1 - floor(x1), xw2 = x2 - floor(x2);
        const int64_t* bst = w.bin_start + si->bin_off;
        uint32_t cnt = 0, run = 0;
        const int64_t base = (MODE == 1) ? offsets[i] : 0;
        const float stx = (float)(L[6] / m[2]), sty = (float)(L[7] / m[2]), stz = (float)(L[8] / m[2]);
        int64_t ncand = 0;
        // one lane range [p0, p3) covering bins z0 .. z0+nz-1 (same wrap u2)
        auto range = [&](int64_t p0, int64_t p1, int64_t p2, int64_t p3, int nb0, int nb1, int z0, int u0,
                         int u1, int u2) {
            const double f0 = (double)nb0 / m[0] + u0 - xw0;
            const double f1 = (double)nb1 / m[1] + u1 - xw1;
            const double f2 = (double)z0 / m[2] + u2 - xw2;
            const float qx = (float)(f0 * L[0] + f1 * L[3] + f2 * L[6]);
            const float qy = (float)(f0 * L[1] + f1 * L[4] + f2 * L[7]);
            const float qz = (float)(f0 * L[2] + f1 * L[5] + f2 * L[8]);
            ncand += p3 - p0;
            for (int64_t pb = p0; pb < p3; pb += WAVE) {
                const int64_t p = pb + lane;
                bool hit = false;
                float l2 = 0.0f, dx = 0.0f, dy = 0.0f, dz = 0.0f;
                int32_t j = -1;
                if (p < p3) {
                    const float4 e = w.slot_pos[p];
                    j = __float_as_int(e.w);
                    const float kz = (float)((p >= p1) + (p >= p2));
                    dx = e.x + fmaf(kz, stx, qx);
                    dy = e.y + fmaf(kz, sty, qy);
                    dz = e.z + fmaf(kz, stz, qz);
                    l2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    hit = l2 < c2 && (int64_t)j != i;
                }
                if (MODE == 0) {
                    cnt += hit ? 1u : 0u;
                } else {
                    const uint64_t msk = ballot(hit);
                    if (hit) {
                        const int64_t e = base + run + mbcnt(msk);
                        if (e < capacity) {
                            const int32_t shj = w.atom_shift[j];
                            dst[e] = j;   // (src comes from row_ptr after the fill)
                            image[3 * e] = u0 - unpack_t0(shj) + si0;
                            image[3 * e + 1] = u1 - unpack_t1(shj) + si1;
                            image[3 * e + 2] = u2 - unpack_t2(shj) + si2;
                            length[e] = sqrtf(l2);
                            if (vec) {
                                vec[3 * e] = dx;
                                vec[3 * e + 1] = dy;
                                vec[3 * e + 2] = dz;
                            }
                        }
                    }
                    run += (uint32_t)__popcll(msk);
                }
            }
        };
        for (int r = 0; r < 9; ++r) {
            int nb0 = b0 + r / 3 - 1, nb1 = b1 + r % 3 - 1;
            const int u0 = nb0 < 0 ? -1 : (nb0 >= m[0] ? 1 : 0);
            const int u1 = nb1 < 0 ? -1 : (nb1 >= m[1] ? 1 : 0);
            nb0 -= u0 * m[0];
            nb1 -= u1 * m[1];
            const int row = (nb0 * m[1] + nb1) * m[2];
            if (b2 >= 1 && b2 <= m[2] - 2) {
                const int64_t p0 = bst[row + b2 - 1], p1 = bst[row + b2], p2 = bst[row + b2 + 1],
                              p3 = bst[row + b2 + 2];
                range(p0, p1, p2, p3, nb0, nb1, b2 - 1, u0, u1, 0);
            } else {
                for (int dz = -1; dz <= 1; ++dz) {
                    int z = b2 + dz;
                    const int u2 = z < 0 ? -1 : (z >= m[2] ? 1 : 0);
                    z -= u2 * m[2];
                    const int64_t p0 = bst[row + z], p3 = bst[row + z + 1];
                    range(p0, p3, p3, p3, nb0, nb1, z, u0, u1, u2);
                }
            }
        }
        if (MODE == 0) {
            const int tot = wave_incl_scan_i32((int)cnt);
            if (lane == WAVE - 1) counts[i] = (uint32_t)tot;
            wave_cand += ncand;
        }
    }
    if (MODE == 0 && lane == 0) partials[grid_wave()] = wave_cand;
}

hipError_t launch_cl_cutoff_sweep(int mode, int B, const StructInfo* info, const ClWs& w,
                                  const float* frac, float c2thr, const float* thr, uint32_t* counts,
                                  const int64_t* offsets, int64_t capacity, int32_t* src,
                                  int32_t* dst, int32_t* image, float* length, float* vec, Counters* ctr,
                                  mg_report* report, int64_t* partials, int grid, hipStream_t s) {
    if (B == 0) return hipSuccess;
    if (mode == 0)
        hipLaunchKernelGGL((k_cl_sweep<0>), dim3(grid), dim3(256), 0, s, B, info, w, frac, c2thr, thr, counts, offsets,
                           capacity, src, dst, image, length, vec, ctr, report, partials);
    else
        hipLaunchKernelGGL((k_cl_sweep<1>), dim3(grid), dim3(256), 0, s, B, info, w, frac, c2thr, thr, counts, offsets,
                           capacity, src, dst, image, length, vec, ctr, report, partials);
    return hipGetLastError();
}

}  // namespace mg

// Cell lists for large structures (the large-cell form of the paper's
// KD-tree-like search, Sec. 1 and Sec. 2.2).
//
// A structure whose lattice planes are far apart compared with the search
// radius R is cut into m_k >= 3 bins per lattice direction, each at least R
// thick, so every neighbour within R of an atom lies in the 27 bins around the
// atom's bin (with the periodic wrap giving the image offset). Atoms are
// counting-sorted into bins (histogram whose atomic also gives each atom its
// arrival slot, scan, scatter, then each bin put in ascending atom order so the
// result does not depend on timing), and the bin-ordered raw coordinates and
// floor(x) are what the sweeps stage: one workgroup per home bin loads the 27
// stencil bins into LDS once and sweeps every atom of the home bin against
// them (cl_tile.h). The image of an edge is t = u - floor(x_j) + floor(x_i),
// u the stencil bin's periodic wrap.
#include <algorithm>

#include "cl_tile.h"

namespace mg {


__global__ __launch_bounds__(256) void k_cl_clear(uint32_t* __restrict__ a, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) a[q] = 0u;
}

// Bin of every atom of every cell-list structure, the bin histogram and the
// atom's arrival order in its bin (the histogram atomic's old value). Grid:
// blockIdx.x = structure, blockIdx.y strides over its atoms.
__global__ __launch_bounds__(256) void k_cl_count(const StructInfo* __restrict__ info,
                                                  const float* __restrict__ frac,
                                                  int32_t* __restrict__ atom_bin,
                                                  int32_t* __restrict__ atom_rank,
                                                  int32_t* __restrict__ atom_struct,
                                                  uint32_t* __restrict__ bin_count) {
    const int b = blockIdx.x;
    const StructInfo* si = info + b;
    if (si->mode != 1) return;
    const int64_t a0 = si->atom0, a1 = a0 + si->n;
    const int mm[3] = {si->m[0], si->m[1], si->m[2]};
    for (int64_t a = a0 + (int64_t)blockIdx.y * blockDim.x + threadIdx.x; a < a1;
         a += (int64_t)gridDim.y * blockDim.x) {
        int bk[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double x = (double)frac[3 * a + k];
            const int q = (int)floor((x - floor(x)) * (double)mm[k]);
            bk[k] = min(max(q, 0), mm[k] - 1);
        }
        const int lb = (bk[0] * mm[1] + bk[1]) * mm[2] + bk[2];
        atom_bin[a] = lb;
        atom_struct[a] = b;
        atom_rank[a] = (int32_t)atomicAdd(&bin_count[si->bin_off + lb], 1u);
    }
}

__global__ __launch_bounds__(256) void k_cl_scatter(const StructInfo* __restrict__ info,
                                                    const int32_t* __restrict__ atom_bin,
                                                    const int32_t* __restrict__ atom_rank,
                                                    const int64_t* __restrict__ bin_start,
                                                    int32_t* __restrict__ slot_atom) {
    const int b = blockIdx.x;
    const StructInfo* si = info + b;
    if (si->mode != 1) return;
    const int64_t a0 = si->atom0, a1 = a0 + si->n;
    for (int64_t a = a0 + (int64_t)blockIdx.y * blockDim.x + threadIdx.x; a < a1;
         a += (int64_t)gridDim.y * blockDim.x)
        slot_atom[bin_start[si->bin_off + atom_bin[a]] + atom_rank[a]] = (int32_t)a;
}

// Every bin in ascending atom order, with the atoms' raw coordinates and
// packed floor(x) written in that order (the arrays the sweeps stage). One
// wave per bin: the rank of an atom is the number of smaller atom indices in
// the bin, counted over the bin (lanes hold up to 64 atoms; larger bins count
// over global memory, a quadratic but rare case).
__global__ __launch_bounds__(256) void k_cl_sort(const int64_t* __restrict__ bin_start,
                                                 const Counters* __restrict__ ctr,
                                                 const int32_t* __restrict__ slot_atom,
                                                 const float* __restrict__ frac,
                                                 float4* __restrict__ slot_x,
                                                 int32_t* __restrict__ slot_shift) {
    const int lane = lane_id();
    const int64_t nb = ctr->total_bins;
    auto put = [&](int64_t pos, int32_t a) {
        const float x0 = frac[3 * (int64_t)a], x1 = frac[3 * (int64_t)a + 1], x2 = frac[3 * (int64_t)a + 2];
        slot_x[pos] = make_float4(x0, x1, x2, __int_as_float(a));
        slot_shift[pos] = pack_t((int)floorf(x0), (int)floorf(x1), (int)floorf(x2));
    };
    for (int64_t q = grid_wave(); q < nb; q += grid_waves()) {
        const int64_t s = uniform64(bin_start[q]);
        const int cnt = __builtin_amdgcn_readfirstlane((int)(bin_start[q + 1] - s));
        if (cnt <= WAVE) {
            const int32_t a = lane < cnt ? slot_atom[s + lane] : INT32_MAX;
            int rank = 0;
            for (int m = 0; m < cnt; ++m) rank += __builtin_amdgcn_readlane(a, m) < a ? 1 : 0;
            if (lane < cnt) put(s + rank, a);
        } else {
            for (int r = lane; r < cnt; r += WAVE) {
                const int32_t a = slot_atom[s + r];
                int rank = 0;
                for (int m = 0; m < cnt; ++m) rank += slot_atom[s + m] < a ? 1 : 0;
                put(s + rank, a);
            }
        }
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
    const int g = (int)std::min<int64_t>((w.cap + 255) / 256, (int64_t)cu * 8);
    // per-structure kernels: enough blocks per structure for the average size
    const int per = (int)std::min<int64_t>(std::max<int64_t>((N / B + 255) / 256, 1), 64);
    hipLaunchKernelGGL(k_cl_clear, dim3(g), dim3(256), 0, s, w.bin_count, w.cap);
    hipLaunchKernelGGL(k_cl_count, dim3(B, per), dim3(256), 0, s, info, frac, w.atom_bin, w.atom_rank, w.atom_struct,
                       w.bin_count);
    Counters* ctr = w.ctr;
    hipLaunchKernelGGL(k_cl_scan_sums, dim3((unsigned)nb), dim3(256), 0, s, w.bin_count, ctr, w.bsum);
    hipLaunchKernelGGL(k_cl_scan_final, dim3((unsigned)nb), dim3(256), 0, s, w.bin_count, ctr, w.bsum, w.bin_start);
    hipLaunchKernelGGL(k_cl_scatter, dim3(B, per), dim3(256), 0, s, info, w.atom_bin, w.atom_rank, w.bin_start,
                       w.slot_atom);
    const int gs = (int)std::min<int64_t>((w.cap + 3) / 4, (int64_t)cu * 16);
    hipLaunchKernelGGL(k_cl_sort, dim3(gs), dim3(256), 0, s, w.bin_start, ctr, w.slot_atom, frac, w.slot_x,
                       w.slot_shift);
    return hipGetLastError();
}

// ------------------------------------------------------- cutoff sweep (cells)

// Count and fill over cell-list tiles: one workgroup per home bin (items
// handed out cyclically over a persistent grid), the stencil staged once, one
// wave per source of the home bin, lane = candidate. The count pass writes
// every source's edge count; after the scan the fill pass repeats the sweep
// and writes each hit at offsets[src] + (its rank among the source's hits),
// ranked with a wave ballot and mbcnt, with 32-bit offsets from a per-source
// scalar base. A candidate whose staged distance lies within a relative 1e-4
// of the threshold (far above the staged form's rounding) is decided, and
// written, in the form the image sweeps use (canon_vec): the edge set does not
// depend on the bins or on which sweep built it.
constexpr float CL_BAND = 1e-4f;

template <int MODE>
__global__ __launch_bounds__(256) void k_cl_sweep(int B, const StructInfo* __restrict__ info, ClWs w,
                                                  const float* __restrict__ frac,
                                                  float c2thr, const float* __restrict__ thr,
                                                  uint32_t* __restrict__ counts,
                                                  const int64_t* __restrict__ offsets, int64_t capacity,
                                                  int32_t* __restrict__ dst, int32_t* __restrict__ image,
                                                  float* __restrict__ length, float* __restrict__ vec,
                                                  int64_t* __restrict__ partials) {
    __shared__ ClTile tile;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t total = w.cl_off[B];
    int64_t wave_cand = 0;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        ClItem it;
        cl_stage(q, B, info, w, tile, it);
        const int T = it.total;
        for (int64_t r = it.hs + wv; r < it.he; r += 4) {
            const ClSource S = cl_source(it, w, r);
            const float c2 = thr ? thr[S.i] : c2thr;   // the source's cutoff
            const int s0 = unpack_t0(S.sh), s1 = unpack_t1(S.sh), s2 = unpack_t2(S.sh);
            uint32_t cnt = 0, run = 0;
            int32_t* dr = nullptr;
            int32_t* ir = nullptr;
            float* lr = nullptr;
            float* vr = nullptr;
            uint32_t room = 0;
            if (MODE == 1) {   // outputs rebased at the source's first edge (wave-uniform)
                const int64_t base = uniform64(offsets[S.i]);
                const int64_t left = capacity - base;
                room = left <= 0 ? 0u : (left >= (int64_t)UINT32_MAX ? UINT32_MAX : (uint32_t)left);
                dr = dst + base;
                ir = image + 3 * base;
                lr = length + base;
                vr = vec ? vec + 3 * base : nullptr;
            }
            const int self = it.home + (int)(r - it.hs);   // the source's own candidate (excluded)
            // below lo: an edge; at or above hi: none; in between the canonical form decides
            const float lo = c2 * (1.0f - CL_BAND), hi = c2 * (1.0f + CL_BAND);
            // the hits of a step: lanes under lo, plus (rarely) the band lanes whose
            // canonical length is under the threshold (they take its vector and length)
            auto decide = [&](float l2, int32_t j, int32_t ct, int cs, float& dx, float& dy, float& dz,
                              float& l2o, bool valid) -> uint64_t {   // cs >= 0: ct is tile.ct[cs]
                const uint64_t sure = ballot(valid && l2 < lo);
                const uint64_t band = ballot(valid && l2 < hi) & ~sure;
                l2o = l2;
                if (band == 0) return sure;   // wave-uniform, the common case
                bool hit = (sure >> lane) & 1ull;
                if ((band >> lane) & 1ull) {
                    if (cs >= 0) ct = tile.ct[cs];
                    const int64_t ja = j;
                    l2o = canon_vec(it.L, (double)S.x0, (double)S.x1, (double)S.x2, (double)frac[3 * ja],
                                    (double)frac[3 * ja + 1], (double)frac[3 * ja + 2], unpack_t0(ct) + s0,
                                    unpack_t1(ct) + s1, unpack_t2(ct) + s2, dx, dy, dz);
                    hit = l2o < c2;
                }
                return ballot(hit);
            };
            auto emit = [&](uint64_t m, float dx, float dy, float dz, float l2, int32_t j, int32_t ct) {
                if (MODE == 0) {
                    cnt += (uint32_t)__popcll(m);
                } else {
                    if ((m >> lane) & 1ull) {
                        const uint32_t e = run + mbcnt(m);
                        if (e < room) {
                            const uint32_t b4 = e << 2, b12 = (e << 3) + (e << 2);
                            *(int32_t*)((char*)dr + b4) = j;   // (src comes from row_ptr after the fill)
                            int32_t* im = (int32_t*)((char*)ir + b12);
                            im[0] = unpack_t0(ct) + s0;
                            im[1] = unpack_t1(ct) + s1;
                            im[2] = unpack_t2(ct) + s2;
                            *(float*)((char*)lr + b4) = sqrt_rn_finite(l2);
                            if (vr) {
                                float* v = (float*)((char*)vr + b12);
                                v[0] = dx;
                                v[1] = dy;
                                v[2] = dz;
                            }
                        }
                    }
                    run += (uint32_t)__popcll(m);
                }
            };
            if (it.staged) {   // full-wave steps over the padded tile, two per trip
                auto step = [&](int cb, const float4 e, int32_t ct) {
                    float dx = e.x - S.px, dy = e.y - S.py, dz = e.z - S.pz;
                    const float l2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    const int32_t j = __float_as_int(e.w);
                    float l2o;
                    const uint64_t m =
                        decide(l2, j, ct, MODE == 1 ? -1 : cb + lane, dx, dy, dz, l2o, true) & ~cl_self_bit(self, cb);
                    emit(m, dx, dy, dz, l2o, j, ct);
                };
                // both steps' candidates are read before the first is used (the
                // tile is padded to whole pairs of steps): one LDS wait per trip
                for (int cb = 0; cb < T; cb += 2 * WAVE) {
                    const float4 e0 = tile.c[cb + lane], e1 = tile.c[cb + WAVE + lane];
                    const int32_t c0 = MODE == 1 ? tile.ct[cb + lane] : 0;
                    const int32_t c1 = MODE == 1 ? tile.ct[cb + WAVE + lane] : 0;
                    step(cb, e0, c0);
                    if (cb + WAVE < T) step(cb + WAVE, e1, c1);   // uniform
                }
            } else {
                for (int cb = 0; cb < T; cb += WAVE) {
                    const int c = cb + lane;
                    float dx = 0.f, dy = 0.f, dz = 0.f, l2 = 0.f;
                    int32_t j = 0, ct = 0;
                    if (c < T) {
                        const float4 e = cl_candidate(tile, it, w, c, ct);
                        j = __float_as_int(e.w);
                        dx = e.x - S.px;
                        dy = e.y - S.py;
                        dz = e.z - S.pz;
                        l2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    }
                    float l2o;
                    const uint64_t m = decide(l2, j, ct, -1, dx, dy, dz, l2o, c < T) & ~cl_self_bit(self, cb);
                    emit(m, dx, dy, dz, l2o, j, ct);
                }
            }
            if (MODE == 0) {
                if (lane == 0) counts[S.i] = cnt;
                wave_cand += T;
            }
        }
        __syncthreads();   // the next item overwrites the tile
    }
    if (MODE == 0 && lane == 0) partials[grid_wave()] = wave_cand;
}

hipError_t launch_cl_cutoff_sweep(int mode, int B, const StructInfo* info, const ClWs& w,
                                  const float* frac, float c2thr, const float* thr, uint32_t* counts,
                                  const int64_t* offsets, int64_t capacity, int32_t* src,
                                  int32_t* dst, int32_t* image, float* length, float* vec, Counters* ctr,
                                  mg_report* report, int64_t* partials, int grid, hipStream_t s) {
    (void)src;
    (void)ctr;
    (void)report;
    if (B == 0) return hipSuccess;
    if (mode == 0)
        hipLaunchKernelGGL((k_cl_sweep<0>), dim3(grid), dim3(256), 0, s, B, info, w, frac, c2thr, thr, counts, offsets,
                           capacity, dst, image, length, vec, partials);
    else
        hipLaunchKernelGGL((k_cl_sweep<1>), dim3(grid), dim3(256), 0, s, B, info, w, frac, c2thr, thr, counts, offsets,
                           capacity, dst, image, length, vec, partials);
    return hipGetLastError();
}

}  // namespace mg

// Cell-list tiles shared by the cell-list sweeps (cutoff count / fill in
// celllist.hip, KNN selection in knn.hip). Internal, not part of the ABI.
//
// A work item is one home bin of a cell-list structure. Its workgroup stages
// the atoms of the (2S+1)^3 bins around it (S = 1: 27 bins, S = 2: 125 bins;
// the periodic stencil that holds every neighbour within S bin thicknesses)
// once in LDS, as positions relative to
// the home bin's origin, and then every source atom of the home bin is swept
// against the staged candidates by one wave, lane = candidate. Staged
// position of atom j in a stencil bin with periodic wrap u:
//     c_j = (x_j - floor(x_j) + u - o) L    (FP64, rounded once to FP32),
// o the home bin's fractional origin; the source's own position p_i is the same
// expression with u = 0, so d = c_j - p_i is the edge vector with t = u -
// floor(x_j) + floor(x_i), and every FP32 quantity is a rounding of an FP64
// value a few bin widths long. Candidates are in stencil order (the stencil's
// bins in a fixed order, each bin's atoms by ascending index), so the edges of
// a source come out in a deterministic order.
#pragma once

#include "mg_internal.h"

namespace mg {

constexpr int CL_TILE = 1024;   // candidates staged per item (a multiple of 128); larger stencils are read from global memory
constexpr int CL_NB_MAX = 125;  // stencil bins at most (half-width 2)

struct ClTile {
    float4 c[CL_TILE];            // staged position (x, y, z) and the atom index (bits of w)
    int32_t ct[CL_TILE];          // packed u - floor(x_j), biased 10-bit fields
    int64_t nb_start[CL_NB_MAX];  // first slot of every stencil bin
    int32_t nb_cum[CL_NB_MAX + 1];   // exclusive prefix of the stencil bins' atom counts; nb_cum[nb] = total
    int32_t nb_u[CL_NB_MAX];      // packed wrap u of every stencil bin
    int32_t wsum;                 // atom count of the first 64 stencil bins (the scan's carry)
};

struct ClItem {
    const StructInfo* si;
    double L[9];
    double o[3];       // fractional origin of the home bin
    int64_t hs, he;    // slot range of the home bin (its atoms are the item's sources)
    int32_t total;     // candidates in the stencil
    int32_t home;      // candidate index of the home bin's first atom (the stencil's centre bin, wrap 0)
    int32_t nb;        // stencil bins, (2S+1)^3
    bool staged;       // total <= CL_TILE: the candidates are in the tile
};

// A source's own candidate (distance 0) sits at candidate index home + (its slot
// - hs); this is its bit in the wave step starting at candidate cb.
__device__ __forceinline__ uint64_t cl_self_bit(int self, int cb) {
    const int sl = self - cb;
    return (sl >= 0 && sl < WAVE) ? (1ull << sl) : 0ull;
}

// Position relative to the home bin origin o (FP64, rounded once) of an atom
// with raw coordinates x and packed floor sh, seen through the wrap u; ct gets
// the packed u - floor(x).
__device__ __forceinline__ float4 cl_rel(const double* L, const double* o, const float4 x, int32_t sh, int u0,
                                         int u1, int u2, int32_t& ct) {
    const int s0 = unpack_t0(sh), s1 = unpack_t1(sh), s2 = unpack_t2(sh);
    const double f0 = ((double)x.x - (double)(s0 - u0)) - o[0];
    const double f1 = ((double)x.y - (double)(s1 - u1)) - o[1];
    const double f2 = ((double)x.z - (double)(s2 - u2)) - o[2];
    ct = pack_t(u0 - s0, u1 - s1, u2 - s2);
    return make_float4((float)(f0 * L[0] + f1 * L[3] + f2 * L[6]), (float)(f0 * L[1] + f1 * L[4] + f2 * L[7]),
                       (float)(f0 * L[2] + f1 * L[5] + f2 * L[8]), x.w);
}

// Stencil bin of concatenated candidate index c: the largest d < nb with nb_cum[d] <= c.
__device__ __forceinline__ int cl_bin_of(const ClTile& tile, int nb, int c) {
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile.nb_cum[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Candidate c of the item (0 <= c < total), from the tile or, for stencils
// larger than the tile, recomputed from the slot arrays (same arithmetic).
__device__ __forceinline__ float4 cl_candidate(const ClTile& tile, const ClItem& it, const ClWs& w, int c,
                                               int32_t& ct) {
    if (it.staged) {
        ct = tile.ct[c];
        return tile.c[c];
    }
    const int d = cl_bin_of(tile, it.nb, c);
    const int64_t p = tile.nb_start[d] + (c - tile.nb_cum[d]);
    const int32_t u = tile.nb_u[d];
    return cl_rel(it.L, it.o, w.slot_x[p], w.slot_shift[p], unpack_t0(u), unpack_t1(u), unpack_t2(u), ct);
}

// Source r (a slot of the home bin): its raw coordinates and packed floor,
// loaded once per wave (the slot is wave-uniform), and its position p_i.
struct ClSource {
    int64_t i;       // atom index
    int32_t sh;      // packed floor(x_i)
    float px, py, pz;
    float x0, x1, x2;   // raw coordinates
};

__device__ __forceinline__ ClSource cl_source(const ClItem& it, const ClWs& w, int64_t r) {
    ClSource s;
    const float4 x = w.slot_x[r];
    s.sh = __builtin_amdgcn_readfirstlane(w.slot_shift[r]);
    const float4 xu = make_float4(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x.x))),
                                  __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x.y))),
                                  __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x.z))),
                                  __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x.w))));
    int32_t ct;
    const float4 p = cl_rel(it.L, it.o, xu, s.sh, 0, 0, 0, ct);
    s.i = (int64_t)__float_as_int(xu.w);
    s.x0 = xu.x;
    s.x1 = xu.y;
    s.x2 = xu.z;
    s.px = p.x;
    s.py = p.y;
    s.pz = p.z;
    return s;
}

// Item q (a bin of the batch's cell-list bins): its structure, home bin and
// stencil, staged into the tile when it fits. Called by every thread of the
// workgroup; ends with a workgroup barrier (the tile is then complete).
__device__ __forceinline__ void cl_stage(int64_t q, int B, const StructInfo* __restrict__ info, const ClWs& w,
                                         ClTile& tile, ClItem& it) {
    const int lane = lane_id();
    const int b = __builtin_amdgcn_readfirstlane(wave_search_le(w.cl_off, B, q, lane));
    const StructInfo* si = info + b;
    it.si = si;
#pragma unroll
    for (int r = 0; r < 9; ++r) it.L[r] = si->L[r];
    const int m0 = si->m[0], m1 = si->m[1], m2 = si->m[2];
    const int lb = (int)(q - w.cl_off[b]);
    const int b2 = lb % m2, b1 = (lb / m2) % m1, b0 = lb / (m2 * m1);
    it.o[0] = (double)b0 / (double)m0;
    it.o[1] = (double)b1 / (double)m1;
    it.o[2] = (double)b2 / (double)m2;
    const int64_t* bst = w.bin_start + si->bin_off;
    it.hs = bst[lb];
    it.he = bst[lb + 1];
    // stencil bin t = (d0, d1, d2) offsets in [-S, S], d2 fastest; m_k >= 2S + 1, so one
    // periodic wrap u in {-1, 0, 1} per direction reaches every stencil bin
    const int S = si->cl_s, W = 2 * S + 1, NB = W * W * W;
    const int t = threadIdx.x;
    int cnt = 0, inc = 0;
    if (t < 2 * WAVE) {
        if (t < NB) {
            int n0 = b0 + t / (W * W) - S, n1 = b1 + (t / W) % W - S, n2 = b2 + t % W - S;
            const int u0 = n0 < 0 ? -1 : (n0 >= m0 ? 1 : 0);
            const int u1 = n1 < 0 ? -1 : (n1 >= m1 ? 1 : 0);
            const int u2 = n2 < 0 ? -1 : (n2 >= m2 ? 1 : 0);
            n0 -= u0 * m0;
            n1 -= u1 * m1;
            n2 -= u2 * m2;
            const int nbin = (n0 * m1 + n1) * m2 + n2;
            const int64_t s0 = bst[nbin];
            cnt = (int)(bst[nbin + 1] - s0);
            tile.nb_start[t] = s0;
            tile.nb_u[t] = pack_t(u0, u1, u2);
        }
        inc = wave_incl_scan_i32(cnt);
        if (t == WAVE - 1) tile.wsum = inc;
    }
    __syncthreads();
    if (t < NB) {
        const int carry = t >= WAVE ? tile.wsum : 0;
        tile.nb_cum[t] = carry + inc - cnt;
        if (t == NB - 1) tile.nb_cum[NB] = carry + inc;
    }
    __syncthreads();
    it.nb = NB;
    it.total = tile.nb_cum[NB];
    it.home = tile.nb_cum[NB / 2];
    it.staged = it.total <= CL_TILE;
    if (it.staged) {
        // the tile is filled up to a multiple of two wave widths with entries no
        // threshold accepts (infinite distance), so full-wave steps (read in pairs)
        // need no bounds test; CL_TILE is a multiple of 128
        const int padded = (it.total + 2 * WAVE - 1) / (2 * WAVE) * (2 * WAVE);
        for (int c = t; c < padded; c += blockDim.x) {
            if (c < it.total) {
                const int d = cl_bin_of(tile, NB, c);
                const int64_t p = tile.nb_start[d] + (c - tile.nb_cum[d]);
                const int32_t u = tile.nb_u[d];
                int32_t ct;
                tile.c[c] = cl_rel(it.L, it.o, w.slot_x[p], w.slot_shift[p], unpack_t0(u), unpack_t1(u),
                                   unpack_t2(u), ct);
                tile.ct[c] = ct;
            } else {
                tile.c[c] = make_float4(1e30f, 1e30f, 1e30f, __int_as_float(-1));
                tile.ct[c] = 0;
            }
        }
    }
    __syncthreads();
}

}  // namespace mg

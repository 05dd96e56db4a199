// Pair x image distance sweep of the cutoff multigraph (Definition def6 with a
// constant cutoff) and its count / fill compaction.
//
// Work item = (structure, group of source atoms). Lanes hold (source,
// destination) pairs; the image loop is uniform over the wave, so every image
// (an FP64-derived shift s_t = t.L rounded once to FP32) is loaded once per
// wave and broadcast to all lanes. The per-pair part p_ij = wrap(x_j - x_i).L is
// computed once per item in FP64 and rounded to FP32; the inner step is
// d = p_ij + s_t, l^2 = d.d and the strict test l < c (as l^2 < c2thr, the
// smallest float whose correctly rounded square root reaches c).
//
// The count pass writes the number of edges of every source; after the scan
// the fill pass repeats the sweep and writes every hit at
// offsets[src] + (rank of the hit inside the source), ranked with a wave
// ballot and mbcnt. The fill visits t = 0 first (the only image with an
// excluded pair, (i, i, 0)) and then the others in table order, so the edges
// of a source are contiguous and their order is deterministic.
// This replaces the ordered stack's concatenate / sort / filter (Sec. 2.2,
// Algorithm 2) for the cutoff graph: nothing is sorted, the output is grouped
// by source as Algorithm 2's stable sort by source index would group it.
#include "mg_internal.h"

namespace mg {

namespace {

struct Pair {
    float px, py, pz;
    int w0, w1, w2;   // wrap of the fractional displacement, plus the packing bias
    bool self;
};

// p_ij in FP32 from the FP64 wrapped fractional displacement. Inactive lanes
// get a displacement no image can bring within the cutoff.
__device__ inline Pair make_pair(const float* __restrict__ frac, const double* L, int64_t atom0,
                                 int il, int j, bool act) {
    Pair P;
    P.self = act && (il == j);
    if (!act) {
        P.px = P.py = P.pz = 1e30f;
        P.w0 = P.w1 = P.w2 = 0;
        return P;
    }
    const int64_t ai = atom0 + il, aj = atom0 + j;
    double d0 = (double)frac[3 * aj] - (double)frac[3 * ai];
    double d1 = (double)frac[3 * aj + 1] - (double)frac[3 * ai + 1];
    double d2 = (double)frac[3 * aj + 2] - (double)frac[3 * ai + 2];
    const double w0 = rint(d0), w1 = rint(d1), w2 = rint(d2);
    d0 -= w0;
    d1 -= w1;
    d2 -= w2;
    double px, py, pz;
    cart64(L, d0, d1, d2, px, py, pz);
    P.px = (float)px;
    P.py = (float)py;
    P.pz = (float)pz;
    P.w0 = (int)w0 + TBIAS;
    P.w1 = (int)w1 + TBIAS;
    P.w2 = (int)w2 + TBIAS;
    return P;
}

// The image loop: every lane uses the same image, so the entries are read
// through the constant address space (scalar loads into SGPRs, waited on by
// their own counter, never behind the fill's vector stores) and the step's
// shift operands are scalar registers. Entries are read in groups of IG
// (one wait per group; 2, 4 or 8, chosen by the tuning), the last few one at
// a time.
typedef const __attribute__((address_space(4))) ImageEntry* ConstTable;

__device__ __forceinline__ ImageEntry image_at(ConstTable tab, int m) {
    ImageEntry e;
    e.sx = tab[m].sx;
    e.sy = tab[m].sy;
    e.sz = tab[m].sz;
    e.tpk = tab[m].tpk;
    return e;
}

template <int IG, class Step>
__device__ __forceinline__ void for_images(const ImageEntry* __restrict__ table, int I, Step&& step) {
    // the table address is wave-uniform; make that explicit so the loads are scalar
    const uint64_t a = (uint64_t)table;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    ConstTable tab = (ConstTable)(((uint64_t)hi << 32) | lo);
    int m = 0;
    for (; m + IG <= I; m += IG) {
        ImageEntry e[IG];
#pragma unroll
        for (int u = 0; u < IG; ++u) e[u] = image_at(tab, m + u);
#pragma unroll
        for (int u = 0; u < IG; ++u) step(e[u]);
    }
    for (; m < I; ++m) step(image_at(tab, m));
}

__device__ inline float dist2(const Pair& P, const ImageEntry& e) {
    const float dx = P.px + e.sx, dy = P.py + e.sy, dz = P.pz + e.sz;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Output arrays rebased at the item's first edge (a wave-uniform offset), so a
// store needs only a 32-bit per-lane offset from a scalar base.
struct OutRel {
    int32_t* src;
    int32_t* dst;
    int32_t* image;
    float* length;
    float* vec;     // nullable
    uint32_t cap;   // capacity - base (clamped to 32 bits): relative edges >= cap are not written
    bool fits;      // every edge of the item lies below capacity (no per-edge test)
};

// item_end: the end of the rows the item writes into (row_ptr past its last source).
__device__ __forceinline__ OutRel rebase(int64_t base, int64_t item_end, int64_t capacity, int32_t* src,
                                         int32_t* dst, int32_t* image, float* length, float* vec) {
    const int64_t b = uniform64(base);
    const int64_t room = capacity - b;
    const uint32_t cap = room <= 0 ? 0u : (room >= (int64_t)UINT32_MAX ? UINT32_MAX : (uint32_t)room);
    const bool fits = __builtin_amdgcn_readfirstlane(uniform64(item_end) <= capacity ? 1 : 0) != 0;
    return OutRel{src + b, dst + b, image + 3 * b, length + b, vec ? vec + 3 * b : nullptr, cap, fits};
}

__device__ __forceinline__ void write_edge(uint32_t e, const OutRel& o, int32_t src_atom, int32_t dst_atom,
                                           const Pair& P, const ImageEntry& t, float l2) {
    const int32_t tpk = t.tpk;
    if (!o.fits && e >= o.cap) return;   // (o.fits is wave-uniform: a scalar branch in the common case)
    // 32-bit byte offsets from the scalar bases (an item's edges are far fewer than
    // 2^28); 12 e as two shifts and an add, not a quarter-rate multiply
    const uint32_t b4 = e << 2;
    uint32_t b8 = e << 3;
    asm volatile("" : "+v"(b8));
    const uint32_t b12 = b8 + b4;
    (void)src_atom;   // src is written densely from row_ptr after the fill (k_src_from_rows)
    *(int32_t*)((char*)o.dst + b4) = dst_atom;
    int32_t* im = (int32_t*)((char*)o.image + b12);
    constexpr int32_t mask = (1 << TBITS) - 1;   // t - w from the biased fields
    im[0] = ((tpk >> (2 * TBITS)) & mask) - P.w0;
    im[1] = ((tpk >> TBITS) & mask) - P.w1;
    im[2] = (tpk & mask) - P.w2;
    *(float*)((char*)o.length + b4) = sqrt_rn_finite(l2);
    if (o.vec) {   // the edge vector p_ij + s_t, as summed for the length
        float* v = (float*)((char*)o.vec + b12);
        v[0] = P.px + t.sx;
        v[1] = P.py + t.sy;
        v[2] = P.pz + t.sz;
    }
}

}  // namespace

constexpr int MODE_COUNT = 0, MODE_FILL = 1;

// Work item = (structure, source group, image chunk). A structure with C > 1
// image chunks splits its table into C consecutive index ranges
// [k I / C, (k+1) I / C); chunk 0 also takes t = 0 first, and no other chunk
// visits t = 0, so a source's chunks, in order, visit exactly the images of the
// unchunked sweep in the same order, and a heavy source group is spread over C
// waves. The count pass writes one count per (source, chunk) into ccount;
// k_chunk_prefix turns them into row totals (counts, scanned into row_ptr) and
// offsets inside the row, and the fill starts chunk k of source i at
// row_ptr[i] + that offset.
template <int MODE, int SLOTS, int IG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_cutoff_sweep(
    int B, const StructInfo* __restrict__ info, const int64_t* __restrict__ item_off,
    uint32_t* __restrict__ ccount, const ImageEntry* __restrict__ table,
    const float* __restrict__ frac, float c2thr,
    const float* __restrict__ thr, uint32_t* __restrict__ counts, const int64_t* __restrict__ offsets, int64_t capacity,
    int32_t* __restrict__ src, int32_t* __restrict__ dst, int32_t* __restrict__ image,
    float* __restrict__ length, float* __restrict__ vec, Counters* __restrict__ ctr, mg_report* __restrict__ rep,
    int64_t* __restrict__ partials) {
    const int lane = lane_id();
    const int64_t* ioff = item_off;
    const int64_t total = ioff[B];
    int64_t ncand = 0;
    for (int64_t q = grid_wave(); q < total; q += grid_waves()) {
        // ioff[lo] <= q < ioff[lo + 1], found by the whole wave in about
        // log65(B) dependent loads (a binary search would chain log2(B))
        const int lo = __builtin_amdgcn_readfirstlane(wave_search_le(ioff, B, q, lane));
        const StructInfo* si = info + lo;
        const int n = si->n;
        const int G = si->G;
        const int C = si->chunks;
        const int li = (int)(q - ioff[lo]);
        const int grp = C == 1 ? li : li / C;
        const int ck_beg = li - grp * C;   // this item's image chunk
        const int ck_end = ck_beg + 1;
        const int i_first = grp * G;
        const int nsrc = min(G, n - i_first);
        const int64_t atom0 = si->atom0;
        const int64_t xoff = si->xoff;
        const int I = si->box == 0 ? 0 : si->images;
        const int zimg = si->zero_img;
        const ImageEntry* tab = table + si->img_off;
        // the lattice is read where the pair offsets are formed (held in scalar
        // registers through the image loop it made the sweep spill more of them)
        const double* L = si->L;
        // (count) where the count of local source a in this item's chunk goes
        auto cslot = [&](int a) -> uint32_t* {
            return C == 1 ? counts + atom0 + a : ccount + xoff + (int64_t)a * C + ck_beg;
        };

        if (I == 0 || zimg < 0) {
            if (MODE == MODE_COUNT && lane < nsrc) *cslot(i_first + lane) = 0u;
            continue;
        }
        // chunk ck's table range; t = 0 goes to chunk 0 only
        auto visit = [&](int ck, auto& step_x, auto& step) {
            const int k0 = (int)((int64_t)ck * I / C), k1 = (int)((int64_t)(ck + 1) * I / C);
            if (ck == 0) step_x(tab[zimg], true);
            if (zimg >= k0 && zimg < k1) {
                for_images<IG>(tab + k0, zimg - k0, step);
                for_images<IG>(tab + zimg + 1, k1 - zimg - 1, step);
            } else {
                for_images<IG>(tab + k0, k1 - k0, step);
            }
        };
        {   // candidates of this item: images of its chunks
            const int k0 = (int)((int64_t)ck_beg * I / C), k1 = (int)((int64_t)ck_end * I / C);
            const bool zin = zimg >= k0 && zimg < k1;
            ncand += (int64_t)nsrc * n * (k1 - k0 - (zin ? 1 : 0) + (ck_beg == 0 ? 1 : 0));
        }
        // (fill) start of this item's chunk of local source a in the output
        auto cstart = [&](int a) -> int64_t {
            return offsets[atom0 + a] + (C == 1 ? 0 : (int64_t)ccount[xoff + (int64_t)a * C + ck_beg]);
        };

        if (n <= WAVE) {
            // ---- several sources per wave: lane = a * n + j
            const int a = lane / n;
            const int j = lane - a * n;
            const bool act = a < nsrc;
            const int il = i_first + a;
            const Pair P = make_pair(frac, L, atom0, il, j, act);
            const float c2 = (thr && act) ? thr[atom0 + il] : c2thr;   // the source's cutoff
            uint32_t cnt = 0;
            uint32_t run = 0;
            uint32_t base = 0;      // this lane's source's first edge, relative to the item's
            uint64_t seg = 0;
            OutRel out{};
            if (MODE == MODE_FILL) {
                const int64_t ibase = cstart(i_first);
                out = rebase(ibase, offsets[atom0 + i_first + nsrc], capacity, src, dst, image, length, vec);
                base = act ? (uint32_t)(cstart(il) - ibase) : 0u;
                seg = (n == WAVE) ? ~0ull : (((1ull << n) - 1ull) << (a * n));
            }
            const int32_t sa = (int32_t)(atom0 + il), da = (int32_t)(atom0 + j);
            auto step_x = [&](const ImageEntry& e, bool zero) {
                const float l2 = dist2(P, e);
                bool hit = l2 < c2;
                if (zero) hit = hit & !P.self;   // the excluded self-image (i, i, 0)
                if (MODE == MODE_COUNT) {
                    cnt += hit ? 1u : 0u;
                } else {
                    const uint64_t m = ballot(hit) & seg;
                    if (hit) write_edge(base + run + mbcnt(m), out, sa, da, P, e, l2);
                    run += (uint32_t)__popcll(m);
                }
            };
            auto step = [&](const ImageEntry& e) { step_x(e, false); };
            visit(ck_beg, step_x, step);   // t = 0 first (the only image with an excluded pair), then table order
            if (MODE == MODE_COUNT) {
                const int inc = wave_incl_scan_i32(act ? (int)cnt : 0);
                const int end = min((lane + 1) * n - 1, WAVE - 1);
                const int beg = lane * n - 1;
                const int hiv = __shfl(inc, end, WAVE);
                const int lov = __shfl(inc, max(beg, 0), WAVE);
                if (lane < nsrc) *cslot(i_first + lane) = (uint32_t)(hiv - (beg >= 0 ? lov : 0));
            }
        } else {
            // ---- one source per item, SLOTS destinations per lane, chunks of 64*SLOTS
            const int il = i_first;
            const float c2 = thr ? thr[atom0 + il] : c2thr;
            uint32_t cnt = 0;   // wave-uniform in this path
            uint32_t run = 0;
            OutRel out{};
            if (MODE == MODE_FILL)
                out = rebase(cstart(il), offsets[atom0 + il + 1], capacity, src, dst, image, length, vec);
            const int32_t sa = (int32_t)(atom0 + il);
            {
                const int ck = ck_beg;
                for (int jc = 0; jc < n; jc += WAVE * SLOTS) {
                    Pair P[SLOTS];
#pragma unroll
                    for (int r = 0; r < SLOTS; ++r) {
                        const int j = jc + r * WAVE + lane;
                        P[r] = make_pair(frac, L, atom0, il, j, j < n);
                    }
                    auto step_x = [&](const ImageEntry& e, bool zero) {
#pragma unroll
                        for (int r = 0; r < SLOTS; ++r) {
                            const float l2 = dist2(P[r], e);
                            bool hit = l2 < c2;
                            if (zero) hit = hit & !P[r].self;
                            if (MODE == MODE_COUNT) {
                                cnt += (uint32_t)__popcll(ballot(hit));
                            } else {
                                const uint64_t m = ballot(hit);
                                if (hit)
                                    write_edge(run + mbcnt(m), out, sa, (int32_t)(atom0 + jc + r * WAVE + lane), P[r],
                                               e, l2);
                                run += (uint32_t)__popcll(m);
                            }
                        }
                    };
                    auto step = [&](const ImageEntry& e) { step_x(e, false); };
                    visit(ck, step_x, step);
                }
            }
            if (MODE == MODE_COUNT && lane == 0) *cslot(il) = cnt;
        }
    }
    if (MODE == MODE_COUNT && lane == 0) partials[grid_wave()] = ncand;
}

hipError_t launch_cutoff_sweep(int mode, int B, const StructInfo* info, const int64_t* item_off,
                               uint32_t* ccount, const ImageEntry* table, const float* frac, float c2thr,
                               const float* thr, uint32_t* counts, const int64_t* offsets, int64_t capacity,
                               int32_t* src, int32_t* dst, int32_t* image, float* length, float* vec,
                               Counters* ctr, mg_report* report, int64_t* partials, int grid, int slots,
                               int img_group, hipStream_t s) {
    if (B == 0) return hipSuccess;
#define MG_SWEEP(M, S, G)                                                                                      \
    hipLaunchKernelGGL((k_cutoff_sweep<M, S, G>), dim3(grid), dim3(256), 0, s, B, info, item_off, ccount, table, \
                       frac, c2thr, thr, counts, offsets, capacity, src, dst, image, length, vec, ctr, report,   \
                       partials)
#define MG_SWEEP_G(M, S)                       \
    do {                                       \
        if (img_group <= 2) MG_SWEEP(M, S, 2); \
        else if (img_group <= 4) MG_SWEEP(M, S, 4); \
        else MG_SWEEP(M, S, 8);                \
    } while (0)
#define MG_SWEEP_SG(M)                       \
    do {                                     \
        if (slots <= 1) MG_SWEEP_G(M, 1);    \
        else if (slots == 2) MG_SWEEP_G(M, 2); \
        else MG_SWEEP_G(M, 4);               \
    } while (0)
    if (mode == MODE_COUNT) MG_SWEEP_SG(MODE_COUNT);
    else MG_SWEEP_SG(MODE_FILL);
#undef MG_SWEEP_SG
#undef MG_SWEEP_G
#undef MG_SWEEP
    return hipGetLastError();
}

// Counts of the chunked structures: the row total of every source goes to
// counts[src] (scanned into row_ptr next) and each (source, chunk) count is
// replaced by the number of the source's edges in the chunks before it. One
// workgroup per structure (unchunked structures return at once); a wave takes
// blocks of floor(64 / C) sources, lane = (source, chunk), and turns the block
// into in-row offsets with one segmented wave scan. The four waves take every
// fourth block, and each loads its next block before storing the current one.
__global__ __launch_bounds__(256) void k_chunk_prefix(int B, const StructInfo* __restrict__ info,
                                                      uint32_t* __restrict__ counts, uint32_t* __restrict__ ccount) {
    const int b = blockIdx.x;
    if (b >= B) return;
    const StructInfo* si = info + b;
    const int C = si->chunks;
    if (C <= 1) return;
    const int n = si->n;
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    uint32_t* cc = ccount + si->xoff;
    const int spb = WAVE / C;                 // sources per block (C <= 64)
    const int al = lane / C, kl = lane - al * C;
    const int nblk = (n + spb - 1) / spb;
    auto load = [&](int blk) -> uint32_t {
        const int a = blk * spb + al;
        return (al < spb && a < n) ? cc[(int64_t)a * C + kl] : 0u;
    };
    uint32_t cn = wv < nblk ? load(wv) : 0u;
    for (int blk = wv; blk < nblk; blk += 4) {
        const uint32_t c = cn;
        if (blk + 4 < nblk) cn = load(blk + 4);   // issued before this block's stores
        const int inc = wave_incl_scan_i32((int)c);
        const int first = al * C;                   // lane of this source's chunk 0
        const int prev = __shfl(inc, max(first - 1, 0), WAVE);   // every lane takes part in the shuffle
        const int before = first > 0 ? prev : 0;
        const uint32_t excl = (uint32_t)inc - (uint32_t)before - c;   // modulo 2^32, like the counts
        const int a = blk * spb + al;
        if (al < spb && a < n) {
            cc[(int64_t)a * C + kl] = excl;
            if (kl == C - 1) counts[si->atom0 + a] = excl + c;
        }
    }
}

hipError_t launch_chunk_prefix(int B, const StructInfo* info, uint32_t* counts, uint32_t* ccount, hipStream_t s) {
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_prefix, dim3((unsigned)B), dim3(256), 0, s, B, info, counts, ccount);
    return hipGetLastError();
}

// src of every cutoff edge from row_ptr: the fill writes no src (a sparse store
// fewer per hit step). One source per wave iteration; the row bounds are
// wave-uniform and come through scalar loads, which wait on their own counter,
// the next row's issued before this row is written. With a 16-byte aligned src
// the row's 16-byte aligned middle is written four edges per lane (a quarter of
// the store instructions), its ends one edge per lane. (Waves that each take a
// contiguous chunk of edges and walk its rows measured slower: the row walk's
// loads sit on each short piece.)
typedef const __attribute__((address_space(4))) int64_t* ConstI64;

__global__ __launch_bounds__(256) void k_src_from_rows(const int64_t* __restrict__ offsets, int64_t N,
                                                       int64_t capacity, int32_t* __restrict__ src) {
    const int lane = lane_id();
    const uint64_t a = (uint64_t)offsets;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    ConstI64 off = (ConstI64)(((uint64_t)hi << 32) | lo);
    const bool wide = ((uint64_t)src & 15u) == 0;
    const int64_t W = grid_waves();
    int64_t i = grid_wave();
    int64_t n0 = i < N ? off[i] : 0, n1 = i < N ? off[i + 1] : 0;
    for (; i < N; i += W) {
        const int64_t e0 = n0;
        const int64_t e1 = min(n1, capacity);
        if (i + W < N) {   // the next row's bounds load while this row is written
            n0 = off[i + W];
            n1 = off[i + W + 1];
        }
        const int32_t v = (int32_t)i;
        if (wide && e1 - e0 >= 8) {
            const int64_t a0 = (e0 + 3) & ~(int64_t)3, a1 = e1 & ~(int64_t)3;   // e0 <= a0 < a1 <= e1
            if (e0 + lane < a0) src[e0 + lane] = v;
            if (a1 + lane < e1) src[a1 + lane] = v;
            const int4 q = make_int4(v, v, v, v);
            for (int64_t e = a0 + 4 * lane; e < a1; e += 4 * WAVE) *(int4*)(src + e) = q;
        } else {
            for (int64_t e = e0 + lane; e < e1; e += WAVE) src[e] = v;
        }
    }
}

hipError_t launch_src_from_rows(const int64_t* offsets, int64_t N, int64_t capacity, int32_t* src, hipStream_t s) {
    if (N == 0 || capacity == 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((N + 3) / 4, (int64_t)device_cu_count() * 16);
    hipLaunchKernelGGL(k_src_from_rows, dim3((unsigned)g), dim3(256), 0, s, offsets, N, capacity, src);
    return hipGetLastError();
}

// ------------------------------------------------------------ prefix sums

constexpr int SCAN_TILE = 2048;   // 256 threads x 8 counts

__device__ inline int64_t block_sum_256(int64_t v, int64_t* sh) {
    v = wave_sum_i64(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    const int64_t t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

// Exclusive scan of N counts (offsets[N] = total). With n_dev set, only the
// first min(N, *n_dev) counts are scanned and offsets[] ends there; launches
// are sized for N so that the count may be known on the device only.
__device__ __forceinline__ int64_t scan_length(int64_t N, const int64_t* n_dev) {
    if (!n_dev) return N;
    const int64_t n = *n_dev;
    return n < 0 ? 0 : (n < N ? n : N);
}

__global__ __launch_bounds__(256) void k_scan_sums(const uint32_t* __restrict__ counts, int64_t N,
                                                   const int64_t* __restrict__ n_dev,
                                                   int64_t* __restrict__ bsum, mg_report* __restrict__ rep,
                                                   const int64_t* __restrict__ partials, int np) {
    __shared__ int64_t sh[4];
    if (partials && rep) {
        // the sweep's per-wave candidate counts: every block sums a slice and
        // adds it with one integer atomic (instead of one block looping over all)
        const int per = (np + (int)gridDim.x - 1) / (int)gridDim.x;
        const int q0 = (int)blockIdx.x * per, q1 = min(np, q0 + per);
        int64_t c = 0;
        for (int q = q0 + (int)threadIdx.x; q < q1; q += 256) c += partials[q];
        c = block_sum_256(c, sh);
        if (threadIdx.x == 0 && c != 0) atomicAdd((unsigned long long*)&rep->candidates, (unsigned long long)c);
        __syncthreads();   // sh is reused below
    }
    const int64_t n = scan_length(N, n_dev);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    if (base >= n) return;            // never read by the final pass
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t idx = base + k * 256 + threadIdx.x;
        if (idx < n) s += counts[idx];
    }
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_scan_final(const uint32_t* __restrict__ counts, int64_t N,
                                                    const int64_t* __restrict__ n_dev,
                                                    const int64_t* __restrict__ bsum,
                                                    int64_t* __restrict__ offsets, int64_t capacity,
                                                    mg_report* __restrict__ rep,
                                                    const int64_t* __restrict__ partials, int np) {
    __shared__ int64_t sh[4];
    __shared__ int64_t swave[4];
    const int64_t n = scan_length(N, n_dev);
    const int64_t last = n > 0 ? (n - 1) / SCAN_TILE : 0;   // the block that writes offsets[n]
    if ((int64_t)blockIdx.x > last) return;
    int64_t p = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) p += bsum[b];
    p = block_sum_256(p, sh);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * 8;
    uint32_t v[8];
    int64_t tsum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = (base + k < n) ? counts[base + k] : 0u;
        tsum += v[k];
    }
    const int64_t inc = wave_incl_scan_i64(tsum);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) swave[w] = inc;
    __syncthreads();
    int64_t excl = p + inc - tsum;
    for (int q = 0; q < w; ++q) excl += swave[q];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (base + k < n) offsets[base + k] = excl;
        excl += v[k];
    }
    if ((int64_t)blockIdx.x == last && threadIdx.x == 255) {
        offsets[n] = excl;
        if (rep) {
            rep->num_edges = excl;
            if (excl > capacity) atomicOr(&rep->flags, (uint32_t)MG_FLAG_CAPACITY);
        }
    }
    if (partials && rep && (int64_t)blockIdx.x == last) {
        // the sweep's per-wave candidate counts, summed here instead of in a launch of their own
        int64_t c = 0;
        for (int q0 = 0; q0 < np; q0 += 256 * 8) {   // eight independent loads per round
            int64_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int q = q0 + k * 256 + threadIdx.x;
                v[k] = q < np ? partials[q] : 0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) c += v[k];
        }
        c = block_sum_256(c, sh);
        if (threadIdx.x == 0) rep->candidates += c;
    }
}

hipError_t launch_scan_counts(const uint32_t* counts, int64_t N, int64_t* offsets, int64_t* bsum,
                              int64_t capacity, mg_report* report, hipStream_t s, const int64_t* n_dev,
                              const int64_t* partials, int np) {
    const int64_t nb = N > 0 ? (N + SCAN_TILE - 1) / SCAN_TILE : 1;
    if (N > 0) {   // the first pass also sums the partials
        hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, s, counts, N, n_dev, bsum, report,
                           partials, np);
        partials = nullptr;
    }
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(256), 0, s, counts, N, n_dev, bsum, offsets,
                       capacity, report, partials, np);
    return hipGetLastError();
}

int64_t scan_block_count(int64_t N) { return N > 0 ? (N + SCAN_TILE - 1) / SCAN_TILE : 1; }

}  // namespace mg

namespace mg {

__global__ __launch_bounds__(256) void k_sum_partials(const int64_t* __restrict__ p, int n,
                                                      mg_report* __restrict__ rep) {
    __shared__ int64_t sh[4];
    int64_t v = 0;
    for (int q0 = 0; q0 < n; q0 += 256 * 8) {   // eight independent loads per round
        int64_t u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = q0 + k * 256 + threadIdx.x;
            u[k] = q < n ? p[q] : 0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) v += u[k];
    }
    v = wave_sum_i64(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) rep->candidates += sh[0] + sh[1] + sh[2] + sh[3];
}

hipError_t launch_sum_partials(const int64_t* partials, int n, mg_report* report, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, n, report);
    return hipGetLastError();
}

}  // namespace mg

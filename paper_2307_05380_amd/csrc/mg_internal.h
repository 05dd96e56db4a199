// Internal declarations shared by the HIP translation units of libmatgraph.
// Not part of the public ABI (include/matgraph.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/matgraph.h"

namespace mg {

constexpr int WAVE = 64;
constexpr int TBITS = 10;                 // bits per packed image component
constexpr int TMAX = (1 << (TBITS - 1)) - 1;   // |t_k| <= 511
constexpr int TBIAS = 1 << (TBITS - 1);

// One lattice translation of a structure's image table: the FP64 product t.L
// rounded once to FP32, and t packed as three biased 10-bit fields (t0 high).
struct alignas(16) ImageEntry {
    float sx, sy, sz;
    int32_t tpk;
};

__host__ __device__ inline int32_t pack_t(int t0, int t1, int t2) {
    return ((t0 + TBIAS) << (2 * TBITS)) | ((t1 + TBIAS) << TBITS) | (t2 + TBIAS);
}
__host__ __device__ inline int unpack_t0(int32_t p) { return ((p >> (2 * TBITS)) & ((1 << TBITS) - 1)) - TBIAS; }
__host__ __device__ inline int unpack_t1(int32_t p) { return ((p >> TBITS) & ((1 << TBITS) - 1)) - TBIAS; }
__host__ __device__ inline int unpack_t2(int32_t p) { return (p & ((1 << TBITS) - 1)) - TBIAS; }

// Per-structure plan, written by the bounds kernel (FP64).
struct alignas(16) StructInfo {
    double L[9];        // lattice rows, FP64 copy of the input
    int64_t atom0;      // first atom
    int64_t box;        // images in the box prod(2 nk + 1); 0 when the structure is skipped
    int64_t img_off;    // first entry in the image table
    int32_t n;          // atoms
    int32_t nk[3];      // box half ranges
    int32_t images;     // entries kept in the table
    int32_t zero_img;   // table index of t = 0 (-1 if absent)
    int32_t G;          // sources per work item
    int32_t groups;     // source groups (work items before image chunks)
    int32_t chunks;     // image chunks per source group in the cutoff sweeps (1 unless the plan splits)
    float rk;           // KNN: k-th neighbour distance of a uniform density n / V (Angstrom)
    int64_t xoff;       // chunks > 1: first of this structure's per-(source, chunk) counts
    float R;            // radius the table was built for, with rounding margin (Angstrom)
    float Rs;           // search radius before the margin (Angstrom)
    uint32_t flags;     // MG_FLAG_* of this structure
    int32_t mode;       // 0: pair x image sweep, 1: cell lists
    int32_t m[3];       // cell lists: bins per lattice direction
    int32_t nbins;      // cell lists: m0 * m1 * m2
    int64_t bin_off;    // cell lists: first bin in the global bin arrays
    int32_t cl_items;   // cell lists: work items (one per bin)
    float wcl;          // cell lists: radius covered by the 27-bin stencil (Angstrom)
    // image tests (FP64): lattice-plane spacings, (R + half the longest cell
    // diagonal)^2 and the metric tensor G = L L^T (00 01 02 11 12 22)
    double hk[3];
    double far2;
    double Gm[6];
    double rGd[3];      // 1 / G_kk
    double rD2[3];      // 1 / det of the 2x2 blocks of G on the index pairs (1,2), (0,2), (0,1)
    int32_t cl_s;       // cell lists: stencil half-width S in bins ((2S+1)^3 bins, each >= R / S thick)
    int32_t pad1;
};

constexpr int CL_MIN_ATOMS = 512;   // structures smaller than this use the image sweep

// The per-structure quantities the batch plan scans, packed for coalesced
// loads (written by the bounds kernel next to StructInfo).
struct alignas(16) PlanRow {
    int32_t box;        // StructInfo::box (at most 1023^3)
    int32_t groups;
    int32_t cl_items;
    int32_t nbins;
    int64_t cost;       // candidates of one source group over the whole box (0: no image sweep)
    int32_t n;
    uint32_t flags;     // StructInfo::flags (the plan kernel ORs them into the report)
};

// Image chunks: a structure whose source groups are heavy gets its image table
// cut into up to MAX_CHUNKS consecutive ranges, each a work item of its own.
constexpr int MAX_CHUNKS = 64;
constexpr int64_t CHUNK_TARGET_DIV = 32768;   // target item cost = total cost / this
constexpr int CHUNK_MIN_BOX = 64;             // at most box / this chunks (short image ranges cost setup)

// Scratch counters at the head of every workspace.
struct alignas(64) Counters {
    uint32_t spare[8];
    uint32_t knn2_count;       // sources queued for the extended KNN search
    uint32_t pad[7];
    int64_t total_box;         // sum of box sizes (image entries needed)
    int64_t total_items;       // work items of the image sweep
    int64_t total_cl_items;    // work items of the cell-list sweep
    int64_t total_bins;        // cell-list bins of the batch
};

// Capacity of the cell-list bin arrays: bins are capped at 2n + 64 per structure.
inline int64_t cl_bin_capacity(int B, int64_t N) { return 2 * N + 64 * (int64_t)B + 1; }

constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------ device helpers

__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set bits of `m` in lanes below the calling lane.
__device__ inline uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline int lane_id() { return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

template <typename T>
__device__ inline T uniform(T v) {
    return (T)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ inline int64_t uniform64(int64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Inclusive wave scan (64 lanes) with DPP row shifts and row broadcasts.
__device__ inline int wave_incl_scan_i32(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Persistent kernels hand out work items cyclically: wave w of the grid takes
// items w, w + W, w + 2W, ... (W waves in the grid). Consecutive items (the
// sources of one structure) land on different waves, which balances uneven
// structures without a shared counter; every loop is bounded by the item count.
// The wave index is made explicitly wave-uniform so that the item loop, its
// structure search and the per-structure loads run on the scalar unit.
__device__ __forceinline__ int64_t grid_wave() {
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    return (int64_t)blockIdx.x * (blockDim.x / WAVE) + w;
}
__device__ __forceinline__ int64_t grid_waves() { return (int64_t)gridDim.x * (blockDim.x / WAVE); }

// Largest s in [0, n) with a[s] <= x, for a non-decreasing a with a[0] <= x,
// found by the whole wave (x wave-uniform): a 65-ary search, each step probing
// 64 positions at once, so the result needs about log65(n) dependent loads.
__device__ __forceinline__ int wave_search_le(const int64_t* __restrict__ a, int n, int64_t x, int lane) {
    int lo = 0, hi = n;   // answer in [lo, hi)
    while (hi - lo > 1) {
        const int span = hi - lo;
        if (span <= WAVE) {
            const int p = lo + lane;
            const uint64_t le = ballot(lane < span && a[min(p, n - 1)] <= x);
            return lo + __popcll(le) - 1;   // a is sorted: the lanes with a[p] <= x are a prefix
        }
        const int p = lo + (int)(((int64_t)span * (lane + 1)) / (WAVE + 1));   // strictly increasing, in (lo, hi)
        const int c = __popcll(ballot(a[p] <= x));                           // probes at or below x
        const int plo = lo + (int)(((int64_t)span * c) / (WAVE + 1));         // probe c - 1, or lo
        const int phi = lo + (int)(((int64_t)span * (c + 1)) / (WAVE + 1));   // probe c, or hi
        lo = c == 0 ? lo : plo;
        hi = c == WAVE ? hi : phi;
    }
    return lo;
}

// Correctly rounded square root of a finite x >= 0: the hardware root (within
// one ulp) and one residual test on each neighbour, r*r against x with a
// single rounding (fma). Checked bit for bit against sqrtf on every float from
// 2^-60 to the largest finite one and on 0; below about 2^-100 the residual
// falls into the range flushed to zero and the hardware root may be kept.
// Squared edge lengths are 0 or far above that.
__device__ __forceinline__ float sqrt_rn_finite(float x) {
    const float r = __builtin_amdgcn_sqrtf(x);
    const float rm = __uint_as_float(__float_as_uint(r) - 1u);
    const float rp = __uint_as_float(__float_as_uint(r) + 1u);
    const float lo = fmaf(-rm, r, x) <= 0.0f ? rm : r;   // x at or below the rm..r midpoint squared
    return fmaf(-rp, r, x) > 0.0f ? rp : lo;             // x above the r..rp midpoint squared
}

// Cartesian vector f L of a fractional vector f (FP64; rows of L are the
// lattice vectors). Every FP32 distance of the image sweeps and the KNN keys
// is built from two such products, each rounded once to FP32: the pair offset
// (x_j - x_i - w) L, w = rint(x_j - x_i), and the image shift t L. All paths
// call this one function (the image tables, the sweeps, the KNN passes), so a
// candidate gets bit for bit the same distance whichever path evaluates it.
__device__ __forceinline__ void cart64(const double* L, double f0, double f1, double f2, double& x, double& y,
                                       double& z) {
    x = f0 * L[0] + f1 * L[3] + f2 * L[6];
    y = f0 * L[1] + f1 * L[4] + f2 * L[7];
    z = f0 * L[2] + f1 * L[5] + f2 * L[8];
}

// FP32 vector and squared length of candidate (j, t) of source i in the form
// the image sweeps compute them (x_i, x_j raw fractional coordinates, t the
// edge's image): pair offset plus image shift as above, summed in FP32. The
// KNN keys of every path use it, and the cell-list cutoff sweep decides with
// it wherever its own staged distance lies near the threshold, so a graph does
// not depend on the path or bin size that built it.
__device__ __forceinline__ float canon_vec(const double* L, double xi0, double xi1, double xi2, double xj0,
                                           double xj1, double xj2, int t0, int t1, int t2, float& dx, float& dy,
                                           float& dz) {
    double d0 = xj0 - xi0, d1 = xj1 - xi1, d2 = xj2 - xi2;
    const double w0 = rint(d0), w1 = rint(d1), w2 = rint(d2);
    d0 -= w0;
    d1 -= w1;
    d2 -= w2;
    double px, py, pz, sx, sy, sz;
    cart64(L, d0, d1, d2, px, py, pz);
    cart64(L, (double)(t0 + (int)w0), (double)(t1 + (int)w1), (double)(t2 + (int)w2), sx, sy, sz);
    dx = (float)px + (float)sx;
    dy = (float)py + (float)sy;
    dz = (float)pz + (float)sz;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Squared KNN key distance of candidate (j, t) of source i (canon_vec's length).
__device__ __forceinline__ float knn_l2(const double* L, double xi0, double xi1, double xi2, double xj0, double xj1,
                                        double xj2, int t0, int t1, int t2) {
    float dx, dy, dz;
    return canon_vec(L, xi0, xi1, xi2, xj0, xj1, xj2, t0, t1, t2, dx, dy, dz);
}

// Orders this wave's LDS writes before its later LDS reads (lanes exchange data
// through LDS without a workgroup barrier).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int64_t wave_incl_scan_i64(int64_t v) {
    // two 32-bit halves would need carries; use shuffles for 64-bit values
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int64_t u = __shfl_up(v, d, WAVE);
        if (lane_id() >= d) v += u;
    }
    return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

__device__ inline double wave_sum_f64(double v) {
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// A DPP lane move of a float (rows of 16 lanes; lanes the pattern leaves
// without a source, or in rows outside ROW_MASK, read 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// Inclusive scan of v over the wave with DPP row shifts and row broadcasts
// (VALU only; lane 63 ends with the total).
__device__ __forceinline__ float wave_incl_scan_f32(float v) {
    v += dpp_f32<0x111, 0xf>(v);   // row_shr:1
    v += dpp_f32<0x112, 0xf>(v);   // row_shr:2
    v += dpp_f32<0x114, 0xf>(v);   // row_shr:4
    v += dpp_f32<0x118, 0xf>(v);   // row_shr:8
    v += dpp_f32<0x142, 0xa>(v);   // row_bcast:15
    v += dpp_f32<0x143, 0xc>(v);   // row_bcast:31
    return v;
}

// Sum of v over the wave, on every lane (the scan's total read from lane 63).
__device__ inline float wave_sum_f32(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_incl_scan_f32(v)), 63));
}

// Structure owning atom `a`: largest b with ptr[b] <= a (ptr non-decreasing, B+1 entries).
__device__ inline int structure_of(const int64_t* __restrict__ ptr, int B, int64_t a) {
    int lo = 0, hi = B;   // invariant: ptr[lo] <= a < ptr[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (ptr[mid] <= a) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace mg

// ------------------------------------------------------- host-side launchers
// Each returns hipSuccess or the launch error. All are asynchronous on `stream`.
namespace mg {

// radii (nullable, cutoff mode only): per-atom cutoffs; then thr[a] receives
// the per-atom threshold on l^2 and the structure's radius is its largest c_a.
// cl_span: cell-list stencil half-width in bins (1: 27 bins at least the radius
// thick; 2: 125 bins at least half the radius thick, where they fit).
hipError_t launch_bounds(const float* lattices, const int64_t* batch_ptr, const float* frac, int B,
                         int64_t N, float radius, const float* radii, float* thr, int knn_k,
                         float knn_lambda, StructInfo* info, PlanRow* plan, Counters* ctr, mg_report* report, int mode,
                         int opts, int cl_span, hipStream_t s);
// Also starts the call's report (num_edges = num_edges0, images_needed, the
// structures' flags, every other field 0) and zeroes the workspace counters:
// no kernel before it may write either.
hipError_t launch_struct_scan(int B, StructInfo* info, const PlanRow* plan, int64_t chunk_cap, int64_t* item_off,
                              int64_t* cl_off,
                              int64_t* box_off, Counters* ctr, mg_report* report, int64_t image_capacity,
                              hipStream_t s, int64_t num_edges0 = 0);
struct ClWs {
    int64_t* cl_off;        // [B+1] scan of cell-list items (one item per bin)
    uint32_t* bin_count;    // [cap] atoms per bin
    int64_t* bin_start;     // [cap+1] first slot of every bin
    int64_t* bsum;          // scan partials
    int32_t* atom_bin;      // [N] bin of every atom (local to its structure)
    int32_t* atom_rank;     // [N] arrival order of every atom in its bin (from the histogram)
    int32_t* slot_atom;     // [N] atoms in bin order, unsorted inside a bin
    float4* slot_x;         // [N] raw coordinates (xyz) and atom index (w) in bin order, ascending atoms inside a bin
    int32_t* slot_shift;    // [N] packed floor(x) in the same order
    int32_t* atom_struct;   // [N] structure of every atom
    Counters* ctr;          // workspace counters (bin totals)
    int64_t cap;            // bin capacity
};
// Cell lists pack floor(x) of every atom (and u - floor(x)) in 10-bit fields:
// a structure with a coordinate outside [-CL_SHIFT_MAX, CL_SHIFT_MAX + 1)
// takes the image sweep.
constexpr int CL_SHIFT_MAX = TMAX - 1;
hipError_t launch_cl_build(int B, int64_t N, const float* frac, const int64_t* batch_ptr,
                           const StructInfo* info, const ClWs& w, hipStream_t s);
// vec (nullable, float [capacity][3]): the fill also writes every edge's vector.
hipError_t launch_cl_cutoff_sweep(int mode, int B, const StructInfo* info, const ClWs& w,
                                  const float* frac, float c2thr, const float* thr, uint32_t* counts,
                                  const int64_t* offsets, int64_t capacity, int32_t* src,
                                  int32_t* dst, int32_t* image, float* length, float* vec, Counters* ctr,
                                  mg_report* report, int64_t* partials, int grid, hipStream_t s);
// tau_scale: the first sweep's threshold is tau_scale times the k-th
// neighbour distance of a uniform density (0: the stencil's covered radius).
hipError_t launch_cl_knn(int B, int k, const StructInfo* info, const ClWs& w, const float* frac,
                         int32_t* src, int32_t* dst, int32_t* image, float* length,
                         int32_t* ext_list, Counters* ctr, mg_report* report, int64_t* partials,
                         int grid, float tau_scale, hipStream_t s);
// Image tables: every structure's box-sized slot (box), keep flags and their
// exclusive scan over the whole capacity, and the compacted tables read by the
// sweeps (table: each structure's kept images contiguous, lexicographic).
struct ImageTables {
    ImageEntry* box;
    uint32_t* kflag;
    int64_t* kscan;   // cap + 1
    int64_t* kbsum;
    ImageEntry* table;
    int64_t cap;
};
// Workspace bytes per image slot (box entry, flag, scan value, compacted entry)
// and a fixed allowance for scan partials and alignment.
constexpr int64_t IMAGE_SLOT_BYTES = 45;
constexpr int64_t IMAGE_FIXED_BYTES = 4096;
hipError_t launch_images(int B, StructInfo* info, const int64_t* box_off, const Counters* ctr, const ImageTables& t,
                         hipStream_t s);
// vec (nullable, float [capacity][3]): the fill also writes every edge's vector.
hipError_t launch_chunk_prefix(int B, const StructInfo* info, uint32_t* counts, uint32_t* ccount, hipStream_t s);
hipError_t launch_cutoff_sweep(int mode, int B, const StructInfo* info, const int64_t* item_off, uint32_t* ccount,
                               const ImageEntry* table, const float* frac, float c2thr,
                               const float* thr, uint32_t* counts, const int64_t* offsets, int64_t capacity,
                               int32_t* src, int32_t* dst, int32_t* image, float* length, float* vec,
                               Counters* ctr, mg_report* report, int64_t* partials, int grid, int slots,
                               int img_group, hipStream_t s);
// src[e] = i for every edge e of source i (offsets = row_ptr), e < capacity.
hipError_t launch_src_from_rows(const int64_t* offsets, int64_t N, int64_t capacity, int32_t* src, hipStream_t s);
// Exclusive scan of counts[0..N) into offsets[0..N]; with a report, also
// records the total as num_edges and flags a capacity overflow, and adds the
// np per-wave candidate counts in partials (if given) to report->candidates.
// With n_dev (a device count), only min(N, *n_dev) counts are scanned.
hipError_t launch_scan_counts(const uint32_t* counts, int64_t N, int64_t* offsets, int64_t* bsum,
                              int64_t capacity, mg_report* report, hipStream_t s,
                              const int64_t* n_dev = nullptr, const int64_t* partials = nullptr, int np = 0);
// tau_scale: the first sweep's threshold is tau_scale times the k-th
// neighbour distance of a uniform density (0: the table's radius).
hipError_t launch_knn(int B, int64_t N, int k, const StructInfo* info, const int64_t* item_off,
                      const ImageEntry* table, const float* frac, int32_t* src, int32_t* dst,
                      int32_t* image, float* length, int32_t* ext_list, Counters* ctr,
                      mg_report* report, int64_t* partials, int grid, float tau_scale, hipStream_t s);
hipError_t launch_knn_extended(int B, int64_t N, int k, const StructInfo* info, const float* frac,
                               const int32_t* atom_struct, int32_t* src, int32_t* dst,
                               int32_t* image, float* length, const int32_t* ext_list,
                               Counters* ctr, mg_report* report, int grid, hipStream_t s);
hipError_t launch_atom_struct(const int64_t* batch_ptr, int B, int64_t N, int32_t* atom_struct,
                              hipStream_t s);
// Workspace of the geometry passes: lattice accumulators (9 B), edge range of
// every structure (B + 1), items per structure (B + 1), order flag.
struct GeomBwdWs {
    double* acc;
    int64_t* start;
    int64_t* item_off;
    int32_t* flag;   // [4]: order flag, structures of the middle LDS window, structures beyond it,
                     // bucket path active
    // Bucket path of the backward pass for structures of more than 512 atoms
    // (all null when the workspace has no room for it): per structure the
    // offsets of its (dst block, chunk) counts and of its gather items, the
    // counts, their exclusive scan, scan partials and one record per edge.
    int64_t* cm_off;     // [B+1]
    int64_t* p3_off;     // [B+1]
    uint32_t* bcount;    // [m_cap]
    int64_t* boff;       // [m_cap + 1]
    int64_t* bsum;
    float4* rec;         // [e_cap]
    int64_t m_cap, e_cap;
};
// Bucket path sizes: atoms per destination block (one LDS accumulator block)
// and the largest structure it takes (more blocks than the per-chunk LDS
// histogram holds go to the atomic kernel).
constexpr int BW_CHUNK = 8192;   // edges per backward item (16384: 1-3 % slower, 4096: 2 % slower)
constexpr int BK_BLOCK = 256;   // atoms per destination block (512: 2-3 % slower on the 64 supercells)
constexpr int BK_MAX_BLOCKS = 256;
// Counts-matrix capacity for a batch of B structures and E edges.
inline int64_t bk_count_capacity(int B, int64_t E) { return ((int64_t)B + E / BW_CHUNK + 1) * BK_MAX_BLOCKS; }
hipError_t launch_geometry_fwd(const float* lattices, const float* frac, const int32_t* atom_struct,
                               const int64_t* batch_ptr, int B, int64_t N, const int32_t* src,
                               const int32_t* dst, const int32_t* image, int64_t E, const int64_t* num_edges,
                               float* vec, float* length, const GeomBwdWs& w, hipStream_t s);
hipError_t launch_geometry_bwd(const float* lattices, const float* frac, int32_t* atom_struct,
                               const int64_t* batch_ptr, int B, int64_t N, const int32_t* src,
                               const int32_t* dst, const int32_t* image, int64_t E,
                               const int64_t* num_edges, const float* grad_vec, const float* grad_length,
                               float* grad_frac, float* grad_lattice, const GeomBwdWs& w, hipStream_t s);
// Workspace of the symmetric closure: per-atom received counts, cursors and
// totals (N), received offsets (N + 1), scan partials, per-edge flags (E) and
// the received-edge buckets (E).
struct SymWs {
    uint32_t* addcnt;
    uint32_t* cursor;
    uint32_t* total;
    int64_t* aoff;
    int64_t* bsum;
    uint8_t* miss;
    uint64_t* bucket;
};
hipError_t launch_symmetrize(const int64_t* row_ptr, int64_t N, int64_t E, const int32_t* dst, const int32_t* image,
                             const float* length, int64_t capacity, int32_t* osrc, int32_t* odst, int32_t* oimg,
                             float* olen, int64_t* out_off, const SymWs& w, mg_report* report, hipStream_t s);
// KNN with ties: the search runs with TIES_K neighbours per source.
constexpr int TIES_K = 64;
hipError_t launch_ties(int64_t N, int k, const int32_t* src, const int32_t* dst, const int32_t* image,
                       const float* length, int64_t capacity, int32_t* osrc, int32_t* odst, int32_t* oimg,
                       float* olen, int64_t* offsets, uint32_t* counts, int64_t* bsum, mg_report* report,
                       hipStream_t s);
hipError_t launch_triplets(const int64_t* row_ptr, int64_t N, int64_t E, const float* vec, int64_t capacity,
                           int32_t* e1, int32_t* e2, float* cosv, int64_t* offsets, uint32_t* counts,
                           int64_t* bsum, mg_report* report, hipStream_t s);
// Per-wave partial counts (candidates evaluated) are written to a workspace
// array and summed by one block afterwards: no shared-counter atomics in the
// sweeps. The array holds MAX_GRID_WAVES entries.
constexpr int MAX_GRID_WAVES = 256 * 64 * 4;
hipError_t launch_sum_partials(const int64_t* partials, int n, mg_report* report, hipStream_t s);
hipError_t launch_zero_report(mg_report* report, Counters* ctr, int64_t num_edges, hipStream_t s);
int64_t scan_block_count(int64_t N);

int device_cu_count();

// Sets the calling thread's mg_last_error() message and returns st.
mg_status api_fail(mg_status st, const char* msg);

}  // namespace mg

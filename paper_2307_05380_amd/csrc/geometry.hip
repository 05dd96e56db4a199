// Edge geometry and its backward pass.
//
// v_e = (x_dst - x_src + t_e) L and l_e = ||v_e|| are the quantities inside the
// norm of Definition def6. The backward pass (edge set held fixed) is what lets
// a generative model move the geometry and rebuild the graph inside its
// forward pass (abstract; Sec. 4):
//   g_e = g_v + g_l v / l (0 when l = 0),
//   grad_x[dst] += g L^T, grad_x[src] -= g L^T, grad_L[s] += f^T g.
// The kernels are bound by HBM traffic on the per-edge arrays. The forward
// pass, whose lengths are held to 2e-5 A, does its per-edge arithmetic in FP64
// (full rate on CDNA) so that thin cells with large image offsets lose no
// accuracy; the backward passes, held to 1e-4 relative, work in FP32 per edge
// with FP64 sums where many edges add up. Results are stored in FP32.
#include "mg_internal.h"

namespace mg {

namespace {

__device__ inline int64_t edge_count(int64_t E, const int64_t* __restrict__ num_edges) {
    if (num_edges == nullptr) return E;
    const int64_t d = *num_edges;
    return d < E ? (d < 0 ? 0 : d) : E;
}

}  // namespace

// Forward pass: four edges per thread with every streamed load (src, dst,
// image) issued before the gathers that depend on them (the source's
// structure, its lattice, both coordinates) and no branch between a load and
// its use (indices are clamped; an edge with an endpoint outside [0, N) gets
// NaN). When a wave's 64 edges share one structure (almost always: the
// builders emit edges grouped by structure) its lattice comes through scalar
// loads. One thread per four edges (no grid cap): the plain streaming shape is
// the fastest here. FP64 arithmetic, FP32 results.
__global__ __launch_bounds__(256) void k_geom_fwd(const float* __restrict__ lattices,
                                                  const float* __restrict__ frac,
                                                  const int32_t* __restrict__ atom_struct, int64_t N,
                                                  const int32_t* __restrict__ src,
                                                  const int32_t* __restrict__ dst,
                                                  const int32_t* __restrict__ image, int64_t E,
                                                  const int64_t* __restrict__ num_edges,
                                                  float* __restrict__ vec, float* __restrict__ length) {
    const int64_t Ee = edge_count(E, num_edges);
    if (Ee == 0) return;
    constexpr int U = 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < Ee; e0 += stride * U) {
        int32_t i[U], j[U], t[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = min(e0 + u * stride, Ee - 1);
            i[u] = src[e];
            j[u] = dst[e];
            t[u][0] = image[3 * e];
            t[u][1] = image[3 * e + 1];
            t[u][2] = image[3 * e + 2];
        }
        bool ok[U];
        int32_t ic[U], jc[U], st[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = (uint64_t)(uint32_t)i[u] < (uint64_t)N && (uint64_t)(uint32_t)j[u] < (uint64_t)N;
            ic[u] = ok[u] ? i[u] : 0;
            jc[u] = ok[u] ? j[u] : 0;
            st[u] = atom_struct[ic[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * stride;
            const float* xi = frac + 3 * (int64_t)ic[u];
            const float* xj = frac + 3 * (int64_t)jc[u];
            const double f0 = (double)xj[0] - (double)xi[0] + (double)t[u][0];
            const double f1 = (double)xj[1] - (double)xi[1] + (double)t[u][1];
            const double f2 = (double)xj[2] - (double)xi[2] + (double)t[u][2];
            const double nan = __builtin_nan("");
            const int su = __builtin_amdgcn_readfirstlane(st[u]);
            double v0, v1, v2;
            if (ballot(st[u] != su) == 0) {
                const float* L = lattices + 9 * (int64_t)su;   // one structure: scalar loads
                v0 = ok[u] ? f0 * (double)L[0] + f1 * (double)L[3] + f2 * (double)L[6] : nan;
                v1 = ok[u] ? f0 * (double)L[1] + f1 * (double)L[4] + f2 * (double)L[7] : nan;
                v2 = ok[u] ? f0 * (double)L[2] + f1 * (double)L[5] + f2 * (double)L[8] : nan;
            } else {
                const float* L = lattices + 9 * (int64_t)st[u];
                v0 = ok[u] ? f0 * (double)L[0] + f1 * (double)L[3] + f2 * (double)L[6] : nan;
                v1 = ok[u] ? f0 * (double)L[1] + f1 * (double)L[4] + f2 * (double)L[7] : nan;
                v2 = ok[u] ? f0 * (double)L[2] + f1 * (double)L[5] + f2 * (double)L[8] : nan;
            }
            if (e < Ee) {
                if (vec) {
                    vec[3 * e] = (float)v0;
                    vec[3 * e + 1] = (float)v1;
                    vec[3 * e + 2] = (float)v2;
                }
                // the FP32 square root of the FP64 square, rounded once: within a few ulps
                if (length) length[e] = sqrtf((float)(v0 * v0 + v1 * v1 + v2 * v2));
            }
        }
    }
}

// Start of the backward pass: coordinate gradients, FP64 lattice sums and the
// plan's flag and counters cleared in one launch.
__global__ __launch_bounds__(256) void k_zero_bwd(float* __restrict__ gf, int64_t n3, double* __restrict__ acc,
                                                  int64_t n9, int32_t* __restrict__ flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 < 4) flag[t0] = 0;
    for (int64_t q = t0; q < n3 + n9; q += stride) {
        if (q < n3) gf[q] = 0.0f;
        else acc[q - n3] = 0.0;
    }
}

// Backward pass.
//
// Global atomics on MI355X are resolved far from the compute units and cost
// far more than LDS traffic, so the backward pass is organised so that almost
// no per-edge value reaches global memory through an atomic:
// - the edges are expected grouped by structure with non-decreasing src (what
//   the graph builders emit); every structure's edge range is found by a
//   search of src for the structure's first atom (no pass over the edges);
// - one workgroup per item (a structure, or a chunk of BW_CHUNK edges of a
//   large one) accumulates the coordinate gradients of the structure's atoms
//   in LDS and the lattice gradient in registers, then writes them with plain
//   stores when the item covers the whole structure (atomics only for split
//   structures). A wave whose 64 edges share the source keeps the source's sum
//   in registers until the run ends. The item kernels check what the grouping
//   promises (both endpoints in the item's structure, src non-decreasing
//   inside every 64-edge step) and raise a flag otherwise;
// - structures with more than BW_WIN atoms take a general kernel: runs of equal
//   dst / src / structure are merged inside the wave by a segmented scan and the
//   run's last lane adds the total with a global atomic. When the flag is
//   raised, whatever the item kernels wrote is cleared and the general kernel
//   takes every edge in chunks of BW_CHUNK, whatever their order.
// Both kernels are launched; each leaves the items of the other at once.
constexpr int BW_SMALL = 128;     // atoms of the small LDS window
constexpr int BW_WIN = 512;       // atoms of a structure held in LDS

// Lane index of the start of this lane's run (runs of equal key over lanes);
// `heads` has bit l set where lane l starts a run (bit 0 always set).
__device__ __forceinline__ int run_start(uint64_t heads, int lane) {
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    return 63 - __builtin_clzll(heads & upto);
}

// key of the lane below (lane 0: its own), by a DPP wave shift
__device__ __forceinline__ int32_t key_below(int32_t key) {
    return __builtin_amdgcn_update_dpp(key, key, 0x138, 0xf, 0xf, false);   // wave_shr:1
}

__device__ __forceinline__ uint64_t run_heads(int32_t key, int lane) {
    const int32_t prev = key_below(key);
    return ballot(lane == 0 || prev != key);
}

__device__ __forceinline__ bool run_tail(uint64_t heads, int lane) {
    return lane == 63 || ((heads >> (lane + 1)) & 1ull);
}

// Inclusive scan of v restricted to this lane's run [rs, lane].
template <typename T>
__device__ __forceinline__ T seg_scan(T v, int rs, int lane) {
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const T y = __shfl_up(v, d, WAVE);
        if (lane - d >= rs) v += y;
    }
    return v;
}

// The same for floats with DPP (VALU only): row shifts inside rows of 16
// lanes, then the last lane of the row below (row_bcast:15) and lane 31
// (row_bcast:31), each added where it lies inside this lane's run.
template <>
__device__ __forceinline__ float seg_scan<float>(float v, int rs, int lane) {
    float y;
    y = dpp_f32<0x111, 0xf>(v);
    v += lane - 1 >= rs ? y : 0.0f;
    y = dpp_f32<0x112, 0xf>(v);
    v += lane - 2 >= rs ? y : 0.0f;
    y = dpp_f32<0x114, 0xf>(v);
    v += lane - 4 >= rs ? y : 0.0f;
    y = dpp_f32<0x118, 0xf>(v);
    v += lane - 8 >= rs ? y : 0.0f;
    y = dpp_f32<0x142, 0xa>(v);
    v += (lane & ~15) - 1 >= rs ? y : 0.0f;
    y = dpp_f32<0x143, 0xc>(v);
    v += 31 >= rs ? y : 0.0f;
    return v;
}

// Edge ranges of the grouped order: start[s] = first edge whose src is at
// least the structure's first atom (start[0] = 0, start[B] = E). One wave per
// structure boundary: a 65-ary search, each step probing 64 positions at once
// (five dependent steps for 50M edges). On edges that are not grouped the
// result is still a set of indices in [0, E]; the item kernels then find edges
// outside their structure and raise the flag.
__global__ __launch_bounds__(256) void k_geom_ranges(const int32_t* __restrict__ src,
                                                     const int64_t* __restrict__ batch_ptr, int B, int64_t E,
                                                     const int64_t* __restrict__ num_edges,
                                                     int64_t* __restrict__ start,
                                                     int32_t* __restrict__ atom_struct) {
    const int64_t Ee = edge_count(E, num_edges);
    const int lane = lane_id();
    const int q = (int)(blockIdx.x * (blockDim.x / WAVE)) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    if (q > B) return;
    if (q < B) {   // the atom -> structure map of the general kernel, written on the way
        const int64_t a1 = batch_ptr[q + 1];
        for (int64_t a = batch_ptr[q] + lane; a < a1; a += WAVE) atom_struct[a] = q;
    }
    if (q == 0 || q == B || Ee == 0) {
        if (lane == 0) start[q] = q == B ? Ee : 0;
        return;
    }
    const int64_t target = batch_ptr[q];
    int64_t lo = 0, hi = Ee;   // the answer lies in [lo, hi]
    while (hi - lo > WAVE) {
        const int64_t span = hi - lo;
        const int64_t p = lo + (span * (lane + 1)) / (WAVE + 1);   // strictly increasing, in [lo, hi)
        const uint64_t below = ballot((int64_t)src[p] < target);
        const int c = __popcll(below);                            // probes below the target
        const int64_t plo = lo + (span * c) / (WAVE + 1);         // probe c - 1, or lo when c = 0
        const int64_t phi = lo + (span * (c + 1)) / (WAVE + 1);   // probe c, or hi when c = 64
        lo = c == 0 ? lo : plo + 1;
        hi = c == WAVE ? hi : phi;
    }
    const int64_t p = lo + lane;
    const uint64_t below = ballot(p < hi && (int64_t)src[min(p, Ee - 1)] < target);
    if (lane == 0) start[q] = lo + __popcll(below);
}

// Items: item_off[s] = number of items of structures < s (one item per
// BW_CHUNK edges, at least one per structure); item_off[B] = total.
// flag[1] and flag[2] count the structures of BW_SMALL < n <= BW_WIN atoms and
// of more than BW_WIN atoms, so that the kernels for those sizes return at
// once when there are none. With the bucket path's workspace (cm_off set), the
// structures of BW_WIN < n <= BK_MAX_BLOCKS * BK_BLOCK atoms get
// nblk = ceil(n / BK_BLOCK) destination blocks: cm_off scans nblk x items
// (their per-(block, chunk) counts) and p3_off scans nblk (their gather
// items); flag[3] = 1 when the counts and the records fit the workspace.
__global__ __launch_bounds__(1024) void k_bwd_items(const int64_t* __restrict__ start,
                                                    const int64_t* __restrict__ batch_ptr, int B,
                                                    int64_t* __restrict__ item_off, int32_t* __restrict__ flag,
                                                    int64_t* __restrict__ cm_off, int64_t* __restrict__ p3_off,
                                                    int64_t m_cap, int64_t e_cap) {
    __shared__ int64_t sh[3][1024];
    const int t = threadIdx.x;
    const int per = (B + 1023) / 1024;
    const int s0 = min(B, t * per), s1 = min(B, s0 + per);
    int64_t sum[3] = {0, 0, 0};
    bool bad = false;   // ranges that are not ordered (edges not grouped)
    int mid = 0, big = 0;
    auto sizes = [&](int q, int64_t& items, int64_t& cm, int64_t& p3) {
        const int64_t n = start[q + 1] - start[q];
        const int64_t na = batch_ptr[q + 1] - batch_ptr[q];
        items = n > BW_CHUNK ? (n + BW_CHUNK - 1) / BW_CHUNK : 1;
        const bool bk = cm_off && na > BW_WIN && na <= (int64_t)BK_MAX_BLOCKS * BK_BLOCK;
        p3 = bk ? (na + BK_BLOCK - 1) / BK_BLOCK : 0;
        cm = p3 * items;
    };
    for (int q = s0; q < s1; ++q) {
        const int64_t n = start[q + 1] - start[q];
        bad |= n < 0;
        int64_t it, cm, p3;
        sizes(q, it, cm, p3);
        sum[0] += it;
        sum[1] += cm;
        sum[2] += p3;
        const int64_t na = batch_ptr[q + 1] - batch_ptr[q];
        mid += (na > BW_SMALL && na <= BW_WIN) ? 1 : 0;
        big += na > BW_WIN ? 1 : 0;
    }
    if (bad) atomicOr(flag, 1);
    if (mid) atomicAdd(flag + 1, mid);
    if (big) atomicAdd(flag + 2, big);
#pragma unroll
    for (int r = 0; r < 3; ++r) sh[r][t] = sum[r];
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t y[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) y[r] = t >= d ? sh[r][t - d] : 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 3; ++r) sh[r][t] += y[r];
        __syncthreads();
    }
    int64_t run[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) run[r] = sh[r][t] - sum[r];
    for (int q = s0; q < s1; ++q) {
        item_off[q] = run[0];
        int64_t it, cm, p3;
        sizes(q, it, cm, p3);
        if (cm_off) {
            cm_off[q] = run[1];
            p3_off[q] = run[2];
        }
        run[0] += it;
        run[1] += cm;
        run[2] += p3;
    }
    if (t == 1023) {
        item_off[B] = sh[0][1023];
        if (cm_off) {
            cm_off[B] = sh[1][1023];
            p3_off[B] = sh[2][1023];
            // every edge of a bucketed structure gets one record; at most start[B] of them
            if (!bad && sh[2][1023] > 0 && sh[1][1023] <= m_cap && start[B] <= e_cap) flag[3] = 1;
        }
    }
}

// Item `item` of the grouped order: its structure, edge range and whether it
// covers the whole structure. False if there is no such item.
struct BwdItem {
    int32_t st;
    int64_t c0, c1, atom0;
    int n;
    bool whole;
};

__device__ __forceinline__ bool bwd_item(int64_t item, int B, const int64_t* __restrict__ start,
                                         const int64_t* __restrict__ item_off,
                                         const int64_t* __restrict__ batch_ptr, BwdItem& it) {
    if (item >= item_off[B]) return false;
    const int lo = wave_search_le(item_off, B, item, lane_id());   // largest s with item_off[s] <= item
    it.st = lo;
    const int64_t k = item - item_off[lo];
    it.c0 = start[lo] + k * BW_CHUNK;
    it.c1 = max(it.c0, min(start[lo + 1], it.c0 + BW_CHUNK));
    it.whole = item_off[lo + 1] - item_off[lo] == 1;
    it.atom0 = batch_ptr[lo];
    it.n = (int)(batch_ptr[lo + 1] - it.atom0);
    return true;
}

// Backward pass of the grouped path, structures of at most WIN atoms. The
// structure's coordinates are staged in LDS; every wave accumulates the
// coordinate gradients of its edges in a private LDS copy with plain
// read-modify-writes (FP32 LDS atomics are several times slower than the
// whole rest of the pass): lanes whose dst is unique in the wave update at
// once, and a lane whose dst another lane of the same step also targets waits
// for a later round (each round every contended atom has one owner, the last
// lane that wrote its tag). Runs of one source are summed in registers (the
// edges are ordered by source), or by a segmented scan when a step mixes
// sources. The length term is evaluated with the metric tensor G = L L^T of
// the structure: |v|^2 = f G f^T, g L^T = c G f^T and f^T g = c f^T f L, so
// no per-edge v is formed and the lattice gradient of the length term is the
// register sum M = sum c f^T f (FP32 per lane, FP64 over lanes and waves),
// multiplied by L once per item. The four
// copies are summed at the end and written with plain stores when the item is
// the whole structure. Each wave walks a contiguous quarter of the item, three
// groups of 64 edges per step with all their loads issued first. A dst outside
// the structure sets flag bit 1, a src outside it (or, where a step mixes
// sources, a src smaller than the previous lane's) sets bit 0 (the results are
// then cleared and recomputed by the general kernel).
template <bool GV, bool GL, int WIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GV ? 5 : 8)))
void k_geom_bwd_lds(const float* __restrict__ lattices, const float* __restrict__ frac,
                    const int64_t* __restrict__ batch_ptr, int B, const int32_t* __restrict__ src,
                    const int32_t* __restrict__ dst, const int32_t* __restrict__ image,
                    const float* __restrict__ gvec, const float* __restrict__ glen,
                    const int64_t* __restrict__ start, const int64_t* __restrict__ item_off,
                    int32_t* __restrict__ flag, float* __restrict__ grad_frac, double* __restrict__ acc, int n_lo) {
    __shared__ float xs[WIN * 3];
    __shared__ float wacc[4][WIN * 3];
    __shared__ int tag[4][WIN];
    __shared__ double red[4][15];
    if (flag[0] != 0) return;
    if (n_lo > 0 && flag[1] == 0) return;   // no structure of this window's sizes
    BwdItem it;
    if (!bwd_item(blockIdx.x, B, start, item_off, batch_ptr, it) || it.n > WIN || it.n <= n_lo) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool gf = grad_frac != nullptr;
    const int n = it.n;
    float* my = wacc[wv];
    int* mytag = tag[wv];
    for (int q = tid; q < 3 * n; q += 256) {
        xs[q] = frac[3 * it.atom0 + q];
        wacc[0][q] = wacc[1][q] = wacc[2][q] = wacc[3][q] = 0.0f;
    }
    __syncthreads();
    const float* Lp = lattices + 9 * (int64_t)it.st;
    float Lf[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Lf[q] = Lp[q];
    // metric tensor G = L L^T (rows of L are the lattice vectors), from FP64
    // rounded once, wave-uniform
    float Gm[6];
    {
        const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const double g = (double)Lf[3 * ia[q]] * Lf[3 * ib[q]] + (double)Lf[3 * ia[q] + 1] * Lf[3 * ib[q] + 1] +
                             (double)Lf[3 * ia[q] + 2] * Lf[3 * ib[q] + 2];
            Gm[q] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int((float)g)));
        }
    }
    const int32_t a0 = (int32_t)it.atom0;
    // this wave's contiguous quarter of the item, as offsets from the item's first edge
    const int64_t qlen = ((it.c1 - it.c0 + 3) / 4 + WAVE - 1) / WAVE * WAVE;
    const int64_t w0 = it.c0 + wv * qlen, w1 = min(it.c1, w0 + qlen);
    const int32_t* srcb = src + it.c0;
    const int32_t* dstb = dst + it.c0;
    const int32_t* imgb = image + 3 * it.c0;
    const float* gvb = GV ? gvec + 3 * it.c0 : nullptr;
    const float* glb = GL ? glen + it.c0 : nullptr;
    const int r1 = (int)(w1 - it.c0);   // end of this wave's range
    int src_cur = -1;   // wave's current source run (local index), -1: none
    float sa0 = 0.f, sa1 = 0.f, sa2 = 0.f;
    // lattice gradient: sum f (x) g_v (upstream vector gradient) and the
    // symmetric M = sum c f f^T of the length term (its part is M L); each lane
    // sums its own edges (at most a 64th of the item) in FP32, the lanes and
    // waves are summed in FP64
    float lv[9], M[6];
#pragma unroll
    for (int q = 0; q < 9; ++q) lv[q] = 0.0f;
#pragma unroll
    for (int q = 0; q < 6; ++q) M[q] = 0.0f;
    bool bad = false, unsorted = false;
    auto add_src_run = [&]() {   // lane 0 adds the wave's source run
        if (src_cur >= 0) {
            const float r0 = wave_sum_f32(sa0), rr1 = wave_sum_f32(sa1), r2 = wave_sum_f32(sa2);
            if (lane == 0) {
                my[3 * src_cur] -= r0;
                my[3 * src_cur + 1] -= rr1;
                my[3 * src_cur + 2] -= r2;
            }
            wave_lds_sync();
        }
        sa0 = sa1 = sa2 = 0.f;
    };
    constexpr int U = 3;   // edge groups in flight per wave (4: 4 % slower, 2: about the same)
    for (int rb = (int)(w0 - it.c0); rb < r1; rb += WAVE * U) {
        int ai[U], aj[U], at[U][3];
        float ag[U][3], al[U];
        // loads without branches (the offset is clamped into the range; lanes past
        // the end are masked later), so all U groups stay in flight together;
        // 32-bit byte offsets from the item's (scalar) bases
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t r = (uint32_t)min(rb + u * WAVE + lane, r1 - 1);
            const uint32_t o4 = r * 4u, o12 = r * 12u;
            ai[u] = *(const int32_t*)((const char*)srcb + o4) - a0;
            aj[u] = *(const int32_t*)((const char*)dstb + o4) - a0;
            const int32_t* ip = (const int32_t*)((const char*)imgb + o12);
            at[u][0] = ip[0];
            at[u][1] = ip[1];
            at[u][2] = ip[2];
            if (GV) {
                const float* gp = (const float*)((const char*)gvb + o12);
                ag[u][0] = gp[0];
                ag[u][1] = gp[1];
                ag[u][2] = gp[2];
            } else {
                ag[u][0] = ag[u][1] = ag[u][2] = 0.0f;
            }
            al[u] = GL ? *(const float*)((const char*)glb + o4) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int base = rb + u * WAVE;
            if (base >= r1) break;                       // uniform
            const bool inr = base + lane < r1;
            const bool oki = (unsigned)ai[u] < (unsigned)n;
            const bool okj = (unsigned)aj[u] < (unsigned)n;
            bad |= inr && !okj;
            unsorted |= inr && !oki;                     // src outside the item's structure
            const bool act = inr && okj && oki;
            const int li = oki ? ai[u] : 0, lj = okj ? aj[u] : 0;
            // FP32 per edge: the gradient is held to 1e-4 relative, and every
            // quantity here is a few roundings away from its FP64 value
            const float f0 = (xs[3 * lj] - xs[3 * li]) + (float)at[u][0];
            const float f1 = (xs[3 * lj + 1] - xs[3 * li + 1]) + (float)at[u][1];
            const float f2 = (xs[3 * lj + 2] - xs[3 * li + 2]) + (float)at[u][2];
            float x0 = 0.f, x1 = 0.f, x2 = 0.f;
            if (GL) {
                // v = f L, |v|^2 = f G f^T and g = c v with c = g_l / |v|; then
                // g L^T = c (G f) and f (x) g = c f f^T L: no per-edge v
                const float h0 = Gm[0] * f0 + Gm[1] * f1 + Gm[2] * f2;
                const float h1 = Gm[1] * f0 + Gm[3] * f1 + Gm[4] * f2;
                const float h2 = Gm[2] * f0 + Gm[4] * f1 + Gm[5] * f2;
                const float l2 = f0 * h0 + f1 * h1 + f2 * h2;
                float c = l2 > 0.0f ? al[u] * __frsqrt_rn(l2) : 0.0f;
                c = act ? c : 0.0f;
                x0 = c * h0;
                x1 = c * h1;
                x2 = c * h2;
                if (acc) {
                    const float c0 = c * f0, c1 = c * f1, c2 = c * f2;
                    M[0] += c0 * f0; M[1] += c0 * f1; M[2] += c0 * f2;
                    M[3] += c1 * f1; M[4] += c1 * f2; M[5] += c2 * f2;
                }
            }
            if (GV) {
                const float g0 = act ? ag[u][0] : 0.0f, g1 = act ? ag[u][1] : 0.0f, g2 = act ? ag[u][2] : 0.0f;
                // g L^T: component k is g . (row k of L)
                x0 += g0 * Lf[0] + g1 * Lf[1] + g2 * Lf[2];
                x1 += g0 * Lf[3] + g1 * Lf[4] + g2 * Lf[5];
                x2 += g0 * Lf[6] + g1 * Lf[7] + g2 * Lf[8];
                if (acc) {
                    lv[0] += f0 * g0; lv[1] += f0 * g1; lv[2] += f0 * g2;
                    lv[3] += f1 * g0; lv[4] += f1 * g1; lv[5] += f1 * g2;
                    lv[6] += f2 * g0; lv[7] += f2 * g1; lv[8] += f2 * g2;
                }
            }
            if (gf) {
                // destination side: rounds of owner lanes (bounded: every round
                // retires at least the owner of each contended atom)
                // (a wave's LDS operations complete in order, so the tag and the
                // accumulator are read back together, one LDS round trip a round)
                bool pend = act;
                for (int round = 0; round < WAVE && ballot(pend) != 0; ++round) {
                    if (pend) mytag[lj] = lane;
                    __builtin_amdgcn_wave_barrier();
                    int tg = -1;
                    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
                    if (pend) {
                        tg = mytag[lj];
                        a0 = my[3 * lj];
                        a1 = my[3 * lj + 1];
                        a2 = my[3 * lj + 2];
                    }
                    const bool own = pend && tg == lane;
                    if (own) {
                        my[3 * lj] = a0 + x0;
                        my[3 * lj + 1] = a1 + x1;
                        my[3 * lj + 2] = a2 + x2;
                    }
                    __builtin_amdgcn_wave_barrier();
                    pend = pend && !own;
                }
                wave_lds_sync();
                // source side
                const int iu = __builtin_amdgcn_readfirstlane(li);   // lane 0 is always in range
                const bool uni = ballot(act && li != iu) == 0;
                if (!(uni && iu == src_cur)) {
                    add_src_run();
                    src_cur = uni ? iu : -1;
                }
                if (src_cur >= 0) {
                    sa0 += x0;
                    sa1 += x1;
                    sa2 += x2;
                } else {
                    // mixed sources: with src non-decreasing over the lanes each
                    // source is one run (checked here: the merge needs it)
                    const int key = act ? li : -1 - lane;   // inactive lanes are runs of their own
                    const int kprev = key_below(key);
                    unsorted |= act && lane > 0 && kprev >= 0 && li < kprev;
                    const uint64_t heads = ballot(lane == 0 || kprev != key);
                    const int rs = run_start(heads, lane);
                    const float y0 = seg_scan(x0, rs, lane), y1 = seg_scan(x1, rs, lane),
                                y2 = seg_scan(x2, rs, lane);
                    if (act && run_tail(heads, lane)) {
                        my[3 * li] -= y0;
                        my[3 * li + 1] -= y1;
                        my[3 * li + 2] -= y2;
                    }
                    wave_lds_sync();
                }
            }
        }
    }
    if (gf) add_src_run();
    if (ballot(bad) != 0 && lane == 0) atomicOr(flag, 2);
    if (ballot(unsorted) != 0 && lane == 0) atomicOr(flag, 1);
    // block sums of lv and M (also orders the LDS updates before the reads below)
#pragma unroll
    for (int q = 0; q < 15; ++q) {
        const double t = wave_sum_f64((double)(q < 9 ? lv[q] : M[q - 9]));
        if (lane == 0) red[wv][q] = t;
    }
    __syncthreads();
    if (acc && tid < 9) {
        const int ra = tid / 3, k = tid - 3 * (tid / 3);
        auto tot = [&](int q) { return (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]); };
        // (M L)[a][k] = sum_b M[a][b] L[b][k], M stored as 00 01 02 11 12 22
        auto msym = [](int x, int y) {   // storage index of M[x][y]
            const int p = x < y ? x : y, q = x < y ? y : x;
            return 3 * p - (p * (p - 1)) / 2 + (q - p);
        };
        double lt = tot(tid);
#pragma unroll
        for (int bq = 0; bq < 3; ++bq) lt += tot(9 + msym(ra, bq)) * (double)Lp[3 * bq + k];
        if (it.whole) acc[9 * (int64_t)it.st + tid] = lt;
        else unsafeAtomicAdd(&acc[9 * (int64_t)it.st + tid], lt);
    }
    if (gf) {
        float* out = grad_frac + 3 * it.atom0;
        for (int q = tid; q < 3 * n; q += 256) {
            const float v = (wacc[0][q] + wacc[1][q]) + (wacc[2][q] + wacc[3][q]);
            if (it.whole) out[q] = v;
            else if (v != 0.0f) unsafeAtomicAdd(&out[q], v);
        }
    }
}

// Bucket path for structures of BW_WIN < n <= BK_MAX_BLOCKS * BK_BLOCK atoms.
// Global float atomics cost about as much per update as a whole edge's
// streaming, and one per destination would dominate the pass, so the
// destination side is transposed instead: every edge's coordinate-gradient
// term is written as a record into the bucket of its destination block
// (BK_BLOCK atoms), and one workgroup per block sums its bucket in LDS and
// adds the block to grad_frac once. Three passes over the items of the
// grouped order: count edges per (block, chunk) in an LDS histogram, a scan of
// the counts in (structure, block, chunk) order gives every bucket's start,
// then the scatter pass computes the terms, places each record at its
// bucket's start plus an LDS cursor, sums the source side per source run (a
// few global atomics per source) and the lattice gradient in registers (nine
// FP64 atomics per item). Edges outside the item's structure set the order
// flag, as in the LDS kernels, and the general kernel then redoes everything.
__device__ __forceinline__ bool bk_layout(const BwdItem& it, int64_t item, const int64_t* __restrict__ item_off,
                                          const int64_t* __restrict__ cm_off, int64_t& k, int64_t& chunks,
                                          int& nblk, int64_t& cmb) {
    k = item - item_off[it.st];
    chunks = item_off[it.st + 1] - item_off[it.st];
    cmb = cm_off[it.st];
    nblk = (int)((cm_off[it.st + 1] - cmb) / chunks);
    return nblk > 0;
}

__global__ __launch_bounds__(256) void k_bk_count(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                                  const int64_t* __restrict__ batch_ptr, int B,
                                                  const int64_t* __restrict__ start,
                                                  const int64_t* __restrict__ item_off,
                                                  const int64_t* __restrict__ cm_off, int32_t* __restrict__ flag,
                                                  uint32_t* __restrict__ bcount) {
    __shared__ uint32_t hist[BK_MAX_BLOCKS];
    if (flag[3] == 0 || flag[0] != 0) return;
    BwdItem it;
    if (!bwd_item(blockIdx.x, B, start, item_off, batch_ptr, it)) return;
    int64_t k, chunks, cmb;
    int nblk;
    if (!bk_layout(it, blockIdx.x, item_off, cm_off, k, chunks, nblk, cmb)) return;
    const int tid = threadIdx.x;
    for (int d = tid; d < nblk; d += 256) hist[d] = 0u;
    __syncthreads();
    const int32_t a0 = (int32_t)it.atom0;
    bool bad = false;
    for (int64_t e = it.c0 + tid; e < it.c1; e += 256) {
        const int i = src[e] - a0, j = dst[e] - a0;
        const bool ok = (unsigned)i < (unsigned)it.n && (unsigned)j < (unsigned)it.n;
        bad |= !ok;
        if (ok) atomicAdd(&hist[j / BK_BLOCK], 1u);
    }
    if (ballot(bad) != 0 && (tid & 63) == 0) atomicOr(flag, 2);
    __syncthreads();
    for (int d = tid; d < nblk; d += 256) bcount[cmb + (int64_t)d * chunks + k] = hist[d];
}

template <bool GV, bool GL>
__global__ __launch_bounds__(256) void k_bk_scatter(const float* __restrict__ lattices, const float* __restrict__ frac,
                                                    const int64_t* __restrict__ batch_ptr, int B,
                                                    const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                                    const int32_t* __restrict__ image,
                                                    const float* __restrict__ gvec, const float* __restrict__ glen,
                                                    const int64_t* __restrict__ start,
                                                    const int64_t* __restrict__ item_off,
                                                    const int64_t* __restrict__ cm_off,
                                                    const int64_t* __restrict__ boff, int32_t* __restrict__ flag,
                                                    float* __restrict__ grad_frac, double* __restrict__ acc,
                                                    float4* __restrict__ rec) {
    __shared__ int64_t base[BK_MAX_BLOCKS];
    __shared__ uint32_t cur[BK_MAX_BLOCKS];
    __shared__ double red[4][15];
    if (flag[3] == 0 || flag[0] != 0) return;
    BwdItem it;
    if (!bwd_item(blockIdx.x, B, start, item_off, batch_ptr, it)) return;
    int64_t k, chunks, cmb;
    int nblk;
    if (!bk_layout(it, blockIdx.x, item_off, cm_off, k, chunks, nblk, cmb)) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int d = tid; d < nblk; d += 256) {
        base[d] = boff[cmb + (int64_t)d * chunks + k];
        cur[d] = 0u;
    }
    __syncthreads();
    const int n = it.n;
    const float* Lp = lattices + 9 * (int64_t)it.st;
    float Lf[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Lf[q] = Lp[q];
    float Gm[6];   // metric tensor G = L L^T from FP64, rounded once, wave-uniform
    {
        const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const double g = (double)Lf[3 * ia[q]] * Lf[3 * ib[q]] + (double)Lf[3 * ia[q] + 1] * Lf[3 * ib[q] + 1] +
                             (double)Lf[3 * ia[q] + 2] * Lf[3 * ib[q] + 2];
            Gm[q] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int((float)g)));
        }
    }
    const int32_t a0 = (int32_t)it.atom0;
    const float* xb = frac + 3 * it.atom0;
    float* gfb = grad_frac + 3 * it.atom0;
    // this wave's contiguous quarter of the item
    const int64_t qlen = ((it.c1 - it.c0 + 3) / 4 + WAVE - 1) / WAVE * WAVE;
    const int64_t w0 = it.c0 + wv * qlen, w1 = min(it.c1, w0 + qlen);
    const int r1 = (int)(w1 - it.c0);
    const int32_t* srcb = src + it.c0;
    const int32_t* dstb = dst + it.c0;
    const int32_t* imgb = image + 3 * it.c0;
    const float* gvb = GV ? gvec + 3 * it.c0 : nullptr;
    const float* glb = GL ? glen + it.c0 : nullptr;
    int src_cur = -1;
    float sa0 = 0.f, sa1 = 0.f, sa2 = 0.f;
    float lv[9], M[6];   // per-lane FP32 sums of this item's edges (FP64 over lanes and waves)
#pragma unroll
    for (int q = 0; q < 9; ++q) lv[q] = 0.0f;
#pragma unroll
    for (int q = 0; q < 6; ++q) M[q] = 0.0f;
    bool bad = false, unsorted = false;
    auto add_src_run = [&]() {   // lane 0 adds the wave's source run
        if (src_cur >= 0) {
            const float r0 = wave_sum_f32(sa0), rr1 = wave_sum_f32(sa1), r2 = wave_sum_f32(sa2);
            if (lane == 0) {
                unsafeAtomicAdd(&gfb[3 * src_cur], -r0);
                unsafeAtomicAdd(&gfb[3 * src_cur + 1], -rr1);
                unsafeAtomicAdd(&gfb[3 * src_cur + 2], -r2);
            }
        }
        sa0 = sa1 = sa2 = 0.f;
    };
    constexpr int U = 4;
    for (int rb = (int)(w0 - it.c0); rb < r1; rb += WAVE * U) {
        int ai[U], aj[U], at[U][3];
        float ag[U][3], al[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t r = (uint32_t)min(rb + u * WAVE + lane, r1 - 1);
            const uint32_t o4 = r * 4u, o12 = r * 12u;
            ai[u] = *(const int32_t*)((const char*)srcb + o4) - a0;
            aj[u] = *(const int32_t*)((const char*)dstb + o4) - a0;
            const int32_t* ip = (const int32_t*)((const char*)imgb + o12);
            at[u][0] = ip[0];
            at[u][1] = ip[1];
            at[u][2] = ip[2];
            if (GV) {
                const float* gp = (const float*)((const char*)gvb + o12);
                ag[u][0] = gp[0];
                ag[u][1] = gp[1];
                ag[u][2] = gp[2];
            } else {
                ag[u][0] = ag[u][1] = ag[u][2] = 0.0f;
            }
            al[u] = GL ? *(const float*)((const char*)glb + o4) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int base_r = rb + u * WAVE;
            if (base_r >= r1) break;   // uniform
            const bool inr = base_r + lane < r1;
            const bool oki = (unsigned)ai[u] < (unsigned)n;
            const bool okj = (unsigned)aj[u] < (unsigned)n;
            bad |= inr && !okj;
            unsorted |= inr && !oki;
            const bool act = inr && okj && oki;
            const int li = oki ? ai[u] : 0, lj = okj ? aj[u] : 0;
            const float f0 = (xb[3 * lj] - xb[3 * li]) + (float)at[u][0];
            const float f1 = (xb[3 * lj + 1] - xb[3 * li + 1]) + (float)at[u][1];
            const float f2 = (xb[3 * lj + 2] - xb[3 * li + 2]) + (float)at[u][2];
            float x0 = 0.f, x1 = 0.f, x2 = 0.f;
            if (GL) {   // g = c v, c = g_l / |v|: g L^T = c (G f), f (x) g = c f f^T L
                const float h0 = Gm[0] * f0 + Gm[1] * f1 + Gm[2] * f2;
                const float h1 = Gm[1] * f0 + Gm[3] * f1 + Gm[4] * f2;
                const float h2 = Gm[2] * f0 + Gm[4] * f1 + Gm[5] * f2;
                const float l2 = f0 * h0 + f1 * h1 + f2 * h2;
                float c = l2 > 0.0f ? al[u] * __frsqrt_rn(l2) : 0.0f;
                c = act ? c : 0.0f;
                x0 = c * h0;
                x1 = c * h1;
                x2 = c * h2;
                if (acc) {
                    const float c0 = c * f0, c1 = c * f1, c2 = c * f2;
                    M[0] += c0 * f0; M[1] += c0 * f1; M[2] += c0 * f2;
                    M[3] += c1 * f1; M[4] += c1 * f2; M[5] += c2 * f2;
                }
            }
            if (GV) {
                const float g0 = act ? ag[u][0] : 0.0f, g1 = act ? ag[u][1] : 0.0f, g2 = act ? ag[u][2] : 0.0f;
                x0 += g0 * Lf[0] + g1 * Lf[1] + g2 * Lf[2];
                x1 += g0 * Lf[3] + g1 * Lf[4] + g2 * Lf[5];
                x2 += g0 * Lf[6] + g1 * Lf[7] + g2 * Lf[8];
                if (acc) {
                    lv[0] += f0 * g0; lv[1] += f0 * g1; lv[2] += f0 * g2;
                    lv[3] += f1 * g0; lv[4] += f1 * g1; lv[5] += f1 * g2;
                    lv[6] += f2 * g0; lv[7] += f2 * g1; lv[8] += f2 * g2;
                }
            }
            if (grad_frac) {
                // destination side: a record in the destination block's bucket at the
                // block's LDS cursor (integer LDS atomics are cheap; float ones are not)
                if (act) {
                    const int db = lj / BK_BLOCK;
                    const int64_t pos = base[db] + (int64_t)atomicAdd(&cur[db], 1u);
                    rec[pos] = make_float4(x0, x1, x2, __int_as_float(lj - db * BK_BLOCK));
                }
                // source side: runs of one source summed in the wave
                const int iu = __builtin_amdgcn_readfirstlane(li);
                const bool uni = ballot(act && li != iu) == 0;
                if (!(uni && iu == src_cur)) {
                    add_src_run();
                    src_cur = uni ? iu : -1;
                }
                if (src_cur >= 0) {
                    sa0 += x0;
                    sa1 += x1;
                    sa2 += x2;
                } else {
                    const int key = act ? li : -1 - lane;
                    const int kprev = key_below(key);
                    unsorted |= act && lane > 0 && kprev >= 0 && li < kprev;
                    const uint64_t heads = ballot(lane == 0 || kprev != key);
                    const int rs = run_start(heads, lane);
                    const float y0 = seg_scan(x0, rs, lane), y1 = seg_scan(x1, rs, lane), y2 = seg_scan(x2, rs, lane);
                    if (act && run_tail(heads, lane)) {
                        unsafeAtomicAdd(&gfb[3 * li], -y0);
                        unsafeAtomicAdd(&gfb[3 * li + 1], -y1);
                        unsafeAtomicAdd(&gfb[3 * li + 2], -y2);
                    }
                }
            }
        }
    }
    if (grad_frac) add_src_run();
    if (ballot(bad) != 0 && lane == 0) atomicOr(flag, 2);
    if (ballot(unsorted) != 0 && lane == 0) atomicOr(flag, 1);
    if (acc) {
#pragma unroll
        for (int q = 0; q < 15; ++q) {
            const double t = wave_sum_f64((double)(q < 9 ? lv[q] : M[q - 9]));
            if (lane == 0) red[wv][q] = t;
        }
        __syncthreads();
        if (tid < 9) {
            const int ra = tid / 3, kk = tid - 3 * (tid / 3);
            auto tot = [&](int q) { return (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]); };
            auto msym = [](int x, int y) {
                const int p = x < y ? x : y, q = x < y ? y : x;
                return 3 * p - (p * (p - 1)) / 2 + (q - p);
            };
            double lt = tot(tid);
#pragma unroll
            for (int bq = 0; bq < 3; ++bq) lt += tot(9 + msym(ra, bq)) * (double)Lp[3 * bq + kk];
            unsafeAtomicAdd(&acc[9 * (int64_t)it.st + tid], lt);
        }
    }
}

// Gather: one workgroup per destination block of a bucketed structure sums
// its bucket's records and adds them to the block's rows of grad_frac (which
// then hold only the source-side sums of the scatter pass). Each wave takes a
// quarter of the bucket into its own LDS copy of the block, with plain
// read-modify-writes in owner rounds (a lane whose atom another lane of the
// same step also targets waits for a later round; LDS float atomics measured
// several times slower); the four copies are summed at the end.
__global__ __launch_bounds__(256) void k_bk_gather(const int64_t* __restrict__ batch_ptr, int B,
                                                   const int64_t* __restrict__ item_off,
                                                   const int64_t* __restrict__ cm_off,
                                                   const int64_t* __restrict__ p3_off,
                                                   const int64_t* __restrict__ boff, const int32_t* __restrict__ flag,
                                                   const float4* __restrict__ rec, float* __restrict__ grad_frac) {
    __shared__ float accl[4][BK_BLOCK * 3];
    __shared__ int tag[4][BK_BLOCK];
    if (flag[3] == 0 || flag[0] != 0) return;
    const int64_t q = blockIdx.x;
    if (q >= p3_off[B]) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int st = __builtin_amdgcn_readfirstlane(wave_search_le(p3_off, B, q, lane));
    const int d = (int)(q - p3_off[st]);
    const int64_t chunks = item_off[st + 1] - item_off[st];
    const int64_t cmb = cm_off[st];
    const int64_t r0 = boff[cmb + (int64_t)d * chunks], r1 = boff[cmb + (int64_t)(d + 1) * chunks];
    for (int x = tid; x < 4 * 3 * BK_BLOCK; x += 256) (&accl[0][0])[x] = 0.0f;
    __syncthreads();
    float* my = accl[wv];
    int* mytag = tag[wv];
    const int64_t qlen = ((r1 - r0 + 3) / 4 + WAVE - 1) / WAVE * WAVE;
    const int64_t w0 = r0 + wv * qlen, w1 = min(r1, w0 + qlen);
    constexpr int U = 4;
    for (int64_t rb = w0; rb < w1; rb += U * WAVE) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t r = rb + u * WAVE + lane;
            v[u] = r < w1 ? rec[r] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (rb + u * WAVE >= w1) break;   // uniform
            bool pend = rb + u * WAVE + lane < w1;
            const int li = pend ? __float_as_int(v[u].w) : 0;
            for (int round = 0; round < WAVE && ballot(pend) != 0; ++round) {
                if (pend) mytag[li] = lane;
                wave_lds_sync();
                const bool own = pend && mytag[li] == lane;
                if (own) {
                    my[3 * li] += v[u].x;
                    my[3 * li + 1] += v[u].y;
                    my[3 * li + 2] += v[u].z;
                }
                wave_lds_sync();
                pend = pend && !own;
            }
        }
    }
    __syncthreads();
    const int64_t a0 = batch_ptr[st] + (int64_t)d * BK_BLOCK;
    const int cnt = (int)min((int64_t)BK_BLOCK, batch_ptr[st + 1] - a0);
    float* out = grad_frac + 3 * a0;
    for (int x = tid; x < 3 * cnt; x += 256) out[x] += (accl[0][x] + accl[1][x]) + (accl[2][x] + accl[3][x]);
}

// After the grouped kernels: if the edges turned out not to be grouped (flag
// set), clear what they wrote so that the general kernel, which then takes
// every edge, starts from zero.
__global__ __launch_bounds__(256) void k_bwd_fix(const int32_t* __restrict__ flag, float* __restrict__ grad_frac,
                                                 int64_t n3, double* __restrict__ acc, int64_t n9) {
    if (*flag == 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n3 + n9; q += stride) {
        if (q < n3) {
            if (grad_frac) grad_frac[q] = 0.0f;
        } else if (acc) {
            acc[q - n3] = 0.0;
        }
    }
}

// General kernel: grouped order with structures of more than BW_WIN atoms
// (one workgroup per item), or any other order (one workgroup per BW_CHUNK
// edges). Per-edge math in FP64; merged runs go to global atomics, and every
// edge's lattice term goes to the structure of its own source, so the result
// does not depend on the item's range being exact.
__global__ __launch_bounds__(256) void k_geom_bwd_any(const float* __restrict__ lattices,
                                                      const float* __restrict__ frac,
                                                      const int32_t* __restrict__ atom_struct,
                                                      const int64_t* __restrict__ batch_ptr, int B, int64_t N,
                                                      const int32_t* __restrict__ src,
                                                      const int32_t* __restrict__ dst,
                                                      const int32_t* __restrict__ image, int64_t E,
                                                      const int64_t* __restrict__ num_edges,
                                                      const float* __restrict__ gvec,
                                                      const float* __restrict__ glen,
                                                      const int64_t* __restrict__ start,
                                                      const int64_t* __restrict__ item_off,
                                                      const int32_t* __restrict__ flag,
                                                      const int64_t* __restrict__ cm_off,
                                                      float* __restrict__ grad_frac,
                                                      double* __restrict__ acc) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool grouped = flag[0] == 0;
    if (grouped && flag[2] == 0) return;   // no structure beyond the LDS window
    int64_t c0, c1;
    BwdItem it;
    it.st = -1;
    it.whole = false;
    if (grouped) {
        if (!bwd_item(blockIdx.x, B, start, item_off, batch_ptr, it) || it.n <= BW_WIN) return;
        if (flag[3] != 0 && cm_off[it.st + 1] > cm_off[it.st]) return;   // taken by the bucket path
        c0 = it.c0;
        c1 = it.c1;
    } else {
        const int64_t Ee = edge_count(E, num_edges);
        c0 = (int64_t)blockIdx.x * BW_CHUNK;
        if (c0 >= Ee) return;
        c1 = min(Ee, c0 + BW_CHUNK);
    }
    const int64_t qlen = ((c1 - c0 + 3) / 4 + WAVE - 1) / WAVE * WAVE;
    const int64_t w0 = c0 + wv * qlen, w1 = min(c1, w0 + qlen);
    int32_t src_cur = -1;   // wave's current source run (uniform), -1: none
    float sa0 = 0.f, sa1 = 0.f, sa2 = 0.f;
    int32_t st_cur = -1;    // wave's current structure run, -1: none
    double la[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) la[q] = 0.0;
    auto add_atom = [&](int32_t a, float y0, float y1, float y2) {
        unsafeAtomicAdd(&grad_frac[3 * (int64_t)a], y0);
        unsafeAtomicAdd(&grad_frac[3 * (int64_t)a + 1], y1);
        unsafeAtomicAdd(&grad_frac[3 * (int64_t)a + 2], y2);
    };
    auto flush_src = [&]() {
        if (src_cur >= 0) {
            const float r0 = wave_sum_f32(sa0), r1 = wave_sum_f32(sa1), r2 = wave_sum_f32(sa2);
            if (lane == 0) add_atom(src_cur, r0, r1, r2);
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
    for (int64_t base = w0; base < w1; base += WAVE) {
        const int64_t e = base + lane;
        int32_t i = -1, j = -1, s = -1;
        bool act = e < w1;
        double f0 = 0, f1 = 0, f2 = 0, g0 = 0, g1 = 0, g2 = 0;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if (act) {
            i = src[e];
            j = dst[e];
            act = i >= 0 && j >= 0 && i < N && j < N;
            if (!act) i = j = -1;
        }
        if (act) {
            s = atom_struct[i];   // per edge: correct whatever the order
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
            x0 = (float)(g0 * (double)L[0] + g1 * (double)L[1] + g2 * (double)L[2]);
            x1 = (float)(g0 * (double)L[3] + g1 * (double)L[4] + g2 * (double)L[5]);
            x2 = (float)(g0 * (double)L[6] + g1 * (double)L[7] + g2 * (double)L[8]);
        }
        if (grad_frac) {
            {   // destination side: merge runs of equal dst; the run's last lane adds
                const uint64_t heads = run_heads(j, lane);
                const int rs = run_start(heads, lane);
                const float y0 = seg_scan(x0, rs, lane), y1 = seg_scan(x1, rs, lane), y2 = seg_scan(x2, rs, lane);
                if (j >= 0 && run_tail(heads, lane)) add_atom(j, y0, y1, y2);
            }
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
            } else if (am) {
                const uint64_t heads = run_heads(i, lane);
                const int rs = run_start(heads, lane);
                const float y0 = seg_scan(x0, rs, lane), y1 = seg_scan(x1, rs, lane), y2 = seg_scan(x2, rs, lane);
                if (i >= 0 && run_tail(heads, lane)) add_atom(i, -y0, -y1, -y2);
            }
        }
        if (acc) {
            {
                const uint64_t am = ballot(act);
                const int fl = am ? __builtin_ctzll(am) : 0;
                const int32_t su = am ? __builtin_amdgcn_readlane(s, fl) : -1;
                const bool uni = su >= 0 && ballot(act && s != su) == 0;
                if (!(uni && su == st_cur)) {
                    flush_lat();
                    st_cur = uni ? su : -1;
                }
                if (st_cur < 0 && am) {
                    const uint64_t heads = run_heads(s, lane);
                    const int rs = run_start(heads, lane);
                    const bool tail = s >= 0 && run_tail(heads, lane);
#pragma unroll 1
                    for (int q = 0; q < 9; ++q) {
                        const int a = q / 3, b = q - 3 * (q / 3);
                        const double Fa = a == 0 ? f0 : (a == 1 ? f1 : f2);
                        const double Gb = b == 0 ? g0 : (b == 1 ? g1 : g2);
                        const double y = seg_scan(Fa * Gb, rs, lane);
                        if (tail) unsafeAtomicAdd(&acc[9 * (int64_t)s + q], y);
                    }
                    continue;
                }
            }
            la[0] += f0 * g0; la[1] += f0 * g1; la[2] += f0 * g2;
            la[3] += f1 * g0; la[4] += f1 * g1; la[5] += f1 * g2;
            la[6] += f2 * g0; la[7] += f2 * g1; la[8] += f2 * g2;
        }
    }
    if (grad_frac) flush_src();
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

// Plan of the grouped path: flag cleared, edge ranges, items.
// (the flag and counters are cleared by the caller's k_zero_bwd)
static void launch_plan(const int32_t* src, const int64_t* batch_ptr, int B, int64_t E, const int64_t* num_edges,
                        const GeomBwdWs& w, int32_t* atom_struct, hipStream_t s) {
    hipLaunchKernelGGL(k_geom_ranges, dim3((unsigned)((B + 1 + 3) / 4)), dim3(256), 0, s, src, batch_ptr, B, E,
                       num_edges, w.start, atom_struct);
    hipLaunchKernelGGL(k_bwd_items, dim3(1), dim3(1024), 0, s, w.start, batch_ptr, B, w.item_off, w.flag, w.cm_off,
                       w.p3_off, w.m_cap, w.e_cap);
}

// Enough workgroups for either order: sum_s max(1, ceil(E_s / chunk)) <= B + ceil(E / chunk).
static unsigned item_grid(int B, int64_t E) { return (unsigned)((int64_t)B + (E + BW_CHUNK - 1) / BW_CHUNK); }

hipError_t launch_geometry_fwd(const float* lattices, const float* frac, const int32_t* atom_struct,
                               const int64_t* batch_ptr, int B, int64_t N, const int32_t* src,
                               const int32_t* dst, const int32_t* image, int64_t E, const int64_t* num_edges,
                               float* vec, float* length, const GeomBwdWs& w, hipStream_t s) {
    (void)batch_ptr;
    (void)w;
    if (E == 0 || B == 0) return hipSuccess;
    const int cu = device_cu_count();
    hipLaunchKernelGGL(k_geom_fwd, dim3(grid_for(E, 256 * 4, 1 << 30)), dim3(256), 0, s, lattices, frac, atom_struct,
                       N, src, dst, image, E, num_edges, vec, length);
    return hipGetLastError();
}

hipError_t launch_geometry_bwd(const float* lattices, const float* frac, int32_t* atom_struct,
                               const int64_t* batch_ptr, int B, int64_t N, const int32_t* src,
                               const int32_t* dst, const int32_t* image, int64_t E,
                               const int64_t* num_edges, const float* grad_vec, const float* grad_length,
                               float* grad_frac, float* grad_lattice, const GeomBwdWs& w, hipStream_t s) {
    const int cu = device_cu_count();
    {
        const int64_t z3 = grad_frac ? 3 * N : 0, z9 = grad_lattice ? 9 * (int64_t)B : 0;
        hipLaunchKernelGGL(k_zero_bwd, dim3(grid_for(z3 + z9 + 4, 256, cu * 4)), dim3(256), 0, s, grad_frac, z3,
                           w.acc, z9, w.flag);
    }
    if (E > 0 && B > 0 && (grad_frac || grad_lattice) && (grad_vec || grad_length)) {
        GeomBwdWs wb = w;
        if (!grad_frac) wb.cm_off = nullptr;   // the bucket path is for the coordinate gradients
        launch_plan(src, batch_ptr, B, E, num_edges, wb, atom_struct, s);
        const unsigned grid = item_grid(B, E);
        double* acc = grad_lattice ? w.acc : nullptr;
        // two LDS sizes: structures of up to 128 atoms (most), and 129..BW_WIN atoms
#define MG_BWD_LDS(GV, GL, WIN, LO)                                                                           \
    hipLaunchKernelGGL((k_geom_bwd_lds<GV, GL, WIN>), dim3(grid), dim3(256), 0, s, lattices, frac, batch_ptr, B, \
                       src, dst, image, grad_vec, grad_length, w.start, w.item_off, w.flag, grad_frac, acc, LO)
#define MG_BWD_LDS2(GV, GL)              \
    do {                                 \
        MG_BWD_LDS(GV, GL, BW_SMALL, 0);        \
        MG_BWD_LDS(GV, GL, BW_WIN, BW_SMALL);   \
    } while (0)
        if (grad_vec && grad_length) MG_BWD_LDS2(true, true);
        else if (grad_vec) MG_BWD_LDS2(true, false);
        else MG_BWD_LDS2(false, true);
#undef MG_BWD_LDS2
#undef MG_BWD_LDS
        if (wb.cm_off) {   // bucket path for the structures of more than BW_WIN atoms
            hipLaunchKernelGGL(k_bk_count, dim3(grid), dim3(256), 0, s, src, dst, batch_ptr, B, w.start, w.item_off,
                               w.cm_off, w.flag, w.bcount);
            hipError_t e = launch_scan_counts(w.bcount, w.m_cap, w.boff, w.bsum, INT64_MAX, nullptr, s, w.cm_off + B);
            if (e != hipSuccess) return e;
#define MG_BK(GV, GL)                                                                                          \
    hipLaunchKernelGGL((k_bk_scatter<GV, GL>), dim3(grid), dim3(256), 0, s, lattices, frac, batch_ptr, B, src, dst, \
                       image, grad_vec, grad_length, w.start, w.item_off, w.cm_off, w.boff, w.flag, grad_frac, acc, \
                       w.rec)
            if (grad_vec && grad_length) MG_BK(true, true);
            else if (grad_vec) MG_BK(true, false);
            else MG_BK(false, true);
#undef MG_BK
            const int64_t p3_grid = (N + BK_BLOCK - 1) / BK_BLOCK + B;   // >= the blocks of all structures
            hipLaunchKernelGGL(k_bk_gather, dim3((unsigned)p3_grid), dim3(256), 0, s, batch_ptr, B, w.item_off,
                               w.cm_off, w.p3_off, w.boff, w.flag, w.rec, grad_frac);
        }
        const int64_t n3 = grad_frac ? 3 * N : 0, n9 = acc ? 9 * (int64_t)B : 0;
        hipLaunchKernelGGL(k_bwd_fix, dim3(grid_for(n3 + n9, 256, cu * 4)), dim3(256), 0, s, w.flag, grad_frac, n3,
                           acc, n9);
        hipLaunchKernelGGL(k_geom_bwd_any, dim3(grid), dim3(256), 0, s, lattices, frac, atom_struct, batch_ptr, B, N,
                           src, dst, image, E, num_edges, grad_vec, grad_length, w.start, w.item_off, w.flag,
                           wb.cm_off, grad_frac, acc);
    }
    if (grad_lattice && B > 0)
        hipLaunchKernelGGL(k_finalize_lattice, dim3(grid_for(9 * (int64_t)B, 256, 1 << 30)), dim3(256), 0, s,
                           w.acc, 9 * (int64_t)B, grad_lattice);
    return hipGetLastError();
}

}  // namespace mg

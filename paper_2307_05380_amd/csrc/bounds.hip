// Per-structure FP64 bounds, batch plan and image tables.
//
// For a displacement with ||v|| <= R, the fractional components f = v L^{-1}
// satisfy |f_k| <= R r_k with r_k the norm of column k of L^{-1}, i.e. one over
// the spacing of the lattice planes spanned by the other two vectors. With the
// pair displacement wrapped into [-1/2, 1/2]^3, every image that can hold a
// neighbour within R has |t_k| <= floor(R r_k + 1/2). That box is the region
// of cells the method evaluates so that it contains the search sphere (Sec.
// 2.2, Fig. 2); the image
// tables then keep only the lattice translations whose cell (t + [-1/2,1/2]^3) L
// comes within R of the origin, tested exactly in FP64.
#include "mg_internal.h"

namespace mg {

// ------------------------------------------------------------------ zeroing

// Clears the report and the workspace counters at the start of a call (a
// kernel rather than a memset, so the call can be captured into a HIP graph).
__global__ void k_zero_report(mg_report* __restrict__ rep, Counters* __restrict__ ctr,
                              int64_t num_edges) {
    const int t = threadIdx.x;
    if (t < (int)(sizeof(mg_report) / 4)) reinterpret_cast<uint32_t*>(rep)[t] = 0u;
    if (ctr && t < (int)(sizeof(Counters) / 4)) reinterpret_cast<uint32_t*>(ctr)[t] = 0u;
    __syncthreads();
    if (t == 0) rep->num_edges = num_edges;
}

hipError_t launch_zero_report(mg_report* report, Counters* ctr, int64_t num_edges, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_report, dim3(1), dim3(64), 0, s, report, ctr, num_edges);
    return hipGetLastError();
}

// ------------------------------------------------------------------- bounds

// Smallest float y whose correctly rounded square root is >= c, so that the
// sweep's test l^2 < y is exactly sqrtf(l^2) < c (the strict cutoff on the
// FP32 length). The FP64 square root rounded to FP32 is the correctly rounded
// FP32 square root (53 >= 2 * 24 + 2 bits).
__device__ inline float cutoff_threshold_dev(float c) {
    auto csqrt = [](float v) { return (float)sqrt((double)v); };
    float y = (float)((double)c * (double)c);
    if (csqrt(y) >= c) {
        for (int it = 0; it < 16; ++it) {
            const float d = nextafterf(y, 0.0f);
            if (d <= 0.0f || csqrt(d) < c) break;
            y = d;
        }
    } else {
        for (int it = 0; it < 16 && csqrt(y) < c; ++it) y = nextafterf(y, INFINITY);
    }
    return y;
}

// mode 0: cutoff, radius = cutoff (or the largest per-atom cutoff of the
// structure); mode 1: KNN first search, radius from density.
// One workgroup per structure (one wave, or four for batches of large
// structures): every thread scans coordinates for non-finite values (and
// per-atom cutoffs), four atoms per round, thread 0 does the FP64 lattice work.
__global__ __launch_bounds__(256) void k_bounds(const float* __restrict__ lattices,
                                                const int64_t* __restrict__ ptr,
                                                const float* __restrict__ frac, int B, float radius,
                                                const float* __restrict__ radii, float* __restrict__ thr,
                                                int knn_k, float knn_lambda,
                                                StructInfo* __restrict__ info, PlanRow* __restrict__ plan,
                                                int mode, int opts, int cl_span) {
    __shared__ int s_bad[4], s_far[4];
    __shared__ float s_rmax[4];
    const int b = blockIdx.x;
    if (b >= B) return;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid >> 6;
    const int64_t a0 = ptr[b], a1 = ptr[b + 1];
    bool bad = false;
    bool far = false;   // a coordinate whose cell floor(x) does not fit the cell lists' packed shift
    float rmax = 0.0f;
    auto out = [](float v) { return !(v >= -(float)CL_SHIFT_MAX && v < (float)(CL_SHIFT_MAX + 1)); };
    constexpr int U = 4;
    const int nt = blockDim.x;
    for (int64_t a = a0 + tid; a < a1; a += U * nt) {
        float x[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {   // all loads of the round first
            const int64_t q = a + u * nt < a1 ? a + u * nt : a;
            x[u][0] = frac[3 * q];
            x[u][1] = frac[3 * q + 1];
            x[u][2] = frac[3 * q + 2];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bad |= !(isfinite(x[u][0]) && isfinite(x[u][1]) && isfinite(x[u][2]));
            far |= out(x[u][0]) || out(x[u][1]) || out(x[u][2]);
        }
        if (radii) {
            for (int u = 0; u < U && a + u * nt < a1; ++u) {
                const int64_t q = a + u * nt;
                const float r = radii[q];
                const bool ok = isfinite(r) && r > 0.0f;
                bad |= !ok;
                rmax = ok ? fmaxf(rmax, r) : rmax;
                thr[q] = ok ? cutoff_threshold_dev(r) : 0.0f;
            }
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) rmax = fmaxf(rmax, __shfl_xor(rmax, d, WAVE));
    const bool wbad = ballot(bad) != 0, wfar = ballot(far) != 0;
    if (lane == 0) {
        s_bad[wv] = wbad;
        s_far[wv] = wfar;
        s_rmax[wv] = rmax;
    }
    __syncthreads();
    if (tid != 0) return;
    bool any_bad = false, any_far = false;
    for (int q = 0; q < nt / WAVE; ++q) {
        any_bad |= s_bad[q] != 0;
        any_far |= s_far[q] != 0;
        rmax = fmaxf(rmax, s_rmax[q]);
    }

    StructInfo si;
    uint32_t flags = any_bad ? (uint32_t)MG_FLAG_NONFINITE : 0u;
    bool finite = true;
    for (int q = 0; q < 9; ++q) {
        float v = lattices[9 * b + q];
        finite &= isfinite(v);
        si.L[q] = (double)v;
    }
    if (!finite) flags |= MG_FLAG_NONFINITE;
    const double* L = si.L;
    // rows of the cofactor matrix: c_k = a_{k+1} x a_{k+2}; r_k = |c_k| / |det|
    double c[3][3];
    for (int k = 0; k < 3; ++k) {
        const double* u = L + 3 * ((k + 1) % 3);
        const double* w = L + 3 * ((k + 2) % 3);
        c[k][0] = u[1] * w[2] - u[2] * w[1];
        c[k][1] = u[2] * w[0] - u[0] * w[2];
        c[k][2] = u[0] * w[1] - u[1] * w[0];
    }
    const double det = L[0] * c[0][0] + L[1] * c[0][1] + L[2] * c[0][2];
    double len[3], lsum = 0.0;
    for (int k = 0; k < 3; ++k) {
        len[k] = sqrt(L[3 * k] * L[3 * k] + L[3 * k + 1] * L[3 * k + 1] + L[3 * k + 2] * L[3 * k + 2]);
        lsum += len[k];
    }
    const double scale = len[0] * len[1] * len[2];
    if (!(fabs(det) >= 1e-9 * scale) || !(scale > 0.0)) flags |= MG_FLAG_SINGULAR;
    const int n = (int)(a1 - a0);

    double R = radii ? (double)rmax : (double)radius;
    if (mode == 1 && n > 0 && !(flags & (MG_FLAG_SINGULAR | MG_FLAG_NONFINITE))) {
        // expected number of candidates inside R for a uniform density n / V is
        // n (4/3) pi R^3 / V; aim for lambda of them
        const double lam = (double)knn_lambda * (double)knn_k + 6.0;
        R = cbrt(3.0 * lam * fabs(det) / (4.0 * 3.14159265358979323846 * (double)n));
    }
    // conservative radius for pruning: covers FP32 rounding of the sweep
    const double Rb = R * (1.0 + 1e-6) + 1e-3 + 1e-5 * lsum;
    const bool valid = n > 0 && !(flags & (MG_FLAG_SINGULAR | MG_FLAG_NONFINITE));
    // Cell lists: m_k bins of thickness h_k / m_k >= Rb along every direction
    // (h_k = |det| / |a_{k+1} x a_{k+2}| is the spacing of the lattice planes),
    // so every neighbour within Rb lies in the 27 bins around the source's bin;
    // m_k >= 3 keeps those 27 bins distinct. With a stencil half-width S = 2
    // the bins are at least Rb / 2 thick and the 125 bins within two of the
    // source's bin hold every neighbour (m_k >= 5; otherwise S = 1). Bins are
    // capped at 2n + 64.
    // Cell lists store every atom's cell floor(x) (and u - floor(x)) packed in
    // 10-bit fields; a structure with a coordinate outside [-510, 511) takes the
    // image sweep, which has no such limit.
    int cm[3] = {0, 0, 0};
    double wcl = 0.0;
    bool use_cl = false;
    int cls = 1;
    if (valid && !any_far && !(opts & MG_OPT_CELL_LIST_OFF) &&
        (n >= CL_MIN_ATOMS || (opts & MG_OPT_CELL_LIST_FORCE))) {
        double h[3];
        for (int k = 0; k < 3; ++k)
            h[k] = fabs(det) / sqrt(c[k][0] * c[k][0] + c[k][1] * c[k][1] + c[k][2] * c[k][2]);
        for (int S = cl_span >= 2 ? 2 : 1; S >= 1 && !use_cl; --S) {
            const int mmin = 2 * S + 1;
            bool ok = true;
            for (int k = 0; k < 3; ++k) {
                const double mk = floor(h[k] * S / Rb);
                ok &= mk >= (double)mmin;
                cm[k] = ok ? (int)fmin(mk, 1024.0) : 0;
            }
            if (!ok) continue;
            // shrink the largest direction until the bins fit 2n + 64 (27 bins always fit;
            // when 125 do not, the stencil falls back to 27)
            const double cap = 2.0 * n + 64.0;
            for (int it = 0; it < 4096; ++it) {
                const double tot = (double)cm[0] * cm[1] * cm[2];
                if (tot <= cap) break;
                const int a = (cm[0] >= cm[1] && cm[0] >= cm[2]) ? 0 : (cm[1] >= cm[2] ? 1 : 2);
                const int shrunk = max(mmin, (int)floor(cm[a] * cap / tot));
                cm[a] = shrunk < cm[a] ? shrunk : cm[a] - 1;
                if (cm[a] < mmin) break;
            }
            if ((double)cm[0] * cm[1] * cm[2] > cap || cm[0] < mmin || cm[1] < mmin || cm[2] < mmin) continue;
            wcl = S * fmin(fmin(h[0] / cm[0], h[1] / cm[1]), h[2] / cm[2]);
            use_cl = true;
            cls = S;
        }
    }
    // quantities of the image tests
    {
        double rh2 = 0.0;
        for (int cnr = 0; cnr < 4; ++cnr) {
            const double e1 = (cnr & 1) ? 0.5 : -0.5, e2 = (cnr & 2) ? 0.5 : -0.5;
            const double dx = 0.5 * L[0] + e1 * L[3] + e2 * L[6];
            const double dy = 0.5 * L[1] + e1 * L[4] + e2 * L[7];
            const double dz = 0.5 * L[2] + e1 * L[5] + e2 * L[8];
            rh2 = fmax(rh2, dx * dx + dy * dy + dz * dz);
        }
        const double far = (double)(float)Rb + sqrt(rh2);   // the radius the image kernel tests with
        si.far2 = far * far;
        for (int k = 0; k < 3; ++k)
            si.hk[k] = fabs(det) / sqrt(c[k][0] * c[k][0] + c[k][1] * c[k][1] + c[k][2] * c[k][2]);
        const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
        for (int q = 0; q < 6; ++q)
            si.Gm[q] = L[3 * ia[q]] * L[3 * ib[q]] + L[3 * ia[q] + 1] * L[3 * ib[q] + 1] +
                       L[3 * ia[q] + 2] * L[3 * ib[q] + 2];
        const double g00 = si.Gm[0], g01 = si.Gm[1], g02 = si.Gm[2], g11 = si.Gm[3], g12 = si.Gm[4],
                     g22 = si.Gm[5];
        si.rGd[0] = 1.0 / g00;
        si.rGd[1] = 1.0 / g11;
        si.rGd[2] = 1.0 / g22;
        si.rD2[0] = 1.0 / (g11 * g22 - g12 * g12);
        si.rD2[1] = 1.0 / (g00 * g22 - g02 * g02);
        si.rD2[2] = 1.0 / (g00 * g11 - g01 * g01);
    }
    int64_t box = 1;
    for (int k = 0; k < 3; ++k) {
        double r = sqrt(c[k][0] * c[k][0] + c[k][1] * c[k][1] + c[k][2] * c[k][2]) / fabs(det);
        double h = floor(Rb * r + 0.5);
        if (!(h <= (double)TMAX)) {     // also catches NaN
            flags |= MG_FLAG_RANGE;
            h = 0.0;
        }
        si.nk[k] = (int)h;
        box *= 2 * (int64_t)si.nk[k] + 1;
    }
    if (use_cl) {
        flags &= ~(uint32_t)MG_FLAG_RANGE;   // the image box is not used
        box = 0;
    }
    if (n == 0 || (flags & (MG_FLAG_SINGULAR | MG_FLAG_NONFINITE | MG_FLAG_RANGE))) box = 0;

    si.atom0 = a0;
    si.n = n;
    si.box = box;
    si.img_off = 0;
    si.images = 0;
    si.zero_img = -1;
    si.R = (float)Rb;
    si.Rs = (float)R;
    si.flags = flags;
    if (mode == 0 && n <= WAVE && n > 0) {
        si.G = WAVE / n;
        si.groups = (n + si.G - 1) / si.G;
    } else {
        si.G = 1;
        si.groups = n;
    }
    // items stay planned for skipped structures (box == 0): the sweeps then
    // write empty results for their sources
    si.mode = use_cl ? 1 : 0;
    si.m[0] = cm[0];
    si.m[1] = cm[1];
    si.m[2] = cm[2];
    si.nbins = use_cl ? cm[0] * cm[1] * cm[2] : 0;
    si.bin_off = 0;
    si.cl_items = use_cl ? si.nbins : 0;   // one work item per bin
    si.wcl = (float)(wcl * (1.0 - 1e-6) - 1e-3);
    si.cl_s = use_cl ? cls : 0;
    si.pad1 = 0;
    if (use_cl) si.groups = 0;
    si.chunks = 1;
    // (4/3) pi rk^3 n / V = k: the KNN passes start below a multiple of it
    si.rk = (mode == 1 && valid) ? (float)cbrt(3.0 * (double)knn_k * fabs(det) / (4.0 * 3.14159265358979323846 * (double)n))
                                 : 0.0f;
    si.xoff = 0;
    info[b] = si;
    const int64_t per = (n <= WAVE) ? (int64_t)min(si.G, n) : 1;   // sources of one group
    const int64_t cost = (si.box > 0 && si.groups > 0) ? per * n * si.box : 0;
    plan[b] = PlanRow{(int32_t)si.box, si.groups, (int32_t)si.cl_items, (int32_t)si.nbins, cost, n, flags};
}

hipError_t launch_bounds(const float* lattices, const int64_t* batch_ptr, const float* frac, int B,
                         int64_t N, float radius, const float* radii, float* thr, int knn_k,
                         float knn_lambda, StructInfo* info, PlanRow* plan, Counters* ctr, mg_report* report, int mode,
                         int opts, int cl_span, hipStream_t s) {
    (void)ctr;
    (void)report;   // the structures' flags reach the report through the plan rows
    if (B == 0) return hipSuccess;
    // four waves per structure only when structures are large on average
    const int nt = (B > 0 && N / B >= 256) ? 256 : 64;
    hipLaunchKernelGGL(k_bounds, dim3(B), dim3(nt), 0, s, lattices, batch_ptr, frac, B, radius, radii, thr,
                       knn_k, knn_lambda, info, plan, mode, opts, cl_span);
    return hipGetLastError();
}

// ------------------------------------------------------- batch plan (scan)

// One workgroup of 1024 threads: exclusive scans over structures of the box
// sizes (image-table offsets) and of the work-item counts. Structures whose
// box does not fit the table capacity are skipped and flagged. Each thread
// takes SCAN_PER consecutive structures per chunk, so a batch of up to
// 1024 * SCAN_PER structures is one round of loads (all in flight together).
//
// Image chunks (chunk_cap > 0, the cutoff sweeps): the items of a batch differ
// in cost by orders of magnitude (densities and sizes spread over decades), and
// one source group is the smallest unit without chunks. A structure whose
// source group costs more than target = (total cost) / CHUNK_TARGET_DIV gets
// C = ceil(cost / target) chunks (at most MAX_CHUNKS and box / CHUNK_MIN_BOX),
// i.e. C items per source group over consecutive ranges of its image table,
// and n * C per-(source, chunk) count slots from a pool of chunk_cap entries;
// while the slots would not fit, the target doubles. Cost = sources of a group
// x destinations x box size (the pruned table size is not known yet).
constexpr int SCAN_PER = 4;
constexpr int SCAN_Q = 5;   // box, items, cell-list items, bins, chunk count slots

__device__ inline int plan_chunks(const PlanRow& pr, int64_t target) {
    if (target <= 0 || pr.cost <= target) return 1;
    const double c = ceil((double)pr.cost / (double)target);   // FP64: no 64-bit integer division
    return (int)fmax(fmin(fmin(c, (double)MAX_CHUNKS), (double)(pr.box / CHUNK_MIN_BOX)), 1.0);
}

__global__ __launch_bounds__(1024) void k_struct_scan(int B, StructInfo* __restrict__ info,
                                                      const PlanRow* __restrict__ plan, int64_t chunk_cap,
                                                      int64_t* __restrict__ item_off,
                                                      int64_t* __restrict__ cl_off,
                                                      int64_t* __restrict__ box_off,
                                                      Counters* __restrict__ ctr,
                                                      mg_report* __restrict__ rep,
                                                      int64_t capacity, int64_t num_edges0) {
    __shared__ int64_t s_part[SCAN_Q][16];
    __shared__ uint32_t s_flags;
    __shared__ int64_t s_base[SCAN_Q];
    __shared__ int64_t s_red[16];
    __shared__ double s_redf[16];
    __shared__ int64_t s_target;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    if (t < SCAN_Q) s_base[t] = 0;
    if (t == 0) s_flags = 0u;
    uint32_t fl = 0u;   // this thread's structures' flags
    // chunk target: total cost, then doubled until the count slots fit
    int64_t target = 0;
    if (chunk_cap > 0) {
        double c = 0.0;   // FP64: the sum is a heuristic and must not overflow
        for (int b = t; b < B; b += 1024) c += (double)plan[b].cost * (double)plan[b].groups;
        c = wave_sum_f64(c);
        if (lane == 0) s_redf[w] = c;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int r = 0; r < 16; ++r) tot += s_redf[r];
            s_target = (int64_t)fmin(fmax(tot / (double)CHUNK_TARGET_DIV, 1.0), 9.0e18);
        }
        __syncthreads();
        target = s_target;
        for (int it = 0; it < 64; ++it) {
            int64_t x = 0;
            for (int b = t; b < B; b += 1024) {
                const int cb = plan_chunks(plan[b], target);
                if (cb > 1) x += (int64_t)plan[b].n * cb;
            }
            x = wave_sum_i64(x);
            __syncthreads();   // s_red reuse
            if (lane == 0) s_red[w] = x;
            __syncthreads();
            int64_t tot = 0;
            for (int r = 0; r < 16; ++r) tot += s_red[r];
            if (tot <= chunk_cap) break;   // uniform over the workgroup
            target = target > (INT64_MAX >> 1) ? INT64_MAX : target * 2;
        }
    }
    __syncthreads();
    bool overflow = false;
    for (int base = 0; base < B; base += 1024 * SCAN_PER) {
        int64_t v[SCAN_PER][SCAN_Q];
        int ch[SCAN_PER];
        int64_t tot[SCAN_Q] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < SCAN_PER; ++u) {
            const int b = base + t * SCAN_PER + u;
            const bool in = b < B;
            const PlanRow pr = plan[in ? b : 0];   // four consecutive rows per thread: coalesced
            fl |= in ? pr.flags : 0u;
            ch[u] = (in && chunk_cap > 0) ? plan_chunks(pr, target) : 1;
            v[u][0] = in ? pr.box : 0;
            v[u][1] = in ? (int64_t)pr.groups * ch[u] : 0;
            v[u][2] = in ? pr.cl_items : 0;
            v[u][3] = in ? pr.nbins : 0;
            v[u][4] = ch[u] > 1 ? (int64_t)pr.n * ch[u] : 0;
#pragma unroll
            for (int q = 0; q < SCAN_Q; ++q) tot[q] += v[u][q];
        }
        int64_t inc[SCAN_Q];
#pragma unroll
        for (int q = 0; q < SCAN_Q; ++q) {
            inc[q] = wave_incl_scan_i64(tot[q]);
            if (lane == 63) s_part[q][w] = inc[q];
        }
        __syncthreads();
        int64_t pre[SCAN_Q];
#pragma unroll
        for (int q = 0; q < SCAN_Q; ++q) {
            pre[q] = s_base[q] + inc[q] - tot[q];
            for (int r = 0; r < w; ++r) pre[q] += s_part[q][r];
        }
#pragma unroll
        for (int u = 0; u < SCAN_PER; ++u) {
            const int b = base + t * SCAN_PER + u;
            if (b < B) {
                const int64_t off = pre[0];
                box_off[b] = off;   // the image scatter turns it into the table offset
                if (off + v[u][0] > capacity && v[u][0] > 0) {
                    overflow = true;
                    info[b].box = 0;           // skipped: no images; its items write empty results
                    info[b].flags |= MG_FLAG_IMAGES;
                }
                item_off[b] = pre[1];
                if (cl_off) cl_off[b] = pre[2];
                if (v[u][3] > 0) info[b].bin_off = pre[3];   // read by the cell-list kernels only
                if (ch[u] > 1) {
                    info[b].chunks = ch[u];
                    info[b].xoff = pre[4];
                }
            }
#pragma unroll
            for (int q = 0; q < SCAN_Q; ++q) pre[q] += v[u][q];
        }
        __syncthreads();
        if (t == 1023) {
#pragma unroll
            for (int q = 0; q < SCAN_Q; ++q) s_base[q] = pre[q];
        }
        __syncthreads();
    }
    // the call's report and counters start here (the kernels after this one add to them)
    if (overflow) fl |= (uint32_t)MG_FLAG_IMAGES;
    if (fl) atomicOr(&s_flags, fl);
    __syncthreads();
    if (t < (int)(sizeof(Counters) / 4)) reinterpret_cast<uint32_t*>(ctr)[t] = 0u;
    if (t >= 64 && t < 64 + (int)(sizeof(mg_report) / 4)) reinterpret_cast<uint32_t*>(rep)[t - 64] = 0u;
    __syncthreads();
    if (t == 0) {
        item_off[B] = s_base[1];
        if (cl_off) cl_off[B] = s_base[2];
        box_off[B] = s_base[0];
        ctr->total_box = s_base[0];
        ctr->total_items = s_base[1];
        ctr->total_cl_items = s_base[2];
        ctr->total_bins = s_base[3];
        rep->num_edges = num_edges0;
        rep->images_needed = s_base[0];
        rep->flags = s_flags;
    }
}

// Skipped structures keep their planned item ranges, so item_off stays a plain
// scan of the planned items.
hipError_t launch_struct_scan(int B, StructInfo* info, const PlanRow* plan, int64_t chunk_cap, int64_t* item_off,
                              int64_t* cl_off,
                              int64_t* box_off, Counters* ctr, mg_report* report, int64_t image_capacity,
                              hipStream_t s, int64_t num_edges0) {
    hipLaunchKernelGGL(k_struct_scan, dim3(1), dim3(1024), 0, s, B, info, plan, chunk_cap, item_off, cl_off, box_off, ctr,
                       report, image_capacity, num_edges0);
    return hipGetLastError();
}

// ------------------------------------------------------------ image tables

// Squared distance from the origin to the cell (t + [-1/2, 1/2]^3) L, exactly:
// the minimum of the convex quadratic q(z) = z G z^T (G = L L^T) over the box
// z in t + [-1/2, 1/2]^3, taken over the faces of the box (vertices, edges,
// 2-faces), each with the unconstrained minimiser of q on the face's affine
// hull when that point lies on the face. The interior is never the answer
// here (t != 0 keeps the origin outside the box). All 26 faces are unrolled;
// the divisions use the structure's precomputed reciprocals.
__device__ __forceinline__ double qform(const double (&G)[3][3], double z0, double z1, double z2) {
    return z0 * (G[0][0] * z0 + 2.0 * (G[0][1] * z1 + G[0][2] * z2)) + z1 * (G[1][1] * z1 + 2.0 * G[1][2] * z2) +
           z2 * G[2][2] * z2;
}

__device__ double cell_min_dist2(const double (&G)[3][3], const double (&rGd)[3], const double (&rD2)[3], int t0,
                                 int t1, int t2) {
    const double t[3] = {(double)t0, (double)t1, (double)t2};
    const double tol = 1e-12;
    double best = 1e300;
    // vertices
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const double z0 = t[0] + ((v & 1) ? 0.5 : -0.5);
        const double z1 = t[1] + ((v & 2) ? 0.5 : -0.5);
        const double z2 = t[2] + ((v & 4) ? 0.5 : -0.5);
        best = fmin(best, qform(G, z0, z1, z2));
    }
    // edges: coordinate f free, the other two at a corner
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const int a = (f + 1) % 3, b = (f + 2) % 3;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double z[3];
            z[a] = t[a] + ((v & 1) ? 0.5 : -0.5);
            z[b] = t[b] + ((v & 2) ? 0.5 : -0.5);
            z[f] = -(G[f][a] * z[a] + G[f][b] * z[b]) * rGd[f];
            const double u = z[f] - t[f];
            if (u >= -0.5 - tol && u <= 0.5 + tol) best = fmin(best, qform(G, z[0], z[1], z[2]));
        }
    }
    // 2-faces: coordinate c fixed at -1/2 or +1/2, the other two free
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int f = (c + 1) % 3, g = (c + 2) % 3;
        const int ff = f < g ? f : g, gg = f < g ? g : f;   // the pair in index order
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            double z[3];
            z[c] = t[c] + (v ? 0.5 : -0.5);
            const double r0 = -G[ff][c] * z[c], r1 = -G[gg][c] * z[c];
            z[ff] = (r0 * G[gg][gg] - G[ff][gg] * r1) * rD2[c];
            z[gg] = (G[ff][ff] * r1 - G[ff][gg] * r0) * rD2[c];
            const double u0 = z[ff] - t[ff], u1 = z[gg] - t[gg];
            if (u0 >= -0.5 - tol && u0 <= 0.5 + tol && u1 >= -0.5 - tol && u1 <= 0.5 + tol)
                best = fmin(best, qform(G, z[0], z[1], z[2]));
        }
    }
    return best;
}

// Every box image of the batch, one thread each: the FP64 shift t.L and a keep
// flag, written into the structure's box-sized slot of the table (tpk = -1 for
// images dropped). Cheap bounds decide most images: the slab bound
// (|t_k| - 1/2) h_k and the sphere bound |t.L| - (half the longest cell
// diagonal) reject, a cell centre inside the ball accepts; the exact distance
// decides the rest. The structure's quantities come precomputed (bounds).
__global__ __launch_bounds__(256) void k_image_flags(int B, const StructInfo* __restrict__ info,
                                                     const int64_t* __restrict__ box_off,
                                                     const Counters* __restrict__ ctr,
                                                     ImageEntry* __restrict__ table, uint32_t* __restrict__ kflag,
                                                     int64_t capacity) {
    const int64_t total = min(ctr->total_box, capacity);
    const int lane = lane_id();
    // whole waves step together over consecutive slots: the wave finds the
    // structures of its first and last slot, each lane then searches only
    // between them
    for (int64_t w0 = grid_wave() * WAVE; w0 < total; w0 += grid_waves() * WAVE) {
        const int64_t idx = w0 + lane;
        const int sa = wave_search_le(box_off, B, w0, lane);
        const int sb = wave_search_le(box_off, B, min(w0 + WAVE, total) - 1, lane);
        if (idx >= total) continue;
        int lo = sa, hi = sb + 1;   // box_off[lo] <= idx < box_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (box_off[mid] <= idx) lo = mid;
            else hi = mid;
        }
        const StructInfo* si = info + lo;
        if (si->box == 0) {               // skipped structure (its slot is never read)
            kflag[idx] = 0u;
            continue;
        }
        const int loc = (int)(idx - box_off[lo]);
        const int n0 = si->nk[0], n1 = si->nk[1], n2 = si->nk[2];
        const int w1 = 2 * n1 + 1, w2 = 2 * n2 + 1;
        const int t2 = loc % w2 - n2;
        const int r = loc / w2;
        const int t1 = r % w1 - n1;
        const int t0 = r / w1 - n0;
        const double* L = si->L;
        const double R = (double)si->R;
        double cx, cy, cz;
        cart64(L, (double)t0, (double)t1, (double)t2, cx, cy, cz);
        const double c2 = cx * cx + cy * cy + cz * cz;
        bool keep;
        if ((t0 | t1 | t2) == 0 || c2 <= R * R) {
            keep = true;
        } else {
            const double slab = fmax(fmax((fabs((double)t0) - 0.5) * si->hk[0], (fabs((double)t1) - 0.5) * si->hk[1]),
                                     (fabs((double)t2) - 0.5) * si->hk[2]);
            if (slab >= R || c2 >= si->far2) {
                keep = false;
            } else {
                const double* g = si->Gm;
                const double G[3][3] = {{g[0], g[1], g[2]}, {g[1], g[3], g[4]}, {g[2], g[4], g[5]}};
                const double rGd[3] = {si->rGd[0], si->rGd[1], si->rGd[2]};
                const double rD2[3] = {si->rD2[0], si->rD2[1], si->rD2[2]};
                keep = cell_min_dist2(G, rGd, rD2, t0, t1, t2) < R * R;
            }
        }
        ImageEntry e;
        e.sx = (float)cx;
        e.sy = (float)cy;
        e.sz = (float)cz;
        e.tpk = keep ? pack_t(t0, t1, t2) : -1;
        table[idx] = e;
        kflag[idx] = keep ? 1u : 0u;
    }
}

// Kept images moved to their compacted slots (kscan: exclusive scan of the keep
// flags over the whole table, so every structure's kept images stay contiguous
// and in lexicographic order); the first B threads also set every structure's
// offset of its compacted images, their number and the index of t = 0 (the
// box centre, always kept).
__global__ __launch_bounds__(256) void k_image_scatter(int B, StructInfo* __restrict__ info,
                                                       const int64_t* __restrict__ box_off,
                                                       const Counters* __restrict__ ctr,
                                                       const ImageEntry* __restrict__ table,
                                                       const uint32_t* __restrict__ kflag,
                                                       const int64_t* __restrict__ kscan,
                                                       ImageEntry* __restrict__ ctable, int64_t capacity) {
    const int64_t total = min(ctr->total_box, capacity);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t idx = t0; idx < total; idx += stride)
        if (kflag[idx]) ctable[kscan[idx]] = table[idx];
    for (int64_t b = t0; b < B; b += stride) {
        StructInfo& si = info[b];
        const int64_t box = si.box, off = box_off[b];
        if (box == 0 || off + box > capacity) {
            si.images = 0;
            si.zero_img = -1;
            continue;
        }
        const int64_t c = ((int64_t)si.nk[0] * (2 * si.nk[1] + 1) + si.nk[1]) * (2 * si.nk[2] + 1) + si.nk[2];
        const int64_t first = kscan[off];
        si.images = (int)(kscan[off + box] - first);
        si.zero_img = kflag[off + c] ? (int)(kscan[off + c] - first) : -1;
        si.img_off = first;
    }
}

hipError_t launch_images(int B, StructInfo* info, const int64_t* box_off, const Counters* ctr, const ImageTables& t,
                         hipStream_t s) {
    if (B == 0) return hipSuccess;
    const int grid = device_cu_count() * 8;
    hipLaunchKernelGGL(k_image_flags, dim3(grid), dim3(256), 0, s, B, info, box_off, ctr, t.box, t.kflag, t.cap);
    // the scan covers the batch's boxes only (their total is known on the device)
    hipError_t e = launch_scan_counts(t.kflag, t.cap, t.kscan, t.kbsum, INT64_MAX, nullptr, s, &ctr->total_box);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_image_scatter, dim3(grid), dim3(256), 0, s, B, info, box_off, ctr, t.box, t.kflag, t.kscan, t.table,
                       t.cap);
    return hipGetLastError();
}

// ----------------------------------------------------- atom -> structure map

__global__ __launch_bounds__(256) void k_atom_struct(const int64_t* __restrict__ ptr, int B,
                                                     int32_t* __restrict__ out) {
    const int b = blockIdx.x;
    if (b >= B) return;
    const int64_t a0 = ptr[b], a1 = ptr[b + 1];
    for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) out[a] = b;
}

hipError_t launch_atom_struct(const int64_t* batch_ptr, int B, int64_t N, int32_t* atom_struct,
                              hipStream_t s) {
    (void)N;
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_atom_struct, dim3(B), dim3(256), 0, s, batch_ptr, B, atom_struct);
    return hipGetLastError();
}

}  // namespace mg

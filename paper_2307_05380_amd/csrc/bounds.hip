// Per-structure FP64 bounds, batch plan and image tables.
//
// For a displacement with ||v|| <= R, the fractional components f = v L^{-1}
// satisfy |f_k| <= R r_k with r_k the norm of column k of L^{-1}, i.e. one over
// the spacing of the lattice planes spanned by the other two vectors. With the
// pair displacement wrapped into [-1/2, 1/2]^3, every image that can hold a
// neighbour within R has |t_k| <= floor(R r_k + 1/2). That box is the paper's
// "evaluated area that covers the search sphere" (Sec. 2.2, Fig. 2); the image
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

// mode 0: cutoff, radius = cutoff; mode 1: KNN first search, radius from density.
// One wave per structure: every lane scans coordinates for non-finite values,
// lane 0 does the FP64 lattice work.
__global__ __launch_bounds__(64) void k_bounds(const float* __restrict__ lattices,
                                               const int64_t* __restrict__ ptr,
                                               const float* __restrict__ frac, int B, float radius,
                                               int knn_k, float knn_lambda,
                                               StructInfo* __restrict__ info,
                                               mg_report* __restrict__ rep, int mode) {
    const int b = blockIdx.x;
    if (b >= B) return;
    const int lane = threadIdx.x;
    const int64_t a0 = ptr[b], a1 = ptr[b + 1];
    bool bad = false;
    for (int64_t a = a0 + lane; a < a1; a += WAVE) {
        float x = frac[3 * a], y = frac[3 * a + 1], z = frac[3 * a + 2];
        bad |= !(isfinite(x) && isfinite(y) && isfinite(z));
    }
    const bool any_bad = ballot(bad) != 0;
    if (lane != 0) return;

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

    double R = (double)radius;
    if (mode == 1 && n > 0 && !(flags & (MG_FLAG_SINGULAR | MG_FLAG_NONFINITE))) {
        // expected number of candidates inside R for a uniform density n / V is
        // n (4/3) pi R^3 / V; aim for lambda of them
        const double lam = (double)knn_lambda * (double)knn_k + 6.0;
        R = cbrt(3.0 * lam * fabs(det) / (4.0 * 3.14159265358979323846 * (double)n));
    }
    // conservative radius for pruning: covers FP32 rounding of the sweep
    const double Rb = R * (1.0 + 1e-6) + 1e-3 + 1e-5 * lsum;
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
    si.pad = 0;
    info[b] = si;
    if (flags) atomicOr(&rep->flags, flags);
}

hipError_t launch_bounds(const float* lattices, const int64_t* batch_ptr, const float* frac, int B,
                         int64_t N, float radius, int knn_k, float knn_lambda, StructInfo* info,
                         Counters* ctr, mg_report* report, int mode, hipStream_t s) {
    (void)N;
    (void)ctr;
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bounds, dim3(B), dim3(64), 0, s, lattices, batch_ptr, frac, B, radius,
                       knn_k, knn_lambda, info, report, mode);
    return hipGetLastError();
}

// ------------------------------------------------------- batch plan (scan)

// One workgroup of 1024 threads: exclusive scans over structures of the box
// sizes (image-table offsets) and of the work-item counts. Structures whose
// box does not fit the table capacity are skipped and flagged.
__global__ __launch_bounds__(1024) void k_struct_scan(int B, StructInfo* __restrict__ info,
                                                      int64_t* __restrict__ item_off,
                                                      Counters* __restrict__ ctr,
                                                      mg_report* __restrict__ rep,
                                                      int64_t capacity) {
    __shared__ int64_t s_box[16], s_item[16];
    __shared__ int64_t s_base_box, s_base_item;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    if (t == 0) {
        s_base_box = 0;
        s_base_item = 0;
    }
    __syncthreads();
    bool overflow = false;
    for (int base = 0; base < B; base += 1024) {
        const int b = base + t;
        int64_t box = 0, items = 0;
        if (b < B) {
            box = info[b].box;
            items = info[b].groups;
        }
        int64_t ib = wave_incl_scan_i64(box);
        int64_t ii = wave_incl_scan_i64(items);
        if (lane == 63) {
            s_box[w] = ib;
            s_item[w] = ii;
        }
        __syncthreads();
        int64_t pb = s_base_box, pi = s_base_item;
        for (int q = 0; q < w; ++q) {
            pb += s_box[q];
            pi += s_item[q];
        }
        if (b < B) {
            const int64_t off = pb + ib - box;
            const bool fits = off + box <= capacity;
            info[b].img_off = off;
            if (!fits && box > 0) {
                overflow = true;
                info[b].box = 0;           // skipped: no images; its items write empty results
                info[b].flags |= MG_FLAG_IMAGES;
            }
            item_off[b] = pi + ii - items;
        }
        __syncthreads();
        if (t == 1023) {
            s_base_box = pb + ib;
            s_base_item = pi + ii;
        }
        __syncthreads();
    }
    if (overflow) atomicOr(&rep->flags, (uint32_t)MG_FLAG_IMAGES);
    if (t == 0) {
        item_off[B] = s_base_item;
        ctr->total_box = s_base_box;
        ctr->total_items = s_base_item;
        rep->images_needed = s_base_box;
    }
}

// Skipped structures keep their planned item ranges, so item_off stays a plain
// scan of the planned items.
hipError_t launch_struct_scan(int B, StructInfo* info, int64_t* item_off, Counters* ctr,
                              mg_report* report, int64_t image_capacity, hipStream_t s) {
    hipLaunchKernelGGL(k_struct_scan, dim3(1), dim3(1024), 0, s, B, info, item_off, ctr, report,
                       image_capacity);
    return hipGetLastError();
}

// ------------------------------------------------------------ image tables

// Squared distance from the origin to the cell (t + [-1/2, 1/2]^3) L, exactly:
// the minimum of the convex quadratic q(z) = z G z^T (G = L L^T) over the box
// z in t + [-1/2, 1/2]^3, taken over all faces of the box (vertices, edges,
// faces, interior), each with the unconstrained minimiser of q on the face's
// affine hull when that point lies on the face.
__device__ double cell_min_dist2(const double G[3][3], int t0, int t1, int t2) {
    const double t[3] = {(double)t0, (double)t1, (double)t2};
    double best = 1e300;
    const double tol = 1e-12;
    // pattern per coordinate: 0 = free, 1 = at -1/2, 2 = at +1/2
    for (int p = 0; p < 27; ++p) {
        int st[3] = {p % 3, (p / 3) % 3, p / 9};
        double z[3];
        int fr[3], nf = 0;
        for (int k = 0; k < 3; ++k) {
            if (st[k] == 0) {
                fr[nf++] = k;
                z[k] = 0.0;
            } else {
                z[k] = t[k] + (st[k] == 1 ? -0.5 : 0.5);
            }
        }
        bool ok = true;
        if (nf == 3) {
            z[0] = z[1] = z[2] = 0.0;       // minimiser of q is the origin
        } else if (nf == 1) {
            const int f = fr[0];
            double rhs = 0.0;
            for (int k = 0; k < 3; ++k)
                if (k != f) rhs -= G[f][k] * z[k];
            z[f] = rhs / G[f][f];
        } else if (nf == 2) {
            const int f = fr[0], g = fr[1];
            const int c = 3 - f - g;
            const double r0 = -G[f][c] * z[c], r1 = -G[g][c] * z[c];
            const double a = G[f][f], bb = G[f][g], d = G[g][g];
            const double det = a * d - bb * bb;
            z[f] = (r0 * d - bb * r1) / det;
            z[g] = (a * r1 - bb * r0) / det;
        }
        for (int q = 0; q < nf; ++q) {
            const int k = fr[q];
            const double u = z[k] - t[k];
            ok &= (u >= -0.5 - tol) && (u <= 0.5 + tol);
        }
        if (!ok) continue;
        double v = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) v += z[i] * G[i][j] * z[j];
        best = fmin(best, v);
    }
    return best;
}

// One workgroup (256 threads) per structure: enumerate the box in
// lexicographic (t0, t1, t2) order, keep the cells within R, compact them in
// order into the table and record where t = 0 landed.
__global__ __launch_bounds__(256) void k_images(int B, StructInfo* __restrict__ info,
                                                ImageEntry* __restrict__ table,
                                                int64_t capacity) {
    __shared__ uint32_t s_cnt[4];
    __shared__ double sL[9];
    __shared__ int s_total;
    const int b = blockIdx.x;
    const int t = threadIdx.x, w = t >> 6;
    const int64_t box = info[b].box;
    const int64_t off = info[b].img_off;
    if (box == 0 || off + box > capacity) {
        if (t == 0) {
            info[b].images = 0;
            info[b].zero_img = -1;
        }
        return;
    }
    if (t < 9) sL[t] = info[b].L[t];
    if (t == 0) s_total = 0;
    const int n0 = info[b].nk[0], n1 = info[b].nk[1], n2 = info[b].nk[2];
    const int w1 = 2 * n1 + 1, w2 = 2 * n2 + 1;
    const double R = (double)info[b].R;
    const double R2 = R * R;
    __syncthreads();
    double G[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            G[i][j] = sL[3 * i] * sL[3 * j] + sL[3 * i + 1] * sL[3 * j + 1] + sL[3 * i + 2] * sL[3 * j + 2];
    ImageEntry* out = table + off;
    for (int64_t base = 0; base < box; base += 256) {
        const int64_t idx = base + t;
        bool keep = false;
        int t0 = 0, t1 = 0, t2 = 0;
        if (idx < box) {
            t2 = (int)(idx % w2) - n2;
            const int64_t r = idx / w2;
            t1 = (int)(r % w1) - n1;
            t0 = (int)(r / w1) - n0;
            keep = (t0 == 0 && t1 == 0 && t2 == 0) || cell_min_dist2(G, t0, t1, t2) < R2;
        }
        const uint64_t m = ballot(keep);
        if ((t & 63) == 0) s_cnt[w] = (uint32_t)__popcll(m);
        __syncthreads();
        int pos = s_total;
        for (int q = 0; q < w; ++q) pos += (int)s_cnt[q];
        pos += (int)mbcnt(m);
        if (keep) {
            ImageEntry e;
            e.sx = (float)(t0 * sL[0] + t1 * sL[3] + t2 * sL[6]);
            e.sy = (float)(t0 * sL[1] + t1 * sL[4] + t2 * sL[7]);
            e.sz = (float)(t0 * sL[2] + t1 * sL[5] + t2 * sL[8]);
            e.tpk = pack_t(t0, t1, t2);
            out[pos] = e;
            if (t0 == 0 && t1 == 0 && t2 == 0) info[b].zero_img = pos;
        }
        __syncthreads();
        if (t == 0) s_total += (int)(s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3]);
        __syncthreads();
    }
    if (t == 0) info[b].images = s_total;
}

hipError_t launch_images(int B, StructInfo* info, ImageEntry* table, int64_t image_capacity,
                         hipStream_t s) {
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_images, dim3(B), dim3(256), 0, s, B, info, table, image_capacity);
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

// k-nearest-neighbour multigraph (Sec. 1; Sec. 2.2, Algorithms 1 and 2).
//
// One wave per source atom. The candidates (j, t) of the source are streamed
// through a per-wave LDS buffer: the paper's ordered stack (new candidates
// joined to the kept ones, ordered by distance, cut to the k nearest), kept on
// chip. A candidate
// survives when its FP32 length is below the current threshold and is
// appended to the buffer; when the buffer is full it is sorted (bitonic, in
// registers across the 64 lanes), cut to the k smallest keys and the threshold
// drops to the k-th length, so the buffer only ever holds plausible
// neighbours. Keys are (length bits << 32 | candidate ordinal); the ordinal
// j * I + image_index follows (dst, t) order because image tables are built in
// lexicographic t order, which gives the tie order (length, dst, t). The
// result is the k smallest keys whatever order the candidates arrive in. A
// candidate is pushed with the bits of its squared length; the length (the
// correctly rounded root) replaces them, with the sign bit set as a marker,
// when the buffer is sorted or ranked, so the root is taken once per key that
// reaches a sort instead of at every sweep step that pushes one.
//
// Lane layout: lane (u, jj) keeps the pair offset of one destination in
// registers and takes every R-th image of the set (R = 64 / min(n, 64) image
// slots), so a batch covers min(n, 64) destinations x R images.
//
// Search area (Algorithm 1). The first pass enumerates the image table built
// for a radius R0 from the structure's density (about lambda * k candidates
// expected), first under a tighter threshold (a multiple of the k-th
// neighbour distance of a uniform density), then, if fewer than k keys lie
// under it, under R0 itself. A source whose stack then holds at least k keys
// is exact: every candidate shorter than R0 lies in the table. Sources with
// fewer than k survivors are queued for the extended pass, which enumerates the
// full image box of radius 2 R0, 4 R0, ... (images computed on the fly in FP64)
// until k are found inside the radius - the expanding search of Algorithm 1,
// which stops once the k-th distance lies inside the region already evaluated.
//
// Every wave-level decision (loop bounds, stack size, threshold, the sort
// branch) is taken on values made explicitly uniform with readfirstlane, every
// helper that shuffles across lanes is force-inlined (no device calls), work is
// handed out cyclically over the grid's waves (loops bounded by the item
// count) and the extended search is capped at
// KNN_MAX_ATTEMPTS radius doublings: every wave reaches its exit.
#include "cl_tile.h"

namespace mg {

namespace {

constexpr int KNN_WAVES = 4;
constexpr int KNN_CAP = 256;   // ordered-stack capacity per wave (keys)
constexpr int KNN_PF = 2;      // table batches read ahead by the first pass
constexpr int KNN_BUF = 256;   // stack room of the first pass (compressed above KNN_BUF - KNN_PF * WAVE keys)
constexpr int KNN_MAX_ATTEMPTS = 24;
constexpr int KNN_BLOCK = 2;   // consecutive first-pass items per wave (4: same time, 8: 15 % slower)

struct KnnShared {
    uint64_t buf[KNN_WAVES][KNN_BUF];
};

__device__ __forceinline__ int ufirst(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float ufirstf(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Value of lane (lane ^ S) without LDS: DPP quad permutes (S = 1, 2), row
// shifts (4), the row rotation by 8 (8) and the gfx950 lane-swap instructions
// (16, 32; the swap of two copies of v leaves the partner's half in the
// returned register that did not keep this lane's own half). Every stride runs
// in the stack compressions of the KNN tests with a wide first radius.
template <int S>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v, int lane) {
    if constexpr (S == 1) {
        return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xf, 0xf, false);   // quad_perm 1,0,3,2
    } else if constexpr (S == 2) {
        return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xf, 0xf, false);   // quad_perm 2,3,0,1
    } else if constexpr (S == 4) {
        const uint32_t up = __builtin_amdgcn_update_dpp(v, v, 0x104, 0xf, 0xf, false);   // row_shl:4
        const uint32_t dn = __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xf, false);   // row_shr:4
        return (lane & 4) ? dn : up;
    } else if constexpr (S == 8) {
        return __builtin_amdgcn_update_dpp(v, v, 0x128, 0xf, 0xf, false);   // row_ror:8
    } else if constexpr (S == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else {
        static_assert(S == 32, "lane strides 1..32");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
}

// The 64-bit key of lane (lane ^ stride), for a stride that is a constant once
// the sorting loops unroll.
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v, int stride, int lane) {
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    uint32_t a, b;
    switch (stride) {
        case 1: a = xor_lane_u32<1>(lo, lane); b = xor_lane_u32<1>(hi, lane); break;
        case 2: a = xor_lane_u32<2>(lo, lane); b = xor_lane_u32<2>(hi, lane); break;
        case 4: a = xor_lane_u32<4>(lo, lane); b = xor_lane_u32<4>(hi, lane); break;
        case 8: a = xor_lane_u32<8>(lo, lane); b = xor_lane_u32<8>(hi, lane); break;
        case 16: a = xor_lane_u32<16>(lo, lane); b = xor_lane_u32<16>(hi, lane); break;
        default: a = xor_lane_u32<32>(lo, lane); b = xor_lane_u32<32>(hi, lane); break;
    }
    return ((uint64_t)b << 32) | a;
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of 64*M keys held as v[r] of lane l = element r*64 + l.
template <int M>
__device__ __forceinline__ void bitonic_sort(uint64_t (&v)[M], int lane) {
#pragma unroll
    for (int size = 2; size <= WAVE * M; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= WAVE) {
                const int rs = stride / WAVE;
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    if ((r & rs) == 0) {
                        const int p = r | rs;
                        const bool asc = (((r * WAVE) & size) == 0);
                        const uint64_t a = v[r], b = v[p];
                        const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
                        v[r] = asc ? lo : hi;
                        v[p] = asc ? hi : lo;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    const uint64_t o = xor_lane_u64(v[r], stride, lane);
                    const bool asc = (((r * WAVE + lane) & size) == 0);
                    const bool lower = (lane & stride) == 0;
                    const bool take_min = (lower == asc);
                    const uint64_t mn = v[r] < o ? v[r] : o, mx = v[r] < o ? o : v[r];
                    v[r] = take_min ? mn : mx;
                }
            }
        }
    }
}

// Key of a pushed candidate: squared length bits (sign bit clear) and ordinal.
// As a ranked key: the correctly rounded length's bits with the sign bit set
// (keys that already are stay as they are; the unused padding key ~0 too).
__device__ __forceinline__ uint64_t len_key(uint64_t key) {
    const uint32_t hi = (uint32_t)(key >> 32);
    const uint32_t lh = __float_as_uint(sqrt_rn_finite(__uint_as_float(hi))) | 0x80000000u;
    return ((uint64_t)((hi >> 31) ? hi : lh) << 32) | (uint32_t)key;
}

template <int M>
__device__ __forceinline__ uint64_t sorted_rank(const uint64_t* buf, int cnt, int lane) {
    uint64_t v[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int e = r * WAVE + lane;
        v[r] = e < cnt ? len_key(buf[e]) : ~0ull;
    }
    bitonic_sort<M>(v, lane);
    return v[0];
}

__device__ __forceinline__ float key_len(uint64_t key) { return __uint_as_float((uint32_t)(key >> 32) & 0x7fffffffu); }

__device__ __forceinline__ float thr_from_len(float l) { return l * l * (1.0f + 3e-6f) + 1e-30f; }

__device__ __forceinline__ void write_invalid(int64_t i, int k, int lane, int32_t* __restrict__ src,
                                              int32_t* __restrict__ dst, int32_t* __restrict__ image,
                                              float* __restrict__ length) {
    if (lane < k) {
        const int64_t e = i * k + lane;
        src[e] = (int32_t)i;
        dst[e] = -1;
        image[3 * e] = image[3 * e + 1] = image[3 * e + 2] = 0;
        length[e] = __builtin_inff();
    }
}

// Image set of one search: either a structure's table (lexicographic) or the
// full box [-n0..n0] x [-n1..n1] x [-n2..n2] enumerated in the same order.
struct ImageSet {
    const ImageEntry* tab;   // table, or nullptr for the box
    uint32_t I;              // number of images
    int zidx;                // index of t = 0
    int n0, n1, n2;          // box half ranges (box only)
};

__device__ __forceinline__ void image_t(const ImageSet& S, uint32_t img, int& t0, int& t1, int& t2) {
    if (S.tab) {
        const int32_t tpk = S.tab[img].tpk;
        t0 = unpack_t0(tpk);
        t1 = unpack_t1(tpk);
        t2 = unpack_t2(tpk);
    } else {
        const uint32_t w1 = 2 * S.n1 + 1, w2 = 2 * S.n2 + 1;
        t2 = (int)(img % w2) - S.n2;
        const uint32_t rr = img / w2;
        t1 = (int)(rr % w1) - S.n1;
        t0 = (int)(rr / w1) - S.n0;
    }
}

// The ordered stack of one wave: cnt keys in buf, threshold tau2 on l^2.
struct Stack {
    int cnt;
    float tau2;
};

// Keep the k smallest of the cnt <= CAP keys in buf (buf[0..k) afterwards) and
// return the threshold their k-th length allows.
template <int CAP>
__device__ __forceinline__ float compress_stack(uint64_t* buf, int cnt, int k, int lane) {
    wave_lds_sync();
    const uint64_t v0 = sorted_rank<CAP / WAVE>(buf, cnt, lane);
    wave_lds_sync();
    if (lane < k) buf[lane] = v0;
    const uint64_t kth = readlane_u64(v0, k - 1);
    return ufirstf(thr_from_len(key_len(kth)));
}

// Push this lane's candidate (pass, l2, ordinal lo) onto the stack of CAP
// keys; when the stack would overflow, keep the k smallest keys and lower the
// threshold first.
template <int CAP = KNN_CAP>
__device__ __forceinline__ void stack_push(Stack& st, bool pass, float l2, uint32_t lo, int k, uint64_t* buf,
                                           int lane) {
    uint64_t m = ballot(pass);
    int c = ufirst(__popcll(m));
    if (c == 0) return;
    if (st.cnt + c > CAP) {
        st.tau2 = ufirstf(fminf(st.tau2, compress_stack<CAP>(buf, st.cnt, k, lane)));
        st.cnt = k;
        pass = pass && l2 < st.tau2;
        m = ballot(pass);
        c = ufirst(__popcll(m));
        wave_lds_sync();
    }
    if (pass) buf[st.cnt + (int)mbcnt(m)] = ((uint64_t)__float_as_uint(l2) << 32) | (uint64_t)lo;
    st.cnt = ufirst(st.cnt + c);
}

// The same push without the capacity test (the caller has made room).
__device__ __forceinline__ void stack_append(Stack& st, bool pass, float l2, uint32_t lo, uint64_t* buf) {
    const uint64_t m = ballot(pass);
    const int c = ufirst(__popcll(m));
    if (c == 0) return;
    if (pass) buf[st.cnt + (int)mbcnt(m)] = ((uint64_t)__float_as_uint(l2) << 32) | (uint64_t)lo;
    st.cnt = ufirst(st.cnt + c);
}

// Stream every candidate (j, t) of source il through the ordered stack with the
// initial threshold tau2. fr: the structure's fractional coordinates. Lane
// (u, jj), lane = u * nn + jj with nn = min(n, 64), holds destination jc + jj
// of the chunk and takes images u, u + R, u + 2R, ... (R = 64 / nn). TAB: the
// images come from the structure's table, KNN_PF batches at a time with every
// load issued before the first is used (indices clamped into the table; a
// second buffer loaded a group ahead measured slower: it costs occupancy); the
// stack is compressed before a group when more than KNN_CAP keys are held, so
// the group's pushes need no test (buf holds KNN_BUF keys). Otherwise the
// images come from the box, computed in FP64, with the test at every push.
// Returns the uniform number of keys left in buf (at most KNN_BUF - KNN_PF * 64,
// which is KNN_CAP).
template <bool TAB>
__device__ __forceinline__ int collect(const ImageSet& S, float tau2, int k, int n, int il, const double* L,
                                       double xi0, double xi1, double xi2, const float* __restrict__ fr,
                                       uint64_t* buf, int lane) {
    Stack st{0, tau2};
    const uint32_t I = S.I;
    const int nn = min(n, WAVE);
    const uint32_t R = (uint32_t)(WAVE / nn);
    const int u = lane / nn;
    const int jj = lane - u * nn;
    for (int jc = 0; jc < n; jc += nn) {
        const int j = jc + jj;
        const bool lok = (uint32_t)u < R && j < n;
        // a lane without a destination sits far away (its squared distances
        // overflow to infinity and pass no threshold)
        float px = 1e30f, py = 1e30f, pz = 1e30f;
        if (lok) {
            double d0 = (double)fr[3 * j] - xi0;
            double d1 = (double)fr[3 * j + 1] - xi1;
            double d2 = (double)fr[3 * j + 2] - xi2;
            d0 -= rint(d0);
            d1 -= rint(d1);
            d2 -= rint(d2);
            double x, y, z;
            cart64(L, d0, d1, d2, x, y, z);
            px = (float)x;
            py = (float)y;
            pz = (float)z;
        }
        // the image of the source's own pair that is the source itself (none: all ones)
        const uint32_t selfm = (lok && j == il) ? (uint32_t)S.zidx : 0xFFFFFFFFu;
        const uint32_t ordj = (uint32_t)j * I;
        auto step = [&](uint32_t m, float sx, float sy, float sz) {
            const float dx = px + sx, dy = py + sy, dz = pz + sz;
            const float l2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const bool pass = l2 < st.tau2 && m < I && m != selfm;
            stack_push(st, pass, l2, ordj + m, k, buf, lane);
        };
        if (TAB) {
            const ImageEntry* tab = S.tab;
            for (uint32_t m0 = 0; m0 < I; m0 += KNN_PF * R) {
                if (st.cnt > KNN_BUF - KNN_PF * WAVE) {
                    st.tau2 = ufirstf(fminf(st.tau2, compress_stack<KNN_BUF>(buf, st.cnt, k, lane)));
                    st.cnt = k;
                    wave_lds_sync();
                }
                float e[KNN_PF][3];
#pragma unroll
                for (int d = 0; d < KNN_PF; ++d) {
                    const uint32_t m = min(m0 + (uint32_t)d * R + (uint32_t)u, I - 1);
                    const ImageEntry t = tab[m];
                    e[d][0] = t.sx;
                    e[d][1] = t.sy;
                    e[d][2] = t.sz;
                }
#pragma unroll
                for (int d = 0; d < KNN_PF; ++d) {
                    const uint32_t mb = m0 + (uint32_t)d * R;
                    if (mb >= I) break;   // uniform
                    const uint32_t m = mb + (uint32_t)u;
                    const float dx = px + e[d][0], dy = py + e[d][1], dz = pz + e[d][2];
                    const float l2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    const bool pass = l2 < st.tau2 && m < I && m != selfm;
                    stack_append(st, pass, l2, ordj + m, buf);
                }
            }
        } else {
            for (uint32_t m = (uint32_t)u, m0 = 0; m0 < I; m0 += R, m += R) {
                float sx = 0.f, sy = 0.f, sz = 0.f;
                if (lok && m < I) {
                    int t0, t1, t2;
                    image_t(S, m, t0, t1, t2);
                    double cx, cy, cz;
                    cart64(L, (double)t0, (double)t1, (double)t2, cx, cy, cz);
                    sx = (float)cx;
                    sy = (float)cy;
                    sz = (float)cz;
                }
                step(m, sx, sy, sz);
            }
        }
    }
    static_assert(KNN_BUF - KNN_PF * WAVE <= KNN_CAP, "the final sort takes at most KNN_CAP keys");
    if (TAB && st.cnt > KNN_BUF - KNN_PF * WAVE) {
        st.tau2 = ufirstf(fminf(st.tau2, compress_stack<KNN_BUF>(buf, st.cnt, k, lane)));
        st.cnt = k;
    }
    wave_lds_sync();
    return st.cnt;
}

// Number of keys among buf[0..cnt) below key, buf padded with all-ones keys up
// to a multiple of 4 (every lane reads the same address: an LDS broadcast).
__device__ __forceinline__ int lds_rank(const uint64_t* buf, int cnt, uint64_t key) {
    int rank = 0;
    for (int q = 0; q < cnt; q += 4) {
        const uint64_t a0 = buf[q], a1 = buf[q + 1], a2 = buf[q + 2], a3 = buf[q + 3];
        rank += (a0 < key ? 1 : 0) + (a1 < key ? 1 : 0) + (a2 < key ? 1 : 0) + (a3 < key ? 1 : 0);
    }
    return rank;
}

// The k smallest of the cnt keys in buf (cnt uniform, k <= cnt <= KNN_CAP):
// returns the rank of this lane's key (k or more: no key for this lane) and the
// key. Up to 128 keys (buf holds at least 128) each key is ranked against all
// of them, read back from LDS (the keys are distinct, their ordinals are): a
// compare and an add per key instead of a sorting network's dependent
// cross-lane exchanges; beyond 64 keys (two per lane) the keys are then placed
// at their ranks. Larger stacks are sorted.
__device__ __forceinline__ int ranked_key(uint64_t* buf, int cnt, int k, int lane, uint64_t& key) {
    if (cnt <= WAVE) {
        key = lane < cnt ? len_key(buf[lane]) : ~0ull;
        wave_lds_sync();
        buf[lane] = key;
        wave_lds_sync();
        const int rank = lds_rank(buf, cnt, key);
        return lane < cnt ? rank : k;
    }
    if (cnt <= 2 * WAVE) {
        const uint64_t a = len_key(buf[lane]);
        const uint64_t b = lane + WAVE < cnt ? len_key(buf[lane + WAVE]) : ~0ull;
        wave_lds_sync();
        buf[lane] = a;
        buf[lane + WAVE] = b;
        wave_lds_sync();
        int ra = 0, rb = 0;
        for (int q = 0; q < cnt; q += 4) {
            const uint64_t a0 = buf[q], a1 = buf[q + 1], a2 = buf[q + 2], a3 = buf[q + 3];
            ra += (a0 < a ? 1 : 0) + (a1 < a ? 1 : 0) + (a2 < a ? 1 : 0) + (a3 < a ? 1 : 0);
            rb += (a0 < b ? 1 : 0) + (a1 < b ? 1 : 0) + (a2 < b ? 1 : 0) + (a3 < b ? 1 : 0);
        }
        wave_lds_sync();
        if (ra < WAVE) buf[ra] = a;
        if (lane + WAVE < cnt && rb < WAVE) buf[rb] = b;
        wave_lds_sync();
        key = buf[lane];   // every rank below 64 is held by one of the cnt > 64 keys
        return lane;
    }
    key = sorted_rank<KNN_CAP / WAVE>(buf, cnt, lane);
    return lane;
}

// Write the k edges of source i from the stack (requires cnt >= k), each key at
// its rank.
__device__ __forceinline__ void emit(const ImageSet& S, int cnt, int k, int64_t i, int64_t atom0,
                                     double xi0, double xi1, double xi2, const float* __restrict__ frac,
                                     uint64_t* buf, int lane, int32_t* __restrict__ src,
                                     int32_t* __restrict__ dst, int32_t* __restrict__ image,
                                     float* __restrict__ length) {
    uint64_t key;
    const int slot = ranked_key(buf, cnt, k, lane, key);
    if (slot < k) {
        const uint32_t qv = (uint32_t)key;
        const uint32_t j = qv / S.I;
        const uint32_t img = qv - j * S.I;
        int t0, t1, t2;
        image_t(S, img, t0, t1, t2);
        const int64_t aj = atom0 + j;
        const double d0 = (double)frac[3 * aj] - xi0, d1 = (double)frac[3 * aj + 1] - xi1,
                     d2 = (double)frac[3 * aj + 2] - xi2;
        const int64_t e = i * k + slot;
        src[e] = (int32_t)i;
        dst[e] = (int32_t)aj;
        image[3 * e] = t0 - (int)rint(d0);
        image[3 * e + 1] = t1 - (int)rint(d1);
        image[3 * e + 2] = t2 - (int)rint(d2);
        length[e] = key_len(key);
    }
}

}  // namespace

// First pass: the sources of image-sweep structures, each with its
// structure's image table (radius R0). Items: item_off scans the sources of
// those structures (skipped structures keep their items and get invalid rows).
// (at most 64 VGPRs: eight waves per SIMD measured 4 % faster than seven)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_knn_first(int B, int k, const StructInfo* __restrict__ info,
                                                   const int64_t* __restrict__ item_off,
                                                   const ImageEntry* __restrict__ table,
                                                   const float* __restrict__ frac,
                                                   int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                   int32_t* __restrict__ image, float* __restrict__ length,
                                                   int32_t* __restrict__ ext_list, Counters* __restrict__ ctr,
                                                   mg_report* __restrict__ rep, int64_t* __restrict__ partials,
                                                   float tau_scale) {
    __shared__ KnnShared sh;
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    uint64_t* buf = sh.buf[wv];
    const uint32_t bad = MG_FLAG_SINGULAR | MG_FLAG_NONFINITE | MG_FLAG_RANGE | MG_FLAG_IMAGES;
    const int64_t total = item_off[B];
    int64_t wave_cand = 0;
    // blocks of KNN_BLOCK consecutive items (mostly sources of one structure)
    // handed out cyclically over the grid's waves; the structure is searched for
    // only when an item lies past the current one's items
    int lo = 0;
    int64_t s_begin = 0, s_end = 0;   // the current structure's items (none yet)
    for (int64_t qb = grid_wave() * KNN_BLOCK; qb < total; qb += grid_waves() * KNN_BLOCK)
    for (int64_t q = qb; q < min(total, qb + KNN_BLOCK); ++q) {
        if (q >= s_end) {   // uniform
            lo = ufirst(wave_search_le(item_off, B, q, lane));
            s_begin = item_off[lo];
            s_end = item_off[lo + 1];
        }
        const StructInfo* si = info + lo;
        const int n = si->n;
        const int64_t atom0 = si->atom0;
        const int il = (int)(q - s_begin);
        const int64_t i = atom0 + il;
        const bool ok = si->box != 0 && si->images > 0 && si->zero_img >= 0 && (si->flags & bad) == 0;
        if (!ok) {
            write_invalid(i, k, lane, src, dst, image, length);
            continue;
        }
        const double* L = si->L;   // read where the pair offsets are formed
        const double xi0 = frac[3 * i], xi1 = frac[3 * i + 1], xi2 = frac[3 * i + 2];
        ImageSet S;
        S.tab = table + si->img_off;
        S.I = (uint32_t)si->images;
        S.zidx = si->zero_img;
        S.n0 = S.n1 = S.n2 = 0;
        if ((uint64_t)n * S.I >= 4294967296ull) {
            if (lane == 0) atomicOr(&rep->flags, (uint32_t)MG_FLAG_RANGE);
            write_invalid(i, k, lane, src, dst, image, length);
            continue;
        }
        wave_cand += (int64_t)n * S.I;
        const double R = (double)si->Rs;
        const float full = (float)(R * R) * (1.0f + 3e-6f);
        // first threshold: tau_scale times the k-th neighbour distance of a
        // uniform density (fewer keys to sort); swept again at the table's
        // radius when fewer than k lie under it
        float first = full;
        {
            const double r = (double)tau_scale * (double)si->rk;
            if (tau_scale > 0.0f && r * r < (double)full) first = ufirstf((float)(r * r));
        }
        const float* fr = frac + 3 * atom0;
        int cnt = 0;
        for (float thr = first;;) {   // one inlined sweep for both thresholds
            cnt = collect<true>(S, thr, k, n, il, L, xi0, xi1, xi2, fr, buf, lane);
            if (cnt >= k || !(thr < full)) break;
            wave_cand += (int64_t)n * S.I;
            thr = full;
        }
        if (cnt >= k) {
            emit(S, cnt, k, i, atom0, xi0, xi1, xi2, frac, buf, lane, src, dst, image, length);
        } else if (lane == 0) {
            const uint32_t pos = atomicAdd(&ctr->knn2_count, 1u);
            ext_list[pos] = (int32_t)i;
            atomicAdd((unsigned long long*)&rep->knn_extended, 1ull);
            atomicOr(&rep->flags, (uint32_t)MG_FLAG_KNN_EXTENDED);
        }
    }
    if (lane == 0) partials[grid_wave()] = wave_cand;
}

// Cell-list pass: one workgroup per home bin of a cell-list structure, the
// stencil bins staged in LDS (cl_tile.h), one wave per source of the home bin.
// Key ordinal: local dst * 32768 + (t0+16, t1+16, t2+16) in 5 bits each, which
// is the (dst, t) order. The sweep keeps candidates by their staged squared
// distance (staged keys: its bits and the candidate's index in the stencil, a
// total order that only has to agree with the distance), within a margin far above
// the staged form's difference from the form every KNN path ranks by
// (knn_l2): (1 + KNN_CL_REL) x the limit + KNN_CL_ABS A^2. At the end the
// staged k-th key and every key within that margin of it get their key
// distance in the shared form, which decides the k nearest and their order, so
// the graph does not depend on the bins or on which pass resolved a source;
// the raw coordinates are read from global memory once per source instead of
// at every sweep step that has a candidate near the threshold. The stencil
// covers every candidate within wcl, so k keys under a threshold at most wcl^2
// are exact. The first sweep uses a tighter threshold, tau_scale times the
// k-th neighbour distance of a uniform density; a source whose k-th key
// distance is not under it is swept again at wcl^2, and one that fails there
// (or has more than 64 keys within the margin of its k-th, or one of them with
// an image component outside [-16, 15]) goes to the extended pass.
constexpr int KNN_CL_CAP = 128;
constexpr float KNN_CL_REL = 1e-4f;   // margin on squared distances: relative part
constexpr float KNN_CL_ABS = 1e-4f;   // and absolute part (A^2)

__device__ __forceinline__ float key_l2(uint64_t key) { return __uint_as_float((uint32_t)(key >> 32)); }
__device__ __forceinline__ float cl_margin(float l2) { return l2 * (1.0f + KNN_CL_REL) + KNN_CL_ABS; }

// Of the k <= cnt <= KNN_CL_CAP staged keys in buf, the keys within the margin
// of the k-th smallest: moved to buf[0..s) in key order (this lane's in v,
// all ones from lane s on), lim = the margin above the k-th. Ranks by LDS
// broadcast as in ranked_key (buf is padded with all-ones keys to 128).
// Returns s, or -1 when more than 64 keys lie within the margin.
__device__ __forceinline__ int cl_near_kth(uint64_t* buf, int cnt, int k, int lane, float& lim, uint64_t& v) {
    const uint64_t a = lane < cnt ? buf[lane] : ~0ull;
    const uint64_t b = lane + WAVE < cnt ? buf[lane + WAVE] : ~0ull;
    wave_lds_sync();
    buf[lane] = a;
    buf[lane + WAVE] = b;
    wave_lds_sync();
    int ra, rb;
    if (cnt <= WAVE) {   // one key per lane (b is the padding: rank cnt)
        ra = lds_rank(buf, cnt, a);
        rb = cnt;
    } else {
        ra = rb = 0;
        for (int q = 0; q < cnt; q += 4) {
            const uint64_t a0 = buf[q], a1 = buf[q + 1], a2 = buf[q + 2], a3 = buf[q + 3];
            ra += (a0 < a ? 1 : 0) + (a1 < a ? 1 : 0) + (a2 < a ? 1 : 0) + (a3 < a ? 1 : 0);
            rb += (a0 < b ? 1 : 0) + (a1 < b ? 1 : 0) + (a2 < b ? 1 : 0) + (a3 < b ? 1 : 0);
        }
    }
    const uint64_t ma = ballot(lane < cnt && ra == k - 1);
    const uint64_t mb = ballot(lane + WAVE < cnt && rb == k - 1);
    const uint64_t kth = ma ? readlane_u64(a, __builtin_ctzll(ma)) : readlane_u64(b, __builtin_ctzll(mb));
    lim = ufirstf(cl_margin(key_l2(kth)));
    const int s = ufirst(__popcll(ballot(lane < cnt && key_l2(a) <= lim)) +
                         __popcll(ballot(lane + WAVE < cnt && key_l2(b) <= lim)));
    if (s > WAVE) return -1;
    wave_lds_sync();
    if (ra < s) buf[ra] = a;   // the keys within the margin are the s smallest
    if (rb < s) buf[rb] = b;
    wave_lds_sync();
    v = lane < s ? buf[lane] : ~0ull;
    return s;
}

__global__ __launch_bounds__(256) void k_knn_cl(int B, int k, const StructInfo* __restrict__ info, ClWs w,
                                                const float* __restrict__ frac,
                                                int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                int32_t* __restrict__ image, float* __restrict__ length,
                                                int32_t* __restrict__ ext_list, Counters* __restrict__ ctr,
                                                mg_report* __restrict__ rep, int64_t* __restrict__ partials,
                                                float tau_scale) {
    __shared__ ClTile tile;
    __shared__ uint64_t sbuf[4][KNN_CL_CAP];
    const int lane = lane_id();
    const int wv = ufirst((int)(threadIdx.x >> 6));
    uint64_t* buf = sbuf[wv];
    const int64_t total = w.cl_off[B];
    int64_t wave_cand = 0;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        ClItem it;
        cl_stage(q, B, info, w, tile, it);
        const StructInfo* si = it.si;
        const int64_t atom0 = si->atom0;
        const int n = si->n;
        const float wc = si->wcl;
        const float full = wc * wc;
        float first = full;
        {   // a multiple of the k-th neighbour distance of a uniform density
            const double r = (double)tau_scale * (double)si->rk;
            if (tau_scale > 0.0f && r * r < (double)full) first = ufirstf((float)(r * r));
        }
        const int T = it.total;
        for (int64_t r = it.hs + wv; r < it.he; r += 4) {
            const ClSource S = cl_source(it, w, r);
            const int s0 = unpack_t0(S.sh), s1 = unpack_t1(S.sh), s2 = unpack_t2(S.sh);
            const int self = it.home + (int)(r - it.hs);   // the source's own candidate (excluded)
            float tau = first;
            bool done = false;
            int overflow = n >= 131072 ? 1 : 0;   // local dst index must fit 17 bits
            for (int attempt = 0; attempt < 2; ++attempt) {
                // staged keys within the margin of the attempt's threshold; when the
                // stack is full only those within the margin of its k-th stay, and
                // the limit drops to that margin
                Stack st{0, ufirstf(cl_margin(tau))};
                auto consider = [&](int c, const float4 e, bool valid) {
                    bool pass = false;
                    float l2 = 0.0f;
                    if (valid) {
                        const float dx = e.x - S.px, dy = e.y - S.py, dz = e.z - S.pz;
                        l2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                        pass = l2 <= st.tau2 && c != self;
                    }
                    uint64_t m = ballot(pass);
                    int cnum = ufirst(__popcll(m));
                    if (cnum == 0) return;
                    if (st.cnt + cnum > KNN_CL_CAP) {   // st.cnt > 64 >= k here
                        float lim;
                        uint64_t v;
                        const int s = cl_near_kth(buf, st.cnt, k, lane, lim, v);
                        if (s < 0) {   // too many near-ties: the extended pass takes the source
                            overflow = 1;
                            st.cnt = 0;
                            st.tau2 = -1.0f;
                        } else {
                            st.cnt = s;
                            st.tau2 = ufirstf(fminf(st.tau2, lim));
                        }
                        pass = pass && l2 <= st.tau2;
                        m = ballot(pass);
                        cnum = ufirst(__popcll(m));
                        wave_lds_sync();
                    }
                    if (pass) buf[st.cnt + (int)mbcnt(m)] = ((uint64_t)__float_as_uint(l2) << 32) | (uint32_t)c;
                    st.cnt = ufirst(st.cnt + cnum);
                };
                if (it.staged) {   // the tile is padded to whole pairs of steps: both read first
                    for (int cb = 0; cb < T; cb += 2 * WAVE) {
                        const float4 e0 = tile.c[cb + lane], e1 = tile.c[cb + WAVE + lane];
                        consider(cb + lane, e0, true);
                        if (cb + WAVE < T) consider(cb + WAVE + lane, e1, true);   // uniform
                    }
                } else {
                    for (int cb = 0; cb < T; cb += WAVE) {
                        const int c = cb + lane;
                        int32_t ct = 0;
                        const float4 e = c < T ? cl_candidate(tile, it, w, c, ct) : make_float4(0.f, 0.f, 0.f, 0.f);
                        consider(c, e, c < T);
                    }
                }
                wave_lds_sync();
                wave_cand += T;
                if (st.cnt >= k && ufirst(ballot(overflow != 0) != 0 ? 1 : 0) == 0) {
                    float lim;
                    uint64_t v;
                    const int s = cl_near_kth(buf, st.cnt, k, lane, lim, v);
                    if (s < 0) {
                        overflow = 1;
                    } else {
                        // the keys within the margin of the k-th: their candidates' image
                        // (each component must fit [-16, 15]) and the shared key form
                        int t0 = 0, t1 = 0, t2 = 0;
                        int64_t ja = 0;
                        float lc = 0.0f;
                        uint64_t ck = ~0ull;
                        if (lane < s) {
                            const int c = (int)(uint32_t)v;
                            int32_t ct;
                            const float4 e = cl_candidate(tile, it, w, c, ct);
                            ja = (int64_t)__float_as_int(e.w);
                            t0 = unpack_t0(ct) + s0;
                            t1 = unpack_t1(ct) + s1;
                            t2 = unpack_t2(ct) + s2;
                            const bool fits = t0 >= -16 && t0 <= 15 && t1 >= -16 && t1 <= 15 && t2 >= -16 && t2 <= 15;
                            overflow |= fits ? 0 : 1;
                            const uint32_t ord = (uint32_t)(ja - atom0) * 32768u +
                                                 (uint32_t)(((t0 + 16) * 32 + (t1 + 16)) * 32 + (t2 + 16));
                            lc = knn_l2(it.L, (double)S.x0, (double)S.x1, (double)S.x2, (double)frac[3 * ja],
                                        (double)frac[3 * ja + 1], (double)frac[3 * ja + 2], t0, t1, t2);
                            ck = ((uint64_t)__float_as_uint(sqrt_rn_finite(lc)) << 32) | (uint64_t)ord;
                        }
                        wave_lds_sync();
                        buf[lane] = ck;   // all ones from lane s on: the padding of the rank loop
                        wave_lds_sync();
                        const int slot = lane < s ? lds_rank(buf, s, ck) : k;
                        // exact when the k-th key distance lies under the attempt's threshold
                        // and every image fits the ordinal
                        if (ballot(overflow != 0) == 0 && ballot(slot == k - 1 && lc < tau) != 0) {
                            if (slot < k) {
                                const int64_t e = S.i * k + slot;
                                src[e] = (int32_t)S.i;
                                dst[e] = (int32_t)ja;
                                image[3 * e] = t0;
                                image[3 * e + 1] = t1;
                                image[3 * e + 2] = t2;
                                length[e] = key_len(ck);
                            }
                            done = true;
                        }
                    }
                }
                wave_lds_sync();   // buf is reused by the next attempt or source
                const int any_overflow = ufirst(ballot(overflow != 0) != 0 ? 1 : 0);
                if (done || any_overflow || !(tau < full)) break;
                tau = full;
            }
            if (!done && lane == 0) {
                const uint32_t pos = atomicAdd(&ctr->knn2_count, 1u);
                ext_list[pos] = (int32_t)S.i;
                atomicAdd((unsigned long long*)&rep->knn_extended, 1ull);
                atomicOr(&rep->flags, (uint32_t)MG_FLAG_KNN_EXTENDED);
            }
        }
        __syncthreads();   // the next item overwrites the tile
    }
    if (lane == 0) partials[grid_wave()] = wave_cand;
}

// Extended pass: the queued sources, full image boxes of radius 2 R0, 4 R0, ...
__global__ __launch_bounds__(256) void k_knn_extended(int k, const StructInfo* __restrict__ info,
                                                      const float* __restrict__ frac,
                                                      const int32_t* __restrict__ atom_struct,
                                                      int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                      int32_t* __restrict__ image, float* __restrict__ length,
                                                      const int32_t* __restrict__ ext_list,
                                                      Counters* __restrict__ ctr, mg_report* __restrict__ rep) {
    __shared__ KnnShared sh;
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    uint64_t* buf = sh.buf[wv];
    const uint32_t total = (uint32_t)ufirst((int)ctr->knn2_count);
    for (int64_t q = grid_wave(); q < (int64_t)total; q += grid_waves()) {
        const int64_t i = (int64_t)ufirst(ext_list[q]);
        const int s = ufirst(atom_struct[i]);
        const StructInfo* si = info + s;
        const int n = si->n;
        const int64_t atom0 = si->atom0;
        const int il = (int)(i - atom0);
        double L[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) L[r] = si->L[r];
        const double xi0 = frac[3 * i], xi1 = frac[3 * i + 1], xi2 = frac[3 * i + 2];
        // plane spacings: r_a = |a_{a+1} x a_{a+2}| / |det|
        double c[3][3], lsum = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double* u = L + 3 * ((a + 1) % 3);
            const double* w = L + 3 * ((a + 2) % 3);
            c[a][0] = u[1] * w[2] - u[2] * w[1];
            c[a][1] = u[2] * w[0] - u[0] * w[2];
            c[a][2] = u[0] * w[1] - u[1] * w[0];
            lsum += sqrt(L[3 * a] * L[3 * a] + L[3 * a + 1] * L[3 * a + 1] + L[3 * a + 2] * L[3 * a + 2]);
        }
        const double det = fabs(L[0] * c[0][0] + L[1] * c[0][1] + L[2] * c[0][2]);
        double rk[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) rk[a] = sqrt(c[a][0] * c[a][0] + c[a][1] * c[a][1] + c[a][2] * c[a][2]) / det;
        double R = (double)si->Rs;
        int done = 0;
        for (int attempt = 0; attempt < KNN_MAX_ATTEMPTS && !done; ++attempt) {
            R *= 2.0;
            const double Rb = R * (1.0 + 1e-6) + 1e-3 + 1e-5 * lsum;
            const double h0 = floor(Rb * rk[0] + 0.5), h1 = floor(Rb * rk[1] + 0.5), h2 = floor(Rb * rk[2] + 0.5);
            const double W = (2 * h0 + 1) * (2 * h1 + 1) * (2 * h2 + 1);
            const int fits = ufirst((h0 <= TMAX && h1 <= TMAX && h2 <= TMAX && (double)n * W < 4294967296.0) ? 1 : 0);
            if (!fits) {
                done = 2;
                break;
            }
            ImageSet S;
            S.tab = nullptr;
            S.n0 = ufirst((int)h0);
            S.n1 = ufirst((int)h1);
            S.n2 = ufirst((int)h2);
            S.I = (uint32_t)((2 * S.n0 + 1) * (2 * S.n1 + 1) * (2 * S.n2 + 1));
            S.zidx = (S.n0 * (2 * S.n1 + 1) + S.n1) * (2 * S.n2 + 1) + S.n2;
            const float tau2 = ufirstf((float)(R * R) * (1.0f + 3e-6f));
            const int cnt = collect<false>(S, tau2, k, n, il, L, xi0, xi1, xi2, frac + 3 * atom0, buf, lane);
            if (cnt >= k) {
                emit(S, cnt, k, i, atom0, xi0, xi1, xi2, frac, buf, lane, src, dst, image, length);
                done = 1;
            }
        }
        if (done != 1) {
            if (lane == 0) atomicOr(&rep->flags, (uint32_t)MG_FLAG_RANGE);
            write_invalid(i, k, lane, src, dst, image, length);
        }
    }
}

hipError_t launch_knn(int B, int64_t N, int k, const StructInfo* info, const int64_t* item_off,
                      const ImageEntry* table, const float* frac, int32_t* src, int32_t* dst,
                      int32_t* image, float* length, int32_t* ext_list, Counters* ctr,
                      mg_report* report, int64_t* partials, int grid, float tau_scale, hipStream_t s) {
    if (N == 0 || B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_knn_first, dim3(grid), dim3(256), 0, s, B, k, info, item_off, table, frac, src, dst,
                       image, length, ext_list, ctr, report, partials, tau_scale);
    return hipGetLastError();
}

hipError_t launch_cl_knn(int B, int k, const StructInfo* info, const ClWs& w, const float* frac,
                         int32_t* src, int32_t* dst, int32_t* image, float* length,
                         int32_t* ext_list, Counters* ctr, mg_report* report, int64_t* partials,
                         int grid, float tau_scale, hipStream_t s) {
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_knn_cl, dim3(grid), dim3(256), 0, s, B, k, info, w, frac, src, dst, image, length,
                       ext_list, ctr, report, partials, tau_scale);
    return hipGetLastError();
}

hipError_t launch_knn_extended(int B, int64_t N, int k, const StructInfo* info, const float* frac,
                               const int32_t* atom_struct, int32_t* src, int32_t* dst,
                               int32_t* image, float* length, const int32_t* ext_list,
                               Counters* ctr, mg_report* report, int grid, hipStream_t s) {
    (void)B;
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_knn_extended, dim3(grid), dim3(256), 0, s, k, info, frac, atom_struct, src, dst,
                       image, length, ext_list, ctr, report);
    return hipGetLastError();
}

}  // namespace mg

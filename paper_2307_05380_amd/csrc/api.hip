// C ABI of libmatgraph (declared in include/matgraph.h): argument validation,
// workspace carving, launch sequencing, tuning state and phase profiling.
// No entry point allocates device memory; every kernel is enqueued on the
// caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mg_internal.h"

namespace {

thread_local std::string g_err;

mg_status fail(mg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

mg_status hip_fail(hipError_t e, const char* what) {
    return fail(MG_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

// The thread's last error message, for entry points outside this file.
mg_status mg::api_fail(mg_status st, const char* msg) { return fail(st, "%s", msg); }

namespace {

std::mutex g_mu;
mg_tuning g_tune = {32, 2, 8, 6, 10, 4, 1, 1};

mg_tuning tuning() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_tune;
}

// ----------------------------------------------------------------- profiling

struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
bool g_prof = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one kernel phase with events on the launch stream when profiling is on.
class Phase {
  public:
    Phase(const char* name, hipStream_t s) : s_(s) {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_prof) return;
        rec_.name = name;
        rec_.a = take_event();
        rec_.b = take_event();
        if (rec_.a && rec_.b && hipEventRecord(rec_.a, s_) == hipSuccess) on_ = true;
    }
    ~Phase() {
        if (!on_) return;
        std::lock_guard<std::mutex> lk(g_mu);
        if (hipEventRecord(rec_.b, s_) == hipSuccess) g_recs.push_back(rec_);
    }

  private:
    hipStream_t s_;
    ProfRec rec_;
    bool on_ = false;
};

template <typename F>
hipError_t phase(const char* name, hipStream_t s, F&& f) {
    Phase p(name, s);
    return f();
}

// ---------------------------------------------------------------- workspace

struct Carver {
    char* base;
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        used = mg::align_up(used, 256);
        T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
        used += count * sizeof(T);
        return p;
    }
};

void carve_cl(Carver& c, int B, int64_t N, mg::Counters* ctr, mg::ClWs& w) {
    w.cap = mg::cl_bin_capacity(B, N);
    w.cl_off = c.take<int64_t>((size_t)B + 1);
    w.bin_count = c.take<uint32_t>((size_t)w.cap);
    w.bin_start = c.take<int64_t>((size_t)w.cap + 1);
    w.bsum = c.take<int64_t>((size_t)((w.cap + 2047) / 2048) + 1);
    w.atom_bin = c.take<int32_t>((size_t)N);
    w.atom_rank = c.take<int32_t>((size_t)N);
    w.slot_atom = c.take<int32_t>((size_t)N);
    w.slot_x = c.take<float4>((size_t)N);
    w.slot_shift = c.take<int32_t>((size_t)N);
    w.atom_struct = c.take<int32_t>((size_t)N);
    w.ctr = ctr;
}

// The image tables take the workspace after the fixed part: per slot a box
// entry, a keep flag, a scan value and a compacted entry.
mg::ImageTables carve_images(Carver& c, size_t bytes) {
    mg::ImageTables t;
    const int64_t room = (int64_t)bytes - (int64_t)c.used - mg::IMAGE_FIXED_BYTES;
    t.cap = room > 0 ? room / mg::IMAGE_SLOT_BYTES : 0;
    if (c.base == nullptr) t.cap = 0;
    t.box = c.take<mg::ImageEntry>((size_t)t.cap);
    t.table = c.take<mg::ImageEntry>((size_t)t.cap);
    t.kscan = c.take<int64_t>((size_t)t.cap + 1);
    t.kflag = c.take<uint32_t>((size_t)t.cap);
    t.kbsum = c.take<int64_t>((size_t)mg::scan_block_count(t.cap) + 1);
    return t;
}

struct CutoffWs {
    mg::Counters* ctr;
    mg::StructInfo* info;
    mg::PlanRow* plan;
    int64_t* item_off;   // sweep items: (structure, source group, image chunk)
    int64_t* box_off;
    uint32_t* counts;
    uint32_t* ccount;    // per-(source, image chunk) counts of chunked structures
    int64_t* offsets;
    int64_t* bsum;
    int64_t* partials;
    float* thr;
    mg::ClWs cl;
    mg::ImageTables img;
    size_t fixed;
};

// Persistent sweep grid: workgroups per CU times the CU count, bounded so the
// per-wave partial array (4 waves per 256-thread workgroup) fits.
int sweep_grid(int wgs_per_cu) {
    const int g = mg::device_cu_count() * (wgs_per_cu > 0 ? wgs_per_cu : 8);
    return std::min(std::max(g, 1), mg::MAX_GRID_WAVES / 4);
}

CutoffWs carve_cutoff(void* ws, size_t bytes, int B, int64_t N) {
    Carver c{static_cast<char*>(ws)};
    CutoffWs w;
    w.ctr = c.take<mg::Counters>(1);
    w.info = c.take<mg::StructInfo>((size_t)B);
    w.plan = c.take<mg::PlanRow>((size_t)B);
    w.item_off = c.take<int64_t>((size_t)B + 1);
    w.box_off = c.take<int64_t>((size_t)B + 1);
    w.counts = c.take<uint32_t>((size_t)N);
    w.ccount = c.take<uint32_t>(4 * (size_t)N + 256);   // per-(source, image chunk) counts
    w.offsets = c.take<int64_t>((size_t)N + 1);
    w.bsum = c.take<int64_t>((size_t)mg::scan_block_count(N) + 1);
    w.partials = c.take<int64_t>(2 * (size_t)mg::MAX_GRID_WAVES);   // image and cell-list sweeps
    w.thr = c.take<float>((size_t)N);
    carve_cl(c, B, N, w.ctr, w.cl);
    w.fixed = c.used;
    w.img = carve_images(c, bytes);
    return w;
}

struct KnnWs {
    mg::Counters* ctr;
    mg::StructInfo* info;
    mg::PlanRow* plan;
    int64_t* item_off;
    int64_t* box_off;
    int32_t* ext_list;
    int64_t* partials;
    mg::ClWs cl;
    mg::ImageTables img;
    size_t fixed;
};

KnnWs carve_knn(void* ws, size_t bytes, int B, int64_t N) {
    Carver c{static_cast<char*>(ws)};
    KnnWs w;
    w.ctr = c.take<mg::Counters>(1);
    w.info = c.take<mg::StructInfo>((size_t)B);
    w.plan = c.take<mg::PlanRow>((size_t)B);
    w.item_off = c.take<int64_t>((size_t)B + 1);
    w.box_off = c.take<int64_t>((size_t)B + 1);
    w.ext_list = c.take<int32_t>((size_t)N);
    w.partials = c.take<int64_t>((size_t)mg::MAX_GRID_WAVES);
    carve_cl(c, B, N, w.ctr, w.cl);
    w.fixed = c.used;
    w.img = carve_images(c, bytes);
    return w;
}

struct GeomWs {
    int32_t* atom_struct;
    mg::GeomBwdWs bwd;
    size_t fixed;
};

// The backward pass's workspace: the fixed part, and with E > 0 the bucket
// path's counts, scan and E edge records after it (same fixed part first, so a
// workspace of either size carves the same fixed layout).
GeomWs carve_geom(void* ws, int B, int64_t N, int64_t E = 0) {
    Carver c{static_cast<char*>(ws)};
    GeomWs w;
    w.atom_struct = c.take<int32_t>((size_t)N);
    w.bwd.acc = c.take<double>((size_t)B * 9);
    w.bwd.start = c.take<int64_t>((size_t)B + 1);
    w.bwd.item_off = c.take<int64_t>((size_t)B + 1);
    w.bwd.flag = c.take<int32_t>(4);   // order flag, item counts by structure size, bucket path (see geometry)
    w.bwd.cm_off = w.bwd.p3_off = nullptr;
    w.bwd.bcount = nullptr;
    w.bwd.boff = w.bwd.bsum = nullptr;
    w.bwd.rec = nullptr;
    w.bwd.m_cap = w.bwd.e_cap = 0;
    if (E > 0) {
        const int64_t m = mg::bk_count_capacity(B, E);
        w.bwd.cm_off = c.take<int64_t>((size_t)B + 1);
        w.bwd.p3_off = c.take<int64_t>((size_t)B + 1);
        w.bwd.bcount = c.take<uint32_t>((size_t)m);
        w.bwd.boff = c.take<int64_t>((size_t)m + 1);
        w.bwd.bsum = c.take<int64_t>((size_t)mg::scan_block_count(m) + 1);
        w.bwd.rec = c.take<float4>((size_t)E);
        w.bwd.m_cap = m;
        w.bwd.e_cap = E;
    }
    w.fixed = mg::align_up(c.used, 256);
    return w;
}

struct TripWs {
    uint32_t* counts;
    int64_t* offsets;
    int64_t* bsum;
    size_t fixed;
};

TripWs carve_triplets(void* ws, int64_t N) {
    Carver c{static_cast<char*>(ws)};
    TripWs w;
    w.counts = c.take<uint32_t>((size_t)N);
    w.offsets = c.take<int64_t>((size_t)N + 1);
    w.bsum = c.take<int64_t>((size_t)mg::scan_block_count(N) + 1);
    w.fixed = mg::align_up(c.used, 256);
    return w;
}

struct SymWsHost {
    mg::SymWs w;
    int64_t* out_off;
    size_t fixed;
};

SymWsHost carve_symmetrize(void* ws, int64_t N, int64_t E) {
    Carver c{static_cast<char*>(ws)};
    SymWsHost h;
    h.w.addcnt = c.take<uint32_t>((size_t)N);
    h.w.cursor = c.take<uint32_t>((size_t)N);
    h.w.total = c.take<uint32_t>((size_t)N);
    h.w.aoff = c.take<int64_t>((size_t)N + 1);
    h.w.bsum = c.take<int64_t>((size_t)mg::scan_block_count(N) + 1);
    h.out_off = c.take<int64_t>((size_t)N + 1);
    h.w.bucket = c.take<uint64_t>((size_t)E);
    h.w.miss = c.take<uint8_t>((size_t)E);
    h.fixed = mg::align_up(c.used, 256);
    return h;
}

struct TiesWs {
    int32_t* src;
    int32_t* dst;
    int32_t* image;
    float* length;
    uint32_t* counts;
    int64_t* offsets;
    int64_t* bsum;
    char* knn;          // the KNN search's own workspace follows
    size_t fixed;
};

TiesWs carve_ties(void* ws, int64_t N) {
    Carver c{static_cast<char*>(ws)};
    TiesWs w;
    const size_t M = (size_t)N * mg::TIES_K;
    w.src = c.take<int32_t>(M);
    w.dst = c.take<int32_t>(M);
    w.image = c.take<int32_t>(3 * M);
    w.length = c.take<float>(M);
    w.counts = c.take<uint32_t>((size_t)N);
    w.offsets = c.take<int64_t>((size_t)N + 1);
    w.bsum = c.take<int64_t>((size_t)mg::scan_block_count(N) + 1);
    w.fixed = mg::align_up(c.used, 256);
    w.knn = static_cast<char*>(ws) + w.fixed;
    return w;
}

// Smallest float y with sqrtf(y) >= c, so that l2 < y  <=>  sqrtf(l2) < c.
float cutoff_threshold(float c) {
    float y = c * c;
    if (std::sqrt(y) >= c) {
        for (;;) {
            const float d = std::nextafter(y, 0.0f);
            if (d <= 0.0f || std::sqrt(d) < c) break;
            y = d;
        }
    } else {
        while (std::sqrt(y) < c) y = std::nextafter(y, INFINITY);
    }
    return y;
}

mg_status check_common(const float* lattices, const float* frac, const int64_t* batch_ptr, int32_t B,
                       int64_t N) {
    if (B < 0) return fail(MG_ERR_INVALID_ARG, "B must be >= 0 (got %d)", B);
    if (N < 0 || N > (int64_t)INT32_MAX) return fail(MG_ERR_INVALID_ARG, "N must be in [0, 2^31) (got %lld)", (long long)N);
    if (B == 0 && N != 0) return fail(MG_ERR_INVALID_ARG, "N must be 0 when B == 0");
    if (!batch_ptr) return fail(MG_ERR_INVALID_ARG, "batch_ptr is NULL");
    if (B > 0 && !lattices) return fail(MG_ERR_INVALID_ARG, "lattices is NULL");
    if (N > 0 && !frac) return fail(MG_ERR_INVALID_ARG, "frac is NULL");
    return MG_OK;
}

}  // namespace

// ============================================================== public ABI

extern "C" {

int32_t mg_abi_version(void) { return MG_ABI_VERSION; }

const char* mg_last_error(void) { return g_err.c_str(); }

size_t mg_cutoff_workspace_bytes(int32_t B, int64_t N, int64_t image_capacity) {
    if (B < 0 || N < 0 || image_capacity < 0) return 0;
    CutoffWs w = carve_cutoff(nullptr, 0, B, N);
    return w.fixed + (size_t)mg::IMAGE_FIXED_BYTES + (size_t)image_capacity * (size_t)mg::IMAGE_SLOT_BYTES;
}

size_t mg_knn_workspace_bytes(int32_t B, int64_t N, int32_t k, int64_t image_capacity) {
    if (B < 0 || N < 0 || image_capacity < 0 || k < 1 || k > 64) return 0;
    KnnWs w = carve_knn(nullptr, 0, B, N);
    return w.fixed + (size_t)mg::IMAGE_FIXED_BYTES + (size_t)image_capacity * (size_t)mg::IMAGE_SLOT_BYTES;
}

size_t mg_knn_ties_workspace_bytes(int32_t B, int64_t N, int32_t k, int64_t image_capacity) {
    if (B < 0 || N < 0 || image_capacity < 0 || k < 1 || k >= mg::TIES_K) return 0;
    return carve_ties(nullptr, N).fixed + mg_knn_workspace_bytes(B, N, mg::TIES_K, image_capacity);
}

size_t mg_symmetrize_workspace_bytes(int64_t N, int64_t E) {
    if (N < 0 || E < 0) return 0;
    return carve_symmetrize(nullptr, N, E).fixed;
}

size_t mg_triplets_workspace_bytes(int64_t N) {
    if (N < 0) return 0;
    return carve_triplets(nullptr, N).fixed;
}

size_t mg_geometry_workspace_bytes(int32_t B, int64_t N) {
    if (B < 0 || N < 0) return 0;
    return carve_geom(nullptr, B, N).fixed;
}

size_t mg_geometry_backward_workspace_bytes(int32_t B, int64_t N, int64_t E) {
    if (B < 0 || N < 0 || E < 0) return 0;
    return carve_geom(nullptr, B, N, E).fixed;
}

}  // extern "C"

namespace {

// Both cutoff entry points: one constant cutoff, or per-atom cutoffs (radii).
mg_status cutoff_graph(const float* lattices, const float* frac, const int64_t* batch_ptr, int32_t B,
                       int64_t N, float cutoff, const float* radii, int64_t capacity, int32_t* src,
                       int32_t* dst, int32_t* image, float* length, float* vec, int64_t* row_ptr,
                       mg_report* report, void* workspace, size_t workspace_bytes, int32_t opts, void* stream) {
    g_err.clear();
    mg_status st = check_common(lattices, frac, batch_ptr, B, N);
    if (st != MG_OK) return st;
    if (!radii && (!(cutoff > 0.0f) || !std::isfinite(cutoff)))
        return fail(MG_ERR_INVALID_ARG, "cutoff must be finite and > 0 (got %g)", (double)cutoff);
    if (capacity < 0) return fail(MG_ERR_INVALID_ARG, "capacity must be >= 0");
    if (capacity > 0 && (!src || !dst || !image || !length))
        return fail(MG_ERR_INVALID_ARG, "src/dst/image/length must be non-NULL when capacity > 0");
    if (!report) return fail(MG_ERR_INVALID_ARG, "report is NULL");
    if (opts & ~(MG_OPT_CELL_LIST_OFF | MG_OPT_CELL_LIST_FORCE))
        return fail(MG_ERR_INVALID_ARG, "unknown opts bits 0x%x", opts);
    if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    CutoffWs w = carve_cutoff(workspace, workspace_bytes, B, N);
    if (workspace_bytes < w.fixed)
        return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    workspace_bytes, w.fixed);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const mg_tuning tu = tuning();
    const float c2 = radii ? 0.0f : cutoff_threshold(cutoff);
    float* thr = radii ? w.thr : nullptr;
    int64_t* offs = row_ptr ? row_ptr : w.offsets;
    const int grid = sweep_grid(tu.cutoff_wgs_per_cu);
    const bool sum = B > 0 && N > 0;
    hipError_t e;
    const bool cl = !(opts & MG_OPT_CELL_LIST_OFF);
    // (the plan kernel starts the report and the workspace counters)
    if ((e = phase("cutoff.bounds", s, [&] {
             return mg::launch_bounds(lattices, batch_ptr, frac, B, N, cutoff, radii, thr, 0, 0.f, w.info,
                                      w.plan, w.ctr, report, 0, opts, tu.cutoff_cl_span, s);
         })) != hipSuccess)
        return hip_fail(e, "bounds");
    if ((e = phase("cutoff.plan", s, [&] {
             return mg::launch_struct_scan(B, w.info, w.plan, 4 * N + 256, w.item_off, w.cl.cl_off, w.box_off, w.ctr, report, w.img.cap, s);
         })) != hipSuccess)
        return hip_fail(e, "plan");
    if ((e = phase("cutoff.images", s, [&] { return mg::launch_images(B, w.info, w.box_off, w.ctr, w.img, s); })) !=
        hipSuccess)
        return hip_fail(e, "images");
    if (cl && (e = phase("cutoff.cells", s, [&] { return mg::launch_cl_build(B, N, frac, batch_ptr, w.info, w.cl, s); })) !=
                  hipSuccess)
        return hip_fail(e, "cell lists");
    // per-wave candidate counts: the image sweep's in partials[0, 4 grid), the
    // cell-list sweep's after them; the scan adds them to the report
    if ((e = phase("cutoff.count", s, [&] {
             const hipError_t r = mg::launch_cutoff_sweep(0, B, w.info, w.item_off, w.ccount, w.img.table, frac, c2,
                                                          thr, w.counts, offs, capacity, src, dst, image, length, vec,
                                                          w.ctr, report, w.partials, grid, tu.cutoff_slots,
                                                          tu.cutoff_img_group, s);
             // row totals and in-row offsets of the image-chunked structures
             return r != hipSuccess ? r : mg::launch_chunk_prefix(B, w.info, w.counts, w.ccount, s);
         })) != hipSuccess)
        return hip_fail(e, "count");
    if (cl && (e = phase("cutoff.cells.count", s, [&] {
                   return mg::launch_cl_cutoff_sweep(0, B, w.info, w.cl, frac, c2, thr, w.counts, offs, capacity,
                                                     src, dst, image, length, vec, w.ctr, report,
                                                     w.partials + grid * 4, grid, s);
               })) != hipSuccess)
        return hip_fail(e, "cell-list count");
    if ((e = phase("cutoff.scan", s, [&] {
             return mg::launch_scan_counts(w.counts, N, offs, w.bsum, capacity, report, s, nullptr,
                                           sum ? w.partials : nullptr, (cl ? 2 : 1) * grid * 4);
         })) != hipSuccess)
        return hip_fail(e, "scan");
    if (capacity == 0) return MG_OK;   // a sizing call: the counts and num_edges are all it needs
    if ((e = phase("cutoff.fill", s, [&] {
             return mg::launch_cutoff_sweep(1, B, w.info, w.item_off, w.ccount, w.img.table, frac, c2, thr, w.counts, offs,
                                            capacity, src, dst, image, length, vec, w.ctr, report, w.partials,
                                            grid, tu.cutoff_slots, tu.cutoff_img_group, s);
         })) != hipSuccess)
        return hip_fail(e, "fill");
    if (cl && (e = phase("cutoff.cells.fill", s, [&] {
                   return mg::launch_cl_cutoff_sweep(1, B, w.info, w.cl, frac, c2, thr, w.counts, offs, capacity, src,
                                                     dst, image, length, vec, w.ctr, report, w.partials, grid, s);
               })) != hipSuccess)
        return hip_fail(e, "cell-list fill");
    if ((e = phase("cutoff.src", s, [&] { return mg::launch_src_from_rows(offs, N, capacity, src, s); })) !=
        hipSuccess)
        return hip_fail(e, "src");
    return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_cutoff_graph(const float* lattices, const float* frac, const int64_t* batch_ptr,
                          int32_t B, int64_t N, float cutoff, int64_t capacity, int32_t* src,
                          int32_t* dst, int32_t* image, float* length, int64_t* row_ptr,
                          mg_report* report, void* workspace, size_t workspace_bytes, int32_t opts,
                          void* stream) {
    return cutoff_graph(lattices, frac, batch_ptr, B, N, cutoff, nullptr, capacity, src, dst, image, length,
                        nullptr, row_ptr, report, workspace, workspace_bytes, opts, stream);
}

mg_status mg_cutoff_graph_vec(const float* lattices, const float* frac, const int64_t* batch_ptr, int32_t B,
                              int64_t N, float cutoff, const float* radii, int64_t capacity, int32_t* src,
                              int32_t* dst, int32_t* image, float* length, float* vec, int64_t* row_ptr,
                              mg_report* report, void* workspace, size_t workspace_bytes, int32_t opts,
                              void* stream) {
    if (capacity > 0 && !vec) {
        g_err.clear();
        return fail(MG_ERR_INVALID_ARG, "vec must be non-NULL when capacity > 0");
    }
    if (radii || N == 0)
        return cutoff_graph(lattices, frac, batch_ptr, B, N, radii ? 1.0f : cutoff, N > 0 ? radii : nullptr,
                            capacity, src, dst, image, length, vec, row_ptr, report, workspace, workspace_bytes,
                            opts, stream);
    return cutoff_graph(lattices, frac, batch_ptr, B, N, cutoff, nullptr, capacity, src, dst, image, length, vec,
                        row_ptr, report, workspace, workspace_bytes, opts, stream);
}

mg_status mg_cutoff_graph_radii(const float* lattices, const float* frac, const int64_t* batch_ptr,
                                int32_t B, int64_t N, const float* radii, int64_t capacity, int32_t* src,
                                int32_t* dst, int32_t* image, float* length, int64_t* row_ptr,
                                mg_report* report, void* workspace, size_t workspace_bytes, int32_t opts,
                                void* stream) {
    if (N > 0 && !radii) {
        g_err.clear();
        return fail(MG_ERR_INVALID_ARG, "radii is NULL");
    }
    // with no atoms there is nothing to read: any valid constant gives the same (empty) graph
    return cutoff_graph(lattices, frac, batch_ptr, B, N, 1.0f, N > 0 ? radii : nullptr, capacity, src, dst,
                        image, length, nullptr, row_ptr, report, workspace, workspace_bytes, opts, stream);
}

mg_status mg_knn_graph(const float* lattices, const float* frac, const int64_t* batch_ptr, int32_t B,
                       int64_t N, int32_t k, int32_t* src, int32_t* dst, int32_t* image,
                       float* length, mg_report* report, void* workspace, size_t workspace_bytes,
                       int32_t opts, void* stream) {
    g_err.clear();
    mg_status st = check_common(lattices, frac, batch_ptr, B, N);
    if (st != MG_OK) return st;
    if (k < 1 || k > 64) return fail(MG_ERR_INVALID_ARG, "k must be in 1..64 (got %d)", k);
    if ((int64_t)N * k > (int64_t)INT32_MAX * 2)
        return fail(MG_ERR_UNSUPPORTED, "N*k = %lld is too large", (long long)N * k);
    if (N > 0 && (!src || !dst || !image || !length))
        return fail(MG_ERR_INVALID_ARG, "src/dst/image/length must be non-NULL");
    if (!report) return fail(MG_ERR_INVALID_ARG, "report is NULL");
    if (opts & ~(MG_OPT_CELL_LIST_OFF | MG_OPT_CELL_LIST_FORCE))
        return fail(MG_ERR_INVALID_ARG, "unknown opts bits 0x%x", opts);
    if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    KnnWs w = carve_knn(workspace, workspace_bytes, B, N);
    if (workspace_bytes < w.fixed)
        return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    workspace_bytes, w.fixed);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const mg_tuning tu = tuning();
    const float lambda = (tu.knn_lambda_x4 > 0 ? tu.knn_lambda_x4 : 6) / 4.0f;
    const int grid = sweep_grid(tu.knn_wgs_per_cu);
    const bool sum = B > 0 && N > 0;
    hipError_t e;
    const bool cl = !(opts & MG_OPT_CELL_LIST_OFF);
    // (the plan kernel starts the report, num_edges = N k, and the workspace counters)
    if ((e = phase("knn.bounds", s, [&] {
             return mg::launch_bounds(lattices, batch_ptr, frac, B, N, 0.f, nullptr, nullptr, k, lambda,
                                      w.info, w.plan, w.ctr, report, 1, opts, tu.knn_cl_span, s);
         })) != hipSuccess)
        return hip_fail(e, "bounds");
    if ((e = phase("knn.plan", s, [&] {
             return mg::launch_struct_scan(B, w.info, w.plan, 0, w.item_off, w.cl.cl_off, w.box_off, w.ctr, report, w.img.cap, s,
                                           N * (int64_t)k);
         })) != hipSuccess)
        return hip_fail(e, "plan");
    if ((e = phase("knn.images", s, [&] { return mg::launch_images(B, w.info, w.box_off, w.ctr, w.img, s); })) !=
        hipSuccess)
        return hip_fail(e, "images");
    if ((e = phase("knn.atoms", s, [&] { return mg::launch_atom_struct(batch_ptr, B, N, w.cl.atom_struct, s); })) !=
        hipSuccess)
        return hip_fail(e, "atom map");
    if (cl && (e = phase("knn.cells", s, [&] { return mg::launch_cl_build(B, N, frac, batch_ptr, w.info, w.cl, s); })) !=
                  hipSuccess)
        return hip_fail(e, "cell lists");
    if ((e = phase("knn.select", s, [&] {
             hipError_t r = mg::launch_knn(B, N, k, w.info, w.item_off, w.img.table, frac, src, dst, image, length,
                                           w.ext_list, w.ctr, report, w.partials, grid, tu.knn_tau_x8 / 8.0f, s);
             if (r != hipSuccess || !sum) return r;
             return mg::launch_sum_partials(w.partials, grid * 4, report, s);
         })) != hipSuccess)
        return hip_fail(e, "knn");
    if (cl && (e = phase("knn.cells.select", s, [&] {
                   hipError_t r = mg::launch_cl_knn(B, k, w.info, w.cl, frac, src, dst, image, length, w.ext_list,
                                                    w.ctr, report, w.partials, grid, tu.knn_tau_x8 / 8.0f, s);
                   if (r != hipSuccess || !sum) return r;
                   return mg::launch_sum_partials(w.partials, grid * 4, report, s);
               })) != hipSuccess)
        return hip_fail(e, "cell-list knn");
    if ((e = phase("knn.extended", s, [&] {
             return mg::launch_knn_extended(B, N, k, w.info, frac, w.cl.atom_struct, src, dst, image, length,
                                            w.ext_list, w.ctr, report, mg::device_cu_count() * 2, s);
         })) != hipSuccess)
        return hip_fail(e, "knn extended");
    return MG_OK;
}

mg_status mg_images_needed(const float* lattices, const float* frac, const int64_t* batch_ptr, int32_t B,
                           int64_t N, float cutoff, const float* radii, int32_t k, mg_report* report,
                           void* workspace, size_t workspace_bytes, int32_t opts, void* stream) {
    g_err.clear();
    mg_status st = check_common(lattices, frac, batch_ptr, B, N);
    if (st != MG_OK) return st;
    if (k < 0 || k > 64) return fail(MG_ERR_INVALID_ARG, "k must be 0 (cutoff graph) or in 1..64 (got %d)", k);
    if (k == 0 && !radii && (!(cutoff > 0.0f) || !std::isfinite(cutoff)))
        return fail(MG_ERR_INVALID_ARG, "cutoff must be finite and > 0 (got %g)", (double)cutoff);
    if (!report) return fail(MG_ERR_INVALID_ARG, "report is NULL");
    if (opts & ~(MG_OPT_CELL_LIST_OFF | MG_OPT_CELL_LIST_FORCE))
        return fail(MG_ERR_INVALID_ARG, "unknown opts bits 0x%x", opts);
    if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const mg_tuning tu = tuning();
    hipError_t e;
    mg::Counters* ctr;
    mg::StructInfo* info;
    mg::PlanRow* plan;
    int64_t *item_off, *cl_off, *box_off;
    float* thr = nullptr;
    if (k == 0) {
        CutoffWs w = carve_cutoff(workspace, workspace_bytes, B, N);
        if (workspace_bytes < w.fixed)
            return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                        workspace_bytes, w.fixed);
        ctr = w.ctr, info = w.info, plan = w.plan, item_off = w.item_off, cl_off = w.cl.cl_off, box_off = w.box_off;
        thr = radii ? w.thr : nullptr;
    } else {
        KnnWs w = carve_knn(workspace, workspace_bytes, B, N);
        if (workspace_bytes < w.fixed)
            return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                        workspace_bytes, w.fixed);
        ctr = w.ctr, info = w.info, plan = w.plan, item_off = w.item_off, cl_off = w.cl.cl_off, box_off = w.box_off;
    }
    const float lambda = (tu.knn_lambda_x4 > 0 ? tu.knn_lambda_x4 : 6) / 4.0f;
    // (the plan kernel starts the report and the workspace counters)
    if ((e = mg::launch_bounds(lattices, batch_ptr, frac, B, N, k == 0 ? (radii ? 1.0f : cutoff) : 0.f,
                               k == 0 ? radii : nullptr, thr, k, lambda, info, plan, ctr, report, k == 0 ? 0 : 1,
                               opts, k == 0 ? tu.cutoff_cl_span : tu.knn_cl_span, s)) != hipSuccess)
        return hip_fail(e, "bounds");
    // the plan with an unbounded table: images_needed is the batch's total, no structure skipped
    if ((e = mg::launch_struct_scan(B, info, plan, 0, item_off, cl_off, box_off, ctr, report, INT64_MAX, s)) !=
        hipSuccess)
        return hip_fail(e, "plan");
    return MG_OK;
}

static mg_status check_edges(const int32_t* src, const int32_t* dst, const int32_t* image, int64_t E) {
    if (E < 0) return fail(MG_ERR_INVALID_ARG, "E must be >= 0");
    if (E > 0 && (!src || !dst || !image)) return fail(MG_ERR_INVALID_ARG, "src/dst/image is NULL");
    return MG_OK;
}

mg_status mg_edge_geometry(const float* lattices, const float* frac, const int64_t* batch_ptr,
                           int32_t B, int64_t N, const int32_t* src, const int32_t* dst,
                           const int32_t* image, int64_t E, const int64_t* num_edges, float* vec,
                           float* length, void* workspace, size_t workspace_bytes, void* stream) {
    g_err.clear();
    mg_status st = check_common(lattices, frac, batch_ptr, B, N);
    if (st != MG_OK) return st;
    if ((st = check_edges(src, dst, image, E)) != MG_OK) return st;
    if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    GeomWs w = carve_geom(workspace, B, N);
    if (workspace_bytes < w.fixed)
        return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    workspace_bytes, w.fixed);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = phase("geometry.atoms", s, [&] { return mg::launch_atom_struct(batch_ptr, B, N, w.atom_struct, s); })) !=
        hipSuccess)
        return hip_fail(e, "atom map");
    if ((e = phase("geometry.fwd", s, [&] {
             return mg::launch_geometry_fwd(lattices, frac, w.atom_struct, batch_ptr, B, N, src, dst, image, E,
                                            num_edges, vec, length, w.bwd, s);
         })) != hipSuccess)
        return hip_fail(e, "geometry");
    return MG_OK;
}

mg_status mg_edge_geometry_backward(const float* lattices, const float* frac, const int64_t* batch_ptr,
                                    int32_t B, int64_t N, const int32_t* src, const int32_t* dst,
                                    const int32_t* image, int64_t E, const int64_t* num_edges,
                                    const float* grad_vec, const float* grad_length, float* grad_frac,
                                    float* grad_lattice, void* workspace, size_t workspace_bytes,
                                    void* stream) {
    g_err.clear();
    mg_status st = check_common(lattices, frac, batch_ptr, B, N);
    if (st != MG_OK) return st;
    if ((st = check_edges(src, dst, image, E)) != MG_OK) return st;
    if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    GeomWs w = carve_geom(workspace, B, N);
    if (workspace_bytes < w.fixed)
        return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    workspace_bytes, w.fixed);
    if (E > 0) {   // room for the bucket path of large structures
        const GeomWs wb = carve_geom(workspace, B, N, E);
        if (workspace_bytes >= wb.fixed) w = wb;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    // (the backward pass writes the atom -> structure map itself)
    if ((e = phase("geometry.bwd", s, [&] {
             return mg::launch_geometry_bwd(lattices, frac, w.atom_struct, batch_ptr, B, N, src, dst, image, E,
                                            num_edges, grad_vec, grad_length, grad_frac, grad_lattice, w.bwd, s);
         })) != hipSuccess)
        return hip_fail(e, "geometry backward");
    return MG_OK;
}

}  // extern "C"

// ------------------------------------------------- allocation-free backward

namespace {

// Scratch of mg_edge_geometry_backward_static: the same workspace layout as
// mg_edge_geometry_backward's, in a device array of the library (one copy per
// GPU, kept until the process ends). Host code never passes the array's name
// to a kernel: it is a host-side stand-in, not a device address. The device
// address comes from hipGetSymbolAddress, once per device with that device
// current, and only that pointer is used.
constexpr size_t kStaticScratchBytes = MG_STATIC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (set-up on the first call on
// each device). Returns nullptr and sets the error message on failure.
void* static_scratch(mg_status* st) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *st = hip_fail(e, "hipGetDevice");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *st = fail(MG_ERR_UNSUPPORTED, "device %d beyond the %d devices the static scratch supports", dev,
                   kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *st = hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

mg_status mg_edge_geometry_backward_static(const float* lattices, const float* frac, const int64_t* batch_ptr,
                                           int32_t B, int64_t N, const int32_t* src, const int32_t* dst,
                                           const int32_t* image, int64_t E, const int64_t* num_edges,
                                           const float* grad_vec, const float* grad_length, float* grad_frac,
                                           float* grad_lattice, void* stream) {
    g_err.clear();
    mg_status st = check_common(lattices, frac, batch_ptr, B, N);
    if (st != MG_OK) return st;
    if ((st = check_edges(src, dst, image, E)) != MG_OK) return st;
    const size_t need = carve_geom(nullptr, B, N).fixed;
    if (need > kStaticScratchBytes)
        return fail(MG_ERR_UNSUPPORTED,
                    "B = %d structures and N = %lld atoms need %zu bytes of scratch; the static scratch holds %zu "
                    "(use mg_edge_geometry_backward with a workspace)",
                    B, (long long)N, need, kStaticScratchBytes);
    void* ws = static_scratch(&st);
    if (!ws) return st;
    GeomWs w = carve_geom(ws, B, N);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = phase("geometry.bwd", s, [&] {
             return mg::launch_geometry_bwd(lattices, frac, w.atom_struct, batch_ptr, B, N, src, dst, image, E,
                                            num_edges, grad_vec, grad_length, grad_frac, grad_lattice, w.bwd, s);
         })) != hipSuccess)
        return hip_fail(e, "geometry backward");
    return MG_OK;
}

mg_status mg_knn_graph_ties(const float* lattices, const float* frac, const int64_t* batch_ptr, int32_t B,
                            int64_t N, int32_t k, int64_t capacity, int32_t* src, int32_t* dst, int32_t* image,
                            float* length, int64_t* row_ptr, mg_report* report, void* workspace,
                            size_t workspace_bytes, int32_t opts, void* stream) {
    g_err.clear();
    if (k < 1 || k >= mg::TIES_K) return fail(MG_ERR_INVALID_ARG, "k must be in 1..%d (got %d)", mg::TIES_K - 1, k);
    if (capacity < 0) return fail(MG_ERR_INVALID_ARG, "capacity must be >= 0");
    if (capacity > 0 && (!src || !dst || !image || !length))
        return fail(MG_ERR_INVALID_ARG, "src/dst/image/length must be non-NULL when capacity > 0");
    if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    if (N < 0) return fail(MG_ERR_INVALID_ARG, "N must be >= 0");
    TiesWs w = carve_ties(workspace, N);
    if (workspace_bytes < w.fixed)
        return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    workspace_bytes, w.fixed);
    mg_status st = mg_knn_graph(lattices, frac, batch_ptr, B, N, mg::TIES_K, w.src, w.dst, w.image, w.length,
                                report, w.knn, workspace_bytes - w.fixed, opts, stream);
    if (st != MG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = phase("knn.ties", s, [&] {
             return mg::launch_ties(N, k, w.src, w.dst, w.image, w.length, capacity, src, dst, image, length,
                                    row_ptr ? row_ptr : w.offsets, w.counts, w.bsum, report, s);
         })) != hipSuccess)
        return hip_fail(e, "ties");
    return MG_OK;
}

mg_status mg_symmetrize(const int64_t* row_ptr, int64_t N, const int32_t* dst, const int32_t* image,
                        const float* length, int64_t E, int64_t capacity, int32_t* out_src, int32_t* out_dst,
                        int32_t* out_image, float* out_length, int64_t* out_row_ptr, mg_report* report,
                        void* workspace, size_t workspace_bytes, void* stream) {
    g_err.clear();
    if (N < 0 || N > (int64_t)INT32_MAX) return fail(MG_ERR_INVALID_ARG, "N must be in [0, 2^31)");
    if (E < 0 || E > (int64_t)INT32_MAX) return fail(MG_ERR_INVALID_ARG, "E must be in [0, 2^31)");
    if (!row_ptr) return fail(MG_ERR_INVALID_ARG, "row_ptr is NULL");
    if (E > 0 && (!dst || !image)) return fail(MG_ERR_INVALID_ARG, "dst/image must be non-NULL when E > 0");
    if (out_length && E > 0 && !length) return fail(MG_ERR_INVALID_ARG, "out_length needs the input lengths");
    if (capacity < 0) return fail(MG_ERR_INVALID_ARG, "capacity must be >= 0");
    if (capacity > 0 && (!out_src || !out_dst || !out_image))
        return fail(MG_ERR_INVALID_ARG, "out_src/out_dst/out_image must be non-NULL when capacity > 0");
    if (!report) return fail(MG_ERR_INVALID_ARG, "report is NULL");
    if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    SymWsHost h = carve_symmetrize(workspace, N, E);
    if (workspace_bytes < h.fixed)
        return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    workspace_bytes, h.fixed);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = mg::launch_zero_report(report, nullptr, 0, s)) != hipSuccess) return hip_fail(e, "zero");
    if ((e = phase("symmetrize", s, [&] {
             return mg::launch_symmetrize(row_ptr, N, E, dst, image, length, capacity, out_src, out_dst, out_image,
                                          out_length, out_row_ptr ? out_row_ptr : h.out_off, h.w, report, s);
         })) != hipSuccess)
        return hip_fail(e, "symmetrize");
    return MG_OK;
}

mg_status mg_triplets(const int64_t* row_ptr, int64_t N, int64_t E, const float* vec, int64_t capacity,
                      int32_t* e1, int32_t* e2, float* cos_theta, int64_t* trip_ptr, mg_report* report,
                      void* workspace, size_t workspace_bytes, void* stream) {
    g_err.clear();
    if (N < 0) return fail(MG_ERR_INVALID_ARG, "N must be >= 0");
    if (E < 0 || E > (int64_t)INT32_MAX) return fail(MG_ERR_INVALID_ARG, "E must be in [0, 2^31) (got %lld)", (long long)E);
    if (!row_ptr) return fail(MG_ERR_INVALID_ARG, "row_ptr is NULL");
    if (capacity < 0) return fail(MG_ERR_INVALID_ARG, "capacity must be >= 0");
    if (capacity > 0 && (!e1 || !e2)) return fail(MG_ERR_INVALID_ARG, "e1/e2 must be non-NULL when capacity > 0");
    if (cos_theta && !vec) return fail(MG_ERR_INVALID_ARG, "cos_theta needs the edge vectors (vec is NULL)");
    if (!report) return fail(MG_ERR_INVALID_ARG, "report is NULL");
    if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is NULL");
    TripWs w = carve_triplets(workspace, N);
    if (workspace_bytes < w.fixed)
        return fail(MG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    workspace_bytes, w.fixed);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = mg::launch_zero_report(report, nullptr, 0, s)) != hipSuccess) return hip_fail(e, "zero");
    if ((e = phase("triplets", s, [&] {
             return mg::launch_triplets(row_ptr, N, E, vec, capacity, e1, e2, cos_theta,
                                        trip_ptr ? trip_ptr : w.offsets, w.counts, w.bsum, report, s);
         })) != hipSuccess)
        return hip_fail(e, "triplets");
    return MG_OK;
}

mg_status mg_get_tuning(mg_tuning* out) {
    if (!out) return fail(MG_ERR_INVALID_ARG, "out is NULL");
    *out = tuning();
    return MG_OK;
}

mg_status mg_set_tuning(const mg_tuning* in) {
    if (!in) return fail(MG_ERR_INVALID_ARG, "in is NULL");
    if (in->cutoff_slots != 0 && in->cutoff_slots != 1 && in->cutoff_slots != 2 && in->cutoff_slots != 4)
        return fail(MG_ERR_INVALID_ARG, "cutoff_slots must be 1, 2 or 4");
    if (in->cutoff_wgs_per_cu < 0 || in->cutoff_wgs_per_cu > 64 || in->knn_wgs_per_cu < 0 ||
        in->knn_wgs_per_cu > 64)
        return fail(MG_ERR_INVALID_ARG, "workgroups per CU must be in 0..64");
    if (in->knn_lambda_x4 < 0 || in->knn_lambda_x4 > 64)
        return fail(MG_ERR_INVALID_ARG, "knn_lambda_x4 must be in 0..64");
    if (in->knn_tau_x8 < 0 || in->knn_tau_x8 > 64)
        return fail(MG_ERR_INVALID_ARG, "knn_tau_x8 must be in 0..64");
    if (in->cutoff_img_group != 0 && in->cutoff_img_group != 2 && in->cutoff_img_group != 4 &&
        in->cutoff_img_group != 8)
        return fail(MG_ERR_INVALID_ARG, "cutoff_img_group must be 2, 4 or 8");
    if (in->cutoff_cl_span < 0 || in->cutoff_cl_span > 2 || in->knn_cl_span < 0 || in->knn_cl_span > 2)
        return fail(MG_ERR_INVALID_ARG, "cell-list spans must be 1 or 2");
    std::lock_guard<std::mutex> lk(g_mu);
    if (in->cutoff_wgs_per_cu) g_tune.cutoff_wgs_per_cu = in->cutoff_wgs_per_cu;
    if (in->cutoff_slots) g_tune.cutoff_slots = in->cutoff_slots;
    if (in->knn_wgs_per_cu) g_tune.knn_wgs_per_cu = in->knn_wgs_per_cu;
    if (in->knn_lambda_x4) g_tune.knn_lambda_x4 = in->knn_lambda_x4;
    if (in->knn_tau_x8) g_tune.knn_tau_x8 = in->knn_tau_x8;
    if (in->cutoff_img_group) g_tune.cutoff_img_group = in->cutoff_img_group;
    if (in->cutoff_cl_span) g_tune.cutoff_cl_span = in->cutoff_cl_span;
    if (in->knn_cl_span) g_tune.knn_cl_span = in->knn_cl_span;
    return MG_OK;
}

mg_status mg_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof = on != 0;
    return MG_OK;
}

int32_t mg_profile_read(char* names, double* ms, int64_t* count, int32_t max) {
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        recs.swap(g_recs);
    }
    std::vector<std::string> nm;
    std::vector<double> tot;
    std::vector<int64_t> cnt;
    for (auto& r : recs) {
        float t = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            size_t q = 0;
            while (q < nm.size() && nm[q] != r.name) ++q;
            if (q == nm.size()) {
                nm.push_back(r.name);
                tot.push_back(0.0);
                cnt.push_back(0);
            }
            tot[q] += t;
            cnt[q] += 1;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& r : recs) {
            g_pool.push_back(r.a);
            g_pool.push_back(r.b);
        }
    }
    const int32_t m = (int32_t)nm.size();
    for (int32_t q = 0; q < m && q < max; ++q) {
        if (names) {
            std::strncpy(names + 32 * q, nm[q].c_str(), 31);
            names[32 * q + 31] = 0;
        }
        if (ms) ms[q] = tot[q];
        if (count) count[q] = cnt[q];
    }
    return m;
}

}  // extern "C"

namespace mg {

int device_cu_count() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
        cache[dev] = cu;
    }
    return cache[dev];
}

}  // namespace mg

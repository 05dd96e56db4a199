/*
 * matgraph.h - periodic cutoff / k-nearest-neighbour multigraphs of crystal
 * batches on AMD MI355X (gfx950), C ABI of libmatgraph.so.
 *
 * What the library computes (arxiv 2307.05380):
 *  - the crystallographic graph of Sec. 2.1, Definition def6: for a material
 *    (rho, x) with n atoms, the edges are the triplets (i, j, t) with t in Z^3
 *    such that || rho (x_j - x_i + t) || < c.  It is a multigraph: a pair may
 *    carry several edges and an atom has edges to its own images (Sec. 1).
 *    The self-image (i, i, 0) is not an edge.
 *  - the k-nearest-neighbour graph, the special case of Definition def6 where
 *    every source keeps exactly its k nearest (j, t) (Sec. 1 and the remark
 *    after Definition def6; Sec. 2.2, Algorithms 1 and 2).
 *  - edge vectors and lengths and their backward pass, so that a model can move
 *    the geometry and rebuild the graph inside its forward pass (abstract,
 *    Sec. 4).
 *
 * Conventions shared by every call
 *  - lattices: float32 [B][3][3], ROW k is lattice vector a_k in Angstrom; the
 *    paper's rho is the transpose. Cartesian = frac @ lattice.
 *  - frac: float32 [N][3] fractional coordinates. Values outside [0, 1) are
 *    accepted; edges follow Definition def6 applied to the coordinates as given
 *    and t is relative to them.
 *  - batch_ptr: int64 [B+1], non-decreasing, batch_ptr[0] = 0, batch_ptr[B] = N.
 *    Structure b owns atoms batch_ptr[b] .. batch_ptr[b+1]-1.
 *  - an edge is (src, dst, image t) with int32 global atom indices and int32
 *    image components; its vector is (frac[dst] - frac[src] + t) @ lattice[b].
 *  - all pointers are DEVICE pointers unless marked [host]. The caller owns
 *    every buffer; the library never allocates or frees memory on these calls
 *    (scratch space comes from the caller's workspace), so they can be
 *    captured into a HIP graph.
 *  - every compute call is asynchronous on `stream` (a hipStream_t; NULL means
 *    the default stream). Host-detectable errors return a non-zero mg_status
 *    immediately, enqueue nothing, and set mg_last_error(). Conditions found on
 *    the device never abort: they set bits of mg_report.flags.
 *  - distances are computed in FP32 from FP64-derived per-pair and per-image
 *    offsets; the per-structure image bounds are computed in FP64 on the GPU.
 */
#ifndef MATGRAPH_H
#define MATGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_ABI_VERSION 1

typedef int32_t mg_status;
enum {
    MG_OK = 0,
    MG_ERR_INVALID_ARG = 1,   /* null required pointer, bad size, bad cutoff / k ... */
    MG_ERR_WORKSPACE = 2,     /* workspace pointer null or smaller than the fixed part */
    MG_ERR_HIP = 3,           /* a HIP runtime call failed (message in mg_last_error) */
    MG_ERR_UNSUPPORTED = 4    /* the request exceeds a documented limit */
};

/* Bits of mg_report.flags (set on the device, never cleared by the library
 * except at the start of a call). */
enum {
    MG_FLAG_CAPACITY = 1u,      /* cutoff: more edges than `capacity`; nothing was written past
                                   capacity, mg_report.num_edges holds the exact count */
    MG_FLAG_SINGULAR = 2u,      /* a lattice with |det| < 1e-9 * |a1||a2||a3|: that structure has no edges */
    MG_FLAG_NONFINITE = 4u,     /* a NaN/Inf lattice entry or coordinate: that structure has no edges */
    MG_FLAG_IMAGES = 8u,        /* the workspace's image table was too small: the graph is incomplete;
                                   mg_report.images_needed holds the slots required */
    MG_FLAG_RANGE = 16u,        /* an image offset beyond |t_k| <= 511 or a KNN key space beyond 2^32
                                   would be needed: that structure (or source) has no edges */
    MG_FLAG_KNN_EXTENDED = 32u, /* informational: some KNN sources needed the extended search */
    MG_FLAG_TIES = 64u          /* keep-ties KNN: a source had more candidates at its k-th distance
                                   than the search keeps (64 keys per source); its set is truncated */
};

/* Device-resident summary written by the graph calls (64 bytes). */
typedef struct mg_report {
    int64_t num_edges;       /* edges the inputs define (cutoff: exact even if > capacity; KNN: N*k) */
    int64_t images_needed;   /* image slots the batch needs (see mg_*_workspace_bytes) */
    int64_t candidates;      /* (source, destination, image) candidates evaluated by the main sweep */
    int64_t knn_extended;    /* KNN sources resolved by the extended search */
    uint32_t flags;          /* MG_FLAG_* */
    uint32_t reserved[7];
} mg_report;

/* Bits of `opts`. */
enum {
    MG_OPT_DEFAULT = 0,
    MG_OPT_CELL_LIST_OFF = 2,   /* never use cell lists (large structures use the image sweep) */
    MG_OPT_CELL_LIST_FORCE = 4  /* use cell lists for every structure where they apply */
};

/* ABI version of the loaded library (MG_ABI_VERSION). */
int32_t mg_abi_version(void);

/* [host] Message of the last non-OK status returned on this thread ("" if none). */
const char* mg_last_error(void);

/* Workspace bytes for mg_cutoff_graph on B structures / N atoms with room for
 * `image_capacity` image slots (45 bytes each). Every structure takes one slot
 * per translation of its search box (the translations its per-axis bounds
 * allow); the table then keeps, per structure, those whose cell can reach
 * within the cutoff. A cutoff call sets MG_FLAG_IMAGES and reports
 * images_needed (the slots the batch needs) when the batch needs more.
 * Returns 0 for negative arguments. */
size_t mg_cutoff_workspace_bytes(int32_t B, int64_t N, int64_t image_capacity);

/* Workspace bytes for mg_knn_graph (same meaning of image_capacity; k in 1..64). */
size_t mg_knn_workspace_bytes(int32_t B, int64_t N, int32_t k, int64_t image_capacity);

/* Workspace bytes for mg_edge_geometry / mg_edge_geometry_backward. */
size_t mg_geometry_workspace_bytes(int32_t B, int64_t N);

/* Workspace bytes with which mg_edge_geometry_backward on E edges takes its
 * faster path for structures of more than 512 (and at most 65536) atoms: the
 * destination side of those structures is transposed through per-block buckets
 * (16 bytes per edge and a small counts table) instead of global atomics.
 * Any workspace of at least mg_geometry_workspace_bytes(B, N) stays valid;
 * the call takes the bucket path only when the workspace is this large. */
size_t mg_geometry_backward_workspace_bytes(int32_t B, int64_t N, int64_t E);

/* Workspace bytes for mg_triplets on a graph of N source atoms (0 if N < 0). */
size_t mg_triplets_workspace_bytes(int64_t N);

/* Workspace bytes for mg_knn_graph_ties (k in 1..63; 0 otherwise). */
size_t mg_knn_ties_workspace_bytes(int32_t B, int64_t N, int32_t k, int64_t image_capacity);

/* Workspace bytes for mg_symmetrize on N atoms and E input edges (0 if negative). */
size_t mg_symmetrize_workspace_bytes(int64_t N, int64_t E);

/*
 * Image-table sizing without building a graph: runs only the per-structure
 * FP64 bounds and the batch plan of a cutoff call (k == 0: constant `cutoff`,
 * or per-atom `radii` as in mg_cutoff_graph_radii) or of a KNN call (k in
 * 1..64; the first search radius comes from the current tuning, see
 * mg_set_tuning) and writes report->images_needed: the image_capacity with
 * which the same call on the same inputs and tuning sets no MG_FLAG_IMAGES.
 * report->flags gets the flags of skipped structures (SINGULAR, NONFINITE,
 * RANGE); every other report field is 0. Together with a cutoff call of
 * capacity 0 (which skips the fill and returns the exact num_edges) it sizes
 * every buffer of a step before that step is captured into a HIP graph.
 *  workspace     mg_cutoff_workspace_bytes(B, N, 0) (k == 0) or
 *                mg_knn_workspace_bytes(B, N, k, 0) bytes suffice.
 * Errors: as mg_cutoff_graph / mg_knn_graph; MG_ERR_INVALID_ARG for k outside 0..64.
 */
mg_status mg_images_needed(const float* lattices, const float* frac, const int64_t* batch_ptr,
                           int32_t B, int64_t N, float cutoff, const float* radii, int32_t k,
                           mg_report* report, void* workspace, size_t workspace_bytes,
                           int32_t opts, void* stream);

/*
 * Periodic cutoff multigraph (Definition def6 with a constant cutoff c_i = cutoff).
 *
 *  cutoff        > 0 and finite, Angstrom; the test is strict (length < cutoff).
 *  capacity      number of edge slots in src/dst/image/length (>= 0). With capacity 0
 *                the call only counts (no fill): report->num_edges is the exact edge
 *                count, and row_ptr (if given) is filled, which sizes the outputs.
 *  src, dst      int32 [capacity]; image int32 [capacity][3]; length float32 [capacity].
 *  row_ptr       int64 [N+1] or NULL: edges of source i are row_ptr[i] .. row_ptr[i+1]-1
 *                (edges are grouped by ascending src; the order inside a source is
 *                deterministic but unspecified).
 *  report        one mg_report (device), overwritten.
 *  workspace     device scratch of workspace_bytes (see mg_cutoff_workspace_bytes);
 *                its contents are not needed between calls.
 *  opts          MG_OPT_* bits.
 * Errors: MG_ERR_INVALID_ARG for null inputs/outputs (outputs may be NULL only when
 * capacity == 0), B < 0, N < 0, N > INT32_MAX, bad cutoff; MG_ERR_WORKSPACE if the
 * workspace is smaller than mg_cutoff_workspace_bytes(B, N, 0).
 */
mg_status mg_cutoff_graph(const float* lattices, const float* frac, const int64_t* batch_ptr,
                          int32_t B, int64_t N, float cutoff, int64_t capacity,
                          int32_t* src, int32_t* dst, int32_t* image, float* length,
                          int64_t* row_ptr, mg_report* report,
                          void* workspace, size_t workspace_bytes, int32_t opts, void* stream);

/*
 * Periodic cutoff multigraph with per-atom cutoffs (Definition def6: the edge
 * (i, j, t) exists when its length is < c_i, the cutoff of its SOURCE atom, so
 * the graph need not be symmetric).
 *
 *  radii         float32 [N] device, c_i in Angstrom for every atom (global index);
 *                each must be finite and > 0, else that structure is skipped and
 *                MG_FLAG_NONFINITE is set. A structure's image range is taken at its
 *                largest c_i. May be NULL only when N == 0.
 *  All other arguments, outputs, ordering and errors as for mg_cutoff_graph; the
 *  workspace size is the same (mg_cutoff_workspace_bytes).
 */
mg_status mg_cutoff_graph_radii(const float* lattices, const float* frac, const int64_t* batch_ptr,
                                int32_t B, int64_t N, const float* radii, int64_t capacity,
                                int32_t* src, int32_t* dst, int32_t* image, float* length,
                                int64_t* row_ptr, mg_report* report,
                                void* workspace, size_t workspace_bytes, int32_t opts, void* stream);

/*
 * Periodic cutoff multigraph that also returns every edge's vector, the
 * displacement whose norm the cutoff test takes (Definition def6): the
 * geometry of the edges comes out of the same sweep, so a model that needs
 * (vec, length) right after building the graph does not stream the edge list
 * again. vec_e = p_ij + s_t in FP32, where p_ij (the wrapped pair
 * displacement times the lattice) and s_t = t L are each computed in FP64 and
 * rounded once; length_e is the correctly rounded norm of that FP32 vector.
 * Compared with mg_edge_geometry (FP64 throughout) the components differ by a
 * few FP32 ulps of |p_ij| + |s_t|.
 *
 *  radii         float32 [N] device per-atom cutoffs as in mg_cutoff_graph_radii,
 *                or NULL for the constant `cutoff` as in mg_cutoff_graph.
 *  vec           float32 [capacity][3]; must be non-NULL when capacity > 0.
 *  All other arguments, outputs, ordering and errors as for mg_cutoff_graph
 *  (mg_cutoff_graph_radii when radii is given); same workspace size.
 */
mg_status mg_cutoff_graph_vec(const float* lattices, const float* frac, const int64_t* batch_ptr,
                              int32_t B, int64_t N, float cutoff, const float* radii, int64_t capacity,
                              int32_t* src, int32_t* dst, int32_t* image, float* length, float* vec,
                              int64_t* row_ptr, mg_report* report,
                              void* workspace, size_t workspace_bytes, int32_t opts, void* stream);

/*
 * Periodic k-nearest-neighbour multigraph (Sec. 1; Sec. 2.2 Algorithms 1-2).
 * Every source gets exactly k edges: the k smallest (length, dst, t0, t1, t2) keys,
 * compared on the FP32 length, then the global dst index, then t lexicographically
 * (signed, ascending). Edge e = i*k + r is the r-th edge of source i in that order.
 *  k             1..64.
 *  src, dst      int32 [N*k]; image int32 [N*k][3]; length float32 [N*k].
 * Errors as for mg_cutoff_graph; MG_ERR_INVALID_ARG for k outside 1..64.
 */
mg_status mg_knn_graph(const float* lattices, const float* frac, const int64_t* batch_ptr,
                       int32_t B, int64_t N, int32_t k,
                       int32_t* src, int32_t* dst, int32_t* image, float* length,
                       mg_report* report, void* workspace, size_t workspace_bytes,
                       int32_t opts, void* stream);

/*
 * Edge vectors and lengths: vec_e = (frac[dst_e] - frac[src_e] + t_e) @ lattice[b(src_e)],
 * length_e = ||vec_e|| (the norm inside Definition def6). Computed in FP64, stored FP32.
 *  E             number of edges (>= 0).
 *  num_edges     int64 [1] device value or NULL: when given, only the first
 *                min(E, *num_edges) edges are processed (capacity-sized buffers).
 *  vec           float32 [E][3] or NULL; length float32 [E] or NULL.
 * src/dst must index atoms of the same structure (not checked).
 */
mg_status mg_edge_geometry(const float* lattices, const float* frac, const int64_t* batch_ptr,
                           int32_t B, int64_t N, const int32_t* src, const int32_t* dst,
                           const int32_t* image, int64_t E, const int64_t* num_edges,
                           float* vec, float* length,
                           void* workspace, size_t workspace_bytes, void* stream);

/*
 * Backward of mg_edge_geometry with the edge set held fixed (abstract, Sec. 4):
 *   g_e = grad_vec_e + grad_length_e * vec_e / length_e   (0 when length_e = 0)
 *   grad_frac[dst_e]  += g_e lattice^T,  grad_frac[src_e] -= g_e lattice^T
 *   grad_lattice[b]   += f_e^T g_e,      f_e = frac[dst_e] - frac[src_e] + t_e
 *  grad_vec      float32 [E][3] or NULL; grad_length float32 [E] or NULL.
 *  grad_frac     float32 [N][3] or NULL, overwritten (FP32 atomics: summation order varies).
 *  grad_lattice  float32 [B][3][3] or NULL, overwritten (accumulated in FP64).
 */
mg_status mg_edge_geometry_backward(const float* lattices, const float* frac,
                                    const int64_t* batch_ptr, int32_t B, int64_t N,
                                    const int32_t* src, const int32_t* dst, const int32_t* image,
                                    int64_t E, const int64_t* num_edges,
                                    const float* grad_vec, const float* grad_length,
                                    float* grad_frac, float* grad_lattice,
                                    void* workspace, size_t workspace_bytes, void* stream);

/*
 * mg_edge_geometry_backward without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the scratch lives in a device
 * array of the library, MG_STATIC_SCRATCH_BYTES per GPU, set up on the first
 * call on each device (with that device current) and kept until the process
 * ends. The call itself allocates nothing.
 *  Arguments, results and device flags as mg_edge_geometry_backward.
 *  Limit: B and N with mg_geometry_workspace_bytes(B, N) <= MG_STATIC_SCRATCH_BYTES
 *  (about 4.1 million atoms with a few thousand structures); larger batches
 *  return MG_ERR_UNSUPPORTED and enqueue nothing.
 *  Every call on one GPU uses that GPU's single scratch array: calls that
 *  overlap in time on one GPU (other streams or host threads) race and give
 *  wrong gradients; serialise them. The scratch keeps the last call's contents;
 *  the call clears what must start at zero itself.
 * Errors: as mg_edge_geometry_backward, MG_ERR_UNSUPPORTED past the limit,
 * MG_ERR_HIP when the scratch's device address cannot be obtained.
 */
#define MG_STATIC_SCRATCH_BYTES (16u << 20)
mg_status mg_edge_geometry_backward_static(const float* lattices, const float* frac,
                                           const int64_t* batch_ptr, int32_t B, int64_t N,
                                           const int32_t* src, const int32_t* dst, const int32_t* image,
                                           int64_t E, const int64_t* num_edges,
                                           const float* grad_vec, const float* grad_length,
                                           float* grad_frac, float* grad_lattice, void* stream);

/*
 * KNN multigraph with ties kept (Sec. 2.2, Algorithm 2: every candidate with
 * d <= d_k): the k nearest of every source plus every further (j, t) whose FP32
 * length equals the k-th one, in (length, dst, t) key order. The search keeps 64
 * keys per source; a source with more candidates at its k-th distance than fit
 * gets the first 64 and sets MG_FLAG_TIES.
 *
 *  k             1..63.
 *  capacity      edge slots in src/dst/image/length (>= 0).
 *  row_ptr       int64 [N+1] or NULL: edges of source i are row_ptr[i] .. row_ptr[i+1]-1.
 *  report        as for mg_knn_graph, except num_edges = the number of edges kept
 *                (exact even past capacity; MG_FLAG_CAPACITY then).
 *  Skipped structures (MG_FLAG_SINGULAR / NONFINITE / RANGE) contribute no edges.
 * Errors: as mg_knn_graph; MG_ERR_INVALID_ARG for k outside 1..63.
 */
mg_status mg_knn_graph_ties(const float* lattices, const float* frac, const int64_t* batch_ptr, int32_t B,
                            int64_t N, int32_t k, int64_t capacity, int32_t* src, int32_t* dst, int32_t* image,
                            float* length, int64_t* row_ptr, mg_report* report, void* workspace,
                            size_t workspace_bytes, int32_t opts, void* stream);

/*
 * Symmetric closure (Sec. 2.2, symmetric-graph procedure): the input edges plus,
 * for every edge (i, j, t) whose reverse (j, i, -t) is not an input edge, the
 * edge (j, i, -t) with the same length. Input edges must be unique; no edge is
 * added twice.
 *
 *  row_ptr       int64 [N+1] device: input edges of source i are row_ptr[i] ..
 *                row_ptr[i+1]-1 (i*k for a KNN graph). A range outside [0, E] is
 *                clamped and sets MG_FLAG_RANGE.
 *  dst, image    int32 [E], int32 [E][3]: the input edges (global atom indices).
 *                An edge with dst outside [0, N) is kept, not reversed, and sets
 *                MG_FLAG_RANGE.
 *  length        float32 [E] or NULL (needed only for out_length).
 *  capacity      slots in the outputs (>= 0).
 *  out_*         src/dst int32 [capacity], image int32 [capacity][3], length float32
 *                [capacity] or NULL. Order: by source; each source's input edges in
 *                input order, then the reverse edges it receives, ordered by the
 *                index of the input edge they reverse.
 *  out_row_ptr   int64 [N+1] or NULL.
 *  report        mg_report: num_edges = edges of the closure (exact even past
 *                capacity; MG_FLAG_CAPACITY then, nothing written past capacity).
 * Cost: each edge scans its destination's out-list, so the call suits modest
 * degrees (KNN graphs); cutoff graphs are already symmetric.
 * Errors: MG_ERR_INVALID_ARG (sizes, NULL pointers), MG_ERR_WORKSPACE.
 */
mg_status mg_symmetrize(const int64_t* row_ptr, int64_t N, const int32_t* dst, const int32_t* image,
                        const float* length, int64_t E, int64_t capacity, int32_t* out_src, int32_t* out_dst,
                        int32_t* out_image, float* out_length, int64_t* out_row_ptr, mg_report* report,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * Triplets (Definition def6, Gamma_2): every ordered pair (e1, e2) of two
 * different edges with the same source, for pair-based (angle) message passing.
 *
 *  row_ptr       int64 [N+1] device: the graph's edges of source i are
 *                row_ptr[i] .. row_ptr[i+1]-1 (mg_cutoff_graph's row_ptr; i*k for a
 *                KNN graph). Sources with an invalid range (negative, decreasing, past
 *                E, or more than 65536 edges) get no triplets and set MG_FLAG_RANGE.
 *  E             number of edges of the graph (< 2^31; edge indices are int32).
 *  vec           float32 [E][3] edge vectors (mg_edge_geometry) or NULL.
 *  capacity      slots in e1/e2/cos_theta (>= 0).
 *  e1, e2        int32 [capacity]: edge indices of the pair, ordered by source, then
 *                e1, then e2 (e2 != e1).
 *  cos_theta     float32 [capacity] or NULL: (v1 . v2) / (|v1| |v2|), 0 if a vector is 0.
 *  trip_ptr      int64 [N+1] or NULL: triplets of source i are trip_ptr[i] .. trip_ptr[i+1]-1.
 *  report        mg_report: num_edges = number of triplets (exact even past capacity;
 *                MG_FLAG_CAPACITY then, and nothing is written past capacity).
 * Errors: MG_ERR_INVALID_ARG (N < 0, E out of range, NULL row_ptr/report, NULL e1/e2
 * with capacity > 0, cos_theta without vec), MG_ERR_WORKSPACE.
 */
mg_status mg_triplets(const int64_t* row_ptr, int64_t N, int64_t E, const float* vec, int64_t capacity,
                      int32_t* e1, int32_t* e2, float* cos_theta, int64_t* trip_ptr, mg_report* report,
                      void* workspace, size_t workspace_bytes, void* stream);

/* ---- launch tuning and profiling (host-side state, per process) ---------- */

/* Tunable launch parameters of the sweeps; 0 in a field keeps the current value. */
typedef struct mg_tuning {
    int32_t cutoff_wgs_per_cu;    /* workgroups per CU for the cutoff sweeps (default 32; more than
                                     stay resident, so the dispatcher balances the items) */
    int32_t cutoff_slots;         /* destination atoms per lane per image step (1, 2 or 4) */
    int32_t knn_wgs_per_cu;       /* persistent workgroups per CU for the KNN sweep */
    int32_t knn_lambda_x4;        /* KNN first-search radius targets (lambda_x4/4)*k + 6 candidates */
    int32_t knn_tau_x8;           /* KNN: the first sweep keeps candidates within (tau_x8/8) times the
                                     k-th neighbour distance of a uniform density (sources with fewer
                                     than k there are swept again at the full search radius); default 10 */
    int32_t cutoff_img_group;     /* image-table entries the cutoff sweep reads per scalar load group
                                     (2, 4 or 8; default 4) */
    int32_t cutoff_cl_span;       /* cell lists of the cutoff calls: stencil half-width in bins, 1 (27
                                     bins at least the radius thick, the default) or 2 (125 bins at
                                     least half the radius thick: fewer candidates, smaller tiles) */
    int32_t knn_cl_span;          /* the same for the KNN calls' cell lists */
} mg_tuning;

/* [host] Read / replace the tuning parameters used by later calls. A field set to 0 in
 * mg_set_tuning keeps its current value. */
mg_status mg_get_tuning(mg_tuning* out);
mg_status mg_set_tuning(const mg_tuning* in);

/* [host] Phase timing: when enabled, every kernel phase of the calls above is
 * bracketed by hipEvents on the call's stream. mg_profile_read synchronises the
 * recorded events, and for up to `max` phases writes a NUL-terminated name
 * (32 bytes each) into names[i*32], the summed milliseconds into ms[i] and the
 * number of launches into count[i]; it returns the number of phases and clears
 * the record. Profiling adds event records, so leave it off outside measurements. */
mg_status mg_profile_enable(int32_t on);
int32_t mg_profile_read(char* names, double* ms, int64_t* count, int32_t max);

#ifdef __cplusplus
}
#endif
#endif /* MATGRAPH_H */

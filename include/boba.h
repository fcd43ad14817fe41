/*
 * boba.h -- C ABI of libboba.so, an MI355X (gfx950) implementation of the
 * data-parallel hot path of BOBA (Batched Order By Attachment, arXiv
 * 2306.10410): first-occurrence reorder -> edge relabel -> COO->CSR -> SpMV,
 * with batched plans, a learned reorder selector, destination binning, the
 * NBR locality metric and PageRank.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers (hipMalloc'd or equivalent), owned by
 *    the caller; the library keeps no reference after the call returns.
 *    Exceptions are marked "host".
 *  - Calls are asynchronous on `stream` (0 = the null stream): they enqueue
 *    kernels and return.  Outputs are valid once the stream reaches that point.
 *  - Vertex IDs are int32 in [0, n); edge counts m and vertex counts n must be
 *    < 2^31.  BOBA positions are uint32, so boba_reorder also needs 2m + n < 2^32.
 *  - Host-detectable errors (null pointers, negative or oversized sizes, a
 *    workspace that is too small) are returned before anything is enqueued.
 *  - Every kernel that indexes memory by a vertex ID bounds-checks it.  An
 *    out-of-range ID is skipped and recorded in a per-device flag; read and
 *    clear it with boba_check_device_error.  Results are unspecified then.
 *  - Results are deterministic: bit-identical across runs, launch shapes and
 *    tuning choices (BOBA_FLAG_RACY excepted, by design).
 *  - boba_last_error() returns a thread-local description of the last failure.
 */
#ifndef BOBA_H
#define BOBA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef BOBA_API
#define BOBA_API __attribute__((visibility("default")))
#endif

typedef int32_t boba_status;
#define BOBA_OK 0
#define BOBA_ERR_ARG 1       /* null pointer, negative size, bad flag */
#define BOBA_ERR_RANGE 2     /* a vertex ID outside [0, n) (device-detected) */
#define BOBA_ERR_OVERFLOW 3  /* m or n >= 2^31, or 2m + n >= 2^32 */
#define BOBA_ERR_WORKSPACE 4 /* workspace null or smaller than the query said */
#define BOBA_ERR_HIP 5       /* a HIP runtime call or kernel launch failed */
#define BOBA_ERR_TIMEOUT 6   /* a batched plan's bounded wait gave up (device-detected) */

/* boba_reorder flags */
#define BOBA_FLAG_INTERLEAVED 0x1u /* flatten as I(0) J(0) I(1) J(1) ... (Fig. 1)
                                      instead of I ++ J (Algorithms 1 and 2) */
#define BOBA_FLAG_RACY 0x2u        /* plain stores instead of AtomicMin in the
                                      scatter, as the paper's GPU kernel writes
                                      r (Sec. 4.4): first(v) becomes some
                                      position of v, not necessarily the first,
                                      and may differ from run to run.  For
                                      measuring what the atomic costs. */
#define BOBA_FLAG_FORCE_GENERAL 0x4u /* graphs of at most 32768 vertices and
                                      2^21 positions (2m + n) are normally
                                      reordered by one workgroup in one launch;
                                      this flag sends them through the
                                      many-workgroup path instead (identical
                                      results).  For testing and timing. */

/* Thread-local, NUL-terminated description of the most recent failure on this
 * thread ("" if none).  The string stays valid until the next call. */
BOBA_API const char *boba_last_error(void);

/* Waits for `stream`, then reports what the kernels on the current device
 * flagged since the last check, and clears it: *code = BOBA_ERR_TIMEOUT if a
 * batched plan's wait for another workgroup gave up (that launch's outputs
 * are then unspecified), else BOBA_ERR_RANGE if a vertex ID was out of range,
 * else BOBA_OK.  `code` is a host pointer. */
BOBA_API boba_status boba_check_device_error(hipStream_t stream, int32_t *code);

/* ------------------------------------------------------------- reorder ---
 * BOBA reordering (Sec. 4.4, Algorithm 2 with AtomicMin, which the paper notes
 * reproduces Algorithm 1 of Sec. 4.3 exactly).  With S = I ++ J (positions
 * 0..2m-1; I = src, J = dst) followed by the tail 0..n-1 (positions 2m..2m+n-1,
 * so vertices that never occur come last, in increasing old ID):
 *     first(v) = min { i : S[i] = v }
 *     perm[v]  = #{ u : first(u) < first(v) }       (new ID of old vertex v)
 *     order[k] = v  such that perm[v] = k           (the paper's permutation p)
 * i.e. vertices are numbered in order of first appearance.
 *   src, dst  int32[m]  edge list (COO); m may be 0 (then src/dst may be NULL).
 *   perm      int32[n]  output, required.
 *   order     int32[n]  output, may be NULL.
 *   ws        workspace of at least boba_reorder_workspace(n, m) bytes,
 *             256-byte aligned; contents on entry are ignored.
 *   flags     0, or any of BOBA_FLAG_INTERLEAVED, BOBA_FLAG_RACY and
 *             BOBA_FLAG_FORCE_GENERAL.
 * Errors: BOBA_ERR_ARG, BOBA_ERR_OVERFLOW, BOBA_ERR_WORKSPACE, BOBA_ERR_HIP. */
BOBA_API size_t boba_reorder_workspace(int64_t n, int64_t m);
BOBA_API boba_status boba_reorder(const int32_t *src, const int32_t *dst, int64_t m, int64_t n,
                         int32_t *perm, int32_t *order, void *ws, size_t ws_bytes,
                         uint32_t flags, hipStream_t stream);

/* boba_reorder for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * results as boba_reorder, with the workspace taken from library-owned device
 * memory instead of a caller buffer.  That memory is a static array of
 * BOBA_REORDER_NOALLOC_MAX_BYTES per device, held from the first call on a
 * device until the process ends.  The call allocates nothing; it accepts a
 * graph iff boba_reorder_workspace(n, m) <= BOBA_REORDER_NOALLOC_MAX_BYTES
 * (e.g. 2^16 vertices with 2^20 edges, or 2^14 vertices with 2^17 edges) and
 * otherwise returns BOBA_ERR_WORKSPACE before enqueuing anything.
 * Every call on a device shares that device's array: calls that overlap in
 * time on one device (two streams, two threads) race and give unspecified
 * results; calls ordered on one stream are safe.  The array keeps the last
 * call's contents, none of which a later call relies on.
 *   Arguments, flags and errors as boba_reorder, without ws / ws_bytes. */
#define BOBA_REORDER_NOALLOC_MAX_BYTES ((size_t)64 << 20)
BOBA_API boba_status boba_reorder_noalloc(const int32_t *src, const int32_t *dst, int64_t m, int64_t n,
                                          int32_t *perm, int32_t *order, uint32_t flags, hipStream_t stream);

/* ------------------------------------------------------------- relabel ---
 * Applies a vertex permutation to an edge list (the step between BOBA and CSR
 * construction, Sec. 5.3): src_out[k] = perm[src[k]], dst_out[k] = perm[dst[k]].
 * Edge order is unchanged.  In place is allowed (src_out == src and/or
 * dst_out == dst); other overlaps are not.
 *   src, dst, src_out, dst_out  int32[m];  perm  int32[n].
 * Errors: BOBA_ERR_ARG, BOBA_ERR_OVERFLOW, BOBA_ERR_HIP. */
BOBA_API boba_status boba_relabel(const int32_t *src, const int32_t *dst, int64_t m,
                         const int32_t *perm, int64_t n, int32_t *src_out, int32_t *dst_out,
                         hipStream_t stream);

/* The same relabel without a random perm read per endpoint: the edge list is
 * first split into vertex buckets (as boba_reorder does), each bucket's perm
 * slice is held on chip while its records get their new IDs, and the IDs go
 * back to edge order.  Same results as boba_relabel; faster on large graphs
 * (RMAT scale 24: 3.3 ms instead of 7.6 ms).  Graphs of more than 2^25
 * vertices take boba_relabel's path.
 *   ws  at least boba_relabel_bucketed_workspace(n, m) bytes, 256-byte aligned
 *       (about 16 bytes per edge).
 * Errors: as boba_relabel, and BOBA_ERR_WORKSPACE. */
BOBA_API size_t boba_relabel_bucketed_workspace(int64_t n, int64_t m);
BOBA_API boba_status boba_relabel_bucketed(const int32_t *src, const int32_t *dst, int64_t m, const int32_t *perm,
                                           int64_t n, int32_t *src_out, int32_t *dst_out, void *ws,
                                           size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------- reorder + relabel ---
 * boba_reorder followed by boba_relabel in one call (same results as the two
 * calls).  For graphs up to 2^25 vertices the relabel reuses the reorder's
 * vertex-bucketed copy of the edge list instead of gathering perm[] once per
 * endpoint.  src_out / dst_out may equal src / dst
 * (in place); other overlaps are not allowed.
 *   ws  at least boba_reorder_relabel_workspace(n, m) bytes, 256-byte aligned.
 * Errors: as boba_reorder. */
BOBA_API size_t boba_reorder_relabel_workspace(int64_t n, int64_t m);
BOBA_API boba_status boba_reorder_relabel(const int32_t *src, const int32_t *dst, int64_t m, int64_t n,
                                          int32_t *perm, int32_t *order, int32_t *src_out, int32_t *dst_out,
                                          void *ws, size_t ws_bytes, uint32_t flags, hipStream_t stream);

/* ---------------------------------------------------------- COO -> CSR ---
 * Builds CSR from COO (the conversion of Sec. 1.1 and Sec. 5.3) by a stable
 * sort on the row: rowptr[r] = #{k : row[k] < r}, and within each row the
 * entries keep their input order k.  Duplicates and self-loops are kept.
 *   row, col  int32[m];  val  float[m] or NULL.
 *   rowptr    int32[n_rows + 1] output;  col_out int32[m];  val_out float[m]
 *             (NULL exactly when val is NULL).  Outputs must not alias inputs.
 *   ws        at least coo_to_csr_workspace(n_rows, m) bytes, 256-byte aligned.
 * Errors: BOBA_ERR_ARG, BOBA_ERR_OVERFLOW, BOBA_ERR_WORKSPACE, BOBA_ERR_HIP. */
BOBA_API size_t coo_to_csr_workspace(int64_t n_rows, int64_t m);
BOBA_API boba_status coo_to_csr(const int32_t *row, const int32_t *col, const float *val, int64_t m,
                       int64_t n_rows, int32_t *rowptr, int32_t *col_out, float *val_out,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- SpMV ---
 * y = A x for CSR A (Algorithm 3, SpMV; rows of CSR as in Sec. 1.2):
 *     y[r] = sum_{e in [rowptr[r], rowptr[r+1])} val[e] * x[col[e]]
 * in FP32.  Work is split evenly over nonzeros, so very long rows cost no more
 * than many short ones; every row is summed in a fixed order, so results are
 * bit-reproducible.  val may be NULL (all ones).
 *   rowptr int32[n_rows+1], col int32[nnz], val float[nnz] or NULL,
 *   x float[n_cols], y float[n_rows] (must not alias x).  col and x may be
 *   NULL when nnz = 0.  rowptr should satisfy rowptr[0] = 0, non-decreasing,
 *   rowptr[n_rows] = nnz; offsets and row indices are clamped, so a malformed
 *   rowptr gives wrong sums, never out-of-bounds accesses.  Column indices
 *   outside [0, n_cols) are skipped and flagged.
 *   ws  at least spmv_csr_workspace(n_rows, nnz) bytes, 256-byte aligned.
 * Errors: BOBA_ERR_ARG, BOBA_ERR_OVERFLOW, BOBA_ERR_WORKSPACE, BOBA_ERR_HIP. */
BOBA_API size_t spmv_csr_workspace(int64_t n_rows, int64_t nnz);
BOBA_API boba_status spmv_csr(const int32_t *rowptr, const int32_t *col, const float *val,
                              int64_t n_rows, int64_t n_cols, int64_t nnz, const float *x, float *y,
                              void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------- batched ---
 * Many graphs reordered (and optionally relabelled) at once by one persistent
 * kernel replayed from a hipGraph.  Per graph the result is exactly that of
 * boba_reorder (+ boba_relabel) on the graph alone; this batching is not in the
 * paper, whose method is per graph (Sec. 4.4).
 *   G             number of graphs.
 *   h_edge_off    host int64[G+1], h_edge_off[0] = 0: graph g owns edges
 *                 [h_edge_off[g], h_edge_off[g+1]) of src/dst (and src_out/dst_out).
 *   h_vert_off    host int64[G+1], h_vert_off[0] = 0: graph g has
 *                 n_g = h_vert_off[g+1] - h_vert_off[g] vertices, local IDs
 *                 [0, n_g); its perm/order live at [h_vert_off[g], ...).
 *   src, dst      int32[total m] concatenated local edge lists.
 *   perm          int32[total n] output (local new IDs);  order may be NULL.
 *   src_out, dst_out  int32[total m] relabelled edges, or both NULL (reorder only).
 *   ws            at least boba_batch_workspace(...) bytes, 256-byte aligned; the
 *                 plan keeps pointers into it, so it must outlive the plan.
 *   tuning        NULL for defaults, else see boba_tuning (0 fields = default).
 * plan_create uploads the plan's tables on `stream` (and waits for them) and
 * captures the hipGraph; the inputs need not be ready yet.  plan_launch
 * replays it on `stream`.  A plan is bound to the pointers given at creation;
 * it is not thread-safe; destroy it before freeing the workspace.  Totals must
 * be < 2^31; each graph must satisfy boba_reorder's limits. */
typedef struct boba_tuning {
    int32_t small_max_n;  /* graphs with n_g <= this run whole in one workgroup (max 32768) */
    int32_t scatter_tile; /* records per (vertex bucket, slice) item of a large graph, at
                             most 4 slices per bucket; positions per item when large
                             graphs scatter with atomics (default 262144) */
    int32_t vertex_tile;  /* vertices per mark / rank item (default 65536) */
    int32_t relabel_tile; /* edges per relabel item (default 262144) */
    int32_t queues;       /* 1..8 ticket queues the graphs are dealt to (default 8, one per
                             XCD); with fewer, the workgroups of the other XCDs run the
                             items by helping.  Never changes results. */
    int32_t spin_limit;   /* sleeps before a wait for another workgroup gives up
                             (default 2^22, about 0.4 s); a give-up is reported as
                             BOBA_ERR_TIMEOUT by boba_check_device_error */
    int32_t scatter_atomic; /* 1: large graphs find first positions by device-wide atomic
                               minima instead of vertex buckets in LDS (the path graphs
                               of more than 2^26 vertices always take); default 0.
                               Never changes results. */
} boba_tuning;
typedef struct boba_batch_plan boba_batch_plan;
BOBA_API size_t boba_batch_workspace(int32_t G, const int64_t *h_edge_off, const int64_t *h_vert_off,
                                     const boba_tuning *tuning);
BOBA_API boba_status boba_batch_plan_create(int32_t G, const int64_t *h_edge_off, const int64_t *h_vert_off,
                                            const int32_t *src, const int32_t *dst, int32_t *perm, int32_t *order,
                                            int32_t *src_out, int32_t *dst_out, void *ws, size_t ws_bytes,
                                            const boba_tuning *tuning, hipStream_t stream, boba_batch_plan **plan);
BOBA_API boba_status boba_batch_plan_launch(boba_batch_plan *plan, hipStream_t stream);
/* info4 (host): items, whole-graph items, r words, bitmap words. */
BOBA_API boba_status boba_batch_plan_info(const boba_batch_plan *plan, int64_t *info4);
BOBA_API boba_status boba_batch_plan_destroy(boba_batch_plan *plan);

/* ------------------------------------------------ binning by destination ---
 * A stable sort of the edges by dst >> shift, shift = max(0, bits(n - 1) -
 * bin_bits): at most 2^bin_bits bins in order of destination, input order
 * kept inside a bin.  Sec. 5.6 suggests binning (or sorting) an edge list that
 * arrives in random order by destination before running BOBA.
 *   src, dst          int32[m] input edges (IDs expected in [0, n); others are
 *                     moved like any ID and reported by the next reorder)
 *   bin_bits          1..31; >= bits(n - 1) gives a full stable sort by dst
 *   src_out, dst_out  int32[m] output; must not alias the inputs
 *   ws                at least boba_bin_by_dst_workspace(n, m) bytes, 256-byte aligned.
 * Errors: ERR_ARG (NULL, aliasing, bin_bits), ERR_OVERFLOW (m or n >= 2^31),
 * ERR_WORKSPACE. */
BOBA_API size_t boba_bin_by_dst_workspace(int64_t n, int64_t m);
BOBA_API boba_status boba_bin_by_dst(const int32_t *src, const int32_t *dst, int64_t m, int64_t n, int32_t bin_bits,
                                     int32_t *src_out, int32_t *dst_out, void *ws, size_t ws_bytes,
                                     hipStream_t stream);

/* ------------------------------------------------------------ PageRank ---
 * PageRank, the iterative application of Sec. 5.1, as repeated SpMV
 * (Algorithm 3, pull form) over the transposed graph:
 *   r_0 = 1/n,  r_{k+1}[v] = (1 - damping)/n + damping * (sum_{u->v} r_k[u] / outdeg(u) + D_k / n)
 * where outdeg(u) counts the edges leaving u and D_k is the rank held by
 * vertices with no out-edge (spread evenly).  FP32 ranks and SpMV; the
 * reductions (D_k, the residual) in FP64 in a fixed order: bit-reproducible.
 *   rowptr, col  CSR of the transposed graph: row v lists the sources u of
 *                the edges u -> v (coo_to_csr(dst, src, ...)); int32[n+1],
 *                int32[nnz] (col NULL when nnz = 0).  Column IDs outside
 *                [0, n) are skipped and flagged (boba_check_device_error).
 *   out_rowptr   int32[n+1] row pointer of the forward CSR (row u lists the
 *                edges leaving u), giving the out-degrees in one coalesced
 *                pass; or NULL: they are then counted from col with one
 *                atomic per distinct vertex of every 8192 edges (much
 *                slower on large graphs: 10 ms for 2^28 edges on 2^24
 *                vertices).  Must describe the same graph.
 *   damping      in [0, 1] (0.85 is the usual choice).
 *   max_iter     iterations to run (>= 0).
 *   tol          > 0: stop after the first iteration k whose L1 change
 *                sum_v |r_{k+1}[v] - r_k[v]| is below tol; 0: run all max_iter.
 *   rank         float[n] output (device).
 *   residual     device double[max_iter] or NULL: the L1 change of every
 *                iteration run (entries past the last one are not written).
 *   iters        device int32[1] or NULL: iterations run.
 *   ws           at least boba_pagerank_workspace(n, nnz) bytes, 256-byte aligned.
 * n = 0 writes nothing.  The call does not wait for the device: the stop
 * test runs on the device, and the iterations after it return at once.
 * Errors: ERR_ARG (NULL, damping, max_iter, tol), ERR_OVERFLOW (a size >= 2^31),
 * ERR_WORKSPACE, ERR_HIP. */
BOBA_API size_t boba_pagerank_workspace(int64_t n, int64_t nnz);
BOBA_API boba_status boba_pagerank(const int32_t *rowptr, const int32_t *col, const int32_t *out_rowptr,
                                   int64_t n, int64_t nnz, float damping, int32_t max_iter, double tol,
                                   float *rank, double *residual, int32_t *iters, void *ws, size_t ws_bytes,
                                   hipStream_t stream);

/* ----------------------------------------------------------------- NBR ---
 * The spatial-locality metric of Sec. 5.2 over the rows of a CSR matrix: for
 * every row v with a non-empty neighbourhood N(v) (its column IDs, duplicates
 * included), the number of distinct cache lines the IDs fall in divided by
 * |N(v)|, where a line holds line_ids consecutive IDs (ID c lies in line
 * c / line_ids).  NBR is the mean of that ratio; lower is more local.
 *   rowptr         int32[n_rows + 1], col int32[nnz] (NULL when nnz = 0),
 *                  rowptr as for spmv_csr (clamped, never read out of bounds).
 *   line_ids       a power of two in [1, 2^30] (32: 128-byte lines of 4-byte values).
 *   lines_per_row  int32[n_rows] output, distinct lines per row (0 for empty
 *                  rows), or NULL.
 *   result         device double[4] output: result[0] = sum of the ratios over
 *                  the non-empty rows, result[1] = how many rows that is,
 *                  result[2] = NBR over all rows (result[0] / n_rows, 0 when
 *                  n_rows = 0), result[3] = NBR over the non-empty rows
 *                  (result[0] / result[1], 0 when there are none).  The sum
 *                  is taken in a fixed order (bit-reproducible).
 *   ws             at least boba_nbr_workspace(n_rows, nnz) bytes, 256-byte aligned.
 * Column IDs outside [0, n_cols) are flagged (boba_check_device_error); the
 * counts of the rows holding them are then unspecified (never an access out
 * of bounds).
 * Errors: ERR_ARG (NULL, line_ids), ERR_OVERFLOW (a size >= 2^31),
 * ERR_WORKSPACE, ERR_HIP. */
BOBA_API size_t boba_nbr_workspace(int64_t n_rows, int64_t nnz);
BOBA_API boba_status boba_nbr(const int32_t *rowptr, const int32_t *col, int64_t n_rows, int64_t n_cols,
                              int64_t nnz, int32_t line_ids, int32_t *lines_per_row, double *result, void *ws,
                              size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------ selector ---
 * A learned "will reordering pay off" selector (not in the paper; it targets
 * the net-speedup question of Sec. 1.1, Problem 2).
 *
 * boba_graph_features: 16 FP32 features of an edge list from n, m, 4096
 * evenly spread samples and 64 windows of min(1024, m) consecutive edges:
 *   0 log2(1+n)  1 log2(1+m)  2 log2(1 + m/max(n,1))
 *   3,4  log2(1 + n*C/(K(K-1)/2)), C = equal pairs among the src (dst) samples
 *   5,6  log2(1 + n*maxcount/K)   7,8  distinct samples / K   (K = 4096)
 *   9    window mean of sum|src-dst| / (L*n)
 *   10,11 window mean of #distinct (id >> 5) / L
 *   12,13 window mean of #(id_e == id_{e-1}) / (L-1)
 *   14,15 window mean of #(|id_e - id_{e-1}| < 32) / (L-1)
 * where sample k is edge floor(k*m/K) and window w starts at edge
 * floor(w*(m-L)/63).  feat16 is a device float[16]; ws at least
 * boba_graph_features_workspace() bytes, 256-byte aligned.
 *
 * MLP 16 -> 64 -> 64 -> 1 with ReLU, FP32, parameters row-major in one device
 * array of boba_mlp_param_count() = 5313 floats: W1[64][16] b1[64] W2[64][64]
 * b2[64] W3[1][64] b3[1].  X is float[B][16], y and yhat float[B].
 * boba_mlp_backward writes grad (float[5313]) of loss = mean((yhat - y)^2) and
 * loss (float[1]); ws at least boba_mlp_backward_workspace(B) bytes.
 * boba_mlp_adam updates params, m1, m2 (float[count]) in place with one Adam
 * step number t >= 1 (bias-corrected).  All reductions have a fixed order. */
BOBA_API size_t boba_graph_features_workspace(void);
BOBA_API boba_status boba_graph_features(const int32_t *src, const int32_t *dst, int64_t m, int64_t n,
                                         float *feat16, void *ws, size_t ws_bytes, hipStream_t stream);
BOBA_API int32_t boba_mlp_param_count(void);
BOBA_API boba_status boba_mlp_forward(const float *params, const float *X, int32_t B, float *yhat,
                                      hipStream_t stream);
BOBA_API size_t boba_mlp_backward_workspace(int32_t B);
BOBA_API boba_status boba_mlp_backward(const float *params, const float *X, const float *y, int32_t B,
                                       float *grad, float *loss, void *ws, size_t ws_bytes, hipStream_t stream);
BOBA_API boba_status boba_mlp_adam(float *params, float *m1, float *m2, const float *grad, int32_t count,
                                   int32_t t, float lr, float b1, float b2, float eps, hipStream_t stream);

/* -------------------------------------------------------------- timing ---
 * Per-kernel timing with HIP events, for benchmarks (off by default).  While
 * enabled, every kernel the library launches outside stream capture is
 * bracketed by a pair of events recorded on its stream. */
BOBA_API boba_status boba_timing_enable(int32_t on);
/* Waits for every recorded event, then writes up to max_entries entries: the
 * kernel names packed NUL-terminated into names_buf (host, buf_len bytes),
 * total_ms[k] (host) the summed durations and launches[k] (host) the launch
 * counts since the last collect.  Clears the records; returns the entry count. */
BOBA_API int32_t boba_timing_collect(char *names_buf, size_t buf_len, double *total_ms, int64_t *launches,
                                     int32_t max_entries);

#ifdef __cplusplus
}
#endif
#endif /* BOBA_H */

// CSR SpMV, y = A x (Algorithm 3, over CSR rows) in FP32.
//
// Rows of scale-free graphs range from empty to hundreds of thousands of
// entries, and reordered graphs put all empty rows together, so the work is
// split evenly over the merge of row ends and nonzeros (merge path): a chunk
// holds kChunk items, each either one nonzero or the end of one row.
//   split   binary search of every chunk's starting (row, nonzero) pair
//   chunk   products val*x[col] of the chunk's nonzeros into LDS (coalesced
//           col/val, gathered x); then each row meeting the chunk is summed:
//           segments of up to kShort entries by one thread, longer ones by a
//           wavefront with a fixed shuffle tree.  A row that lies inside the
//           chunk is written; a row crossing the chunk's start (head) or end
//           (tail) leaves a partial sum.
//   fixup   every row crossing chunk boundaries is summed from its tail
//           partial and the following head partials, in chunk order.
// Every sum has a fixed order, so results are bit-reproducible.
//
// PageRank as repeated SpMV (the PR application of Sec. 5.1; the paper's PR
// pushes ranks along edges with atomics, here the same iteration is pulled
// with Algorithm 3 over the transposed CSR, which needs no atomics):
//   r_{k+1}[v] = (1 - a)/n + a * (sum_{u -> v} r_k[u] / outdeg(u) + D_k / n)
// with damping a, r_0 = 1/n, and D_k the rank on vertices without out-edges.
//   init / outdeg   r = 1/n, out-degrees counted from the columns
//   step            per part of the vertices: x = r / outdeg (the SpMV's
//                   input), the partial dangling mass and, after an SpMV,
//                   the new rank and the partial L1 change (fused)
//   finish          one workgroup sums the partials in a fixed order, keeps
//                   D and the residual, and raises the stop flag once the
//                   residual is below the tolerance; every later kernel of
//                   the call then returns at once.
#include "internal.h"

namespace boba {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr uint32_t kChunk = kThreads * kItems;  // nonzeros per chunk
constexpr uint32_t kShort = 64;                  // longer segments: one wavefront each
constexpr uint32_t kNoRow = 0xFFFFFFFFu;
constexpr uint32_t kLongCap = kChunk / kShort + 1;  // disjoint rows of > kShort nonzeros in a chunk

// Merge-path split of diagonal d = c * kChunk: the number i of row ends and
// j = d - i of nonzeros that come before it, where row r ends after nonzero
// rowptr[r+1] - 1 and a row end is taken before an equal nonzero index.
__global__ __launch_bounds__(kThreads) void k_spmv_split(const int32_t *__restrict__ rowptr, uint32_t n_rows,
                                                         int32_t nnz, uint32_t nchunk, uint32_t *__restrict__ split_i,
                                                         uint32_t *__restrict__ split_j) {
    const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c > nchunk) return;
    const uint64_t total = (uint64_t)n_rows + (uint64_t)nnz;
    const uint64_t d = min((uint64_t)c * kChunk, total);
    uint64_t lo = d > (uint64_t)nnz ? d - (uint64_t)nnz : 0, hi = min(d, (uint64_t)n_rows);
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const int64_t end = min(max(rowptr[mid + 1], 0), nnz);  // row mid ends after nonzero end-1
        if (end <= (int64_t)(d - mid - 1)) lo = mid + 1;
        else hi = mid;
    }
    split_i[c] = (uint32_t)lo;
    split_j[c] = (uint32_t)(d - lo);
}

// Where the sum of row r's segment in chunk [e0, e1) goes.
__device__ __forceinline__ void emit(uint32_t r, uint32_t rb, uint32_t re, uint32_t e0, uint32_t e1, float acc,
                                     uint32_t c, float *__restrict__ y, uint32_t *__restrict__ head_row,
                                     float *__restrict__ head_sum, uint32_t *__restrict__ tail_row,
                                     float *__restrict__ tail_sum) {
    if (rb >= e0 && re <= e1) {
        y[r] = acc;  // whole row (or an empty row) in this chunk
    } else if (rb < e0) {
        head_row[c] = r;  // began in an earlier chunk
        head_sum[c] = acc;
    } else {
        tail_row[c] = r;  // begins here, continues in later chunks
        tail_sum[c] = acc;
    }
}

template <bool HAS_VAL>
__global__ __launch_bounds__(kThreads) void k_spmv_chunk(const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col,
                                                         const float *__restrict__ val, uint32_t n_rows,
                                                         uint32_t n_cols, int32_t nnz, const float *__restrict__ x,
                                                         const uint32_t *__restrict__ split_i,
                                                         const uint32_t *__restrict__ split_j,
                                                         float *__restrict__ y, uint32_t *__restrict__ head_row,
                                                         float *__restrict__ head_sum, uint32_t *__restrict__ tail_row,
                                                         float *__restrict__ tail_sum, int32_t *flag,
                                                         const uint32_t *__restrict__ skip) {
    if (skip && *skip) return;  // a converged PageRank iteration
    __shared__ float prod[kChunk];
    __shared__ uint32_t long_rows[kLongCap];
    __shared__ uint32_t n_long;
    const uint32_t c = blockIdx.x;
    const uint32_t e0 = split_j[c];
    const uint32_t e1 = max(e0, min(split_j[c + 1], e0 + kChunk));  // at most kChunk nonzeros
    if (threadIdx.x == 0) {
        n_long = 0;
        head_row[c] = kNoRow;
        tail_row[c] = kNoRow;
    }

    // Branch-free: every load of a thread is issued before the first use (out
    // of range entries read a clamped, valid address and are masked after).
    bool bad = false;
    if (e1 > e0) {  // uniform; a chunk of row ends only has no nonzero to read
        int32_t cc[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t e = e0 + j * kThreads + threadIdx.x;
            cc[j] = col[e < e1 ? e : e0];
        }
        float xv[kItems], vv[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t e = e0 + j * kThreads + threadIdx.x;
            xv[j] = x[(uint32_t)cc[j] < n_cols ? (uint32_t)cc[j] : 0u];
            vv[j] = HAS_VAL ? val[e < e1 ? e : e0] : 1.f;
        }
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t i = j * kThreads + threadIdx.x;
            const bool live = e0 + i < e1;
            const bool ok = (uint32_t)cc[j] < n_cols;
            bad |= live && !ok;
            prod[i] = live && ok ? (HAS_VAL ? vv[j] * xv[j] : xv[j]) : 0.f;
        }
    }
    if (bad) flag_range_error(flag);
    __syncthreads();

    // rows meeting this chunk: those ending in it, plus the open row at its end
    // (clamped: a malformed rowptr cannot index out of bounds)
    const uint32_t last = n_rows - 1;
    const uint32_t open_row = split_i[c + 1];  // row still open at the chunk's end
    const uint32_t row_lo = min(split_i[c], last);
    const uint32_t row_hi = min(min(open_row, last), row_lo + kChunk);
    for (uint32_t r = row_lo + threadIdx.x; r <= row_hi; r += kThreads) {
        const uint32_t rb = (uint32_t)min(max(rowptr[r], 0), nnz), re = (uint32_t)min(max(rowptr[r + 1], 0), nnz);
        const uint32_t sb = max(rb, e0), se = min(re, e1);
        if (r == open_row && sb >= se) continue;  // the open row has no entries here
        if (sb < se && se - sb > kShort) {
            const uint32_t q = atomicAdd(&n_long, 1u);
            if (q < kLongCap) {
                long_rows[q] = r;
                continue;
            }
            // more long rows than disjoint ones can be: only overlapping rows
            // of a malformed rowptr get here, and are summed by this thread
        }
        float acc = 0.f;
        for (uint32_t k = sb; k < se; ++k) acc += prod[k - e0];
        emit(r, rb, re, e0, e1, acc, c, y, head_row, head_sum, tail_row, tail_sum);
    }
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    for (uint32_t q = wave; q < min(n_long, kLongCap); q += kThreads / kWave) {
        const uint32_t r = long_rows[q];
        const uint32_t rb = (uint32_t)min(max(rowptr[r], 0), nnz), re = (uint32_t)min(max(rowptr[r + 1], 0), nnz);
        const uint32_t sb = max(rb, e0), se = min(re, e1);
        float acc = 0.f;
        for (uint32_t k = sb + lane; k < se; k += kWave) acc += prod[k - e0];
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, kWave);
        if (lane == 0) emit(r, rb, re, e0, e1, acc, c, y, head_row, head_sum, tail_row, tail_sum);
    }
}

__global__ __launch_bounds__(kThreads) void k_spmv_fixup(uint32_t nchunk, const uint32_t *__restrict__ head_row,
                                                         const float *__restrict__ head_sum,
                                                         const uint32_t *__restrict__ tail_row,
                                                         const float *__restrict__ tail_sum, float *__restrict__ y,
                                                         const uint32_t *__restrict__ skip) {
    if (skip && *skip) return;
    const uint32_t stride = gridDim.x * kThreads;
    for (uint32_t c = blockIdx.x * kThreads + threadIdx.x; c < nchunk; c += stride) {
        const uint32_t r = tail_row[c];
        if (r == kNoRow) continue;
        float acc = tail_sum[c];
        for (uint32_t d = c + 1; d < nchunk && head_row[d] == r; ++d) acc += head_sum[d];
        y[r] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void k_fill_f32(float *__restrict__ a, uint32_t count, float v) {
    const uint32_t stride = gridDim.x * kThreads;
    for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) a[i] = v;
}

constexpr uint32_t kPrParts = 4096;  // parts of the vertices in the reductions

__global__ __launch_bounds__(kThreads) void k_pr_init(uint32_t n, float *__restrict__ rank,
                                                      uint32_t *__restrict__ outdeg, uint32_t *__restrict__ state) {
    const uint32_t stride = gridDim.x * kThreads;
    const float r0 = 1.f / (float)n;
    for (uint32_t v = blockIdx.x * kThreads + threadIdx.x; v < n; v += stride) {
        rank[v] = r0;
        outdeg[v] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        state[0] = 0;  // stop flag
        state[1] = 0;  // iterations done
    }
}

// Out-degrees from the forward graph's row pointer (one coalesced pass).
__global__ __launch_bounds__(kThreads) void k_pr_outdeg_rowptr(const int32_t *__restrict__ out_rowptr, uint32_t n,
                                                               uint32_t nnz, uint32_t *__restrict__ outdeg) {
    const uint32_t stride = gridDim.x * kThreads;
    for (uint32_t u = blockIdx.x * kThreads + threadIdx.x; u < n; u += stride) {
        const int32_t a = out_rowptr[u], b = out_rowptr[u + 1];
        outdeg[u] = b > a ? min((uint32_t)(b - a), nnz) : 0u;
    }
}

// Out-degrees counted from the transposed graph's columns.  A workgroup takes
// kOutChunk entries at a time and first counts them in an LDS hash table
// (up to kProbe slots tried; an entry that finds none is counted in global
// memory directly), then adds one global atomic per distinct vertex: the
// hubs of a power-law graph, which occur many times in every chunk, no longer
// queue on one counter.  Counts are integers, so the order does not matter.
constexpr uint32_t kOutHash = 4096;
constexpr uint32_t kOutChunk = 8192;
constexpr uint32_t kProbe = 8;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

__global__ __launch_bounds__(kThreads) void k_pr_outdeg(const int32_t *__restrict__ col, uint32_t nnz, uint32_t n,
                                                        uint32_t *__restrict__ outdeg, int32_t *flag) {
    __shared__ uint32_t keys[kOutHash];
    __shared__ uint32_t cnts[kOutHash];
    bool bad = false;
    for (uint64_t c0 = (uint64_t)blockIdx.x * kOutChunk; c0 < nnz; c0 += (uint64_t)gridDim.x * kOutChunk) {
        for (uint32_t i = threadIdx.x; i < kOutHash; i += kThreads) {
            keys[i] = kEmptyKey;
            cnts[i] = 0;
        }
        __syncthreads();
        const uint32_t c1 = (uint32_t)min<uint64_t>(nnz, c0 + kOutChunk);
        for (uint32_t e = (uint32_t)c0 + threadIdx.x; e < c1; e += kThreads) {
            const uint32_t u = (uint32_t)col[e];
            if (u >= n) {
                bad = true;
                continue;
            }
            uint32_t h = (u * 2654435761u) >> 20;  // 12 bits: a slot of the 4096
            bool done = false;
            for (uint32_t t = 0; t < kProbe && !done; ++t) {
                const uint32_t old = atomicCAS(&keys[h], kEmptyKey, u);
                if (old == kEmptyKey || old == u) {
                    atomicAdd(&cnts[h], 1u);
                    done = true;
                }
                h = (h + 1) & (kOutHash - 1);
            }
            if (!done) atomicAdd(&outdeg[u], 1u);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kOutHash; i += kThreads)
            if (keys[i] != kEmptyKey) atomicAdd(&outdeg[keys[i]], cnts[i]);
        __syncthreads();
    }
    if (bad) flag_range_error(flag);
}

// Fixed-order sum over the workgroup of two doubles per thread; thread 0 gets
// the totals.
template <int BLOCK>
__device__ inline void block_sum2(double &a, double &b, double *la, double *lb) {
    la[threadIdx.x] = a;
    lb[threadIdx.x] = b;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            la[threadIdx.x] += la[threadIdx.x + h];
            lb[threadIdx.x] += lb[threadIdx.x + h];
        }
        __syncthreads();
    }
    a = la[0];
    b = lb[0];
}

// Part p of the vertices.  UPDATE: the new rank from y (the SpMV of x) and
// the dangling mass D kept by the last finish.  Then x = r / outdeg for the
// next SpMV and the part's dangling mass (and L1 change).
template <bool UPDATE>
__global__ __launch_bounds__(kThreads) void k_pr_step(uint32_t n, uint32_t per_part, float base, float damping,
                                                      const double *__restrict__ dangling,
                                                      const float *__restrict__ y, float *__restrict__ rank,
                                                      const uint32_t *__restrict__ outdeg, float *__restrict__ x,
                                                      double *__restrict__ part_dang, double *__restrict__ part_diff,
                                                      const uint32_t *__restrict__ skip) {
    if (UPDATE && *skip) return;
    __shared__ double la[kThreads], lb[kThreads];
    const float dn = UPDATE ? (float)(*dangling / (double)n) : 0.f;
    const uint32_t v0 = blockIdx.x * per_part, v1 = min(n, v0 + per_part);
    double dang = 0.0, diff = 0.0;
    for (uint32_t v = v0 + threadIdx.x; v < v1; v += kThreads) {
        float r = rank[v];
        if (UPDATE) {
            const float nr = base + damping * (y[v] + dn);
            diff += fabs((double)nr - (double)r);
            rank[v] = nr;
            r = nr;
        }
        const uint32_t d = outdeg[v];
        x[v] = d ? r / (float)d : 0.f;
        if (!d) dang += r;
    }
    block_sum2<kThreads>(dang, diff, la, lb);
    if (threadIdx.x == 0) {
        part_dang[blockIdx.x] = dang;
        part_diff[blockIdx.x] = diff;
    }
}

// Sums the partials (thread t takes parts t, t + 1024, ... in order, then a
// fixed tree).  it < 0: after init (no residual).
__global__ __launch_bounds__(1024) void k_pr_finish(uint32_t parts, const double *__restrict__ part_dang,
                                                    const double *__restrict__ part_diff, int32_t it, double tol,
                                                    double *__restrict__ dangling, double *__restrict__ residual,
                                                    uint32_t *__restrict__ state, int32_t *__restrict__ iters_out) {
    if (it >= 0 && state[0]) return;
    __shared__ double la[1024], lb[1024];
    double dang = 0.0, diff = 0.0;
    for (uint32_t p = threadIdx.x; p < parts; p += 1024) {
        dang += part_dang[p];
        diff += part_diff[p];
    }
    block_sum2<1024>(dang, diff, la, lb);
    if (threadIdx.x == 0) {
        *dangling = dang;
        if (it >= 0) {
            if (residual) residual[it] = diff;
            state[1] = (uint32_t)it + 1;
            if (tol > 0.0 && diff < tol) state[0] = 1;
        }
        if (iters_out) *iters_out = (int32_t)state[1];
    }
}

struct SpmvLayout {
    uint32_t *split_i, *split_j, *head_row, *tail_row;
    float *head_sum, *tail_sum;
    size_t bytes;
    uint32_t nchunk;
};

SpmvLayout spmv_layout(void *ws, int64_t n_rows, int64_t nnz) {
    SpmvLayout L;
    L.nchunk = ceil_div((uint64_t)n_rows + (uint64_t)nnz, kChunk);
    Carver c(ws);
    L.split_i = c.take<uint32_t>(L.nchunk + 1);
    L.split_j = c.take<uint32_t>(L.nchunk + 1);
    L.head_row = c.take<uint32_t>(L.nchunk);
    L.tail_row = c.take<uint32_t>(L.nchunk);
    L.head_sum = c.take<float>(L.nchunk);
    L.tail_sum = c.take<float>(L.nchunk);
    L.bytes = c.bytes();
    return L;
}

}  // namespace
}  // namespace boba

using namespace boba;

extern "C" size_t spmv_csr_workspace(int64_t n_rows, int64_t nnz) {
    if (n_rows < 0 || nnz < 0) return 0;
    return spmv_layout(nullptr, n_rows, nnz).bytes;
}

extern "C" boba_status spmv_csr(const int32_t *rowptr, const int32_t *col, const float *val, int64_t n_rows,
                                int64_t n_cols, int64_t nnz, const float *x, float *y, void *ws, size_t ws_bytes,
                                hipStream_t stream) {
    clear_error();
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(BOBA_ERR_ARG, "spmv_csr: negative size");
    if (n_rows >= (1ll << 31) || n_cols >= (1ll << 31) || nnz >= (1ll << 31))
        return fail(BOBA_ERR_OVERFLOW, "spmv_csr: sizes must be < 2^31");
    if (n_rows == 0) return BOBA_OK;
    if (!rowptr || !y) return fail(BOBA_ERR_ARG, "spmv_csr: rowptr or y is NULL");
    if (nnz > 0 && (!col || !x)) return fail(BOBA_ERR_ARG, "spmv_csr: col or x is NULL");
    const size_t need = spmv_csr_workspace(n_rows, nnz);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "spmv_csr: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)", need,
                    ws_bytes, ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    const uint32_t nr = (uint32_t)n_rows, nc = (uint32_t)n_cols;
    if (nnz == 0) {
        BOBA_LAUNCH("spmv_fill", k_fill_f32, dim3(grid_for(nr, kThreads * 4)), dim3(kThreads), stream, y, nr, 0.f);
        return BOBA_OK;
    }
    const SpmvLayout L = spmv_layout(ws, n_rows, nnz);
    BOBA_LAUNCH("spmv_split", k_spmv_split, dim3(ceil_div(L.nchunk + 1ull, kThreads)), dim3(kThreads), stream, rowptr,
                nr, (int32_t)nnz, L.nchunk, L.split_i, L.split_j);
    if (val)
        BOBA_LAUNCH("spmv", (k_spmv_chunk<true>), dim3(L.nchunk), dim3(kThreads), stream, rowptr, col, val, nr, nc,
                    (int32_t)nnz, x, (const uint32_t *)L.split_i, (const uint32_t *)L.split_j, y, L.head_row,
                    L.head_sum, L.tail_row, L.tail_sum, flag, (const uint32_t *)nullptr);
    else
        BOBA_LAUNCH("spmv", (k_spmv_chunk<false>), dim3(L.nchunk), dim3(kThreads), stream, rowptr, col, val, nr, nc,
                    (int32_t)nnz, x, (const uint32_t *)L.split_i, (const uint32_t *)L.split_j, y, L.head_row,
                    L.head_sum, L.tail_row, L.tail_sum, flag, (const uint32_t *)nullptr);
    BOBA_LAUNCH("spmv_fixup", k_spmv_fixup, dim3(grid_for(L.nchunk, kThreads)), dim3(kThreads), stream, L.nchunk,
                (const uint32_t *)L.head_row, (const float *)L.head_sum, (const uint32_t *)L.tail_row,
                (const float *)L.tail_sum, y, (const uint32_t *)nullptr);
    return BOBA_OK;
}

// ------------------------------------------------------------- PageRank ---
struct PrLayout {
    uint32_t parts = 0, per_part = 0;
    uint32_t *outdeg = nullptr, *state = nullptr;
    float *x = nullptr, *y = nullptr;
    double *part_dang = nullptr, *part_diff = nullptr, *dangling = nullptr;
    void *spmv_ws = nullptr;
    size_t spmv_bytes = 0, bytes = 0;
};

static PrLayout pr_layout(void *ws, int64_t n, int64_t nnz) {
    PrLayout L;
    L.per_part = n > 0 ? ceil_div((uint64_t)n, kPrParts) : 1;
    L.parts = n > 0 ? ceil_div((uint64_t)n, L.per_part) : 0;
    Carver c(ws);
    L.outdeg = c.take<uint32_t>((size_t)n);
    L.x = c.take<float>((size_t)n);
    L.y = c.take<float>((size_t)n);
    L.part_dang = c.take<double>(kPrParts);
    L.part_diff = c.take<double>(kPrParts);
    L.dangling = c.take<double>(1);
    L.state = c.take<uint32_t>(2);
    L.spmv_bytes = spmv_layout(nullptr, n, nnz).bytes;
    L.spmv_ws = c.take<char>(L.spmv_bytes);
    L.bytes = c.bytes();
    return L;
}

extern "C" size_t boba_pagerank_workspace(int64_t n, int64_t nnz) {
    if (n < 0 || nnz < 0) return 0;
    return pr_layout(nullptr, n, nnz).bytes;
}

extern "C" boba_status boba_pagerank(const int32_t *rowptr, const int32_t *col, const int32_t *out_rowptr,
                                     int64_t n, int64_t nnz, float damping, int32_t max_iter, double tol,
                                     float *rank, double *residual, int32_t *iters, void *ws, size_t ws_bytes,
                                     hipStream_t stream) {
    clear_error();
    if (n < 0 || nnz < 0) return fail(BOBA_ERR_ARG, "boba_pagerank: negative size");
    if (n >= (1ll << 31) || nnz >= (1ll << 31)) return fail(BOBA_ERR_OVERFLOW, "boba_pagerank: sizes must be < 2^31");
    if (!(damping >= 0.f && damping <= 1.f))
        return fail(BOBA_ERR_ARG, "boba_pagerank: damping must lie in [0, 1] (got %g)", (double)damping);
    if (max_iter < 0) return fail(BOBA_ERR_ARG, "boba_pagerank: max_iter < 0");
    if (!(tol >= 0.0)) return fail(BOBA_ERR_ARG, "boba_pagerank: tol must be >= 0");
    if (n == 0) return BOBA_OK;
    if (!rowptr || !rank) return fail(BOBA_ERR_ARG, "boba_pagerank: rowptr or rank is NULL");
    if (nnz > 0 && !col) return fail(BOBA_ERR_ARG, "boba_pagerank: col is NULL");
    const size_t need = boba_pagerank_workspace(n, nnz);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "boba_pagerank: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)",
                    need, ws_bytes, ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    const PrLayout L = pr_layout(ws, n, nnz);
    const SpmvLayout S = spmv_layout(L.spmv_ws, n, nnz);
    const uint32_t un = (uint32_t)n, ue = (uint32_t)nnz;
    const float base = (1.f - damping) / (float)un;
    BOBA_LAUNCH("pr_init", k_pr_init, dim3(grid_for(un, kThreads * 4)), dim3(kThreads), stream, un, rank, L.outdeg,
                L.state);
    if (ue > 0) {
        if (out_rowptr)
            BOBA_LAUNCH("pr_outdeg", k_pr_outdeg_rowptr, dim3(grid_for(un, kThreads * 4)), dim3(kThreads), stream,
                        out_rowptr, un, ue, L.outdeg);
        else
            BOBA_LAUNCH("pr_outdeg", k_pr_outdeg, dim3(grid_for(ue, kOutChunk, 2048)), dim3(kThreads), stream, col,
                        ue, un, L.outdeg, flag);
        BOBA_LAUNCH("spmv_split", k_spmv_split, dim3(ceil_div(S.nchunk + 1ull, kThreads)), dim3(kThreads), stream,
                    rowptr, un, (int32_t)ue, S.nchunk, S.split_i, S.split_j);
    }
    BOBA_LAUNCH("pr_step", k_pr_step<false>, dim3(L.parts), dim3(kThreads), stream, un, L.per_part, base, damping,
                (const double *)L.dangling, (const float *)L.y, rank, (const uint32_t *)L.outdeg, L.x, L.part_dang,
                L.part_diff, (const uint32_t *)L.state);
    BOBA_LAUNCH("pr_finish", k_pr_finish, dim3(1), dim3(1024), stream, L.parts, (const double *)L.part_dang,
                (const double *)L.part_diff, -1, tol, L.dangling, residual, L.state, iters);
    for (int32_t it = 0; it < max_iter; ++it) {
        if (ue > 0) {
            BOBA_LAUNCH("spmv", (k_spmv_chunk<false>), dim3(S.nchunk), dim3(kThreads), stream, rowptr, col,
                        (const float *)nullptr, un, un, (int32_t)ue, (const float *)L.x,
                        (const uint32_t *)S.split_i, (const uint32_t *)S.split_j, L.y, S.head_row, S.head_sum,
                        S.tail_row, S.tail_sum, flag, (const uint32_t *)L.state);
            BOBA_LAUNCH("spmv_fixup", k_spmv_fixup, dim3(grid_for(S.nchunk, kThreads)), dim3(kThreads), stream,
                        S.nchunk, (const uint32_t *)S.head_row, (const float *)S.head_sum,
                        (const uint32_t *)S.tail_row, (const float *)S.tail_sum, L.y, (const uint32_t *)L.state);
        } else {
            BOBA_LAUNCH("spmv_fill", k_fill_f32, dim3(grid_for(un, kThreads * 4)), dim3(kThreads), stream, L.y, un,
                        0.f);
        }
        BOBA_LAUNCH("pr_step", k_pr_step<true>, dim3(L.parts), dim3(kThreads), stream, un, L.per_part, base, damping,
                    (const double *)L.dangling, (const float *)L.y, rank, (const uint32_t *)L.outdeg, L.x,
                    L.part_dang, L.part_diff, (const uint32_t *)L.state);
        BOBA_LAUNCH("pr_finish", k_pr_finish, dim3(1), dim3(1024), stream, L.parts, (const double *)L.part_dang,
                    (const double *)L.part_diff, it, tol, L.dangling, residual, L.state, iters);
    }
    return BOBA_OK;
}

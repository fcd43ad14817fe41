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
#include "internal.h"

namespace boba {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr uint32_t kChunk = kThreads * kItems;  // nonzeros per chunk
constexpr uint32_t kShort = 64;                  // longer segments: one wavefront each
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

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
                                                         float *__restrict__ tail_sum, int32_t *flag) {
    __shared__ float prod[kChunk];
    __shared__ uint32_t long_rows[kChunk / kShort + 1];
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
            long_rows[atomicAdd(&n_long, 1u)] = r;
            continue;
        }
        float acc = 0.f;
        for (uint32_t k = sb; k < se; ++k) acc += prod[k - e0];
        emit(r, rb, re, e0, e1, acc, c, y, head_row, head_sum, tail_row, tail_sum);
    }
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    for (uint32_t q = wave; q < n_long; q += kThreads / kWave) {
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
                                                         const float *__restrict__ tail_sum, float *__restrict__ y) {
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
                    L.head_sum, L.tail_row, L.tail_sum, flag);
    else
        BOBA_LAUNCH("spmv", (k_spmv_chunk<false>), dim3(L.nchunk), dim3(kThreads), stream, rowptr, col, val, nr, nc,
                    (int32_t)nnz, x, (const uint32_t *)L.split_i, (const uint32_t *)L.split_j, y, L.head_row,
                    L.head_sum, L.tail_row, L.tail_sum, flag);
    BOBA_LAUNCH("spmv_fixup", k_spmv_fixup, dim3(grid_for(L.nchunk, kThreads)), dim3(kThreads), stream, L.nchunk,
                (const uint32_t *)L.head_row, (const float *)L.head_sum, (const uint32_t *)L.tail_row,
                (const float *)L.tail_sum, y);
    return BOBA_OK;
}

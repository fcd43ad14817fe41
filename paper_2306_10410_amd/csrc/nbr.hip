// NBR spatial-locality metric over CSR rows (Sec. 5.2): for every row v with
// a non-empty neighbourhood N(v), the number of distinct cache lines its
// column IDs fall in (a line holds line_ids consecutive IDs) divided by
// |N(v)|, duplicates counted in |N(v)| as they occur; the metric is the mean
// of that ratio.
//   split   the first row of every chunk: chunks hold kChunkE items, an item
//           being a row or an entry (row r starts at item r + rowptr[r]), so
//           runs of empty rows are shared out like entries
//   chunk   a workgroup per chunk stages the line IDs of its rows' entries in
//           LDS and finds each entry's row by a max-scan of the rows' first
//           entries; a lane per entry then inserts (row, line) into an LDS
//           hash set (the insertion that finds the pair absent is a new
//           line), and the first lane of each row's run in a wavefront adds
//           the run's new lines to the row's count.  Rows longer than kSmall
//           are put on lists, by length.
//   mid     a workgroup per listed row of up to kMid entries with an LDS hash
//           set of its lines; the insertion that finds a line absent counts.
//   big     a workgroup per longer listed row with an LDS bitmap: over all
//           lines in one pass when they number at most 2^20, else one pass
//           per 2^20 lines of the row's [min, max] line span; an entry is new
//           when its bit was clear.
//   reduce  the per-row ratios summed in a fixed order (per part of the rows,
//           then over the parts), so the result is bit-reproducible.
#include <algorithm>

#include "internal.h"

namespace boba {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kChunkE = 1024;                // items (rows + entries) per chunk
constexpr uint32_t kSmall = 256;                  // longest row the chunk kernel counts
constexpr uint32_t kWin = kChunkE + kSmall;       // entries a chunk stages
constexpr uint32_t kPerThread = kWin / kThreads;  // staged entries per thread in the row scan
constexpr uint32_t kRowsPerThread = kChunkE / kThreads;  // rows of a chunk per thread
constexpr uint32_t kLists = kWave;                // lists of rows longer than kSmall
constexpr uint32_t kBigPerChunk = (kChunkE + kSmall + 1) / (kSmall + 2);  // ceil(kChunkE / (kSmall + 2))
constexpr uint32_t kMid = 2048;                   // longest row the hash-set kernel counts
constexpr uint32_t kMidThreads = 256;
constexpr uint32_t kMidTableBits = 12;            // 4096 slots: at most half full
constexpr uint32_t kMidTable = 1u << kMidTableBits;
constexpr uint32_t kNotCounted = 0xFFFFFFFFu;     // count slot of rows the chunk does not count
constexpr uint32_t kTableBits = 11;               // hash set of a chunk's (row, line) pairs
constexpr uint32_t kTable = 1u << kTableBits;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
static_assert(kWin % kThreads == 0 && kChunkE % kThreads == 0 && kThreads % kWave == 0,
              "the window and the rows split evenly over the threads");
static_assert(kTable > kWin && kMidTable > kMid, "a free slot is always left");
constexpr int kBigThreads = 1024;
constexpr uint32_t kBitmapWords = 32768;          // 128 KB: 2^20 lines per pass
constexpr uint32_t kParts = 1024;                 // parts of the rows in the reduction

__device__ __forceinline__ uint32_t clamp_ptr(int32_t p, uint32_t nnz) {
    return p < 0 ? 0u : min((uint32_t)p, nnz);
}

// chunk[c] = {r, rowptr[r]} for the first row r with r + rowptr[r] >=
// c * kChunkE (r = n_rows for c = nchunk); also clears the big-row counters.
__global__ __launch_bounds__(kThreads) void k_nbr_split(const int32_t *__restrict__ rowptr, uint32_t n_rows,
                                                        uint32_t nnz, uint32_t nchunk, uint2 *__restrict__ chunk,
                                                        uint32_t *__restrict__ list_count) {
    const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c < 2 * kLists) list_count[c] = 0;
    if (c > nchunk) return;
    uint32_t lo = 0, hi = n_rows;
    if (c == nchunk) {
        lo = n_rows;
    } else {
        const uint32_t target = c * kChunkE;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (mid + clamp_ptr(rowptr[mid], nnz) < target) lo = mid + 1;
            else hi = mid;
        }
    }
    chunk[c] = make_uint2(lo, clamp_ptr(rowptr[lo], nnz));
}

__global__ __launch_bounds__(kThreads) void k_nbr_chunk(const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ col, uint32_t n_cols,
                                                        uint32_t nnz, uint32_t shift,
                                                        const uint2 *__restrict__ chunk,
                                                        uint32_t *__restrict__ nd_out,
                                                        uint32_t *__restrict__ lists, uint32_t per_list,
                                                        uint32_t *__restrict__ list_count, int32_t *flag) {
    __shared__ uint32_t lines[kWin];
    __shared__ uint16_t rowof[kWin];      // 1 + the chunk-local row of each staged entry (0: none)
    __shared__ uint32_t rcnt[kChunkE];    // distinct lines of each counted row; kNotCounted for the others
    __shared__ uint32_t table[kTable];    // hash set of (row, line): the staged entry that holds the pair
    __shared__ uint32_t red[kThreads / kWave];
    __shared__ uint32_t list_at[4];       // the chunk's listed rows per class, and their first slots
    const uint2 first = chunk[blockIdx.x], next = chunk[blockIdx.x + 1];
    const uint32_t r_lo = first.x, r_hi = next.x;
    if (r_lo >= r_hi) return;
    // the chunk's rows start within kChunkE entries of the first one, so
    // every row that is not listed ends by base + kChunkE + kSmall
    const uint32_t base = first.y;
    const uint32_t wend = min(next.y, min(nnz, base + kChunkE + kSmall));
    const uint32_t cnt = wend > base ? min(wend - base, kWin) : 0u;
    // a chunk holds at most kChunkE rows (r + rowptr[r] grows with r); more
    // can only come from a malformed rowptr and are given 0 below
    const uint32_t nrows = r_hi - r_lo;
    // every load of the window and of the rows' bounds in flight at once:
    // unconditional loads at clamped (always valid) indices, so that no
    // branch makes one wait before the next is issued
    uint32_t v[kPerThread], s[kRowsPerThread], e[kRowsPerThread];
    if (cnt > 0) {  // the same for the whole workgroup
#pragma unroll
        for (uint32_t k = 0; k < kPerThread; ++k)
            v[k] = (uint32_t)col[base + min(threadIdx.x + k * kThreads, cnt - 1)];
    }
    int32_t ps[kRowsPerThread], pe[kRowsPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerThread; ++k) {
        const uint32_t j = threadIdx.x + k * kThreads;
        ps[k] = rowptr[r_lo + min(j, nrows)];
        pe[k] = rowptr[r_lo + min(j + 1, nrows)];
    }
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerThread; ++k) {
        const bool ok = threadIdx.x + k * kThreads < nrows;
        s[k] = ok ? clamp_ptr(ps[k], nnz) : 0u;
        e[k] = ok ? clamp_ptr(pe[k], nnz) : 0u;
    }
#pragma unroll
    for (uint32_t k = 0; k < kPerThread; ++k) {
        const uint32_t i = threadIdx.x + k * kThreads;
        if (i < cnt) {
            if (v[k] >= n_cols) flag_range_error(flag);
            lines[i] = v[k] >> shift;
        }
        rowof[i] = 0;
    }
    for (uint32_t h = threadIdx.x; h < kTable; h += kThreads) table[h] = kEmpty;
    if (threadIdx.x < 2) list_at[threadIdx.x] = 0;
    __syncthreads();
    // rows longer than kSmall go on list c mod kLists of their class (up to
    // kMid entries: class 0, the hash-set kernel's; longer: class 1, the
    // bitmap kernel's), with one counter update per class and chunk whose
    // reply is not waited for until the end (kLists counters, so that the
    // updates of neighbouring chunks do not queue on one address); empty
    // rows get 0, the others mark their first entry
    uint32_t slot[kRowsPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerThread; ++k) {
        const uint32_t j = threadIdx.x + k * kThreads;
        const bool ok = j < nrows;
        const uint32_t d = e[k] > s[k] ? e[k] - s[k] : 0u;
        const bool big = ok && d > kSmall;
        const uint32_t cls = d > kMid;
        slot[k] = big ? (cls << 31) | atomicAdd(&list_at[cls], 1u) : ~0u;
        const bool staged = ok && d > 0 && s[k] >= base && s[k] - base < cnt;
        const bool counted = staged && !big && s[k] - base + d <= cnt;
        if (staged) rowof[s[k] - base] = (uint16_t)(j + 1);  // listed rows too: their entries are skipped
        if (ok) rcnt[j] = counted ? 0u : kNotCounted;
        if (ok && !big && !counted) nd_out[r_lo + j] = 0;
    }
    for (uint32_t j = kChunkE + threadIdx.x; j < nrows; j += kThreads) {  // malformed rowptr only
        const uint32_t r = r_lo + j;
        const uint32_t rs = clamp_ptr(rowptr[r], nnz), re = clamp_ptr(rowptr[r + 1], nnz);
        if (re > rs && re - rs > kSmall) {
            const uint32_t li = (re - rs > kMid) * kLists + blockIdx.x % kLists;
            const uint32_t i = atomicAdd(&list_count[li], 1u);
            if (i < per_list) lists[(size_t)li * per_list + i] = r;
        } else {
            nd_out[r] = 0;
        }
    }
    __syncthreads();
    uint32_t base0 = 0, base1 = 0;
    if (threadIdx.x == 0) {
        if (list_at[0] > 0) base0 = atomicAdd(&list_count[blockIdx.x % kLists], list_at[0]);
        if (list_at[1] > 0) base1 = atomicAdd(&list_count[kLists + blockIdx.x % kLists], list_at[1]);
    }
    // the row of entry i is the last row marked at or before i (max-scan)
    {
        uint32_t loc[kPerThread], m = 0;
#pragma unroll
        for (uint32_t k = 0; k < kPerThread; ++k) {
            loc[k] = rowof[threadIdx.x * kPerThread + k];
            m = max(m, loc[k]);
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan<kThreads>(m, OpMax{}, red, total);
#pragma unroll
        for (uint32_t k = 0; k < kPerThread; ++k) {
            run = max(run, loc[k]);
            rowof[threadIdx.x * kPerThread + k] = (uint16_t)run;
        }
    }
    __syncthreads();
    // a lane per entry inserts (row, line) into the hash set; the entry whose
    // insertion finds the pair absent is the row's first in that line
    const uint32_t lane = threadIdx.x & (kWave - 1);
    for (uint32_t i0 = (threadIdx.x / kWave) * kWave; i0 < cnt; i0 += kThreads) {
        const uint32_t i = i0 + lane;  // < kWin: cnt <= kWin, a multiple of kWave
        const bool in = i < cnt;
        const uint32_t j1 = in ? rowof[i] : 0u;
        const bool act = j1 != 0 && rcnt[j1 - 1] != kNotCounted;
        bool is_new = false;
        if (act) {
            const uint32_t my = lines[i];
            // linear probing ends: the table has more slots than a chunk has entries
            uint32_t h = ((my * 0x9E3779B1u) ^ (j1 * 0x85EBCA77u)) >> (32 - kTableBits);
            for (;;) {
                const uint32_t old = atomicCAS(&table[h], kEmpty, i);
                if (old == kEmpty) {
                    is_new = true;
                    break;
                }
                if (lines[old] == my && rowof[old] == j1) break;  // old < cnt: a staged entry
                h = (h + 1) & (kTable - 1);
            }
        }
        // the lanes of one row are consecutive: the first lane of each run
        // adds the run's new lines to the row's count
        const uint64_t fresh = __ballot(is_new);
        const uint32_t jp = in && lane > 0 ? rowof[i - 1] : 0u;
        const bool head = in && (lane == 0 || jp != j1);
        const uint64_t heads = __ballot(head);
        if (act && head) {
            const uint64_t above = lane + 1 < kWave ? (heads >> (lane + 1)) << (lane + 1) : 0ull;
            const uint64_t end = above & (~above + 1);  // lowest head above this lane, 0 if none
            const uint64_t run = (end ? end - 1 : ~0ull) & (~0ull << lane);
            const uint32_t n = (uint32_t)__popcll(fresh & run);
            if (n) atomicAdd(&rcnt[j1 - 1], n);
        }
    }
    if (threadIdx.x == 0) {
        list_at[2] = base0;
        list_at[3] = base1;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerThread; ++k) {
        const uint32_t j = threadIdx.x + k * kThreads;
        if (j < nrows && rcnt[j] != kNotCounted) nd_out[r_lo + j] = rcnt[j];
        if (slot[k] != ~0u) {
            const uint32_t cls = slot[k] >> 31, at = list_at[2 + cls] + (slot[k] & 0x7FFFFFFFu);
            if (at < per_list)  // always, unless rowptr is malformed
                lists[(size_t)(cls * kLists + blockIdx.x % kLists) * per_list + at] = r_lo + j;
        }
    }
}

// The lengths of the kLists lists of one class (read by the first
// wavefront) and the number of visits that covers the longest.  Visit v is
// entry v / kLists of list v % kLists: about the order of the chunks that
// filled the lists, so the rows of the first chunks, BOBA's hubs, are handed
// out first.  Every thread of the workgroup calls it.
__device__ uint64_t list_visits(const uint32_t *__restrict__ counts, uint32_t per_list, uint32_t *len,
                                uint32_t *longest) {
    if (threadIdx.x < kWave) {
        const uint32_t n = min(counts[threadIdx.x], per_list);
        len[threadIdx.x] = n;
        const uint32_t m = wave_reduce(n, OpMax{});
        if (threadIdx.x == 0) *longest = m;
    }
    __syncthreads();
    return (uint64_t)kLists * *longest;
}

// A workgroup per listed row of kSmall < d <= kMid entries: the row's lines
// go into an LDS hash set (linear probing, compare-and-swap of the line);
// the insertion that finds the line absent counts it.
__global__ __launch_bounds__(kMidThreads) void k_nbr_mid(const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col, uint32_t n_cols,
                                                         uint32_t nnz, uint32_t shift,
                                                         const uint32_t *__restrict__ list, uint32_t per_list,
                                                         const uint32_t *__restrict__ counts,
                                                         uint32_t *__restrict__ nd_out, int32_t *flag) {
    __shared__ uint32_t tab[kMidTable];
    __shared__ uint32_t red[kMidThreads / kWave];
    __shared__ uint32_t len[kLists];
    __shared__ uint32_t longest;
    const uint64_t visits = list_visits(counts, per_list, len, &longest);
    for (uint64_t vi = blockIdx.x; vi < visits; vi += gridDim.x) {
        const uint32_t l = (uint32_t)(vi % kLists), p = (uint32_t)(vi / kLists);
        if (p >= len[l]) continue;  // the same for the whole workgroup
        const uint32_t r = list[(size_t)l * per_list + p];
        const uint32_t s = clamp_ptr(rowptr[r], nnz);
        // at most kMid < kMidTable insertions, so a free slot is always left
        const uint32_t e = min(max(s, clamp_ptr(rowptr[r + 1], nnz)), s + kMid);
        for (uint32_t h = threadIdx.x; h < kMidTable; h += kMidThreads) tab[h] = kEmpty;
        __syncthreads();
        uint32_t fresh = 0;
        for (uint32_t k = s + threadIdx.x; k < e; k += kMidThreads) {
            const uint32_t v = (uint32_t)col[k];
            if (v >= n_cols) {
                flag_range_error(flag);
                continue;
            }
            const uint32_t line = v >> shift;  // < 2^31, never kEmpty
            uint32_t h = (line * 0x9E3779B1u) >> (32 - kMidTableBits);
            for (;;) {
                const uint32_t old = atomicCAS(&tab[h], kEmpty, line);
                if (old == kEmpty) {
                    ++fresh;
                    break;
                }
                if (old == line) break;
                h = (h + 1) & (kMidTable - 1);
            }
        }
        // (its first barrier also keeps the next row's clearing after every insertion)
        const uint32_t nd = block_reduce<kMidThreads>(fresh, OpSum{}, red);
        if (threadIdx.x == 0) nd_out[r] = nd;
    }
}

// A workgroup per listed row longer than kMid.  The bitmap (dynamic LDS,
// `words` words) covers lines [p0, p0 + 32*words).  When all lines fit
// (`whole`), one pass over [0, 32*words) serves every row; otherwise the
// row's [min, max] line span is found first and covered in as many passes as
// it takes.
__global__ __launch_bounds__(kBigThreads) void k_nbr_big(const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col, uint32_t n_cols,
                                                         uint32_t nnz, uint32_t shift, uint32_t words, bool whole,
                                                         const uint32_t *__restrict__ big_list, uint32_t per_list,
                                                         const uint32_t *__restrict__ big_count,
                                                         uint32_t *__restrict__ nd_out, int32_t *flag) {
    extern __shared__ uint32_t bm[];
    __shared__ uint32_t red[kBigThreads / kWave];
    __shared__ uint32_t len[kLists];
    __shared__ uint32_t longest;
    const uint64_t visits = list_visits(big_count, per_list, len, &longest);
    const uint64_t cover = 32ull * words;
    for (uint64_t vi = blockIdx.x; vi < visits; vi += gridDim.x) {
        const uint32_t l = (uint32_t)(vi % kLists), p = (uint32_t)(vi / kLists);
        if (p >= len[l]) continue;  // the same for the whole workgroup
        const uint32_t r = big_list[(size_t)l * per_list + p];
        const uint32_t s = clamp_ptr(rowptr[r], nnz), e = max(s, clamp_ptr(rowptr[r + 1], nnz));
        uint64_t lo = 0, hi = cover - 1;
        if (!whole) {
            // the row's line span (max of ~line gives the minimum)
            uint32_t h = 0, nl = 0;
            for (uint32_t k = s + threadIdx.x; k < e; k += kBigThreads) {
                const uint32_t v = (uint32_t)col[k];
                if (v >= n_cols) {
                    flag_range_error(flag);
                    continue;
                }
                h = max(h, v >> shift);
                nl = max(nl, ~(v >> shift));
            }
            hi = block_reduce<kBigThreads>(h, OpMax{}, red);
            lo = ~block_reduce<kBigThreads>(nl, OpMax{}, red);
        }
        uint32_t fresh = 0;
        for (uint64_t p0 = lo; p0 <= hi; p0 += cover) {
            const uint64_t span = min(hi - p0 + 1, cover);
            const uint32_t nw = (uint32_t)((span + 31) / 32);
            for (uint32_t w = threadIdx.x; w < nw; w += kBigThreads) bm[w] = 0;
            __syncthreads();
            for (uint32_t k = s + threadIdx.x; k < e; k += kBigThreads) {
                const uint32_t v = (uint32_t)col[k];
                if (v >= n_cols) {
                    if (whole) flag_range_error(flag);
                    continue;
                }
                const uint64_t l = v >> shift;
                if (l < p0 || l >= p0 + span) continue;
                const uint32_t b = (uint32_t)(l - p0);
                const uint32_t bit = 1u << (b & 31);
                fresh += (atomicOr(&bm[b >> 5], bit) & bit) == 0;
            }
            __syncthreads();
        }
        const uint32_t nd = block_reduce<kBigThreads>(fresh, OpSum{}, red);
        if (threadIdx.x == 0) nd_out[r] = nd;
    }
}

// Part p of the rows: the sum of nd/|N(v)| over its non-empty rows (each
// thread in row order, then a fixed tree) and their number.
__global__ __launch_bounds__(kThreads) void k_nbr_reduce(const int32_t *__restrict__ rowptr, uint32_t n_rows,
                                                         uint32_t nnz, uint32_t per_part,
                                                         const uint32_t *__restrict__ nd,
                                                         double *__restrict__ part_sum,
                                                         uint32_t *__restrict__ part_cnt) {
    __shared__ double ls[kThreads];
    __shared__ uint32_t lc[kThreads / kWave];
    const uint32_t r0 = blockIdx.x * per_part;
    const uint32_t r1 = min(n_rows, r0 + per_part);
    double acc = 0.0;
    uint32_t cnt = 0;
    uint32_t r = r0 + threadIdx.x;
    // four rows' loads in flight at a time; the sum still runs in row order
    for (; r + 3 * kThreads < r1; r += 4 * kThreads) {
        int32_t ps[4], pe[4];
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ps[u] = rowptr[r + u * kThreads];
            pe[u] = rowptr[r + u * kThreads + 1];
            v[u] = nd[r + u * kThreads];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t s = clamp_ptr(ps[u], nnz), e = clamp_ptr(pe[u], nnz);
            if (e <= s) continue;
            acc += (double)v[u] / (double)(e - s);
            ++cnt;
        }
    }
    for (; r < r1; r += kThreads) {
        const uint32_t s = clamp_ptr(rowptr[r], nnz), e = clamp_ptr(rowptr[r + 1], nnz);
        if (e <= s) continue;
        acc += (double)nd[r] / (double)(e - s);
        ++cnt;
    }
    ls[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) ls[threadIdx.x] += ls[threadIdx.x + h];
        __syncthreads();
    }
    cnt = block_reduce<kThreads>(cnt, OpSum{}, lc);
    if (threadIdx.x == 0) {
        part_sum[blockIdx.x] = ls[0];
        part_cnt[blockIdx.x] = cnt;
    }
}

__global__ __launch_bounds__(kParts) void k_nbr_final(const double *__restrict__ part_sum,
                                                      const uint32_t *__restrict__ part_cnt, uint32_t parts,
                                                      uint32_t n_rows, double *__restrict__ result) {
    __shared__ double ls[kParts];
    __shared__ uint32_t lc[kParts / kWave];
    const uint32_t t = threadIdx.x;
    ls[t] = t < parts ? part_sum[t] : 0.0;
    const uint32_t c = t < parts ? part_cnt[t] : 0u;
    __syncthreads();
    for (uint32_t h = kParts / 2; h > 0; h >>= 1) {
        if (t < h) ls[t] += ls[t + h];
        __syncthreads();
    }
    const uint32_t total = block_reduce<kParts>(c, OpSum{}, lc);
    if (t == 0) {
        // the sum, the rows it covers, and NBR over all rows and over the
        // non-empty rows (0 where there is no row to average over)
        result[0] = ls[0];
        result[1] = (double)total;
        result[2] = n_rows ? ls[0] / (double)n_rows : 0.0;
        result[3] = total ? ls[0] / (double)total : 0.0;
    }
}

struct NbrLayout {
    uint32_t nchunk = 0, parts = 0, per_part = 0, max_big = 0, per_list = 0;
    uint2 *chunk = nullptr;
    uint32_t *nd = nullptr, *lists = nullptr, *list_count = nullptr, *part_cnt = nullptr;
    double *part_sum = nullptr;
    size_t bytes = 0;
};

NbrLayout nbr_layout(void *ws, int64_t n_rows, int64_t nnz) {
    NbrLayout L;
    L.nchunk = ceil_div((uint64_t)n_rows + (uint64_t)nnz, kChunkE);
    if (L.nchunk == 0) L.nchunk = 1;
    L.per_part = n_rows > 0 ? ceil_div((uint64_t)n_rows, kParts) : 1;
    L.parts = n_rows > 0 ? ceil_div((uint64_t)n_rows, L.per_part) : 0;
    L.max_big = (uint32_t)((uint64_t)nnz / (kSmall + 1) + 1);
    Carver c(ws);
    L.chunk = c.take<uint2>(L.nchunk + 1ull);
    L.nd = c.take<uint32_t>((size_t)n_rows);
    // a chunk holds at most kBigPerChunk rows longer than kSmall: their first
    // items lie more than kSmall + 1 apart
    L.per_list = (uint32_t)std::min<uint64_t>(L.max_big, (uint64_t)kBigPerChunk * ceil_div(L.nchunk, kLists));
    L.lists = c.take<uint32_t>(2ull * kLists * L.per_list);  // class 0 (kSmall < d <= kMid), then class 1
    L.list_count = c.take<uint32_t>(2 * kLists);
    L.part_sum = c.take<double>(kParts);
    L.part_cnt = c.take<uint32_t>(kParts);
    L.bytes = c.bytes();
    return L;
}

}  // namespace
}  // namespace boba

using namespace boba;

extern "C" size_t boba_nbr_workspace(int64_t n_rows, int64_t nnz) {
    if (n_rows < 0 || nnz < 0) return 0;
    return nbr_layout(nullptr, n_rows, nnz).bytes;
}

extern "C" boba_status boba_nbr(const int32_t *rowptr, const int32_t *col, int64_t n_rows, int64_t n_cols,
                                int64_t nnz, int32_t line_ids, int32_t *lines_per_row, double *result, void *ws,
                                size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(BOBA_ERR_ARG, "boba_nbr: negative size");
    if (n_rows >= (1ll << 31) || n_cols >= (1ll << 31) || nnz >= (1ll << 31))
        return fail(BOBA_ERR_OVERFLOW, "boba_nbr: sizes must be < 2^31");
    if (line_ids < 1 || line_ids > (1 << 30) || (line_ids & (line_ids - 1)))
        return fail(BOBA_ERR_ARG, "boba_nbr: line_ids must be a power of two in [1, 2^30] (got %d)", line_ids);
    if (!result) return fail(BOBA_ERR_ARG, "boba_nbr: result is NULL");
    if (n_rows > 0 && !rowptr) return fail(BOBA_ERR_ARG, "boba_nbr: rowptr is NULL");
    if (nnz > 0 && !col) return fail(BOBA_ERR_ARG, "boba_nbr: col is NULL");
    const size_t need = boba_nbr_workspace(n_rows, nnz);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "boba_nbr: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)", need,
                    ws_bytes, ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    const NbrLayout L = nbr_layout(ws, n_rows, nnz);
    const uint32_t nr = (uint32_t)n_rows, nc = (uint32_t)n_cols, ne = (uint32_t)nnz;
    const uint32_t shift = (uint32_t)__builtin_ctz((unsigned)line_ids);
    uint32_t *nd = lines_per_row ? (uint32_t *)lines_per_row : L.nd;
    if (nr > 0) {
        BOBA_LAUNCH("nbr_split", k_nbr_split, dim3(ceil_div(L.nchunk + 1ull, kThreads)), dim3(kThreads), stream,
                    rowptr, nr, ne, L.nchunk, L.chunk, L.list_count);
        BOBA_LAUNCH("nbr_chunk", k_nbr_chunk, dim3(L.nchunk), dim3(kThreads), stream, rowptr, col, nc, ne, shift,
                    (const uint2 *)L.chunk, nd, L.lists, L.per_list, L.list_count, flag);
        const uint32_t grid_mid = std::max<uint64_t>(1, std::min<uint64_t>(L.max_big, (uint64_t)device_cus() * 8));
        BOBA_LAUNCH("nbr_mid", k_nbr_mid, dim3(grid_mid), dim3(kMidThreads), stream, rowptr, col, nc, ne, shift,
                    (const uint32_t *)L.lists, L.per_list, (const uint32_t *)L.list_count, nd, flag);
        // a bitmap over all lines when they fit in 128 KB (2^20 lines), so
        // that smaller ones let two or more workgroups share a CU
        const uint64_t nlines = ((uint64_t)nc + (uint64_t)line_ids - 1) >> shift;
        const bool whole = nlines <= 32ull * kBitmapWords;
        const uint32_t words = whole ? (uint32_t)std::max<uint64_t>(1, (nlines + 31) / 32) : kBitmapWords;
        const uint32_t per_cu = std::max<uint32_t>(1, std::min<uint32_t>(2, (uint32_t)(147456 / (4ull * words))));
        const uint32_t grid_big = std::min<uint64_t>(L.max_big, (uint64_t)device_cus() * per_cu);
        const int tok = timing_begin("nbr_big", stream);
        hipLaunchKernelGGL(k_nbr_big, dim3(grid_big), dim3(kBigThreads), 4ull * words, stream, rowptr, col, nc, ne,
                           shift, words, whole, (const uint32_t *)L.lists + (size_t)kLists * L.per_list,
                           L.per_list, (const uint32_t *)L.list_count + kLists, nd, flag);
        timing_end(tok, stream);
        if (boba_status e = check_launch("nbr_big")) return e;
        BOBA_LAUNCH("nbr_reduce", k_nbr_reduce, dim3(L.parts), dim3(kThreads), stream, rowptr, nr, ne, L.per_part,
                    (const uint32_t *)nd, L.part_sum, L.part_cnt);
    }
    BOBA_LAUNCH("nbr_final", k_nbr_final, dim3(1), dim3(kParts), stream, (const double *)L.part_sum,
                (const uint32_t *)L.part_cnt, L.parts, nr, result);
    return BOBA_OK;
}

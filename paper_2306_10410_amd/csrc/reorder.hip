// BOBA reordering (Sec. 4.4, Algorithm 2 with AtomicMin) and edge relabelling.
//
// boba_reorder computes, for every vertex v, r[v] = its first position in the
// flattened edge list S = I ++ J (Algorithm 2, the lines that write r, with an
// exact minimum), then perm[v] = the rank of key(v) = r[v] among all keys, where
// a vertex that never occurs has key 2m + v (it follows all others in
// increasing ID).  Two paths:
//   bucketed (n <= 2^25; the normal case)
//     split     per tile of S, records {offset, v mod 2^15} sorted by vertex
//               bucket (v >> 15) in LDS, written segment by segment
//     min       per (bucket, slice): the bucket's r in LDS, every record folded
//               in with an LDS minimum
//     rank      keys grouped by key block, each block ranked with an LDS
//               bitmap and prefix popcounts (ParMapKeys without a hash table)
//   direct (otherwise)
//     init      r[v] <- inf, bitmap <- 0
//     scatter   r[S[i]] <- min(r[S[i]], i), one global atomic per new position
//     mark      set bit key(v) in a bitmap over [0, 2m + n)
//     scan      prefix popcount of the bitmap words
//     rank      perm[v] = number of set bits before key(v)
//   The direct path's bitmap holds, per 32 positions, {bits, exclusive prefix
//   popcount} as one uint2 so that rank needs one 8-byte load per vertex.
#include <mutex>

#include "internal.h"
#include "scan.h"

namespace boba {
namespace {

constexpr int kBlock = 256;
constexpr int kScatterChunks = 4;  // int4 chunks per thread per tile
constexpr uint32_t kScatterTile = kBlock * kScatterChunks;  // chunks per workgroup

__global__ __launch_bounds__(kBlock) void k_reorder_init(uint32_t *__restrict__ r, uint32_t n,
                                                         uint2 *__restrict__ W, uint32_t nw) {
    const uint32_t stride = gridDim.x * kBlock;
    const uint32_t total = n > nw ? n : nw;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < total; i += stride) {
        if (i < n) r[i] = kInf;
        if (i < nw) W[i] = make_uint2(0u, 0u);
    }
}

// r[v] <- min(r[v], pos), skipping the atomic when a (possibly stale) read
// already shows a smaller position: r only decreases, so a stale value is
// never smaller than the current one and the skip is always safe.  All probe
// reads of a thread are issued before its first atomic so that they overlap.
// RACY: a plain store after the comparison, the non-atomic write of the
// paper's GPU kernel (Sec. 4.4): r[v] ends up at one of v's positions, not
// necessarily the first.
template <bool RACY>
__device__ __forceinline__ void lower(uint32_t *r, uint32_t pos) {
    if (RACY) *r = pos;
    else atomicMin(r, pos);
}

template <bool RACY, int K>
__device__ __forceinline__ void visit_all(uint32_t *__restrict__ r, const int32_t (&v)[K], const uint32_t (&pos)[K],
                                          const bool (&live)[K], uint32_t n, int32_t *flag) {
    // Unconditional loads (index clamped to 0 when unused) keep the probes in
    // straight-line code, so they are all in flight together.
    uint32_t cur[K];
#pragma unroll
    for (int q = 0; q < K; ++q) cur[q] = r[(live[q] && (uint32_t)v[q] < n) ? (uint32_t)v[q] : 0u];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        if (!live[q]) continue;
        if ((uint32_t)v[q] < n) {
            if (pos[q] < cur[q]) lower<RACY>(&r[v[q]], pos[q]);
        } else {
            flag_range_error(flag);
        }
    }
}

template <bool RACY>
__device__ __forceinline__ void visit(uint32_t *__restrict__ r, int32_t v, uint32_t pos, uint32_t n,
                                      int32_t *flag) {
    if ((uint32_t)v < n) {
        if (pos < r[v]) lower<RACY>(&r[v], pos);
    } else {
        flag_range_error(flag);
    }
}

// Chunk c < m4 covers src[4c .. 4c+3]; chunk c >= m4 covers dst[4(c-m4) .. +3].
template <bool INTERLEAVED, bool RACY>
__global__ __launch_bounds__(kBlock) void k_scatter_min_vec(const v4i *__restrict__ src4,
                                                            const v4i *__restrict__ dst4, uint32_t m4,
                                                            uint32_t m, uint32_t n, uint32_t *__restrict__ r,
                                                            int32_t *flag) {
    const uint32_t base = blockIdx.x * kScatterTile + threadIdx.x;
    const uint32_t nchunks = 2 * m4;
    constexpr int K = 4 * kScatterChunks;
    int32_t v[K];
    uint32_t pos[K];
    bool live[K];
#pragma unroll
    for (int u = 0; u < kScatterChunks; ++u) {
        const uint32_t c = base + u * kBlock;
        const bool ok = c < nchunks;
        const uint32_t cc = ok ? c : 0u;
        const v4i x = __builtin_nontemporal_load(cc < m4 ? &src4[cc] : &dst4[cc - m4]);
        const bool is_dst = c >= m4;
        const uint32_t k = 4 * (is_dst ? c - m4 : c);
        const uint32_t p0 = INTERLEAVED ? 2 * k + (is_dst ? 1 : 0) : (is_dst ? m + k : k);
        const uint32_t step = INTERLEAVED ? 2 : 1;
        v[4 * u + 0] = x.x;
        v[4 * u + 1] = x.y;
        v[4 * u + 2] = x.z;
        v[4 * u + 3] = x.w;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pos[4 * u + q] = p0 + q * step;
            live[4 * u + q] = ok;
        }
    }
    visit_all<RACY>(r, v, pos, live, n, flag);
}

// Edges k in [k0, m): both endpoints, scalar loads (tails and unaligned input).
template <bool INTERLEAVED, bool RACY>
__global__ __launch_bounds__(kBlock) void k_scatter_min_scalar(const int32_t *__restrict__ src,
                                                               const int32_t *__restrict__ dst, uint32_t k0,
                                                               uint32_t m, uint32_t n, uint32_t *__restrict__ r,
                                                               int32_t *flag) {
    const uint64_t cnt = m - k0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t t = blockIdx.x * kBlock + threadIdx.x; t < 2 * cnt; t += stride) {
        const bool is_dst = t >= cnt;
        const uint32_t k = k0 + (uint32_t)(is_dst ? t - cnt : t);
        const uint32_t pos = INTERLEAVED ? 2 * k + (is_dst ? 1 : 0) : (is_dst ? m + k : k);
        visit<RACY>(r, is_dst ? dst[k] : src[k], pos, n, flag);
    }
}

__device__ __forceinline__ uint32_t key_of(const uint32_t *__restrict__ r, uint32_t v, uint32_t tail) {
    uint32_t p = r[v];
    return p == kInf ? tail + v : p;
}

__global__ __launch_bounds__(kBlock) void k_mark(const uint32_t *__restrict__ r, uint32_t n, uint32_t tail,
                                                 uint2 *__restrict__ W) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        uint32_t p = key_of(r, v, tail);
        atomicOr(&W[p >> 5].x, 1u << (p & 31));
    }
}

struct LoadPopc {
    const uint2 *W;
    __device__ uint32_t operator()(uint32_t i) const { return __popc(W[i].x); }
};
struct StorePrefix {
    uint2 *W;
    __device__ void operator()(uint32_t i, uint32_t v) const { W[i].y = v; }
};

__global__ __launch_bounds__(kBlock) void k_rank(const uint32_t *__restrict__ r, uint32_t n, uint32_t tail,
                                                 const uint2 *__restrict__ W, int32_t *__restrict__ perm,
                                                 int32_t *__restrict__ order) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        uint32_t p = key_of(r, v, tail);
        uint2 w = W[p >> 5];
        uint32_t k = w.y + __popc(w.x & ((1u << (p & 31)) - 1u));
        perm[v] = (int32_t)k;
        if (order) order[k] = (int32_t)v;
    }
}

// ------------------------------------------------------------------ relabel
__device__ __forceinline__ int32_t lookup(const int32_t *__restrict__ perm, int32_t v, uint32_t n,
                                          int32_t *flag) {
    if ((uint32_t)v < n) return perm[v];
    flag_range_error(flag);
    return v;
}

constexpr int kRelabelChunks = 4;
constexpr uint32_t kRelabelTile = kBlock * kRelabelChunks;

__global__ __launch_bounds__(kBlock) void k_relabel_vec(const v4i *src4, const v4i *dst4, uint32_t m4,
                                                        const int32_t *__restrict__ perm, uint32_t n,
                                                        v4i *so4, v4i *do4, int32_t *flag) {
    const uint32_t base = blockIdx.x * kRelabelTile + threadIdx.x;
    const uint32_t nchunks = 2 * m4;
    v4i v[kRelabelChunks];
#pragma unroll
    for (int u = 0; u < kRelabelChunks; ++u) {
        const uint32_t c = base + u * kBlock;
        const uint32_t cc = c < nchunks ? c : 0u;
        v[u] = __builtin_nontemporal_load(cc < m4 ? &src4[cc] : &dst4[cc - m4]);
    }
    // all gathers before any store, in straight-line code, so they overlap
    bool bad = false;
#pragma unroll
    for (int u = 0; u < kRelabelChunks; ++u) {
        v4i g;
        g.x = perm[(uint32_t)v[u].x < n ? (uint32_t)v[u].x : 0u];
        g.y = perm[(uint32_t)v[u].y < n ? (uint32_t)v[u].y : 0u];
        g.z = perm[(uint32_t)v[u].z < n ? (uint32_t)v[u].z : 0u];
        g.w = perm[(uint32_t)v[u].w < n ? (uint32_t)v[u].w : 0u];
        bad |= (uint32_t)v[u].x >= n || (uint32_t)v[u].y >= n || (uint32_t)v[u].z >= n || (uint32_t)v[u].w >= n;
        v[u] = g;
    }
#pragma unroll
    for (int u = 0; u < kRelabelChunks; ++u) {
        const uint32_t c = base + u * kBlock;
        if (c < nchunks) __builtin_nontemporal_store(v[u], c < m4 ? &so4[c] : &do4[c - m4]);
    }
    if (bad) flag_range_error(flag);
}

__global__ __launch_bounds__(kBlock) void k_relabel_scalar(const int32_t *src, const int32_t *dst, uint32_t k0,
                                                           uint32_t m, const int32_t *__restrict__ perm,
                                                           uint32_t n, int32_t *so, int32_t *dso, int32_t *flag) {
    const uint64_t cnt = m - k0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t t = blockIdx.x * kBlock + threadIdx.x; t < 2 * cnt; t += stride) {
        if (t < cnt) {
            uint32_t k = k0 + (uint32_t)t;
            so[k] = lookup(perm, src[k], n, flag);
        } else {
            uint32_t k = k0 + (uint32_t)(t - cnt);
            dso[k] = lookup(perm, dst[k], n, flag);
        }
    }
}


// ------------------------------------------------- small graphs, one launch
// A graph of at most kSmallN vertices and kSmallPositions positions is
// reordered (and, if asked, relabelled) by one workgroup in one launch:
// first positions by LDS atomic min over S, every vertex's key (its first
// position, or 2m + v when it never occurs) marked in a position bitmap in the
// workspace (small enough to stay in L2), prefix popcounts of the bitmap words
// by the workgroup, ranks, and the relabel by LDS gathers of the ranks.  The
// many-kernel path spends most of its time between launches at these sizes.
constexpr int kSmallThreads = 1024;
constexpr uint32_t kSmallN = 32768;              // r in LDS: 128 KB
constexpr uint64_t kSmallPositions = 1ull << 21; // 2m + n: at most 8 MB of edges
constexpr int kSmallU = 8;                       // loads in flight per thread and array
constexpr int kSmallScanPer = 4;                 // bitmap words per thread per scan round

inline bool small_graph(int64_t n, int64_t m) {
    return n <= kSmallN && 2 * (uint64_t)m + (uint64_t)n <= kSmallPositions;
}

// Coherent loads of the bitmap (other threads wrote it through L2).
__device__ __forceinline__ uint32_t ld_l2(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint2 ld_l2_2(const uint2 *p) {
    const uint64_t v = __hip_atomic_load((const uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

template <bool INTERLEAVED, bool RACY>
__global__ __launch_bounds__(kSmallThreads) void k_small_reorder(const int32_t *src, const int32_t *dst, uint32_t m,
                                                                  uint32_t n, uint2 *__restrict__ W, uint32_t nw,
                                                                  int32_t *__restrict__ perm,
                                                                  int32_t *__restrict__ order, int32_t *so,
                                                                  int32_t *dso, int32_t *flag) {
    __shared__ uint32_t lr[kSmallN];
    __shared__ uint32_t stage[kSmallThreads * kSmallScanPer];
    __shared__ uint32_t scan_lds[kSmallThreads / kWave];
    const uint32_t tid = threadIdx.x;
    for (uint32_t v = tid; v < n; v += kSmallThreads) lr[v] = kInf;
    for (uint32_t i = tid; i < nw; i += kSmallThreads) W[i] = make_uint2(0u, 0u);
    __syncthreads();
    bool bad = false;
    // first positions: a round's loads are all issued before its LDS atomics
    for (uint32_t k0 = tid; k0 < m; k0 += kSmallThreads * kSmallU) {
        int32_t a[kSmallU], b[kSmallU];
#pragma unroll
        for (int j = 0; j < kSmallU; ++j) {
            const uint32_t k = min(k0 + j * kSmallThreads, m - 1);
            a[j] = src[k];
            b[j] = dst[k];
        }
#pragma unroll
        for (int j = 0; j < kSmallU; ++j) {
            const uint32_t k = k0 + j * kSmallThreads;
            if (k >= m) break;
            const uint32_t pa = INTERLEAVED ? 2 * k : k, pb = INTERLEAVED ? 2 * k + 1 : m + k;
            if ((uint32_t)a[j] < n) {
                if (pa < lr[a[j]]) lower<RACY>(&lr[a[j]], pa);
            } else {
                bad = true;
            }
            if ((uint32_t)b[j] < n) {
                if (pb < lr[b[j]]) lower<RACY>(&lr[b[j]], pb);
            } else {
                bad = true;
            }
        }
    }
    __syncthreads();
    // keys into the bitmap (never-occurring vertices after every position)
    for (uint32_t v = tid; v < n; v += kSmallThreads) {
        uint32_t p = lr[v];
        if (p == kInf) p = 2 * m + v;
        lr[v] = p;
        atomicOr(&W[p >> 5].x, 1u << (p & 31));
    }
    __syncthreads();
    // W[i].y = keys in words [0, i): rounds of kSmallThreads * kSmallScanPer
    // words, each thread a run of kSmallScanPer consecutive words
    uint32_t carry = 0;
    for (uint32_t w0 = 0; w0 < nw; w0 += kSmallThreads * kSmallScanPer) {
#pragma unroll
        for (int j = 0; j < kSmallScanPer; ++j) {
            const uint32_t i = w0 + j * kSmallThreads + tid;
            stage[j * kSmallThreads + tid] = i < nw ? ld_l2(&W[i].x) : 0u;
        }
        __syncthreads();
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < kSmallScanPer; ++j) cnt += __popc(stage[tid * kSmallScanPer + j]);
        uint32_t total;
        uint32_t run = carry + block_exclusive_scan<kSmallThreads>(cnt, OpSum{}, scan_lds, total);
#pragma unroll
        for (int j = 0; j < kSmallScanPer; ++j) {
            const uint32_t bits = stage[tid * kSmallScanPer + j];
            stage[tid * kSmallScanPer + j] = run;
            run += __popc(bits);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSmallScanPer; ++j) {
            const uint32_t i = w0 + j * kSmallThreads + tid;
            if (i < nw) W[i].y = stage[j * kSmallThreads + tid];
        }
        carry += total;
        __syncthreads();
    }
    // ranks; each thread rewrites only its own vertices' LDS entries
    for (uint32_t v = tid; v < n; v += kSmallThreads) {
        const uint32_t p = lr[v];
        const uint2 w = ld_l2_2(&W[p >> 5]);
        const uint32_t k = w.y + __popc(w.x & ((1u << (p & 31)) - 1u));
        perm[v] = (int32_t)k;
        if (order) order[k] = (int32_t)v;
        lr[v] = k;
    }
    if (so) {
        __syncthreads();
        for (uint32_t k0 = tid; k0 < m; k0 += kSmallThreads * kSmallU) {
            int32_t a[kSmallU], b[kSmallU];
#pragma unroll
            for (int j = 0; j < kSmallU; ++j) {
                const uint32_t k = min(k0 + j * kSmallThreads, m - 1);
                a[j] = src[k];
                b[j] = dst[k];
            }
#pragma unroll
            for (int j = 0; j < kSmallU; ++j) {
                const uint32_t k = k0 + j * kSmallThreads;
                if (k >= m) break;
                // an out-of-range ID (flagged above) is passed through
                so[k] = (uint32_t)a[j] < n ? (int32_t)lr[a[j]] : a[j];
                dso[k] = (uint32_t)b[j] < n ? (int32_t)lr[b[j]] : b[j];
            }
        }
    }
    if (bad) flag_range_error(flag);
}

// ------------------------------------------------------- bucketed scatter-min
// The direct scatter above issues one random 4-byte read of r per position;
// for a 64 MB r those reads run at HBM random-access speed.  The bucketed path
// never touches r per position:
//   split     each workgroup takes a tile of kTileT consecutive elements of
//             one half (src or dst), groups them by vertex bucket
//             v >> kVBits in LDS (counting sort, bucket segments padded to
//             4 records) and writes the tile's records + segment offsets.
//             A record packs (element offset in tile) << kVBits | (v mod W).
//   transpose the per-tile offsets to bucket-major order.
//   bucket    one workgroup per (bucket, slice of tiles) keeps the bucket's
//             2^kVBits r values in LDS and folds every record in with an LDS
//             atomic min; the slice's minima are written out coalesced.
// Slices (several workgroups per bucket) keep the GPU busy when there are few
// buckets; their partial minima are merged by the mark kernel.
constexpr int kSplitThreads = 1024;
constexpr int kSplitPer = 32;                                   // elements per thread
constexpr uint32_t kTileT = kSplitThreads * kSplitPer;          // 32768 elements per tile
constexpr int kVBits = 15;
constexpr uint32_t kBucketW = 1u << kVBits;                     // vertices per bucket
constexpr uint32_t kMaxBuckets = 1024;                          // LDS budget of split
constexpr uint32_t kSentinel = 0xFFFFFFFFu;
constexpr int kMinThreads = 1024;
constexpr int kMinGroup = 16;                                   // segments in flight per wave
constexpr uint32_t kLongMax = 512;                              // long segments a workgroup can queue
constexpr uint32_t kChunk = 16 * kWave;                         // records per wave step, 8 loads of 2 per lane
constexpr uint32_t kInlineMax = 2 * kChunk;                     // longer segment rests go to the queue

// Queue of segment rests longer than kInlineMax records: an entry is {tile,
// first record, end, first chunk}; one 64-bit LDS atomic hands out the slot
// (high word) and the chunks (low word) together, so chunk bases grow with
// the slot and a wave can walk the entries in order.
struct LongQueue {
    uint32_t e[kLongMax][4];
    unsigned long long top;
};

// Pushes the rest [k1, e1) of tile's segment; false when the queue is full
// (the caller then works through it itself).  Wave-uniform arguments.
__device__ inline bool long_push(LongQueue &q, uint32_t tile, uint32_t k1, uint32_t e1, uint32_t lane) {
    unsigned long long t = 0;
    if (lane == 0) t = atomicAdd(&q.top, (1ull << 32) | ((e1 - k1 + kChunk - 1) / kChunk));
    t = __shfl(t, 0, kWave);
    const uint32_t slot = (uint32_t)(t >> 32);
    if (slot >= kLongMax) return false;
    if (lane == 0) {
        q.e[slot][0] = tile;
        q.e[slot][1] = k1;
        q.e[slot][2] = e1;
        q.e[slot][3] = (uint32_t)t;
    }
    return true;
}

// Calls f(tile, first record, end) for every chunk of the queued rests,
// chunks dealt round-robin over the waves.  After a barrier.
template <class F>
__device__ inline void long_drain(const LongQueue &q, uint32_t wave, uint32_t nwave, F &&f) {
    const uint32_t nq = min((uint32_t)(q.top >> 32), kLongMax);
    if (nq == 0) return;
    const uint32_t units = q.e[nq - 1][3] + (q.e[nq - 1][2] - q.e[nq - 1][1] + kChunk - 1) / kChunk;
    uint32_t i = 0;
    for (uint32_t u = wave; u < units; u += nwave) {
        while (i + 1 < nq && q.e[i + 1][3] <= u) ++i;
        f(q.e[i][0], q.e[i][1] + (u - q.e[i][3]) * kChunk, q.e[i][2]);
    }
}

inline uint32_t split_region(uint32_t nb) { return (kTileT + 3 * nb + 3) & ~3u; }

// Loads tile t (32 elements per thread, element k0 + j*4096 + 4*tid + q, so
// that every load instruction is coalesced; 16-byte loads when src and dst
// are 16-byte aligned).  Past the end: -1.
__device__ __forceinline__ void split_load(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                                           uint32_t m, uint32_t tiles_half, uint32_t t, bool vec,
                                           int32_t (&v)[kSplitPer]) {
    const bool h = t >= tiles_half;
    const uint32_t k0 = (t - (h ? tiles_half : 0u)) * kTileT;
    const int32_t *a = h ? dst : src;
#pragma unroll
    for (int j = 0; j < kSplitPer / 4; ++j) {
        const uint32_t e = k0 + j * (4 * kSplitThreads) + 4 * threadIdx.x;
        if (vec && e + 3 < m) {
            const v4i x = __builtin_nontemporal_load((const v4i *)(a + e));
            v[4 * j] = x.x;
            v[4 * j + 1] = x.y;
            v[4 * j + 2] = x.z;
            v[4 * j + 3] = x.w;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[4 * j + q] = e + q < m ? a[e + q] : -1;
        }
    }
}

// Persistent: workgroup g takes a contiguous run of tiles.  The next tile's
// loads are issued right after the current tile has been sorted into LDS, so
// they are in flight while the current tile's records are written out.
__global__ __launch_bounds__(kSplitThreads) void k_bucket_split(const int32_t *__restrict__ src,
                                                                 const int32_t *__restrict__ dst, uint32_t m,
                                                                 uint32_t tiles_half, uint32_t n, uint32_t nb,
                                                                 uint32_t region, bool vec,
                                                                 uint32_t *__restrict__ recs,
                                                                 uint32_t *__restrict__ tile_off, int32_t *flag) {
    __shared__ __align__(16) uint32_t stage[kTileT + 3 * kMaxBuckets];
    __shared__ uint32_t hist[kMaxBuckets];
    __shared__ uint32_t cur[kMaxBuckets];
    __shared__ uint32_t scan_lds[kSplitThreads / kWave];
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = 2 * tiles_half;
    const uint32_t per = (nt + gridDim.x - 1) / gridDim.x;
    const uint32_t t_begin = blockIdx.x * per;
    const uint32_t t_end = min(nt, t_begin + per);
    int32_t v[kSplitPer];
    if (t_begin < t_end) split_load(src, dst, m, tiles_half, t_begin, vec, v);
    bool bad = false;
    for (uint32_t t = t_begin; t < t_end; ++t) {
        const bool h = t >= tiles_half;
        const uint32_t k0 = (t - (h ? tiles_half : 0u)) * kTileT;
        for (uint32_t i = tid; i < nb; i += kSplitThreads) hist[i] = 0;
        __syncthreads();
        // A wave's 256 consecutive elements of one step j often share a
        // bucket when the input is sorted (a bucket spans 32768 IDs); then one
        // atomic counts them all instead of 256 same-address LDS atomics.
        const uint32_t lane = tid & (kWave - 1);
        bool same[kSplitPer / 4];
#pragma unroll
        for (int j = 0; j < kSplitPer / 4; ++j) {
            bool all_ok = true;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t e = k0 + j * (4 * kSplitThreads) + 4 * tid + q;
                const int32_t x = v[4 * j + q];
                const bool ok = e < m && (uint32_t)x < n;
                if (e < m && !ok) {
                    bad = true;
                    v[4 * j + q] = -1;
                }
                all_ok = all_ok && ok;
            }
            const uint32_t b0 = (uint32_t)__shfl(v[4 * j], 0, kWave) >> kVBits;
            const bool mine = all_ok && ((uint32_t)v[4 * j] >> kVBits) == b0 &&
                              ((uint32_t)v[4 * j + 1] >> kVBits) == b0 && ((uint32_t)v[4 * j + 2] >> kVBits) == b0 &&
                              ((uint32_t)v[4 * j + 3] >> kVBits) == b0;
            same[j] = __ballot(mine) == ~0ull;
            if (same[j]) {
                if (lane == 0) atomicAdd(&hist[b0], 4u * kWave);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t x = v[4 * j + q];
                    if (x >= 0 && k0 + j * (4 * kSplitThreads) + 4 * tid + q < m)
                        atomicAdd(&hist[(uint32_t)x >> kVBits], 1u);
                }
            }
        }
        __syncthreads();

        const uint32_t c = tid < nb ? hist[tid] : 0u;
        const uint32_t pc = (c + 3) & ~3u;
        uint32_t total;
        const uint32_t start = block_exclusive_scan<kSplitThreads>(pc, OpSum{}, scan_lds, total);
        uint32_t *off = tile_off + (size_t)t * (nb + 1);
        if (tid < nb) {
            off[tid] = start;
            cur[tid] = start;
            for (uint32_t q = c; q < pc; ++q) stage[start + q] = kSentinel;
        }
        if (tid == 0) off[nb] = total;
        __syncthreads();

#pragma unroll
        for (int j = 0; j < kSplitPer / 4; ++j) {
            if (same[j]) {  // one bucket: 256 slots in element order
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&cur[(uint32_t)v[4 * j] >> kVBits], 4u * kWave);
                base = __shfl(base, 0, kWave) + 4 * lane;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t o = j * (4 * kSplitThreads) + 4 * tid + q;
                    stage[base + q] = (o << kVBits) | ((uint32_t)v[4 * j + q] & (kBucketW - 1));
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t x = v[4 * j + q];
                    if (x >= 0) {
                        const uint32_t o = j * (4 * kSplitThreads) + 4 * tid + q;
                        const uint32_t slot = atomicAdd(&cur[(uint32_t)x >> kVBits], 1u);
                        stage[slot] = (o << kVBits) | ((uint32_t)x & (kBucketW - 1));
                    }
                }
            }
        }
        __syncthreads();
        if (t + 1 < t_end) split_load(src, dst, m, tiles_half, t + 1, vec, v);
        v4u *out = (v4u *)(recs + (size_t)t * region);
        const v4u *st = (const v4u *)stage;
        for (uint32_t i = tid; i < total / 4; i += kSplitThreads) __builtin_nontemporal_store(st[i], &out[i]);
    }
    if (bad) flag_range_error(flag);
}

// out[c][r] = in[r][c] for an rows x cols matrix of uint32.
__global__ __launch_bounds__(256) void k_transpose(const uint32_t *__restrict__ in, uint32_t rows, uint32_t cols,
                                                   uint32_t *__restrict__ out) {
    __shared__ uint32_t tile[32][33];
    const uint32_t c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const uint32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (uint32_t y = ty; y < 32; y += 8) {
        const uint32_t r = r0 + y, c = c0 + tx;
        if (r < rows && c < cols) tile[y][tx] = in[(size_t)r * cols + c];
    }
    __syncthreads();
    for (uint32_t y = ty; y < 32; y += 8) {
        const uint32_t c = c0 + y, r = r0 + tx;
        if (r < rows && c < cols) out[(size_t)c * rows + r] = tile[tx][y];
    }
}

// Workgroup (bucket b, slice s) folds the records of tiles [s*tps, (s+1)*tps)
// into an LDS copy of r for vertices [b*W, (b+1)*W).  Element k of half h has
// position hbase[h] + stride * k.
template <bool RACY>
__global__ __launch_bounds__(kMinThreads) void k_bucket_min(const uint32_t *__restrict__ recs,
                                                            const uint32_t *__restrict__ off_t, uint32_t nt,
                                                            uint32_t tiles_half, uint32_t region, uint32_t nb,
                                                            uint32_t tps, uint32_t batch, uint32_t n,
                                                            uint32_t hbase1, uint32_t stride,
                                                            uint32_t *__restrict__ out) {
    __shared__ uint32_t lr[kBucketW];
    __shared__ LongQueue longq;
    const uint32_t b = blockIdx.x % nb;
    const uint32_t s = blockIdx.x / nb;
    const uint32_t t0 = s * tps;
    const uint32_t t1 = min(nt, t0 + tps);
    for (uint32_t i = threadIdx.x; i < kBucketW; i += kMinThreads) lr[i] = kInf;
    if (threadIdx.x == 0) longq.top = 0;
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    constexpr uint32_t NWAVE = kMinThreads / kWave;
    // Most records are not first occurrences (at RMAT-24 98% of positions):
    // a plain LDS read rejects them, and only a smaller position pays for an
    // atomic.  The read may be stale, but r only decreases, so a stale value
    // never rejects a record that would lower r.
    auto fold = [&](uint32_t rec, uint32_t pb) {
        if (rec == kSentinel) return;
        const uint32_t i = rec & (kBucketW - 1);
        const uint32_t p = pb + stride * (rec >> kVBits);
        if (p < lr[i]) lower<RACY>(&lr[i], p);
    };
    // records [kb, min(kb + kChunk, e1)) of a tile's segment, 8 loads in
    // flight per lane
    auto fold_chunk = [&](uint32_t tile, uint32_t kb, uint32_t e1) {
        const bool h = tile >= tiles_half;
        const uint32_t pb = (h ? hbase1 : 0u) + stride * ((tile - (h ? tiles_half : 0u)) * kTileT);
        uint2 xs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t k = kb + 2 * (u * kWave + lane);
            xs[u] = k < e1 ? *(const uint2 *)(recs + (size_t)tile * region + k) : make_uint2(kSentinel, kSentinel);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            fold(xs[u].x, pb);
            fold(xs[u].y, pb);
        }
    };
    const uint32_t *beg = off_t + (size_t)b * nt;
    const uint32_t *end = off_t + (size_t)(b + 1) * nt;
    // A wave takes `batch` (<= 64) tiles at a time: one coalesced load of
    // their segment bounds, then groups of kMinGroup segments with the next
    // group's loads issued before the current group is folded in.
    for (uint32_t tb = t0 + wave * batch; tb < t1; tb += NWAVE * batch) {
        const uint32_t cnt = min(batch, t1 - tb);
        const uint32_t my = tb + lane;
        const uint32_t sb = lane < cnt ? beg[my] : 0u;
        const uint32_t se = lane < cnt ? end[my] : 0u;
        const uint64_t longs = __ballot(se - sb > 2 * kWave);  // segments past one load per lane
        uint2 cur[kMinGroup], nxt[kMinGroup];
        auto load_group = [&](uint32_t g0, uint2 (&dst)[kMinGroup]) {
#pragma unroll
            for (int g = 0; g < kMinGroup; ++g) {
                const uint32_t gi = g0 + g;
                const uint32_t b0 = __shfl(sb, gi & (kWave - 1), kWave);
                const uint32_t e0 = __shfl(se, gi & (kWave - 1), kWave);
                const uint32_t k = b0 + 2 * lane;
                dst[g] = (gi < cnt && k < e0) ? *(const uint2 *)(recs + (size_t)(tb + gi) * region + k)
                                              : make_uint2(kSentinel, kSentinel);
            }
        };
        load_group(0, cur);
        for (uint32_t g0 = 0; g0 < cnt; g0 += kMinGroup) {
            if (g0 + kMinGroup < cnt) load_group(g0 + kMinGroup, nxt);
#pragma unroll
            for (int g = 0; g < kMinGroup; ++g) {
                const uint32_t gi = g0 + g;
                const uint32_t tile = tb + gi;
                const bool h = tile >= tiles_half;
                const uint32_t pb = (h ? hbase1 : 0u) + stride * ((tile - (h ? tiles_half : 0u)) * kTileT);
                uint2 x = cur[g];
                fold(x.x, pb);
                fold(x.y, pb);
            }
            // the rest of a segment longer than 128 records: folded here up
            // to kInlineMax records, queued beyond (a sorted input makes whole
            // tiles one segment) and shared out over all waves at the end
            for (uint64_t mk = (longs >> g0) & ((1ull << kMinGroup) - 1); mk; mk &= mk - 1) {
                const uint32_t gi = g0 + (uint32_t)__builtin_ctzll(mk);
                const uint32_t e0 = __shfl(se, gi, kWave);
                const uint32_t k1 = __shfl(sb, gi, kWave) + 2 * kWave;
                if (e0 - k1 <= kInlineMax || !long_push(longq, tb + gi, k1, e0, lane))
                    for (uint32_t kb = k1; kb < e0; kb += kChunk) fold_chunk(tb + gi, kb, e0);
            }
#pragma unroll
            for (int g = 0; g < kMinGroup; ++g) cur[g] = nxt[g];
        }
    }
    __syncthreads();
    long_drain(longq, wave, NWAVE, fold_chunk);
    __syncthreads();
    uint32_t *o = out + (size_t)s * n + (size_t)b * kBucketW;
    const uint32_t cnt = min(kBucketW, n - b * kBucketW);
    for (uint32_t i = threadIdx.x; i < cnt; i += kMinThreads) o[i] = lr[i];
}


// -------------------------------------------------- fused relabel (bucketed)
// After the ranks are known, the split's records relabel the edges without a
// random perm gather per endpoint:
//   bucket_relabel  workgroup (bucket, slice): perm of the bucket's vertices in
//                   LDS; every record of the bucket gets its new ID, written
//                   to `vals` in the record's own slot (coalesced).
//   tile_unsplit    workgroup per tile: scatters the tile's new IDs back to
//                   element order in LDS, then writes them out coalesced.
__global__ __launch_bounds__(kMinThreads) void k_bucket_relabel(const uint32_t *__restrict__ recs,
                                                                const uint32_t *__restrict__ off_t, uint32_t nt,
                                                                uint32_t region, uint32_t nb, uint32_t tps,
                                                                uint32_t batch, uint32_t n,
                                                                const int32_t *__restrict__ perm,
                                                                uint32_t *__restrict__ vals) {
    __shared__ uint32_t lp[kBucketW];
    __shared__ LongQueue longq;
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);  // neighbouring buckets share lines
    const uint32_t b = w % nb;
    const uint32_t s = w / nb;
    const uint32_t t0 = s * tps;
    const uint32_t t1 = min(nt, t0 + tps);
    const uint32_t cntv = min(kBucketW, n - b * kBucketW);
    for (uint32_t i = threadIdx.x; i < cntv; i += kMinThreads) lp[i] = (uint32_t)perm[(size_t)b * kBucketW + i];
    if (threadIdx.x == 0) longq.top = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    constexpr uint32_t NWAVE = kMinThreads / kWave;
    // new IDs of records [kb, min(kb + kChunk, e1)) of a tile's segment, 8
    // loads in flight per lane
    auto relabel_chunk = [&](uint32_t tile, uint32_t kb, uint32_t e1) {
        uint2 xs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t kk = kb + 2 * (u * kWave + lane);
            xs[u] = kk < e1 ? *(const uint2 *)(recs + (size_t)tile * region + kk) : make_uint2(kSentinel, kSentinel);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t kk = kb + 2 * (u * kWave + lane);
            if (kk >= e1) continue;
            uint2 v;
            v.x = xs[u].x != kSentinel ? lp[xs[u].x & (kBucketW - 1)] : kSentinel;
            v.y = xs[u].y != kSentinel ? lp[xs[u].y & (kBucketW - 1)] : kSentinel;
            *(uint2 *)(vals + (size_t)tile * region + kk) = v;
        }
    };
    const uint32_t *beg = off_t + (size_t)b * nt;
    const uint32_t *end = off_t + (size_t)(b + 1) * nt;
    // same batching and software pipelining as bucket_min
    for (uint32_t tb = t0 + wave * batch; tb < t1; tb += NWAVE * batch) {
        const uint32_t cnt = min(batch, t1 - tb);
        const uint32_t sb = lane < cnt ? beg[tb + lane] : 0u;
        const uint32_t se = lane < cnt ? end[tb + lane] : 0u;
        const uint64_t longs = __ballot(se - sb > 2 * kWave);
        uint2 cur[kMinGroup], nxt[kMinGroup];
        auto load_group = [&](uint32_t g0, uint2 (&dst)[kMinGroup]) {
#pragma unroll
            for (int g = 0; g < kMinGroup; ++g) {
                const uint32_t gi = g0 + g;
                const uint32_t b0 = __shfl(sb, gi & (kWave - 1), kWave);
                const uint32_t e0 = __shfl(se, gi & (kWave - 1), kWave);
                const uint32_t k = b0 + 2 * lane;
                dst[g] = (gi < cnt && k < e0) ? *(const uint2 *)(recs + (size_t)(tb + gi) * region + k)
                                              : make_uint2(kSentinel, kSentinel);
            }
        };
        load_group(0, cur);
        for (uint32_t g0 = 0; g0 < cnt; g0 += kMinGroup) {
            if (g0 + kMinGroup < cnt) load_group(g0 + kMinGroup, nxt);
#pragma unroll
            for (int g = 0; g < kMinGroup; ++g) {
                const uint32_t gi = g0 + g;
                const uint32_t tile = tb + gi;
                const uint32_t e0 = __shfl(se, gi & (kWave - 1), kWave);
                uint32_t k = __shfl(sb, gi & (kWave - 1), kWave) + 2 * lane;
                const uint2 r2 = cur[g];
                if (gi < cnt && k < e0) {
                    uint2 v;
                    v.x = r2.x != kSentinel ? lp[r2.x & (kBucketW - 1)] : kSentinel;
                    v.y = r2.y != kSentinel ? lp[r2.y & (kBucketW - 1)] : kSentinel;
                    *(uint2 *)(vals + (size_t)tile * region + k) = v;
                }
            }
            // the rest of a segment longer than 128 records, as in
            // bucket_min: here up to kInlineMax records, else queued
            for (uint64_t mk = (longs >> g0) & ((1ull << kMinGroup) - 1); mk; mk &= mk - 1) {
                const uint32_t gi = g0 + (uint32_t)__builtin_ctzll(mk);
                const uint32_t e0 = __shfl(se, gi, kWave);
                const uint32_t k1 = __shfl(sb, gi, kWave) + 2 * kWave;
                if (e0 - k1 <= kInlineMax || !long_push(longq, tb + gi, k1, e0, lane))
                    for (uint32_t kb = k1; kb < e0; kb += kChunk) relabel_chunk(tb + gi, kb, e0);
            }
#pragma unroll
            for (int g = 0; g < kMinGroup; ++g) cur[g] = nxt[g];
        }
    }
    __syncthreads();
    long_drain(longq, wave, NWAVE, relabel_chunk);
}

__global__ __launch_bounds__(kSplitThreads) void k_tile_unsplit(const uint32_t *__restrict__ recs,
                                                                 const uint32_t *__restrict__ vals,
                                                                 const uint32_t *__restrict__ tile_off, uint32_t nb,
                                                                 uint32_t region, uint32_t m, uint32_t tiles_half,
                                                                 int32_t *__restrict__ src_out,
                                                                 int32_t *__restrict__ dst_out) {
    __shared__ __align__(16) uint32_t out[kTileT];
    // elements without a record (out-of-range IDs) come out as -1
    for (uint32_t i = threadIdx.x; i < kTileT; i += kSplitThreads) out[i] = kSentinel;
    __syncthreads();
    const uint32_t t = xcd_work_index(blockIdx.x, gridDim.x);
    const bool h = t >= tiles_half;
    const uint32_t k0 = (t - (h ? tiles_half : 0u)) * kTileT;
    const uint32_t total = tile_off[(size_t)t * (nb + 1) + nb];
    const v4u *r4 = (const v4u *)(recs + (size_t)t * region);
    const v4u *v4 = (const v4u *)(vals + (size_t)t * region);
    for (uint32_t i = threadIdx.x; i < total / 4; i += kSplitThreads) {
        const v4u r = __builtin_nontemporal_load(&r4[i]);
        const v4u v = __builtin_nontemporal_load(&v4[i]);
        if (r.x != kSentinel) out[r.x >> kVBits] = v.x;
        if (r.y != kSentinel) out[r.y >> kVBits] = v.y;
        if (r.z != kSentinel) out[r.z >> kVBits] = v.z;
        if (r.w != kSentinel) out[r.w >> kVBits] = v.w;
    }
    __syncthreads();
    int32_t *o = (h ? dst_out : src_out) + k0;
    const uint32_t count = min(kTileT, m - k0);
    if ((((uintptr_t)o) & 15u) == 0) {
        const v4i *o4s = (const v4i *)out;
        for (uint32_t i = threadIdx.x; i < count / 4; i += kSplitThreads)
            __builtin_nontemporal_store(o4s[i], (v4i *)o + i);
        for (uint32_t i = (count & ~3u) + threadIdx.x; i < count; i += kSplitThreads) o[i] = (int32_t)out[i];
    } else {
        for (uint32_t i = threadIdx.x; i < count; i += kSplitThreads) o[i] = (int32_t)out[i];
    }
}

// ------------------------------------------- ranking by key blocks (bucketed)
// After bucket_min, r holds every vertex's first position (kInf when it never
// occurs).  perm[v] counts the vertices with a smaller key (key = r, or 2m + v
// in the tail).  Keys below 2m are grouped into key blocks of 2^kbits
// positions (about 4096 blocks); the isolated vertices form one extra block
// after them.  The ranking's vertex buckets ("rank buckets", 2^rbits vertices,
// rbits <= kVBits) are its own: narrower than the split's when the graph has
// few split buckets, so that these kernels still spread over the GPU.
//   rank_count    per rank bucket: its vertices per key block (LDS counters),
//                 stored bucket-major; with several bucket_min slices it
//                 also writes the merged minimum back to slice 0
//   scan          transposed to block-major, exclusive scan: where bucket b's
//                 entries of key block k start in the entry list E (and how
//                 many keys precede the block); transposed back for the
//                 per-bucket kernels
//   rank_scatter  per rank bucket: {r, v} of every occurring vertex into E
//   rank_block    per key block: its keys as an LDS bitmap with prefix
//                 popcounts; rank = keys in earlier blocks + keys before it in
//                 the block; writes order[rank] = v and the rank beside E
//   rank_perm     per rank bucket: the ranks back into an LDS perm slice;
//                 isolated vertices take the tail ranks in increasing ID
// Every step streams or works in LDS: no device-wide random atomics.
constexpr uint32_t kMinKeyBits = 15;
constexpr uint32_t kPermChunk = 1024;  // key blocks rank_perm takes at a time (= its threads)
constexpr uint32_t kMaxKeyBits = 18;                            // rank_block LDS <= 48 KB
constexpr uint32_t kTargetKeyBlocks = 4096;                    // bounds a key block's entries
constexpr uint32_t kMaxKeyBlocks = 1u << (32 - kMaxKeyBits);    // 2m < 2^32
// Key blocks: the first nsmall blocks span 2^ks positions each, the rest
// 2^kbits.  First occurrences are densest at the start of S, where a block of
// 2^kbits positions can hold that many keys for one workgroup to rank (at
// RMAT-24 the first 2^17-position block took 0.14 ms, alone at the end of
// rank_block), so the start is cut 4x finer.
struct KeyBlocks {
    uint32_t kbits, ks, nsmall;
    __host__ __device__ uint32_t lead() const { return nsmall << ks; }
    __device__ uint32_t block(uint32_t p) const { return p < lead() ? p >> ks : nsmall + ((p - lead()) >> kbits); }
    __device__ uint32_t base(uint32_t b) const { return b < nsmall ? b << ks : lead() + ((b - nsmall) << kbits); }
    __device__ uint32_t bits(uint32_t b) const { return b < nsmall ? ks : kbits; }
};
constexpr uint32_t kSmallKeyBlocks = 64;
constexpr uint32_t kMinSmallKeyBits = 12;
constexpr uint32_t kMinRankBits = 10;                           // a rank bucket spans at least kMinThreads vertices
constexpr uint64_t kTargetRankBuckets = 512;
constexpr uint64_t kMaxRankTable = 1u << 21;
static_assert((1u << kMinRankBits) == (uint32_t)kMinThreads, "rank_perm's flag words assume it");

__device__ __forceinline__ uint32_t merged_r(const uint32_t *__restrict__ rpart, uint32_t slices, uint32_t n,
                                             uint32_t v) {
    uint32_t p = rpart[v];
    for (uint32_t s = 1; s < slices; ++s) p = min(p, rpart[(size_t)s * n + v]);
    return p;
}

// cnt_b[b][k]: bucket-major (coalesced rows); cnt gets its final zero, where
// the scan of the transposed counts leaves the total.
__global__ __launch_bounds__(kMinThreads) void k_rank_count(uint32_t *__restrict__ rpart, uint32_t slices,
                                                            uint32_t n, uint32_t nb, uint32_t rbits, uint32_t nblk,
                                                            KeyBlocks kb, uint32_t *__restrict__ cnt_b,
                                                            uint32_t *__restrict__ cnt) {
    __shared__ uint32_t h[kMaxKeyBlocks + 1];
    const uint32_t b = blockIdx.x;
    const uint32_t w = 1u << rbits;
    const uint32_t v0 = b << rbits;
    const uint32_t cntv = min(w, n - v0);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    for (uint32_t k = threadIdx.x; k <= nblk; k += kMinThreads) h[k] = 0;
    if (b == 0 && threadIdx.x == 0) cnt[(size_t)(nblk + 1) * nb] = 0;  // the scan's total lands here
    __syncthreads();
    for (uint32_t q = 0; q < cntv; q += kMinThreads) {
        const uint32_t i = q + threadIdx.x;
        const uint32_t p = i < cntv ? merged_r(rpart, slices, n, v0 + i) : 0u;
        if (slices > 1 && i < cntv) rpart[v0 + i] = p;  // each vertex is read and written by this thread only
        const bool iso = i < cntv && p == kInf;
        // isolated vertices are common (about 38% in RMAT): one atomic per wave
        const uint64_t bal = __ballot(iso);
        if (iso && lane == (uint32_t)(__ffsll((long long)bal) - 1)) atomicAdd(&h[nblk], (uint32_t)__popcll(bal));
        if (i < cntv && !iso) atomicAdd(&h[kb.block(p)], 1u);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k <= nblk; k += kMinThreads) cnt_b[(size_t)b * (nblk + 1) + k] = h[k];
}

// r: the merged minima (slice 0 after rank_count)
__global__ __launch_bounds__(kMinThreads) void k_rank_scatter(const uint32_t *__restrict__ r, uint32_t n,
                                                              uint32_t rbits, uint32_t nblk, KeyBlocks kb,
                                                              const uint32_t *__restrict__ off_b, uint2 *__restrict__ E) {
    __shared__ uint32_t cur[kMaxKeyBlocks];
    const uint32_t b = blockIdx.x;
    const uint32_t v0 = b << rbits;
    const uint32_t cntv = min(1u << rbits, n - v0);
    for (uint32_t k = threadIdx.x; k < nblk; k += kMinThreads) cur[k] = off_b[(size_t)b * (nblk + 1) + k];
    __syncthreads();
    constexpr int U = 8;
    for (uint32_t i0 = threadIdx.x; i0 < cntv; i0 += U * kMinThreads) {
        uint32_t p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * kMinThreads;
            p[u] = i < cntv ? r[v0 + i] : kInf;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p[u] != kInf) {
                const uint32_t slot = atomicAdd(&cur[kb.block(p[u])], 1u);
                E[slot] = make_uint2(p[u], v0 + i0 + u * kMinThreads);
            }
        }
    }
}

// One 1024-thread workgroup per key block, LDS sized to the block (dynamic):
// bits[2^(kbits-5)], then uint16 pre[same], then uint32 gbase[2^(kbits-11)].
// At 2^17 positions per block that is 24 KB, so two blocks share a CU.
constexpr int kRankThreads = 1024;

inline size_t rank_block_lds(uint32_t kbits) {
    const size_t words = (size_t)1 << (kbits - 5);
    return words * 4 + words * 2 + (words / kWave) * 4;
}

__global__ __launch_bounds__(kRankThreads) void k_rank_block(uint2 *__restrict__ E,
                                                             const uint32_t *__restrict__ off, uint32_t nb,
                                                             KeyBlocks kb, int32_t *__restrict__ order) {
    extern __shared__ __align__(16) uint32_t dyn[];
    // LDS sized for a regular block; a small one uses the front of each array
    const uint32_t kbits = kb.bits(blockIdx.x);
    const uint32_t nwords = 1u << (kbits - 5);
    const uint32_t ngroups = nwords / kWave;  // 2 .. 256
    uint32_t *bits = dyn;
    uint16_t *pre = (uint16_t *)(dyn + nwords);      // exclusive popcount within a 64-word group
    uint32_t *gbase = dyn + nwords + nwords / 2;     // exclusive popcount of the groups
    // plain order: the dense first key blocks go round-robin to all XCDs
    const uint32_t blk = blockIdx.x;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    constexpr uint32_t NWAVE = kRankThreads / kWave;
    for (uint32_t i = threadIdx.x; i < nwords; i += kRankThreads) bits[i] = 0;
    __syncthreads();
    const uint32_t e0 = off[(size_t)blk * nb];
    const uint32_t e1 = off[(size_t)(blk + 1) * nb];
    const uint32_t base = kb.base(blk);
    constexpr int U = 8;  // entries in flight per thread
    // a block of at most U * kRankThreads entries (nearly all) stays in
    // registers between setting the bits and ranking
    const bool one_pass = e1 - e0 <= U * kRankThreads;
    uint2 held[U];
    if (one_pass) {
        // loads at clamped indices, the guard applied afterwards: all U in
        // flight before the first is waited for
        if (e1 > e0) {  // the same for the whole workgroup
#pragma unroll
            for (int u = 0; u < U; ++u) held[u] = E[min(e0 + threadIdx.x + u * kRankThreads, e1 - 1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + threadIdx.x + u * kRankThreads >= e1) held[u] = make_uint2(base, 0u);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t p = held[u].x - base;
            if (e0 + threadIdx.x + u * kRankThreads < e1) atomicOr(&bits[p >> 5], 1u << (p & 31));
        }
    } else {
        for (uint32_t e = e0 + threadIdx.x; e < e1; e += U * kRankThreads) {
            uint32_t p[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t i = e + u * kRankThreads;
                p[u] = i < e1 ? E[i].x - base : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (e + u * kRankThreads < e1) atomicOr(&bits[p[u] >> 5], 1u << (p[u] & 31));
        }
    }
    __syncthreads();
    for (uint32_t g = wave; g < ngroups; g += NWAVE) {
        const uint32_t w = g * kWave + lane;
        const uint32_t c = __popc(bits[w]);
        const uint32_t incl = wave_inclusive_scan(c, OpSum{});
        pre[w] = (uint16_t)(incl - c);
        if (lane == kWave - 1) gbase[g] = incl;
    }
    __syncthreads();
    // exclusive scan of the group sums (at most 256 groups): one wave, four per lane
    if (wave == 0) {
        uint32_t v[4], t = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t g = lane * 4 + q;
            v[q] = g < ngroups ? gbase[g] : 0u;
            t += v[q];
        }
        uint32_t run = wave_inclusive_scan(t, OpSum{}) - t;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t g = lane * 4 + q;
            if (g < ngroups) gbase[g] = run;
            run += v[q];
        }
    }
    __syncthreads();
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += U * kRankThreads) {
        uint2 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = e + u * kRankThreads;
            x[u] = one_pass ? held[u] : (i < e1 ? E[i] : make_uint2(base, 0u));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (e + u * kRankThreads >= e1) continue;
            const uint32_t p = x[u].x - base;
            const uint32_t w = p >> 5;
            const uint32_t k = e0 + gbase[w / kWave] + pre[w] + __popc(bits[w] & ((1u << (p & 31)) - 1u));
            E[e + u * kRankThreads] = make_uint2(k, x[u].y);  // the rank replaces the key (coalesced)
            if (order) order[k] = (int32_t)x[u].y;  // within the block's rank range
        }
    }
}

// Per rank bucket: the ranks of its occurring vertices come back from the
// entry list into an LDS perm slice (segment bounds 64 at a time, the first 64
// entries of 8 segments in flight); isolated vertices (still unset) take the
// tail ranks from iso_base on in increasing ID, via one ballot bitmap and one
// scan; the slice is written out coalesced.
__global__ __launch_bounds__(kMinThreads) void k_rank_perm(const uint2 *__restrict__ E,
                                                           const uint32_t *__restrict__ off_b,
                                                           const uint32_t *__restrict__ cnt_b, uint32_t nblk,
                                                           uint32_t n, uint32_t rbits, int32_t *__restrict__ perm,
                                                           int32_t *__restrict__ order) {
    __shared__ uint32_t lp[kBucketW];
    __shared__ uint32_t pre[kPermChunk + 1];  // entries of the bucket in earlier key blocks of the chunk
    __shared__ uint32_t obs[kPermChunk];      // where the bucket's slice of each key block starts in E
    __shared__ uint32_t flags[kBucketW / 32];
    __shared__ uint32_t scan_lds[kMinThreads / kWave];
    // neighbouring buckets on one XCD: their slices of a key block lie side by
    // side in E and are read through the same L2 (0.12 -> 0.106 ms at RMAT-24)
    const uint32_t b = xcd_work_index(blockIdx.x, gridDim.x);
    const uint32_t w = 1u << rbits;  // kMinThreads .. kBucketW vertices
    const uint32_t v0 = b << rbits;
    const uint32_t cntv = min(w, n - v0);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    for (uint32_t i = threadIdx.x; i < w; i += kMinThreads) lp[i] = kInf;
    const uint32_t *ob = off_b + (size_t)b * (nblk + 1);
    const uint32_t *cb = cnt_b + (size_t)b * (nblk + 1);
    // The bucket's entries lie in one small slice per key block.  Per chunk of
    // kPermChunk key blocks, the slices are numbered through in order and each
    // thread takes a contiguous run of them, 8 loads in flight.
    constexpr int U = 8;
    for (uint32_t k0 = 0; k0 < nblk; k0 += kPermChunk) {
        const uint32_t kc = min(kPermChunk, nblk - k0);
        const uint32_t t = threadIdx.x;
        const uint32_t c = t < kc ? cb[k0 + t] : 0u;
        if (t < kc) obs[t] = ob[k0 + t];
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<kMinThreads>(c, OpSum{}, scan_lds, tot);
        pre[t] = ex;  // = tot for t >= kc
        if (t == 0) pre[kPermChunk] = tot;
        __syncthreads();
        const uint32_t per = (tot + kMinThreads - 1) / kMinThreads;
        uint32_t i = t * per;
        const uint32_t iend = min(tot, i + per);
        if (i < iend) {
            uint32_t k = 0, hi = kc - 1;  // the last slice starting at or before entry i
            while (k < hi) {
                const uint32_t mid = (k + hi + 1) >> 1;
                if (pre[mid] <= i) k = mid;
                else hi = mid - 1;
            }
            for (; i < iend; i += U) {
                uint2 x[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t ii = i + u;
                    if (ii < iend) {
                        while (pre[k + 1] <= ii) ++k;
                        x[u] = E[obs[k] + (ii - pre[k])];
                    } else {
                        x[u] = make_uint2(0u, kInf);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (x[u].y != kInf) lp[(x[u].y - v0) & (w - 1)] = x[u].x;
            }
        }
        __syncthreads();  // pre and obs are rewritten by the next chunk
    }
    // isolated flags: vertices [u*1024 + wave*64, +64) -> words 32u + 2 wave, +1
    for (uint32_t u = 0; u < w / kMinThreads; ++u) {
        const uint32_t i = u * kMinThreads + threadIdx.x;
        const uint64_t bal = __ballot(i < cntv && lp[i] == kInf);
        if (lane == 0) {
            const uint32_t w = (u * kMinThreads + wave * kWave) / 32;
            flags[w] = (uint32_t)bal;
            flags[w + 1] = (uint32_t)(bal >> 32);
        }
    }
    __syncthreads();
    const uint32_t word = threadIdx.x < w / 32 ? flags[threadIdx.x] : 0u;  // vertices 32 t .. 32 t + 31
    uint32_t tot;
    const uint32_t before = block_exclusive_scan<kMinThreads>(__popc(word), OpSum{}, scan_lds, tot);
    uint32_t left = word, k = ob[nblk] + before;
    while (left) {
        const uint32_t j = __ffs(left) - 1;
        left &= left - 1;
        lp[threadIdx.x * 32 + j] = k;
        if (order) order[k] = (int32_t)(v0 + threadIdx.x * 32 + j);
        ++k;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cntv; i += kMinThreads) perm[v0 + i] = (int32_t)lp[i];
}

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Host-side plan: which scatter path runs and the bucketed path's shape.
struct ReorderPlan {
    bool small;     // one workgroup, one launch (small_graph), unless BOBA_FLAG_FORCE_GENERAL
    bool bucketed;
    uint32_t nb, tiles_half, nt, region, slices, tps;
    KeyBlocks kb;          // key blocks of the bucketed ranking
    uint32_t nblk;
    uint32_t rbits, nbr;   // rank buckets: 2^rbits vertices each, nbr of them
};

ReorderPlan reorder_plan(int64_t n, int64_t m) {
    ReorderPlan P{};
    P.small = small_graph(n, m);
    P.nb = ceil_div((uint64_t)n, kBucketW);
    P.tiles_half = ceil_div((uint64_t)m, kTileT);
    P.nt = 2 * P.tiles_half;
    P.bucketed = m > 0 && n > 0 && P.nb <= kMaxBuckets;
    P.slices = 1;
    if (P.bucketed) {
        // Enough (bucket, slice) workgroups to fill 256 CUs; up to four per CU
        // so that uneven buckets (hubs of a power-law graph land in a few) are
        // balanced by the dispatcher, as long as the partial minima (slices x
        // 4n bytes) stay below an eighth of the record traffic (8m bytes).
        const uint64_t fill = ceil_div(256, P.nb), spread = ceil_div(1024, P.nb);
        const uint64_t cap = (uint64_t)m / (4 * (uint64_t)n) > 1 ? (uint64_t)m / (4 * (uint64_t)n) : 1;
        uint64_t s = spread < cap ? spread : cap;
        if (s < fill) s = fill;
        P.slices = (uint32_t)(s < P.nt ? s : P.nt);
        if (P.slices < 1) P.slices = 1;
        P.region = split_region(P.nb);
        // about 4096 key blocks of 2^15 .. 2^18 positions: the first blocks of
        // a graph hold most first occurrences, and a small block bounds the
        // work of the workgroup that ranks it
        const uint64_t keys = 2 * (uint64_t)m;
        uint32_t kbits = kMinKeyBits;
        while (kbits < kMaxKeyBits && (keys >> kbits) > kTargetKeyBlocks) ++kbits;
        // the leading blocks 4x finer (at most kSmallKeyBlocks of them)
        const uint32_t ks = kbits - 2 > kMinSmallKeyBits ? kbits - 2 : kMinSmallKeyBits;
        const uint64_t lead_max = (uint64_t)kSmallKeyBlocks << ks;
        uint64_t nblk;
        if (keys <= lead_max) {
            P.kb = KeyBlocks{kbits, ks, (uint32_t)ceil_div(keys, 1ull << ks)};
            nblk = P.kb.nsmall;
        } else {
            P.kb = KeyBlocks{kbits, ks, kSmallKeyBlocks};
            nblk = kSmallKeyBlocks + ceil_div(keys - lead_max, 1ull << kbits);
        }
        if (nblk > kMaxKeyBlocks) {  // only near 2m = 2^32: regular blocks throughout
            P.kb = KeyBlocks{kbits, kbits, 0};
            nblk = ceil_div(keys, 1ull << kbits);
        }
        P.nblk = (uint32_t)nblk;
        // rank buckets: narrower than the split's until there are about 512
        // (two 1024-thread workgroups per CU), while the count table
        // (key blocks + 1) x rank buckets stays within 2^21 words
        P.rbits = kVBits;
        auto nbr_at = [&](uint32_t bits) { return ceil_div((uint64_t)n, 1ull << bits); };
        while (P.rbits > kMinRankBits && nbr_at(P.rbits) < kTargetRankBuckets &&
               (uint64_t)(P.nblk + 1) * nbr_at(P.rbits - 1) <= kMaxRankTable)
            --P.rbits;
        P.nbr = (uint32_t)nbr_at(P.rbits);
    }
    P.tps = P.nt ? ceil_div(P.nt, P.slices) : 0;
    return P;
}

struct ReorderLayout {
    uint32_t *r;  // r = slice 0 of the partial minima
    uint2 *W;
    uint32_t *partial;
    uint32_t *recs, *tile_off, *off_t;
    uint32_t *vals;  // new IDs in record layout (fused relabel only)
    uint32_t *cnt, *cnt_b, *off_b, *cnt_partial;  // bucketed ranking
    uint2 *E;
    uint32_t ncnt;
    size_t bytes;
    uint32_t nw;
};

ReorderLayout reorder_layout(void *ws, int64_t n, int64_t m, const ReorderPlan &P, bool with_vals = false) {
    ReorderLayout L{};
    const uint64_t positions = 2 * (uint64_t)m + (uint64_t)n;
    L.nw = ceil_div(positions, 32);
    Carver c(ws);
    L.W = c.take<uint2>(L.nw);
    L.partial = c.take<uint32_t>(scan_partials(L.nw));
    L.r = c.take<uint32_t>((size_t)n * P.slices);
    L.recs = c.take<uint32_t>(P.bucketed ? (size_t)P.nt * P.region : 0);
    L.tile_off = c.take<uint32_t>(P.bucketed ? (size_t)P.nt * (P.nb + 1) : 0);
    L.off_t = c.take<uint32_t>(P.bucketed ? (size_t)P.nt * (P.nb + 1) : 0);
    L.vals = c.take<uint32_t>(P.bucketed && with_vals ? (size_t)P.nt * P.region : 0);
    L.ncnt = P.bucketed ? (P.nblk + 1) * P.nbr + 1 : 0;
    L.cnt = c.take<uint32_t>(L.ncnt);
    L.cnt_b = c.take<uint32_t>(P.bucketed ? L.ncnt - 1 : 0);
    L.off_b = c.take<uint32_t>(P.bucketed ? L.ncnt - 1 : 0);
    L.cnt_partial = c.take<uint32_t>(P.bucketed ? scan_partials(L.ncnt) : 0);
    L.E = c.take<uint2>(P.bucketed ? (size_t)n : 0);
    L.bytes = c.bytes();
    return L;
}

// Tiles per wave step of the bucket kernels: spread a slice's tiles over all 16 waves.
uint32_t min_batch(const ReorderPlan &P) {
    uint32_t batch = ceil_div(P.tps, kMinThreads / kWave);
    batch = (batch + kMinGroup - 1) / kMinGroup * kMinGroup;
    return batch < (uint32_t)kMinGroup ? kMinGroup : (batch > (uint32_t)kWave ? kWave : batch);
}

boba_status check_sizes(int64_t m, int64_t n, bool positions) {
    if (m < 0 || n < 0) return fail(BOBA_ERR_ARG, "negative size (m=%lld, n=%lld)", (long long)m, (long long)n);
    if (m >= (1ll << 31) || n >= (1ll << 31))
        return fail(BOBA_ERR_OVERFLOW, "m and n must be < 2^31 (m=%lld, n=%lld)", (long long)m, (long long)n);
    if (positions && 2 * m + n >= (1ll << 32))
        return fail(BOBA_ERR_OVERFLOW, "2m + n must be < 2^32 (m=%lld, n=%lld)", (long long)m, (long long)n);
    return BOBA_OK;
}

// Which path a reorder took.
enum ReorderPath { PATH_SMALL, PATH_BUCKETED, PATH_DIRECT };

// Launches the reorder; *path tells which path ran.  so / dso (nullable): the
// small path also writes the relabelled edges there.
boba_status reorder_run(const int32_t *src, const int32_t *dst, uint32_t um, uint32_t un, int32_t *perm,
                        int32_t *order, bool inter, bool racy, bool general, const ReorderPlan &P,
                        const ReorderLayout &L, int32_t *flag, hipStream_t stream, ReorderPath *path,
                        int32_t *so = nullptr,
                        int32_t *dso = nullptr) {
    if (P.small && !general) {
        *path = PATH_SMALL;
        if (inter && racy)
            BOBA_LAUNCH("small_reorder", (k_small_reorder<true, true>), dim3(1), dim3(kSmallThreads), stream, src, dst,
                        um, un, L.W, L.nw, perm, order, so, dso, flag);
        else if (inter)
            BOBA_LAUNCH("small_reorder", (k_small_reorder<true, false>), dim3(1), dim3(kSmallThreads), stream, src,
                        dst, um, un, L.W, L.nw, perm, order, so, dso, flag);
        else if (racy)
            BOBA_LAUNCH("small_reorder", (k_small_reorder<false, true>), dim3(1), dim3(kSmallThreads), stream, src,
                        dst, um, un, L.W, L.nw, perm, order, so, dso, flag);
        else
            BOBA_LAUNCH("small_reorder", (k_small_reorder<false, false>), dim3(1), dim3(kSmallThreads), stream, src,
                        dst, um, un, L.W, L.nw, perm, order, so, dso, flag);
        return BOBA_OK;
    }
    const bool bucketed = P.bucketed;
    *path = bucketed ? PATH_BUCKETED : PATH_DIRECT;
    const uint32_t tail = 2 * um;
    if (bucketed) {
        BOBA_LAUNCH("bucket_split", k_bucket_split, dim3(P.nt < device_cus() ? P.nt : device_cus()),
                    dim3(kSplitThreads), stream, src, dst, um,
                    P.tiles_half, un, P.nb, P.region, aligned16(src) && aligned16(dst), L.recs, L.tile_off, flag);
        BOBA_LAUNCH("bucket_transpose", k_transpose, dim3(ceil_div(P.nb + 1, 32), ceil_div(P.nt, 32)), dim3(256),
                    stream, (const uint32_t *)L.tile_off, P.nt, P.nb + 1, L.off_t);
        if (racy)
            BOBA_LAUNCH("bucket_min", k_bucket_min<true>, dim3(P.nb * P.slices), dim3(kMinThreads), stream,
                        (const uint32_t *)L.recs, (const uint32_t *)L.off_t, P.nt, P.tiles_half, P.region, P.nb,
                        P.tps, min_batch(P), un, inter ? 1u : um, inter ? 2u : 1u, L.r);
        else
            BOBA_LAUNCH("bucket_min", k_bucket_min<false>, dim3(P.nb * P.slices), dim3(kMinThreads), stream,
                        (const uint32_t *)L.recs, (const uint32_t *)L.off_t, P.nt, P.tiles_half, P.region, P.nb,
                        P.tps, min_batch(P), un, inter ? 1u : um, inter ? 2u : 1u, L.r);
        const uint32_t kcols = P.nblk + 1;  // key blocks and the tail block
        BOBA_LAUNCH("rank_count", k_rank_count, dim3(P.nbr), dim3(kMinThreads), stream, L.r, P.slices, un, P.nbr,
                    P.rbits, P.nblk, P.kb, L.cnt_b, L.cnt);
        // bucket-major counts -> block-major, scanned in place -> bucket-major offsets
        BOBA_LAUNCH("rank_transpose", k_transpose, dim3(ceil_div(kcols, 32), ceil_div(P.nbr, 32)), dim3(256), stream,
                    (const uint32_t *)L.cnt_b, P.nbr, kcols, L.cnt);
        if (boba_status e = device_scan<OpSum, false>("rank_scan", LoadArr{L.cnt}, StoreArr{L.cnt}, L.ncnt,
                                                      L.cnt_partial, stream))
            return e;
        BOBA_LAUNCH("rank_transpose", k_transpose, dim3(ceil_div(P.nbr, 32), ceil_div(kcols, 32)), dim3(256), stream,
                    (const uint32_t *)L.cnt, kcols, P.nbr, L.off_b);
        BOBA_LAUNCH("rank_scatter", k_rank_scatter, dim3(P.nbr), dim3(kMinThreads), stream, (const uint32_t *)L.r,
                    un, P.rbits, P.nblk, P.kb, (const uint32_t *)L.off_b, L.E);
        {
            const size_t lds = rank_block_lds(P.kb.kbits);
            const int tok = timing_begin("rank_block", stream);
            hipLaunchKernelGGL(k_rank_block, dim3(P.nblk), dim3(kRankThreads), lds, stream, L.E,
                               (const uint32_t *)L.cnt, P.nbr, P.kb, order);
            timing_end(tok, stream);
            if (boba_status e = check_launch("rank_block")) return e;
        }
        BOBA_LAUNCH("rank_perm", k_rank_perm, dim3(P.nbr), dim3(kMinThreads), stream, (const uint2 *)L.E,
                    (const uint32_t *)L.off_b, (const uint32_t *)L.cnt_b, P.nblk, un, P.rbits, perm, order);
        return BOBA_OK;
    } else {
        BOBA_LAUNCH("reorder_init", k_reorder_init, dim3(grid_for(un > L.nw ? un : L.nw, kBlock * 4)),
                    dim3(kBlock), stream, L.r, un, L.W, L.nw);
        uint32_t k0 = 0;
        if (um > 0 && aligned16(src) && aligned16(dst)) {
            const uint32_t m4 = um / 4;
            if (m4 > 0) {
                dim3 grid(ceil_div(2ull * m4, kScatterTile));
                const v4i *s4 = (const v4i *)src, *d4 = (const v4i *)dst;
                if (inter && racy)
                    BOBA_LAUNCH("scatter_min", (k_scatter_min_vec<true, true>), grid, dim3(kBlock), stream, s4, d4,
                                m4, um, un, L.r, flag);
                else if (inter)
                    BOBA_LAUNCH("scatter_min", (k_scatter_min_vec<true, false>), grid, dim3(kBlock), stream, s4, d4,
                                m4, um, un, L.r, flag);
                else if (racy)
                    BOBA_LAUNCH("scatter_min", (k_scatter_min_vec<false, true>), grid, dim3(kBlock), stream, s4, d4,
                                m4, um, un, L.r, flag);
                else
                    BOBA_LAUNCH("scatter_min", (k_scatter_min_vec<false, false>), grid, dim3(kBlock), stream, s4, d4,
                                m4, um, un, L.r, flag);
            }
            k0 = 4 * m4;
        }
        if (k0 < um) {
            dim3 grid(grid_for(2ull * (um - k0), kBlock));
            if (inter && racy)
                BOBA_LAUNCH("scatter_min_scalar", (k_scatter_min_scalar<true, true>), grid, dim3(kBlock), stream,
                            src, dst, k0, um, un, L.r, flag);
            else if (inter)
                BOBA_LAUNCH("scatter_min_scalar", (k_scatter_min_scalar<true, false>), grid, dim3(kBlock), stream,
                            src, dst, k0, um, un, L.r, flag);
            else if (racy)
                BOBA_LAUNCH("scatter_min_scalar", (k_scatter_min_scalar<false, true>), grid, dim3(kBlock), stream,
                            src, dst, k0, um, un, L.r, flag);
            else
                BOBA_LAUNCH("scatter_min_scalar", (k_scatter_min_scalar<false, false>), grid, dim3(kBlock), stream,
                            src, dst, k0, um, un, L.r, flag);
        }
        BOBA_LAUNCH("mark", k_mark, dim3(grid_for(un, kBlock * 4)), dim3(kBlock), stream, (const uint32_t *)L.r, un,
                    tail, L.W);
    }
    if (boba_status e = device_scan<OpSum, false>("bitmap_scan", LoadPopc{L.W}, StorePrefix{L.W}, L.nw, L.partial,
                                                  stream))
        return e;
    BOBA_LAUNCH("rank", k_rank, dim3(grid_for(un, kBlock * 4)), dim3(kBlock), stream, (const uint32_t *)L.r, un, tail,
                (const uint2 *)L.W, perm, order);
    return BOBA_OK;
}

boba_status relabel_run(const int32_t *src, const int32_t *dst, uint32_t um, const int32_t *perm, uint32_t un,
                        int32_t *src_out, int32_t *dst_out, int32_t *flag, hipStream_t stream) {
    uint32_t k0 = 0;
    if (aligned16(src) && aligned16(dst) && aligned16(src_out) && aligned16(dst_out)) {
        const uint32_t m4 = um / 4;
        if (m4 > 0) {
            BOBA_LAUNCH("relabel", k_relabel_vec, dim3(ceil_div(2ull * m4, kRelabelTile)), dim3(kBlock), stream,
                        (const v4i *)src, (const v4i *)dst, m4, perm, un, (v4i *)src_out, (v4i *)dst_out, flag);
        }
        k0 = 4 * m4;
    }
    if (k0 < um) {
        BOBA_LAUNCH("relabel_scalar", k_relabel_scalar, dim3(grid_for(2ull * (um - k0), kBlock)), dim3(kBlock), stream,
                    src, dst, k0, um, perm, un, src_out, dst_out, flag);
    }
    return BOBA_OK;
}

boba_status reorder_args(const int32_t *src, const int32_t *dst, int64_t m, int64_t n, int32_t *perm, uint32_t flags,
                         const char *who) {
    if (boba_status e = check_sizes(m, n, true)) return e;
    if (flags & ~(BOBA_FLAG_INTERLEAVED | BOBA_FLAG_RACY | BOBA_FLAG_FORCE_GENERAL))
        return fail(BOBA_ERR_ARG, "%s: unknown flags 0x%x", who, flags);
    if (m > 0 && (!src || !dst)) return fail(BOBA_ERR_ARG, "%s: src/dst is NULL", who);
    if (m > 0 && n == 0) return fail(BOBA_ERR_ARG, "%s: edges given but n = 0", who);
    if (n > 0 && !perm) return fail(BOBA_ERR_ARG, "%s: perm is NULL", who);
    return BOBA_OK;
}

}  // namespace
}  // namespace boba

using namespace boba;

extern "C" size_t boba_reorder_workspace(int64_t n, int64_t m) {
    if (n < 0 || m < 0) return 0;
    return reorder_layout(nullptr, n, m, reorder_plan(n, m)).bytes;
}

extern "C" boba_status boba_reorder(const int32_t *src, const int32_t *dst, int64_t m, int64_t n, int32_t *perm,
                                    int32_t *order, void *ws, size_t ws_bytes, uint32_t flags, hipStream_t stream) {
    clear_error();
    if (boba_status e = reorder_args(src, dst, m, n, perm, flags, "boba_reorder")) return e;
    if (n == 0) return BOBA_OK;
    const size_t need = boba_reorder_workspace(n, m);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "boba_reorder: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)",
                    need, ws_bytes, ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    const ReorderPlan P = reorder_plan(n, m);
    const ReorderLayout L = reorder_layout(ws, n, m, P);
    ReorderPath path;
    return reorder_run(src, dst, (uint32_t)m, (uint32_t)n, perm, order, flags & BOBA_FLAG_INTERLEAVED,
                       flags & BOBA_FLAG_RACY, flags & BOBA_FLAG_FORCE_GENERAL, P, L, flag, stream, &path);
}

// ------------------------------------------------ allocation-free reorder
// Workspace of boba_reorder_noalloc.  In host code this name is only a
// stand-in for the device array: the device address comes from
// hipGetSymbolAddress, once per device (each device holds its own copy).
static __device__ __align__(256) unsigned char scratch[BOBA_REORDER_NOALLOC_MAX_BYTES];

namespace {
constexpr int kScratchDevices = 64;
void *g_scratch_ptr[kScratchDevices] = {};
std::mutex g_scratch_mu;

// Device address of this device's scratch (nullptr and a message on failure).
void *scratch_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) {
        fail(BOBA_ERR_HIP, "boba_reorder_noalloc: hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fail(BOBA_ERR_HIP, "boba_reorder_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" boba_status boba_reorder_noalloc(const int32_t *src, const int32_t *dst, int64_t m, int64_t n,
                                            int32_t *perm, int32_t *order, uint32_t flags, hipStream_t stream) {
    clear_error();
    if (boba_status e = reorder_args(src, dst, m, n, perm, flags, "boba_reorder_noalloc")) return e;
    if (n == 0) return BOBA_OK;
    const size_t need = boba_reorder_workspace(n, m);
    if (need > BOBA_REORDER_NOALLOC_MAX_BYTES)
        return fail(BOBA_ERR_WORKSPACE,
                    "boba_reorder_noalloc: n=%lld, m=%lld needs %zu bytes of workspace; the static scratch "
                    "holds %zu",
                    (long long)n, (long long)m, need, (size_t)BOBA_REORDER_NOALLOC_MAX_BYTES);
    void *ws = scratch_ptr();
    if (!ws) return BOBA_ERR_HIP;
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    TimingSuspend no_events;
    const ReorderPlan P = reorder_plan(n, m);
    const ReorderLayout L = reorder_layout(ws, n, m, P);
    ReorderPath path;
    return reorder_run(src, dst, (uint32_t)m, (uint32_t)n, perm, order, flags & BOBA_FLAG_INTERLEAVED,
                       flags & BOBA_FLAG_RACY, flags & BOBA_FLAG_FORCE_GENERAL, P, L, flag, stream, &path);
}

extern "C" size_t boba_reorder_relabel_workspace(int64_t n, int64_t m) {
    if (n < 0 || m < 0) return 0;
    return reorder_layout(nullptr, n, m, reorder_plan(n, m), true).bytes;
}

extern "C" boba_status boba_reorder_relabel(const int32_t *src, const int32_t *dst, int64_t m, int64_t n,
                                            int32_t *perm, int32_t *order, int32_t *src_out, int32_t *dst_out,
                                            void *ws, size_t ws_bytes, uint32_t flags, hipStream_t stream) {
    clear_error();
    if (boba_status e = reorder_args(src, dst, m, n, perm, flags, "boba_reorder_relabel")) return e;
    if (m > 0 && (!src_out || !dst_out)) return fail(BOBA_ERR_ARG, "boba_reorder_relabel: src_out/dst_out is NULL");
    if (n == 0) return BOBA_OK;
    const size_t need = boba_reorder_relabel_workspace(n, m);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE,
                    "boba_reorder_relabel: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)", need, ws_bytes,
                    ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    const uint32_t um = (uint32_t)m, un = (uint32_t)n;
    const ReorderPlan P = reorder_plan(n, m);
    const ReorderLayout L = reorder_layout(ws, n, m, P, true);
    ReorderPath path;
    if (boba_status e = reorder_run(src, dst, um, un, perm, order, flags & BOBA_FLAG_INTERLEAVED,
                                    flags & BOBA_FLAG_RACY, flags & BOBA_FLAG_FORCE_GENERAL, P, L, flag, stream,
                                    &path, m > 0 ? src_out : nullptr,
                                    m > 0 ? dst_out : nullptr))
        return e;
    if (m == 0 || path == PATH_SMALL) return BOBA_OK;
    if (path == PATH_DIRECT) return relabel_run(src, dst, um, perm, un, src_out, dst_out, flag, stream);
    BOBA_LAUNCH("bucket_relabel", k_bucket_relabel, dim3(P.nb * P.slices), dim3(kMinThreads), stream,
                (const uint32_t *)L.recs, (const uint32_t *)L.off_t, P.nt, P.region, P.nb, P.tps, min_batch(P), un,
                (const int32_t *)perm, L.vals);
    BOBA_LAUNCH("tile_unsplit", k_tile_unsplit, dim3(P.nt), dim3(kSplitThreads), stream, (const uint32_t *)L.recs,
                (const uint32_t *)L.vals, (const uint32_t *)L.tile_off, P.nb, P.region, um, P.tiles_half, src_out,
                dst_out);
    return BOBA_OK;
}

extern "C" boba_status boba_relabel(const int32_t *src, const int32_t *dst, int64_t m, const int32_t *perm, int64_t n,
                                    int32_t *src_out, int32_t *dst_out, hipStream_t stream) {
    clear_error();
    if (boba_status e = check_sizes(m, n, false)) return e;
    if (m == 0) return BOBA_OK;
    if (!src || !dst || !src_out || !dst_out || !perm)
        return fail(BOBA_ERR_ARG, "boba_relabel: NULL pointer");
    if (n == 0) return fail(BOBA_ERR_ARG, "boba_relabel: edges given but n = 0");
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    return relabel_run(src, dst, (uint32_t)m, perm, (uint32_t)n, src_out, dst_out, flag, stream);
}

// The records, segment offsets and new IDs of the bucketed relabel (no ranking).
struct RelabelLayout {
    uint32_t *recs, *tile_off, *off_t, *vals;
    size_t bytes;
};

static RelabelLayout relabel_layout(void *ws, const ReorderPlan &P) {
    RelabelLayout L;
    Carver c(ws);
    L.recs = c.take<uint32_t>(P.bucketed ? (size_t)P.nt * P.region : 0);
    L.tile_off = c.take<uint32_t>(P.bucketed ? (size_t)P.nt * (P.nb + 1) : 0);
    L.off_t = c.take<uint32_t>(P.bucketed ? (size_t)P.nt * (P.nb + 1) : 0);
    L.vals = c.take<uint32_t>(P.bucketed ? (size_t)P.nt * P.region : 0);
    L.bytes = c.bytes() > 0 ? c.bytes() : 256;
    return L;
}

extern "C" size_t boba_relabel_bucketed_workspace(int64_t n, int64_t m) {
    if (n < 0 || m < 0 || n >= (1ll << 31) || m >= (1ll << 31)) return 0;
    return relabel_layout(nullptr, reorder_plan(n, m)).bytes;
}

extern "C" boba_status boba_relabel_bucketed(const int32_t *src, const int32_t *dst, int64_t m, const int32_t *perm,
                                             int64_t n, int32_t *src_out, int32_t *dst_out, void *ws,
                                             size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (boba_status e = check_sizes(m, n, false)) return e;
    if (m == 0) return BOBA_OK;
    if (!src || !dst || !src_out || !dst_out || !perm)
        return fail(BOBA_ERR_ARG, "boba_relabel_bucketed: NULL pointer");
    if (n == 0) return fail(BOBA_ERR_ARG, "boba_relabel_bucketed: edges given but n = 0");
    const size_t need = boba_relabel_bucketed_workspace(n, m);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE,
                    "boba_relabel_bucketed: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)", need,
                    ws_bytes, ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    const uint32_t um = (uint32_t)m, un = (uint32_t)n;
    const ReorderPlan P = reorder_plan(n, m);
    if (!P.bucketed) return relabel_run(src, dst, um, perm, un, src_out, dst_out, flag, stream);
    const RelabelLayout L = relabel_layout(ws, P);
    BOBA_LAUNCH("bucket_split", k_bucket_split, dim3(P.nt < device_cus() ? P.nt : device_cus()), dim3(kSplitThreads),
                stream, src, dst, um, P.tiles_half, un, P.nb, P.region, aligned16(src) && aligned16(dst), L.recs,
                L.tile_off, flag);
    BOBA_LAUNCH("bucket_transpose", k_transpose, dim3(ceil_div(P.nb + 1, 32), ceil_div(P.nt, 32)), dim3(256), stream,
                (const uint32_t *)L.tile_off, P.nt, P.nb + 1, L.off_t);
    BOBA_LAUNCH("bucket_relabel", k_bucket_relabel, dim3(P.nb * P.slices), dim3(kMinThreads), stream,
                (const uint32_t *)L.recs, (const uint32_t *)L.off_t, P.nt, P.region, P.nb, P.tps, min_batch(P), un,
                perm, L.vals);
    BOBA_LAUNCH("tile_unsplit", k_tile_unsplit, dim3(P.nt), dim3(kSplitThreads), stream, (const uint32_t *)L.recs,
                (const uint32_t *)L.vals, (const uint32_t *)L.tile_off, P.nb, P.region, um, P.tiles_half, src_out,
                dst_out);
    return BOBA_OK;
}

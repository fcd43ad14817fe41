// Batched BOBA: many graphs of uneven sizes reordered (and relabelled) by one
// persistent kernel, replayed from a hipGraph.
//
// Every graph g has its own edge list src/dst[edge_off[g] .. edge_off[g+1]) of
// local vertex IDs in [0, n_g), n_g = vert_off[g+1] - vert_off[g]; its outputs
// are perm/order[vert_off[g] ..] and, when relabelling, src_out/dst_out over
// the same edge range.  The semantics per graph are exactly boba_reorder's
// (flattening I ++ J, isolated vertices last in increasing ID).
//
// Work is a ticket-ordered list of items.  Workgroups of the persistent
// kernel take tickets from a global counter and run items in ticket order:
//   SMALL    a whole graph with n_g <= small_max_n in one workgroup: first
//            positions by LDS atomic min, ranks through a bitmap in the graph's
//            workspace (L2-resident), relabel by LDS gathers.
//   SPLIT    a tile of 16384 positions of a large graph: records {offset in
//            tile, v mod 2^15} sorted by vertex bucket (v >> 15) in LDS and
//            written with the tile's segment offsets (as boba_reorder's split).
//   FOLD     (vertex bucket, slice of tiles): the bucket's r in LDS, every
//            record of its segments folded in with an LDS minimum; the
//            slice's minima written out.
//   SCATTER  (graphs of more than 2^26 vertices, or when asked for) a tile of
//            positions: global atomic min into the graph's r.  Contended
//            device-wide atomics made this several times slower than
//            SPLIT + FOLD on the batch workloads.
//   MARK     a tile of vertices: r = minimum over the FOLD slices, then set
//            the bitmap bit of each key.
//   SCAN     the graph's bitmap prefix popcounts, one workgroup.
//   RANK     a tile of vertices: perm (and order).
//   RELABEL  a tile of edges: src_out = perm[src], dst_out = perm[dst].
// A large graph's stage-s items wait for all its stage-(s-1) items.  Items are
// ordered so that every dependency has a smaller ticket; a ticket is only taken
// by a running workgroup, so every wait ends even without co-residency.  Waits
// are bounded anyway: past the spin limit the kernel flags an error and moves
// on.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace boba {
namespace {

constexpr int kThreads = 1024;
constexpr uint32_t kSmallMax = 32768;  // LDS capacity of the SMALL path (uint32 per vertex)
constexpr uint32_t kSpinLimit = 1u << 22;  // default: about 0.4 s of sleeping
constexpr uint32_t kQueues = 8;            // one per XCD: workgroup b starts on queue b % 8

enum ItemType : uint32_t { ITEM_SMALL = 0, ITEM_SCATTER = 1, ITEM_MARK = 2, ITEM_SCAN = 3, ITEM_RANK = 4,
                           ITEM_RELABEL = 5, ITEM_SPLIT = 6, ITEM_FOLD = 7 };
constexpr uint32_t kStages = 8;

// SPLIT / FOLD geometry: tiles of kTileP positions, vertex buckets of 2^kVB
// vertices (the FOLD's LDS r), at most kFoldBuckets buckets (the SPLIT's LDS
// counters), at most kMaxSlices slices per bucket.
constexpr uint32_t kTileP = 16384;
constexpr int kVB = 15;
constexpr uint32_t kBucketV = 1u << kVB;
constexpr uint32_t kFoldBuckets = 2048;
constexpr uint32_t kMaxSlices = 4;
constexpr uint32_t kSentinel = 0xFFFFFFFFu;
inline uint32_t fold_region(uint32_t nb) { return (kTileP + 3 * nb + 3) & ~3u; }

struct GraphDesc {
    int64_t edge_off;   // first edge
    int64_t vert_off;   // first vertex
    uint32_t m, n;
    uint32_t nw;        // bitmap words
    uint32_t pad;
    int64_t r_off;      // r (uint32 words) in the workspace, large graphs only
    int64_t w_off;      // bitmap (uint2 words) in the workspace
    int64_t p_off;      // line-aligned private copy of perm, large graphs only
    uint32_t need[kStages];  // items per stage (index = ItemType)
    // SPLIT / FOLD graphs (fold != 0)
    uint32_t fold, nb, tiles, region, slices, fold_tiles;
    int64_t rec_off;    // records: tiles x region words
    int64_t toff_off;   // segment offsets: tiles x (nb + 1) words
    int64_t rp_off;     // FOLD minima: slices x n words
};

struct Item {
    uint32_t type, graph, begin, end;
    uint32_t bucket, slice;  // FOLD only
};

struct BatchArgs {
    const int32_t *src, *dst;
    int32_t *perm, *order, *src_out, *dst_out;
    const GraphDesc *graphs;
    const Item *items;    // queue q owns items [qstart[q], qstart[q+1])
    uint32_t qstart[kQueues + 1];
    uint32_t *queue;      // [kQueues] ticket counters
    uint32_t *abort;      // [1] set when a wait gave up
    uint32_t spin_limit;  // sleeps before a wait gives up
    uint32_t *done;       // [G * 6] finished items per (graph, stage)
    uint32_t *r_pool;     // large-graph r arrays
    uint2 *w_pool;        // bitmaps
    int32_t *p_pool;      // large-graph perm copies read by RELABEL
    uint32_t *rec_pool;   // SPLIT records
    uint32_t *toff_pool;  // SPLIT segment offsets
    uint32_t *rp_pool;    // FOLD minima
    int32_t *flag;
};

// Cross-workgroup data goes through relaxed agent-scope atomic accesses,
// which are coherent across the XCDs without the L2 write-back / invalidate
// that agent-scope fences cost (those would evict every workgroup's L2-resident
// r and perm).  A producer waits for its own accesses to complete before a
// workgroup barrier and the counter increment; a consumer spins on the counter
// with relaxed loads and then reads with coherent loads, or with plain loads
// of lines no L2 can hold yet (first touch within the kernel).
__device__ __forceinline__ uint32_t ld_coh(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint2 ld_coh2(const uint2 *p) {
    const uint64_t v = __hip_atomic_load((const uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}
__device__ __forceinline__ void st_coh(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh2(uint32_t *p, uint32_t lo, uint32_t hi) {
    __hip_atomic_store((uint64_t *)p, (uint64_t)lo | ((uint64_t)hi << 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void drain() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);  // all of this wave's memory operations complete
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Thread 0 waits until `need` items of (graph, stage) have finished.
__device__ void wait_stage(const BatchArgs &A, uint32_t g, uint32_t stage, uint32_t need) {
    if (threadIdx.x == 0) {
        const uint32_t *c = A.done + (size_t)g * kStages + stage;
        uint32_t spins = 0;
        while (ld_coh(c) < need) {
            __builtin_amdgcn_s_sleep(4);
            // give up past the limit, or at once after another wait gave up
            if (++spins > A.spin_limit || ld_coh(A.abort) != 0) {
                atomicOr(A.abort, 1u);
                flag_timeout(A.flag);
                break;
            }
        }
    }
    __syncthreads();
}

__device__ void signal_stage(const BatchArgs &A, uint32_t g, uint32_t stage) {
    drain();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(A.done + (size_t)g * kStages + stage, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bitmap prefix popcounts of words [0, nw) by one workgroup.  Words are read
// in tiles of kThreads * kScanPer (coalesced, staged in LDS); each thread
// scans kScanPer consecutive words, the tile carries its total forward.
constexpr int kScanPer = 4;
__device__ void scan_bitmap(uint2 *W, uint32_t nw, uint32_t *lds, uint32_t *stage) {
    uint32_t carry = 0;
    for (uint32_t t0 = 0; t0 < nw; t0 += kThreads * kScanPer) {
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const uint32_t i = t0 + j * kThreads + threadIdx.x;
            stage[j * kThreads + threadIdx.x] = i < nw ? ld_coh(&W[i].x) : 0u;
        }
        __syncthreads();
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) s += __popc(stage[threadIdx.x * kScanPer + j]);
        uint32_t total;
        uint32_t run = carry + block_exclusive_scan<kThreads>(s, OpSum{}, lds, total);
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const uint32_t bits = stage[threadIdx.x * kScanPer + j];
            stage[threadIdx.x * kScanPer + j] = run;
            run += __popc(bits);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const uint32_t i = t0 + j * kThreads + threadIdx.x;
            if (i < nw) st_coh(&W[i].y, stage[j * kThreads + threadIdx.x]);
        }
        carry += total;
        __syncthreads();
    }
}

__device__ __forceinline__ uint32_t rank_of(const uint2 *W, uint32_t key) {
    const uint2 w = ld_coh2(W + (key >> 5));
    return w.y + __popc(w.x & ((1u << (key & 31)) - 1u));
}

constexpr int kU = 8;  // loads in flight per thread in streaming loops

__device__ void run_small(const BatchArgs &A, const GraphDesc &G, uint32_t *lr, uint32_t *lds, uint32_t *stage) {
    const uint32_t n = G.n, m = G.m;
    const int32_t *src = A.src + G.edge_off, *dst = A.dst + G.edge_off;
    uint2 *W = A.w_pool + G.w_off;
    bool bad = false;
    for (uint32_t v = threadIdx.x; v < n; v += kThreads) lr[v] = kInf;
    __syncthreads();
    // first positions: all loads of a round before its LDS atomics
    for (uint32_t k0 = threadIdx.x; k0 < m; k0 += kThreads * kU) {
        int32_t a[kU], b[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const uint32_t k = min(k0 + j * kThreads, m - 1);
            a[j] = __builtin_nontemporal_load(src + k);
            b[j] = __builtin_nontemporal_load(dst + k);
        }
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const uint32_t k = k0 + j * kThreads;
            if (k >= m) break;
            if ((uint32_t)a[j] < n) atomicMin(&lr[a[j]], k); else bad = true;
            if ((uint32_t)b[j] < n) atomicMin(&lr[b[j]], m + k); else bad = true;
        }
    }
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < n; v += kThreads) {
        uint32_t p = lr[v];
        if (p == kInf) p = 2 * m + v;
        lr[v] = p;
        atomicOr(&W[p >> 5].x, 1u << (p & 31));
    }
    drain();
    __syncthreads();
    scan_bitmap(W, G.nw, lds, stage);
    drain();
    __syncthreads();
    int32_t *perm = A.perm + G.vert_off;
    int32_t *order = A.order ? A.order + G.vert_off : nullptr;
    for (uint32_t v = threadIdx.x; v < n; v += kThreads) {
        const uint32_t k = rank_of(W, lr[v]);
        perm[v] = (int32_t)k;
        if (order && k < n) order[k] = (int32_t)v;
        lr[v] = k;  // each thread rewrites only its own vertices
    }
    __syncthreads();
    if (A.src_out && m > 0) {
        int32_t *so = A.src_out + G.edge_off, *dso = A.dst_out + G.edge_off;
        for (uint32_t k0 = threadIdx.x; k0 < m; k0 += kThreads * kU) {
            int32_t a[kU], b[kU];
#pragma unroll
            for (int j = 0; j < kU; ++j) {
                const uint32_t k = min(k0 + j * kThreads, m - 1);
                a[j] = __builtin_nontemporal_load(src + k);
                b[j] = __builtin_nontemporal_load(dst + k);
            }
#pragma unroll
            for (int j = 0; j < kU; ++j) {
                const uint32_t k = k0 + j * kThreads;
                if (k >= m) break;
                // ranks are < n: a valid ID
                __builtin_nontemporal_store((uint32_t)a[j] < n ? (int32_t)lr[a[j]] : a[j], so + k);
                __builtin_nontemporal_store((uint32_t)b[j] < n ? (int32_t)lr[b[j]] : b[j], dso + k);
            }
        }
    }
    if (bad) flag_range_error(A.flag);
}

// Exclusive sum over the workgroup of 64-bit values (lds: kThreads / kWave
// uint64); two barriers.
__device__ uint64_t block_exclusive_sum64(uint64_t x, uint64_t *lds, uint64_t &total) {
    constexpr int NW = kThreads / kWave;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint64_t incl = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) lds[wave] = incl;
    __syncthreads();
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint64_t s = lds[w];
        if (w < wave) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + incl - x;
}

// SPLIT of a graph with at most kFewBuckets buckets (every graph of up to
// 2^18 vertices): per-thread counts in 16-bit fields of two registers and one
// packed scan give every element its slot, with no LDS atomics (with so few
// buckets, per-element atomics on the counters serialize).  Tile counts fit
// in 16 bits (kTileP = 2^14).
constexpr uint32_t kFewBuckets = 8;
__device__ bool split_few(const BatchArgs &A, const GraphDesc &G, uint32_t t, const int32_t (&v)[kTileP / kThreads],
                          uint32_t *st) {
    const uint32_t nb = G.nb;
    uint64_t c[2] = {0, 0};
#pragma unroll
    for (int j = 0; j < (int)(kTileP / kThreads); ++j) {
        if (v[j] < 0) continue;
        const uint32_t b = (uint32_t)v[j] >> kVB;
        const uint64_t inc = 1ull << (16 * (b & 3));
        if (b < 4) c[0] += inc;
        else c[1] += inc;
    }
    uint64_t tot[2];
    __shared__ uint64_t scan64[kThreads / kWave];
    uint64_t e[2];
    e[0] = block_exclusive_sum64(c[0], scan64, tot[0]);
    e[1] = block_exclusive_sum64(c[1], scan64, tot[1]);
    // bucket b's segment starts at fstart[b], padded to 4 records;
    // fstart[kFewBuckets] = the tile's total
    __shared__ uint32_t fstart[kFewBuckets + 1];
    if (threadIdx.x == 0) {
        uint32_t total = 0;
        for (uint32_t b = 0; b < kFewBuckets; ++b) {
            const uint32_t cb = b < nb ? (uint32_t)(tot[b >> 2] >> (16 * (b & 3))) & 0xFFFFu : 0u;
            fstart[b] = total;
            for (uint32_t q = cb; q < ((cb + 3) & ~3u); ++q) st[total + q] = kSentinel;
            total += (cb + 3) & ~3u;
        }
        fstart[kFewBuckets] = total;
    }
    __syncthreads();
    uint32_t *toff = A.toff_pool + G.toff_off + (size_t)t * (nb + 1);
    if (threadIdx.x <= nb) st_coh(toff + threadIdx.x, fstart[threadIdx.x < nb ? threadIdx.x : kFewBuckets]);
#pragma unroll
    for (int j = 0; j < (int)(kTileP / kThreads); ++j) {
        if (v[j] < 0) continue;
        const uint32_t b = (uint32_t)v[j] >> kVB;
        const uint32_t sh = 16 * (b & 3);
        const uint64_t eb = b < 4 ? e[0] : e[1];
        const uint32_t slot = fstart[b] + ((uint32_t)(eb >> sh) & 0xFFFFu);
        if (b < 4) e[0] = eb + (1ull << sh);
        else e[1] = eb + (1ull << sh);
        const uint32_t o = j * kThreads + threadIdx.x;
        st[slot] = (o << kVB) | ((uint32_t)v[j] & (kBucketV - 1));
    }
    const uint32_t total = fstart[kFewBuckets];
    __syncthreads();
    uint32_t *rec = A.rec_pool + G.rec_off + (size_t)t * G.region;
    for (uint32_t i = threadIdx.x; i < total / 2; i += kThreads) st_coh2(rec + 2 * i, st[2 * i], st[2 * i + 1]);
    return false;
}

// SPLIT: tile t = positions [t * kTileP, +kTileP) of I ++ J.  Records are
// staged in `st` (LDS, fold_region(nb) words), bucket counters in `cnt`
// (2 * kFoldBuckets words).  Records and offsets are written with coherent
// stores: a FOLD item on another XCD reads them.
constexpr int kSplitPer = kTileP / kThreads;  // 16
__device__ bool run_split(const BatchArgs &A, const GraphDesc &G, uint32_t t, uint32_t *st, uint32_t *cnt,
                          uint32_t *lds) {
    const uint32_t n = G.n, m = G.m, nb = G.nb;
    const int32_t *src = A.src + G.edge_off, *dst = A.dst + G.edge_off;
    uint32_t *hist = cnt, *cur = cnt + kFoldBuckets;
    const uint32_t p0 = t * kTileP;
    const uint32_t np = min(kTileP, 2 * m - p0);
    bool bad = false;
    for (uint32_t i = threadIdx.x; i < nb; i += kThreads) hist[i] = 0;
    int32_t v[kSplitPer];
#pragma unroll
    for (int j = 0; j < kSplitPer; ++j) {
        const uint32_t o = j * kThreads + threadIdx.x;
        const uint32_t p = p0 + min(o, np - 1);
        v[j] = __builtin_nontemporal_load(p < m ? src + p : dst + (p - m));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSplitPer; ++j) {
        const uint32_t o = j * kThreads + threadIdx.x;
        if (o >= np) {
            v[j] = -1;
        } else if ((uint32_t)v[j] >= n) {
            bad = true;
            v[j] = -1;
        }
    }
    if (nb <= kFewBuckets) return split_few(A, G, t, v, st) || bad;
#pragma unroll
    for (int j = 0; j < kSplitPer; ++j)
        if (v[j] >= 0) atomicAdd(&hist[(uint32_t)v[j] >> kVB], 1u);
    __syncthreads();
    // segments padded to 4 records; two buckets per thread (nb <= 2 * kThreads)
    const uint32_t b0 = 2 * threadIdx.x;
    const uint32_t c0 = b0 < nb ? hist[b0] : 0u, c1 = b0 + 1 < nb ? hist[b0 + 1] : 0u;
    const uint32_t q0 = (c0 + 3) & ~3u, q1 = (c1 + 3) & ~3u;
    uint32_t total;
    const uint32_t s0 = block_exclusive_scan<kThreads>(q0 + q1, OpSum{}, lds, total);
    uint32_t *toff = A.toff_pool + G.toff_off + (size_t)t * (nb + 1);
    if (b0 < nb) {
        cur[b0] = s0;
        st_coh(toff + b0, s0);
        for (uint32_t q = c0; q < q0; ++q) st[s0 + q] = kSentinel;
    }
    if (b0 + 1 < nb) {
        cur[b0 + 1] = s0 + q0;
        st_coh(toff + b0 + 1, s0 + q0);
        for (uint32_t q = c1; q < q1; ++q) st[s0 + q0 + q] = kSentinel;
    }
    if (threadIdx.x == 0) st_coh(toff + nb, total);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSplitPer; ++j) {
        if (v[j] >= 0) {
            const uint32_t o = j * kThreads + threadIdx.x;
            const uint32_t slot = atomicAdd(&cur[(uint32_t)v[j] >> kVB], 1u);
            st[slot] = (o << kVB) | ((uint32_t)v[j] & (kBucketV - 1));
        }
    }
    __syncthreads();
    uint32_t *rec = A.rec_pool + G.rec_off + (size_t)t * G.region;
    for (uint32_t i = threadIdx.x; i < total / 2; i += kThreads) st_coh2(rec + 2 * i, st[2 * i], st[2 * i + 1]);
    return bad;
}

// FOLD: bucket b over tiles [t0, t1) into LDS r (lr), written to slice s.
constexpr int kFoldU = 4;  // 8-byte loads in flight per lane
__device__ void run_fold(const BatchArgs &A, const GraphDesc &G, uint32_t b, uint32_t t0, uint32_t t1, uint32_t s,
                         uint32_t *lr) {
    const uint32_t n = G.n, nb = G.nb;
    const uint32_t v0 = b * kBucketV;
    const uint32_t cntv = min(kBucketV, n - v0);
    for (uint32_t i = threadIdx.x; i < cntv; i += kThreads) lr[i] = kInf;
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    constexpr uint32_t NW = kThreads / kWave;
    const uint32_t *toff = A.toff_pool + G.toff_off;
    const uint32_t *recs = A.rec_pool + G.rec_off;
    for (uint32_t t = t0 + wave; t < t1; t += NW) {
        // clamped: after a wait that gave up the offsets may not be this launch's
        const uint32_t se = min(ld_coh(toff + (size_t)t * (nb + 1) + b + 1), G.region);
        const uint32_t sb = min(ld_coh(toff + (size_t)t * (nb + 1) + b), se);
        const uint32_t pb = t * kTileP;
        const uint32_t *rt = recs + (size_t)t * G.region;
        for (uint32_t k0 = sb + 2 * lane; k0 < se; k0 += kFoldU * 2 * kWave) {
            uint2 x[kFoldU];
#pragma unroll
            for (int u = 0; u < kFoldU; ++u) {
                const uint32_t k = k0 + u * 2 * kWave;
                x[u] = k < se ? ld_coh2((const uint2 *)(rt + k)) : make_uint2(kSentinel, kSentinel);
            }
#pragma unroll
            for (int u = 0; u < kFoldU; ++u) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t r = h ? x[u].y : x[u].x;
                    if (r == kSentinel) continue;
                    const uint32_t i = r & (kBucketV - 1);
                    const uint32_t p = pb + (r >> kVB);
                    if (p < lr[i]) atomicMin(&lr[i], p);
                }
            }
        }
    }
    __syncthreads();
    uint32_t *out = A.rp_pool + G.rp_off + (size_t)s * n + v0;
    for (uint32_t i = threadIdx.x; i < cntv; i += kThreads) st_coh(out + i, lr[i]);
}

__global__ __launch_bounds__(kThreads) void k_batch(BatchArgs A) {
    __shared__ uint32_t lr[kSmallMax];
    __shared__ uint32_t stage[kThreads * kScanPer];
    __shared__ uint32_t lds[kThreads / kWave];
    __shared__ uint32_t ticket;
    // A workgroup serves the queue of the XCD it runs on, so a graph's items
    // stay on one XCD and its r / bitmap / perm in that XCD's L2.  A
    // workgroup whose queue is empty helps the next queues.
    uint32_t xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    uint32_t q = xcc % kQueues, tried = 0;
    while (true) {
        if (threadIdx.x == 0) ticket = atomicAdd(A.queue + q, 1u);
        __syncthreads();
        const uint32_t t = A.qstart[q] + ticket;
        __syncthreads();
        if (t >= A.qstart[q + 1]) {
            if (++tried == kQueues) break;
            q = (q + 1) % kQueues;
            continue;
        }
        const Item it = A.items[t];
        const GraphDesc G = A.graphs[it.graph];
        const uint32_t n = G.n, m = G.m;
        uint32_t *r = A.r_pool + G.r_off;
        uint2 *W = A.w_pool + G.w_off;
        bool bad = false;
        switch (it.type) {
        case ITEM_SMALL:
            run_small(A, G, lr, lds, stage);
            break;
        case ITEM_SCATTER: {
            // positions p in [begin, end) of I ++ J; probes before atomics
            const int32_t *src = A.src + G.edge_off, *dst = A.dst + G.edge_off;
            for (uint32_t p0 = it.begin + threadIdx.x; p0 < it.end; p0 += kThreads * kU) {
                int32_t v[kU];
                uint32_t cur[kU];
#pragma unroll
                for (int j = 0; j < kU; ++j) {
                    const uint32_t p = min(p0 + j * kThreads, it.end - 1);
                    v[j] = __builtin_nontemporal_load(p < m ? src + p : dst + (p - m));
                }
#pragma unroll
                for (int j = 0; j < kU; ++j) cur[j] = r[(uint32_t)v[j] < n ? (uint32_t)v[j] : 0u];
#pragma unroll
                for (int j = 0; j < kU; ++j) {
                    const uint32_t p = p0 + j * kThreads;
                    if (p >= it.end) break;
                    if ((uint32_t)v[j] < n) {
                        if (p < cur[j]) atomicMin(&r[v[j]], p);
                    } else {
                        bad = true;
                    }
                }
            }
            signal_stage(A, it.graph, ITEM_SCATTER);
            break;
        }
        case ITEM_SPLIT:
            bad = run_split(A, G, it.begin / kTileP, lr, stage, lds);
            signal_stage(A, it.graph, ITEM_SPLIT);
            break;
        case ITEM_FOLD:
            wait_stage(A, it.graph, ITEM_SPLIT, G.need[ITEM_SPLIT]);
            run_fold(A, G, it.bucket, it.begin, it.end, it.slice, lr);
            signal_stage(A, it.graph, ITEM_FOLD);
            break;
        case ITEM_MARK:
            if (G.fold) wait_stage(A, it.graph, ITEM_FOLD, G.need[ITEM_FOLD]);
            else wait_stage(A, it.graph, ITEM_SCATTER, G.need[ITEM_SCATTER]);
            for (uint32_t v0 = it.begin + threadIdx.x; v0 < it.end; v0 += kThreads * kU) {
                uint32_t p[kU];
                if (G.fold) {
                    // r = the minimum over the FOLD slices, kept for RANK
                    const uint32_t *rp = A.rp_pool + G.rp_off;
#pragma unroll
                    for (int j = 0; j < kU; ++j) p[j] = ld_coh(rp + min(v0 + j * kThreads, it.end - 1));
                    for (uint32_t sl = 1; sl < G.slices; ++sl) {
#pragma unroll
                        for (int j = 0; j < kU; ++j)
                            p[j] = min(p[j], ld_coh(rp + (size_t)sl * n + min(v0 + j * kThreads, it.end - 1)));
                    }
#pragma unroll
                    for (int j = 0; j < kU; ++j)
                        if (v0 + j * kThreads < it.end) st_coh(r + v0 + j * kThreads, p[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < kU; ++j) p[j] = ld_coh(r + min(v0 + j * kThreads, it.end - 1));
                }
#pragma unroll
                for (int j = 0; j < kU; ++j) {
                    const uint32_t v = v0 + j * kThreads;
                    if (v >= it.end) break;
                    const uint32_t key = p[j] == kInf ? 2 * m + v : p[j];
                    atomicOr(&W[key >> 5].x, 1u << (key & 31));
                }
            }
            signal_stage(A, it.graph, ITEM_MARK);
            break;
        case ITEM_SCAN:
            wait_stage(A, it.graph, ITEM_MARK, G.need[ITEM_MARK]);
            scan_bitmap(W, G.nw, lds, stage);
            signal_stage(A, it.graph, ITEM_SCAN);
            break;
        case ITEM_RANK: {
            wait_stage(A, it.graph, ITEM_SCAN, 1);
            int32_t *perm = A.perm + G.vert_off;
            int32_t *pcopy = A.p_pool + G.p_off;
            int32_t *order = A.order ? A.order + G.vert_off : nullptr;
            for (uint32_t v0 = it.begin + threadIdx.x; v0 < it.end; v0 += kThreads * kU) {
                uint32_t key[kU];
                uint2 w[kU];
#pragma unroll
                for (int j = 0; j < kU; ++j) {
                    const uint32_t v = min(v0 + j * kThreads, it.end - 1);
                    const uint32_t p = ld_coh(r + v);
                    key[j] = p == kInf ? 2 * m + v : p;
                }
#pragma unroll
                for (int j = 0; j < kU; ++j) w[j] = ld_coh2(W + (key[j] >> 5));
#pragma unroll
                for (int j = 0; j < kU; ++j) {
                    const uint32_t v = v0 + j * kThreads;
                    if (v >= it.end) break;
                    const uint32_t k = w[j].y + __popc(w[j].x & ((1u << (key[j] & 31)) - 1u));
                    perm[v] = (int32_t)k;
                    st_coh((uint32_t *)pcopy + v, k);
                    if (order && k < n) order[k] = (int32_t)v;
                }
            }
            signal_stage(A, it.graph, ITEM_RANK);
            break;
        }
        case ITEM_RELABEL: {
            wait_stage(A, it.graph, ITEM_RANK, G.need[ITEM_RANK]);
            const int32_t *src = A.src + G.edge_off, *dst = A.dst + G.edge_off;
            // the graph's own line-aligned perm copy: no L2 holds its lines
            // before RANK finished, so cached plain loads are safe here
            const int32_t *perm = A.p_pool + G.p_off;
            int32_t *so = A.src_out + G.edge_off, *dso = A.dst_out + G.edge_off;
            for (uint32_t k0 = it.begin + threadIdx.x; k0 < it.end; k0 += kThreads * kU) {
                int32_t a[kU], b[kU], pa[kU], pb[kU];
#pragma unroll
                for (int j = 0; j < kU; ++j) {
                    const uint32_t k = min(k0 + j * kThreads, it.end - 1);
                    a[j] = __builtin_nontemporal_load(src + k);
                    b[j] = __builtin_nontemporal_load(dst + k);
                }
#pragma unroll
                for (int j = 0; j < kU; ++j) {
                    pa[j] = perm[(uint32_t)a[j] < n ? (uint32_t)a[j] : 0u];
                    pb[j] = perm[(uint32_t)b[j] < n ? (uint32_t)b[j] : 0u];
                }
#pragma unroll
                for (int j = 0; j < kU; ++j) {
                    const uint32_t k = k0 + j * kThreads;
                    if (k >= it.end) break;
                    __builtin_nontemporal_store((uint32_t)a[j] < n ? pa[j] : a[j], so + k);
                    __builtin_nontemporal_store((uint32_t)b[j] < n ? pb[j] : b[j], dso + k);
                }
            }
            break;
        }
        default:
            break;
        }
        if (bad) flag_range_error(A.flag);
        __syncthreads();
    }
}

// r = inf for large graphs, bitmaps and counters = 0 (replayed before every run).
__global__ __launch_bounds__(256) void k_batch_init(uint32_t *__restrict__ r, uint64_t nr, uint2 *__restrict__ w,
                                                    uint64_t nw, uint32_t *__restrict__ counters, uint32_t nc) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    const uint64_t i0 = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    for (uint64_t i = i0; i < nr; i += stride) r[i] = kInf;
    for (uint64_t i = i0; i < nw; i += stride) w[i] = make_uint2(0u, 0u);
    for (uint64_t i = i0; i < nc; i += stride) counters[i] = 0;
}

}  // namespace
}  // namespace boba

using namespace boba;

struct boba_batch_plan {
    int32_t G;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int device;
    uint32_t n_items, n_small;
    uint64_t r_words, w_words;
};

namespace {

struct HostPlan {
    std::vector<GraphDesc> graphs;
    std::vector<Item> items;
    uint32_t qstart[kQueues + 1] = {};
    uint64_t r_words = 0, w_words = 0, p_words = 0;
    uint64_t rec_words = 0, toff_words = 0, rp_words = 0;
    uint32_t n_small = 0;
};

boba_status build_host_plan(int32_t G, const int64_t *eo, const int64_t *vo, bool relabel, const boba_tuning *tu,
                            HostPlan &H) {
    const uint32_t small_max = tu && tu->small_max_n > 0 ? (uint32_t)std::min<int64_t>(tu->small_max_n, kSmallMax)
                                                         : kSmallMax;
    const uint32_t scatter_tile = tu && tu->scatter_tile > 0 ? (uint32_t)tu->scatter_tile : 262144u;
    const uint32_t vertex_tile = tu && tu->vertex_tile > 0 ? (uint32_t)tu->vertex_tile : 65536u;
    const uint32_t relabel_tile = tu && tu->relabel_tile > 0 ? (uint32_t)tu->relabel_tile : 262144u;
    const uint32_t nq = tu && tu->queues > 0 ? (uint32_t)std::min<int32_t>(tu->queues, (int32_t)kQueues) : kQueues;
    const bool atomic_scatter = tu && tu->scatter_atomic > 0;
    H.graphs.resize(G);
    std::vector<int32_t> big, small;
    for (int32_t g = 0; g < G; ++g) {
        const int64_t m = eo[g + 1] - eo[g], n = vo[g + 1] - vo[g];
        if (m < 0 || n < 0) return fail(BOBA_ERR_ARG, "batch: offsets of graph %d decrease", g);
        if (m >= (1ll << 31) || n >= (1ll << 31) || 2 * m + n >= (1ll << 32))
            return fail(BOBA_ERR_OVERFLOW, "batch: graph %d too large (m=%lld, n=%lld)", g, (long long)m,
                        (long long)n);
        if (m > 0 && n == 0) return fail(BOBA_ERR_ARG, "batch: graph %d has edges but no vertices", g);
        GraphDesc &D = H.graphs[g];
        memset(&D, 0, sizeof(D));
        D.edge_off = eo[g];
        D.vert_off = vo[g];
        D.m = (uint32_t)m;
        D.n = (uint32_t)n;
        D.nw = ceil_div(2 * (uint64_t)m + (uint64_t)n, 32);
        D.w_off = (int64_t)H.w_words;
        H.w_words += D.nw;
        if (n == 0) continue;
        if ((uint32_t)n <= small_max) {
            small.push_back(g);
        } else {
            D.r_off = (int64_t)H.r_words;
            H.r_words += (uint64_t)n;
            D.p_off = (int64_t)H.p_words;
            H.p_words += ((uint64_t)n + 63) & ~63ull;  // 256-byte lines of its own
            const uint32_t nb = (uint32_t)ceil_div((uint64_t)n, kBucketV);
            if (!atomic_scatter && m > 0 && nb <= kFoldBuckets) {
                D.fold = 1;
                D.nb = nb;
                D.tiles = (uint32_t)ceil_div(2 * (uint64_t)m, kTileP);
                D.region = fold_region(nb);
                // slices of about scatter_tile records per (bucket, slice)
                uint64_t sl = ceil_div(2 * (uint64_t)m, (uint64_t)nb * scatter_tile);
                sl = std::min<uint64_t>({std::max<uint64_t>(sl, 1), kMaxSlices, D.tiles});
                const uint32_t ft = (uint32_t)ceil_div(D.tiles, sl);
                D.slices = (uint32_t)ceil_div(D.tiles, ft);
                D.fold_tiles = ft;
                D.rec_off = (int64_t)H.rec_words;
                H.rec_words += (uint64_t)D.tiles * D.region;
                D.toff_off = (int64_t)H.toff_words;
                H.toff_words += (uint64_t)D.tiles * (nb + 1);
                D.rp_off = (int64_t)H.rp_words;
                H.rp_words += (uint64_t)D.slices * (uint64_t)n;
            }
            big.push_back(g);
        }
    }
    // larger work first (longest-processing-time order), graphs dealt to the
    // least-loaded queue
    auto by_m = [&](int32_t a, int32_t b) { return H.graphs[a].m > H.graphs[b].m || (H.graphs[a].m == H.graphs[b].m && a < b); };
    std::sort(big.begin(), big.end(), by_m);
    std::sort(small.begin(), small.end(), by_m);
    // queues past nq stay empty (their workgroups help the others)
    std::vector<uint64_t> load(nq, 0);
    std::vector<std::vector<int32_t>> qbig(kQueues), qsmall(kQueues);
    auto deal = [&](int32_t g, std::vector<std::vector<int32_t>> &dst) {
        const size_t q = std::min_element(load.begin(), load.end()) - load.begin();
        load[q] += 2ull * H.graphs[g].m + H.graphs[g].n + 1;
        dst[q].push_back(g);
    };
    for (int32_t g : big) deal(g, qbig);
    for (int32_t g : small) deal(g, qsmall);
    auto tiles = [&](uint32_t type, int32_t g, uint64_t count, uint32_t tile) {
        uint32_t k = 0;
        for (uint64_t b = 0; b < count; b += tile, ++k)
            H.items.push_back(Item{type, (uint32_t)g, (uint32_t)b, (uint32_t)std::min<uint64_t>(count, b + tile)});
        H.graphs[g].need[type] = k;
    };
    for (uint32_t q = 0; q < kQueues; ++q) {
        H.qstart[q] = (uint32_t)H.items.size();
        for (int32_t g : qbig[q]) {
            if (H.graphs[g].fold) tiles(ITEM_SPLIT, g, 2ull * H.graphs[g].m, kTileP);
            else tiles(ITEM_SCATTER, g, 2ull * H.graphs[g].m, scatter_tile);
        }
        for (int32_t g : qsmall[q]) H.items.push_back(Item{ITEM_SMALL, (uint32_t)g, 0, 0});
        for (int32_t g : qbig[q]) {
            GraphDesc &D = H.graphs[g];
            if (!D.fold) continue;
            for (uint32_t b = 0; b < D.nb; ++b)
                for (uint32_t sl = 0; sl < D.slices; ++sl)
                    H.items.push_back(Item{ITEM_FOLD, (uint32_t)g, sl * D.fold_tiles, std::min(D.tiles, (sl + 1) * D.fold_tiles), b, sl});
            D.need[ITEM_FOLD] = D.nb * D.slices;
        }
        for (int32_t g : qbig[q]) tiles(ITEM_MARK, g, H.graphs[g].n, vertex_tile);
        for (int32_t g : qbig[q]) tiles(ITEM_SCAN, g, 1, 1);
        for (int32_t g : qbig[q]) tiles(ITEM_RANK, g, H.graphs[g].n, vertex_tile);
        if (relabel)
            for (int32_t g : qbig[q]) tiles(ITEM_RELABEL, g, H.graphs[g].m, relabel_tile);
    }
    H.qstart[kQueues] = (uint32_t)H.items.size();
    H.n_small = (uint32_t)small.size();
    return BOBA_OK;
}

struct BatchLayout {
    GraphDesc *graphs;
    Item *items;
    uint32_t *queue_and_done;
    uint32_t *r;
    uint2 *w;
    int32_t *p;
    uint32_t *rec, *toff, *rp;
    size_t bytes;
};

BatchLayout batch_layout(void *ws, const HostPlan &H) {
    BatchLayout L;
    Carver c(ws);
    L.graphs = c.take<GraphDesc>(H.graphs.size());
    L.items = c.take<Item>(H.items.size());
    L.queue_and_done = c.take<uint32_t>(kQueues + 1 + kStages * H.graphs.size());
    L.r = c.take<uint32_t>(H.r_words);
    L.w = c.take<uint2>(H.w_words);
    L.p = c.take<int32_t>(H.p_words);
    L.rec = c.take<uint32_t>(H.rec_words);
    L.toff = c.take<uint32_t>(H.toff_words);
    L.rp = c.take<uint32_t>(H.rp_words);
    L.bytes = c.bytes();
    return L;
}

}  // namespace

extern "C" size_t boba_batch_workspace(int32_t G, const int64_t *h_edge_off, const int64_t *h_vert_off,
                                       const boba_tuning *tuning) {
    if (G < 0 || (G > 0 && (!h_edge_off || !h_vert_off))) return 0;
    HostPlan H;
    if (build_host_plan(G, h_edge_off, h_vert_off, true, tuning, H) != BOBA_OK) return 0;
    return batch_layout(nullptr, H).bytes;
}

extern "C" boba_status boba_batch_plan_create(int32_t G, const int64_t *h_edge_off, const int64_t *h_vert_off,
                                              const int32_t *src, const int32_t *dst, int32_t *perm, int32_t *order,
                                              int32_t *src_out, int32_t *dst_out, void *ws, size_t ws_bytes,
                                              const boba_tuning *tuning, hipStream_t stream,
                                              boba_batch_plan **plan) {
    clear_error();
    if (!plan) return fail(BOBA_ERR_ARG, "batch: plan is NULL");
    *plan = nullptr;
    if (G < 0 || (G > 0 && (!h_edge_off || !h_vert_off))) return fail(BOBA_ERR_ARG, "batch: bad graph offsets");
    if ((src_out == nullptr) != (dst_out == nullptr))
        return fail(BOBA_ERR_ARG, "batch: src_out and dst_out must both be given or both be NULL");
    if (G > 0 && (h_edge_off[0] != 0 || h_vert_off[0] != 0)) return fail(BOBA_ERR_ARG, "batch: offsets must start at 0");
    const int64_t M = G > 0 ? h_edge_off[G] : 0, N = G > 0 ? h_vert_off[G] : 0;
    if (M >= (1ll << 31) || N >= (1ll << 31)) return fail(BOBA_ERR_OVERFLOW, "batch: totals must be < 2^31");
    if (M > 0 && (!src || !dst)) return fail(BOBA_ERR_ARG, "batch: src/dst is NULL");
    if (N > 0 && !perm) return fail(BOBA_ERR_ARG, "batch: perm is NULL");
    HostPlan H;
    if (boba_status e = build_host_plan(G, h_edge_off, h_vert_off, src_out != nullptr, tuning, H)) return e;
    const BatchLayout L = batch_layout(ws, H);
    if (!ws || ws_bytes < L.bytes || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "batch: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)",
                    L.bytes, ws_bytes, ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(BOBA_ERR_HIP, "batch: cannot query the device");

    // the plan's tables live in the caller's workspace; copy them once
    hipError_t e = hipMemcpyAsync(L.graphs, H.graphs.data(), H.graphs.size() * sizeof(GraphDesc),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !H.items.empty())
        e = hipMemcpyAsync(L.items, H.items.data(), H.items.size() * sizeof(Item), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(BOBA_ERR_HIP, "batch: table upload failed: %s", hipGetErrorString(e));

    BatchArgs A;
    A.src = src;
    A.dst = dst;
    A.perm = perm;
    A.order = order;
    A.src_out = src_out;
    A.dst_out = dst_out;
    A.graphs = L.graphs;
    A.items = L.items;
    for (uint32_t q = 0; q <= kQueues; ++q) A.qstart[q] = H.qstart[q];
    A.queue = L.queue_and_done;
    A.abort = L.queue_and_done + kQueues;
    A.done = L.queue_and_done + kQueues + 1;
    const uint32_t n_items = (uint32_t)H.items.size();
    A.r_pool = L.r;
    A.w_pool = L.w;
    A.p_pool = L.p;
    A.rec_pool = L.rec;
    A.toff_pool = L.toff;
    A.rp_pool = L.rp;
    A.flag = flag;
    A.spin_limit = tuning && tuning->spin_limit > 0 ? (uint32_t)tuning->spin_limit : kSpinLimit;

    // capture: init node + persistent kernel (one workgroup per CU)
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(BOBA_ERR_HIP, "batch: stream create failed: %s", hipGetErrorString(e));
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const uint32_t nc = kQueues + 1 + kStages * (uint32_t)G;
        hipLaunchKernelGGL(k_batch_init, dim3(grid_for(std::max<uint64_t>({H.r_words, H.w_words, (uint64_t)nc}), 1024)),
                           dim3(256), 0, cap, L.r, H.r_words, L.w, H.w_words, L.queue_and_done, nc);
        if (n_items > 0)
            hipLaunchKernelGGL(k_batch, dim3(std::max(1, cus)), dim3(kThreads), 0, cap, A);
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        e = e2 != hipSuccess ? e2 : hipGetLastError();
    }
    hipStreamDestroy(cap);
    if (e != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return fail(BOBA_ERR_HIP, "batch: graph capture failed: %s", hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return fail(BOBA_ERR_HIP, "batch: graph instantiate failed: %s", hipGetErrorString(e));
    }
    boba_batch_plan *P = (boba_batch_plan *)calloc(1, sizeof(boba_batch_plan));
    if (!P) {
        hipGraphExecDestroy(exec);
        hipGraphDestroy(graph);
        return fail(BOBA_ERR_ARG, "batch: out of host memory");
    }
    P->G = G;
    P->graph = graph;
    P->exec = exec;
    P->device = dev;
    P->n_items = n_items;
    P->n_small = H.n_small;
    P->r_words = H.r_words;
    P->w_words = H.w_words;
    *plan = P;
    return BOBA_OK;
}

extern "C" boba_status boba_batch_plan_launch(boba_batch_plan *plan, hipStream_t stream) {
    clear_error();
    if (!plan) return fail(BOBA_ERR_ARG, "batch: plan is NULL");
    const int tok = timing_begin("batch_graph", stream);
    hipError_t e = hipGraphLaunch(plan->exec, stream);
    timing_end(tok, stream);
    if (e != hipSuccess) return fail(BOBA_ERR_HIP, "batch: graph launch failed: %s", hipGetErrorString(e));
    return BOBA_OK;
}

extern "C" boba_status boba_batch_plan_info(const boba_batch_plan *plan, int64_t *info4) {
    clear_error();
    if (!plan || !info4) return fail(BOBA_ERR_ARG, "batch: NULL argument");
    info4[0] = plan->n_items;
    info4[1] = plan->n_small;
    info4[2] = (int64_t)plan->r_words;
    info4[3] = (int64_t)plan->w_words;
    return BOBA_OK;
}

extern "C" boba_status boba_batch_plan_destroy(boba_batch_plan *plan) {
    clear_error();
    if (!plan) return BOBA_OK;
    if (plan->exec) hipGraphExecDestroy(plan->exec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    free(plan);
    return BOBA_OK;
}

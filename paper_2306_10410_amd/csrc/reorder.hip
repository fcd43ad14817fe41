// BOBA reordering (Sec. 4.4, Algorithm 2 with AtomicMin) and edge relabelling.
//
// Pipeline of boba_reorder on one stream:
//   init      r[v] <- inf, bitmap <- 0
//   scatter   for every position i of the flattened edge list S = I ++ J,
//             r[S[i]] <- min(r[S[i]], i)          (Algorithm 2, lines with r)
//   mark      key(v) = r[v], or 2m + v when v never occurs (tail); set bit
//             key(v) in a bitmap over [0, 2m + n)
//   scan      prefix popcount of the bitmap words      } ParMapKeys: the rank
//   rank      perm[v] = number of set bits before key(v) } of each unique key
// The bitmap holds, per 32 positions, {bits, exclusive prefix popcount} as one
// uint2 so that rank needs one 8-byte load per vertex.
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
template <int K>
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
            if (pos[q] < cur[q]) atomicMin(&r[v[q]], pos[q]);
        } else {
            flag_range_error(flag);
        }
    }
}

__device__ __forceinline__ void visit(uint32_t *__restrict__ r, int32_t v, uint32_t pos, uint32_t n,
                                      int32_t *flag) {
    if ((uint32_t)v < n) {
        if (pos < r[v]) atomicMin(&r[v], pos);
    } else {
        flag_range_error(flag);
    }
}

// Chunk c < m4 covers src[4c .. 4c+3]; chunk c >= m4 covers dst[4(c-m4) .. +3].
template <bool INTERLEAVED>
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
    visit_all(r, v, pos, live, n, flag);
}

// Edges k in [k0, m): both endpoints, scalar loads (tails and unaligned input).
template <bool INTERLEAVED>
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
        visit(r, is_dst ? dst[k] : src[k], pos, n, flag);
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

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

struct ReorderLayout {
    uint32_t *r;
    uint2 *W;
    uint32_t *partial;
    size_t bytes;
    uint32_t nw;
};

ReorderLayout reorder_layout(void *ws, int64_t n, int64_t m) {
    ReorderLayout L;
    const uint64_t positions = 2 * (uint64_t)m + (uint64_t)n;
    L.nw = ceil_div(positions, 32);
    Carver c(ws);
    L.r = c.take<uint32_t>((size_t)n);
    L.W = c.take<uint2>(L.nw);
    L.partial = c.take<uint32_t>(scan_partials(L.nw));
    L.bytes = c.bytes();
    return L;
}

boba_status check_sizes(int64_t m, int64_t n, bool positions) {
    if (m < 0 || n < 0) return fail(BOBA_ERR_ARG, "negative size (m=%lld, n=%lld)", (long long)m, (long long)n);
    if (m >= (1ll << 31) || n >= (1ll << 31))
        return fail(BOBA_ERR_OVERFLOW, "m and n must be < 2^31 (m=%lld, n=%lld)", (long long)m, (long long)n);
    if (positions && 2 * m + n >= (1ll << 32))
        return fail(BOBA_ERR_OVERFLOW, "2m + n must be < 2^32 (m=%lld, n=%lld)", (long long)m, (long long)n);
    return BOBA_OK;
}

}  // namespace
}  // namespace boba

using namespace boba;

extern "C" size_t boba_reorder_workspace(int64_t n, int64_t m) {
    if (n < 0 || m < 0) return 0;
    return reorder_layout(nullptr, n, m).bytes;
}

extern "C" boba_status boba_reorder(const int32_t *src, const int32_t *dst, int64_t m, int64_t n, int32_t *perm,
                                    int32_t *order, void *ws, size_t ws_bytes, uint32_t flags, hipStream_t stream) {
    clear_error();
    if (boba_status e = check_sizes(m, n, true)) return e;
    if (flags & ~BOBA_FLAG_INTERLEAVED) return fail(BOBA_ERR_ARG, "boba_reorder: unknown flags 0x%x", flags);
    if (m > 0 && (!src || !dst)) return fail(BOBA_ERR_ARG, "boba_reorder: src/dst is NULL");
    if (m > 0 && n == 0) return fail(BOBA_ERR_ARG, "boba_reorder: edges given but n = 0");
    if (n == 0) return BOBA_OK;
    if (!perm) return fail(BOBA_ERR_ARG, "boba_reorder: perm is NULL");
    const size_t need = boba_reorder_workspace(n, m);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "boba_reorder: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)",
                    need, ws_bytes, ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;

    const bool inter = flags & BOBA_FLAG_INTERLEAVED;
    const uint32_t un = (uint32_t)n, um = (uint32_t)m;
    ReorderLayout L = reorder_layout(ws, n, m);

    BOBA_LAUNCH("reorder_init", k_reorder_init, dim3(grid_for(un > L.nw ? un : L.nw, kBlock * 4)), dim3(kBlock),
                stream, L.r, un, L.W, L.nw);

    uint32_t k0 = 0;
    if (m > 0 && aligned16(src) && aligned16(dst)) {
        const uint32_t m4 = um / 4;
        if (m4 > 0) {
            dim3 grid(ceil_div(2ull * m4, kScatterTile));
            if (inter)
                BOBA_LAUNCH("scatter_min", k_scatter_min_vec<true>, grid, dim3(kBlock), stream, (const v4i *)src,
                            (const v4i *)dst, m4, um, un, L.r, flag);
            else
                BOBA_LAUNCH("scatter_min", k_scatter_min_vec<false>, grid, dim3(kBlock), stream, (const v4i *)src,
                            (const v4i *)dst, m4, um, un, L.r, flag);
        }
        k0 = 4 * m4;
    }
    if (k0 < um) {
        dim3 grid(grid_for(2ull * (um - k0), kBlock));
        if (inter)
            BOBA_LAUNCH("scatter_min_scalar", k_scatter_min_scalar<true>, grid, dim3(kBlock), stream, src, dst, k0, um,
                        un, L.r, flag);
        else
            BOBA_LAUNCH("scatter_min_scalar", k_scatter_min_scalar<false>, grid, dim3(kBlock), stream, src, dst, k0,
                        um, un, L.r, flag);
    }

    const uint32_t tail = 2 * um;
    BOBA_LAUNCH("mark", k_mark, dim3(grid_for(un, kBlock * 4)), dim3(kBlock), stream, (const uint32_t *)L.r, un, tail,
                L.W);
    if (boba_status e = device_scan<OpSum, false>("bitmap_scan", LoadPopc{L.W}, StorePrefix{L.W}, L.nw, L.partial, stream))
        return e;
    BOBA_LAUNCH("rank", k_rank, dim3(grid_for(un, kBlock * 4)), dim3(kBlock), stream, (const uint32_t *)L.r, un, tail,
                (const uint2 *)L.W, perm, order);
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
    const uint32_t um = (uint32_t)m, un = (uint32_t)n;
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

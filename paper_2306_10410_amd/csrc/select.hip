// Reorder selector (not in the paper): 16 cheap graph features and a
// 16-64-64-1 ReLU MLP with its training kernels (mean squared error, Adam).
//
// Features use K = 4096 spread samples p_k = floor(k m / K) and 64 windows of
// L = min(1024, m) consecutive edges starting at floor(w (m - L) / 63):
//   0 log2(1+n)  1 log2(1+m)  2 log2(1 + m/max(n,1))
//   3,4  log2(1 + n * C / (K(K-1)/2)), C = equal pairs among src (dst) samples
//   5,6  log2(1 + n * maxcount / K)       7,8  distinct / K
//   9    mean over windows of sum |src-dst| / (L n)
//   10,11 mean over windows of #distinct (id >> 5) / L   (src, dst)
//   12,13 mean over windows of #(id_e == id_{e-1}) / (L-1)
//   14,15 mean over windows of #(|id_e - id_{e-1}| < 32) / (L-1)
// Counts are exact integers (equal samples and distinct lines are counted in
// LDS hash tables); the final combination is done in FP64 in a fixed order and
// rounded to FP32.  No value is used as an index, so any input is safe.
//
// MLP parameters, row-major, FP32: W1[64][16] b1[64] W2[64][64] b2[64] W3[1][64] b3[1].
// Forward: one wavefront per sample, a lane per hidden unit.  Backward: per-sample
// activations and deltas, then one thread per parameter summing over the batch
// in sample order (deterministic).  Adam: elementwise with bias correction.
#include <math.h>

#include "internal.h"

namespace boba {
namespace {

constexpr int kSpread = 4096;
constexpr int kWin = 64;
constexpr int kWinLen = 1024;
constexpr int kT = 1024;  // threads of the feature kernels

// per-window counters, then per-spread-side counters (uint64 each)
constexpr int kWinStats = 7;    // absdiff, lines src, lines dst, eq src, eq dst, near src, near dst
constexpr int kSpreadStats = 3; // collisions, max count, distinct
constexpr size_t kFeatWsWords = (size_t)kWin * kWinStats + 2 * kSpreadStats;

__device__ uint64_t block_sum64(uint64_t x, uint64_t *lds) {
    for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane == 0) lds[wave] = x;
    __syncthreads();
    uint64_t t = 0;
    for (int w = 0; w < kT / kWave; ++w) t += lds[w];
    __syncthreads();
    return t;
}

__device__ uint32_t block_max32(uint32_t x, uint32_t *lds) {
    for (int d = kWave / 2; d >= 1; d >>= 1) x = max(x, (uint32_t)__shfl_xor(x, d, kWave));
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane == 0) lds[wave] = x;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < kT / kWave; ++w) t = max(t, lds[w]);
    __syncthreads();
    return t;
}

// Exact counting with open-addressing hash tables in LDS (linear probing; a
// table has at least twice as many slots as keys, so every insert ends).
__device__ __forceinline__ uint32_t fib_hash(uint32_t k, int bits) { return (k * 0x9E3779B1u) >> (32 - bits); }

constexpr int kSpreadBits = 13;  // 8192 slots for 4096 samples
constexpr int kWinBits = 11;     // 2048 slots for <= 1024 keys
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;
constexpr unsigned long long kEmpty64 = ~0ull;

// Workgroups 0 .. kWin-1: windows; kWin, kWin+1: spread samples of src, dst.
// One launch; every workgroup writes its own counters.
__global__ __launch_bounds__(kT) void k_feat_stats(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                                                   uint32_t m, uint64_t *__restrict__ out) {
    __shared__ unsigned long long key[1 << kSpreadBits];  // spread keys; windows use the first words as uint32
    __shared__ uint32_t cnt[1 << kSpreadBits];
    __shared__ uint64_t red[kT / kWave];
    __shared__ uint32_t red32[kT / kWave];
    const uint32_t t = threadIdx.x;
    if (blockIdx.x < kWin) {
        uint32_t *tab = (uint32_t *)key;  // two tables of 2^kWinBits words
        for (uint32_t i = t; i < (2u << kWinBits); i += kT) tab[i] = kEmpty32;
        const uint32_t L = min((uint32_t)kWinLen, m);
        const uint32_t s0 = (uint32_t)(((uint64_t)blockIdx.x * (m - L)) / (kWin - 1));
        const bool live = t < L;
        const int32_t vs = live ? src[s0 + t] : 0, vd = live ? dst[s0 + t] : 0;
        const int32_t ps = live && t > 0 ? src[s0 + t - 1] : 0, pd = live && t > 0 ? dst[s0 + t - 1] : 0;
        uint64_t st[kWinStats];
        st[0] = live ? (uint64_t)llabs((long long)vs - (long long)vd) : 0;
        const bool pair = live && t > 0;
        st[3] = pair && vs == ps;
        st[4] = pair && vd == pd;
        st[5] = pair && llabs((long long)vs - (long long)ps) < 32;
        st[6] = pair && llabs((long long)vd - (long long)pd) < 32;
        __syncthreads();
        // distinct cache lines (id >> 5 < 2^27, never the empty marker)
        for (int side = 0; side < 2; ++side) {
            uint32_t *tb = tab + (side << kWinBits);
            uint32_t fresh = 0;
            if (live) {
                const uint32_t k = (uint32_t)(side == 0 ? vs : vd) >> 5;
                uint32_t h = fib_hash(k, kWinBits);
                while (true) {
                    const uint32_t prev = atomicCAS(&tb[h], kEmpty32, k);
                    if (prev == kEmpty32) {
                        fresh = 1;
                        break;
                    }
                    if (prev == k) break;
                    h = (h + 1) & ((1u << kWinBits) - 1);
                }
            }
            st[1 + side] = fresh;
        }
        uint64_t *o = out + (size_t)blockIdx.x * kWinStats;
        for (int q = 0; q < kWinStats; ++q) {
            const uint64_t tot = block_sum64(st[q], red);
            if (t == 0) o[q] = tot;
        }
        return;
    }
    const uint32_t side = blockIdx.x - kWin;
    const int32_t *arr = side == 0 ? src : dst;
    for (uint32_t i = t; i < (1u << kSpreadBits); i += kT) {
        key[i] = kEmpty64;
        cnt[i] = 0;
    }
    __syncthreads();
    for (uint32_t k = t; k < (uint32_t)kSpread; k += kT) {
        const unsigned long long v = (uint32_t)arr[((uint64_t)k * m) / kSpread];
        uint32_t h = fib_hash((uint32_t)v, kSpreadBits);
        while (true) {
            const unsigned long long prev = atomicCAS(&key[h], kEmpty64, v);
            if (prev == kEmpty64 || prev == v) {
                atomicAdd(&cnt[h], 1u);
                break;
            }
            h = (h + 1) & ((1u << kSpreadBits) - 1);
        }
    }
    __syncthreads();
    uint64_t coll = 0, distinct = 0;
    uint32_t mx = 0;
    for (uint32_t i = t; i < (1u << kSpreadBits); i += kT) {
        const uint64_t c = cnt[i];
        coll += c * (c - (c > 0)) / 2;  // c (c - 1) / 2 equal pairs
        distinct += c > 0;
        mx = max(mx, (uint32_t)c);
    }
    coll = block_sum64(coll, red);
    distinct = block_sum64(distinct, red);
    mx = block_max32(mx, red32);
    if (t == 0) {
        uint64_t *o = out + (size_t)kWin * kWinStats + side * kSpreadStats;
        o[0] = coll;
        o[1] = mx;
        o[2] = distinct;
    }
}

// One wavefront: lane w < 64 holds window w's counters; their sums over the
// windows are exact integers (wavefront reductions), so each mean is one FP64
// division of an exact count; lane 0 combines everything.
__global__ __launch_bounds__(kWave) void k_feat_final(const uint64_t *__restrict__ st, uint32_t m, uint32_t n,
                                                      float *__restrict__ f) {
    static_assert(kWin == kWave, "one window per lane");
    const uint32_t lane = threadIdx.x;
    uint64_t sum[kWinStats];
#pragma unroll
    for (int q = 0; q < kWinStats; ++q) {
        uint64_t x = m > 0 ? st[(size_t)lane * kWinStats + q] : 0;
        for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
        sum[q] = x;
    }
    if (lane != 0) return;
    const double dn = (double)n, dm = (double)m;
    double F[16] = {};
    F[0] = log2(1.0 + dn);
    F[1] = log2(1.0 + dm);
    F[2] = log2(1.0 + dm / (n > 0 ? dn : 1.0));
    if (m > 0) {
        const double P = (double)kSpread * (kSpread - 1) / 2.0;
        for (int side = 0; side < 2; ++side) {
            const uint64_t *sp = st + (size_t)kWin * kWinStats + side * kSpreadStats;
            F[3 + side] = log2(1.0 + dn * (double)sp[0] / P);
            F[5 + side] = log2(1.0 + dn * (double)sp[1] / kSpread);
            F[7 + side] = (double)sp[2] / kSpread;
        }
        const double L = (double)min((uint32_t)kWinLen, m);
        F[9] = (double)sum[0] / (L * (n > 0 ? dn : 1.0) * kWin);
        F[10] = (double)sum[1] / (L * kWin);
        F[11] = (double)sum[2] / (L * kWin);
        if (L > 1) {
            for (int q = 3; q < 7; ++q) F[9 + q] = (double)sum[q] / ((L - 1.0) * kWin);
        }
    }
    for (int q = 0; q < 16; ++q) f[q] = (float)F[q];
}

// ----------------------------------------------------------------------- MLP
constexpr int IN = 16, H = 64;
constexpr int OW1 = 0, OB1 = OW1 + H * IN, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int NP = OB3 + 1;  // 5313
constexpr int kMT = 256;

// One wavefront per sample, lane o owning hidden unit o of both layers: each
// dot product runs in input order in its lane, the output sums the 64 lanes'
// terms with a fixed shuffle tree.  The weights come straight from global
// memory (21 KB, cache-resident after the first sample).
constexpr int kFwdWaves = kMT / kWave;  // samples per workgroup

__global__ __launch_bounds__(kMT) void k_mlp_forward(const float *__restrict__ P, const float *__restrict__ X,
                                                     int32_t B, float *__restrict__ yhat) {
    static_assert(H == kWave, "one hidden unit per lane");
    __shared__ float h1s[kFwdWaves][H];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int b = blockIdx.x * kFwdWaves + wave;
    if (b >= B) return;  // wave-uniform; no barrier follows
    float x[IN];
#pragma unroll
    for (int i = 0; i < IN; ++i) x[i] = X[(size_t)b * IN + i];
    float s = P[OB1 + lane];
#pragma unroll
    for (int i = 0; i < IN; ++i) s = fmaf(P[OW1 + lane * IN + i], x[i], s);
    h1s[wave][lane] = s > 0.f ? s : 0.f;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float z = P[OB2 + lane];
#pragma unroll 16
    for (int i = 0; i < H; ++i) z = fmaf(P[OW2 + lane * H + i], h1s[wave][i], z);
    float t = P[OW3 + lane] * (z > 0.f ? z : 0.f);
    for (int d = kWave / 2; d >= 1; d >>= 1) t += __shfl_xor(t, d, kWave);
    if (lane == 0) yhat[b] = P[OB3] + t;
}

// Per sample: h1, h2 and the deltas g1 = dL/dz1, g2 = dL/dz2, go = dL/dout.
__global__ __launch_bounds__(kMT) void k_mlp_back_sample(const float *__restrict__ P, const float *__restrict__ X,
                                                         const float *__restrict__ y, int32_t B,
                                                         float *__restrict__ h1o, float *__restrict__ h2o,
                                                         float *__restrict__ g1o, float *__restrict__ g2o,
                                                         float *__restrict__ goo, float *__restrict__ sq) {
    __shared__ float w[NP];
    for (int i = threadIdx.x; i < NP; i += kMT) w[i] = P[i];
    __syncthreads();
    const int b = blockIdx.x * kMT + threadIdx.x;
    if (b >= B) return;
    float x[IN], h1[H], z2[H];
#pragma unroll
    for (int i = 0; i < IN; ++i) x[i] = X[(size_t)b * IN + i];
    for (int o = 0; o < H; ++o) {
        float s = w[OB1 + o];
#pragma unroll
        for (int i = 0; i < IN; ++i) s = fmaf(w[OW1 + o * IN + i], x[i], s);
        h1[o] = s > 0.f ? s : 0.f;
        h1o[(size_t)b * H + o] = h1[o];
    }
    float out = w[OB3];
    for (int o = 0; o < H; ++o) {
        float s = w[OB2 + o];
        for (int i = 0; i < H; ++i) s = fmaf(w[OW2 + o * H + i], h1[i], s);
        z2[o] = s;
        const float h = s > 0.f ? s : 0.f;
        h2o[(size_t)b * H + o] = h;
        out = fmaf(w[OW3 + o], h, out);
    }
    const float d = out - y[b];
    sq[b] = d * d;
    const float go = 2.f * d / (float)B;
    goo[b] = go;
    float g1[H];
#pragma unroll
    for (int i = 0; i < H; ++i) g1[i] = 0.f;
    for (int o = 0; o < H; ++o) {
        const float g2 = z2[o] > 0.f ? go * w[OW3 + o] : 0.f;
        g2o[(size_t)b * H + o] = g2;
        for (int i = 0; i < H; ++i) g1[i] = fmaf(g2, w[OW2 + o * H + i], g1[i]);
    }
    for (int i = 0; i < H; ++i) g1o[(size_t)b * H + i] = h1[i] > 0.f ? g1[i] : 0.f;
}

// One thread per parameter (plus one for the loss), summing over samples in order.
__global__ __launch_bounds__(kMT) void k_mlp_back_param(const float *__restrict__ X, int32_t B,
                                                        const float *__restrict__ h1, const float *__restrict__ h2,
                                                        const float *__restrict__ g1, const float *__restrict__ g2,
                                                        const float *__restrict__ go, const float *__restrict__ sq,
                                                        float *__restrict__ grad, float *__restrict__ loss) {
    const int p = blockIdx.x * kMT + threadIdx.x;
    if (p > NP) return;
    float s = 0.f;
    if (p == NP) {
        for (int b = 0; b < B; ++b) s += sq[b];
        loss[0] = B > 0 ? s / (float)B : 0.f;
        return;
    }
    if (p < OB1) {
        const int o = p / IN, i = p % IN;
        for (int b = 0; b < B; ++b) s = fmaf(g1[(size_t)b * H + o], X[(size_t)b * IN + i], s);
    } else if (p < OW2) {
        const int o = p - OB1;
        for (int b = 0; b < B; ++b) s += g1[(size_t)b * H + o];
    } else if (p < OB2) {
        const int q = p - OW2, o = q / H, i = q % H;
        for (int b = 0; b < B; ++b) s = fmaf(g2[(size_t)b * H + o], h1[(size_t)b * H + i], s);
    } else if (p < OW3) {
        const int o = p - OB2;
        for (int b = 0; b < B; ++b) s += g2[(size_t)b * H + o];
    } else if (p < OB3) {
        const int i = p - OW3;
        for (int b = 0; b < B; ++b) s = fmaf(go[b], h2[(size_t)b * H + i], s);
    } else {
        for (int b = 0; b < B; ++b) s += go[b];
    }
    grad[p] = s;
}

__global__ __launch_bounds__(kMT) void k_adam(float *__restrict__ P, float *__restrict__ m1, float *__restrict__ m2,
                                              const float *__restrict__ g, int32_t count, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * kMT + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    P[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

}  // namespace
}  // namespace boba

using namespace boba;

extern "C" size_t boba_graph_features_workspace(void) { return align_up(kFeatWsWords * sizeof(uint64_t), 256); }

extern "C" boba_status boba_graph_features(const int32_t *src, const int32_t *dst, int64_t m, int64_t n, float *feat16,
                                           void *ws, size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (m < 0 || n < 0) return fail(BOBA_ERR_ARG, "boba_graph_features: negative size");
    if (m >= (1ll << 31) || n >= (1ll << 31)) return fail(BOBA_ERR_OVERFLOW, "boba_graph_features: sizes must be < 2^31");
    if (!feat16) return fail(BOBA_ERR_ARG, "boba_graph_features: feat16 is NULL");
    if (m > 0 && (!src || !dst)) return fail(BOBA_ERR_ARG, "boba_graph_features: src/dst is NULL");
    if (!ws || ws_bytes < boba_graph_features_workspace() || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "boba_graph_features: workspace needs %zu bytes, 256-byte aligned",
                    boba_graph_features_workspace());
    uint64_t *st = (uint64_t *)ws;
    const uint32_t um = (uint32_t)m;
    if (m > 0) {
        BOBA_LAUNCH("feat_stats", k_feat_stats, dim3(kWin + 2), dim3(kT), stream, src, dst, um, st);
    }
    BOBA_LAUNCH("feat_final", k_feat_final, dim3(1), dim3(kWave), stream, (const uint64_t *)st, um, (uint32_t)n, feat16);
    return BOBA_OK;
}

extern "C" int32_t boba_mlp_param_count(void) { return NP; }

extern "C" boba_status boba_mlp_forward(const float *params, const float *X, int32_t B, float *yhat,
                                        hipStream_t stream) {
    clear_error();
    if (B < 0) return fail(BOBA_ERR_ARG, "boba_mlp_forward: negative batch");
    if (B == 0) return BOBA_OK;
    if (!params || !X || !yhat) return fail(BOBA_ERR_ARG, "boba_mlp_forward: NULL pointer");
    BOBA_LAUNCH("mlp_forward", k_mlp_forward, dim3(ceil_div(B, kFwdWaves)), dim3(kMT), stream, params, X, B, yhat);
    return BOBA_OK;
}

extern "C" size_t boba_mlp_backward_workspace(int32_t B) {
    if (B < 0) return 0;
    Carver c(nullptr);
    for (int k = 0; k < 4; ++k) c.take<float>((size_t)B * H);
    c.take<float>(B);
    c.take<float>(B);
    return c.bytes();
}

extern "C" boba_status boba_mlp_backward(const float *params, const float *X, const float *y, int32_t B, float *grad,
                                         float *loss, void *ws, size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (B <= 0) return fail(BOBA_ERR_ARG, "boba_mlp_backward: batch must be positive");
    if (!params || !X || !y || !grad || !loss) return fail(BOBA_ERR_ARG, "boba_mlp_backward: NULL pointer");
    if (!ws || ws_bytes < boba_mlp_backward_workspace(B) || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "boba_mlp_backward: workspace needs %zu bytes, 256-byte aligned",
                    boba_mlp_backward_workspace(B));
    Carver c(ws);
    float *h1 = c.take<float>((size_t)B * H), *h2 = c.take<float>((size_t)B * H);
    float *g1 = c.take<float>((size_t)B * H), *g2 = c.take<float>((size_t)B * H);
    float *go = c.take<float>(B), *sq = c.take<float>(B);
    BOBA_LAUNCH("mlp_back_sample", k_mlp_back_sample, dim3(ceil_div(B, kMT)), dim3(kMT), stream, params, X, y, B, h1,
                h2, g1, g2, go, sq);
    BOBA_LAUNCH("mlp_back_param", k_mlp_back_param, dim3(ceil_div(NP + 1, kMT)), dim3(kMT), stream, X, B,
                (const float *)h1, (const float *)h2, (const float *)g1, (const float *)g2, (const float *)go,
                (const float *)sq, grad, loss);
    return BOBA_OK;
}

extern "C" boba_status boba_mlp_adam(float *params, float *m1, float *m2, const float *grad, int32_t count, int32_t t,
                                     float lr, float b1, float b2, float eps, hipStream_t stream) {
    clear_error();
    if (count < 0 || t < 1) return fail(BOBA_ERR_ARG, "boba_mlp_adam: count >= 0 and step t >= 1 required");
    if (count == 0) return BOBA_OK;
    if (!params || !m1 || !m2 || !grad) return fail(BOBA_ERR_ARG, "boba_mlp_adam: NULL pointer");
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    BOBA_LAUNCH("mlp_adam", k_adam, dim3(ceil_div(count, kMT)), dim3(kMT), stream, params, m1, m2, grad, count, lr, b1,
                b2, eps, c1, c2);
    return BOBA_OK;
}

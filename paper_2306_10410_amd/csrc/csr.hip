// COO -> CSR by a stable least-significant-digit radix sort on the row
// (the conversion step of Sec. 1.1 / Sec. 5.3, moved from the CPU to the GPU).
//
// Per digit pass:
//   hist     per 8192-edge tile, a histogram of the digit (LDS atomics),
//            stored tile-major: hist[t * 256 + d]
//   offsets  column scan of hist -> where tile t's digit-d run starts
//   scatter  stable rank inside the tile (wave ballots + per-wave LDS
//            counters, waves own contiguous 1024-edge runs), local sort in
//            LDS, then coalesced writes of key / col / val runs
// After the last pass rowptr comes from the sorted rows: the end of each row's
// run is written at rowptr[row + 1], then an inclusive max-scan fills rows
// without entries.
#include "internal.h"
#include "scan.h"

namespace boba {
namespace {

constexpr int kBlock = 1024;
constexpr int kNWave = kBlock / kWave;
constexpr int kItems = 8;
constexpr uint32_t kTile = kBlock * kItems;       // 8192 edges per workgroup: ~128-byte digit runs
constexpr uint32_t kWaveRun = kWave * kItems;     // contiguous edges per wave

// Histogram: 256 threads x 32 keys per tile (int4 loads when aligned), one
// LDS sub-histogram per wave (skewed digits -- hub rows -- contend less).
constexpr int kHistThreads = 256;
constexpr int kHistPer = kTile / kHistThreads;  // 32
static_assert(kHistPer % 4 == 0, "int4 loads");

template <int BITS>
__global__ __launch_bounds__(kHistThreads) void k_radix_hist(const int32_t *__restrict__ keys, uint32_t m,
                                                             uint32_t shift, uint32_t tiles,
                                                             uint32_t *__restrict__ hist) {
    constexpr uint32_t BINS = 1u << BITS;
    constexpr int NW = kHistThreads / kWave;
    __shared__ uint32_t h[NW][BINS];
    for (uint32_t d = threadIdx.x; d < NW * BINS; d += kHistThreads) (&h[0][0])[d] = 0;
    __syncthreads();
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t base = blockIdx.x * kTile;
    const bool vec = (((uintptr_t)keys) & 15u) == 0;
    uint32_t k[kHistPer];
#pragma unroll
    for (int j = 0; j < kHistPer / 4; ++j) {
        const uint32_t e = base + j * (4 * kHistThreads) + 4 * threadIdx.x;
        if (vec && e + 3 < m) {
            const v4i x = *(const v4i *)(keys + e);
            k[4 * j] = (uint32_t)x.x;
            k[4 * j + 1] = (uint32_t)x.y;
            k[4 * j + 2] = (uint32_t)x.z;
            k[4 * j + 3] = (uint32_t)x.w;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) k[4 * j + q] = e + q < m ? (uint32_t)keys[e + q] : 0u;
        }
    }
    // Digit 0 is counted in a register: after BOBA the smallest row IDs are
    // the hubs, so in the upper digits 0 is by far the most frequent, and
    // equal-address LDS atomics from one wave serialize.
    uint32_t zeros = 0;
#pragma unroll
    for (int j = 0; j < kHistPer / 4; ++j) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (base + j * (4 * kHistThreads) + 4 * threadIdx.x + q < m) {
                const uint32_t d = (k[4 * j + q] >> shift) & (BINS - 1);
                if (d == 0) ++zeros;
                else atomicAdd(&h[wave][d], 1u);
            }
        }
    }
    zeros = wave_reduce(zeros, OpSum{});
    if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&h[wave][0], zeros);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < BINS; d += kHistThreads) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += h[w][d];
        hist[(size_t)blockIdx.x * BINS + d] = t;  // tile-major: coalesced
    }
}

// amdgpu_waves_per_eu(8): at most 64 VGPRs, so that two workgroups share a CU
// LAST (the final pass of coo_to_csr): the sorted keys themselves are not
// needed, only where rows end.  Inside a tile's digit run consecutive slots
// are consecutive output positions, so a key change there is a row end and
// rowptr[key + 1] is written directly; only the first and last key of every
// run are stored (into keys_out at their positions), for k_run_ends to
// settle the row ends that fall on run boundaries.
template <int BITS, bool HAS_VAL, bool LAST = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_radix_scatter(const int32_t *__restrict__ keys_in,
                                                          const int32_t *__restrict__ col_in,
                                                          const float *__restrict__ val_in, uint32_t m,
                                                          uint32_t shift, uint32_t tiles,
                                                          const uint32_t *__restrict__ offs,
                                                          int32_t *__restrict__ keys_out,
                                                          int32_t *__restrict__ col_out,
                                                          float *__restrict__ val_out,
                                                          uint32_t n_rows = 0, uint32_t *__restrict__ rowptr = nullptr,
                                                          int32_t *flag = nullptr) {
    constexpr uint32_t BINS = 1u << BITS;
    constexpr uint32_t MASK = BINS - 1;
    // digits per thread in the tile scan (threads beyond BINS hold none)
    constexpr uint32_t DPT = BINS >= (uint32_t)kBlock ? BINS / kBlock : 1;
    static_assert(BINS % kBlock == 0 || kBlock % BINS == 0, "digit count and block size must divide");
    __shared__ uint32_t s_cnt[kNWave][BINS];  // per-wave counts, then run starts
    __shared__ uint32_t s_gofs[BINS];         // global start of the digit's run minus its tile-local start
    __shared__ uint32_t s_scan[kNWave];
    // One tile-sized buffer, reused for keys, columns and values in turn, keeps
    // the LDS footprint near 58 KB: two workgroups per CU overlap one
    // another's load, rank and store phases.
    __shared__ int32_t s_buf[kTile];
    __shared__ uint8_t s_dig[kTile];          // digit of every sorted slot

    const uint32_t tile = xcd_work_index(blockIdx.x, gridDim.x);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = threadIdx.x / kWave;
    for (uint32_t i = threadIdx.x; i < kNWave * BINS; i += kBlock) (&s_cnt[0][0])[i] = 0;
    for (uint32_t d = threadIdx.x; d < BINS; d += kBlock) s_gofs[d] = offs[(size_t)tile * BINS + d];
    __syncthreads();

    const uint32_t tile_base = tile * kTile;
    const uint32_t wbase = tile_base + wave * kWaveRun;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    // Only the keys are held through the ranking; columns and values are
    // loaded later, each shortly before its own phase (fewer live registers).
    int32_t key[kItems], col[kItems];
    float val[kItems];
    uint32_t pos[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t i = wbase + j * kWave + lane;
        key[j] = i < m ? keys_in[i] : 0;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const bool valid = wbase + j * kWave + lane < m;
        const uint32_t d = ((uint32_t)key[j] >> shift) & MASK;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t below = __popcll(peers & lt_mask);
        const uint32_t prior = s_cnt[wave][d];
        if (valid && below == 0) s_cnt[wave][d] = prior + (uint32_t)__popcll(peers);
        pos[j] = prior + below;  // rank among the wave's equal digits so far
    }
    __syncthreads();

    // Tile-local start of every (digit, wave) run, digit-major.
    {
        const bool owns = threadIdx.x * DPT < BINS;
        uint32_t s = 0;
#pragma unroll
        for (uint32_t q = 0; q < DPT; ++q) {
            const uint32_t d = threadIdx.x * DPT + q;
            if (!owns) break;
#pragma unroll
            for (int w = 0; w < kNWave; ++w) s += s_cnt[w][d];
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan<kBlock>(s, OpSum{}, s_scan, total);
#pragma unroll
        for (uint32_t q = 0; q < DPT; ++q) {
            const uint32_t d = threadIdx.x * DPT + q;
            if (!owns) break;
            s_gofs[d] -= run;  // modulo 2^32; adding back a position in [run, run + count) is exact
#pragma unroll
            for (int w = 0; w < kNWave; ++w) {
                const uint32_t c = s_cnt[w][d];
                s_cnt[w][d] = run;
                run += c;
            }
        }
    }
    __syncthreads();

    const uint32_t count = m - tile_base < kTile ? m - tile_base : kTile;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t i = wbase + j * kWave + lane;
        col[j] = i < m ? col_in[i] : 0;
    }
    // keys: local sort, then the destination of every sorted slot
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        if (wbase + j * kWave + lane < m) {
            const uint32_t d = ((uint32_t)key[j] >> shift) & MASK;
            pos[j] += s_cnt[wave][d];
            s_buf[pos[j]] = key[j];
            s_dig[pos[j]] = (uint8_t)d;
        }
    }
    __syncthreads();
    // destination of sorted slot p (m: none; never the case when the offsets
    // are consistent)
    auto dest = [&](uint32_t p) -> uint32_t {
        if (p >= count) return m;
        const uint32_t g = s_gofs[s_dig[p]] + p;
        return g < m ? g : m;
    };
    if (LAST) {
        bool bad = false;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t p = j * kBlock + threadIdx.x;
            const uint32_t g = dest(p);
            if (g >= m) continue;
            const int32_t key = s_buf[p];
            const uint8_t dg = s_dig[p];
            const bool run_end = p + 1 == count || s_dig[p + 1] != dg;
            if (p == 0 || s_dig[p - 1] != dg || run_end) keys_out[g] = key;
            if ((uint32_t)key >= n_rows) {
                bad = true;
                continue;
            }
            if (!run_end && s_buf[p + 1] != key) rowptr[key + 1] = g + 1;
        }
        if (bad) flag_range_error(flag);
    } else {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t p = j * kBlock + threadIdx.x;
            const uint32_t g = dest(p);
            if (g < m) keys_out[g] = s_buf[p];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j)
        if (wbase + j * kWave + lane < m) s_buf[pos[j]] = col[j];
    if (HAS_VAL) {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t i = wbase + j * kWave + lane;
            val[j] = i < m ? val_in[i] : 0.f;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t p = j * kBlock + threadIdx.x;
        const uint32_t g = dest(p);
        if (g < m) col_out[g] = s_buf[p];
    }
    if (HAS_VAL) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kItems; ++j)
            if (wbase + j * kWave + lane < m) s_buf[pos[j]] = __float_as_int(val[j]);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t p = j * kBlock + threadIdx.x;
            const uint32_t g = dest(p);
            if (g < m) val_out[g] = __int_as_float(s_buf[p]);
        }
    }
}

// Offsets from the tile-major histograms: offs[t][d] = start of digit d's
// bucket + count of digit d in tiles before t.  Per block of kColTiles tiles
// the column sums are written digit-major (partial[d * blocks + b]); a plain
// exclusive scan of that array gives every (digit, block) its start; then each
// block's running sums are written in place.  Rows of the histogram are read
// coalesced, one thread per digit, kColUnroll rows in flight.
constexpr uint32_t kColTiles = 64;
constexpr int kColUnroll = 16;

template <int BINS>
__global__ __launch_bounds__(BINS) void k_col_reduce(const uint32_t *__restrict__ hist, uint32_t tiles,
                                                     uint32_t blocks, uint32_t *__restrict__ partial) {
    const uint32_t b = blockIdx.x, d = threadIdx.x;
    const uint32_t t0 = b * kColTiles, t1 = min(tiles, t0 + kColTiles);
    uint32_t s = 0;
    for (uint32_t t = t0; t < t1; t += kColUnroll) {
        uint32_t v[kColUnroll];
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u) v[u] = t + u < t1 ? hist[(size_t)(t + u) * BINS + d] : 0u;
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u) s += v[u];
    }
    partial[(size_t)d * blocks + b] = s;
}

template <int BINS>
__global__ __launch_bounds__(BINS) void k_col_down(uint32_t *__restrict__ hist, uint32_t tiles, uint32_t blocks,
                                                   const uint32_t *__restrict__ partial) {
    const uint32_t b = blockIdx.x, d = threadIdx.x;
    const uint32_t t0 = b * kColTiles, t1 = min(tiles, t0 + kColTiles);
    uint32_t run = partial[(size_t)d * blocks + b];
    for (uint32_t t = t0; t < t1; t += kColUnroll) {
        uint32_t v[kColUnroll];
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u) v[u] = t + u < t1 ? hist[(size_t)(t + u) * BINS + d] : 0u;
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u) {
            if (t + u < t1) hist[(size_t)(t + u) * BINS + d] = run;
            run += v[u];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *__restrict__ a, uint32_t count, uint32_t v) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) a[i] = v;
}

// The row ends on digit-run boundaries of the last pass: run (t, d) of the
// output (runs lie digit-major, then by tile) ends just before the next run
// starts; if its last key differs from the next run's first key (or it is the
// last run), that key's row ends there.  The first and last key of every run
// were stored by the last pass.  offs holds each run's global start.
template <int BITS>
__global__ __launch_bounds__(256) void k_run_ends(const uint32_t *__restrict__ offs, uint32_t tiles,
                                                  const int32_t *__restrict__ keys, uint32_t m, uint32_t n_rows,
                                                  uint32_t *__restrict__ rowptr) {
    constexpr uint32_t BINS = 1u << BITS;
    const uint64_t runs = (uint64_t)tiles * BINS;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < runs; q += stride) {
        const uint32_t t = (uint32_t)(q / BINS), d = (uint32_t)(q % BINS);
        const uint32_t start = offs[q];
        const uint32_t next = t + 1 < tiles ? offs[q + BINS] : (d + 1 < BINS ? offs[d + 1] : m);
        if (next <= start || next > m) continue;  // empty run
        const int32_t key = keys[next - 1];
        if ((uint32_t)key >= n_rows) continue;    // flagged by the scatter
        if (next == m || keys[next] != key) rowptr[key + 1] = next;
    }
}

constexpr int kBits = 8;

struct CsrLayout {
    int32_t *keys_a, *keys_b, *col_x;
    float *val_x;
    uint32_t *hist, *partial, *colpart;
    size_t bytes;
    uint32_t tiles, colblocks;
};

CsrLayout csr_layout(void *ws, int64_t n_rows, int64_t m, bool has_val) {
    CsrLayout L;
    L.tiles = ceil_div((uint64_t)m, kTile);
    const uint64_t hist_count = (uint64_t)(1u << kBits) * L.tiles;
    const uint64_t scan_count = hist_count > (uint64_t)n_rows + 1 ? hist_count : (uint64_t)n_rows + 1;
    Carver c(ws);
    L.keys_a = c.take<int32_t>((size_t)m);
    L.keys_b = c.take<int32_t>((size_t)m);
    L.col_x = c.take<int32_t>((size_t)m);
    L.val_x = c.take<float>(has_val ? (size_t)m : 0);
    L.hist = c.take<uint32_t>((size_t)hist_count);
    L.partial = c.take<uint32_t>(scan_partials(scan_count));
    L.colblocks = ceil_div(L.tiles, kColTiles);
    L.colpart = c.take<uint32_t>((size_t)L.colblocks << kBits);
    L.bytes = c.bytes();
    return L;
}

}  // namespace
}  // namespace boba

using namespace boba;

extern "C" size_t coo_to_csr_workspace(int64_t n_rows, int64_t m) {
    if (n_rows < 0 || m < 0) return 0;
    return csr_layout(nullptr, n_rows, m, true).bytes;
}

extern "C" boba_status coo_to_csr(const int32_t *row, const int32_t *col, const float *val, int64_t m,
                                  int64_t n_rows, int32_t *rowptr, int32_t *col_out, float *val_out, void *ws,
                                  size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (m < 0 || n_rows < 0) return fail(BOBA_ERR_ARG, "coo_to_csr: negative size");
    if (m >= (1ll << 31) || n_rows >= (1ll << 31)) return fail(BOBA_ERR_OVERFLOW, "coo_to_csr: m and n_rows must be < 2^31");
    if (!rowptr) return fail(BOBA_ERR_ARG, "coo_to_csr: rowptr is NULL");
    if ((val == nullptr) != (val_out == nullptr))
        return fail(BOBA_ERR_ARG, "coo_to_csr: val and val_out must both be given or both be NULL");
    if (m > 0 && (!row || !col || !col_out)) return fail(BOBA_ERR_ARG, "coo_to_csr: NULL pointer");
    if (m > 0 && n_rows == 0) return fail(BOBA_ERR_ARG, "coo_to_csr: edges given but n_rows = 0");
    const size_t need = coo_to_csr_workspace(n_rows, m);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "coo_to_csr: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)",
                    need, ws_bytes, ws);
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    const bool has_val = val != nullptr;
    CsrLayout L = csr_layout(ws, n_rows, m, has_val);
    const uint32_t um = (uint32_t)m, nr = (uint32_t)n_rows;

    BOBA_LAUNCH("csr_fill", k_fill_u32, dim3(grid_for(nr + 1ull, kBlock * 4)), dim3(kBlock), stream,
                (uint32_t *)rowptr, nr + 1, 0u);
    if (m == 0) return BOBA_OK;

    uint32_t bits = 0;
    while (bits < 31 && (1ull << bits) < (uint64_t)nr) ++bits;
    const int passes = bits == 0 ? 1 : (int)((bits + kBits - 1) / kBits);

    const int32_t *kin = row;
    const int32_t *cin = col;
    const float *vin = val;
    for (int p = 0; p < passes; ++p) {
        const uint32_t shift = (uint32_t)(p * kBits);
        const bool last = p + 1 == passes;
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        int32_t *kout = (p % 2 == 0) ? L.keys_a : L.keys_b;
        int32_t *cout = to_out ? col_out : L.col_x;
        float *vout = to_out ? val_out : L.val_x;
        BOBA_LAUNCH("radix_hist", k_radix_hist<kBits>, dim3(L.tiles), dim3(kHistThreads), stream, kin, um, shift, L.tiles,
                    L.hist);
        BOBA_LAUNCH("radix_offsets", k_col_reduce<1 << kBits>, dim3(L.colblocks), dim3(1 << kBits), stream,
                    (const uint32_t *)L.hist, L.tiles, L.colblocks, L.colpart);
        if (boba_status e = device_scan<OpSum, false>("radix_offsets", LoadArr{L.colpart}, StoreArr{L.colpart},
                                                      L.colblocks << kBits, L.partial, stream))
            return e;
        BOBA_LAUNCH("radix_offsets", k_col_down<1 << kBits>, dim3(L.colblocks), dim3(1 << kBits), stream, L.hist,
                    L.tiles, L.colblocks, (const uint32_t *)L.colpart);
        const uint32_t *offs = L.hist;
        if (has_val && last)
            BOBA_LAUNCH("radix_scatter", (k_radix_scatter<kBits, true, true>), dim3(L.tiles), dim3(kBlock), stream,
                        kin, cin, vin, um, shift, L.tiles, offs, kout, cout, vout, nr, (uint32_t *)rowptr, flag);
        else if (last)
            BOBA_LAUNCH("radix_scatter", (k_radix_scatter<kBits, false, true>), dim3(L.tiles), dim3(kBlock), stream,
                        kin, cin, vin, um, shift, L.tiles, offs, kout, cout, vout, nr, (uint32_t *)rowptr, flag);
        else if (has_val)
            BOBA_LAUNCH("radix_scatter", (k_radix_scatter<kBits, true>), dim3(L.tiles), dim3(kBlock), stream, kin, cin,
                        vin, um, shift, L.tiles, offs, kout, cout, vout);
        else
            BOBA_LAUNCH("radix_scatter", (k_radix_scatter<kBits, false>), dim3(L.tiles), dim3(kBlock), stream, kin, cin,
                        vin, um, shift, L.tiles, offs, kout, cout, vout);
        kin = kout;
        cin = cout;
        vin = vout;
    }
    BOBA_LAUNCH("row_ends", k_run_ends<kBits>, dim3(grid_for((uint64_t)L.tiles << kBits, 256)), dim3(256), stream,
                (const uint32_t *)L.hist, L.tiles, kin, um, nr, (uint32_t *)rowptr);
    return device_scan<OpMax, true>("rowptr_scan", LoadArr{(const uint32_t *)rowptr}, StoreArr{(uint32_t *)rowptr}, nr + 1,
                                    L.partial, stream);
}

// ------------------------------------------------ binning by destination
// A stable sort of the edges by dst >> shift: the remedy the paper suggests
// for edge lists in random order (Sec. 5.6) -- bin (or sort) the COO by
// destination before running BOBA.  shift = max(0, bits(n - 1) - bin_bits),
// so the edges fall into at most 2^bin_bits bins in order of destination and
// keep their input order inside a bin.  LSD radix passes of 8 bits over the
// bin number, with the same kernels as coo_to_csr (key dst, payload src).
namespace boba {
namespace {

struct BinLayout {
    int32_t *keys_x, *vals_x;
    uint32_t *hist, *partial, *colpart;
    size_t bytes;
    uint32_t tiles, colblocks;
};

BinLayout bin_layout(void *ws, int64_t m) {
    BinLayout L;
    L.tiles = ceil_div((uint64_t)m, kTile);
    L.colblocks = ceil_div(L.tiles, kColTiles);
    Carver c(ws);
    L.keys_x = c.take<int32_t>((size_t)m);
    L.vals_x = c.take<int32_t>((size_t)m);
    L.hist = c.take<uint32_t>((size_t)L.tiles << kBits);
    L.colpart = c.take<uint32_t>((size_t)L.colblocks << kBits);
    L.partial = c.take<uint32_t>(scan_partials((uint64_t)L.colblocks << kBits));
    L.bytes = c.bytes();
    return L;
}

inline uint32_t id_bits(int64_t n) {
    uint32_t bits = 0;
    while (bits < 31 && (1ull << bits) < (uint64_t)n) ++bits;
    return bits;
}

}  // namespace
}  // namespace boba

extern "C" size_t boba_bin_by_dst_workspace(int64_t n, int64_t m) {
    if (n < 0 || m < 0) return 0;
    return bin_layout(nullptr, m).bytes;
}

extern "C" boba_status boba_bin_by_dst(const int32_t *src, const int32_t *dst, int64_t m, int64_t n,
                                       int32_t bin_bits, int32_t *src_out, int32_t *dst_out, void *ws,
                                       size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (m < 0 || n < 0) return fail(BOBA_ERR_ARG, "boba_bin_by_dst: negative size");
    if (m >= (1ll << 31) || n >= (1ll << 31))
        return fail(BOBA_ERR_OVERFLOW, "boba_bin_by_dst: m and n must be < 2^31");
    if (bin_bits < 1 || bin_bits > 31) return fail(BOBA_ERR_ARG, "boba_bin_by_dst: bin_bits must be in 1..31");
    if (m == 0) return BOBA_OK;
    if (!src || !dst || !src_out || !dst_out) return fail(BOBA_ERR_ARG, "boba_bin_by_dst: NULL pointer");
    if (src_out == src || src_out == dst || dst_out == src || dst_out == dst)
        return fail(BOBA_ERR_ARG, "boba_bin_by_dst: outputs may not alias the inputs");
    const size_t need = boba_bin_by_dst_workspace(n, m);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u))
        return fail(BOBA_ERR_WORKSPACE, "boba_bin_by_dst: workspace needs %zu bytes, 256-byte aligned (got %zu at %p)",
                    need, ws_bytes, ws);
    const BinLayout L = bin_layout(ws, m);
    const uint32_t um = (uint32_t)m;
    const uint32_t total = id_bits(n);
    const uint32_t key_bits = (uint32_t)bin_bits < total ? (uint32_t)bin_bits : total;
    const uint32_t shift = total - key_bits;
    const int passes = key_bits == 0 ? 0 : (int)((key_bits + kBits - 1) / kBits);
    if (passes == 0) {  // a single bin: the edge list is unchanged
        if (hipMemcpyAsync(src_out, src, (size_t)m * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(dst_out, dst, (size_t)m * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return fail(BOBA_ERR_HIP, "boba_bin_by_dst: copy failed");
        return BOBA_OK;
    }
    const int32_t *kin = dst, *vin = src;
    for (int p = 0; p < passes; ++p) {
        const uint32_t sh = shift + (uint32_t)(p * kBits);
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        int32_t *kout = to_out ? dst_out : L.keys_x;
        int32_t *vout = to_out ? src_out : L.vals_x;
        BOBA_LAUNCH("bin_hist", k_radix_hist<kBits>, dim3(L.tiles), dim3(kHistThreads), stream, kin, um, sh, L.tiles,
                    L.hist);
        BOBA_LAUNCH("bin_offsets", k_col_reduce<1 << kBits>, dim3(L.colblocks), dim3(1 << kBits), stream,
                    (const uint32_t *)L.hist, L.tiles, L.colblocks, L.colpart);
        if (boba_status e = device_scan<OpSum, false>("bin_offsets", LoadArr{L.colpart}, StoreArr{L.colpart},
                                                      L.colblocks << kBits, L.partial, stream))
            return e;
        BOBA_LAUNCH("bin_offsets", k_col_down<1 << kBits>, dim3(L.colblocks), dim3(1 << kBits), stream, L.hist,
                    L.tiles, L.colblocks, (const uint32_t *)L.colpart);
        BOBA_LAUNCH("bin_scatter", (k_radix_scatter<kBits, false>), dim3(L.tiles), dim3(kBlock), stream, kin, vin,
                    (const float *)nullptr, um, sh, L.tiles, (const uint32_t *)L.hist, kout, vout, (float *)nullptr);
        kin = kout;
        vin = vout;
    }
    return BOBA_OK;
}

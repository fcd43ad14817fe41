// Device-wide scan over uint32 sequences given by load/store functors:
// reduce (one partial per tile) -> scan of the partials in one workgroup ->
// rescan of every tile with its carry.  Tiles are 256 threads x 16 items,
// read striped so that every load instruction is coalesced.
#pragma once

#include "internal.h"

namespace boba {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr uint32_t kScanTile = kScanBlock * kScanItems;
constexpr int kScanTopBlock = 1024;

inline uint32_t scan_tiles(uint64_t count) { return ceil_div(count, kScanTile); }
// Workspace words needed by device_scan for `count` items.
inline size_t scan_partials(uint64_t count) { return (size_t)scan_tiles(count) + 1; }

template <class Load, class Op>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(Load load, uint32_t count, uint32_t *partial) {
    __shared__ uint32_t lds[kScanBlock / kWave];
    Op op;
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x;
    // loads at clamped indices (count >= 1 in a launched workgroup), so that
    // all of them are in flight before the first is waited for
    uint32_t v[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) v[j] = load(min(base + j * kScanBlock, count - 1));
    uint32_t acc = Op::identity;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j * kScanBlock < count) acc = op(acc, v[j]);
    acc = block_reduce<kScanBlock>(acc, op, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Exclusive scan of partial[0..nt) in place by one workgroup; partial[nt] gets
// the total.  Each thread scans a contiguous run sequentially.
template <class Op>
__global__ __launch_bounds__(kScanTopBlock) void k_scan_top(uint32_t *partial, uint32_t nt) {
    __shared__ uint32_t lds[kScanTopBlock / kWave];
    Op op;
    const uint32_t per = (nt + kScanTopBlock - 1) / kScanTopBlock;
    const uint32_t b = threadIdx.x * per;
    const uint32_t e = min(nt, b + per);
    uint32_t s = Op::identity;
    for (uint32_t i = b; i < e; ++i) s = op(s, partial[i]);
    uint32_t total;
    uint32_t run = block_exclusive_scan<kScanTopBlock>(s, op, lds, total);
    for (uint32_t i = b; i < e; ++i) {
        uint32_t v = partial[i];
        partial[i] = run;
        run = op(run, v);
    }
    if (threadIdx.x == 0) partial[nt] = total;
}

template <class Load, class Store, class Op, bool INCLUSIVE>
__global__ __launch_bounds__(kScanBlock) void k_scan_down(Load load, Store store, uint32_t count,
                                                          const uint32_t *partial) {
    __shared__ uint32_t lds[kScanBlock / kWave];
    Op op;
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x;
    uint32_t carry = partial[blockIdx.x];
    uint32_t x[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) x[j] = load(min(base + j * kScanBlock, count - 1));
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j * kScanBlock >= count) x[j] = Op::identity;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint32_t total;
        uint32_t ex = block_exclusive_scan<kScanBlock>(x[j], op, lds, total);
        uint32_t i = base + j * kScanBlock;
        if (i < count) store(i, INCLUSIVE ? op(carry, op(ex, x[j])) : op(carry, ex));
        carry = op(carry, total);
    }
}

// Enqueues the scan; `partial` must hold scan_partials(count) words.
// `name` labels the three launches for timing and error messages.
template <class Op, bool INCLUSIVE, class Load, class Store>
boba_status device_scan(const char *name, Load load, Store store, uint32_t count, uint32_t *partial, hipStream_t s) {
    const uint32_t nt = scan_tiles(count);
    if (nt == 0) return BOBA_OK;
    BOBA_LAUNCH(name, (k_scan_reduce<Load, Op>), dim3(nt), dim3(kScanBlock), s, load, count, partial);
    BOBA_LAUNCH(name, (k_scan_top<Op>), dim3(1), dim3(kScanTopBlock), s, partial, nt);
    BOBA_LAUNCH(name, (k_scan_down<Load, Store, Op, INCLUSIVE>), dim3(nt), dim3(kScanBlock), s, load, store, count,
                (const uint32_t *)partial);
    return BOBA_OK;
}

// Plain array load / store functors.
struct LoadArr {
    const uint32_t *a;
    __device__ uint32_t operator()(uint32_t i) const { return a[i]; }
};
struct StoreArr {
    uint32_t *a;
    __device__ void operator()(uint32_t i, uint32_t v) const { a[i] = v; }
};

}  // namespace boba

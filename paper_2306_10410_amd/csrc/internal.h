// Internal helpers shared by the translation units of libboba.so.
// gfx950 / CDNA4 only: wave64, 256-thread workgroups unless stated.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "boba.h"

namespace boba {

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr int kWave = 64;

// ---------------------------------------------------------------- host side
// Records a thread-local message and returns `code` (printf-style).
boba_status fail(boba_status code, const char *fmt, ...);
void clear_error();
// Device address of the per-device "vertex ID out of range" flag (nullptr and
// an error message on failure).
int32_t *range_flag();
// Compute units of the current device (256 on the MI355X; 256 if the query fails).
uint32_t device_cus();

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Carves 256-byte aligned sub-buffers out of a caller workspace.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *p) : base((char *)p) {}
    template <class T> T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return align_up(off, 256); }
};

// Returns BOBA_ERR_HIP (with the kernel name) if the last launch failed.
boba_status check_launch(const char *what);

// Optional event timing around launches (see boba_timing_enable).
int timing_begin(const char *name, hipStream_t s);
void timing_end(int token, hipStream_t s);
// While one is alive, launches on this thread are not timed (creating the
// events can allocate; the allocation-free entry point must not).
struct TimingSuspend {
    TimingSuspend();
    ~TimingSuspend();
};

// Launches a kernel (parenthesise template kernels), times it when timing is
// on, and returns BOBA_ERR_HIP from the enclosing function if the launch fails.
#define BOBA_LAUNCH(name, kernel, grid, block, stream, ...)                        \
    do {                                                                          \
        const int tok_ = ::boba::timing_begin(name, stream);                      \
        hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);          \
        ::boba::timing_end(tok_, stream);                                         \
        if (boba_status e_ = ::boba::check_launch(name)) return e_;               \
    } while (0)

// Grid size for a grid-stride kernel: enough workgroups to fill 256 CUs
// several times over, never more than the work needs.
inline uint32_t grid_for(uint64_t items, uint32_t per_block, uint32_t cap = 8192) {
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

// ---------------------------------------------------------------- device side
constexpr uint32_t kXcds = 8;  // MI355X: 8 XCDs, each with its own L2

// Workgroups are handed to the XCDs round-robin by workgroup ID.  This maps
// workgroup i of a grid of g to a work index such that every XCD gets one
// contiguous range of work indices, taken in increasing order: neighbouring
// work items (which share cache lines at their edges) then run on the same
// XCD at about the same time and meet in its L2.  A bijection on [0, g).
__device__ __forceinline__ uint32_t xcd_work_index(uint32_t i, uint32_t g) {
    const uint32_t x = i % kXcds, j = i / kXcds, q = g / kXcds, r = g % kXcds;
    return x * q + (x < r ? x : r) + j;
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

struct OpSum {
    static constexpr uint32_t identity = 0;
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};
struct OpMax {
    static constexpr uint32_t identity = 0;
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};

template <class Op>
__device__ inline uint32_t wave_inclusive_scan(uint32_t x, Op op) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x = op(x, y);
    }
    return x;
}

template <class Op>
__device__ inline uint32_t wave_reduce(uint32_t x, Op op) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x = op(x, __shfl_xor(x, d, kWave));
    return x;
}

// Exclusive scan over a workgroup of BLOCK threads.  `lds` holds BLOCK/64
// words.  Returns the exclusive prefix of this thread; `total` gets the
// reduction over the whole workgroup.  Contains two barriers: every thread of
// the workgroup must call it.
template <int BLOCK, class Op>
__device__ inline uint32_t block_exclusive_scan(uint32_t x, Op op, uint32_t *lds, uint32_t &total) {
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    uint32_t incl = wave_inclusive_scan(x, op);
    if (lane == kWave - 1) lds[wave] = incl;
    __syncthreads();
    uint32_t before = Op::identity, tot = Op::identity;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        uint32_t s = lds[w];
        if (w < wave) before = op(before, s);
        tot = op(tot, s);
    }
    __syncthreads();
    uint32_t excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = Op::identity;
    total = tot;
    return op(before, excl);
}

template <int BLOCK, class Op>
__device__ inline uint32_t block_reduce(uint32_t x, Op op, uint32_t *lds) {
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    x = wave_reduce(x, op);
    if (lane == 0) lds[wave] = x;
    __syncthreads();
    uint32_t tot = Op::identity;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot = op(tot, lds[w]);
    __syncthreads();
    return tot;
}

// Bits of the per-device error flag read by boba_check_device_error.
constexpr int32_t kFlagRange = 1;    // a vertex ID out of range
constexpr int32_t kFlagTimeout = 2;  // a bounded wait for another workgroup gave up

__device__ inline void flag_range_error(int32_t *flag) {
    if (flag) atomicOr(flag, kFlagRange);
}

__device__ inline void flag_timeout(int32_t *flag) {
    if (flag) atomicOr(flag, kFlagTimeout);
}

}  // namespace boba

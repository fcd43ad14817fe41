// CSR SpMV, y = A x (Algorithm 3, over CSR rows) in FP32.
//
// A group of L lanes (L in {4, 8, 16, 32, 64}; 64 = one wavefront) owns a row:
// lanes stride over the row's entries, accumulate with FMA, then reduce with
// cross-lane xor shuffles in a fixed tree, so the result is deterministic.
// The random reads of x are what the reordering makes local.
#include "internal.h"

namespace boba {
namespace {

constexpr int kBlock = 256;

template <int L, bool HAS_VAL>
__global__ __launch_bounds__(kBlock) void k_spmv(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                 const float *__restrict__ val, uint32_t n_rows, uint32_t n_cols,
                                                 const float *__restrict__ x, float *__restrict__ y, int32_t *flag) {
    constexpr uint32_t G = kBlock / L;  // row groups per workgroup
    const uint32_t lane = threadIdx.x % L;
    const uint32_t stride = gridDim.x * G;
    for (uint32_t row = blockIdx.x * G + threadIdx.x / L; row < n_rows; row += stride) {
        const int32_t b = rowptr[row], e = rowptr[row + 1];
        float acc = 0.f;
        for (int32_t k = b + (int32_t)lane; k < e; k += L) {
            const int32_t c = col[k];
            if ((uint32_t)c < n_cols) {
                acc = fmaf(HAS_VAL ? val[k] : 1.f, x[c], acc);
            } else {
                flag_range_error(flag);
            }
        }
#pragma unroll
        for (int d = L / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, L);
        if (lane == 0) y[row] = acc;
    }
}

template <int L>
boba_status launch(const int32_t *rowptr, const int32_t *col, const float *val, uint32_t nr, uint32_t nc,
                   const float *x, float *y, int32_t *flag, hipStream_t s) {
    constexpr uint32_t G = kBlock / L;
    const uint32_t grid = grid_for(nr, G, 65535u);
    if (val)
        BOBA_LAUNCH("spmv", (k_spmv<L, true>), dim3(grid), dim3(kBlock), s, rowptr, col, val, nr, nc, x, y, flag);
    else
        BOBA_LAUNCH("spmv", (k_spmv<L, false>), dim3(grid), dim3(kBlock), s, rowptr, col, val, nr, nc, x, y, flag);
    return BOBA_OK;
}

}  // namespace

boba_status spmv_launch(const int32_t *rowptr, const int32_t *col, const float *val, int64_t n_rows, int64_t n_cols,
                        const float *x, float *y, int lanes, hipStream_t stream) {
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    const uint32_t nr = (uint32_t)n_rows, nc = (uint32_t)n_cols;
    switch (lanes) {
    case 4: return launch<4>(rowptr, col, val, nr, nc, x, y, flag, stream);
    case 8: return launch<8>(rowptr, col, val, nr, nc, x, y, flag, stream);
    case 16: return launch<16>(rowptr, col, val, nr, nc, x, y, flag, stream);
    case 32: return launch<32>(rowptr, col, val, nr, nc, x, y, flag, stream);
    case 64: return launch<64>(rowptr, col, val, nr, nc, x, y, flag, stream);
    default: return fail(BOBA_ERR_ARG, "spmv: lanes per row must be 4, 8, 16, 32 or 64 (got %d)", lanes);
    }
}

}  // namespace boba

using namespace boba;

extern "C" boba_status spmv_csr(const int32_t *rowptr, const int32_t *col, const float *val, int64_t n_rows,
                                int64_t n_cols, const float *x, float *y, hipStream_t stream) {
    clear_error();
    if (n_rows < 0 || n_cols < 0) return fail(BOBA_ERR_ARG, "spmv_csr: negative size");
    if (n_rows >= (1ll << 31) || n_cols >= (1ll << 31)) return fail(BOBA_ERR_OVERFLOW, "spmv_csr: sizes must be < 2^31");
    if (n_rows == 0) return BOBA_OK;
    if (!rowptr || !col || !x || !y) return fail(BOBA_ERR_ARG, "spmv_csr: NULL pointer");
    // Mean row length is unknown without reading rowptr; a quarter wavefront
    // suits the mean degrees 4..32 of the graphs this library targets.
    return spmv_launch(rowptr, col, val, n_rows, n_cols, x, y, 16, stream);
}

// Error reporting and the per-device range-error flag.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "internal.h"

namespace boba {

namespace {
thread_local char g_msg[512] = "";

// Set by any kernel that meets a vertex ID outside its valid range.
__device__ int32_t g_range_error = 0;

constexpr int kMaxDevices = 64;
int32_t *g_flag_ptr[kMaxDevices] = {};
std::mutex g_flag_mu;
}  // namespace

boba_status fail(boba_status code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_msg[0] = 0; }

boba_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BOBA_ERR_HIP, "%s: launch failed: %s", what, hipGetErrorString(e));
    return BOBA_OK;
}

int32_t *range_flag() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        fail(BOBA_ERR_HIP, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_flag_mu);
    if (!g_flag_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_range_error));
        if (e != hipSuccess) {
            fail(BOBA_ERR_HIP, "hipGetSymbolAddress(range flag): %s", hipGetErrorString(e));
            return nullptr;
        }
        g_flag_ptr[dev] = (int32_t *)p;
    }
    return g_flag_ptr[dev];
}

uint32_t device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return (uint32_t)cus;
}

}  // namespace boba

extern "C" const char *boba_last_error(void) { return boba::g_msg; }

extern "C" boba_status boba_check_device_error(hipStream_t stream, int32_t *code) {
    using namespace boba;
    clear_error();
    if (!code) return fail(BOBA_ERR_ARG, "boba_check_device_error: code is NULL");
    int32_t *flag = range_flag();
    if (!flag) return BOBA_ERR_HIP;
    int32_t h = 0;
    hipError_t e = hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(BOBA_ERR_HIP, "boba_check_device_error: %s", hipGetErrorString(e));
    if (h) {
        const int32_t zero = 0;
        e = hipMemcpyAsync(flag, &zero, sizeof(zero), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(BOBA_ERR_HIP, "boba_check_device_error: %s", hipGetErrorString(e));
    }
    *code = (h & kFlagTimeout) ? BOBA_ERR_TIMEOUT : (h & kFlagRange) ? BOBA_ERR_RANGE : BOBA_OK;
    return BOBA_OK;
}

// Optional per-kernel timing with HIP events recorded on the launch stream.
// Off by default; when on, every kernel launch of the library is bracketed by
// an event pair.  Collection waits for the events and sums durations per name.
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace boba {
namespace {

struct Record {
    const char *name;
    hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;
thread_local int g_suspended = 0;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

TimingSuspend::TimingSuspend() { ++g_suspended; }
TimingSuspend::~TimingSuspend() { --g_suspended; }

int timing_begin(const char *name, hipStream_t s) {
    if (g_suspended) return -1;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_on) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    Record r{name, take_event(), take_event()};
    if (!r.start || !r.stop || hipEventRecord(r.start, s) != hipSuccess) return -1;
    g_records.push_back(r);
    return (int)g_records.size() - 1;
}

void timing_end(int token, hipStream_t s) {
    if (token < 0) return;
    std::lock_guard<std::mutex> lock(g_mu);
    if (token < (int)g_records.size()) hipEventRecord(g_records[token].stop, s);
}

}  // namespace boba

using namespace boba;

extern "C" boba_status boba_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_on = on != 0;
    return BOBA_OK;
}

extern "C" int32_t boba_timing_collect(char *names_buf, size_t buf_len, double *total_ms, int64_t *launches,
                                       int32_t max_entries) {
    clear_error();
    std::lock_guard<std::mutex> lock(g_mu);
    std::vector<std::string> names;
    std::vector<double> ms;
    std::vector<int64_t> cnt;
    for (const Record &r : g_records) {
        float t = 0.f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) {
            t = 0.f;
        }
        size_t k = 0;
        while (k < names.size() && names[k] != r.name) ++k;
        if (k == names.size()) {
            names.emplace_back(r.name);
            ms.push_back(0.0);
            cnt.push_back(0);
        }
        ms[k] += t;
        cnt[k] += 1;
        g_pool.push_back(r.start);
        g_pool.push_back(r.stop);
    }
    g_records.clear();
    int32_t out = 0;
    size_t off = 0;
    for (size_t k = 0; k < names.size() && out < max_entries; ++k) {
        const size_t len = names[k].size() + 1;
        if (!names_buf || off + len > buf_len) break;
        memcpy(names_buf + off, names[k].c_str(), len);
        off += len;
        if (total_ms) total_ms[out] = ms[k];
        if (launches) launches[out] = cnt[k];
        ++out;
    }
    return out;
}

// Error reporting and device queries shared by the C entry points.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>
#include <vector>

#include "qd_internal.h"

namespace qd {

static thread_local char g_err[512] = "";
static thread_local const volatile int *g_abort = nullptr;

bool abort_requested() { return g_abort && *g_abort != 0; }

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

int device_cus() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

struct TimedLaunch {
    const char *name;
    hipEvent_t a, b;
};
struct KernelTotal {
    std::string name;
    double ms;
    uint64_t launches;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<TimedLaunch> g_pending;
static std::vector<KernelTotal> g_totals;

bool profiling() { return g_prof_on; }

KernelTimer::KernelTimer(const char *name, hipStream_t s) : name_(name), s_(s) {
    if (!g_prof_on || !name) return;  // a null name times nothing (and creates no events)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s_, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;  // no events in graphs
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
        a_ = b_ = nullptr;
        return;
    }
    (void)hipEventRecord(a_, s_);
}

KernelTimer::~KernelTimer() {
    if (!a_) return;
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_pending.push_back({name_, a_, b_});
}

static void drain_pending() {
    for (auto &t : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            bool found = false;
            for (auto &k : g_totals)
                if (k.name == t.name) {
                    k.ms += ms;
                    k.launches++;
                    found = true;
                }
            if (!found) g_totals.push_back({t.name, (double)ms, 1});
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_pending.clear();
}

static std::vector<std::pair<std::string, uint64_t>> g_counters;

void profile_count(const char *name, uint64_t amount) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    for (auto &c : g_counters)
        if (c.first == name) {
            c.second += amount;
            return;
        }
    g_counters.push_back({name, amount});
}

}  // namespace qd

extern "C" int qd_profile_counter(const char *name, uint64_t *total) {
    if (!name || !total) return qd::fail(QD_ERR_INVALID, "null pointer");
    std::lock_guard<std::mutex> lock(qd::g_prof_mu);
    *total = 0;
    for (auto &c : qd::g_counters)
        if (c.first == name) *total = c.second;
    return QD_OK;
}

extern "C" int qd_profile_enable(int on) {
    std::lock_guard<std::mutex> lock(qd::g_prof_mu);
    qd::drain_pending();
    qd::g_totals.clear();
    qd::g_counters.clear();
    qd::g_prof_on = on != 0;
    return QD_OK;
}

extern "C" int qd_profile_read(const char *kernel, double *total_ms, uint64_t *launches) {
    if (!kernel || !total_ms || !launches) return qd::fail(QD_ERR_INVALID, "null pointer");
    std::lock_guard<std::mutex> lock(qd::g_prof_mu);
    qd::drain_pending();
    *total_ms = 0.0;
    *launches = 0;
    for (auto &k : qd::g_totals)
        if (k.name == kernel) {
            *total_ms = k.ms;
            *launches = k.launches;
        }
    return QD_OK;
}

extern "C" const char *qd_last_error(void) { return qd::g_err; }

extern "C" int qd_set_abort_flag(const volatile int *flag) {
    qd::g_abort = flag;
    return QD_OK;
}

extern "C" int qd_version(void) { return 200; }

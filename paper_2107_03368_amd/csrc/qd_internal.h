// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qd.h"

namespace qd {

typedef unsigned long long u64;

// Candidate key: (K << 32) | database row.  K < 2^24, so a real key is below
// 2^56 and KEY_NONE sorts after every real candidate.
constexpr u64 KEY_NONE = ~0ull;

// Record a message for qd_last_error() and return `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
// The calling thread's abort flag (qd_set_abort_flag) is set.
bool abort_requested();

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Number of compute units of the current device (cached per device).
int device_cus();

// Optional per-kernel timing with HIP events on the launch stream.  While
// profiling is on, a KernelTimer brackets one launch; durations are summed
// per kernel name when read.
bool profiling();
// Adds to a named counter while profiling is on (read with qd_profile_counter).
void profile_count(const char *name, uint64_t amount);
class KernelTimer {
  public:
    KernelTimer(const char *name, hipStream_t s);
    ~KernelTimer();

  private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace qd

#define QD_HIP_CHECK(call)                                                                             \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return qd::fail(e_ == hipErrorOutOfMemory ? QD_ERR_OOM : QD_ERR_DEVICE, "%s: %s", #call, \
                            hipGetErrorString(e_));                                                    \
    } while (0)

// Host-side launchers of the guard kernels (internal to libagile_guard.so).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "guard_device.h"

namespace agile {

struct DevInfo {
    int num_cu;
    size_t lds_per_block;  // largest dynamic LDS one workgroup may take
    size_t lds_per_cu;
};

// Maximum number of radix entries (plus one) the validation index may use.
constexpr uint32_t MAX_RADIX = (1u << 14) + 1;

hipError_t launch_validate(const DevTable& t, const DevInfo& d, const void* q, uint64_t n,
                           uint8_t* verdict, int32_t* owner, hipStream_t s);

hipError_t launch_copy(bool guard, const DevTable& t, DevLog* log, void* dst, const void* src,
                       uint64_t n, unsigned long long seq, int logon, const DevInfo& d,
                       hipStream_t s);

hipError_t launch_triad(bool guard, const DevTable& t, DevLog* log, float* a, const float* b,
                        const float* c, float sc, uint64_t n, unsigned long long seq, int logon,
                        const DevInfo& d, hipStream_t s);

hipError_t launch_gather(bool guard, const DevTable& t, DevLog* log, void* out, const void* tab,
                         uint64_t row_bytes, const int64_t* idx, uint64_t n, uint32_t w,
                         unsigned long long seq, int logon, const DevInfo& d, hipStream_t s);

hipError_t launch_scatter(bool guard, const DevTable& t, DevLog* log, void* dst,
                          uint64_t row_bytes, const int64_t* idx, const void* src, uint64_t n,
                          uint32_t w, int accumulate, unsigned long long seq, int logon,
                          const DevInfo& d, hipStream_t s);

hipError_t launch_scatter_add(bool guard, const DevTable& t, DevLog* log, void* dst, uint64_t rb,
                              const int64_t* idx, const void* src, uint64_t n, uint32_t w,
                              unsigned long long seq, int logon, const DevInfo& d, hipStream_t s);

hipError_t launch_log_reset(DevLog* log, hipStream_t s);

}  // namespace agile

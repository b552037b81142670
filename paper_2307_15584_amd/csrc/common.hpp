// Shared host-side plumbing of the library: status/error reporting, the context object,
// device guards and launch checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "qmc.h"

namespace qmc {

// Per-thread text of the last failure, returned by qmc_last_error().
std::string& last_error_slot();

inline qmc_status fail(qmc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error_slot() = buf;
    return st;
}

inline qmc_status ok() { return QMC_OK; }

// Launch parameters chosen for one kernel family (defaults, or picked by the autotuner).
struct GenTune {
    uint32_t chunks_per_wave = 1;  // consecutive 256-index chunks of one dimension per wavefront
    uint32_t nontemporal = 0;      // streaming (non-temporal) stores for materialised points
};

struct IntegrateTune {
    uint32_t waves_per_cu = 16;  // persistent grid size, in wavefronts per compute unit
    uint32_t dynamic = 1;       // 1: atomic task queue, 0: static interleave of tiles
};

// A captured sequence of progressive passes, replayed with hipGraphLaunch.
struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace qmc

struct qmc_context_s {
    int device = 0;
    int num_cus = 256;
    int max_threads_per_cu = 2048;
    qmc::GenTune sobol_tune;
    qmc::GenTune lattice_tune;
    std::map<uint32_t, qmc::IntegrateTune> integrate_tunes;  // key: (kind, d, backward)
    hipStream_t capture_stream = nullptr;                    // private stream used only for graph capture
    std::vector<qmc::GraphEntry> graphs;
    void* static_scratch = nullptr;  // device address of the library's static scratch on this device
};

namespace qmc {

// Makes the context's device current for the duration of a call, restoring the caller's.
struct DeviceGuard {
    int prev = -1;
    bool switched = false;
    qmc_status status = QMC_OK;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) {
            status = fail(QMC_ERR_DEVICE, "hipGetDevice failed");
            return;
        }
        if (prev != dev) {
            if (hipSetDevice(dev) != hipSuccess) {
                status = fail(QMC_ERR_DEVICE, "hipSetDevice(%d) failed", dev);
                return;
            }
            switched = true;
        }
    }
    ~DeviceGuard() {
        if (switched) (void)hipSetDevice(prev);
    }
};

// Clears a stale error before a launch and reports the launch's own error after it.
inline void clear_launch_error() { (void)hipGetLastError(); }

inline qmc_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QMC_ERR_DEVICE, "%s: launch failed: %s", what, hipGetErrorString(e));
    return QMC_OK;
}

inline hipStream_t as_stream(qmc_stream s) { return reinterpret_cast<hipStream_t>(s); }

// Device address of the static scratch of qmc_integrate_pixels_l2_step_noalloc on `device`, which
// must be the current device; looked up once per device.
qmc_status static_scratch_address(int device, void** ptr);

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace qmc

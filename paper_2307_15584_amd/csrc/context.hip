// Context lifetime and error reporting.
#include "common.hpp"

namespace qmc {
std::string& last_error_slot() {
    static thread_local std::string slot;
    return slot;
}
}  // namespace qmc

extern "C" qmc_status qmc_create(int device, qmc_context* out) {
    if (!out) return qmc::fail(QMC_ERR_INVALID_ARGUMENT, "qmc_create: out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return qmc::fail(QMC_ERR_DEVICE, "qmc_create: no HIP device %d (%d visible)", device, count);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return qmc::fail(QMC_ERR_DEVICE, "qmc_create: hipGetDeviceProperties(%d) failed", device);
    void* scratch = nullptr;
    {
        qmc::DeviceGuard guard(device);
        if (guard.status != QMC_OK) return guard.status;
        const qmc_status st = qmc::static_scratch_address(device, &scratch);
        if (st != QMC_OK) return st;
    }
    auto* ctx = new qmc_context_s();
    ctx->device = device;
    ctx->num_cus = prop.multiProcessorCount;
    ctx->max_threads_per_cu = prop.maxThreadsPerMultiProcessor;
    ctx->static_scratch = scratch;
    *out = ctx;
    return QMC_OK;
}

extern "C" qmc_status qmc_destroy(qmc_context ctx) {
    if (!ctx) return QMC_OK;
    {
        qmc::DeviceGuard guard(ctx->device);
        for (auto& g : ctx->graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
        }
        if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    }
    delete ctx;
    return QMC_OK;
}

extern "C" const char* qmc_last_error(void) { return qmc::last_error_slot().c_str(); }

extern "C" const char* qmc_version(void) { return "qmc-gfx950 1.0"; }

// kdcd_krr_solve_noalloc: the s-step BDCD solve with its workspace in a
// fixed device array of the library instead of memory allocated per call, for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid allocation).
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"

namespace {

// The workspace of every no-allocation solve on a device; each device holds
// its own copy from the library's first use on it until the process ends.
__device__ __align__(256) char scratch[KDCD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of `scratch` per device, looked up once per device with that
// device current.  In host code the array's name is only a host-side stand-in:
// kernels and copies must be given this address instead.
struct ScratchTable {
    std::mutex mu;
    void *ptr[kMaxDevices] = {};
};

ScratchTable &scratch_table()
{
    static ScratchTable t;
    return t;
}

kdcd_status scratch_on_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return KDCD_ERR_HIP;
    if (dev >= kMaxDevices) return KDCD_ERR_UNSUPPORTED;
    ScratchTable &t = scratch_table();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KDCD_ERR_HIP;
        t.ptr[dev] = p;
    }
    *out = t.ptr[dev];
    return KDCD_OK;
}

}  // namespace

extern "C" {

kdcd_status kdcd_krr_solve_noalloc(const kdcd_matrix *A, const double *y,
                                   const kdcd_kernel *kernel, double lambda, int32_t b, int32_t s,
                                   int64_t H, const int32_t *idx, double *alpha,
                                   const kdcd_options *opt, kdcd_stream stream)
{
    kdcd_options o{};
    if (opt) {
        // each of these would allocate: a caller workspace is replaced by the
        // fixed array; the monitor's host poller, graph replay and the stage
        // timer allocate memory or events of their own
        if (opt->workspace || opt->workspace_bytes || opt->monitor_every || opt->flags ||
            opt->profile)
            return KDCD_ERR_UNSUPPORTED;
        o = *opt;
    }
    if (!A || b < 1 || s < 1) return KDCD_ERR_INVALID_ARG;
    const size_t need = kdcd_workspace_bytes(1, A, kernel, b, s, o.compute);
    if (need == 0) return KDCD_ERR_INVALID_ARG;
    if (need > (size_t)KDCD_NOALLOC_SCRATCH_BYTES) return KDCD_ERR_WORKSPACE;
    void *ws = nullptr;
    const kdcd_status rc = scratch_on_current_device(&ws);
    if (rc != KDCD_OK) return rc;
    o.workspace = ws;
    o.workspace_bytes = (size_t)KDCD_NOALLOC_SCRATCH_BYTES;
    return kdcd_krr_solve(A, y, kernel, lambda, b, s, H, idx, alpha, &o, stream);
}

}  // extern "C"

// Optimality Criteria update for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): otm_oc_update_noalloc.
//
// It computes what otm_oc_update computes (Sec. 3.3, OCOptimizer; Sec. 3.4
// step 6) from caller-owned device buffers, with the bisection's scratch --
// the per-block partial sums and the device scalars -- in one file-scope
// device array instead of a context's allocations.  q_e is recomputed from
// (rho_e, s_e) wherever it is needed, so no n^3-sized buffer is involved and
// the scratch is the same for every n.
//
// The array is per GPU and lives until the process ends.  Its device address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) at the first call there; host code uses that address, never the
// array's name.  Every call on a GPU shares the array, so calls that overlap
// on one GPU (two streams, two threads) race: the caller serialises them.
// Nothing in it has to start at zero: the bracket kernel initialises the
// bisection state and every partial is written before it is read.
#include <hip/hip_runtime.h>

#include <mutex>

#include "otm_internal.h"

namespace otm {
namespace {

// layout: [Scalars, padded to 4 KiB][partials]
constexpr size_t kScalarsBytes = 4096;
constexpr int kNoAllocBlocks = 1024;  // grid cap of the OC kernels' reductions
constexpr size_t kPartialDoubles = 512 * kMaxReduce;
constexpr size_t kScratchBytes = kScalarsBytes + kPartialDoubles * sizeof(double);
static_assert(sizeof(Scalars) <= kScalarsBytes, "device scalars exceed their slot");
static_assert(2 * kNoAllocBlocks <= (int)kPartialDoubles, "bracket partials exceed the scratch");
static_assert(512 * kOcCands <= (int)kPartialDoubles, "bisection partials exceed the scratch");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (set-up on first use).
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return OTM_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) return OTM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return OTM_EDEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return OTM_OK;
}

}  // namespace
}  // namespace otm

extern "C" int otm_oc_update_noalloc(int32_t n, const void* rho_dev, const void* sens_dev, double vstar,
                                     const otm_oc_opts* oc, void* rho_out_dev, void* lambda_dev, void* stream) {
    using namespace otm;
    if (!rho_dev || !sens_dev || !rho_out_dev || !oc) return OTM_EINVAL;
    if (n < 4 || n > 1024) return OTM_EINVAL;
    if (!(vstar > 0.0 && vstar <= 1.0)) return OTM_EINVAL;
    if (!(oc->move > 0.0 && oc->eta > 0.0 && oc->rho_min > 0.0 && oc->rho_min < 1.0)) return OTM_EINVAL;
    if (rho_out_dev == sens_dev || lambda_dev == rho_dev || lambda_dev == sens_dev || lambda_dev == rho_out_dev)
        return OTM_EINVAL;
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    Workspace ws{};
    ws.sc = (Scalars*)base;
    ws.partials = (double*)((unsigned char*)base + kScalarsBytes);
    ws.counter = nullptr;  // the OC kernels keep no completion counters
    ws.max_blocks = kNoAllocBlocks;
    (void)hipGetLastError();  // a stale error from earlier work is not this call's
    launch_oc_from_sens(n, (const double*)rho_dev, (const double*)sens_dev, (double*)rho_out_dev,
                        (double*)lambda_dev, vstar, oc->eta, oc->move, oc->rho_min, ws, (hipStream_t)stream);
    if (hipGetLastError() != hipSuccess) return OTM_EDEVICE;
    return OTM_OK;
}

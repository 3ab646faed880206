// pa_contract_noalloc: pa_contract for callers that cannot allocate device
// memory (code under hipGraph capture, serving loops, harnesses that forbid
// hipMalloc).  The one scratch buffer pa_contract needs -- the latent-entry
// table of a streamed contraction, otherwise a stream-ordered allocation
// filled from the host -- lives in a file-scope device array instead, and a
// kernel on the caller's stream writes it.  Every call on a GPU shares that
// GPU's array: calls that overlap on one GPU (on different streams, or from
// different threads) race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "pa_plan.h"

namespace pa {

// int64 entries of the static table: two per latent entry, so contractions
// with at most kNoAllocTabEntries latent entries (1 MiB per GPU, held until the
// process ends).
constexpr int64_t kNoAllocTabEntries = (int64_t)1 << 16;

static __device__ __align__(256) int64_t scratch[2 * kNoAllocTabEntries];

// The array's device address on each GPU (its host-side name is no device
// address), resolved once per device with that device current.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static int64_t *g_scratch_ptr[kMaxDevices] = {nullptr};

static int scratch_on_current_device(int64_t **ptr) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PA_EHIP, "contract_noalloc: no current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(PA_EUNSUPPORTED, "contract_noalloc: device index too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PA_EHIP, std::string("contract_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<int64_t *>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return PA_OK;
}

}  // namespace pa

using namespace pa;

extern "C" int pa_contract_noalloc(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B,
                                   const int32_t *b_vars, const int32_t *out_vars, int32_t n_out, pa_bitarray *C,
                                   const pa_opts *opts, void *stream) {
    int64_t *tab = nullptr;
    int rc = scratch_on_current_device(&tab);
    if (rc) return rc;
    return contract_impl(A, a_vars, B, b_vars, out_vars, n_out, C, opts, stream, tab, 2 * kNoAllocTabEntries);
}

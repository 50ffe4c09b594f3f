// Allocation-free fitness entry point: hpmocd_eval with its scratch in a fixed device array
// instead of a caller workspace, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.hpp"
#include "run.hpp"

// The eval workspace of hpmocd_eval_noalloc: the transposed labels, the histogram areas, the
// accumulators, the label-range flag and the item table. One copy per device, held by the
// loaded code object until the process ends. Host code never uses this name as an address
// (on the host it names a stand-in, not device memory): it asks each device for the array's
// address once and passes that.
static __device__ __align__(256) unsigned char scratch[HPMOCD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be the current device. Looked up on
// the first call for that device and kept.
int scratch_on(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return HPMOCD_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return HPMOCD_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HPMOCD_OK;
}

}  // namespace

using namespace hpm;

extern "C" int hpmocd_eval_noalloc(const hpmocd_graph *G, const int32_t *d_labels,
                                   int32_t n_ind, void *stream, int64_t *A, int64_t *S,
                                   double *f1, double *f2)
{
    return c_guard([&]() -> int {
        if (!G || !d_labels || n_ind < 1 || !A || !S || !f1 || !f2) return HPMOCD_ERR_ARG;
        int rc = check_device(G);
        if (rc) return rc;
        size_t need = 0;
        if ((rc = hpmocd_eval_workspace_size(G, n_ind, &need))) return rc;
        if (need > HPMOCD_NOALLOC_SCRATCH_BYTES) return HPMOCD_ERR_SCRATCH;
        void *ws = nullptr;
        if ((rc = scratch_on(G->device, &ws))) return rc;
        return eval_on(G, d_labels, n_ind, ws, (hipStream_t)stream, A, S, f1, f2, nullptr);
    });
}

// hs_noalloc.hip -- hs_price_greeks_noalloc: the Greek set of hs_price_greeks
// run in a workspace the library holds itself, for callers that cannot
// allocate device memory.  The workspace is a file-scope device array,
// `scratch`, of HS_NOALLOC_SCRATCH_BYTES; every GPU the library runs on holds
// its own copy until the process ends.  Its device address is looked up once
// per device (hipGetSymbolAddress, with that device current) on the first
// call there, and only that address is handed to the kernels: in host code
// the array's name is a host-side stand-in, not a device address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/hs_api.h"
#include "hs_plan.hpp"
#include "hs_run.hpp"

namespace hs {
namespace {

__device__ __align__(256) unsigned char scratch[HS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch array (looked up on first use).
hs_status scratch_of(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("hs_price_greeks_noalloc: device %d outside 0..%d", dev, kMaxDevices - 1);
        return HS_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hs_price_greeks_noalloc: hipGetSymbolAddress of the scratch array failed: %s",
                      hipGetErrorString(e));
            return HS_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HS_OK;
}

}  // namespace
}  // namespace hs

using namespace hs;

extern "C" hs_status hs_price_greeks_noalloc(const hs_model* model, const double* corr,
                                             const hs_option* option, int64_t n_paths,
                                             int32_t n_steps, const hs_bumps* bumps,
                                             const hs_opts* opts, void* hip_stream,
                                             hs_greeks* out)
{
    if (!out) {
        set_error("hs_price_greeks_noalloc: null out");
        return HS_EINVAL;
    }
    Request q;
    hs_status rc = copy_request(model, corr, option, n_paths, n_steps, bumps, opts, q);
    if (rc != HS_OK) return rc;
    rc = validate(q);
    if (rc != HS_OK) return rc;
    if (q.opts.flags & (HS_FLAG_GRAPH | HS_FLAG_TIMING)) {
        set_error("hs_price_greeks_noalloc: HS_FLAG_GRAPH and HS_FLAG_TIMING create runtime "
                  "objects and are not accepted here");
        return HS_EINVAL;
    }
    const size_t need = workspace_bound(q, true);
    if (need == 0 || need > HS_NOALLOC_SCRATCH_BYTES) {
        set_error("hs_price_greeks_noalloc: the request needs at least %zu bytes of workspace, "
                  "the static scratch holds %zu",
                  need, static_cast<size_t>(HS_NOALLOC_SCRATCH_BYTES));
        return HS_ENOMEM;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hs_price_greeks_noalloc: no current device");
        return HS_EDEVICE;
    }
    void* ws = nullptr;
    rc = scratch_of(dev, &ws);
    if (rc != HS_OK) return rc;
    RunResult res;
    rc = run_greek_set(q, ws, HS_NOALLOC_SCRATCH_BYTES, static_cast<hipStream_t>(hip_stream), res,
                       nullptr);
    if (rc != HS_OK) return rc;
    fill_greeks(q, res, out);
    return HS_OK;
}

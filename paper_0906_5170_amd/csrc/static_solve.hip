// cf_solve_static: the force solve of cf_solve for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its workspace is a fixed array in
// device memory that the library holds on every device it runs on, instead
// of a buffer the caller passes or the library allocates.
//
// The array's address differs per device and is not the host-side symbol:
// the first call on a device looks it up with hipGetSymbolAddress (with that
// device current) and keeps it; every later use passes that address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/casimir_fdtd.h"
#include "solver.hpp"

namespace {

constexpr size_t kScratchBytes = CF_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// One lock per device: calls on the same device run one after another, since
// they share that device's array.
std::mutex g_mu[kMaxDevices];
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device (set up on first use)

}  // namespace

extern "C" cf_status cf_solve_static(cf_problem* p, const cf_opts* o, cf_result* out) {
    return cfi::guarded([&]() -> cf_status {
        if (!p || !o || !out) return cfi::fail(CF_E_ARG, "null argument");
        if (o->flags & CF_FLAG_GRAPH)
            return cfi::fail(CF_E_UNSUPPORTED, "cf_solve_static does not take CF_FLAG_GRAPH (instantiating a graph allocates)");
        size_t need = 0;
        const cf_status st = cf_workspace_size(p, o, &need);
        if (st != CF_OK) return st;
        if (need > kScratchBytes)
            return cfi::fail(CF_E_BUDGET, "this solve needs " + std::to_string(need) +
                                              " bytes of workspace; cf_solve_static holds at most " +
                                              std::to_string(kScratchBytes) + " (use cf_solve with a workspace)");
        int dev = -1;
        const hipError_t ed = hipGetDevice(&dev);
        if (ed != hipSuccess) return cfi::fail(CF_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(ed));
        if (dev < 0 || dev >= kMaxDevices) return cfi::fail(CF_E_DEVICE, "device ordinal beyond the supported range");
        std::lock_guard<std::mutex> lk(g_mu[dev]);
        if (!g_scratch[dev]) {
            void* ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return cfi::fail(CF_E_DEVICE, std::string("hipGetSymbolAddress of the static workspace: ") +
                                                  hipGetErrorString(e));
            g_scratch[dev] = ptr;
        }
        // cf_solve allocates nothing when it is given a workspace; it clears
        // the accumulators, Gamma rows and field arrays it reads first, so the
        // previous call's contents do not matter
        return cf_solve(p, o, g_scratch[dev], kScratchBytes, out);
    });
}

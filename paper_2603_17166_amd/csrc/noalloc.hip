// Synthesis without any device allocation (psht_synth_noalloc, include/psht.h).
//
// The workspace of the synthesis (the ring coefficients F, the Theta-stage
// output V and the used NUFFT grid rows U, see capi.cpp) comes from a
// file-scope device array instead of a caller buffer.  Each GPU the library
// runs on holds its own copy of the array for the lifetime of the process.
// Host code never passes the array's name to a kernel (in host code it names
// a host-side stand-in): the device address of each GPU's copy is looked up
// once per device with hipGetSymbolAddress and that address is used.
//
// The synthesis stages write every element of the workspace they later read
// (F on the active rings, every used row of V and U), so nothing has to be
// cleared between calls.
#include <mutex>

#include "psht_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // PSHT_NOALLOC_SCRATCH_BYTES in include/psht.h
static_assert(kScratchBytes == PSHT_NOALLOC_SCRATCH_BYTES, "scratch size and header disagree");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of this device's scratch array (looked up on first use).
psht_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return psht::set_error(PSHT_ERR_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return psht::set_error(PSHT_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return psht::set_error(PSHT_ERR_DEVICE, (std::string("hipGetSymbolAddress(scratch): ") +
                                                     hipGetErrorString(e)).c_str());
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PSHT_OK;
}

}  // namespace

extern "C" psht_status psht_synth_noalloc(psht_plan plan, int nmaps, const void *alm, void *map, void *hip_stream) {
    if (!plan) return psht::set_error(PSHT_ERR_ARG, "plan is NULL");
    if (nmaps < 0) return psht::set_error(PSHT_ERR_ARG, "nmaps < 0");
    const size_t need = (size_t)nmaps * plan->ws_per_map;
    if (need > kScratchBytes)
        return psht::set_error(PSHT_ERR_WORKSPACE,
                               ("psht_synth_noalloc: the plan needs " + std::to_string(need) +
                                " bytes of workspace, above the static scratch of " + std::to_string(kScratchBytes) +
                                " bytes; use psht_synth with a caller workspace")
                                   .c_str());
    void *ws = nullptr;
    psht_status s = scratch_address(&ws);
    if (s != PSHT_OK) return s;
    return psht::synth_run(plan, nmaps, alm, map, ws, kScratchBytes, 1.0, hip_stream);
}

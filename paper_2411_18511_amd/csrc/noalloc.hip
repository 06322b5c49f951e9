// hrd_dirac_apply_static: hrd_dirac_apply for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// allocation).  The even/odd operator's odd temporary lives in a file-scope
// device array instead of a caller workspace; every other parity mode needs
// no temporary.  The array is per device, shared by every call on that
// device, and sized once for the process (kScratchBytes).
#include <mutex>

#include "api_util.h"
#include "hrd.h"

namespace hrd {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // the largest odd temporary accepted
constexpr int kMaxDevices = 64;

// Device memory of the odd temporary.  In host code this name is only a
// handle for hipGetSymbolAddress: the kernels receive the device address
// looked up once per device below, never the name itself.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
hrd_status scratch_on_current_device(void **ptr)
{
    int dev = -1;
    HRD_TRY(check_hip(hipGetDevice(&dev), "hipGetDevice"));
    if (dev < 0 || dev >= kMaxDevices) return fail(HRD_EINVAL, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HRD_TRY(check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
        if (!p) return fail(HRD_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return HRD_OK;
}

}  // namespace
}  // namespace hrd

using namespace hrd;

extern "C" {

size_t hrd_dirac_static_scratch_bytes(void) { return kScratchBytes; }

hrd_status hrd_dirac_apply_static(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, const void *U,
                                  const void *psi, void *out, double m0, hrd_parity parity, int dagger, void *stream)
{
    void *work = nullptr;
    if (parity == HRD_EO) {
        HRD_TRY(check_lattice(lat));
        HRD_TRY(check_rep_prec_any(rep, prec));
        const size_t need = spinor_bytes(lat, rep, prec, 1);
        if (need > kScratchBytes)
            return fail(HRD_ESIZE, "dirac_apply_static: HRD_EO needs a %zu-byte odd temporary, beyond the %zu bytes "
                        "of the static scratch (use hrd_dirac_apply with a workspace)", need, kScratchBytes);
        HRD_TRY(scratch_on_current_device(&work));
    }
    return dirac_apply_checked(lat, rep, prec, U, psi, out, m0, parity, dagger, work, stream);
}

}  // extern "C"

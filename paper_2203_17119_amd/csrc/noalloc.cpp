// The Schur operator on internal fields without any device allocation.
//
// dwf_schur_apply_internal applies Mpc (or Mpc^+) in two fused stencil stages
// with one or two intermediate fields, which it takes from the context's
// workspaces (allocated on first use).  This variant takes them from a fixed
// device array instead, so that callers that cannot allocate device memory
// (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc) can apply the operator.  The array is one per device for the
// whole process; its device address is looked up once per device when a
// context is created there.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dwf_internal.h"

namespace dwf {

// the largest intermediate storage one call may need: two fields of the
// call's precision (FP32 at 16^4 x 12, 75.5 MB, fits)
constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;

// File-scope device array; in host code its name is only a stand-in for the
// symbol, never an address: every use below goes through the pointer that
// hipGetSymbolAddress returns for the device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex scratch_mutex;
static void *scratch_dev[kMaxDevices] = {};

// Looks up the array's address on `device`, which must be the current device.
void scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) fail(DWF_ENOTSUP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (scratch_dev[device]) return;
    void *p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(DWF_EDEVICE, "no device address for the scratch array");
    scratch_dev[device] = p;
}

static void *scratch_of(int device)
{
    std::lock_guard<std::mutex> lock(scratch_mutex);
    return (device >= 0 && device < kMaxDevices) ? scratch_dev[device] : nullptr;
}

}  // namespace dwf

using namespace dwf;

extern "C" dwf_status dwf_schur_apply_internal_noalloc(dwf_ctx ctx, int prec, int dagger, const void *in, void *out)
{
    DWF_API_BEGIN
    if (!ctx) fail(DWF_EINVAL, "null context");
    if (!in || !out) fail(DWF_EINVAL, "null field pointer");
    if (in == out) fail(DWF_EINVAL, "in and out must differ");
    if (prec < P_F64 || prec > P_BF16) fail(DWF_EINVAL, "unknown precision");
    dwf::Context &c = *ctx;
    if (!c.links[prec][0] || !c.links[prec][1])
        fail(DWF_EINVAL, "links of this precision are not prepared: call an operator or solver of this precision "
                         "once beforehand (this entry point allocates nothing)");
    // the fused stages write every byte of both intermediates (payload and,
    // for FP16, the site scales) before reading them: nothing needs clearing
    const long stride = batch_stride(c, prec);
    const int nfields = dagger ? 1 : 2;
    if ((size_t)stride * nfields > kScratchBytes)
        fail(DWF_EINVAL, "lattice too large for the fixed scratch array (" + std::to_string(kScratchBytes >> 20) +
                             " MiB: two intermediate fields of the precision)");
    char *base = (char *)scratch_of(c.device);
    if (!base) fail(DWF_EDEVICE, "scratch array not resolved on this device");
    Field ta = make_field(c, base, prec);
    Field y = make_field(c, base + (dagger ? 0 : stride), prec);
    // kernel timing would create events: off for this call
    const int timing = c.timing;
    c.timing = 0;
    try {
        apply_mpc(c, prec, dagger != 0, make_field(c, (void *)in, prec), make_field(c, out, prec), false, false,
                  Field{}, 1, 0, -1, ta, y);
    } catch (...) {
        c.timing = timing;
        throw;
    }
    c.timing = timing;
    DWF_API_END
}

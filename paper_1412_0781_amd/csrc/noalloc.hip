// fb_expand_noalloc: the expansion a = T* I with its pass buffers in a fixed device array of
// this library instead of a caller-provided workspace, for callers that cannot allocate.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ffbspca.h"
#include "plan.h"

namespace {

// One array per device, loaded with the library's code object and held until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy: on the host the
// name is a stand-in, and its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[FB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// Device address of `scratch` on the current device `dev` (looked up once per device,
// with that device current).
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int fb_expand_noalloc(fb_plan_t plan, const float* images, int64_t n, float* coeffs, int precision,
                                 void* stream) {
  if (!plan || n < 0) return FB_ERR_INVALID_ARG;
  if (precision != FB_FP32 && precision != FB_BF16X3) return FB_ERR_INVALID_ARG;
  fb::Plan& pl = plan->pl;
  // one pass holds at least one group of 16 images (plus the alignment slack of the split)
  const size_t need = fb::pass_layout(pl).per_image * (size_t)fb::kImgGroup + 2 * 256;
  if (need > (size_t)FB_NOALLOC_SCRATCH_BYTES) return FB_ERR_SCRATCH_LIMIT;
  if (!pl.has_device) return FB_ERR_NO_DEVICE;
  // the per-kernel timer creates HIP events, i.e. allocates: not allowed here
  if (pl.prof.on) return FB_ERR_INVALID_ARG;
  if (n == 0) return FB_OK;
  if (!images || !coeffs) return FB_ERR_INVALID_ARG;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
  if (e != hipSuccess) {
    pl.last_hip = e;
    return FB_ERR_HIP;
  }
  // the plan's tables live on the device it was built on; the array used must be that device's
  if (dev != pl.device) return FB_ERR_INVALID_ARG;
  void* ws = nullptr;
  e = scratch_address(dev, &ws);
  if (e != hipSuccess) {
    pl.last_hip = e;
    return FB_ERR_HIP;
  }
  return fb_expand(plan, images, n, coeffs, precision, ws, (size_t)FB_NOALLOC_SCRATCH_BYTES, stream);
}

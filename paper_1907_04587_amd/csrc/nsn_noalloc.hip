// The loss/gradient entry point that allocates nothing (nsn_mlp_loss_grad_noalloc):
// the same kernels as nsn_mlp_loss_grad, with their per-block partial gradients in a
// file-scope device array instead of a caller-given scratch buffer.
#include <hip/hip_runtime.h>

#include <string>

#include "nsn_layout.h"

// Room for the partial gradients of the loss kernel's largest grid (256 workgroups of
// 9347 floats, plus their loss terms): about 9.6 MB per device, held until the process
// ends.  In host code the name is only the runtime's handle of this array; kernels get
// its device address from hipGetSymbolAddress.
static constexpr size_t kScratchBytes = 10u << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace nsn {
namespace {

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, taken once

nsn_status scratch_of_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return set_error(NSN_EDEVICE, "nsn_mlp_loss_grad_noalloc: no current device (or more than 64)");
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(NSN_EDEVICE, std::string("nsn_mlp_loss_grad_noalloc: hipGetSymbolAddress: ") +
                                        hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return NSN_OK;
}

}  // namespace
}  // namespace nsn

using namespace nsn;

extern "C" {

size_t nsn_mlp_noalloc_scratch_bytes(void) { return kScratchBytes; }

nsn_status nsn_mlp_loss_grad_noalloc(const float *w, const float *x, const float *t, int64_t n, float *grad,
                                     float *loss_out, void *stream) {
  if (!w || !x || !t || !grad || n <= 0) return set_error(NSN_EINVAL, "nsn_mlp_loss_grad_noalloc: bad arguments");
  const size_t need = nsn_mlp_scratch_bytes(n);
  if (need > kScratchBytes)
    return set_error(NSN_EUNSUPPORTED, "nsn_mlp_loss_grad_noalloc: " + std::to_string(n) + " samples need " +
                                           std::to_string(need) + " bytes of scratch, more than the " +
                                           std::to_string(kScratchBytes) + " it holds");
  void *ptr = nullptr;
  const nsn_status st = scratch_of_current_device(&ptr);
  if (st) return st;
  // every call rewrites all the partials it reads (nothing needs clearing); calls that
  // overlap on one device share the array and race
  return nsn_mlp_loss_grad(w, x, t, n, grad, loss_out, ptr, stream);
}

}  // extern "C"

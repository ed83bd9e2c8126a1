// Interpolation without allocation: the derivative buffer of apc_interpolate_force
// (n x p doubles) lives in a file-scope device array instead of the temporary
// cache, so the call makes no hipMalloc / hipFree (for callers that cannot
// allocate: graph capture, tight serving loops).
//
// Each GPU holds its own copy of the array, at its own address, until the process
// ends.  In host code the array's name is not a device address, so the address is
// taken once per device with hipGetSymbolAddress (that device current) and kept
// in g_dev; kernels only ever receive that address.  Calls that overlap on one
// GPU share the array and race; the derivative kernel writes every row the
// particle kernel reads, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "apc_internal.h"

namespace {
constexpr int64_t SCRATCH_DOUBLES = APC_NOALLOC_BYTES / 8;
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_dev[MAX_DEVICES] = {};
} // namespace

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

// The device address of this GPU's array (taken on the first call per device).
static int scratch_ptr(double **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    apc_set_error_msg("interpolate_force_noalloc: device index out of range");
    return APC_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_dev[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_dev[dev] = (double *)p;
  }
  *out = g_dev[dev];
  return APC_OK;
}

int apc_interp_noalloc_impl(apc_cloud *c, const double *phi, double *phi_p, double *grad_p,
                            hipStream_t s) {
  const int64_t need = c->n * (int64_t)c->p;
  if (need > SCRATCH_DOUBLES) {
    apc_set_error_msg("interpolate_force_noalloc: n x p derivatives exceed the fixed "
                      "buffer (APC_NOALLOC_BYTES)");
    return APC_EINVAL;
  }
  double *D = nullptr;
  APCCHK(scratch_ptr(&D));
  return apc_interp_with(c, phi, phi_p, grad_p, D, s);
}

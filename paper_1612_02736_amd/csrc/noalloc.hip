// Allocation-free variant of hps_solve: the solve's work vectors and split-K
// partials live in one fixed device array of this library instead of
// buffers the handle allocates on demand.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>

#include "../../include/hps.h"

// defined in hps_api.cpp
int hps_solve_on_scratch(hps_handle *h, const double *f, const double *g, int nrhs, double *u,
                         const hps_solve_opts *opts, double *work, size_t bytes);
int hps_set_error(int code, const char *msg);

constexpr size_t kScratchBytes = HPS_SOLVE_NOALLOC_MAX_BYTES;

// Each device that loads the library holds its own copy until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host it
// names a stand-in, not device memory): it uses the address that
// hipGetSymbolAddress returns on each device.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of this device's array, looked up once per device with the
// device current (the caller's current device).
int scratch_address(double **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return hps_set_error(HPS_EHIP, "hipGetDevice failed or device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return hps_set_error(HPS_EHIP, "hipGetSymbolAddress of the solve work array failed");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double *>(g_scratch_ptr[dev]);
  return HPS_OK;
}

}  // namespace

extern "C" int hps_solve_noalloc(hps_handle *h, const double *f, const double *g, int nrhs,
                                 double *u, const hps_solve_opts *opts) {
  double *work = nullptr;
  const int rc = scratch_address(&work);
  if (rc) return rc;
  return hps_solve_on_scratch(h, f, g, nrhs, u, opts, work, kScratchBytes);
}

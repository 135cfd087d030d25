// lb_adjoint_step_noalloc: the reverse mode of one step (as lb_adjoint_step)
// for callers that cannot allocate device memory, with the adjoint's scratch
// (the predictor state, its adjoint, R0_bar, the ln M gradient adjoint and
// the per-site eta/s partials) in a file-scope device array instead of a
// caller's workspace.
//
// The array is a device symbol: in host code its name is not a device
// address, so the entry point looks its address up once per device
// (hipGetSymbolAddress with that device current) and passes only that
// address to the kernels.  Every call on a device shares the device's copy;
// nothing in it has to start at zero (each call writes every scratch value
// before it reads it), and calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/lb.h"

namespace lbmi {
int set_error(int code, const char* msg);
int context_device(const lb_ctx* c);
size_t context_adjoint_bytes(const lb_ctx* c);
}  // namespace lbmi

namespace {

// 80 MiB: the 128 x 128 grid of the gradient workload needs 75.6 MiB
// (4840 bytes per site and 256-byte alignment).  Held by every device the
// library is loaded on until the process ends.
constexpr size_t kScratchBytes = (size_t)80 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of scratch (looked up once).
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != dev) {
      const hipError_t e2 = hipSetDevice(prev);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int lb_adjoint_step_noalloc(lb_ctx* c, double tau_fm, double dtau_fm, const double* d_F,
                                       const double* d_lnM, double* d_adj_F, double* d_adj_lnM,
                                       double* d_grad_eta_over_s) {
  if (!c) return lbmi::set_error(LB_E_STATE, "context not initialised");
  const size_t need = lbmi::context_adjoint_bytes(c);
  if (need == 0) return lbmi::set_error(LB_E_STATE, "context not initialised");
  if (need > kScratchBytes)
    return lbmi::set_error(LB_E_ARG, ("grid too large for the static adjoint scratch: needs " + std::to_string(need) +
                                      " bytes, the maximum is " + std::to_string(kScratchBytes) +
                                      " (about 17000 sites); use lb_adjoint_step with a workspace")
                                         .c_str());
  const int dev = lbmi::context_device(c);
  if (dev < 0 || dev >= kMaxDevices) return lbmi::set_error(LB_E_ARG, "device index out of range");
  void* p = nullptr;
  const hipError_t e = scratch_address(dev, &p);
  if (e != hipSuccess)
    return lbmi::set_error(LB_E_HIP, (std::string("hipGetSymbolAddress: ") + hipGetErrorString(e)).c_str());
  return lb_adjoint_step(c, tau_fm, dtau_fm, d_F, d_lnM, d_adj_F, d_adj_lnM, d_grad_eta_over_s, p, kScratchBytes);
}

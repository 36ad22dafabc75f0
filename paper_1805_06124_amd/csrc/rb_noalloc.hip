// rb_greedy_z_noalloc: the FP64 greedy for callers that cannot allocate
// memory.  Its workspace is a fixed device array of this library, `scratch`;
// each device holds its own copy at its own address, which the host learns
// once per device from hipGetSymbolAddress (the array's name in host code is
// only a host-side stand-in, never a device address).
#include <mutex>

#include "rb_host.h"

using namespace rb;

namespace {

__device__ __align__(256) unsigned char scratch[RB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// The current device's address of `scratch` (looked up on its first use on
// that device, with that device current).
int scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(RB_EDEVICE, "rb_greedy_z_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(RB_EDEVICE, "rb_greedy_z_noalloc: device %d not supported", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(RB_EDEVICE, "rb_greedy_z_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RB_OK;
}

}  // namespace

extern "C" {

int rb_greedy_z_noalloc(const void* S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, void* W,
                        int64_t ldW, void* E, int64_t ldE, int64_t* piv, double* err, double* rho, int32_t* nu,
                        int64_t* k_out, const rb_opts* opts, rb_stats* stats, hipStream_t stream) {
  last_error().clear();
  if (!W) return set_error(RB_EINVAL, "rb_greedy_z_noalloc: W is required (it may be S)");
  rb_opts o;
  rb_default_opts(&o);
  if (opts) o = *opts;
  o.collect_stats = 0;  // HIP events are runtime objects: not created here
  const size_t need = greedy_z_ws_bytes(N, M, kmax, &o);
  if (need > RB_NOALLOC_SCRATCH_BYTES)
    return set_error(RB_ENOMEM, "rb_greedy_z_noalloc: workspace of %zu bytes exceeds the fixed %zu (lower anchor_max)",
                     need, (size_t)RB_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  int rc = scratch_for_current_device(&ws);
  if (rc != RB_OK) return rc;
  return greedy_z_core("rb_greedy_z_noalloc", S, N, M, ldS, tol, kmax, W, ldW, E, ldE, 0, piv, err, rho, nu, k_out,
                       ws, RB_NOALLOC_SCRATCH_BYTES, &o, stats, stream);
}

}  // extern "C"

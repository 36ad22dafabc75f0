// Host-side helpers shared by the C-ABI translation units (error state,
// RAII device/pinned buffers, event timers).
#pragma once

#include <cstdarg>
#include <cstdio>
#include <string>

#include "rb_internal.h"

namespace rb {

// per-thread message of the last failing call
std::string& last_error();
int set_error(int code, const char* fmt, ...);

// The FP64 greedy started from k0 >= 0 orthonormal vectors in E[:, 0..k0-1]
// (rb_greedy_z for k0 = 0, rb_greedy_resume_z otherwise); fn names the entry
// point in error messages.
int greedy_z_core(const char* fn, const void* S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax,
                  void* W, int64_t ldW, void* E, int64_t ldE, int64_t k0, int64_t* piv, double* err, double* rho,
                  int32_t* nu, int64_t* k_out, void* ws, size_t ws_bytes, const rb_opts* opts, rb_stats* stats,
                  hipStream_t stream);
// Workspace bytes of greedy_z_core (0 for invalid sizes or options).
size_t greedy_z_ws_bytes(int64_t N, int64_t M, int64_t kmax, const rb_opts* opts);

#define RB_HIP(expr)                                                                                \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return ::rb::set_error(RB_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Device buffer owned by one call.
struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1); }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

// Pinned host buffer owned by one call.
struct HostBuf {
  void* p = nullptr;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipHostMalloc(&p, bytes, hipHostMallocDefault); }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

#define RB_ALLOC(buf, bytes)                                                                         \
  do {                                                                                               \
    if ((buf).alloc(bytes) != hipSuccess) {                                                          \
      (void)hipGetLastError();                                                                       \
      return ::rb::set_error(RB_ENOMEM, "device allocation of %zu bytes failed", (size_t)(bytes));   \
    }                                                                                                \
  } while (0)

// Accumulates device time between start() and stop() with HIP events on one
// stream (stop() synchronises on its event); inactive unless enabled.
struct EventTimer {
  bool on = false;
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s = nullptr;
  EventTimer(bool enable, hipStream_t st) : on(enable), s(st) {
    if (on) {
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) on = false;
    }
  }
  ~EventTimer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  void start() {
    if (on) (void)hipEventRecord(a, s);
  }
  void stop(double* acc) {
    if (!on) return;
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    *acc += ms;
  }
};

inline bool valid_ld(int64_t N, int64_t ld) { return ld >= N && ld > 0; }

// Slices of one workspace buffer, each 256-byte aligned.  With base ==
// nullptr only the size is counted (the same sequence of take() calls sizes
// a workspace and then carves it).
struct Carve {
  char* base = nullptr;
  size_t used = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    const size_t off = (used + 255) & ~static_cast<size_t>(255);
    used = off + sizeof(T) * (count ? count : 1);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// Host words the greedies read back after each step: pinned memory when the
// call may allocate, else a buffer on the caller's stack (a synchronous copy
// to pageable memory; no allocation).
struct HostWords {
  HostBuf pinned;
  alignas(64) unsigned char local[1024];
  unsigned char* p = local;
  // bytes <= sizeof local
  hipError_t init(bool may_alloc, size_t bytes) {
    if (!may_alloc) return hipSuccess;
    hipError_t e = pinned.alloc(bytes);
    if (e == hipSuccess) p = pinned.as<unsigned char>();
    return e;
  }
  template <class T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(p + off);
  }
};

// Per-step and total device time of one phase (collect_stats): adds the
// timer's interval to *total and, if slot is non-null, to *slot.
inline void lap(EventTimer& tm, double* total, double* slot) {
  if (!tm.on) return;
  double t = 0.0;
  tm.stop(&t);
  *total += t;
  if (slot) *slot += t;
}

}  // namespace rb

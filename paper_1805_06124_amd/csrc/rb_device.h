// Device-side helpers inlined into the kernels of librb.so: the chirp
// phase, streaming loads, wave reductions, the pivot search's coefficient
// arithmetic, error-free sums and the (value, index) argmax.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rb {

constexpr int kWave = 64;

// ---------------------------------------------------------------- device --

// Phase of the chirp family, Psi(f) = -pi/4 + A f^(-5/3) + B f^(-1) (the
// leading and first post-Newtonian terms) for total mass m (solar masses)
// and mass ratio q, evaluated from the grid table (tab[3n+1] = f_n^(-5/3),
// tab[3n+2] = 1/f_n).  One definition for every kernel that forms the
// surrogate's phase inputs, rounded step by step, so they agree bit for bit.
constexpr double kChirpTsun = 4.925490947641267e-6;  // GM_sun / c^3 [s]
constexpr double kChirpPi = 3.14159265358979323846;
__device__ __forceinline__ void chirp_phase_coeffs(double m, double q, double& A, double& B) {
#pragma clang fp contract(off)
  const double pm = kChirpPi * m * kChirpTsun;
  const double eta = q / ((1.0 + q) * (1.0 + q));
  const double a0 = 3.0 / (128.0 * eta);
  A = a0 * pow(pm, -5.0 / 3.0);
  B = a0 * (3715.0 / 756.0 + 55.0 * eta / 9.0) / pm;
}
__device__ __forceinline__ double chirp_phase(double A, double B, const double* tab, int64_t n) {
#pragma clang fp contract(off)
  return -kChirpPi / 4.0 + A * tab[3 * n + 1] + B * tab[3 * n + 2];
}
// the surrogate's inputs of a sample: the parameters mapped onto [-1, 1]
__device__ __forceinline__ float box_map(double v, double lo, double hi) {
#pragma clang fp contract(off)
  return (float)(2.0 * (v - lo) / (hi - lo) - 1.0);
}

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

// Streaming 16-byte load that bypasses cache retention (S is read once per
// sweep; keeping it out of L2/MALL leaves room for the basis vector).
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return make_float2(v.x, v.y);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// The pivot search's coefficient arithmetic, shared by every kernel that
// forms c = e^H x for it: each lane accumulates conj(e_n) x_n over its rows
// n = lane, lane + 64, lane + 128, ... in increasing order with explicit
// fused multiply-adds, then wave_sum adds the 64 lane sums.  Any two kernels
// that keep this order produce the same bits for the same (e, x), whatever
// their unrolling or how many columns and vectors a wave carries.
__device__ __forceinline__ void sweep_cmac(const double2 e, const double2 s, double& re, double& im) {
  re = __builtin_fma(e.y, s.y, __builtin_fma(e.x, s.x, re));
  im = __builtin_fma(-e.y, s.x, __builtin_fma(e.x, s.y, im));
}
// acc + |c|^2, rounded the same way wherever the running sum of Eq. (6.3)
// is advanced
__device__ __forceinline__ double sweep_acc_add(double a, double cr, double ci) {
#pragma clang fp contract(off)
  return a + __builtin_fma(cr, cr, ci * ci);
}

// Error-free transformations (Knuth two-sum; fma product) for the exact
// squared norms.  Contraction is switched off in each of them: fusing the
// product v*v into the following sum would break the two-sum identity.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
struct dd {
  double hi, lo;
};
__device__ __forceinline__ void dd_add_sq(dd& x, double v) {
#pragma clang fp contract(off)
  double p = v * v;
  double pe = __builtin_fma(v, v, -p);
  double s, e;
  two_sum(x.hi, p, s, e);
  x.hi = s;
  x.lo += e + pe;
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
  double s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  dd r;
  r.hi = s + e;  // fast two-sum renormalisation
  r.lo = e - (r.hi - s);
  return r;
}
__device__ __forceinline__ dd wave_dd_sum(dd x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dd y;
    y.hi = __shfl_xor(x.hi, o, kWave);
    y.lo = __shfl_xor(x.lo, o, kWave);
    x = dd_add(x, y);
  }
  return x;
}

// (value, index) argmax with ties to the lowest index.  A NaN value ranks
// above every number (so a non-finite estimate reaches the host instead of
// dropping out of the search).  The combination is a maximum under a total
// order, hence associative and commutative: every reduction order gives the
// same result.
struct vi {
  double v;
  int64_t i;
};
// An index < 0 marks "no candidate".
__device__ __forceinline__ vi vi_max(vi a, vi b) {
  if (a.i < 0) return b;
  if (b.i < 0) return a;
  const bool an = a.v != a.v, bn = b.v != b.v;
  if (an != bn) return an ? a : b;
  if (!an) {
    if (b.v > a.v) return b;
    if (b.v < a.v) return a;
  }
  return (b.i < a.i) ? b : a;
}
__device__ __forceinline__ vi wave_vi_max(vi x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    vi y;
    y.v = __shfl_xor(x.v, o, kWave);
    y.i = __shfl_xor(x.i, o, kWave);
    x = vi_max(x, y);
  }
  return x;
}

}  // namespace rb

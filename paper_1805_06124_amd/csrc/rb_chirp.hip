// Synthetic snapshot family standing in for the paper's gravitational-wave
// model (Sec. 6.1.1): column j is the leading-1PN frequency-domain chirp
//   h(f) = f^(-7/6) exp(-i Psi(f)),
//   Psi  = -pi/4 + 3/(128 eta v^5) (1 + (3715/756 + 55 eta/9) v^2),
//   v    = (pi Mtot f)^(1/3),  eta = q/(1+q)^2,
// with Mtot = total mass (solar masses) * GM_sun/c^3 seconds, on the uniform
// grid f_n = flo + n (fhi - flo)/(N - 1), divided by its L2 norm.  FP64
// throughout; complex64 output is the rounded normalised value.
// One workgroup per column: pass 1 evaluates the column and accumulates its
// exact squared norm, pass 2 writes the normalised values.
#include "rb_internal.h"

namespace rb {

namespace {

constexpr double kTsun = 4.925490947641267e-6;  // GM_sun / c^3 [s]
constexpr double kPi = 3.14159265358979323846;
constexpr int kChirpThreads = 256;

struct ChirpCol {
  double Mt, eta;
};

__device__ __forceinline__ double2 chirp_value(const ChirpCol p, double flo, double fhi, int64_t N, int64_t n) {
#pragma clang fp contract(off)
  const double f = (N > 1) ? flo + (double)n * (fhi - flo) / (double)(N - 1) : flo;
  const double v = cbrt(kPi * p.Mt * f);
  const double v2 = v * v;
  const double v5 = v2 * v2 * v;
  const double psi = -kPi / 4.0 + 3.0 / (128.0 * p.eta * v5) * (1.0 + (3715.0 / 756.0 + 55.0 * p.eta / 9.0) * v2);
  const double amp = pow(f, -7.0 / 6.0);
  double s, c;
  sincos(psi, &s, &c);
  return make_double2(amp * c, -(amp * s));
}

// Output column j is the snapshot of parameter set pj = cols ? cols[j] : j.
template <int kDtype>
__global__ __launch_bounds__(kChirpThreads) void k_chirp(const double* __restrict__ params,
                                                         const int64_t* __restrict__ cols, double flo, double fhi,
                                                         int64_t N, void* __restrict__ out, int64_t ld) {
  const int64_t j = blockIdx.x;
  const int64_t pj = cols ? cols[j] : j;
  ChirpCol p;
  p.Mt = params[2 * pj] * kTsun;
  const double q = params[2 * pj + 1];
  p.eta = q / ((1.0 + q) * (1.0 + q));
  dd acc = {0.0, 0.0};
  double2* o64 = reinterpret_cast<double2*>(out) + j * ld;
  float2* o32 = reinterpret_cast<float2*>(out) + j * ld;
  for (int64_t n = threadIdx.x; n < N; n += kChirpThreads) {
    const double2 h = chirp_value(p, flo, fhi, N, n);
    if (kDtype == 0) o64[n] = h;
    dd_add_sq(acc, h.x);
    dd_add_sq(acc, h.y);
  }
  acc = wave_dd_sum(acc);
  __shared__ dd sh[kChirpThreads / 64];
  __shared__ double snrm;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    dd t = sh[0];
    for (int w = 1; w < kChirpThreads / 64; ++w) t = dd_add(t, sh[w]);
    snrm = sqrt(t.hi + t.lo);
  }
  __syncthreads();
  const double nrm = snrm;
  for (int64_t n = threadIdx.x; n < N; n += kChirpThreads) {
    if (kDtype == 0) {
      const double2 h = o64[n];
      o64[n] = make_double2(h.x / nrm, h.y / nrm);
    } else {
      const double2 h = chirp_value(p, flo, fhi, N, n);
      o32[n] = make_float2((float)(h.x / nrm), (float)(h.y / nrm));
    }
  }
}

}  // namespace

hipError_t launch_chirp_fill(const double* params, const int64_t* cols, int64_t M, double flo, double fhi, int64_t N,
                             int dtype, void* out, int64_t ld, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (M > 0x7fffffffLL) return hipErrorInvalidValue;
  if (dtype == 0)
    hipLaunchKernelGGL(k_chirp<0>, dim3((unsigned)M), dim3(kChirpThreads), 0, s, params, cols, flo, fhi, N, out, ld);
  else
    hipLaunchKernelGGL(k_chirp<1>, dim3((unsigned)M), dim3(kChirpThreads), 0, s, params, cols, flo, fhi, N, out, ld);
  return hipGetLastError();
}

}  // namespace rb

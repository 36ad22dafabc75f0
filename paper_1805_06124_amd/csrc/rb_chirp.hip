// Synthetic snapshot family standing in for the paper's gravitational-wave
// model (Sec. 6.1.1): column j is the leading-1PN frequency-domain chirp
//   h(f) = f^(-7/6) exp(-i Psi(f)),
//   Psi  = -pi/4 + 3/(128 eta v^5) (1 + (3715/756 + 55 eta/9) v^2),
//   v    = (pi Mtot f)^(1/3),  eta = q/(1+q)^2,
// with Mtot = total mass (solar masses) * GM_sun/c^3 seconds, on the uniform
// grid f_n = flo + n (fhi - flo)/(N - 1), divided by its L2 norm.  FP64
// throughout; complex64 output is the rounded normalised value.
//
// Evaluation form.  |h(f_n)| = f_n^(-7/6) does not depend on the phase, so
// every column has the same norm ||h|| = (sum_n f_n^(-7/3))^(1/2) (computed
// once, exactly).  With v^2 = (pi Mtot f)^(2/3) the phase separates into a
// per-column and a per-row factor:
//   Psi = -pi/4 + A f^(-5/3) + B f^(-1),
//   A = 3/(128 eta) (pi Mtot)^(-5/3),  B = 3/(128 eta) (3715/756 + 55 eta/9) / (pi Mtot).
// A row table (f_n^(-7/6)/||h||, f_n^(-5/3), 1/f_n) is built once; each
// element then costs two FMAs, one sincos and two products, in one pass.
#include <cmath>

#include "rb_host.h"

namespace rb {

namespace {

constexpr double kTsun = 4.925490947641267e-6;  // GM_sun / c^3 [s]
constexpr double kPi = 3.14159265358979323846;
constexpr int kChirpThreads = 256;

// table[3n] = f^(-7/6) / ||h||, table[3n+1] = f^(-5/3), table[3n+2] = 1/f
__global__ __launch_bounds__(1024) void k_chirp_table(double flo, double fhi, int64_t N, double* __restrict__ tab) {
  dd acc = {0.0, 0.0};
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x) {
    const double f = (N > 1) ? flo + (double)n * (fhi - flo) / (double)(N - 1) : flo;
    const double amp = pow(f, -7.0 / 6.0);
    tab[3 * n] = amp;
    tab[3 * n + 1] = pow(f, -5.0 / 3.0);
    tab[3 * n + 2] = 1.0 / f;
    dd_add_sq(acc, amp);
  }
  acc = wave_dd_sum(acc);
  __shared__ dd sh[16];
  __shared__ double sinv;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    dd t = sh[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) t = dd_add(t, sh[w]);
    sinv = 1.0 / sqrt(t.hi + t.lo);
  }
  __syncthreads();
  const double inv = sinv;
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x) tab[3 * n] *= inv;
}

// Output column j is the snapshot of parameter set pj = cols ? cols[j] : j.
template <int kDtype>
__global__ __launch_bounds__(kChirpThreads) void k_chirp(const double* __restrict__ params,
                                                         const int64_t* __restrict__ cols,
                                                         const double* __restrict__ tab, int64_t N,
                                                         void* __restrict__ out, int64_t ld) {
  const int64_t j = blockIdx.x;
  const int64_t pj = cols ? cols[j] : j;
  const double pm = kPi * params[2 * pj] * kTsun;
  const double q = params[2 * pj + 1];
  const double eta = q / ((1.0 + q) * (1.0 + q));
  const double a0 = 3.0 / (128.0 * eta);
  const double A = a0 * pow(pm, -5.0 / 3.0);
  const double B = a0 * (3715.0 / 756.0 + 55.0 * eta / 9.0) / pm;
  double2* o64 = reinterpret_cast<double2*>(out) + j * ld;
  float2* o32 = reinterpret_cast<float2*>(out) + j * ld;
  for (int64_t n = threadIdx.x; n < N; n += kChirpThreads) {
    const double amp = tab[3 * n];
    const double psi = -kPi / 4.0 + A * tab[3 * n + 1] + B * tab[3 * n + 2];
    double s, c;
    sincos(psi, &s, &c);
    if (kDtype == 0)
      o64[n] = make_double2(amp * c, -(amp * s));
    else
      o32[n] = make_float2((float)(amp * c), (float)(-(amp * s)));
  }
}

// Surrogate inputs of sample b (one workgroup): the affinely mapped
// parameters and, at each of the F rows n = rows[r], the unit-modulus phase
// factor exp(-i Psi(f_n)) of the snapshot (the chirp's value divided by its
// amplitude, which is the same for every snapshot):
//   X[b][0..1] = 2 (Mtot, q) - 1 on the parameter box, X[b][2 + 2r] =
//   cos Psi(f_n), X[b][3 + 2r] = -sin Psi(f_n)  (FP64, rounded to FP32);
//   T[b] = targets[idx[b]] (dout floats) when targets != NULL.
__global__ __launch_bounds__(kChirpThreads) void k_phase_features(
    const double* __restrict__ params, const float* __restrict__ targets, const int64_t* __restrict__ idx,
    int dout, double mlo, double mhi, double qlo, double qhi, const int64_t* __restrict__ rows, int64_t F,
    const double* __restrict__ tab, float* __restrict__ X, float* __restrict__ T) {
  const int64_t b = blockIdx.x;
  const int64_t pj = idx[b];
  const int64_t din = 2 + 2 * F;
  const double m = params[2 * pj], q = params[2 * pj + 1];
  double A, B;
  chirp_phase_coeffs(m, q, A, B);
  float* x = X + b * din;
  if (threadIdx.x == 0) {
    x[0] = box_map(m, mlo, mhi);
    x[1] = box_map(q, qlo, qhi);
  }
  for (int64_t r = threadIdx.x; r < F; r += kChirpThreads) {
    double sn, cs;
    sincos(chirp_phase(A, B, tab, rows[r]), &sn, &cs);
    x[2 + 2 * r] = (float)cs;
    x[3 + 2 * r] = (float)(-sn);
  }
  if (targets)
    for (int t = threadIdx.x; t < dout; t += kChirpThreads) T[b * dout + t] = targets[pj * dout + t];
}

}  // namespace

hipError_t launch_phase_features(const double* params, const float* targets, const int64_t* idx, int64_t batch,
                                 int dout, const double* ranges, const int64_t* rows, int64_t F, const double* table,
                                 float* X, float* T, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (batch > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_phase_features, dim3((unsigned)batch), dim3(kChirpThreads), 0, s, params, targets, idx, dout,
                     ranges[0], ranges[1], ranges[2], ranges[3], rows, F, table, X, T);
  return hipGetLastError();
}

hipError_t launch_chirp_table(double flo, double fhi, int64_t N, double* table, hipStream_t s) {
  hipLaunchKernelGGL(k_chirp_table, dim3(1), dim3(1024), 0, s, flo, fhi, N, table);
  return hipGetLastError();
}

hipError_t launch_chirp_fill(const double* params, const int64_t* cols, int64_t M, const double* table, int64_t N,
                             int dtype, void* out, int64_t ld, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (M > 0x7fffffffLL) return hipErrorInvalidValue;
  if (dtype == 0)
    hipLaunchKernelGGL(k_chirp<0>, dim3((unsigned)M), dim3(kChirpThreads), 0, s, params, cols, table, N, out, ld);
  else
    hipLaunchKernelGGL(k_chirp<1>, dim3((unsigned)M), dim3(kChirpThreads), 0, s, params, cols, table, N, out, ld);
  return hipGetLastError();
}

}  // namespace rb

// ---------------------------------------------------------------------------
// Parameters of the chirp family from a seed: SplitMix64 (Steele, Lea &
// Flood 2014) counter outputs mapped to uniform doubles (z >> 11) 2^-53;
// column j takes Mtot from counter 2 j and q from counter 2 j + 1.  The
// affine maps are rounded step by step (contraction into fused
// multiply-adds is switched off), so the values are the same bits as any
// other implementation of these formulas.
namespace rb {
namespace {

__device__ __forceinline__ double splitmix_uniform(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1p-53;
}

__global__ __launch_bounds__(256) void k_chirp_params(uint64_t seed, int64_t start, int64_t M, double mlo, double mhi,
                                                      double qlo, double qhi, double* __restrict__ params) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= M) return;
  {
#pragma clang fp contract(off)
    const uint64_t j = (uint64_t)(start + t);
    const double um = splitmix_uniform(seed, 2ull * j), uq = splitmix_uniform(seed, 2ull * j + 1ull);
    const double dm = mhi - mlo, dq = qhi - qlo;
    const double pm = dm * um, pq = dq * uq;
    params[2 * t] = mlo + pm;
    params[2 * t + 1] = qlo + pq;
  }
}

// sum of every double of a buffer read once with 16-byte streaming loads
// (the plain read whose rate is the achievable HBM bandwidth); one partial
// sum per block
__global__ __launch_bounds__(256) void k_stream_read(const double2* __restrict__ p, int64_t n2,
                                                     double* __restrict__ partial) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += stride) {
    const double2 a = ld_stream(p + i);
    s0 += a.x;
    s1 += a.y;
  }
  const double s = wave_sum(s0 + s1);
  __shared__ double ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

}  // namespace
}  // namespace rb

extern "C" {

int rb_chirp_params(uint64_t seed, int64_t start, int64_t M, double mlo, double mhi, double qlo, double qhi,
                    double* params, hipStream_t stream) {
  rb::last_error().clear();
  if (!params || M <= 0 || start < 0 || !(mhi >= mlo) || !(qhi >= qlo) || !std::isfinite(mlo) ||
      !std::isfinite(mhi) || !std::isfinite(qlo) || !std::isfinite(qhi))
    return rb::set_error(RB_EINVAL, "rb_chirp_params: bad arguments");
  hipLaunchKernelGGL(rb::k_chirp_params, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, stream, seed, start, M, mlo,
                     mhi, qlo, qhi, params);
  RB_HIP(hipGetLastError());
  return RB_OK;
}

int rb_stream_read(const void* p, size_t bytes, double* partial, int64_t npartial, hipStream_t stream) {
  rb::last_error().clear();
  if (!p || !partial || bytes < 16 || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(p) % 16) != 0 ||
      npartial < 1 || npartial > 65535)
    return rb::set_error(RB_EINVAL, "rb_stream_read: bad arguments");
  hipLaunchKernelGGL(rb::k_stream_read, dim3((unsigned)npartial), dim3(256), 0, stream,
                     static_cast<const double2*>(p), (int64_t)(bytes / 16), partial);
  RB_HIP(hipGetLastError());
  return RB_OK;
}

}  // extern "C"

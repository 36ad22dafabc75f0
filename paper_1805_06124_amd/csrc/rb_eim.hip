// Empirical-interpolation (EI) nodes of a reduced basis and out-of-sample
// validation of the empirical interpolant (Sec. 6.1: the code selects EI
// nodes and validates the basis and its interpolant).
//
// Standard EIM on a discrete basis e_1..e_k: node p_1 maximises |e_1|.  Node
// p_j maximises |r_j|, where r_j = e_j - I_{j-1}[e_j] is the part of e_j
// that interpolation through the earlier nodes misses.  Ties go to the
// lowest index.
//
// Computed in elimination form.  Each residual is stored normalised,
// r_i <- r_i / r_i(p_i).  Then T[l, i] = r_i(p_l) is unit lower triangular
// (r_i vanishes at the earlier nodes), and
//   r_j = e_j - sum_{i<j} alpha_i r_i,  alpha = T^{-1} e_j(p_1..p_{j-1}),
// which vanishes at p_1..p_{j-1} and lies in span(e_1..e_j).  It is
// therefore the EI residual.
// T^{-1} grows by one row per step:
//   Tinv[j, l] = -sum_{l <= i < j} r_i(p_j) Tinv[i, l].
// E = R U with U upper triangular, so the interpolation matrix
// B = E(P, :) = T U.  The interpolant is then
//   I[v] = E B^{-1} v(P) = R (T^{-1} v(P)),
// which needs no solve with U.
//
// Per node: four small launches, enqueued without host synchronisation:
// the coefficients alpha, the residual and its block maxima, the node and
// the new row of T^{-1}, the normalisation.
#include <algorithm>
#include <cmath>
#include <vector>

#include "rb_host.h"

using namespace rb;

namespace rb {
namespace {

struct Peak {
  double v;   // |r|^2
  int64_t i;  // row
  double e;   // max |e_j|^2 over the same rows
};

__device__ __forceinline__ bool peak_better(double v, int64_t i, double bv, int64_t bi) {
  return v > bv || (v == bv && i < bi);
}

// alpha[i] = sum_{l <= i} Tinv[i, l] e_j(p_l), i < j
__global__ __launch_bounds__(256) void k_eim_alpha(const double2* __restrict__ E, int64_t ldE, int64_t j,
                                                   const int64_t* __restrict__ nodes, const double2* __restrict__ Ti,
                                                   int64_t ldT, double2* __restrict__ alpha) {
  __shared__ double2 ev[1024];
  const double2* ej = E + j * ldE;
  for (int64_t l0 = 0; l0 < j; l0 += 1024) {
    // gather e_j at the nodes in chunks of 1024
    for (int64_t l = l0 + threadIdx.x; l < std::min<int64_t>(j, l0 + 1024); l += 256) ev[l - l0] = ej[nodes[l]];
    __syncthreads();
    for (int64_t i = threadIdx.x; i < j; i += 256) {
      double2 s = (l0 == 0) ? make_double2(0.0, 0.0) : alpha[i];
      const int64_t lend = std::min<int64_t>(i + 1, std::min<int64_t>(j, l0 + 1024));
      for (int64_t l = l0; l < lend; ++l) {
        const double2 t = Ti[i + l * ldT], e = ev[l - l0];
        s.x = fma(t.x, e.x, fma(-t.y, e.y, s.x));
        s.y = fma(t.x, e.y, fma(t.y, e.x, s.y));
      }
      alpha[i] = s;
    }
    __syncthreads();
  }
}

// R[:, j] = e_j - R[:, :j] alpha; per-block max of |r|^2 (lowest row on ties)
__global__ __launch_bounds__(256) void k_eim_resid(const double2* __restrict__ E, int64_t ldE, int64_t N, int64_t j,
                                                   const double2* __restrict__ alpha, double2* __restrict__ R,
                                                   int64_t ldR, Peak* __restrict__ part) {
  __shared__ double2 sa[256];
  __shared__ Peak wp[4];
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double2 r = make_double2(0.0, 0.0);
  if (n < N) r = E[n + j * ldE];
  for (int64_t i0 = 0; i0 < j; i0 += 256) {
    if (i0 + threadIdx.x < j) sa[threadIdx.x] = alpha[i0 + threadIdx.x];
    __syncthreads();
    if (n < N) {
      const int64_t iend = std::min<int64_t>(256, j - i0);
      for (int64_t q = 0; q < iend; ++q) {
        const double2 a = sa[q], x = R[n + (i0 + q) * ldR];
        r.x = fma(-a.x, x.x, fma(a.y, x.y, r.x));
        r.y = fma(-a.x, x.y, fma(-a.y, x.x, r.y));
      }
    }
    __syncthreads();
  }
  double v = -1.0, em = 0.0;
  int64_t idx = INT64_MAX;
  if (n < N) {
    R[n + j * ldR] = r;
    v = r.x * r.x + r.y * r.y;
    idx = n;
    const double2 e = E[n + j * ldE];
    em = e.x * e.x + e.y * e.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off);
    const int64_t oi = __shfl_down(idx, off);
    em = fmax(em, __shfl_down(em, off));
    if (peak_better(ov, oi, v, idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wp[wave] = Peak{v, idx, em};
  __syncthreads();
  if (threadIdx.x == 0) {
    Peak b = wp[0];
    for (int w = 1; w < 4; ++w) {
      if (peak_better(wp[w].v, wp[w].i, b.v, b.i)) {
        b.v = wp[w].v;
        b.i = wp[w].i;
      }
      b.e = fmax(b.e, wp[w].e);
    }
    part[blockIdx.x] = b;
  }
}

// node j = argmax of the block maxima; new row j of Tinv; the pivot r_j(p_j)
__global__ __launch_bounds__(256) void k_eim_select(const Peak* __restrict__ part, int64_t nblk, int64_t j,
                                                    const double2* __restrict__ R, int64_t ldR,
                                                    int64_t* __restrict__ nodes, double* __restrict__ peak,
                                                    double2* __restrict__ pivot, double2* __restrict__ Ti,
                                                    int64_t ldT, int* __restrict__ info) {
  __shared__ Peak wp[4];
  __shared__ int64_t s_p;
  __shared__ double2 trow[1024];
  double v = -1.0, em = 0.0;
  int64_t idx = INT64_MAX;
  for (int64_t b = threadIdx.x; b < nblk; b += 256) {
    if (peak_better(part[b].v, part[b].i, v, idx)) {
      v = part[b].v;
      idx = part[b].i;
    }
    em = fmax(em, part[b].e);
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off);
    const int64_t oi = __shfl_down(idx, off);
    em = fmax(em, __shfl_down(em, off));
    if (peak_better(ov, oi, v, idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wp[wave] = Peak{v, idx, em};
  __syncthreads();
  if (threadIdx.x == 0) {
    Peak b = wp[0];
    for (int w = 1; w < 4; ++w) {
      if (peak_better(wp[w].v, wp[w].i, b.v, b.i)) {
        b.v = wp[w].v;
        b.i = wp[w].i;
      }
      b.e = fmax(b.e, wp[w].e);
    }
    s_p = b.i;
    nodes[j] = b.i;
    peak[j] = sqrt(b.v);
    *pivot = R[b.i + j * ldR];
    // r_j at rounding level of e_j: e_j depends on e_1..e_{j-1}
    const double thr = 64.0 * (double)(j + 1) * 0x1p-53;
    if (!(b.v > thr * thr * b.e) && *info < 0) *info = (int)j;
  }
  __syncthreads();
  const int64_t p = s_p;
  // new row of Tinv: Tinv[j, l] = -sum_{l <= i < j} r_i(p_j) Tinv[i, l]
  for (int64_t l0 = 0; l0 < j; l0 += 1024) {
    for (int64_t i = l0 + threadIdx.x; i < std::min<int64_t>(j, l0 + 1024); i += 256) trow[i - l0] = R[p + i * ldR];
    __syncthreads();
    for (int64_t l = threadIdx.x; l < j; l += 256) {
      double2 s = (l0 == 0) ? make_double2(0.0, 0.0) : Ti[j + l * ldT];
      const int64_t ibeg = std::max<int64_t>(l, l0), iend = std::min<int64_t>(j, l0 + 1024);
      for (int64_t i = ibeg; i < iend; ++i) {
        const double2 t = trow[i - l0], x = Ti[i + l * ldT];
        s.x = fma(-t.x, x.x, fma(t.y, x.y, s.x));
        s.y = fma(-t.x, x.y, fma(-t.y, x.x, s.y));
      }
      Ti[j + l * ldT] = s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) Ti[j + j * ldT] = make_double2(1.0, 0.0);
}

// R[:, j] /= r_j(p_j); the node's own entry is set to exactly 1
__global__ __launch_bounds__(256) void k_eim_scale(double2* __restrict__ R, int64_t ldR, int64_t N, int64_t j,
                                                   const double2* __restrict__ pivot,
                                                   const int64_t* __restrict__ nodes) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const double2 pv = *pivot;
  const double den = pv.x * pv.x + pv.y * pv.y;
  if (!(den > 0.0)) return;
  double2* x = R + n + j * ldR;
  if (n == nodes[j]) {
    *x = make_double2(1.0, 0.0);
    return;
  }
  const double2 a = *x;
  // a / pv = a conj(pv) / |pv|^2
  *x = make_double2((a.x * pv.x + a.y * pv.y) / den, (a.y * pv.x - a.x * pv.y) / den);
}

__global__ __launch_bounds__(256) void k_fill_zero(double2* __restrict__ x, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) x[t] = make_double2(0.0, 0.0);
}

// G[l, m] = V[nodes[l], m]   (k x M, ld k)
__global__ __launch_bounds__(256) void k_gather_rows(const double2* __restrict__ V, int64_t ldV,
                                                     const int64_t* __restrict__ nodes, int64_t k, int64_t M,
                                                     double2* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= k * M) return;
  const int64_t l = e % k, m = e / k;
  G[e] = V[nodes[l] + m * ldV];
}

// out = A^H (n x n, ld n)
__global__ __launch_bounds__(256) void k_conj_transpose(const double2* __restrict__ A, int64_t n,
                                                        double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e % n, c = e / n;
  const double2 a = A[c + r * n];
  out[e] = make_double2(a.x, -a.y);
}

}  // namespace
}  // namespace rb

extern "C" {

int rb_eim_z(const void* E_, int64_t N, int64_t k, int64_t ldE, int64_t* nodes, double* peak, void* R_, void* Tinv_,
             int64_t* k_out, hipStream_t stream) {
  last_error().clear();
  if (!E_ || !nodes || !k_out || N <= 0 || k <= 0 || k > N || !valid_ld(N, ldE))
    return set_error(RB_EINVAL, "rb_eim_z: bad arguments");
  const double2* E = static_cast<const double2*>(E_);
  const int64_t nblk = (N + 255) / 256;
  DevBuf d_R, d_T, d_alpha, d_part, d_nodes, d_peak, d_piv, d_info;
  double2* R = static_cast<double2*>(R_);
  double2* Ti = static_cast<double2*>(Tinv_);
  if (!R) {
    RB_ALLOC(d_R, sizeof(double2) * (size_t)N * (size_t)k);
    R = d_R.as<double2>();
  }
  if (!Ti) {
    RB_ALLOC(d_T, sizeof(double2) * (size_t)k * (size_t)k);
    Ti = d_T.as<double2>();
  }
  RB_ALLOC(d_alpha, sizeof(double2) * (size_t)k);
  RB_ALLOC(d_part, sizeof(Peak) * (size_t)nblk);
  RB_ALLOC(d_nodes, sizeof(int64_t) * (size_t)k);
  RB_ALLOC(d_peak, sizeof(double) * (size_t)k);
  RB_ALLOC(d_piv, sizeof(double2));
  RB_ALLOC(d_info, sizeof(int));
  const int minus1 = -1;
  RB_HIP(hipMemcpyAsync(d_info.p, &minus1, sizeof(int), hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((k * k + 255) / 256)), dim3(256), 0, stream, Ti, k * k);
  RB_HIP(hipGetLastError());
  for (int64_t j = 0; j < k; ++j) {
    if (j > 0) {
      hipLaunchKernelGGL(k_eim_alpha, dim3(1), dim3(256), 0, stream, E, ldE, j, d_nodes.as<int64_t>(), Ti, k,
                         d_alpha.as<double2>());
      RB_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_eim_resid, dim3((unsigned)nblk), dim3(256), 0, stream, E, ldE, N, j, d_alpha.as<double2>(),
                       R, N, d_part.as<Peak>());
    RB_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_eim_select, dim3(1), dim3(256), 0, stream, d_part.as<Peak>(), nblk, j, R, N,
                       d_nodes.as<int64_t>(), d_peak.as<double>(), d_piv.as<double2>(), Ti, k, d_info.as<int>());
    RB_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_eim_scale, dim3((unsigned)nblk), dim3(256), 0, stream, R, N, N, j, d_piv.as<double2>(),
                       d_nodes.as<int64_t>());
    RB_HIP(hipGetLastError());
  }
  int info = -1;
  RB_HIP(hipMemcpyAsync(nodes, d_nodes.p, sizeof(int64_t) * k, hipMemcpyDeviceToHost, stream));
  if (peak) RB_HIP(hipMemcpyAsync(peak, d_peak.p, sizeof(double) * k, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipMemcpyAsync(&info, d_info.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  if (info >= 0) {
    *k_out = info;
    return RB_RANK;
  }
  *k_out = k;
  return RB_OK;
}

int rb_eim_errors_z(const void* R_, int64_t N, int64_t k, int64_t ldR, const void* Tinv_, const int64_t* nodes,
                    const void* V_, int64_t M, int64_t ldV, double* out, hipStream_t stream) {
  last_error().clear();
  if (!R_ || !Tinv_ || !nodes || !V_ || !out || N <= 0 || k <= 0 || k > N || M <= 0 || !valid_ld(N, ldR) ||
      !valid_ld(N, ldV))
    return set_error(RB_EINVAL, "rb_eim_errors_z: bad arguments");
  const double2* R = static_cast<const double2*>(R_);
  const double2* Ti = static_cast<const double2*>(Tinv_);
  const double2* V = static_cast<const double2*>(V_);
  const int64_t chunk = std::min<int64_t>(M, 65536);
  DevBuf d_TH, d_G, d_W, d_bad;
  RB_ALLOC(d_TH, sizeof(double2) * (size_t)k * (size_t)k);
  RB_ALLOC(d_G, sizeof(double2) * (size_t)k * (size_t)chunk);
  RB_ALLOC(d_W, sizeof(double2) * (size_t)k * (size_t)chunk);
  RB_ALLOC(d_bad, sizeof(int));
  RB_HIP(hipMemsetAsync(d_bad.p, 0, sizeof(int), stream));
  hipLaunchKernelGGL(k_conj_transpose, dim3((unsigned)((k * k + 255) / 256)), dim3(256), 0, stream, Ti, k,
                     d_TH.as<double2>());
  RB_HIP(hipGetLastError());
  for (int64_t j0 = 0; j0 < M; j0 += chunk) {
    const int64_t mc = std::min(chunk, M - j0);
    // G = V(P, chunk); W = Tinv G = (Tinv^H)^H G; out = ||V - R W||^2
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((k * mc + 255) / 256)), dim3(256), 0, stream, V + j0 * ldV,
                       ldV, nodes, k, mc, d_G.as<double2>());
    RB_HIP(hipGetLastError());
    RB_HIP(launch_project_z(d_TH.as<double2>(), k, k, k, d_G.as<double2>(), mc, k, d_W.as<double2>(), k, stream));
    RB_HIP(launch_resid(V + j0 * ldV, ldV, static_cast<double2*>(nullptr), 0, N, mc, R, ldR, k, d_W.as<double2>(), 1,
                        k, out + j0, d_bad.as<int>(), stream));
  }
  RB_HIP(launch_sqrt_inplace(out, M, stream));
  int hbad = 0;
  RB_HIP(hipMemcpyAsync(&hbad, d_bad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  if (hbad) return set_error(RB_ENONFINITE, "rb_eim_errors_z: non-finite value");
  return RB_OK;
}

}  // extern "C"

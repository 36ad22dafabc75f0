// Out-of-sample validation of a reduced basis and enrichment of the basis by
// the columns that fail it (Sec. 6.1: the code validates the basis on fresh
// parameter samples and enriches it by iterative refinement).
//
// Validation of a column v against the orthonormal basis E (N x k):
// r(v) = ||v - E (E^H v)||_2, computed explicitly.  This takes two FP64
// matrix-core passes over the validation columns:
//   1. C = E^H V (k_project_z);
//   2. ||V - E C|| per column (k_resid in its norms-only form).
// The Pythagorean form ||v||^2 - ||E^H v||^2 would need only one pass.  Its
// rounding floor, about sqrt(k u) ||v|| ~ 1e-7 for k in the hundreds, is far
// above the tolerances a validation has to decide (1e-10 and below), so it
// is not used.
//
// Enrichment: the columns with r >= tol continue the greedy from E (the
// greedy's own pivot rule and stopping test, see greedy_z_core).  Residuals
// can only shrink as the basis grows, so afterwards every column of the
// validation set is below tol.  A run may take several validation rounds,
// each on a fresh set of columns.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rb_host.h"

using namespace rb;

namespace rb {
namespace {

__global__ __launch_bounds__(256) void k_sqrt_inplace(double* __restrict__ x, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) x[t] = sqrt(x[t]);
}

// a column fails validation when its residual is not below tol (NaN fails)
__device__ __forceinline__ bool fails(double r, double tol) { return !(r < tol); }

// failing columns per block of 256
__global__ __launch_bounds__(256) void k_fail_count(const double* __restrict__ r, int64_t n, double tol,
                                                    int* __restrict__ count) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int f = (t < n && fails(r[t], tol)) ? 1 : 0;
  const int c = __syncthreads_count(f);
  if (threadIdx.x == 0) count[blockIdx.x] = c;
}

// exclusive prefix sum of count[0..nb) into off[0..nb], off[nb] = total; one
// block of 1024 threads, each owning a contiguous segment
__global__ __launch_bounds__(1024) void k_scan_counts(const int* __restrict__ count, int64_t nb,
                                                      int64_t* __restrict__ off) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t seg = (nb + 1023) / 1024;
  const int64_t b0 = std::min<int64_t>(nb, t * seg), b1 = std::min<int64_t>(nb, b0 + seg);
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += count[b];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 1024 segment sums
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t v = (t >= d) ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;  // exclusive
  for (int64_t b = b0; b < b1; ++b) {
    off[b] = run;
    run += count[b];
  }
  if (t == 1023) off[nb] = part[1023];
}

// idx[off[block] + rank] = base + t for each failing t, in increasing order
__global__ __launch_bounds__(256) void k_fail_scatter(const double* __restrict__ r, int64_t n, double tol,
                                                      const int64_t* __restrict__ off, int64_t base,
                                                      int64_t* __restrict__ idx) {
  __shared__ int wave_tot[4];
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool f = t < n && fails(r[t], tol);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t bal = __ballot(f);
  const int below = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wave_tot[wave] = __popcll(bal);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wave_tot[w];
  if (f) idx[off[blockIdx.x] + before + below] = base + t;
}

}  // namespace

hipError_t launch_sqrt_inplace(double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sqrt_inplace, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

// out[j] = ||v_j - E (E^H v_j)||^2 for the M columns of V, in chunks of at
// most `chunk` columns; Cw holds k x chunk coefficients.
static hipError_t residual_sq(const double2* E, int64_t N, int64_t k, int64_t ldE, const double2* V, int64_t M,
                              int64_t ldV, double* out, double2* Cw, int64_t chunk, int* bad, hipStream_t s) {
  for (int64_t j0 = 0; j0 < M; j0 += chunk) {
    const int64_t mc = std::min(chunk, M - j0);
    hipError_t e;
    if (k > 0) {
      e = launch_project_z(E, N, k, ldE, V + j0 * ldV, mc, ldV, Cw, k, s);
      if (e != hipSuccess) return e;
    }
    e = launch_resid(V + j0 * ldV, ldV, static_cast<double2*>(nullptr), 0, N, mc, E, ldE, k, Cw, 1, k, out + j0, bad,
                     s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rb

extern "C" {

int rb_residual_norms_z(const void* E_, int64_t N, int64_t k, int64_t ldE, const void* V_, int64_t M, int64_t ldV,
                        double* out, hipStream_t stream) {
  last_error().clear();
  if (!V_ || !out || N <= 0 || M <= 0 || k < 0 || k > N || !valid_ld(N, ldV) || (k > 0 && (!E_ || !valid_ld(N, ldE))))
    return set_error(RB_EINVAL, "rb_residual_norms_z: bad arguments");
  const int64_t chunk = std::min<int64_t>(M, 65536);
  DevBuf Cw, bad;
  RB_ALLOC(Cw, sizeof(double2) * (size_t)std::max<int64_t>(k, 1) * (size_t)chunk);
  RB_ALLOC(bad, sizeof(int));
  RB_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), stream));
  RB_HIP(residual_sq(static_cast<const double2*>(E_), N, k, ldE, static_cast<const double2*>(V_), M, ldV, out,
                     Cw.as<double2>(), chunk, bad.as<int>(), stream));
  RB_HIP(launch_sqrt_inplace(out, M, stream));
  int hbad = 0;
  RB_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  if (hbad) return set_error(RB_ENONFINITE, "rb_residual_norms_z: non-finite value in V");
  return RB_OK;
}

int rb_enrich_z(rb_regen_fn regen, void* regen_ctx, int64_t N, int64_t Mv, int64_t rounds, double tol, int64_t kmax,
                void* E_, int64_t ldE, int64_t k_in, int64_t* piv, double* err, double* rho, int32_t* nu,
                int64_t* k_out, int64_t* n_fail, double* resid_max, double* resid, const rb_opts* opts_in,
                rb_stats* stats, hipStream_t stream) {
  last_error().clear();
  rb_opts o;
  rb_default_opts(&o);
  if (opts_in) o = *opts_in;
  int64_t kcap = std::min(kmax, N);
  if (!regen || !E_ || N <= 0 || Mv <= 0 || rounds < 1 || !(tol >= 0.0) || !std::isfinite(tol) || k_in < 0 ||
      k_in > kcap || !valid_ld(N, ldE) || !piv || !err || !rho || !k_out || !n_fail || !resid_max ||
      o.regen_chunk < 1)
    return set_error(RB_EINVAL, "rb_enrich_z: bad arguments");
  double2* E = static_cast<double2*>(E_);
  const int64_t chunk = std::min<int64_t>(Mv, o.regen_chunk);
  const int64_t nb = (Mv + 255) / 256;

  DevBuf Vc, Cw, d_cols, d_r, d_cnt, d_off, d_bad;
  RB_ALLOC(Vc, sizeof(double2) * (size_t)N * (size_t)chunk);
  RB_ALLOC(Cw, sizeof(double2) * (size_t)std::max<int64_t>(kcap, 1) * (size_t)chunk);
  RB_ALLOC(d_cols, sizeof(int64_t) * (size_t)chunk);
  RB_ALLOC(d_r, sizeof(double) * (size_t)Mv);
  RB_ALLOC(d_cnt, sizeof(int) * (size_t)nb);
  RB_ALLOC(d_off, sizeof(int64_t) * (size_t)(nb + 1));
  RB_ALLOC(d_bad, sizeof(int));
  double* r = d_r.as<double>();

  rb_stats tot;
  std::memset(&tot, 0, sizeof tot);
  int64_t k = k_in;
  int status = RB_OK;
  for (int64_t round = 0; round < rounds; ++round) {
    const int64_t base = round * Mv;
    // ---- 1. validation residuals of this round's columns ----
    RB_HIP(hipMemsetAsync(d_bad.p, 0, sizeof(int), stream));
    for (int64_t j0 = 0; j0 < Mv; j0 += chunk) {
      const int64_t mc = std::min(chunk, Mv - j0);
      RB_HIP(launch_iota(d_cols.as<int64_t>(), base + j0, mc, stream));
      if (regen(regen_ctx, d_cols.as<int64_t>(), mc, Vc.p, N, stream) != 0)
        return set_error(RB_EDEVICE, "rb_enrich_z: the regenerator failed");
      RB_HIP(residual_sq(E, N, k, ldE, Vc.as<double2>(), mc, N, r + j0, Cw.as<double2>(), mc, d_bad.as<int>(),
                         stream));
    }
    RB_HIP(launch_sqrt_inplace(r, Mv, stream));
    if (resid) RB_HIP(hipMemcpyAsync(resid + base, r, sizeof(double) * Mv, hipMemcpyDeviceToDevice, stream));
    // ---- 2. the failing columns, in index order ----
    hipLaunchKernelGGL(k_fail_count, dim3((unsigned)nb), dim3(256), 0, stream, r, Mv, tol, d_cnt.as<int>());
    RB_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, stream, d_cnt.as<int>(), nb, d_off.as<int64_t>());
    RB_HIP(hipGetLastError());
    // largest residual (the est_argmax kernel over a mask of zeros)
    int64_t nf = 0;
    int hbad = 0;
    RB_HIP(hipMemcpyAsync(&nf, d_off.as<int64_t>() + nb, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipMemcpyAsync(&hbad, d_bad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    {
      DevBuf part, res, zmask;
      const int64_t np = sweep_partials_needed(Mv);
      RB_ALLOC(part, sizeof(ArgMax) * np);
      RB_ALLOC(res, sizeof(ArgMax));
      RB_ALLOC(zmask, (size_t)Mv);
      RB_HIP(hipMemsetAsync(zmask.p, 0, (size_t)Mv, stream));
      RB_HIP(launch_est_argmax(r, nullptr, zmask.as<uint8_t>(), Mv, part.as<ArgMax>(), np, res.as<ArgMax>(), stream));
      ArgMax h;
      RB_HIP(hipMemcpyAsync(&h, res.p, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
      RB_HIP(hipStreamSynchronize(stream));
      resid_max[round] = h.v;
    }
    if (hbad) return set_error(RB_ENONFINITE, "rb_enrich_z: non-finite value in a validation column");
    n_fail[round] = nf;
    if (nf == 0) continue;
    if (k == kcap) {
      status = RB_KMAX;
      continue;
    }
    // ---- 3. regenerate the failing columns and continue the greedy ----
    DevBuf d_fidx, F;
    RB_ALLOC(d_fidx, sizeof(int64_t) * (size_t)nf);
    RB_ALLOC(F, sizeof(double2) * (size_t)N * (size_t)nf);
    hipLaunchKernelGGL(k_fail_scatter, dim3((unsigned)nb), dim3(256), 0, stream, r, Mv, tol, d_off.as<int64_t>(),
                       base, d_fidx.as<int64_t>());
    RB_HIP(hipGetLastError());
    if (regen(regen_ctx, d_fidx.as<int64_t>(), nf, F.p, N, stream) != 0)
      return set_error(RB_EDEVICE, "rb_enrich_z: the regenerator failed");
    std::vector<int64_t> fidx((size_t)nf);
    RB_HIP(hipMemcpyAsync(fidx.data(), d_fidx.p, sizeof(int64_t) * nf, hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    int64_t k_new = k;
    rb_stats st;
    const int rc = greedy_z_core("rb_enrich_z", F.p, N, nf, N, tol, kcap, F.p, N, E, ldE, k, piv, err, rho, nu,
                                 &k_new, nullptr, 0, &o, &st, stream);
    if (rc < 0) return rc;
    for (int64_t i = k; i < k_new; ++i) piv[i] = fidx[(size_t)piv[i]];
    tot.sweeps += st.sweeps;
    tot.anchors += st.anchors;
    tot.gs_passes += st.gs_passes;
    tot.ms_sweep += st.ms_sweep;
    tot.ms_gs += st.ms_gs;
    tot.ms_anchor += st.ms_anchor;
    k = k_new;
    if (rc == RB_KMAX || rc == RB_RANK) status = rc;
  }
  *k_out = k;
  if (stats) *stats = tot;
  return status;
}

}  // extern "C"

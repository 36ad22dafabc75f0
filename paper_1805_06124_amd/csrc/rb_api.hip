// C ABI of librb.so and the host driver of the RB-greedy (Alg. 3).
//
// One greedy step k (Sec. 6.1.2):
//   1. orthonormalise the pivot column x_J of the working matrix X against
//      the basis by iterated Gram-Schmidt with Hoffmann's kappa criterion;
//      e_{k+1} = v/||v||, rho_k = ||v|| = |R_{k+1,k+1}|;
//   2. one fused sweep of X with e_{k+1} (Eq. (6.3)): c_j, acc_j += |c_j|^2,
//      est_j = nrm_j - acc_j and the masked argmax (est_max, J);
//   3. host decision: err_{k+1} = sqrt(est_max); stop when err < tol or at
//      kmax.
// Resolution of Eq. (6.3): est_j carries an absolute rounding error of a few
// (k+1) u max_j nrm_j, so once est_max drops below theta times the largest
// nrm since the last anchoring the estimate can no longer be trusted.  The
// working columns are then re-anchored: X <- X - E_panel C_panel (explicit
// residuals against the vectors swept since the last anchoring), nrm <-
// ||x_j||^2 exactly, acc <- 0.  This is the stored-residual form of the same
// greedy (the matrix V of Alg. 2, Remark 5.5) entered only when needed; the
// pivots and errors are those of Alg. 2/3 (Proposition 5.3).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "rb_host.h"

using namespace rb;

namespace rb {

std::string& last_error() {
  static thread_local std::string msg;
  return msg;
}

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error() = buf;
  return code;
}

}  // namespace rb

extern "C" {

void rb_default_opts(rb_opts* o) {
  if (!o) return;
  o->kappa = 2.0;
  o->nu_max = 4;
  o->nu_min = 1;
  o->theta = 1e-3;
  o->anchor_max = 128;
  o->collect_stats = 0;
  o->theta32 = 1e-4;
  o->regen_chunk = 32768;
  o->certify = 2;
}

const char* rb_strerror(int status) {
  switch (status) {
    case RB_OK: return "converged (err < tol)";
    case RB_KMAX: return "stopped at kmax";
    case RB_RANK: return "rank exhausted (pivot in the span of the basis)";
    case RB_EINVAL: return "invalid argument";
    case RB_ENOMEM: return "device allocation failed";
    case RB_EDEVICE: return "HIP runtime error";
    case RB_ENONFINITE: return "non-finite value in S";
    case RB_ENOCONV: return "an iterative eigen-solve did not converge";
    default: return "unknown status";
  }
}

const char* rb_last_error(void) { return last_error().c_str(); }

int rb_colnorms_z(const void* S, int64_t N, int64_t M, int64_t ldS, double* nrm, hipStream_t stream) {
  last_error().clear();
  if (!S || !nrm || N <= 0 || M <= 0 || !valid_ld(N, ldS)) return set_error(RB_EINVAL, "rb_colnorms_z: bad arguments");
  DevBuf bad;
  RB_ALLOC(bad, sizeof(int));
  RB_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), stream));
  RB_HIP(launch_colnorms_z(static_cast<const double2*>(S), N, M, ldS, nrm, bad.as<int>(), stream));
  int hbad = 0;
  RB_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  if (hbad) return set_error(RB_ENONFINITE, "rb_colnorms_z: non-finite column norm");
  return RB_OK;
}

int rb_sweep_z(const void* S, int64_t N, int64_t M, int64_t ldS, const void* e, const double* nrm, double* acc,
               const uint8_t* mask, void* c_out, int64_t ldc, double* est_max, int64_t* J, hipStream_t stream) {
  last_error().clear();
  if (!S || !e || !nrm || !acc || !est_max || !J || N <= 0 || M <= 0 || !valid_ld(N, ldS) || (c_out && ldc <= 0))
    return set_error(RB_EINVAL, "rb_sweep_z: bad arguments");
  const int64_t np = sweep_partials_needed(M);
  DevBuf part, res;
  RB_ALLOC(part, sizeof(ArgMax) * np);
  RB_ALLOC(res, sizeof(ArgMax));
  RB_HIP(launch_sweep_z(static_cast<const double2*>(S), N, M, ldS, static_cast<const double2*>(e), nrm, acc, mask,
                        static_cast<double2*>(c_out), ldc, part.as<ArgMax>(), np, res.as<ArgMax>(), stream));
  ArgMax h;
  RB_HIP(hipMemcpyAsync(&h, res.p, sizeof h, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  *est_max = h.v;
  *J = h.i;
  return RB_OK;
}

int rb_project_z(const void* E, int64_t N, int64_t k, int64_t ldE, const void* S, int64_t M, int64_t ldS, void* C,
                 int64_t ldC, hipStream_t stream) {
  last_error().clear();
  if (!E || !S || !C || N <= 0 || k <= 0 || M <= 0 || !valid_ld(N, ldE) || !valid_ld(N, ldS) || ldC < k)
    return set_error(RB_EINVAL, "rb_project_z: bad arguments");
  if ((k + 159) / 160 > 65535) return set_error(RB_EINVAL, "rb_project_z: k too large");
  RB_HIP(launch_project_z(static_cast<const double2*>(E), N, k, ldE, static_cast<const double2*>(S), M, ldS,
                          static_cast<double2*>(C), ldC, stream));
  RB_HIP(hipStreamSynchronize(stream));
  return RB_OK;
}

int rb_chirp_fill(const double* params, int64_t M, double flo, double fhi, int64_t N, int dtype, void* out, int64_t ld,
                  hipStream_t stream) {
  last_error().clear();
  if (!params || !out || M <= 0 || N <= 0 || !valid_ld(N, ld) || (dtype != 0 && dtype != 1) || !(flo > 0.0) ||
      !(fhi >= flo) || M > 0x7fffffffLL)
    return set_error(RB_EINVAL, "rb_chirp_fill: bad arguments");
  DevBuf tab;
  RB_ALLOC(tab, sizeof(double) * 3 * (size_t)N);
  RB_HIP(launch_chirp_table(flo, fhi, N, tab.as<double>(), stream));
  RB_HIP(launch_chirp_fill(params, nullptr, M, tab.as<double>(), N, dtype, out, ld, stream));
  RB_HIP(hipStreamSynchronize(stream));
  return RB_OK;
}

}  // extern "C"

namespace rb {

// The FP64 greedy, started from k0 >= 0 orthonormal vectors already in
// E[:, 0..k0-1] (k0 = 0: the greedy of Alg. 3 itself).
int greedy_z_core(const char* fn, const void* S_, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax,
                  void* W_, int64_t ldW, void* E_, int64_t ldE, int64_t k0, int64_t* piv, double* err, double* rho,
                  int32_t* nu, int64_t* k_out, const rb_opts* opts_in, rb_stats* stats, hipStream_t stream) {
  const auto t_begin = std::chrono::steady_clock::now();
  rb_opts o;
  rb_default_opts(&o);
  if (opts_in) o = *opts_in;
  char msg[160];
  auto bad = [&](const char* what) {
    std::snprintf(msg, sizeof msg, "%s: %s", fn, what);
    return set_error(RB_EINVAL, msg);
  };
  if (!S_ || N <= 0 || M <= 0 || !valid_ld(N, ldS) || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol) || !piv ||
      !err || !rho || !k_out || k0 < 0)
    return bad("bad arguments");
  if ((kmax > 0 || k0 > 0) && (!E_ || !valid_ld(N, ldE))) return bad("bad basis buffer");
  if (W_ && !valid_ld(N, ldW)) return bad("bad working-matrix leading dimension");
  if (W_ == S_ && W_ && ldW != ldS) return bad("W == S needs ldW == ldS");
  if (!(o.kappa > 1.0) || o.nu_max < 1 || o.nu_min < 1 || o.nu_min > o.nu_max || !(o.theta > 0.0) ||
      !(o.theta < 1.0) || o.anchor_max < 1)
    return bad("bad options");

  const double2* S = static_cast<const double2*>(S_);
  double2* E = static_cast<double2*>(E_);
  int64_t kcap = kmax;
  if (kcap > N) kcap = N;
  if (kcap > k0 + M) kcap = k0 + M;
  if (k0 > kcap) return bad("the starting basis is larger than kmax or N");
  const int64_t panel = o.anchor_max;
  const int64_t np = sweep_partials_needed(M);

  rb_stats st;
  std::memset(&st, 0, sizeof st);
  EventTimer tm(o.collect_stats != 0, stream);

  DevBuf d_nrm, d_nrm0, d_acc, d_mask, d_part, d_res, d_cpan, d_v, d_g, d_sq, d_bad, d_Wown;
  RB_ALLOC(d_nrm, sizeof(double) * M);
  RB_ALLOC(d_nrm0, sizeof(double) * M);
  RB_ALLOC(d_acc, sizeof(double) * M);
  RB_ALLOC(d_mask, M);
  RB_ALLOC(d_part, sizeof(ArgMax) * np);
  RB_ALLOC(d_res, sizeof(ArgMax));
  RB_ALLOC(d_cpan, sizeof(double2) * (size_t)panel * (size_t)M);
  RB_ALLOC(d_v, sizeof(double2) * N);
  RB_ALLOC(d_g, sizeof(double2) * (kcap > 0 ? kcap : 1));
  RB_ALLOC(d_sq, sizeof(double) * 4);
  RB_ALLOC(d_bad, sizeof(int));
  HostBuf h;
  if (h.alloc(64) != hipSuccess) return set_error(RB_ENOMEM, "pinned host allocation failed");
  ArgMax* h_res = h.as<ArgMax>();                          // 16 B
  double* h_sc = reinterpret_cast<double*>(h.as<char>() + 16);  // scalars
  int* h_bad = reinterpret_cast<int*>(h.as<char>() + 48);

  double* nrm = d_nrm.as<double>();
  double* nrm0 = d_nrm0.as<double>();
  double* acc = d_acc.as<double>();
  uint8_t* mask = d_mask.as<uint8_t>();
  ArgMax* part = d_part.as<ArgMax>();
  ArgMax* res = d_res.as<ArgMax>();
  double2* cpan = d_cpan.as<double2>();  // panel row r (vector a + r) at cpan + r*M
  double2* v = d_v.as<double2>();
  double2* g = d_g.as<double2>();
  double* sq = d_sq.as<double>();

  // ---- initial norms (Alg. 3: sigma_0(s_i) = ||s_i||) ----
  tm.start();
  RB_HIP(hipMemsetAsync(d_bad.p, 0, sizeof(int), stream));
  RB_HIP(launch_colnorms_z(S, N, M, ldS, nrm, d_bad.as<int>(), stream));
  RB_HIP(hipMemcpyAsync(h_bad, d_bad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipMemcpyAsync(nrm0, nrm, sizeof(double) * M, hipMemcpyDeviceToDevice, stream));
  RB_HIP(hipMemsetAsync(acc, 0, sizeof(double) * M, stream));
  RB_HIP(hipMemsetAsync(mask, 0, M, stream));
  RB_HIP(launch_est_argmax(nrm, nullptr, mask, M, part, np, res, stream));
  RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  tm.stop(&st.ms_anchor);
  if (*h_bad) {
    std::snprintf(msg, sizeof msg, "%s: S holds a non-finite value", fn);
    return set_error(RB_ENONFINITE, msg);
  }

  // working matrix X: S until the first anchoring, W afterwards
  const double2* X = S;
  int64_t ldX = ldS;
  bool written = false;   // X has been written (an anchoring or the start)
  double2* W = static_cast<double2*>(W_);
  int64_t ldWk = ldW;
  double A_w = h_res->v;  // largest nrm since the last anchoring
  int64_t J = h_res->i;
  int64_t k = 0;          // basis vectors so far
  int64_t a = 0;          // first basis vector in the coefficient panel
  int64_t m = 0;          // vectors swept since the last anchoring
  int status = RB_KMAX;

  // ---- continuation: reduce every column against the k0 given vectors ----
  // X <- S - E0 (E0^H S), a block at a time (at most `panel` vectors per
  // block; blocks in order), then nrm = ||x||^2 and the pivot search starts
  // from there with k = k0.
  if (k0 > 0) {
    tm.start();
    if (!W) {
      RB_ALLOC(d_Wown, sizeof(double2) * (size_t)N * (size_t)M);
      W = d_Wown.as<double2>();
      ldWk = N;
    }
    for (int64_t b0 = 0; b0 < k0; b0 += panel) {
      const int64_t pb = std::min<int64_t>(panel, k0 - b0);
      RB_HIP(launch_project_z(E + b0 * ldE, N, pb, ldE, X, M, ldX, cpan, pb, stream));
      RB_HIP(launch_resid(X, ldX, W, ldWk, N, M, E + b0 * ldE, ldE, pb, cpan, 1, pb, nrm, d_bad.as<int>(), stream));
      X = W;
      ldX = ldWk;
    }
    written = true;
    RB_HIP(launch_est_argmax(nrm, nullptr, mask, M, part, np, res, stream));
    RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    tm.stop(&st.ms_anchor);
    st.anchors++;
    A_w = h_res->v;
    J = h_res->i;
    k = a = k0;
  }
  err[k] = std::sqrt(A_w > 0.0 ? A_w : 0.0);

  // Re-anchoring against the m panel vectors a..a+m-1 swept since the last
  // writing anchoring.  write: X <- X - E_p C_p (the panel restarts);
  // otherwise only nrm_j <- ||x_j - E_p c_j||^2 (one read of X; the panel
  // keeps growing: later sweep coefficients of x_j differ from those of the
  // deflated column by at most u ||x_j|| per vector, an error m u sqrt(A_X)
  // in err that stays far below the rounding of the explicit form).
  // Either way acc <- 0 and the pivot is the argmax of the fresh norms.
  double A_X = A_w;  // largest nrm of X when it was last written
  auto anchor = [&](bool write) -> int {
    tm.start();
    if (write && !W) {
      const size_t bytes = sizeof(double2) * (size_t)N * (size_t)M;
      RB_ALLOC(d_Wown, bytes);
      W = d_Wown.as<double2>();
      ldWk = N;
    }
    if (write) {
      RB_HIP(launch_resid(X, ldX, W, ldWk, N, M, E + a * ldE, ldE, m, cpan, M, 1, nrm, d_bad.as<int>(), stream));
      X = W;
      ldX = ldWk;
      written = true;
    } else {
      RB_HIP(launch_resid(X, ldX, static_cast<double2*>(nullptr), 0, N, M, E + a * ldE, ldE, m, cpan, M, 1, nrm,
                          d_bad.as<int>(), stream));
    }
    RB_HIP(hipMemsetAsync(acc, 0, sizeof(double) * M, stream));
    RB_HIP(launch_est_argmax(nrm, nullptr, mask, M, part, np, res, stream));
    RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    tm.stop(&st.ms_anchor);
    if (write) {
      a = k;
      m = 0;
      A_X = h_res->v;
    }
    A_w = h_res->v;
    st.anchors++;
    return RB_OK;
  };
  // a norms-only anchoring keeps the extra estimate error 2 m u sqrt(A_X)
  // rho below a tenth of the resolution threshold theta rho^2
  auto norms_only_ok = [&](double est) -> bool {
    if (!written) return false;
    const double rho = std::sqrt(est > 0.0 ? est : 0.0);
    return 2.0 * (double)panel * 0x1p-53 * std::sqrt(A_X) <= 0.1 * o.theta * rho;
  };

  while (true) {
    if (err[k] < tol) {
      status = RB_OK;
      break;
    }
    if (k == kcap) break;
    if (J < 0) break;  // every column pivoted

    // ---- 1. orthonormalise x_J (iterated Gram-Schmidt, kappa criterion) ----
    tm.start();
    RB_HIP(hipMemcpyAsync(v, X + J * ldX, sizeof(double2) * N, hipMemcpyDeviceToDevice, stream));
    // ||v|| before the first pass: the stored column (its norm differs from
    // nrm[J] after a norms-only re-anchoring)
    if (k > 0) {
      RB_HIP(launch_sqnorms_small(v, N, 1, N, sq + 1, stream));
      RB_HIP(hipMemcpyAsync(&h_sc[0], sq + 1, sizeof(double), hipMemcpyDeviceToHost, stream));
    } else {
      RB_HIP(hipMemcpyAsync(&h_sc[0], nrm + J, sizeof(double), hipMemcpyDeviceToHost, stream));
    }
    RB_HIP(hipMemcpyAsync(&h_sc[1], nrm0 + J, sizeof(double), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    double before = std::sqrt(h_sc[0]);
    const double s_norm = std::sqrt(h_sc[1]);
    double after = before;
    const double* scale_src = nrm + J;  // k == 0: the exact column norm
    int passes = 0;
    if (k == 0) {
      passes = 1;  // a pass against an empty basis changes nothing
    } else {
      while (passes < o.nu_max) {
        RB_HIP(launch_gemv_ch(E, ldE, k, v, N, 1, N, g, stream));
        RB_HIP(launch_gemv_n_sub(E, ldE, k, g, v, N, 1, N, stream));
        RB_HIP(launch_sqnorms_small(v, N, 1, N, sq, stream));
        RB_HIP(hipMemcpyAsync(&h_sc[2], sq, sizeof(double), hipMemcpyDeviceToHost, stream));
        RB_HIP(hipStreamSynchronize(stream));
        ++passes;
        after = std::sqrt(h_sc[2]);
        if (passes >= o.nu_min && after > before / o.kappa) break;
        before = after;
      }
      scale_src = sq;
    }
    st.gs_passes += passes;
    const double r = after;
    if (!(r > 64.0 * 0x1p-53 * s_norm)) {  // numerically in span(E)
      tm.stop(&st.ms_gs);
      status = RB_RANK;
      break;
    }
    RB_HIP(launch_scale_into(v, N, scale_src, E + k * ldE, stream));
    RB_HIP(hipMemsetAsync(mask + J, 1, 1, stream));
    tm.stop(&st.ms_gs);
    piv[k] = J;
    rho[k] = r;
    if (nu) nu[k] = passes;
    ++k;

    // ---- 2. fused sweep with the new vector (panel row m) ----
    if (m == panel) {
      int rc = anchor(true);
      if (rc != RB_OK) return rc;
      // the new vector has not been swept yet: the panel restarts at it
      a = k - 1;
    }
    tm.start();
    RB_HIP(launch_sweep_z(X, N, M, ldX, E + (k - 1) * ldE, nrm, acc, mask, cpan + m * M, 1, part, np, nullptr,
                          stream));
    tm.stop(&st.ms_sweep);  // the sweep kernel alone
    RB_HIP(launch_sweep_final(M, part, res, stream));
    RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    st.sweeps++;
    ++m;
    double est_max = h_res->v;
    J = h_res->i;

    // ---- 3. resolution check and error ----
    if (J >= 0 && est_max < o.theta * A_w) {
      int rc = anchor(!norms_only_ok(est_max));
      if (rc != RB_OK) return rc;
      est_max = h_res->v;
      J = h_res->i;
    }
    err[k] = (J >= 0) ? std::sqrt(est_max > 0.0 ? est_max : 0.0) : 0.0;
  }
  if (status == RB_KMAX && err[k] < tol) status = RB_OK;
  *k_out = k;
  st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
  if (stats) *stats = st;
  return status;
}

}  // namespace rb

extern "C" {

int rb_greedy_z(const void* S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, void* W, int64_t ldW,
                void* E, int64_t ldE, int64_t* piv, double* err, double* rho, int32_t* nu, int64_t* k_out,
                const rb_opts* opts, rb_stats* stats, hipStream_t stream) {
  last_error().clear();
  return greedy_z_core("rb_greedy_z", S, N, M, ldS, tol, kmax, W, ldW, E, ldE, 0, piv, err, rho, nu, k_out, opts,
                       stats, stream);
}

int rb_greedy_resume_z(const void* S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, void* W,
                       int64_t ldW, void* E, int64_t ldE, int64_t k0, int64_t* piv, double* err, double* rho,
                       int32_t* nu, int64_t* k_out, const rb_opts* opts, rb_stats* stats, hipStream_t stream) {
  last_error().clear();
  return greedy_z_core("rb_greedy_resume_z", S, N, M, ldS, tol, kmax, W, ldW, E, ldE, k0, piv, err, rho, nu, k_out,
                       opts, stats, stream);
}

}  // extern "C"

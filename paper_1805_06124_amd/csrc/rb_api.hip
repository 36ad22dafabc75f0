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
  o->theta = 1e-7;
  o->anchor_max = 128;
  o->collect_stats = 0;
  o->theta32 = 1e-4;
  o->regen_chunk = 32768;
  o->certify = 2;
  o->step_ms = nullptr;
  o->fuse = 1;
  o->lookahead = 5;
  o->look_k = 4096;
  o->lookahead32 = -1;
}

const char* rb_strerror(int status) {
  switch (status) {
    case RB_OK: return "converged (err < tol)";
    case RB_KMAX: return "stopped at kmax";
    case RB_RANK: return "rank exhausted (pivot in the span of the basis)";
    case RB_EINVAL: return "invalid argument";
    case RB_ENOMEM: return "device allocation failed";
    case RB_EDEVICE: return "HIP runtime error";
    case RB_ENONFINITE: return "non-finite value (input, re-anchored column or estimate)";
    case RB_EBREAKDOWN: return "iterated Gram-Schmidt did not settle within nu_max passes";
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

namespace {

// Device scratch of the FP64 greedy, carved from one workspace.
struct ZScratch {
  double *nrm, *nrm0, *acc, *sq;
  uint8_t* mask;
  ArgMax *part, *res;
  double2 *cpan, *v, *g;
  int* bad;
  // pivot lookahead: candidate list and its scratch, list-local sums, rerank partials
  ArgMax *list = nullptr, *rpart = nullptr, *lres = nullptr, *coarse = nullptr;
  double* acc_l = nullptr;
  GsState* gst = nullptr;  // [0]: the step's own orthogonalisation, [1 + d]: prediction d
  // returns the bytes used (base == nullptr: sizing only); look_k = 0: no lookahead
  size_t carve(void* base, int64_t N, int64_t M, int64_t kcap, int64_t panel, int look_k) {
    Carve c(base);
    nrm = c.take<double>(M);
    nrm0 = c.take<double>(M);
    acc = c.take<double>(M);
    mask = c.take<uint8_t>(M);
    part = c.take<ArgMax>(2 * sweep_partials_needed(M));  // the fused pass keeps two maxima per workgroup
    res = c.take<ArgMax>(2);
    cpan = c.take<double2>((size_t)panel * (size_t)M);  // panel row r (vector a + r) at r*M
    v = c.take<double2>(N);
    g = c.take<double2>(kcap > 0 ? kcap : 1);
    sq = c.take<double>(4);
    bad = c.take<int>(1);
    gst = c.take<GsState>(kLookMax + 1);
    if (look_k > 0) {
      list = c.take<ArgMax>(look_k);
      const int64_t nc = look_list_scratch((M + kPivotGroup - 1) / kPivotGroup);
      if (nc > 0) coarse = c.take<ArgMax>(nc);
      acc_l = c.take<double>(look_k);
      rpart = c.take<ArgMax>(rerank_partials(look_k));
      lres = c.take<ArgMax>(1);
    }
    return c.used;
  }
};

bool z_opts_ok(const rb_opts& o) {
  return o.kappa > 1.0 && o.nu_max >= 1 && o.nu_min >= 1 && o.nu_min <= o.nu_max && o.theta > 0.0 &&
         o.theta < 1.0 && o.anchor_max >= 1 && o.lookahead >= 0 && o.lookahead <= kLookMax &&
         (o.lookahead == 0 || (o.look_k >= 1 && o.look_k <= kLookListMax));
}
int z_look_k(const rb_opts& o) { return o.lookahead > 0 ? o.look_k : 0; }

}  // namespace

size_t greedy_z_ws_bytes(int64_t N, int64_t M, int64_t kmax, const rb_opts* opts_in) {
  rb_opts o;
  rb_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (N <= 0 || M <= 0 || kmax < 0 || !z_opts_ok(o)) return 0;
  ZScratch z;
  return z.carve(nullptr, N, M, std::min(kmax, N), o.anchor_max, z_look_k(o));
}

// The FP64 greedy, started from k0 >= 0 orthonormal vectors already in
// E[:, 0..k0-1] (k0 = 0: the greedy of Alg. 3 itself).
int greedy_z_core(const char* fn, const void* S_, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax,
                  void* W_, int64_t ldW, void* E_, int64_t ldE, int64_t k0, int64_t* piv, double* err, double* rho,
                  int32_t* nu, int64_t* k_out, void* ws, size_t ws_bytes, const rb_opts* opts_in, rb_stats* stats,
                  hipStream_t stream) {
  const auto t_begin = std::chrono::steady_clock::now();
  rb_opts o;
  rb_default_opts(&o);
  if (opts_in) o = *opts_in;
  auto fail = [&](int code, const char* what) { return set_error(code, "%s: %s", fn, what); };
  if (!S_ || N <= 0 || M <= 0 || !valid_ld(N, ldS) || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol) || !piv ||
      !err || !rho || !k_out || k0 < 0)
    return fail(RB_EINVAL, "bad arguments");
  if ((kmax > 0 || k0 > 0) && (!E_ || !valid_ld(N, ldE))) return fail(RB_EINVAL, "bad basis buffer");
  if (W_ && !valid_ld(N, ldW)) return fail(RB_EINVAL, "bad working-matrix leading dimension");
  if (W_ == S_ && W_ && ldW != ldS) return fail(RB_EINVAL, "W == S needs ldW == ldS");
  if (!z_opts_ok(o)) return fail(RB_EINVAL, "bad options");
  if (ws && !W_) return fail(RB_EINVAL, "a caller workspace needs a working matrix W (W may be S)");
  if (ws && reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(RB_EINVAL, "workspace not 256-byte aligned");

  const double2* S = static_cast<const double2*>(S_);
  double2* E = static_cast<double2*>(E_);
  int64_t kcap = kmax;
  if (kcap > N) kcap = N;
  if (kcap > k0 + M) kcap = k0 + M;
  if (k0 > kcap) return fail(RB_EINVAL, "the starting basis is larger than kmax or N");
  const int64_t panel = o.anchor_max;
  const int64_t np = sweep_partials_needed(M);
  const int64_t np2 = 2 * np;  // capacity of the partials for a fused pass

  // scratch: the caller's workspace, or one allocation of the same layout
  ZScratch z;
  const size_t need = z.carve(nullptr, N, M, std::min(kmax, N), panel, z_look_k(o));
  DevBuf d_ws, d_Wown;
  if (ws) {
    if (ws_bytes < need) {
      char m[160];
      std::snprintf(m, sizeof m, "workspace of %zu bytes, %zu needed", ws_bytes, need);
      return fail(RB_ENOMEM, m);
    }
  } else {
    RB_ALLOC(d_ws, need);
    ws = d_ws.p;
  }
  z.carve(ws, N, M, std::min(kmax, N), panel, z_look_k(o));
  HostWords hw;
  if (hw.init(d_ws.p != nullptr, 96 + sizeof(GsState) * (kLookMax + 1)) != hipSuccess)
    return fail(RB_ENOMEM, "pinned host allocation failed");
  ArgMax* h_res = hw.at<ArgMax>(0);     // 2 x 16 B
  double* h_sc = hw.at<double>(32);     // scalars
  int* h_bad = hw.at<int>(64);
  GsState* h_gs = hw.at<GsState>(96);   // kLookMax + 1 records

  rb_stats st;
  std::memset(&st, 0, sizeof st);
  EventTimer tm(o.collect_stats != 0, stream);
  double* step_ms = (tm.on && o.step_ms) ? o.step_ms : nullptr;
  auto slot = [&](int64_t i, int part) -> double* {
    return (step_ms && i <= kcap) ? step_ms + 3 * i + part : nullptr;
  };

  double* nrm = z.nrm;
  double* nrm0 = z.nrm0;
  double* acc = z.acc;
  uint8_t* mask = z.mask;
  ArgMax* part = z.part;
  ArgMax* res = z.res;
  double2* cpan = z.cpan;
  double2* v = z.v;
  double2* g_coef = z.g;
  double* sq = z.sq;

  // ---- initial norms (Alg. 3: sigma_0(s_i) = ||s_i||) ----
  tm.start();
  RB_HIP(launch_fill(z.bad, 0, 1, stream));
  RB_HIP(launch_colnorms_z(S, N, M, ldS, nrm, z.bad, stream));
  RB_HIP(hipMemcpyAsync(h_bad, z.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipMemcpyAsync(nrm0, nrm, sizeof(double) * M, hipMemcpyDeviceToDevice, stream));
  RB_HIP(launch_fill(acc, 0.0, M, stream));
  RB_HIP(launch_fill(mask, (uint8_t)0, M, stream));
  RB_HIP(launch_est_argmax(nrm, nullptr, mask, M, part, np, res, stream));
  RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  lap(tm, &st.ms_anchor, nullptr);
  if (*h_bad) return fail(RB_ENONFINITE, "S holds a non-finite value");

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
  // an error found after the run started: the outputs of the k completed
  // vectors stay valid
  auto fail_run = [&](int code, const char* what) {
    char m2[200];
    std::snprintf(m2, sizeof m2, "%s (after %lld basis vectors)", what, (long long)k);
    *k_out = k;
    if (stats) *stats = st;
    return fail(code, m2);
  };

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
      RB_HIP(launch_resid(X, ldX, W, ldWk, N, M, E + b0 * ldE, ldE, pb, cpan, 1, pb, nrm, z.bad, stream));
      X = W;
      ldX = ldWk;
    }
    written = true;
    RB_HIP(launch_est_argmax(nrm, nullptr, mask, M, part, np, res, stream));
    RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipMemcpyAsync(h_bad, z.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    lap(tm, &st.ms_anchor, nullptr);
    st.anchors++;
    k = a = k0;
    if (*h_bad) return fail_run(RB_ENONFINITE, "a reduced column is not finite");
    A_w = h_res->v;
    J = h_res->i;
  }
  err[k] = std::sqrt(A_w > 0.0 ? A_w : 0.0);

  double A_X = A_w;  // largest nrm of X when it was last written

  // Pivot lookahead (rb_look.hip): predictions spec[spec_at .. nspec) made
  // at the last sweep, each with its vector in E[:, k + d] already and its
  // coefficients in panel row m + d.  fine_part: part holds the per-group
  // partials of the current estimates (the list's source).
  struct Spec {
    int64_t J;
    double r;
    int passes;
  };
  Spec spec[kLookMax];
  int nspec = 0, spec_at = 0;
  bool fine_part = false;
  const int look_k = z_look_k(o);
  const int64_t ngroups = (M + kPivotGroup - 1) / kPivotGroup;

  // Re-anchoring against the m panel vectors a..a+m-1 swept since the last
  // writing anchoring.  write: X <- X - E_p C_p (the panel restarts);
  // otherwise only nrm_j <- ||x_j - E_p c_j||^2 (one read of X; the panel
  // keeps growing: later sweep coefficients of x_j differ from those of the
  // deflated column by at most u ||x_j|| per vector, an error m u sqrt(A_X)
  // in err that stays far below the rounding of the explicit form).
  // Either way acc <- 0 and the pivot is the argmax of the fresh norms.
  auto anchor = [&](bool write, double* slot_ms) -> int {
    nspec = spec_at = 0;
    fine_part = false;
    tm.start();
    if (write && !W) {
      const size_t bytes = sizeof(double2) * (size_t)N * (size_t)M;
      RB_ALLOC(d_Wown, bytes);
      W = d_Wown.as<double2>();
      ldWk = N;
    }
    if (write) {
      RB_HIP(launch_resid(X, ldX, W, ldWk, N, M, E + a * ldE, ldE, m, cpan, M, 1, nrm, z.bad, stream));
      X = W;
      ldX = ldWk;
      written = true;
    } else {
      RB_HIP(launch_resid(X, ldX, static_cast<double2*>(nullptr), 0, N, M, E + a * ldE, ldE, m, cpan, M, 1, nrm,
                          z.bad, stream));
    }
    RB_HIP(launch_fill(acc, 0.0, M, stream));
    RB_HIP(launch_est_argmax(nrm, nullptr, mask, M, part, np, res, stream));
    RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipMemcpyAsync(h_bad, z.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    lap(tm, &st.ms_anchor, slot_ms);
    st.anchors++;
    if (*h_bad) return fail_run(RB_ENONFINITE, "a re-anchored column is not finite");
    if (write) {
      a = k;
      m = 0;
      A_X = h_res->v;
    }
    A_w = h_res->v;
    return RB_OK;
  };
  // a norms-only anchoring keeps the extra estimate error 2 m u sqrt(A_X)
  // rho below a tenth of the resolution threshold theta rho^2
  auto norms_only_ok = [&](double est) -> bool {
    if (!written) return false;
    const double r = std::sqrt(est > 0.0 ? est : 0.0);
    return 2.0 * (double)panel * 0x1p-53 * std::sqrt(A_X) <= 0.1 * o.theta * r;
  };
  // Re-anchoring ahead of time, fused with the next sweep: when the next
  // estimate is predicted (from the last step's decrease) to fall within a
  // factor kFusePredict of the resolution threshold, the panel holds at most
  // kFuseMaxM vectors and a norms-only anchoring is accurate enough, the
  // next sweep also recomputes every column's residual norm against the
  // panel, in the same read of X.  A step that still ends below the
  // threshold falls back to the separate re-anchoring above.
  constexpr double kFusePredict = 4.0;
  bool fuse_next = false;
  double est_prev = A_w;
  // the fused pass with the newest vector (column k - 1 of E)
  auto fused_sweep = [&](double* slot_ms, double* est_out, int64_t* J_out) -> int {
    nspec = spec_at = 0;
    fine_part = false;
    tm.start();
    RB_HIP(launch_anchor_sweep(X, ldX, N, M, E + a * ldE, ldE, m, cpan, M, E + (k - 1) * ldE, nrm, acc, mask,
                               cpan + m * M, part, np2, res, z.bad, stream));
    ++m;
    RB_HIP(hipMemcpyAsync(h_res, res, 2 * sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipMemcpyAsync(h_bad, z.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    lap(tm, &st.ms_fused, slot_ms);
    st.anchors++;
    st.fused++;
    if (*h_bad) return fail_run(RB_ENONFINITE, "a re-anchored column is not finite");
    A_w = h_res[1].v;
    *est_out = h_res[0].v;
    *J_out = h_res[0].i;
    return RB_OK;
  };

  // Orthogonalisation of the pivot (iterated classical Gram-Schmidt with
  // Hoffmann's kappa criterion, Sec. 6.1.2) against E[:, 0..kk-1], kk >= 1,
  // driven from the device (GsState): a step's own reads its outcome back
  // once, a predicted one (rb_look.hip) not at all, and both run the same
  // kernels.  jsrc (device) or jhost names the column; prev chains
  // predictions; an accepted vector goes to E[:, kk].
  // passes: how many passes to queue (at most nu_max); an orthogonalisation
  // that would need more is not accepted.
  auto gs_launch = [&](const ArgMax* jsrc, int64_t jhost, const GsState* prev, int64_t kk, GsState* gs,
                       int passes) -> int {
    RB_HIP(launch_gs_begin(X, ldX, N, jsrc, jhost, prev, nrm0, v, sq + 1, gs, stream));
    for (int p = 0; p < passes; ++p)
      RB_HIP(launch_gs_pass(E, ldE, kk, v, N, g_coef, sq, gs, o.nu_min, o.nu_max, o.kappa, stream));
    RB_HIP(launch_gs_finish(gs, tol, sq, v, N, E + kk * ldE, stream));
    return RB_OK;
  };

  // Predict the next dmax pivots before the sweep with E[:, k-1]: the best
  // listed column after reranking with E[:, k-1] (then with each predicted
  // vector in turn), orthogonalised into E[:, k + d] as its own step would
  // do it; a prediction that step would not accept ends the chain.  No
  // host round trip: the outcomes are read back with the sweep's argmax.
  // A predicted orthogonalisation queues at most kLookPasses passes (with
  // kappa = 2 a pivot's orthogonalisation settles after one or two: every
  // step of the 10,000 x 409,600 chirp run does); one that needs more ends
  // the chain and its step runs its own.
  const int look_passes = std::min(o.nu_max, std::max(o.nu_min, kLookPasses));
  auto predict = [&](int dmax) -> int {
    tm.start();
    if (!fine_part) RB_HIP(launch_est_apply(nrm, acc, mask, nullptr, M, part, np, stream));
    RB_HIP(launch_look_list(part, ngroups, look_k, z.list, z.coarse, stream));
    for (int d = 0; d < dmax; ++d) {
      GsState* gd = z.gst + 1 + d;
      RB_HIP(launch_rerank(X, N, ldX, E + (k - 1 + d) * ldE, z.list, look_k, nrm, acc, z.acc_l, d == 0 ? 1 : 0,
                           mask, z.gst + 1, d, z.rpart, z.lres, stream));
      int rc = gs_launch(z.lres, -1, d > 0 ? gd - 1 : nullptr, k + d, gd, look_passes);
      if (rc != RB_OK) return rc;
    }
    lap(tm, &st.ms_look, nullptr);
    return RB_OK;
  };

  while (true) {
    if (err[k] < tol) {
      status = RB_OK;
      break;
    }
    if (k == kcap) break;
    if (J < 0) break;

    // A step whose pivot was predicted at the last sweep: its vector and its
    // coefficients are already there, unless this step would not run a
    // plain sweep (a fused re-anchoring is due).
    bool taken = false;
    if (spec_at < nspec) {
      const bool fused_due = fuse_next && m <= kFuseMaxM && norms_only_ok(est_prev);
      if (spec[spec_at].J == J && m < panel && !fused_due) taken = true;
      else nspec = spec_at = 0;
    }
    double est_max = 0.0;
    if (taken) {
      const Spec sp = spec[spec_at++];
      tm.start();
      RB_HIP(launch_fill(mask + J, (uint8_t)1, 1, stream));
      RB_HIP(launch_est_apply(nrm, acc, mask, cpan + m * M, M, part, np, stream));
      RB_HIP(launch_sweep_final(M, part, res, stream));
      RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
      RB_HIP(hipStreamSynchronize(stream));
      lap(tm, &st.ms_apply, slot(k, 1));
      piv[k] = J;
      rho[k] = sp.r;
      if (nu) nu[k] = sp.passes;
      st.gs_passes += sp.passes;
      st.look_steps++;
      ++k;
      ++m;
      fine_part = true;
      est_max = h_res->v;
      J = h_res->i;
    } else {
      nspec = spec_at = 0;
      // ---- 1. orthonormalise x_J (iterated Gram-Schmidt, kappa criterion) ----
      tm.start();
      double r = 0.0;
      int passes = 1;
      if (k == 0) {
        // against an empty basis: e = s_J / ||s_J|| with the exact norm
        RB_HIP(hipMemcpyAsync(v, X + J * ldX, sizeof(double2) * N, hipMemcpyDeviceToDevice, stream));
        RB_HIP(hipMemcpyAsync(&h_sc[0], nrm + J, sizeof(double), hipMemcpyDeviceToHost, stream));
        RB_HIP(hipStreamSynchronize(stream));
        r = std::sqrt(h_sc[0]);
        if (!std::isfinite(r)) return fail_run(RB_ENONFINITE, "an orthogonalised pivot is not finite");
        if (!(r > 0.0)) {
          status = RB_RANK;
          break;
        }
        RB_HIP(launch_scale_into(v, N, nrm + J, E, stream));
      } else {
        // the passes a pivot usually needs first; the rest only if it has not
        // finished (they continue from the device state)
        int rc = gs_launch(nullptr, J, nullptr, k, z.gst, look_passes);
        if (rc != RB_OK) return rc;
        RB_HIP(hipMemcpyAsync(h_gs, z.gst, sizeof(GsState), hipMemcpyDeviceToHost, stream));
        RB_HIP(hipStreamSynchronize(stream));
        if (!h_gs->done) {
          for (int p = look_passes; p < o.nu_max; ++p)
            RB_HIP(launch_gs_pass(E, ldE, k, v, N, g_coef, sq, z.gst, o.nu_min, o.nu_max, o.kappa, stream));
          RB_HIP(launch_gs_finish(z.gst, tol, sq, v, N, E + k * ldE, stream));
          RB_HIP(hipMemcpyAsync(h_gs, z.gst, sizeof(GsState), hipMemcpyDeviceToHost, stream));
          RB_HIP(hipStreamSynchronize(stream));
        }
        const GsState& g = *h_gs;
        r = g.after;
        passes = g.passes;
        if (!g.finite) return fail_run(RB_ENONFINITE, "an orthogonalised pivot is not finite");
        if (g.in_span) {  // numerically in span(E)
          status = RB_RANK;
          break;
        }
        if (!g.settled && r >= tol) {
          char m2[160];
          std::snprintf(m2, sizeof m2, "Gram-Schmidt of pivot %lld still shrank ||v|| by kappa after %d passes",
                        (long long)J, passes);
          return fail_run(RB_EBREAKDOWN, m2);
        }
      }
      st.gs_passes += passes;
      RB_HIP(launch_fill(mask + J, (uint8_t)1, 1, stream));
      lap(tm, &st.ms_gs, slot(k, 0));
      piv[k] = J;
      rho[k] = r;
      if (nu) nu[k] = passes;
      ++k;

      // ---- 2. sweep with the new vector (panel row m) ----
      if (m == panel) {
        int rc = anchor(true, slot(k - 1, 2));
        if (rc != RB_OK) return rc;
        // the new vector has not been swept yet: the panel restarts at it
        a = k - 1;
      }
      if (fuse_next && m <= kFuseMaxM && norms_only_ok(est_prev)) {
        int rc = fused_sweep(slot(k - 1, 1), &est_max, &J);
        if (rc != RB_OK) return rc;
      } else {
        // predicted vectors ride along in the same read of X, within the
        // panel and the basis capacity (one that was not accepted is read
        // too and its coefficients are never used)
        const int64_t dmax = std::min<int64_t>(std::min<int64_t>(o.lookahead, panel - m - 1), kcap - k);
        if (dmax > 0) {
          int rc2 = predict((int)dmax);
          if (rc2 != RB_OK) return rc2;
        }
        tm.start();
        if (dmax > 0)
          RB_HIP(launch_sweep_look(X, N, M, ldX, E + (k - 1) * ldE, ldE, 1 + (int)dmax, nrm, acc, mask,
                                   cpan + m * M, part, np, stream));
        else
          RB_HIP(launch_sweep_z(X, N, M, ldX, E + (k - 1) * ldE, nrm, acc, mask, cpan + m * M, 1, part, np,
                                nullptr, stream));
        const double ms_before = st.ms_sweep;
        lap(tm, &st.ms_sweep, slot(k - 1, 1));  // the sweep kernel alone
        if (dmax > 0) st.ms_look_sweep += st.ms_sweep - ms_before;
        RB_HIP(launch_sweep_final(M, part, res, stream));
        RB_HIP(hipMemcpyAsync(h_res, res, sizeof(ArgMax), hipMemcpyDeviceToHost, stream));
        if (dmax > 0)
          RB_HIP(hipMemcpyAsync(h_gs + 1, z.gst + 1, sizeof(GsState) * dmax, hipMemcpyDeviceToHost, stream));
        RB_HIP(hipStreamSynchronize(stream));
        st.sweeps++;
        int nd = 0;
        if (dmax > 0) {
          st.look_sweeps++;
          st.look_vectors += dmax;
          for (int d = 0; d < (int)dmax; ++d) st.look_gs += h_gs[1 + d].live;
          while (nd < (int)dmax && h_gs[1 + nd].accept) {
            spec[nd] = Spec{h_gs[1 + nd].J, h_gs[1 + nd].after, h_gs[1 + nd].passes};
            ++nd;
          }
        }
        ++m;
        fine_part = true;
        nspec = nd;
        spec_at = 0;
        est_max = h_res->v;
        J = h_res->i;
      }
    }
    if (J >= 0 && std::isnan(est_max)) return fail_run(RB_ENONFINITE, "a swept estimate is not finite");

    // ---- 3. resolution check and error ----
    if (J >= 0 && est_max < o.theta * A_w) {
      int rc = anchor(!norms_only_ok(est_max), slot(k - 1, 2));
      if (rc != RB_OK) return rc;
      est_max = h_res->v;
      J = h_res->i;
    }
    err[k] = (J >= 0) ? std::sqrt(est_max > 0.0 ? est_max : 0.0) : 0.0;
    // ---- 4. fuse a re-anchoring into the next sweep? ----
    {
      const double e_now = est_max > 0.0 ? est_max : 0.0;
      const double ratio = (est_prev > 0.0 && e_now < est_prev) ? e_now / est_prev : 1.0;
      fuse_next = o.fuse != 0 && J >= 0 && e_now * ratio < kFusePredict * o.theta * A_w;
      est_prev = e_now;
    }
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
                void* E, int64_t ldE, int64_t* piv, double* err, double* rho, int32_t* nu, int64_t* k_out, void* ws,
                size_t ws_bytes, const rb_opts* opts, rb_stats* stats, hipStream_t stream) {
  last_error().clear();
  return greedy_z_core("rb_greedy_z", S, N, M, ldS, tol, kmax, W, ldW, E, ldE, 0, piv, err, rho, nu, k_out, ws,
                       ws_bytes, opts, stats, stream);
}

size_t rb_greedy_z_workspace(int64_t N, int64_t M, int64_t kmax, const rb_opts* opts) {
  return greedy_z_ws_bytes(N, M, kmax, opts);
}

int rb_greedy_resume_z(const void* S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, void* W,
                       int64_t ldW, void* E, int64_t ldE, int64_t k0, int64_t* piv, double* err, double* rho,
                       int32_t* nu, int64_t* k_out, void* ws, size_t ws_bytes, const rb_opts* opts, rb_stats* stats,
                       hipStream_t stream) {
  last_error().clear();
  return greedy_z_core("rb_greedy_resume_z", S, N, M, ldS, tol, kmax, W, ldW, E, ldE, k0, piv, err, rho, nu, k_out,
                       ws, ws_bytes, opts, stats, stream);
}

}  // extern "C"

// Mixed-precision RB-greedy (complex64 storage, FP64 basis) and the built-in
// chirp regenerator.
//
// One step k:
//   1. the candidate chosen at the previous step becomes e_k (FP64), with an
//      FP32 copy for the sweep;
//   2. one complex64 sweep with the FP32 copy (FP32 products and row-tile
//      sums, FP64 across tiles; acc/est FP64) nominates the 8 columns of
//      largest estimated residual;
//   3. the 8 are regenerated in FP64 and orthogonalised against the FP64
//      basis (iterated Gram-Schmidt, kappa criterion); the pivot is the
//      candidate with the largest exact residual rho, and err_k = rho
//      (Corollary 5.6).
// Re-anchoring (the stored-residual form, as in the FP64 driver) happens when
// the complex64 estimate falls below theta32 times its anchored scale or the
// coefficient panel is full.  Two kinds:
//   deflation : X32 <- round32(X32 - E_panel C_panel), cheap (one read and one
//               write of the complex64 matrix), but it leaves a perturbation
//               of up to kDelta32 * sigma in the stored columns;
//   exact     : X32 <- round32(s64 - E (E^H s64)) from columns regenerated in
//               FP64, which resets the perturbation to the storage rounding.
// A deflation is used while the accumulated perturbation stays below
// tol / 10, or while sigma is so large that a later anchoring must still
// come before the error can reach tol; otherwise the anchoring is exact.
#include <chrono>
#include <cmath>
#include <cstring>

#include "rb_host.h"

using namespace rb;

namespace {

// perturbation one complex64 re-anchoring may leave in a stored residual
// column, relative to that residual's norm: storage rounding (2^-24 per
// component) plus coefficients known to FP32 accuracy, with margin
constexpr double kDelta32 = 2.4e-7;

}  // namespace

extern "C" {

int rb_chirp_table(double flo, double fhi, int64_t N, double* table, hipStream_t stream) {
  last_error().clear();
  if (!table || N <= 0 || !(flo > 0.0) || !(fhi >= flo)) return set_error(RB_EINVAL, "rb_chirp_table: bad arguments");
  RB_HIP(launch_chirp_table(flo, fhi, N, table, stream));
  return RB_OK;
}

int rb_chirp_regen(void* ctx, const int64_t* cols, int64_t n, void* out, int64_t ldo, hipStream_t stream) {
  const rb_chirp_ctx* c = static_cast<const rb_chirp_ctx*>(ctx);
  if (!c || !c->params || !cols || !out || n <= 0 || c->N <= 0 || ldo < c->N) return RB_EINVAL;
  if (c->table) {
    hipError_t e = launch_chirp_fill(c->params, cols, n, c->table, c->N, 0, out, ldo, stream);
    return e == hipSuccess ? 0 : RB_EDEVICE;
  }
  DevBuf tab;  // no prepared table: build one for this call
  if (tab.alloc(sizeof(double) * 3 * (size_t)c->N) != hipSuccess) return RB_ENOMEM;
  hipError_t e = launch_chirp_table(c->flo, c->fhi, c->N, tab.as<double>(), stream);
  if (e == hipSuccess) e = launch_chirp_fill(c->params, cols, n, tab.as<double>(), c->N, 0, out, ldo, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);  // the table is freed on return
  return e == hipSuccess ? 0 : RB_EDEVICE;
}

int rb_sweep_c(const void* S32, int64_t N, int64_t M, int64_t ldS, const void* e32, const double* nrm, double* acc,
               const uint8_t* mask, void* c_out, int64_t ldc, double* est_top, int64_t* J_top, hipStream_t stream) {
  last_error().clear();
  if (!S32 || !e32 || !nrm || !acc || !est_top || !J_top || N <= 0 || M <= 0 || !valid_ld(N, ldS) ||
      (c_out && ldc <= 0))
    return set_error(RB_EINVAL, "rb_sweep_c: bad arguments");
  const int64_t np = sweep32_partials_needed(M);
  DevBuf part, top;
  RB_ALLOC(part, sizeof(ArgMax) * np);
  RB_ALLOC(top, sizeof(ArgMax) * kTop);
  RB_HIP(launch_sweep_c(static_cast<const float2*>(S32), N, M, ldS, static_cast<const float2*>(e32), nrm, acc, mask,
                        static_cast<double2*>(c_out), ldc, part.as<ArgMax>(), np, top.as<ArgMax>(), stream));
  ArgMax h[kTop];
  RB_HIP(hipMemcpyAsync(h, top.p, sizeof h, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  for (int r = 0; r < kTop; ++r) {
    est_top[r] = h[r].v;
    J_top[r] = h[r].i;
  }
  return RB_OK;
}

int rb_greedy_c(const void* S32_, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, rb_regen_fn regen,
                void* regen_ctx, void* W32_, int64_t ldW, void* E_, int64_t ldE, int64_t* piv, double* err,
                double* rho, int32_t* nu, int64_t* k_out, const rb_opts* opts_in, rb_stats* stats,
                hipStream_t stream) {
  last_error().clear();
  const auto t_begin = std::chrono::steady_clock::now();
  rb_opts o;
  rb_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (!S32_ || N <= 0 || M <= 0 || !valid_ld(N, ldS) || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol) ||
      !piv || !err || !rho || !k_out || !regen)
    return set_error(RB_EINVAL, "rb_greedy_c: bad arguments");
  if (kmax > 0 && (!E_ || !valid_ld(N, ldE))) return set_error(RB_EINVAL, "rb_greedy_c: bad basis buffer");
  if (W32_ && !valid_ld(N, ldW)) return set_error(RB_EINVAL, "rb_greedy_c: bad working-matrix leading dimension");
  if (W32_ == S32_ && W32_ && ldW != ldS) return set_error(RB_EINVAL, "rb_greedy_c: W32 == S32 needs ldW == ldS");
  if (!(o.kappa > 1.0) || o.nu_max < 1 || o.nu_min < 1 || o.nu_min > o.nu_max || !(o.theta32 > 0.0) ||
      !(o.theta32 < 1.0) || o.anchor_max < 1 || o.regen_chunk < 1)
    return set_error(RB_EINVAL, "rb_greedy_c: bad options");

  const float2* S32 = static_cast<const float2*>(S32_);
  double2* E = static_cast<double2*>(E_);
  int64_t kcap = kmax;
  if (kcap > N) kcap = N;
  if (kcap > M) kcap = M;
  const int64_t panel = o.anchor_max;
  const int64_t np = sweep32_partials_needed(M);
  const int64_t chunk = o.regen_chunk < M ? o.regen_chunk : M;

  rb_stats st;
  std::memset(&st, 0, sizeof st);
  EventTimer tm(o.collect_stats != 0, stream);

  DevBuf d_nrm, d_acc, d_mask, d_part, d_top, d_cpan, d_V, d_G, d_sq, d_cols, d_e32, d_bad;
  DevBuf d_Wown, d_S64c, d_Cc, d_iota;
  RB_ALLOC(d_nrm, sizeof(double) * M);
  RB_ALLOC(d_acc, sizeof(double) * M);
  RB_ALLOC(d_mask, M);
  RB_ALLOC(d_part, sizeof(ArgMax) * np);
  RB_ALLOC(d_top, sizeof(ArgMax) * kTop);
  RB_ALLOC(d_cpan, sizeof(double2) * (size_t)panel * (size_t)M);
  RB_ALLOC(d_V, sizeof(double2) * (size_t)N * kTop);
  RB_ALLOC(d_G, sizeof(double2) * (size_t)(kcap > 0 ? kcap : 1) * kTop);
  RB_ALLOC(d_sq, sizeof(double) * 2 * kTop);
  RB_ALLOC(d_cols, sizeof(int64_t) * kTop);
  RB_ALLOC(d_e32, sizeof(float2) * N);
  RB_ALLOC(d_bad, sizeof(int));
  HostBuf h;
  const size_t h_bytes = sizeof(ArgMax) * kTop + sizeof(double) * 2 * kTop + sizeof(int64_t) * kTop + 64;
  if (h.alloc(h_bytes) != hipSuccess) return set_error(RB_ENOMEM, "pinned host allocation failed");
  ArgMax* h_top = h.as<ArgMax>();
  double* h_sq = reinterpret_cast<double*>(h_top + kTop);
  int64_t* h_cols = reinterpret_cast<int64_t*>(h_sq + 2 * kTop);
  int* h_bad = reinterpret_cast<int*>(h_cols + kTop);

  double* nrm = d_nrm.as<double>();
  double* acc = d_acc.as<double>();
  uint8_t* mask = d_mask.as<uint8_t>();
  ArgMax* part = d_part.as<ArgMax>();
  ArgMax* top = d_top.as<ArgMax>();
  double2* cpan = d_cpan.as<double2>();
  double2* V = d_V.as<double2>();
  double2* G = d_G.as<double2>();
  double* sq = d_sq.as<double>();
  int64_t* cols = d_cols.as<int64_t>();
  float2* e32 = d_e32.as<float2>();

  const float2* X32 = S32;  // working matrix: S32 until the first anchoring
  int64_t ldX = ldS;
  float2* W32 = static_cast<float2*>(W32_);
  int64_t ldWk = ldW;

  // ---- initial norms and candidates ----
  tm.start();
  RB_HIP(hipMemsetAsync(d_bad.p, 0, sizeof(int), stream));
  RB_HIP(launch_colnorms_c(S32, N, M, ldS, nrm, d_bad.as<int>(), stream));
  RB_HIP(hipMemsetAsync(acc, 0, sizeof(double) * M, stream));
  RB_HIP(hipMemsetAsync(mask, 0, M, stream));
  RB_HIP(launch_est_topk(nrm, nullptr, mask, M, part, np, top, stream));
  RB_HIP(hipMemcpyAsync(h_bad, d_bad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipMemcpyAsync(h_top, top, sizeof(ArgMax) * kTop, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  tm.stop(&st.ms_anchor);
  if (*h_bad) return set_error(RB_ENONFINITE, "rb_greedy_c: S holds a non-finite value");
  double A_w = h_top[0].v > 0.0 ? h_top[0].v : 0.0;
  double P = 0.5 * kDelta32 * std::sqrt(A_w);  // perturbation bound of the stored columns

  int64_t k = 0, a = 0, m = 0;
  int status = RB_KMAX;

  // ---- confirmation of the candidates in h_top against E[:, 0:k] ----
  int64_t Jbest = -1;
  double rbest = 0.0;
  int slot = 0, passes = 0;
  bool rank_flag = false;
  const double* sq_final = sq;
  auto confirm = [&](int64_t kcur) -> int {
    tm.start();
    int nv = 0;
    for (int r = 0; r < kTop; ++r)
      if (h_top[r].i >= 0) h_cols[nv++] = h_top[r].i;
    Jbest = -1;
    rbest = 0.0;
    rank_flag = false;
    if (nv == 0) {
      tm.stop(&st.ms_gs);
      return RB_OK;
    }
    RB_HIP(hipMemcpyAsync(cols, h_cols, sizeof(int64_t) * nv, hipMemcpyHostToDevice, stream));
    if (regen(regen_ctx, cols, nv, V, N, stream) != 0)
      return set_error(RB_EDEVICE, "rb_greedy_c: regeneration callback failed");
    RB_HIP(launch_sqnorms_small(V, N, nv, N, sq, stream));
    RB_HIP(hipMemcpyAsync(h_sq, sq, sizeof(double) * nv, hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    double orig[kTop], before[kTop], after[kTop];
    for (int r = 0; r < nv; ++r) orig[r] = before[r] = after[r] = std::sqrt(h_sq[r]);
    sq_final = sq;
    passes = 1;
    if (kcur > 0) {
      passes = 0;
      while (passes < o.nu_max) {
        RB_HIP(launch_gemv_ch(E, ldE, kcur, V, N, nv, N, G, stream));
        RB_HIP(launch_gemv_n_sub(E, ldE, kcur, G, V, N, nv, N, stream));
        RB_HIP(launch_sqnorms_small(V, N, nv, N, sq + kTop, stream));
        RB_HIP(hipMemcpyAsync(h_sq + kTop, sq + kTop, sizeof(double) * nv, hipMemcpyDeviceToHost, stream));
        RB_HIP(hipStreamSynchronize(stream));
        ++passes;
        bool all_ok = true;
        for (int r = 0; r < nv; ++r) {
          after[r] = std::sqrt(h_sq[kTop + r]);
          if (!(after[r] > before[r] / o.kappa)) all_ok = false;
        }
        if (passes >= o.nu_min && all_ok) break;
        for (int r = 0; r < nv; ++r) before[r] = after[r];
      }
      sq_final = sq + kTop;
    }
    st.gs_passes += passes;
    int b = 0;
    for (int r = 1; r < nv; ++r)
      if (after[r] > after[b] || (after[r] == after[b] && h_cols[r] < h_cols[b])) b = r;
    slot = b;
    Jbest = h_cols[b];
    rbest = after[b];
    rank_flag = !(rbest > 64.0 * 0x1p-53 * orig[b]);
    tm.stop(&st.ms_gs);
    return RB_OK;
  };

  // ---- re-anchoring ----
  auto ensure_w = [&]() -> int {
    if (!W32) {
      RB_ALLOC(d_Wown, sizeof(float2) * (size_t)N * (size_t)M);
      W32 = d_Wown.as<float2>();
      ldWk = N;
    }
    return RB_OK;
  };
  auto anchor = [&](bool exact) -> int {
    tm.start();
    int rc = ensure_w();
    if (rc != RB_OK) return rc;
    if (exact) {
      if (!d_S64c.p) {
        RB_ALLOC(d_S64c, sizeof(double2) * (size_t)N * (size_t)chunk);
        RB_ALLOC(d_Cc, sizeof(double2) * (size_t)(kcap > 0 ? kcap : 1) * (size_t)chunk);
        RB_ALLOC(d_iota, sizeof(int64_t) * (size_t)chunk);
      }
      double2* S64c = d_S64c.as<double2>();
      double2* Cc = d_Cc.as<double2>();
      int64_t* iota = d_iota.as<int64_t>();
      for (int64_t c0 = 0; c0 < M; c0 += chunk) {
        const int64_t mc = (M - c0 < chunk) ? M - c0 : chunk;
        RB_HIP(launch_iota(iota, c0, mc, stream));
        if (regen(regen_ctx, iota, mc, S64c, N, stream) != 0)
          return set_error(RB_EDEVICE, "rb_greedy_c: regeneration callback failed");
        if (k > 0) RB_HIP(launch_project_z(E, N, k, ldE, S64c, mc, N, Cc, k, stream));
        RB_HIP(launch_resid(S64c, N, W32 + c0 * ldWk, ldWk, N, mc, E, ldE, k, Cc, 1, k, nrm + c0,
                            d_bad.as<int>(), stream));
      }
      st.regen_anchors++;
    } else {
      RB_HIP(launch_resid(X32, ldX, W32, ldWk, N, M, E + a * ldE, ldE, m, cpan, M, 1, nrm, d_bad.as<int>(),
                          stream));
    }
    X32 = W32;
    ldX = ldWk;
    RB_HIP(hipMemsetAsync(acc, 0, sizeof(double) * M, stream));
    RB_HIP(launch_est_topk(nrm, nullptr, mask, M, part, np, top, stream));
    RB_HIP(hipMemcpyAsync(h_top, top, sizeof(ArgMax) * kTop, hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    tm.stop(&st.ms_anchor);
    a = k;
    m = 0;
    A_w = h_top[0].v > 0.0 ? h_top[0].v : 0.0;
    const double sig = std::sqrt(A_w);
    P = exact ? 0.5 * kDelta32 * sig : P + kDelta32 * sig;
    st.anchors++;
    return RB_OK;
  };
  auto choose_exact = [&](double sigma) -> bool {
    const double budget = 0.1 * tol;
    if (P + kDelta32 * sigma <= budget) return false;  // deflation error stays negligible
    if (kDelta32 * sigma > budget) return false;       // a later anchoring comes before tol
    return true;
  };

  int rc = confirm(0);
  if (rc != RB_OK) return rc;
  err[0] = (Jbest >= 0) ? rbest : 0.0;
  bool certified = false;

  // Bound on |est_j - true residual_j^2| for the stored columns since the
  // last anchoring: FP32 coefficients (|dc| <= 9 u32 ||x_j||, so the m
  // accumulated |c|^2 terms are off by <= 18 sqrt(m) u32 nrm_j) plus the
  // stored-column perturbation P (|d ||r||^2| <= 2 ||r|| P + P^2).
  auto est_bound = [&](double est) -> double {
    const double u32 = 0x1p-24;
    const double r = std::sqrt(est > 0.0 ? est : 0.0);
    return 18.0 * std::sqrt((double)(m > 0 ? m : 1)) * u32 * A_w + 2.0 * r * P + P * P;
  };

  while (true) {
    if (err[k] < tol) {
      // certify == 2: the sweep's largest estimate already bounds every
      // column's true residual below tol
      const bool bounded_ok = o.certify == 2 && h_top[0].i >= 0 &&
                              h_top[0].v + est_bound(h_top[0].v) < tol * tol;
      if (o.certify && !certified && !bounded_ok && k < kcap && Jbest >= 0) {
        rc = anchor(true);
        if (rc != RB_OK) return rc;
        certified = true;
        rc = confirm(k);
        if (rc != RB_OK) return rc;
        err[k] = (Jbest >= 0) ? rbest : 0.0;
        continue;
      }
      status = RB_OK;
      break;
    }
    if (k == kcap || Jbest < 0) break;
    if (rank_flag) {
      status = RB_RANK;
      break;
    }
    // ---- 1. the confirmed candidate becomes e_k ----
    tm.start();
    RB_HIP(launch_scale_into(V + slot * N, N, sq_final + slot, E + k * ldE, stream));
    RB_HIP(launch_round32(E + k * ldE, N, e32, stream));
    RB_HIP(hipMemsetAsync(mask + Jbest, 1, 1, stream));
    tm.stop(&st.ms_gs);
    piv[k] = Jbest;
    rho[k] = rbest;
    if (nu) nu[k] = passes;
    ++k;
    certified = false;

    // ---- 2. complex64 sweep with the FP32 copy (panel row m) ----
    if (m == panel) {
      rc = anchor(choose_exact(rbest));
      if (rc != RB_OK) return rc;
      a = k - 1;  // the new vector has not been swept yet
    }
    tm.start();
    RB_HIP(launch_sweep_c(X32, N, M, ldX, e32, nrm, acc, mask, cpan + m * M, 1, part, np, nullptr, stream));
    tm.stop(&st.ms_sweep);  // the sweep kernel alone
    RB_HIP(launch_sweep_c_final(M, part, top, stream));
    RB_HIP(hipMemcpyAsync(h_top, top, sizeof(ArgMax) * kTop, hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    st.sweeps++;
    ++m;
    if (h_top[0].i >= 0 && h_top[0].v < o.theta32 * A_w) {
      rc = anchor(choose_exact(std::sqrt(h_top[0].v > 0.0 ? h_top[0].v : 0.0)));
      if (rc != RB_OK) return rc;
    }
    // ---- 3. FP64 confirmation of the candidates ----
    const int64_t top1 = h_top[0].i;
    rc = confirm(k);
    if (rc != RB_OK) return rc;
    if (Jbest >= 0 && Jbest != top1) st.misses++;
    err[k] = (Jbest >= 0) ? rbest : 0.0;
  }
  if (status == RB_KMAX && err[k] < tol) status = RB_OK;
  *k_out = k;
  st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
  if (stats) *stats = st;
  return status;
}

}  // extern "C"

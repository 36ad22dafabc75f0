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
#include <algorithm>
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

}  // extern "C"

namespace {

// Device scratch of the mixed greedy, carved from one workspace: the part
// every run uses, and the exact re-anchoring's regeneration chunk.
struct CScratch {
  double *nrm, *acc, *sq;
  uint8_t* mask;
  ArgMax *part, *top;
  double2 *cpan, *V, *G;
  int64_t* cols;
  float2* e32;  // the sweep's FP32 vector, then (lookahead) the predicted ones, N apart
  int* bad;
  // pivot lookahead: candidate list, list-local sums, rerank partials, predicted top-8
  ArgMax *list = nullptr, *rpart = nullptr, *ptop = nullptr, *coarse = nullptr;
  double* acc_l = nullptr;
  size_t carve(void* base, int64_t N, int64_t M, int64_t kcap, int64_t panel, int look_k) {
    Carve c(base);
    nrm = c.take<double>(M);
    acc = c.take<double>(M);
    mask = c.take<uint8_t>(M);
    part = c.take<ArgMax>(sweep32_partials_needed(M));
    top = c.take<ArgMax>(kTop);
    cpan = c.take<double2>((size_t)panel * (size_t)M);
    V = c.take<double2>((size_t)N * kTop);
    G = c.take<double2>((size_t)(kcap > 0 ? kcap : 1) * kTop);
    sq = c.take<double>(2 * kTop);
    cols = c.take<int64_t>(kTop);
    e32 = c.take<float2>((size_t)N * (look_k > 0 ? 1 + kLookMax : 1));
    bad = c.take<int>(1);
    if (look_k > 0) {
      list = c.take<ArgMax>(look_k);
      acc_l = c.take<double>(look_k);
      rpart = c.take<ArgMax>(rerank32_partials(look_k));
      ptop = c.take<ArgMax>(kTop);
      const int64_t nc = look_list_scratch((M + 15) / 16);
      if (nc > 0) coarse = c.take<ArgMax>(nc);
    }
    return c.used;
  }
};
struct CRegen {
  double2 *S64c, *Cc;
  int64_t* iota;
  size_t carve(void* base, int64_t N, int64_t kcap, int64_t chunk) {
    Carve c(base);
    S64c = c.take<double2>((size_t)N * (size_t)chunk);
    Cc = c.take<double2>((size_t)(kcap > 0 ? kcap : 1) * (size_t)chunk);
    iota = c.take<int64_t>(chunk);
    return c.used;
  }
};

bool c_opts_ok(const rb_opts& o) {
  return o.kappa > 1.0 && o.nu_max >= 1 && o.nu_min >= 1 && o.nu_min <= o.nu_max && o.theta32 > 0.0 &&
         o.theta32 < 1.0 && o.anchor_max >= 1 && o.regen_chunk >= 1 && o.lookahead32 >= -1 &&
         o.lookahead32 <= kLookMax && (o.lookahead32 == 0 || (o.look_k >= 1 && o.look_k <= kLookListMax));
}
// the mixed greedy's prediction depth (lookahead32 = -1: by the column count)
int c_depth(const rb_opts& o, int64_t M) { return o.lookahead32 >= 0 ? o.lookahead32 : (M < 1000000 ? 2 : 5); }
int c_look_k(const rb_opts& o) { return o.lookahead32 != 0 ? o.look_k : 0; }

// both parts, 256-byte aligned one after the other
size_t c_ws_bytes(int64_t N, int64_t M, int64_t kcap, const rb_opts& o, size_t* base_bytes) {
  CScratch c;
  CRegen r;
  const int64_t chunk = o.regen_chunk < M ? o.regen_chunk : M;
  const size_t b = (c.carve(nullptr, N, M, kcap, o.anchor_max, c_look_k(o)) + 255) & ~static_cast<size_t>(255);
  if (base_bytes) *base_bytes = b;
  return b + r.carve(nullptr, N, kcap, chunk);
}

}  // namespace

extern "C" {

size_t rb_greedy_c_workspace(int64_t N, int64_t M, int64_t kmax, const rb_opts* opts_in) {
  rb_opts o;
  rb_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (N <= 0 || M <= 0 || kmax < 0 || !c_opts_ok(o)) return 0;
  return c_ws_bytes(N, M, std::min(std::min(kmax, N), M), o, nullptr);
}

int rb_greedy_c(const void* S32_, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax, rb_regen_fn regen,
                void* regen_ctx, void* W32_, int64_t ldW, void* E_, int64_t ldE, int64_t* piv, double* err,
                double* rho, int32_t* nu, int64_t* k_out, void* ws, size_t ws_bytes, const rb_opts* opts_in,
                rb_stats* stats, hipStream_t stream) {
  last_error().clear();
  const auto t_begin = std::chrono::steady_clock::now();
  rb_opts o;
  rb_default_opts(&o);
  if (opts_in) o = *opts_in;
  auto fail = [&](int code, const char* what) { return set_error(code, "rb_greedy_c: %s", what); };
  if (!S32_ || N <= 0 || M <= 0 || !valid_ld(N, ldS) || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol) ||
      !piv || !err || !rho || !k_out || !regen)
    return fail(RB_EINVAL, "bad arguments");
  if (kmax > 0 && (!E_ || !valid_ld(N, ldE))) return fail(RB_EINVAL, "bad basis buffer");
  if (W32_ && !valid_ld(N, ldW)) return fail(RB_EINVAL, "bad working-matrix leading dimension");
  if (W32_ == S32_ && W32_ && ldW != ldS) return fail(RB_EINVAL, "W32 == S32 needs ldW == ldS");
  if (!c_opts_ok(o)) return fail(RB_EINVAL, "bad options");
  if (ws && !W32_) return fail(RB_EINVAL, "a caller workspace needs a working matrix W32 (W32 may be S32)");
  if (ws && reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(RB_EINVAL, "workspace not 256-byte aligned");

  const float2* S32 = static_cast<const float2*>(S32_);
  double2* E = static_cast<double2*>(E_);
  int64_t kcap = kmax;
  if (kcap > N) kcap = N;
  if (kcap > M) kcap = M;
  const int64_t panel = o.anchor_max;
  const int64_t np = sweep32_partials_needed(M);
  const int64_t chunk = o.regen_chunk < M ? o.regen_chunk : M;

  // scratch: the caller's workspace (both parts), or an allocation of the
  // base part now and of the regeneration part at the first exact anchoring
  CScratch z;
  CRegen rg = {nullptr, nullptr, nullptr};
  size_t base_bytes = 0;
  const size_t need = c_ws_bytes(N, M, kcap, o, &base_bytes);
  DevBuf d_ws, d_regen, d_Wown;
  if (ws) {
    if (ws_bytes < need) {
      char m[160];
      std::snprintf(m, sizeof m, "workspace of %zu bytes, %zu needed", ws_bytes, need);
      return fail(RB_ENOMEM, m);
    }
    z.carve(ws, N, M, kcap, panel, c_look_k(o));
    rg.carve(static_cast<char*>(ws) + base_bytes, N, kcap, chunk);
  } else {
    RB_ALLOC(d_ws, base_bytes);
    z.carve(d_ws.p, N, M, kcap, panel, c_look_k(o));
  }
  HostWords hw;
  const size_t h_bytes = sizeof(ArgMax) * kTop + sizeof(double) * 2 * kTop + sizeof(int64_t) * kTop + 64;
  if (hw.init(d_ws.p != nullptr, h_bytes) != hipSuccess) return fail(RB_ENOMEM, "pinned host allocation failed");
  ArgMax* h_top = hw.at<ArgMax>(0);
  double* h_sq = reinterpret_cast<double*>(h_top + kTop);
  int64_t* h_cols = reinterpret_cast<int64_t*>(h_sq + 2 * kTop);
  int* h_bad = reinterpret_cast<int*>(h_cols + kTop);

  rb_stats st;
  std::memset(&st, 0, sizeof st);
  EventTimer tm(o.collect_stats != 0, stream);
  double* step_ms = (tm.on && o.step_ms) ? o.step_ms : nullptr;
  auto slot = [&](int64_t i, int part) -> double* {
    return (step_ms && i <= kcap) ? step_ms + 3 * i + part : nullptr;
  };

  double* nrm = z.nrm;
  double* acc = z.acc;
  uint8_t* mask = z.mask;
  ArgMax* part = z.part;
  ArgMax* top = z.top;
  double2* cpan = z.cpan;
  double2* V = z.V;
  double2* G = z.G;
  double* sq = z.sq;
  int64_t* cols = z.cols;
  float2* e32 = z.e32;

  const float2* X32 = S32;  // working matrix: S32 until the first anchoring
  int64_t ldX = ldS;
  float2* W32 = static_cast<float2*>(W32_);
  int64_t ldWk = ldW;

  // ---- initial norms and candidates ----
  tm.start();
  RB_HIP(launch_fill(z.bad, 0, 1, stream));
  RB_HIP(launch_colnorms_c(S32, N, M, ldS, nrm, z.bad, stream));
  RB_HIP(launch_fill(acc, 0.0, M, stream));
  RB_HIP(launch_fill(mask, (uint8_t)0, M, stream));
  RB_HIP(launch_est_topk(nrm, nullptr, mask, M, part, np, top, stream));
  RB_HIP(hipMemcpyAsync(h_bad, z.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  RB_HIP(hipMemcpyAsync(h_top, top, sizeof(ArgMax) * kTop, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  lap(tm, &st.ms_anchor, nullptr);
  if (*h_bad) return fail(RB_ENONFINITE, "S holds a non-finite value");
  double A_w = h_top[0].v > 0.0 ? h_top[0].v : 0.0;
  double P = 0.5 * kDelta32 * std::sqrt(A_w);  // perturbation bound of the stored columns

  int64_t k = 0, a = 0, m = 0;
  int status = RB_KMAX;
  auto fail_run = [&](int code, const char* what) {
    char m2[200];
    std::snprintf(m2, sizeof m2, "%s (after %lld basis vectors)", what, (long long)k);
    *k_out = k;
    if (stats) *stats = st;
    return fail(code, m2);
  };

  // ---- confirmation of the candidates in h_top against E[:, 0:k] ----
  int64_t Jbest = -1;
  double rbest = 0.0;
  int slot_b = 0, passes = 0;
  bool rank_flag = false, settled_b = true;
  const double* sq_final = sq;
  // slot_ms: where the confirmation's time goes (the vector it chooses)
  // spec: a predicted set (rb_look.hip's lookahead): a non-finite candidate
  // ends the prediction instead of the run, and the time and passes count
  // as prediction
  auto confirm = [&](int64_t kcur, double* slot_ms, bool spec = false) -> int {
    tm.start();
    int nv = 0;
    for (int r = 0; r < kTop; ++r)
      if (h_top[r].i >= 0) h_cols[nv++] = h_top[r].i;
    Jbest = -1;
    rbest = 0.0;
    rank_flag = false;
    settled_b = true;
    if (nv == 0) {
      lap(tm, spec ? &st.ms_look : &st.ms_gs, slot_ms);
      return RB_OK;
    }
    RB_HIP(hipMemcpyAsync(cols, h_cols, sizeof(int64_t) * nv, hipMemcpyHostToDevice, stream));
    if (regen(regen_ctx, cols, nv, V, N, stream) != 0) return fail_run(RB_EDEVICE, "regeneration callback failed");
    RB_HIP(launch_sqnorms_small(V, N, nv, N, sq, stream));
    RB_HIP(hipMemcpyAsync(h_sq, sq, sizeof(double) * nv, hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    double orig[kTop], before[kTop], after[kTop];
    bool settled[kTop];
    for (int r = 0; r < nv; ++r) {
      orig[r] = before[r] = after[r] = std::sqrt(h_sq[r]);
      settled[r] = true;
      if (!std::isfinite(orig[r])) {
        if (spec) {
          lap(tm, &st.ms_look, nullptr);
          return RB_OK;  // Jbest < 0: no prediction
        }
        return fail_run(RB_ENONFINITE, "a regenerated candidate is not finite");
      }
    }
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
          settled[r] = after[r] > before[r] / o.kappa;
          if (!settled[r]) all_ok = false;
        }
        if (passes >= o.nu_min && all_ok) break;
        for (int r = 0; r < nv; ++r) before[r] = after[r];
      }
      sq_final = sq + kTop;
    }
    if (spec) {
      st.look_gs++;
    } else {
      st.gs_passes += passes;
    }
    for (int r = 0; r < nv; ++r)
      if (!std::isfinite(after[r])) {
        if (spec) {
          lap(tm, &st.ms_look, nullptr);
          return RB_OK;
        }
        return fail_run(RB_ENONFINITE, "an orthogonalised candidate is not finite");
      }
    int b = 0;
    for (int r = 1; r < nv; ++r)
      if (after[r] > after[b] || (after[r] == after[b] && h_cols[r] < h_cols[b])) b = r;
    slot_b = b;
    Jbest = h_cols[b];
    rbest = after[b];
    settled_b = settled[b];
    rank_flag = !(rbest > 64.0 * 0x1p-53 * orig[b]);
    lap(tm, spec ? &st.ms_look : &st.ms_gs, slot_ms);
    return RB_OK;
  };

  // ---- pivot lookahead (rb_look.hip): predictions spec[spec_at .. nspec)
  // made at the last sweep, each with its predicted top-8 set, the outcome
  // of confirming that set, its vector in E[:, k + d] and its coefficients
  // in panel row m + d.  A step takes a prediction when the top-8 set of
  // the estimates equals the predicted one: its confirmation, which
  // depends on nothing else, then gives the same pivot and vector. ----
  struct Spec32 {
    int64_t top[kTop];
    int64_t J;
    double r;
    int passes;
    bool settled, rank;
  };
  Spec32 spec[kLookMax];
  int nspec = 0, spec_at = 0;
  bool taken = false;  // the step about to start was predicted
  const int look_k = c_look_k(o);
  const int64_t ngroups = (M + 15) / 16;

  // ---- re-anchoring ----
  auto ensure_w = [&]() -> int {
    if (!W32) {
      RB_ALLOC(d_Wown, sizeof(float2) * (size_t)N * (size_t)M);
      W32 = d_Wown.as<float2>();
      ldWk = N;
    }
    return RB_OK;
  };
  auto anchor = [&](bool exact, double* slot_ms) -> int {
    nspec = spec_at = 0;
    taken = false;
    tm.start();
    int rc = ensure_w();
    if (rc != RB_OK) return rc;
    if (exact) {
      if (!rg.S64c) {
        const size_t rb = rg.carve(nullptr, N, kcap, chunk);
        RB_ALLOC(d_regen, rb);
        rg.carve(d_regen.p, N, kcap, chunk);
      }
      for (int64_t c0 = 0; c0 < M; c0 += chunk) {
        const int64_t mc = (M - c0 < chunk) ? M - c0 : chunk;
        RB_HIP(launch_iota(rg.iota, c0, mc, stream));
        if (regen(regen_ctx, rg.iota, mc, rg.S64c, N, stream) != 0)
          return fail_run(RB_EDEVICE, "regeneration callback failed");
        if (k > 0) RB_HIP(launch_project_z(E, N, k, ldE, rg.S64c, mc, N, rg.Cc, k, stream));
        RB_HIP(launch_resid(rg.S64c, N, W32 + c0 * ldWk, ldWk, N, mc, E, ldE, k, rg.Cc, 1, k, nrm + c0, z.bad,
                            stream));
      }
      st.regen_anchors++;
    } else {
      RB_HIP(launch_resid(X32, ldX, W32, ldWk, N, M, E + a * ldE, ldE, m, cpan, M, 1, nrm, z.bad, stream));
    }
    X32 = W32;
    ldX = ldWk;
    RB_HIP(launch_fill(acc, 0.0, M, stream));
    RB_HIP(launch_est_topk(nrm, nullptr, mask, M, part, np, top, stream));
    RB_HIP(hipMemcpyAsync(h_top, top, sizeof(ArgMax) * kTop, hipMemcpyDeviceToHost, stream));
    RB_HIP(hipMemcpyAsync(h_bad, z.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    RB_HIP(hipStreamSynchronize(stream));
    lap(tm, &st.ms_anchor, slot_ms);
    st.anchors++;
    if (*h_bad) return fail_run(RB_ENONFINITE, "a re-anchored column is not finite");
    a = k;
    m = 0;
    A_w = h_top[0].v > 0.0 ? h_top[0].v : 0.0;
    const double sig = std::sqrt(A_w);
    P = exact ? 0.5 * kDelta32 * sig : P + kDelta32 * sig;
    return RB_OK;
  };
  auto choose_exact = [&](double sigma) -> bool {
    const double budget = 0.1 * tol;
    if (P + kDelta32 * sigma <= budget) return false;  // deflation error stays negligible
    if (kDelta32 * sigma > budget) return false;       // a later anchoring comes before tol
    return true;
  };
  // the confirmed candidate's Gram-Schmidt must have settled unless its
  // residual is already below tol
  auto check_breakdown = [&]() -> int {
    if (Jbest >= 0 && !rank_flag && !settled_b && rbest >= tol) {
      char m2[160];
      std::snprintf(m2, sizeof m2, "Gram-Schmidt of candidate %lld still shrank ||v|| by kappa after %d passes",
                    (long long)Jbest, passes);
      return fail_run(RB_EBREAKDOWN, m2);
    }
    return RB_OK;
  };

  // Predict the next dmax steps before the sweep with e32 (E[:, k-1]): the
  // top-8 of the listed columns after reranking with the newest FP32 vector
  // (then with each predicted one), confirmed in FP64 against E[:, 0..k+d-1]
  // exactly as its step would confirm it; the chosen vector goes to
  // E[:, k + d] and its FP32 copy to e32 + (d + 1) N.  A prediction its step
  // would not accept ends the chain.  Returns the number made.
  auto predict = [&](int dmax, int* nd_out) -> int {
    *nd_out = 0;
    tm.start();
    RB_HIP(launch_est_apply(nrm, acc, mask, nullptr, M, part, np, stream));
    RB_HIP(launch_look_list(part, ngroups, look_k, z.list, z.coarse, stream));
    lap(tm, &st.ms_look, nullptr);
    int64_t ex[kLookMax];
    int nd = 0;
    for (int d = 0; d < dmax; ++d) {
      tm.start();
      RB_HIP(launch_rerank32(X32, N, ldX, e32 + d * N, z.list, look_k, nrm, acc, z.acc_l, d == 0 ? 1 : 0, mask, ex, d,
                             z.rpart, z.ptop, stream));
      RB_HIP(hipMemcpyAsync(h_top, z.ptop, sizeof(ArgMax) * kTop, hipMemcpyDeviceToHost, stream));
      RB_HIP(hipStreamSynchronize(stream));
      lap(tm, &st.ms_look, nullptr);
      if (h_top[0].i < 0 || std::isnan(h_top[0].v)) break;
      int rc2 = confirm(k + d, nullptr, true);
      if (rc2 != RB_OK) return rc2;
      if (Jbest < 0 || rank_flag || (!settled_b && rbest >= tol)) break;
      tm.start();
      RB_HIP(launch_scale_into(V + slot_b * N, N, sq_final + slot_b, E + (k + d) * ldE, stream));
      RB_HIP(launch_round32(E + (k + d) * ldE, N, e32 + (d + 1) * N, stream));
      lap(tm, &st.ms_look, nullptr);
      Spec32& sp = spec[d];
      for (int r = 0; r < kTop; ++r) sp.top[r] = h_top[r].i;
      sp.J = Jbest;
      sp.r = rbest;
      sp.passes = passes;
      sp.settled = settled_b;
      sp.rank = rank_flag;
      ex[d] = Jbest;
      nd = d + 1;
    }
    *nd_out = nd;
    return RB_OK;
  };
  auto same_top = [&](const Spec32& sp) -> bool {
    for (int r = 0; r < kTop; ++r)
      if (h_top[r].i != sp.top[r]) return false;
    return true;
  };

  int rc = confirm(0, slot(0, 0));
  if (rc != RB_OK) return rc;
  err[0] = (Jbest >= 0) ? rbest : 0.0;
  bool certified = false;

  // Bound on |est_j - true residual_j^2| for the stored columns since the
  // last anchoring.  The complex64 sweep sums, per lane and row tile, 8
  // complex products (16 real ones per component) in FP32 with the FP32
  // copy e32 of a unit vector, then adds the partials in FP64.  Per
  // component the error is at most (gamma_16 + u32 (1 + gamma_16)) times
  // sum_n |e_n| |x_n| <= ||x_j|| (Cauchy-Schwarz, ||e|| = 1), just over
  // 17 u32 ||x_j||, so |dc| <= 17 sqrt(2) u32 ||x_j|| < 25 u32 ||x_j||; the m
  // accumulated |c|^2 terms are off by at most sum (2 |c_i| |dc_i| +
  // |dc_i|^2) <= 50 sqrt(m) u32 nrm_j + 625 m u32^2 nrm_j <= 51 sqrt(m) u32
  // nrm_j (m <= anchor_max).  Plus the stored-column perturbation P
  // (|d ||r||^2| <= 2 ||r|| P + P^2).
  auto est_bound = [&](double est) -> double {
    const double u32 = 0x1p-24;
    const double r = std::sqrt(est > 0.0 ? est : 0.0);
    return 51.0 * std::sqrt((double)(m > 0 ? m : 1)) * u32 * A_w + 2.0 * r * P + P * P;
  };

  while (true) {
    if (err[k] < tol) {
      // certify == 2: the sweep's largest estimate already bounds every
      // column's true residual below tol
      const bool bounded_ok = o.certify == 2 && h_top[0].i >= 0 &&
                              h_top[0].v + est_bound(h_top[0].v) < tol * tol;
      if (o.certify && !certified && !bounded_ok && k < kcap && Jbest >= 0) {
        rc = anchor(true, slot(k > 0 ? k - 1 : 0, 2));
        if (rc != RB_OK) return rc;
        certified = true;
        rc = confirm(k, slot(k, 0));
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
    rc = check_breakdown();
    if (rc != RB_OK) return rc;
    // ---- 1. the confirmed candidate becomes e_k (a predicted one is there already) ----
    tm.start();
    bool step_taken = taken;
    taken = false;
    if (!step_taken) {
      RB_HIP(launch_scale_into(V + slot_b * N, N, sq_final + slot_b, E + k * ldE, stream));
      RB_HIP(launch_round32(E + k * ldE, N, e32, stream));
    }
    RB_HIP(launch_fill(mask + Jbest, (uint8_t)1, 1, stream));
    lap(tm, &st.ms_gs, slot(k, 0));
    piv[k] = Jbest;
    rho[k] = rbest;
    if (nu) nu[k] = passes;
    ++k;
    certified = false;

    // ---- 2. complex64 sweep with the FP32 copy (panel row m) ----
    bool apply_taken = step_taken;
    if (m == panel) {
      rc = anchor(choose_exact(rbest), slot(k - 1, 2));
      if (rc != RB_OK) return rc;
      a = k - 1;  // the new vector has not been swept yet
      apply_taken = false;
    }
    if (apply_taken) {
      // its coefficients are panel row m already
      tm.start();
      RB_HIP(launch_est_apply32(nrm, acc, mask, cpan + m * M, M, part, np, top, stream));
      RB_HIP(hipMemcpyAsync(h_top, top, sizeof(ArgMax) * kTop, hipMemcpyDeviceToHost, stream));
      RB_HIP(hipStreamSynchronize(stream));
      lap(tm, &st.ms_apply, slot(k - 1, 1));
      st.look_steps++;
      ++m;
    } else {
      if (step_taken) {  // a re-anchoring came in between: sweep with its FP32 copy
        RB_HIP(launch_round32(E + (k - 1) * ldE, N, e32, stream));
      }
      nspec = spec_at = 0;
      int64_t dmax = 0;
      if (look_k > 0 && sweep_c_look_ok(X32, ldX, e32, N))
        dmax = std::min<int64_t>(std::min<int64_t>(c_depth(o, M), panel - m - 1), kcap - k);
      int nd = 0;
      if (dmax > 0) {
        rc = predict((int)dmax, &nd);
        if (rc != RB_OK) return rc;
      }
      tm.start();
      if (nd > 0)
        RB_HIP(launch_sweep_c_look(X32, N, M, ldX, e32, N, 1 + nd, nrm, acc, mask, cpan + m * M, part, np, nullptr,
                                   stream));
      else
        RB_HIP(launch_sweep_c(X32, N, M, ldX, e32, nrm, acc, mask, cpan + m * M, 1, part, np, nullptr, stream));
      const double ms_before = st.ms_sweep;
      lap(tm, &st.ms_sweep, slot(k - 1, 1));  // the sweep kernel alone
      if (nd > 0) {
        st.ms_look_sweep += st.ms_sweep - ms_before;
        st.look_sweeps++;
        st.look_vectors += nd;
      }
      RB_HIP(launch_sweep_c_final(M, part, top, stream));
      RB_HIP(hipMemcpyAsync(h_top, top, sizeof(ArgMax) * kTop, hipMemcpyDeviceToHost, stream));
      RB_HIP(hipStreamSynchronize(stream));
      st.sweeps++;
      ++m;
      nspec = nd;
      spec_at = 0;
    }
    if (h_top[0].i >= 0 && std::isnan(h_top[0].v)) return fail_run(RB_ENONFINITE, "a swept estimate is not finite");
    if (h_top[0].i >= 0 && h_top[0].v < o.theta32 * A_w) {
      rc = anchor(choose_exact(std::sqrt(h_top[0].v > 0.0 ? h_top[0].v : 0.0)), slot(k - 1, 2));
      if (rc != RB_OK) return rc;
    }
    // ---- 3. FP64 confirmation of the candidates (or the predicted one's) ----
    const int64_t top1 = h_top[0].i;
    if (spec_at < nspec && same_top(spec[spec_at])) {
      const Spec32& sp = spec[spec_at++];
      Jbest = sp.J;
      rbest = sp.r;
      passes = sp.passes;
      settled_b = sp.settled;
      rank_flag = sp.rank;
      st.gs_passes += passes;
      taken = true;
    } else {
      nspec = spec_at = 0;
      rc = confirm(k, slot(k, 0));
      if (rc != RB_OK) return rc;
    }
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

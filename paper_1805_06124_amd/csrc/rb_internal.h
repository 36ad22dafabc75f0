// Internal declarations shared by the HIP translation units of librb.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rb.h"

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

// ------------------------------------------------------------------ host --

// Device argmax result record.
struct ArgMax {
  double v;
  int64_t i;
};

// Candidates kept by the mixed-precision sweep for FP64 confirmation.
constexpr int kTop = 8;

// launchers (each defined in the translation unit that holds the kernel)
hipError_t launch_colnorms_z(const double2* S, int64_t N, int64_t M, int64_t ldS, double* nrm, int* bad,
                             hipStream_t s);
hipError_t launch_colnorms_c(const float2* S, int64_t N, int64_t M, int64_t ldS, double* nrm, int* bad,
                             hipStream_t s);
hipError_t launch_sweep_z(const double2* S, int64_t N, int64_t M, int64_t ldS, const double2* e,
                          const double* nrm, double* acc, const uint8_t* mask, double2* c_out, int64_t ldc,
                          ArgMax* partial, int64_t npartial_cap, ArgMax* result, hipStream_t s);
// result == NULL: only the per-workgroup partials; launch_sweep_final then
// reduces them (lets the host time the sweep kernel alone)
hipError_t launch_sweep_final(int64_t M, const ArgMax* partial, ArgMax* result, hipStream_t s);
hipError_t launch_est_argmax(const double* nrm, const double* acc, const uint8_t* mask, int64_t M,
                             ArgMax* partial, int64_t npartial_cap, ArgMax* result, hipStream_t s);
int64_t sweep_partials_needed(int64_t M);
// the final reduction alone, over n partial records
hipError_t launch_argmax_records(const ArgMax* partial, int64_t n, ArgMax* result, hipStream_t s);

// Pivot lookahead of the FP64 greedy (rb_look.hip).  The sweep kernels keep
// one partial argmax per kPivotGroup consecutive columns.
//   launch_sweep_look: the sweep with V = 1 + d vectors E[:, 0..V-1] (d <=
//     kLookMax predicted ones): vector 0 advances acc and gives the per-group
//     partials (reduce with launch_sweep_final), vector v's coefficients go
//     to c_out[v * M + j];
//   launch_est_apply: acc_j += |c_j|^2 from stored coefficients (c == NULL:
//     none) and the per-group partials of nrm - acc;
//   launch_look_list: the best K of n partial records (K <= kLookListMax);
//   launch_rerank: for the K listed columns, c = e^H x_q and a = acc + |c|^2
//     (acc_g[q] when first, else acc_l[slot]; a -> acc_l[slot]) and the argmax
//     of nrm_q - a over listed columns neither masked nor predicted before
//     (chain[0..nprev).J; no candidate if chain[nprev-1] was not accepted);
//     partial holds rerank_partials(K) records.
constexpr int kPivotGroup = 16;
constexpr int kLookMax = 5;
constexpr int kLookListMax = 8192;
hipError_t launch_sweep_look(const double2* S, int64_t N, int64_t M, int64_t ldS, const double2* E, int64_t ldE,
                             int V, const double* nrm, double* acc, const uint8_t* mask, double2* c_out,
                             ArgMax* partial, int64_t npartial_cap, hipStream_t s);
hipError_t launch_est_apply(const double* nrm, double* acc, const uint8_t* mask, const double2* c, int64_t M,
                            ArgMax* partial, int64_t npartial_cap, hipStream_t s);
hipError_t launch_look_list(const ArgMax* partial, int64_t n, int K, ArgMax* list, hipStream_t s);
int64_t rerank_partials(int K);
struct GsState;
hipError_t launch_rerank(const double2* X, int64_t N, int64_t ldX, const double2* e, const ArgMax* list, int K,
                         const double* nrm, const double* acc_g, double* acc_l, int first, const uint8_t* mask,
                         const GsState* chain, int nprev, ArgMax* partial, ArgMax* result, hipStream_t s);

// mixed precision: complex64 sweep with FP32 basis copy -> kTop best
// (est, index) in top[0..kTop) (descending, ties to the lower index)
hipError_t launch_sweep_c(const float2* S, int64_t N, int64_t M, int64_t ldS, const float2* e, const double* nrm,
                          double* acc, const uint8_t* mask, double2* c_out, int64_t ldc, ArgMax* partial,
                          int64_t cap, ArgMax* top, hipStream_t s);
hipError_t launch_sweep_c_final(int64_t M, ArgMax* partial, ArgMax* top, hipStream_t s);
hipError_t launch_est_topk(const double* nrm, const double* acc, const uint8_t* mask, int64_t M, ArgMax* partial,
                           int64_t cap, ArgMax* top, hipStream_t s);
int64_t sweep32_partials_needed(int64_t M);
hipError_t launch_round32(const double2* x, int64_t N, float2* y, hipStream_t s);
hipError_t launch_iota(int64_t* cols, int64_t start, int64_t n, hipStream_t s);
// x[i] <- sqrt(x[i]), i < n
hipError_t launch_sqrt_inplace(double* x, int64_t n, hipStream_t s);
// p[i] <- v for i < n (a kernel, so that no memset node enters a captured
// stream)
hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t s);
hipError_t launch_fill(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
hipError_t launch_fill(int* p, int v, int64_t n, hipStream_t s);

// Gram-Schmidt building blocks over the basis E (N x k, ldE) and nv vectors
// V (N x nv, ldV):  G = E^H V ;  V -= E G ;  norms.
hipError_t launch_gemv_ch(const double2* E, int64_t ldE, int64_t k, const double2* V, int64_t ldV,
                          int64_t nv, int64_t N, double2* G, hipStream_t s);
hipError_t launch_gemv_n_sub(const double2* E, int64_t ldE, int64_t k, const double2* G, double2* V,
                             int64_t ldV, int64_t nv, int64_t N, hipStream_t s);
hipError_t launch_sqnorms_small(const double2* V, int64_t ldV, int64_t nv, int64_t N, double* out,
                                hipStream_t s);
hipError_t launch_scale_into(const double2* v, int64_t N, const double* sq, double2* out, hipStream_t s);

// The Gram-Schmidt of one pivot column driven from the device, so that a
// chain of them (the pivot lookahead) runs without host round trips, and a
// regular step reads its outcome back once.  launch_gs_begin copies column
// J (*jsrc when jsrc != NULL, else jhost) of X into v and sets ||v|| before
// the first pass (sq1 receives ||v||^2); prev (NULL: none) is the previous
// link of a chain, whose rejection makes this one dead.  Each
// launch_gs_pass is one classical pass against E[:, 0..kk-1], kk >= 1
// (G: kk coefficients, sq: ||v||^2 after it), followed by Hoffmann's test;
// passes after the test is met (or after nu_max) do nothing, so a caller
// launches nu_max of them.  launch_gs_finish sets the outcome flags and
// writes e = v / ||v|| into out when accepted.
struct GsState {
  double before;   // ||v|| before the pass under way
  double after;    // ||v|| after the last pass: the residual rho of the pivot
  double s_norm2;  // ||s_J||^2 of the original column (rank test)
  int64_t J;       // the column (< 0: none)
  int32_t passes;
  int32_t done;     // no further pass runs
  int32_t settled;  // the last pass met Hoffmann's criterion
  int32_t live;     // this orthogonalisation runs at all
  int32_t finite;   // ||v|| is finite
  int32_t in_span;  // ||v|| <= 64 u ||s_J||: numerically in span(E)
  int32_t accept;   // live, finite, not in the span, settled unless ||v|| < tol
  int32_t pad;
};
hipError_t launch_gs_begin(const double2* X, int64_t ldX, int64_t N, const ArgMax* jsrc, int64_t jhost,
                           const GsState* prev, const double* nrm0, double2* v, double* sq1, GsState* st,
                           hipStream_t s);
hipError_t launch_gs_pass(const double2* E, int64_t ldE, int64_t kk, double2* v, int64_t N, double2* G, double* sq,
                          GsState* st, int nu_min, int nu_max, double kappa, hipStream_t s);
hipError_t launch_gs_finish(GsState* st, double tol, const double* sq, const double2* v, int64_t N, double2* out,
                            hipStream_t s);

// Re-anchoring: W[:, j] = X[:, j] - sum_{i<m} E[:, i] C(i, j) with
// C(i, j) = C[i*cI + j*cJ] (X may equal W; W == NULL: norms only),
// nrm[j] = ||W[:, j]||^2; *bad set to 1 if a norm is not finite.
hipError_t launch_resid(const double2* X, int64_t ldX, double2* W, int64_t ldW, int64_t N, int64_t M,
                        const double2* E, int64_t ldE, int64_t m, const double2* C, int64_t cI, int64_t cJ,
                        double* nrm, int* bad, hipStream_t s);
hipError_t launch_resid(const double2* X, int64_t ldX, float2* W, int64_t ldW, int64_t N, int64_t M,
                        const double2* E, int64_t ldE, int64_t m, const double2* C, int64_t cI, int64_t cJ,
                        double* nrm, int* bad, hipStream_t s);
hipError_t launch_resid(const float2* X, int64_t ldX, float2* W, int64_t ldW, int64_t N, int64_t M,
                        const double2* E, int64_t ldE, int64_t m, const double2* C, int64_t cI, int64_t cJ,
                        double* nrm, int* bad, hipStream_t s);
// Norms-only re-anchoring fused with the next sweep (FP64 working matrix
// X, not written): against the m <= kFuseMaxM panel vectors E
// (coefficients C(i, j) = Cp[i*ldCp + j]) nrm_j = ||x_j - E c_j||^2
// explicitly, c_out[j] = e^H x_j, acc_j = |c_out[j]|^2; result[0] = the
// masked argmax of nrm - acc, result[1] = the largest unmasked nrm.
// partial needs 2 * anchor_sweep_partials(M) entries.
constexpr int kFuseMaxM = 16;
int64_t anchor_sweep_partials(int64_t M);
hipError_t launch_anchor_sweep(const double2* X, int64_t ldX, int64_t N, int64_t M,
                               const double2* E, int64_t ldE, int64_t m, const double2* Cp, int64_t ldCp,
                               const double2* e, double* nrm, double* acc, const uint8_t* mask, double2* c_out,
                               ArgMax* partial, int64_t npartial_cap, ArgMax* result, int* bad, hipStream_t s);
// C = E^H S on FP64 matrix cores
hipError_t launch_project_z(const double2* E, int64_t N, int64_t k, int64_t ldE, const double2* S, int64_t M,
                            int64_t ldS, double2* C, int64_t ldC, hipStream_t s);

// surrogate inputs: mapped parameters and the phase factors at F rows
// (X: batch x (2 + 2F) floats), targets gathered into T (see rb_chirp.hip)
hipError_t launch_phase_features(const double* params, const float* targets, const int64_t* idx, int64_t batch,
                                 int dout, const double* ranges, const int64_t* rows, int64_t F, const double* table,
                                 float* X, float* T, hipStream_t s);
// chirp row table (3 N doubles, see rb_chirp.hip) for launch_chirp_fill
hipError_t launch_chirp_table(double flo, double fhi, int64_t N, double* table, hipStream_t s);
// cols (device, may be NULL): output column j uses parameter set cols[j]
hipError_t launch_chirp_fill(const double* params, const int64_t* cols, int64_t M, const double* table, int64_t N,
                             int dtype, void* out, int64_t ld, hipStream_t s);

}  // namespace rb

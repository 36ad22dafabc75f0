// Internal declarations shared by the HIP translation units of librb.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rb.h"
#include "rb_device.h"

namespace rb {

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
//     above 32,768 records they are first reduced to the maxima of equal
//     runs, into scratch (look_list_scratch(n) records, 0 when not needed);
//   launch_rerank: for the K listed columns, c = e^H x_q and a = acc + |c|^2
//     (acc_g[q] when first, else acc_l[slot]; a -> acc_l[slot]) and the argmax
//     of nrm_q - a over listed columns neither masked nor predicted before
//     (chain[0..nprev).J; no candidate if chain[nprev-1] was not accepted);
//     partial holds rerank_partials(K) records.
constexpr int kPivotGroup = 16;
constexpr int kLookMax = 5;
constexpr int kLookPasses = 2;  // Gram-Schmidt passes queued for a predicted pivot
constexpr int kLookListMax = 8192;
hipError_t launch_sweep_look(const double2* S, int64_t N, int64_t M, int64_t ldS, const double2* E, int64_t ldE,
                             int V, const double* nrm, double* acc, const uint8_t* mask, double2* c_out,
                             ArgMax* partial, int64_t npartial_cap, hipStream_t s);
hipError_t launch_est_apply(const double* nrm, double* acc, const uint8_t* mask, const double2* c, int64_t M,
                            ArgMax* partial, int64_t npartial_cap, hipStream_t s);
int64_t look_list_scratch(int64_t n);
hipError_t launch_look_list(const ArgMax* partial, int64_t n, int K, ArgMax* list, ArgMax* scratch, hipStream_t s);
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
// Pivot lookahead of the mixed greedy (rb_sweep32.hip), the complex64 forms
// of launch_sweep_look / launch_est_apply / launch_rerank: the same tile
// arithmetic as launch_sweep_c on 16-byte aligned columns (even ldS) and
// vectors (sweep_c_look_ok), top-8 candidates instead of one argmax.
//   launch_sweep_c_look: V = 1 + d vectors e[v * ldv ..]; vector 0 advances
//     acc and gives the top-8 (into top when != NULL), vector v's
//     coefficients go to c_out[v * M + j];
//   launch_est_apply32: acc += |c|^2 (c == NULL: none), top-8 into top;
//   launch_rerank32: the listed columns' updated estimates (acc_l as in
//     launch_rerank) and their top-8 into top, excluding masked columns and
//     excl[0..nexcl); partial holds rerank32_partials(K) records.
bool sweep_c_look_ok(const float2* S, int64_t ldS, const float2* e, int64_t ldv);
hipError_t launch_sweep_c_look(const float2* S, int64_t N, int64_t M, int64_t ldS, const float2* e, int64_t ldv, int V,
                               const double* nrm, double* acc, const uint8_t* mask, double2* c_out, ArgMax* partial,
                               int64_t cap, ArgMax* top, hipStream_t s);
hipError_t launch_est_apply32(const double* nrm, double* acc, const uint8_t* mask, const double2* c, int64_t M,
                              ArgMax* partial, int64_t cap, ArgMax* top, hipStream_t s);
int64_t rerank32_partials(int K);
hipError_t launch_rerank32(const float2* X, int64_t N, int64_t ldX, const float2* e, const ArgMax* list, int K,
                           const double* nrm, const double* acc_g, double* acc_l, int first, const uint8_t* mask,
                           const int64_t* excl, int nexcl, ArgMax* partial, ArgMax* top, hipStream_t s);
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

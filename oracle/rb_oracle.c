/*
 * CPU FP64 oracle for the reduced-basis greedy of Antil, Chen & Field,
 * "A Note on QR-Based Model Reduction" (arXiv 1805.06124).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP path.
 *
 * Everything here is plain, slow and literal:
 *   - oracle_sqnorm        : ||x||^2 accumulated exactly (double-double),
 *                            rounded once to double.
 *   - oracle_chirp         : the leading-1PN chirp snapshot family used as the
 *                            stand-in workload (unit-L2-normalised columns).
 *   - oracle_greedy_explicit: Alg. 2 (MGS with column pivoting, Sec. 5.2.1) in
 *                            its explicit residual-matrix form; the pivot is the
 *                            column of largest residual norm (equivalently
 *                            Alg. 3, Proposition 5.3), the new basis vector is
 *                            orthonormalised by Hoffmann's iterated MGS
 *                            ("MGSCI", kappa = 2, Sec. 6.1.2).
 *   - oracle_greedy_resume : the explicit greedy continued from a given
 *                            orthonormal basis (enrichment after
 *                            out-of-sample validation, Sec. 6.1).
 *   - oracle_greedy_pythag : the same greedy with the pivot search done by the
 *                            Pythagorean residual update of Eq. (6.3) (stored
 *                            ||s_i||^2 and running sum of |c|^2; no residual
 *                            matrix), as in the paper's own code.
 *   - oracle_project       : C = E^H S, a plain triple loop.
 *   - oracle_residual_norms: ||s_j - E E^H s_j||_2 per column, explicitly.
 *
 * Complex arithmetic follows the paper's real-valued statements with the
 * transpose read as the conjugate transpose: <e, s> = e^H s, |c|^2 = c c*.
 *
 * Layout: a complex N x M matrix is column-major with leading dimension ld,
 * i.e. column j starts at x + j*ld; elements are C99 double complex
 * (interleaved re, im).
 *
 * Optional OpenMP (compile with -fopenmp) parallelises loops over independent
 * columns only; every reduction over columns (argmax, max) is sequential, so
 * results do not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;

/* Status codes (same meaning as the product library's; defined here on
 * their own so the two sides share no header). */
#define OR_OK 0
#define OR_KMAX 1
#define OR_RANK 2
#define OR_EINVAL -1
#define OR_ENOMEM -2
#define OR_ENONFINITE -4
#define OR_EREPLAY -6

/* ------------------------------------------------------------------ */
/* exact squared norm: error-free products (fma) accumulated as a     */
/* double-double (hi, lo) and rounded to double once at the end.      */
/* ------------------------------------------------------------------ */
static void dd_add(double *hi, double *lo, double a) {
  double s = *hi + a;
  double bb = s - *hi;
  double err = (*hi - (s - bb)) + (a - bb);
  *lo += err;
  *hi = s;
}

double oracle_sqnorm(const zc *x, int64_t n) {
  double hi = 0.0, lo = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double re = creal(x[i]), im = cimag(x[i]);
    double p1 = re * re, e1 = fma(re, re, -p1);
    double p2 = im * im, e2 = fma(im, im, -p2);
    dd_add(&hi, &lo, p1);
    lo += e1;
    dd_add(&hi, &lo, p2);
    lo += e2;
  }
  /* one rounding of hi + lo */
  return hi + lo;
}

void oracle_sqnorms(const zc *S, int64_t N, int64_t M, int64_t ld, double *out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t j = 0; j < M; ++j) out[j] = oracle_sqnorm(S + j * ld, N);
}

static zc dotc(const zc *e, const zc *v, int64_t n) { /* e^H v */
  zc s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += conj(e[i]) * v[i];
  return s;
}

static double plain_norm(const zc *v, int64_t n) { return sqrt(oracle_sqnorm(v, n)); }

/* ------------------------------------------------------------------ */
/* Chirp snapshot family (stand-in for the paper's IMRPhenomPv2 data, */
/* Sec. 6.1.1): h(f) = f^(-7/6) exp(-i Psi(f)),                        */
/* Psi = -pi/4 + 3/(128 eta v^5) (1 + (3715/756 + 55 eta/9) v^2),      */
/* v = (pi Mtot f)^(1/3), Mtot in seconds (solar masses * GM_sun/c^3), */
/* eta = q/(1+q)^2.  Uniform grid f_n = flo + n (fhi-flo)/(N-1).       */
/* Each column is divided by its L2 norm.                              */
/* ------------------------------------------------------------------ */
#define ORACLE_TSUN 4.925490947641267e-6 /* GM_sun / c^3 in seconds */

void oracle_chirp(const double *params, int64_t M, double flo, double fhi, int64_t N, zc *out, int64_t ld) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t j = 0; j < M; ++j) {
    double Mtot = params[2 * j] * ORACLE_TSUN;
    double q = params[2 * j + 1];
    double eta = q / ((1.0 + q) * (1.0 + q));
    zc *col = out + j * ld;
    for (int64_t n = 0; n < N; ++n) {
      double f = (N > 1) ? flo + (double)n * (fhi - flo) / (double)(N - 1) : flo;
      double v = cbrt(M_PI * Mtot * f);
      double v2 = v * v;
      double v5 = v2 * v2 * v;
      double psi = -M_PI / 4.0 + 3.0 / (128.0 * eta * v5) * (1.0 + (3715.0 / 756.0 + 55.0 * eta / 9.0) * v2);
      double amp = pow(f, -7.0 / 6.0);
      col[n] = amp * cos(psi) - I * (amp * sin(psi));
    }
    double nrm = plain_norm(col, N);
    for (int64_t n = 0; n < N; ++n) col[n] = col[n] / nrm;
  }
}

/* ------------------------------------------------------------------ */
/* Hoffmann's iterated MGS, criterion form ("MGSCI"), Sec. 6.1.2:      */
/* repeat a full modified Gram-Schmidt pass of v against e_1..e_k     */
/* while the pass shrinks ||v|| by at least the factor kappa; at most */
/* nu_max passes.  Returns the number of passes; *rho_out = ||v||.    */
/* ------------------------------------------------------------------ */
static int mgsci(const zc *E, int64_t ldE, int64_t k, zc *v, int64_t N, double kappa, int nu_max, double *rho_out) {
  double before = plain_norm(v, N);
  int nu = 0;
  double after = before;
  while (nu < nu_max) {
    for (int64_t i = 0; i < k; ++i) {
      const zc *e = E + i * ldE;
      zc c = dotc(e, v, N);
      for (int64_t n = 0; n < N; ++n) v[n] -= c * e[n];
    }
    ++nu;
    after = plain_norm(v, N);
    if (after > before / kappa) break;
    before = after;
  }
  *rho_out = after;
  return nu;
}

/* argmax over unpivoted columns of val[]; ties go to the lowest index.
 * Returns -1 if every column is pivoted. */
static int64_t argmax_unpivoted(const double *val, const unsigned char *piv_mask, int64_t M) {
  int64_t best = -1;
  for (int64_t j = 0; j < M; ++j) {
    if (piv_mask[j]) continue;
    if (best < 0 || val[j] > val[best]) best = j;
  }
  return best;
}

static int any_nonfinite(const zc *S, int64_t N, int64_t M, int64_t ld) {
  for (int64_t j = 0; j < M; ++j)
    for (int64_t n = 0; n < N; ++n) {
      double re = creal(S[j * ld + n]), im = cimag(S[j * ld + n]);
      if (!isfinite(re) || !isfinite(im)) return 1;
    }
  return 0;
}

/*
 * Shared result record of both greedy forms.
 *   E     : N x kmax basis, column-major, ld = N (caller-owned)
 *   piv   : kmax pivots (0-based column indices)
 *   err   : kmax+1 greedy errors; err[i] = max over unpivoted columns of the
 *           residual norm after i basis vectors (err[0] = max ||s_j||)
 *   rho   : kmax explicit pivot residual norms ||v|| after MGSCI (= |R_ii|)
 *   nu    : kmax MGSCI pass counts
 *   pick  : kmax pairs (residual^2 of the chosen pivot, max residual^2) as
 *           seen by this oracle at that step (used by the replay check)
 *   C     : optional kmax x M coefficients R(i, j) = e_i^H (residual of s_j
 *           after i-1 vectors), column-major with ld = kmax (NULL to skip)
 */

/*
 * Alg. 2 / Alg. 3 in explicit residual form, started from k0 >= 0 given
 * orthonormal basis vectors E[:, 0..k0-1].
 * k0 = 0 is the greedy itself.  k0 > 0 continues a greedy whose basis
 * already holds k0 vectors: every column of S is first reduced against
 * e_1..e_k0 by the same column updates Alg. 2 makes after each pivot (one
 * MGS step per vector, in order), and the loop then runs from k = k0.  This
 * is the enrichment step of out-of-sample validation (Sec. 6.1): columns
 * that fail validation continue the greedy of the existing basis.
 * Stopping rule: continue while err[k] >= tol and k < kmax; return k basis
 * vectors in total (err[k] < tol, or k = kmax).  If the largest residual is
 * already below tol no vector is added.  force_piv (length nforce, may be
 * NULL) replays a given pivot sequence: at step k0 + i, i < nforce, the pivot
 * is force_piv[i] instead of the argmax (the argmax and the forced value are
 * both recorded in pick).  Entries of piv, err, rho, nu, pick below k0 are
 * left untouched.
 */
static int greedy_explicit(const zc *S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax,
                           double kappa, int nu_max, const int64_t *force_piv, int64_t nforce, int64_t k0,
                           zc *E, int64_t *piv, double *err, double *rho, int *nu, double *pick,
                           zc *C, int64_t *k_out) {
  if (N <= 0 || M <= 0 || ldS < N || kmax < 0 || k0 < 0 || k0 > N || !S || !E || !piv || !err || !rho || !k_out)
    return OR_EINVAL;
  if (any_nonfinite(S, N, M, ldS)) return OR_ENONFINITE;
  int64_t kcap = kmax;
  if (kcap > N) kcap = N;
  if (kcap > k0 + M) kcap = k0 + M;
  if (kcap < k0) return OR_EINVAL;
  zc *V = (zc *)malloc(sizeof(zc) * (size_t)N * (size_t)M);
  double *res2 = (double *)malloc(sizeof(double) * (size_t)M);
  unsigned char *mask = (unsigned char *)calloc((size_t)M, 1);
  zc *v = (zc *)malloc(sizeof(zc) * (size_t)N);
  if (!V || !res2 || !mask || !v) { free(V); free(res2); free(mask); free(v); return OR_ENOMEM; }
  for (int64_t j = 0; j < M; ++j) memcpy(V + j * N, S + j * ldS, sizeof(zc) * (size_t)N);
  /* reduce every column against the k0 given vectors, one MGS step each */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t j = 0; j < M; ++j) {
    zc *Vj = V + j * N;
    for (int64_t i = 0; i < k0; ++i) {
      const zc *ei = E + i * N;
      zc c = dotc(ei, Vj, N);
      if (C) C[j * kcap + i] = c;
      for (int64_t n = 0; n < N; ++n) Vj[n] -= c * ei[n];
    }
  }

  int status = OR_KMAX;
  int64_t k = k0;
  oracle_sqnorms(V, N, M, N, res2);
  int64_t p = argmax_unpivoted(res2, mask, M);
  err[k0] = sqrt(res2[p]);
  if (err[k0] < tol) { status = OR_OK; goto done; }
  while (k < kcap) {
    if (err[k] < tol) { status = OR_OK; break; }
    /* pivot: argmax of the explicit residual norms (Alg. 2) */
    int64_t pk = p;
    if (force_piv && k - k0 < nforce) {
      pk = force_piv[k - k0];
      if (pk < 0 || pk >= M || mask[pk]) { status = OR_EREPLAY; break; }
    }
    if (pick) { pick[2 * k] = res2[pk]; pick[2 * k + 1] = res2[p]; }
    memcpy(v, V + pk * N, sizeof(zc) * (size_t)N);
    double s_norm = plain_norm(S + pk * ldS, N);
    double r;
    int passes = mgsci(E, N, k, v, N, kappa, nu_max, &r);
    /* numerically in the span of the basis: rank exhausted */
    if (r <= 64.0 * 0x1p-53 * s_norm || r == 0.0) { status = OR_RANK; break; }
    zc *ek = E + k * N;
    for (int64_t n = 0; n < N; ++n) ek[n] = v[n] / r;
    piv[k] = pk;
    rho[k] = r;
    if (nu) nu[k] = passes;
    mask[pk] = 1;
    /* MGS update of every remaining residual column against e_{k+1} */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t j = 0; j < M; ++j) {
      zc *Vj = V + j * N;
      zc c = dotc(ek, Vj, N);
      if (C) C[j * kcap + k] = c;
      if (mask[j]) continue;
      for (int64_t n = 0; n < N; ++n) Vj[n] -= c * ek[n];
      res2[j] = oracle_sqnorm(Vj, N);
    }
    ++k;
    p = argmax_unpivoted(res2, mask, M);
    /* every column pivoted (k = M): nothing is left to approximate */
    err[k] = (p >= 0) ? sqrt(res2[p]) : 0.0;
  }
  if (k == kcap && status == OR_KMAX && err[k] < tol) status = OR_OK;
done:
  *k_out = k;
  free(V); free(res2); free(mask); free(v);
  return status;
}

int oracle_greedy_explicit(const zc *S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax,
                           double kappa, int nu_max, const int64_t *force_piv, int64_t nforce,
                           zc *E, int64_t *piv, double *err, double *rho, int *nu, double *pick,
                           zc *C, int64_t *k_out) {
  return greedy_explicit(S, N, M, ldS, tol, kmax, kappa, nu_max, force_piv, nforce, 0, E, piv, err, rho, nu,
                         pick, C, k_out);
}

/* The greedy continued from the k0 orthonormal vectors in E[:, 0..k0-1]
 * (ld = N); see greedy_explicit. */
int oracle_greedy_resume(const zc *S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax,
                         double kappa, int nu_max, const int64_t *force_piv, int64_t nforce, int64_t k0,
                         zc *E, int64_t *piv, double *err, double *rho, int *nu, double *pick,
                         zc *C, int64_t *k_out) {
  return greedy_explicit(S, N, M, ldS, tol, kmax, kappa, nu_max, force_piv, nforce, k0, E, piv, err, rho, nu,
                         pick, C, k_out);
}

/*
 * Same greedy with the pivot search by the Pythagorean residual update of
 * Eq. (6.3): est_j = ||s_j||^2 - sum_i |e_i^H s_j|^2, the two terms stored
 * separately; the pivot column s_J itself (not a residual) is orthonormalised
 * against the basis by MGSCI, as in Alg. 3.
 */
int oracle_greedy_pythag(const zc *S, int64_t N, int64_t M, int64_t ldS, double tol, int64_t kmax,
                         double kappa, int nu_max, const int64_t *force_piv, int64_t nforce,
                         zc *E, int64_t *piv, double *err, double *rho, int *nu, double *pick,
                         zc *C, int64_t *k_out) {
  if (N <= 0 || M <= 0 || ldS < N || kmax < 0 || !S || !E || !piv || !err || !rho || !k_out) return OR_EINVAL;
  if (any_nonfinite(S, N, M, ldS)) return OR_ENONFINITE;
  int64_t kcap = kmax;
  if (kcap > N) kcap = N;
  if (kcap > M) kcap = M;
  double *nrm = (double *)malloc(sizeof(double) * (size_t)M);
  double *acc = (double *)calloc((size_t)M, sizeof(double));
  double *est = (double *)malloc(sizeof(double) * (size_t)M);
  unsigned char *mask = (unsigned char *)calloc((size_t)M, 1);
  zc *v = (zc *)malloc(sizeof(zc) * (size_t)N);
  if (!nrm || !acc || !est || !mask || !v) { free(nrm); free(acc); free(est); free(mask); free(v); return OR_ENOMEM; }
  oracle_sqnorms(S, N, M, ldS, nrm);
  memcpy(est, nrm, sizeof(double) * (size_t)M);
  int status = OR_KMAX;
  int64_t k = 0;
  int64_t p = argmax_unpivoted(est, mask, M);
  err[0] = sqrt(est[p]);
  while (k < kcap) {
    if (err[k] < tol) { status = OR_OK; break; }
    int64_t pk = p;
    if (force_piv && k < nforce) {
      pk = force_piv[k];
      if (pk < 0 || pk >= M || mask[pk]) { status = OR_EREPLAY; break; }
    }
    if (pick) { pick[2 * k] = est[pk]; pick[2 * k + 1] = est[p]; }
    memcpy(v, S + pk * ldS, sizeof(zc) * (size_t)N);
    double s_norm = plain_norm(v, N);
    double r;
    int passes = mgsci(E, N, k, v, N, kappa, nu_max, &r);
    if (r <= 64.0 * 0x1p-53 * s_norm || r == 0.0) { status = OR_RANK; break; }
    zc *ek = E + k * N;
    for (int64_t n = 0; n < N; ++n) ek[n] = v[n] / r;
    piv[k] = pk;
    rho[k] = r;
    if (nu) nu[k] = passes;
    mask[pk] = 1;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t j = 0; j < M; ++j) {
      zc c = dotc(ek, S + j * ldS, N);
      if (C) C[j * kcap + k] = c;
      if (mask[j]) continue;
      double cr = creal(c), ci = cimag(c);
      acc[j] += cr * cr + ci * ci;
      est[j] = nrm[j] - acc[j];
    }
    ++k;
    p = argmax_unpivoted(est, mask, M);
    err[k] = (p >= 0) ? sqrt(est[p] > 0.0 ? est[p] : 0.0) : 0.0;
  }
  if (k == kcap && status == OR_KMAX && err[k] < tol) status = OR_OK;
  *k_out = k;
  free(nrm); free(acc); free(est); free(mask); free(v);
  return status;
}

/* C = E^H S : k x M, column-major with ldC (plain triple loop). */
void oracle_project(const zc *E, int64_t N, int64_t k, int64_t ldE, const zc *S, int64_t M, int64_t ldS,
                    zc *C, int64_t ldC) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t j = 0; j < M; ++j)
    for (int64_t i = 0; i < k; ++i) C[j * ldC + i] = dotc(E + i * ldE, S + j * ldS, N);
}

/* out[j] = || s_j - E (E^H s_j) ||_2 for every column (explicit residual). */
void oracle_residual_norms(const zc *E, int64_t N, int64_t k, int64_t ldE, const zc *S, int64_t M, int64_t ldS,
                           double *out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t j = 0; j < M; ++j) {
    zc *r = (zc *)malloc(sizeof(zc) * (size_t)N);
    zc *c = (zc *)malloc(sizeof(zc) * (size_t)(k > 0 ? k : 1));
    const zc *s = S + j * ldS;
    for (int64_t i = 0; i < k; ++i) c[i] = dotc(E + i * ldE, s, N);
    for (int64_t n = 0; n < N; ++n) {
      zc t = s[n];
      for (int64_t i = 0; i < k; ++i) t -= E[i * ldE + n] * c[i];
      r[n] = t;
    }
    out[j] = plain_norm(r, N);
    free(r);
    free(c);
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

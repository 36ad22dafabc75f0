// The reconstruction algorithm (Alg. 4, Sec. 5.2.2; Theorem 5.8): after the
// greedy has produced Q_j and R(1:j, :) = Q_j^H S Pi, take the SVD of
// R(1:j, :) = V Sigma W^H, keep the k singular values >= tau2 and return
// X_k = Q_j V(:, 1:k).  The rows of R are the coefficients C = E^H S up to
// the column order, which changes neither the singular values nor V.
//
// The SVD's left factor on the GPU:
//   1. G = C C^H (j x j, FP64, split over the M columns, partial sums added
//      in a fixed order);
//   2. V0 = eigenvectors of G by cyclic Jacobi in parallel (round-robin)
//      order.  A rotation is skipped when |G_pq| <= eps sqrt(G_pp G_qq), the
//      relative test;
//   3. refinement: B = V0^H C (matrix cores), G2 = B B^H, Jacobi on G2 gives
//      V1 and the eigenvalues; V = V0 V1, sigma_i = sqrt(lambda_i), sorted
//      descending.
// The Gram matrix squares the condition number.  On its own it fixes the
// small sigma only to about sqrt(u) sigma_1, unless the rows of C are graded
// as the greedy orders them.  After the refinement the rows of B are
// orthogonal to working accuracy, so the second Gram matrix is determined
// entry by entry to relative accuracy.  Its Jacobi eigenvalues then carry an
// absolute error of a few u sigma_1, the accuracy of an SVD of C taken
// directly.
#include <algorithm>
#include <cmath>
#include <vector>

#include "rb_host.h"

using namespace rb;

namespace rb {
namespace {

constexpr int kGT = 64;   // Gram tile (rows of C per side)
constexpr int kGK = 16;   // columns of C staged per step

// Partial Gram tiles: for tile pair tp = (ti >= tl) and column split sp,
// P[(sp * ntp + tp) * 4096 + a * 64 + b] = sum over m in the split of
// C[ti*64 + a, m] conj(C[tl*64 + b, m]).
__global__ __launch_bounds__(256) void k_gram_partial(const double2* __restrict__ C, int64_t j, int64_t M,
                                                      int64_t ldC, int64_t chunk, int ntile,
                                                      double2* __restrict__ P) {
  __shared__ double2 sA[kGK][kGT + 1];
  __shared__ double2 sB[kGK][kGT + 1];
  const int tp = blockIdx.x;
  // tile pair index -> (ti, tl), ti >= tl, row-major over the lower triangle
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= tp) ++ti;
  const int tl = tp - ti * (ti + 1) / 2;
  const int ntp = ntile * (ntile + 1) / 2;
  const int64_t m0 = (int64_t)blockIdx.y * chunk;
  const int64_t m1 = std::min<int64_t>(M, m0 + chunk);
  const int t = threadIdx.x;
  const int ta = t & 15, tb = t >> 4;
  const int64_t i0 = (int64_t)ti * kGT, l0 = (int64_t)tl * kGT;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);

  for (int64_t mb = m0; mb < m1; mb += kGK) {
    // stage 16 columns x 64 rows of each side (4 elements per thread)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = t + 256 * q;
      const int r = idx & 63, c = idx >> 6;
      const int64_t m = mb + c;
      const bool okm = m < m1;
      sA[c][r] = (okm && i0 + r < j) ? C[(i0 + r) + m * ldC] : make_double2(0.0, 0.0);
      sB[c][r] = (okm && l0 + r < j) ? C[(l0 + r) + m * ldC] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < kGK; ++c) {
      double2 av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sA[c][ta + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sB[c][tb + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          // a * conj(b)
          acc[a][b].x = fma(av[a].x, bv[b].x, fma(av[a].y, bv[b].y, acc[a][b].x));
          acc[a][b].y = fma(av[a].y, bv[b].x, fma(-av[a].x, bv[b].y, acc[a][b].y));
        }
    }
    __syncthreads();
  }
  double2* out = P + ((int64_t)blockIdx.y * ntp + tp) * (kGT * kGT);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) out[(ta + 16 * a) * kGT + (tb + 16 * b)] = acc[a][b];
}

// G (j x j, ld j, full Hermitian) from the partials, splits added in order.
// Element (i, l) with i >= l is summed once; G[l, i] is its conjugate and
// the diagonal is real.
__global__ __launch_bounds__(256) void k_gram_reduce(const double2* __restrict__ P, int ns, int ntp, int64_t j,
                                                     double2* __restrict__ G) {
  const int tp = blockIdx.x;
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= tp) ++ti;
  const int tl = tp - ti * (ti + 1) / 2;
  for (int e = threadIdx.x; e < kGT * kGT; e += 256) {
    const int a = e / kGT, b = e % kGT;
    const int64_t i = (int64_t)ti * kGT + a, l = (int64_t)tl * kGT + b;
    if (i >= j || l >= j || i < l) continue;
    double2 s = make_double2(0.0, 0.0);
    for (int sp = 0; sp < ns; ++sp) {
      const double2 v = P[((int64_t)sp * ntp + tp) * (kGT * kGT) + e];
      s.x += v.x;
      s.y += v.y;
    }
    if (i == l) s.y = 0.0;
    G[i + l * j] = s;
    G[l + i * j] = make_double2(s.x, -s.y);
  }
}

// Cyclic Jacobi for the Hermitian j x j matrix G (ld j, overwritten: its
// diagonal ends as the eigenvalues) accumulating V (ld j) = the
// eigenvectors.  One block; each round applies n/2 disjoint rotations
// (round-robin pairing), columns then rows.  info: sweeps used, or -1 if
// max_sweeps passed without a rotation-free sweep.
constexpr int kJT = 1024;
constexpr int kJU = 2;           // elements per thread per pass (loads first)
constexpr int kMaxPairs = 1024;  // j <= 2048

__global__ __launch_bounds__(kJT) void k_jacobi(double2* __restrict__ G, int64_t n, double2* __restrict__ V,
                                                int max_sweeps, double eps, int* __restrict__ info) {
  __shared__ int sp[kMaxPairs], sq[kMaxPairs];
  __shared__ double sc[kMaxPairs], ss[kMaxPairs], sa[kMaxPairs], sd[kMaxPairs];
  __shared__ double2 sph[kMaxPairs];
  __shared__ int sact[kMaxPairs];
  __shared__ int rotated;
  const int t = threadIdx.x;
  for (int64_t e = t; e < n * n; e += kJT) {
    const int64_t r = e % n, c = e / n;
    V[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  const int64_t npr = n + (n & 1);
  const int64_t half = npr / 2;
  const uint32_t nu = (uint32_t)n;  // n <= 2048: pair-element indices fit 32 bits
  int sweep = 0;
  bool done = false;
  for (; sweep < max_sweeps && !done; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int64_t r = 0; r < npr - 1; ++r) {
      // ---- rotation parameters of every pair ----
      for (int64_t i = t; i < half; i += kJT) {
        int64_t p, q;
        if (i == 0) {
          p = r;
          q = npr - 1;
        } else {
          p = (r + i) % (npr - 1);
          q = (r - i + (npr - 1)) % (npr - 1);
        }
        if (p > q) {
          const int64_t tmp = p;
          p = q;
          q = tmp;
        }
        int act = 0;
        if (q < n) {
          const double a = G[p + p * n].x, d = G[q + q * n].x;
          const double2 b = G[p + q * n];
          const double ab = hypot(b.x, b.y);
          if (ab > 0.0 && ab > eps * sqrt(fabs(a * d))) {
            const double zeta = (d - a) / (2.0 * ab);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + tt * tt);
            sc[i] = c;
            ss[i] = tt * c;
            sph[i] = make_double2(b.x / ab, b.y / ab);
            sa[i] = a - tt * ab;
            sd[i] = d + tt * ab;
            act = 1;
          }
        }
        sp[i] = (int)p;
        sq[i] = (int)q;
        sact[i] = act;
        if (act) atomicOr(&rotated, 1);
      }
      __syncthreads();
      // ---- columns p, q of G and V: [x_p, x_q] <- [x_p, x_q] J ----
      // each thread takes kJU elements at a time, all loads issued first
      const int64_t total = half * n;
      for (int64_t base = t; base < total; base += (int64_t)kJT * kJU) {
        double2 gp[kJU], gq[kJU], vp[kJU], vq[kJU];
        bool ok[kJU];
#pragma unroll
        for (int u = 0; u < kJU; ++u) {
          const int64_t e = base + (int64_t)u * kJT;
          ok[u] = false;
          if (e < total) {
            const int64_t i = (uint32_t)e / nu, row = (uint32_t)e % nu;
            if (sact[i]) {
              ok[u] = true;
              const int64_t p = sp[i], q = sq[i];
              gp[u] = G[row + p * n];
              gq[u] = G[row + q * n];
              vp[u] = V[row + p * n];
              vq[u] = V[row + q * n];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kJU; ++u) {
          if (!ok[u]) continue;
          const int64_t e = base + (int64_t)u * kJT;
          const int64_t i = (uint32_t)e / nu, row = (uint32_t)e % nu;
          const int64_t p = sp[i], q = sq[i];
          const double c = sc[i], s = ss[i];
          const double2 ph = sph[i];  // J = [[c, s], [-s conj(ph), c conj(ph)]]
          // xq * conj(ph)
          const double2 y = make_double2(gq[u].x * ph.x + gq[u].y * ph.y, gq[u].y * ph.x - gq[u].x * ph.y);
          G[row + p * n] = make_double2(c * gp[u].x - s * y.x, c * gp[u].y - s * y.y);
          G[row + q * n] = make_double2(s * gp[u].x + c * y.x, s * gp[u].y + c * y.y);
          const double2 z = make_double2(vq[u].x * ph.x + vq[u].y * ph.y, vq[u].y * ph.x - vq[u].x * ph.y);
          V[row + p * n] = make_double2(c * vp[u].x - s * z.x, c * vp[u].y - s * z.y);
          V[row + q * n] = make_double2(s * vp[u].x + c * z.x, s * vp[u].y + c * z.y);
        }
      }
      __syncthreads();
      // ---- rows p, q of G: [y_p; y_q] <- J^H [y_p; y_q] ----
      // element e = (column, pair) with the pair varying fastest, so the
      // threads of a wave touch the rows of one column (a few cache lines)
      const uint32_t hu = (uint32_t)half;
      for (int64_t base = t; base < total; base += (int64_t)kJT * kJU) {
        double2 yp[kJU], yq[kJU];
        bool ok[kJU];
#pragma unroll
        for (int u = 0; u < kJU; ++u) {
          const int64_t e = base + (int64_t)u * kJT;
          ok[u] = false;
          if (e < total) {
            const int64_t i = (uint32_t)e % hu, col = (uint32_t)e / hu;
            if (sact[i]) {
              ok[u] = true;
              const int64_t p = sp[i], q = sq[i];
              if (col != p && col != q) {
                yp[u] = G[p + col * n];
                yq[u] = G[q + col * n];
              }
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kJU; ++u) {
          if (!ok[u]) continue;
          const int64_t e = base + (int64_t)u * kJT;
          const int64_t i = (uint32_t)e % hu, col = (uint32_t)e / hu;
          const int64_t p = sp[i], q = sq[i];
          if (col == p) {
            G[p + p * n] = make_double2(sa[i], 0.0);
            G[q + p * n] = make_double2(0.0, 0.0);
            continue;
          }
          if (col == q) {
            G[q + q * n] = make_double2(sd[i], 0.0);
            G[p + q * n] = make_double2(0.0, 0.0);
            continue;
          }
          const double c = sc[i], s = ss[i];
          const double2 ph = sph[i];
          // yq * ph
          const double2 z = make_double2(yq[u].x * ph.x - yq[u].y * ph.y, yq[u].x * ph.y + yq[u].y * ph.x);
          G[p + col * n] = make_double2(c * yp[u].x - s * z.x, c * yp[u].y - s * z.y);
          G[q + col * n] = make_double2(s * yp[u].x + c * z.x, s * yp[u].y + c * z.y);
        }
      }
      __syncthreads();
    }
    done = (rotated == 0);
    __syncthreads();
  }
  if (t == 0) *info = done ? sweep : -1;
}

// Descending order of the eigenvalues diag(G) (ties to the lower index):
// sigma[r] = sqrt(max(lambda, 0)) and perm[r] = the eigenvalue's index.
__global__ __launch_bounds__(256) void k_eig_order(const double2* __restrict__ G, int64_t n,
                                                   double* __restrict__ sigma, int64_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double li = G[i + i * n].x;
  int64_t rank = 0;
  for (int64_t l = 0; l < n; ++l) {
    const double ll = G[l + l * n].x;
    rank += (ll > li || (ll == li && l < i)) ? 1 : 0;
  }
  sigma[rank] = sqrt(li > 0.0 ? li : 0.0);
  perm[rank] = i;
}

// Out[:, r] = A[:, perm[r]] for r < ncols (complex columns of length n)
__global__ __launch_bounds__(256) void k_permute_cols(const double2* __restrict__ A, int64_t n, int64_t lda,
                                                      const int64_t* __restrict__ perm, int64_t ncols,
                                                      double2* __restrict__ Out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t row = e % n, r = e / n;
  Out[row + r * ldo] = A[row + perm[r] * lda];
}

// Out (m x nn) = A (m x kk) B (kk x nn), complex, column-major; 16 x 16
// output tile per block, kk staged 16 at a time.
__global__ __launch_bounds__(256) void k_gemm_nn(const double2* __restrict__ A, int64_t lda,
                                                 const double2* __restrict__ B, int64_t ldb, int64_t m, int64_t nn,
                                                 int64_t kk, double2* __restrict__ Out, int64_t ldo) {
  __shared__ double2 sA[16][17], sB[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t row = (int64_t)blockIdx.x * 16 + tx, col = (int64_t)blockIdx.y * 16 + ty;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t k0 = 0; k0 < kk; k0 += 16) {
    {
      const int64_t ka = k0 + ty;  // A tile: rows of this block, 16 k's
      sA[ty][tx] = (row < m && ka < kk) ? A[row + ka * lda] : make_double2(0.0, 0.0);
      const int64_t kb = k0 + tx;  // B tile: 16 k's, columns of this block
      sB[ty][tx] = (kb < kk && col < nn) ? B[kb + col * ldb] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double2 a = sA[q][tx], b = sB[ty][q];
      acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
      acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
    }
    __syncthreads();
  }
  if (row < m && col < nn) Out[row + col * ldo] = acc;
}

}  // namespace

// G = C C^H for C j x M (ldC); P holds the partial tiles.
static hipError_t gram(const double2* C, int64_t j, int64_t M, int64_t ldC, double2* P, int ns, double2* G,
                       hipStream_t s) {
  const int ntile = (int)((j + kGT - 1) / kGT);
  const int ntp = ntile * (ntile + 1) / 2;
  int64_t chunk = (M + ns - 1) / ns;
  chunk = (chunk + kGK - 1) / kGK * kGK;
  const int nsu = (int)((M + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_gram_partial, dim3(ntp, nsu), dim3(256), 0, s, C, j, M, ldC, chunk, ntile, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3(ntp), dim3(256), 0, s, P, nsu, ntp, j, G);
  return hipGetLastError();
}

static int gram_splits(int64_t j, int64_t M) {
  const int ntile = (int)((j + kGT - 1) / kGT);
  const int ntp = ntile * (ntile + 1) / 2;
  int ns = std::max(1, 2048 / ntp);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, (M + 1023) / 1024));
  return std::min(ns, 256);
}

static hipError_t gemm_nn(const double2* A, int64_t lda, const double2* B, int64_t ldb, int64_t m, int64_t nn,
                          int64_t kk, double2* Out, int64_t ldo, hipStream_t s) {
  if (m <= 0 || nn <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_nn, dim3((unsigned)((m + 15) / 16), (unsigned)((nn + 15) / 16)), dim3(256), 0, s, A,
                     lda, B, ldb, m, nn, kk, Out, ldo);
  return hipGetLastError();
}

}  // namespace rb

extern "C" {

int rb_reconstruct_z(const void* E_, int64_t N, int64_t j, int64_t ldE, const void* C_, int64_t M, int64_t ldC,
                     double tau2, void* X_, int64_t ldX, double* sigma, void* Vout, int64_t* k_out,
                     hipStream_t stream) {
  last_error().clear();
  if (!E_ || !C_ || !X_ || !sigma || !k_out || N <= 0 || j <= 0 || M <= 0 || j > N || j > 2 * kMaxPairs ||
      !valid_ld(N, ldE) || ldC < j || !valid_ld(N, ldX) || !(tau2 >= 0.0) || !std::isfinite(tau2))
    return set_error(RB_EINVAL, "rb_reconstruct_z: bad arguments");
  const double2* E = static_cast<const double2*>(E_);
  const double2* C = static_cast<const double2*>(C_);
  double2* X = static_cast<double2*>(X_);
  const int ntile = (int)((j + kGT - 1) / kGT);
  const int ntp = ntile * (ntile + 1) / 2;
  const int ns = gram_splits(j, M);
  const size_t jj = (size_t)j * (size_t)j;

  DevBuf P, G, V0, V1, V, B, d_sig, d_perm, d_info;
  RB_ALLOC(P, sizeof(double2) * (size_t)ns * ntp * kGT * kGT);
  RB_ALLOC(G, sizeof(double2) * jj);
  RB_ALLOC(V0, sizeof(double2) * jj);
  RB_ALLOC(V1, sizeof(double2) * jj);
  RB_ALLOC(V, sizeof(double2) * jj);
  RB_ALLOC(B, sizeof(double2) * (size_t)j * (size_t)M);
  RB_ALLOC(d_sig, sizeof(double) * j);
  RB_ALLOC(d_perm, sizeof(int64_t) * j);
  RB_ALLOC(d_info, sizeof(int) * 2);
  const double eps = 4.0 * 0x1p-53;
  const int max_sweeps = 60;

  // 1. G = C C^H and its Jacobi eigenvectors V0
  RB_HIP(gram(C, j, M, ldC, P.as<double2>(), ns, G.as<double2>(), stream));
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kJT), 0, stream, G.as<double2>(), j, V0.as<double2>(), max_sweeps, eps,
                     d_info.as<int>());
  RB_HIP(hipGetLastError());
  // 2. refinement: B = V0^H C, G2 = B B^H, Jacobi -> V1, lambda
  RB_HIP(launch_project_z(V0.as<double2>(), j, j, j, C, M, ldC, B.as<double2>(), j, stream));
  RB_HIP(gram(B.as<double2>(), j, M, j, P.as<double2>(), ns, G.as<double2>(), stream));
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kJT), 0, stream, G.as<double2>(), j, V1.as<double2>(), max_sweeps, eps,
                     d_info.as<int>() + 1);
  RB_HIP(hipGetLastError());
  // 3. V = V0 V1, ordered by descending eigenvalue
  RB_HIP(gemm_nn(V0.as<double2>(), j, V1.as<double2>(), j, j, j, j, V.as<double2>(), j, stream));
  hipLaunchKernelGGL(k_eig_order, dim3((unsigned)((j + 255) / 256)), dim3(256), 0, stream, G.as<double2>(), j,
                     d_sig.as<double>(), d_perm.as<int64_t>());
  RB_HIP(hipGetLastError());
  int info[2];
  RB_HIP(hipMemcpyAsync(info, d_info.p, sizeof info, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipMemcpyAsync(sigma, d_sig.p, sizeof(double) * j, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  if (info[0] < 0 || info[1] < 0) return set_error(RB_ENOCONV, "rb_reconstruct_z: Jacobi did not converge");
  for (int64_t i = 0; i < j; ++i)
    if (!std::isfinite(sigma[i])) return set_error(RB_ENONFINITE, "rb_reconstruct_z: non-finite singular value");
  // 4. k = #{sigma_i >= tau2}; X_k = E V(:, 1:k)
  int64_t k = 0;
  while (k < j && sigma[k] >= tau2) ++k;
  double2* Vs = Vout ? static_cast<double2*>(Vout) : V1.as<double2>();  // V1 is free now
  hipLaunchKernelGGL(k_permute_cols, dim3((unsigned)((jj + 255) / 256)), dim3(256), 0, stream, V.as<double2>(), j,
                     j, d_perm.as<int64_t>(), j, Vs, j);
  RB_HIP(hipGetLastError());
  RB_HIP(gemm_nn(E, ldE, Vs, j, N, k, j, X, ldX, stream));
  RB_HIP(hipStreamSynchronize(stream));
  *k_out = k;
  return RB_OK;
}

}  // extern "C"

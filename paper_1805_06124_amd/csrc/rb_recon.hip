// The reconstruction algorithm (Alg. 4, Sec. 5.2.2; Theorem 5.8): after the
// greedy has produced Q_j and R(1:j, :) = Q_j^H S Pi, take the SVD of
// R(1:j, :) = V Sigma W^H, keep the k singular values >= tau2 and return
// X_k = Q_j V(:, 1:k).  The rows of R are the coefficients C = E^H S up to
// the column order, which changes neither the singular values nor V.
//
// The SVD's left factor on the GPU:
//   1. G = C C^H (j x j, FP64 matrix cores, split over the M columns,
//      partial sums added in a fixed order);
//   2. V0 = eigenvectors of G by cyclic Jacobi in parallel (round-robin)
//      order.  A rotation is skipped when |G_pq| <= eps sqrt(G_pp G_qq), the
//      relative test.  For j <= 141 the matrix lives in one CU's LDS and the
//      rotations are logged and multiplied out afterwards; larger j use a
//      global-memory solve;
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

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kGT = 32;   // Gram tile (rows of C per side)
constexpr int kGK = 16;   // columns of C staged per step

// Partial Gram tiles on FP64 matrix cores (v_mfma_f64_16x16x4f64): for tile
// pair tp = (ti >= tl) and column split sp,
// P[(sp * ntp + tp) * kGT^2 + a * kGT + b] = sum over m in the split of
// C[ti*kGT + a, m] conj(C[tl*kGT + b, m]).  Four waves, each a 16 x 16
// quarter of the tile; the reduction runs over m in LDS-staged chunks of 16
// columns (stored [m][row]), the next chunk loaded into registers while the
// matrix cores work on the current one.  MFMA operands (64 lanes):
// A(16x4) lane l holds A[l%16][l/16], B(4x16) lane l holds B[l/16][l%16],
// result lane l register r holds D[l/16 + 4r][l%16].
//   c_i conj(c_l):  re = ri rl + ii il,  im = ii rl - ri il
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
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wi = (wave >> 1) * 16, wl = (wave & 1) * 16;
  const int64_t i0 = (int64_t)ti * kGT, l0 = (int64_t)tl * kGT;
  // staging: thread t takes row t % 32 of columns t / 32 and t / 32 + 8
  const int sr = t & (kGT - 1), sc = t / kGT;
  d4v accr = (d4v){0.0, 0.0, 0.0, 0.0}, acci = (d4v){0.0, 0.0, 0.0, 0.0};
  double2 av[2], bv[2];
  auto load = [&](int64_t mb) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int64_t m = mb + sc + 8 * q;
      const bool okm = m < m1;
      av[q] = (okm && i0 + sr < j) ? C[(i0 + sr) + m * ldC] : make_double2(0.0, 0.0);
      bv[q] = (okm && l0 + sr < j) ? C[(l0 + sr) + m * ldC] : make_double2(0.0, 0.0);
    }
  };
  if (m0 < m1) load(m0);
  for (int64_t mb = m0; mb < m1; mb += kGK) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      sA[sc + 8 * q][sr] = av[q];
      sB[sc + 8 * q][sr] = bv[q];
    }
    __syncthreads();
    if (mb + kGK < m1) load(mb + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      const int r = kk + (lane >> 4);
      const double2 a = sA[r][wi + (lane & 15)];
      const double2 b = sB[r][wl + (lane & 15)];
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, accr, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acci, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.x, b.y, acci, 0, 0, 0);
    }
    __syncthreads();
  }
  double2* out = P + ((int64_t)blockIdx.y * ntp + tp) * (kGT * kGT);
#pragma unroll
  for (int r = 0; r < 4; ++r) out[(wi + (lane >> 4) + 4 * r) * kGT + wl + (lane & 15)] = make_double2(accr[r], acci[r]);
}

// G (j x j, ld j, full Hermitian) from the partials, splits added in order;
// one thread per element of a tile pair.  Element (i, l) with i >= l is
// summed once; G[l, i] is its conjugate and the diagonal is real.
__global__ __launch_bounds__(256) void k_gram_reduce(const double2* __restrict__ P, int ns, int ntp, int64_t j,
                                                     double2* __restrict__ G) {
  const int tp = blockIdx.x;
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= tp) ++ti;
  const int tl = tp - ti * (ti + 1) / 2;
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= kGT * kGT) return;
  const int a = e / kGT, b = e % kGT;
  const int64_t i = (int64_t)ti * kGT + a, l = (int64_t)tl * kGT + b;
  if (i >= j || l >= j || i < l) return;
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

// Round-robin pairing shared by the Jacobi kernels: in round r of a sweep
// (npr = n rounded up to even, npr - 1 rounds) slot i pairs p < q; q >= n is
// the dummy index of odd n.
__device__ __forceinline__ void rr_pair(int r, int i, int npr, int& p, int& q) {
  const int R = npr - 1;
  if (i == 0) {
    p = r;
    q = R;
  } else {
    p = r + i;
    if (p >= R) p -= R;
    q = r - i;
    if (q < 0) q += R;
  }
  if (p > q) {
    const int tmp = p;
    p = q;
    q = tmp;
  }
}

// Rotation of the pair (p, q) that zeroes G_pq (a = G_pp, d = G_qq, b =
// G_pq): J = [[c, s], [-s conj(ph), c conj(ph)]] with ph = b / |b|,
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (d - a) / (2 |b|),
// c = 1 / sqrt(1 + t^2), s = t c; afterwards G_pp = a - t |b|,
// G_qq = d + t |b|.  Skipped (returns false) when |b| <= eps sqrt(|a d|).
__device__ __forceinline__ bool jacobi_rot(double a, double d, double2 b, double eps, double& c, double& s,
                                           double2& ph, double& tb) {
  double ab = sqrt(b.x * b.x + b.y * b.y);
  if (!(ab > 0x1p-480 && ab < 0x1p480)) ab = hypot(b.x, b.y);  // squares out of range
  if (!(ab > 0.0 && ab > eps * sqrt(fabs(a * d)))) return false;
  const double rab = 1.0 / ab;
  const double zeta = 0.5 * (d - a) * rab;
  const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  c = 1.0 / sqrt(1.0 + tt * tt);
  s = tt * c;
  ph = make_double2(b.x * rab, b.y * rab);
  tb = tt * ab;
  return true;
}

// Workgroup barrier that orders LDS only: the rotation log's global stores
// are never read back inside the solve, so the barrier need not wait for them.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Cyclic Jacobi with the matrix resident in LDS (n <= kLdsN: the lower
// triangle of n x n complex FP64 values fills the 160 KB of one CU).  Each
// round's n/2 rotations touch disjoint pairs, so the update splits into
// independent 2 x 2 blocks: block (i, i') of rows {p_i, q_i} and columns
// {p_i', q_i'} becomes J_i^H B J_i', and the diagonal block of an active
// pair becomes diag(a - t|b|, d + t|b|).  Every stored entry belongs to
// exactly one block, so a round is one barrier for the rotation parameters
// and one for the update.  The eigenvectors are not formed here: every
// round's rotations are appended to rot (identity for skipped pairs) and
// k_apply_rot multiplies them out afterwards, which keeps the sequential
// loop in LDS.  On exit G (full, ld n) holds the rotated matrix (its
// diagonal the eigenvalues) and info the sweeps used (the last one
// rotation-free), or -1 if max_sweeps passed without a rotation-free sweep.
constexpr int kLdsN = 141;
constexpr int kLdsHalf = (kLdsN + 1) / 2;
constexpr int kLdsTri = kLdsN * (kLdsN + 1) / 2;
constexpr int kLdsT = 1024;
constexpr int kLdsBlk = (kLdsHalf * (kLdsHalf + 1) / 2 + kLdsT - 1) / kLdsT;  // blocks per thread

__device__ __forceinline__ int tri(int r, int c) { return r * (r + 1) / 2 + c; }  // r >= c

__global__ __launch_bounds__(kLdsT) void k_jacobi_lds(double2* __restrict__ G, int n, double4* __restrict__ rot,
                                                      int max_sweeps, double eps, int* __restrict__ info) {
  __shared__ double2 g[kLdsTri];
  __shared__ double4 sj[kLdsHalf];  // c, s, ph of each slot's rotation
  __shared__ double stb[kLdsHalf];  // t |b|
  __shared__ int spq[kLdsHalf];     // p | q << 8 | active << 16
  __shared__ int rotated;
  const int t = threadIdx.x;
  for (int r = 0; r < n; ++r)
    for (int c = t; c <= r; c += kLdsT) g[tri(r, c)] = G[r + (int64_t)c * n];
  __syncthreads();
  const int npr = n + (n & 1), half = npr / 2, R = npr - 1;
  // this thread's blocks (i >= i'), fixed for the whole solve
  const int nb = half * (half + 1) / 2;
  int bi[kLdsBlk], bj[kLdsBlk];
#pragma unroll
  for (int u = 0; u < kLdsBlk; ++u) {
    const int e = t + u * kLdsT;
    bi[u] = -1;
    bj[u] = 0;
    if (e < nb) {
      int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while (i * (i + 1) / 2 > e) --i;
      while ((i + 1) * (i + 2) / 2 <= e) ++i;
      bi[u] = i;
      bj[u] = e - i * (i + 1) / 2;
    }
  }
  // entry (r, c) of the Hermitian matrix: stored at tri(max, min), conjugated
  // when r < c
  auto get = [&](int r, int c) -> double2 {
    const bool lo = r >= c;
    const double2 v = g[lo ? tri(r, c) : tri(c, r)];
    return make_double2(v.x, lo ? v.y : -v.y);
  };
  auto put = [&](int r, int c, double2 v) {
    const bool lo = r >= c;
    g[lo ? tri(r, c) : tri(c, r)] = make_double2(v.x, lo ? v.y : -v.y);
  };
  int sweep = 0;
  bool done = false;
  for (; sweep < max_sweeps && !done; ++sweep) {
    if (t == 0) rotated = 0;
    lds_barrier();
    for (int r = 0; r < R; ++r) {
      if (t < half) {
        int p, q;
        rr_pair(r, t, npr, p, q);
        double c = 1.0, s = 0.0, tb = 0.0;
        double2 ph = make_double2(1.0, 0.0);
        bool act = false;
        if (q < n) {
          const double2 bl = g[tri(q, p)];  // G_qp = conj(G_pq)
          act = jacobi_rot(g[tri(p, p)].x, g[tri(q, q)].x, make_double2(bl.x, -bl.y), eps, c, s, ph, tb);
        }
        const double4 J = make_double4(c, s, ph.x, ph.y);
        sj[t] = J;
        stb[t] = tb;
        spq[t] = p | (q << 8) | (act ? 1 << 16 : 0);
        if (act) rotated = 1;
        rot[((int64_t)sweep * R + r) * half + t] = J;
      }
      lds_barrier();
#pragma unroll
      for (int u = 0; u < kLdsBlk; ++u) {
        const int i = bi[u], i2 = bj[u];
        if (i < 0) continue;
        const int w1 = spq[i], w2 = spq[i2];
        const bool ai = (w1 >> 16) != 0, aj = (w2 >> 16) != 0;
        if (!ai && !aj) continue;
        const int p = w1 & 255, q = (w1 >> 8) & 255;
        if (i == i2) {  // diagonal block of an active pair
          const double tb = stb[i];
          g[tri(p, p)] = make_double2(g[tri(p, p)].x - tb, 0.0);
          g[tri(q, q)] = make_double2(g[tri(q, q)].x + tb, 0.0);
          g[tri(q, p)] = make_double2(0.0, 0.0);
          continue;
        }
        const int p2 = w2 & 255, q2 = (w2 >> 8) & 255;
        const bool hq = q < n, hq2 = q2 < n;  // the dummy row / column is absent
        double2 x11 = get(p, p2);
        double2 x12 = hq2 ? get(p, q2) : make_double2(0.0, 0.0);
        double2 x21 = hq ? get(q, p2) : make_double2(0.0, 0.0);
        double2 x22 = (hq && hq2) ? get(q, q2) : make_double2(0.0, 0.0);
        if (aj) {  // columns: [x_p', x_q'] <- [x_p', x_q'] J'
          const double4 J = sj[i2];
          const double c = J.x, s = J.y;
          const double2 y1 = make_double2(x12.x * J.z + x12.y * J.w, x12.y * J.z - x12.x * J.w);
          const double2 y2 = make_double2(x22.x * J.z + x22.y * J.w, x22.y * J.z - x22.x * J.w);
          const double2 n11 = make_double2(c * x11.x - s * y1.x, c * x11.y - s * y1.y);
          const double2 n12 = make_double2(s * x11.x + c * y1.x, s * x11.y + c * y1.y);
          const double2 n21 = make_double2(c * x21.x - s * y2.x, c * x21.y - s * y2.y);
          const double2 n22 = make_double2(s * x21.x + c * y2.x, s * x21.y + c * y2.y);
          x11 = n11;
          x12 = n12;
          x21 = n21;
          x22 = n22;
        }
        if (ai) {  // rows: [y_p; y_q] <- J^H [y_p; y_q]
          const double4 J = sj[i];
          const double c = J.x, s = J.y;
          const double2 z1 = make_double2(x21.x * J.z - x21.y * J.w, x21.x * J.w + x21.y * J.z);
          const double2 z2 = make_double2(x22.x * J.z - x22.y * J.w, x22.x * J.w + x22.y * J.z);
          const double2 n11 = make_double2(c * x11.x - s * z1.x, c * x11.y - s * z1.y);
          const double2 n21 = make_double2(s * x11.x + c * z1.x, s * x11.y + c * z1.y);
          const double2 n12 = make_double2(c * x12.x - s * z2.x, c * x12.y - s * z2.y);
          const double2 n22 = make_double2(s * x12.x + c * z2.x, s * x12.y + c * z2.y);
          x11 = n11;
          x12 = n12;
          x21 = n21;
          x22 = n22;
        }
        put(p, p2, x11);
        if (hq2) put(p, q2, x12);
        if (hq) put(q, p2, x21);
        if (hq && hq2) put(q, q2, x22);
      }
      lds_barrier();
    }
    done = (rotated == 0);
    lds_barrier();
  }
  for (int r = 0; r < n; ++r)
    for (int c = t; c <= r; c += kLdsT) {
      const double2 v = g[tri(r, c)];
      G[r + (int64_t)c * n] = v;
      G[c + (int64_t)r * n] = make_double2(v.x, -v.y);
    }
  if (t == 0) *info = done ? sweep : -1;
}

// V = J_1 J_2 ... J_T (n x n, ld n) from the rotation log of k_jacobi_lds:
// row rho of V starts as e_rho^T and every round updates its pairs,
// [v_p, v_q] <- [v_p, v_q] J.  One wave per row with the row in LDS (a
// wave's LDS accesses complete in order, so the rounds need no barrier);
// the workgroup's four waves share the log, staged kRotStage rounds at a
// time and double-buffered.  Rounds: info sweeps (all logged sweeps when
// info < 0).
constexpr int kRotStage = 8;

__global__ __launch_bounds__(256) void k_apply_rot(const double4* __restrict__ rot, const int* __restrict__ info,
                                                   int max_sweeps, int n, double2* __restrict__ V) {
  __shared__ double2 row[4][kLdsN + 1];
  __shared__ double4 st[2][kRotStage * kLdsHalf];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int rho = blockIdx.x * 4 + wave;
  const int npr = n + (n & 1), half = npr / 2, R = npr - 1;
  const int sweeps = (*info >= 0) ? *info : max_sweeps;
  const int64_t rounds = (int64_t)sweeps * R;
  for (int c = lane; c < n; c += 64) row[wave][c] = make_double2(c == rho ? 1.0 : 0.0, 0.0);
  auto stage = [&](int64_t r0, int buf) {
    const int64_t nr = rounds - r0 < kRotStage ? rounds - r0 : kRotStage;
    for (int e = t; e < nr * half; e += 256) st[buf][e] = rot[r0 * half + e];
  };
  if (rounds > 0) stage(0, 0);
  __syncthreads();
  int buf = 0;
  for (int64_t r0 = 0; r0 < rounds; r0 += kRotStage, buf ^= 1) {
    if (r0 + kRotStage < rounds) stage(r0 + kRotStage, buf ^ 1);
    const int64_t nr = rounds - r0 < kRotStage ? rounds - r0 : kRotStage;
    if (rho < n) {
      int r = (int)(r0 % R);
      for (int64_t rr = 0; rr < nr; ++rr, r = (r + 1 == R) ? 0 : r + 1) {
        for (int i = lane; i < half; i += 64) {
          int p, q;
          rr_pair(r, i, npr, p, q);
          if (q >= n) continue;
          const double4 J = st[buf][rr * half + i];
          if (J.y == 0.0 && J.z == 1.0 && J.w == 0.0) continue;  // skipped pair: identity
          const double2 vp = row[wave][p], vq = row[wave][q];
          const double2 y = make_double2(vq.x * J.z + vq.y * J.w, vq.y * J.z - vq.x * J.w);  // vq conj(ph)
          row[wave][p] = make_double2(J.x * vp.x - J.y * y.x, J.x * vp.y - J.y * y.y);
          row[wave][q] = make_double2(J.y * vp.x + J.x * y.x, J.y * vp.y + J.x * y.y);
        }
      }
    }
    __syncthreads();
  }
  if (rho < n)
    for (int c = lane; c < n; c += 64) V[rho + (int64_t)c * n] = row[wave][c];
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

// Out (m x nn) = A (m x kk) B (kk x nn), complex, column-major, on FP64
// matrix cores.  A workgroup owns 64 rows x 32 columns; wave w the rows
// 16w..16w+15 as two 16 x 16 MFMA tiles; the reduction runs over kk in
// LDS-staged chunks of 16.   a b:  re = ar br - ai bi,  im = ar bi + ai br
__global__ __launch_bounds__(256) void k_gemm_nn(const double2* __restrict__ A, int64_t lda,
                                                 const double2* __restrict__ B, int64_t ldb, int64_t m, int64_t nn,
                                                 int64_t kk, double2* __restrict__ Out, int64_t ldo) {
  __shared__ double2 sA[16][64 + 1];
  __shared__ double2 sB[16][32 + 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 32;
  d4v accr[2] = {(d4v){0.0, 0.0, 0.0, 0.0}, (d4v){0.0, 0.0, 0.0, 0.0}};
  d4v acci[2] = {(d4v){0.0, 0.0, 0.0, 0.0}, (d4v){0.0, 0.0, 0.0, 0.0}};
  for (int64_t k0 = 0; k0 < kk; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // A: 64 rows x 16 k, lanes along rows
      const int e = t + 256 * q, r = e & 63, k = e >> 6;
      sA[k][r] = (r0 + r < m && k0 + k < kk) ? A[(r0 + r) + (k0 + k) * lda] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {  // B: 16 k x 32 columns, lanes along k
      const int e = t + 256 * q, k = e & 15, c = e >> 4;
      sB[k][c] = (k0 + k < kk && c0 + c < nn) ? B[(k0 + k) + (c0 + c) * ldb] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k += 4) {
      const double2 a = sA[k + (lane >> 4)][16 * wave + (lane & 15)];
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
        const double2 b = sB[k + (lane >> 4)][16 * tb + (lane & 15)];
        accr[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, accr[tb], 0, 0, 0);
        accr[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, accr[tb], 0, 0, 0);
        acci[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, acci[tb], 0, 0, 0);
        acci[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acci[tb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int tb = 0; tb < 2; ++tb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 16 * wave + (lane >> 4) + 4 * r, col = c0 + 16 * tb + (lane & 15);
      if (row < m && col < nn) Out[row + col * ldo] = make_double2(accr[tb][r], acci[tb][r]);
    }
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
  hipLaunchKernelGGL(k_gram_reduce, dim3(ntp, (kGT * kGT + 255) / 256), dim3(256), 0, s, P, nsu, ntp, j, G);
  return hipGetLastError();
}

static int gram_splits(int64_t j, int64_t M) {
  const int ntile = (int)((j + kGT - 1) / kGT);
  const int ntp = ntile * (ntile + 1) / 2;
  int ns = std::max(1, 2048 / ntp);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, (M + 1023) / 1024));
  return std::min(ns, 256);
}

// Eigenvectors V (ld n) of the Hermitian G (overwritten, diagonal = the
// eigenvalues); info: sweeps used or -1.  The LDS-resident solve with a
// rotation log (rot: max_sweeps (n + 1) (n + 1) / 2 double4, rounded up to
// even n) when n fits one CU's LDS, else the global-memory solve.
static size_t jacobi_log_count(int64_t n, int max_sweeps) {
  const int64_t npr = n + (n & 1);
  return n <= kLdsN ? (size_t)max_sweeps * (size_t)(npr - 1) * (size_t)(npr / 2) : 0;
}
static hipError_t jacobi(double2* G, int64_t n, double2* V, double4* rot, int max_sweeps, double eps, int* info,
                         hipStream_t s) {
  if (n <= kLdsN) {
    hipLaunchKernelGGL(k_jacobi_lds, dim3(1), dim3(kLdsT), 0, s, G, (int)n, rot, max_sweeps, eps, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_apply_rot, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, rot, info, max_sweeps, (int)n,
                       V);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kJT), 0, s, G, n, V, max_sweeps, eps, info);
  return hipGetLastError();
}

static hipError_t gemm_nn(const double2* A, int64_t lda, const double2* B, int64_t ldb, int64_t m, int64_t nn,
                          int64_t kk, double2* Out, int64_t ldo, hipStream_t s) {
  if (m <= 0 || nn <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_nn, dim3((unsigned)((m + 63) / 64), (unsigned)((nn + 31) / 32)), dim3(256), 0, s, A,
                     lda, B, ldb, m, nn, kk, Out, ldo);
  return hipGetLastError();
}

}  // namespace rb

// The reconstruction's device buffers, carved from one workspace (the same
// sequence of take() calls sizes it and lays it out).
struct ReconBufs {
  double2 *P, *G, *V0, *V1, *V, *B;
  double* sig;
  int64_t* perm;
  int* info;
  double4* rot;
};
constexpr double kReconEps = 4.0 * 0x1p-53;
constexpr int kReconSweeps = 60;

static bool recon_sizes_ok(int64_t j, int64_t M) { return j >= 1 && j <= 2 * kMaxPairs && M >= 1; }

static size_t recon_carve(void* base, int64_t j, int64_t M, ReconBufs& b) {
  const int ntile = (int)((j + kGT - 1) / kGT);
  const int ntp = ntile * (ntile + 1) / 2;
  const int ns = gram_splits(j, M);
  const size_t jj = (size_t)j * (size_t)j;
  Carve c(base);
  b.P = c.take<double2>((size_t)ns * ntp * kGT * kGT);
  b.G = c.take<double2>(jj);
  b.V0 = c.take<double2>(jj);
  b.V1 = c.take<double2>(jj);
  b.V = c.take<double2>(jj);
  b.B = c.take<double2>((size_t)j * (size_t)M);
  b.sig = c.take<double>(j);
  b.perm = c.take<int64_t>(j);
  b.info = c.take<int>(2);
  const size_t nrot = jacobi_log_count(j, kReconSweeps);
  b.rot = nrot ? c.take<double4>(nrot) : nullptr;
  return c.used;
}

extern "C" {

size_t rb_reconstruct_z_workspace(int64_t j, int64_t M) {
  if (!recon_sizes_ok(j, M)) return 0;
  ReconBufs b;
  return recon_carve(nullptr, j, M, b);
}

int rb_reconstruct_z(const void* E_, int64_t N, int64_t j, int64_t ldE, const void* C_, int64_t M, int64_t ldC,
                     double tau2, void* X_, int64_t ldX, double* sigma, void* Vout, int64_t* k_out, void* ws,
                     size_t ws_bytes, hipStream_t stream) {
  last_error().clear();
  if (!E_ || !C_ || !X_ || !sigma || !k_out || N <= 0 || !recon_sizes_ok(j, M) || j > N || !valid_ld(N, ldE) ||
      ldC < j || !valid_ld(N, ldX) || !(tau2 >= 0.0) || !std::isfinite(tau2))
    return set_error(RB_EINVAL, "rb_reconstruct_z: bad arguments");
  const double2* E = static_cast<const double2*>(E_);
  const double2* C = static_cast<const double2*>(C_);
  double2* X = static_cast<double2*>(X_);
  const int ns = gram_splits(j, M);
  const size_t jj = (size_t)j * (size_t)j;

  ReconBufs b;
  const size_t need = recon_carve(nullptr, j, M, b);
  DevBuf own;
  if (ws) {
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
      return set_error(RB_EINVAL, "rb_reconstruct_z: workspace not 256-byte aligned");
    if (ws_bytes < need)
      return set_error(RB_ENOMEM, "rb_reconstruct_z: workspace of %zu bytes, %zu needed", ws_bytes, need);
  } else {
    RB_ALLOC(own, need);
    ws = own.p;
  }
  recon_carve(ws, j, M, b);

  // 1. G = C C^H and its Jacobi eigenvectors V0
  RB_HIP(gram(C, j, M, ldC, b.P, ns, b.G, stream));
  RB_HIP(jacobi(b.G, j, b.V0, b.rot, kReconSweeps, kReconEps, b.info, stream));
  // 2. refinement: B = V0^H C, G2 = B B^H, Jacobi -> V1, lambda
  RB_HIP(launch_project_z(b.V0, j, j, j, C, M, ldC, b.B, j, stream));
  RB_HIP(gram(b.B, j, M, j, b.P, ns, b.G, stream));
  RB_HIP(jacobi(b.G, j, b.V1, b.rot, kReconSweeps, kReconEps, b.info + 1, stream));
  // 3. V = V0 V1, ordered by descending eigenvalue
  RB_HIP(gemm_nn(b.V0, j, b.V1, j, j, j, j, b.V, j, stream));
  hipLaunchKernelGGL(k_eig_order, dim3((unsigned)((j + 255) / 256)), dim3(256), 0, stream, b.G, j, b.sig, b.perm);
  RB_HIP(hipGetLastError());
  int info[2];
  RB_HIP(hipMemcpyAsync(info, b.info, sizeof info, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipMemcpyAsync(sigma, b.sig, sizeof(double) * j, hipMemcpyDeviceToHost, stream));
  RB_HIP(hipStreamSynchronize(stream));
  if (info[0] < 0 || info[1] < 0) return set_error(RB_ENOCONV, "rb_reconstruct_z: Jacobi did not converge");
  for (int64_t i = 0; i < j; ++i)
    if (!std::isfinite(sigma[i])) return set_error(RB_ENONFINITE, "rb_reconstruct_z: non-finite singular value");
  // 4. k = #{sigma_i >= tau2}; X_k = E V(:, 1:k)
  int64_t k = 0;
  while (k < j && sigma[k] >= tau2) ++k;
  double2* Vs = Vout ? static_cast<double2*>(Vout) : b.V1;  // V1 is free now
  hipLaunchKernelGGL(k_permute_cols, dim3((unsigned)((jj + 255) / 256)), dim3(256), 0, stream, b.V, j, j, b.perm, j,
                     Vs, j);
  RB_HIP(hipGetLastError());
  RB_HIP(gemm_nn(E, ldE, Vs, j, N, k, j, X, ldX, stream));
  RB_HIP(hipStreamSynchronize(stream));
  *k_out = k;
  return RB_OK;
}

}  // extern "C"

// Dense complex FP64 products of the greedy:
//   project : C = E^H S  (k x M), the coefficients of every snapshot on the
//             basis (the projection E E^H s of Sec. 4), on FP64 matrix cores
//             (v_mfma_f64_16x16x4f64);
//   resid   : W = X - E C (N x M) with exact norms of the result, the
//             explicit re-anchoring of the working columns onto their
//             residuals against m basis vectors, i.e. the stored-residual
//             form of the greedy (the residual matrix V of Alg. 2;
//             Remark 5.5).
#include "rb_internal.h"

namespace rb {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------- project --
// C = E^H S.  A workgroup owns a block of 32*kTA basis vectors (i) x 64
// columns (j); 4 waves as 2 x 2, each wave 16*kTA x 32 = kTA x 2 MFMA 16x16
// tiles.  With kTA up to 7 a block covers k <= 224, so S is read once.  The
// reduction runs over rows n in chunks of 16 staged through LDS as
// [n][col]; the next chunk is loaded into registers while the matrix cores
// work on the current one.
//
// v_mfma_f64_16x16x4f64 operand layout (64 lanes): A(16x4) lane l holds
// A[l%16][l/16]; B(4x16) lane l holds B[l/16][l%16]; the 16x16 result
// lane l, register r holds D[l/16 + 4r][l%16].
//   conj(e) s:  re = er sr + ei si,  im = er si - ei sr
constexpr int kPJ = 64;  // columns per block
constexpr int kPK = 16;  // rows per LDS chunk

template <int kTA>
__global__ __launch_bounds__(256) void k_project_z(const double2* __restrict__ E, int64_t N, int64_t k, int64_t ldE,
                                                   const double2* __restrict__ S, int64_t M, int64_t ldS,
                                                   double2* __restrict__ C, int64_t ldC) {
  constexpr int kTI = 32 * kTA;                      // basis vectors per block
  constexpr int kQE = (kPK * kTI) / 256;             // staged E values per thread
  constexpr int kQS = (kPK * kPJ) / 256;             // staged S values per thread
  __shared__ double2 sE[kPK][kTI + 1];
  __shared__ double2 sS[kPK][kPJ + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * kPJ;
  const int64_t i0 = (int64_t)blockIdx.y * kTI;
  const int wi = (wave >> 1) * (16 * kTA), wj = (wave & 1) * 32;

  d4v accr[kTA][2], acci[kTA][2];
#pragma unroll
  for (int a = 0; a < kTA; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
      acci[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
    }
  // thread t stages row (t % 16) of columns t / 16 + 16 q
  const int rr = tid % kPK, cc = tid / kPK;
  double2 ev[kQE], sv[kQS];
  auto load = [&](int64_t n0) {
    const int64_t n = n0 + rr;
#pragma unroll
    for (int q = 0; q < kQE; ++q) {
      const int64_t i = i0 + cc + 16 * q;
      ev[q] = (n < N && i < k) ? E[n + i * ldE] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < kQS; ++q) {
      const int64_t j = j0 + cc + 16 * q;
      sv[q] = (n < N && j < M) ? ld_stream(S + n + j * ldS) : make_double2(0.0, 0.0);
    }
  };
  load(0);
  for (int64_t n0 = 0; n0 < N; n0 += kPK) {
#pragma unroll
    for (int q = 0; q < kQE; ++q) sE[rr][cc + 16 * q] = ev[q];
#pragma unroll
    for (int q = 0; q < kQS; ++q) sS[rr][cc + 16 * q] = sv[q];
    __syncthreads();
    if (n0 + kPK < N) load(n0 + kPK);
#pragma unroll
    for (int kk = 0; kk < kPK; kk += 4) {
      const int r = kk + (lane >> 4);
      double2 a[kTA], b[2];
#pragma unroll
      for (int t = 0; t < kTA; ++t) a[t] = sE[r][wi + 16 * t + (lane & 15)];
#pragma unroll
      for (int t = 0; t < 2; ++t) b[t] = sS[r][wj + 16 * t + (lane & 15)];
#pragma unroll
      for (int ta = 0; ta < kTA; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
          accr[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, b[tb].x, accr[ta][tb], 0, 0, 0);
          accr[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].y, b[tb].y, accr[ta][tb], 0, 0, 0);
          acci[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, b[tb].y, acci[ta][tb], 0, 0, 0);
          acci[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[ta].y, b[tb].x, acci[ta][tb], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int ta = 0; ta < kTA; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi + 16 * ta + (lane >> 4) + 4 * r;
        const int64_t j = j0 + wj + 16 * tb + (lane & 15);
        if (i < k && j < M) C[i + j * ldC] = make_double2(accr[ta][tb][r], acci[ta][tb][r]);
      }
}

// ------------------------------------------------------------- residual --
// Explicit re-anchoring of a block of working columns:
//   W[:, j] = X[:, j] - E[:, 0:m] C(0:m, j),  nrm[j] = ||W[:, j]||^2
// with C(i, j) = C[i*cI + j*cJ].  X and W may alias (in-place); W == NULL
// computes the norms only.  The norm is that of the stored W values (after
// rounding to the output type), summed
// in FP64 (relative error ~ N u of the anchored norm itself, far below what
// the pivot search resolves).
//
// One workgroup owns a strip of 64 columns and walks down all rows in 64-row
// tiles, so each column's norm is finished inside the workgroup (no partial
// buffers, deterministic).  The next chunk of E (and C) is loaded into
// registers while the matrix cores work on the current one; with m <= 16
// the C tile is staged once for the whole strip.  The product E C for a row tile runs on FP64
// matrix cores: 4 waves as 2 x 2, each 32 x 32 = 2 x 2 MFMA 16x16 tiles,
// the reduction over basis vectors in LDS-staged chunks of 16.
//   E C, complex:  re = Er Cr - Ei Ci,  im = Er Ci + Ei Cr.
constexpr int kRT = 64;   // rows per tile, columns per strip
constexpr int kRK = 16;   // basis vectors per LDS chunk

__device__ __forceinline__ double2 ld_x(const double2* p) { return ld_stream(p); }
__device__ __forceinline__ double2 ld_x(const float2* p) {
  float2 v = ld_stream(p);
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 st_w(double2* p, double re, double im) {
  *p = make_double2(re, im);
  return make_double2(re, im);
}
__device__ __forceinline__ double2 st_w(float2* p, double re, double im) {
  float2 v = make_float2((float)re, (float)im);
  *p = v;
  return make_double2((double)v.x, (double)v.y);
}

// kVec (complex64 X only): the epilogue moves two consecutive rows per lane
// with 16-byte accesses (X, and W when written, 16-byte aligned with even
// leading dimensions); otherwise one row per lane.
template <class XT, class WT, bool kVec>
__global__ __launch_bounds__(256) void k_resid(const XT* X, int64_t ldX, WT* W, int64_t ldW, int64_t N, int64_t M,
                                               const double2* __restrict__ E, int64_t ldE, int64_t m,
                                               const double2* __restrict__ Cc, int64_t cI, int64_t cJ,
                                               double* __restrict__ nrm, int* __restrict__ bad) {
  // LDS: the staging chunks of E and C, reused as a half tile (32 columns x
  // 64 rows) of the product for a coalesced epilogue.
  constexpr int kStage = 2 * kRK * (kRT + 1);
  constexpr int kHalf = (kRT / 2) * (kRT + 1);
  __shared__ double2 smem[kStage > kHalf ? kStage : kHalf];
  __shared__ double2 sC1[kRK][kRT + 1];  // C tile when m <= kRK (staged once)
  double2 (*sE)[kRT + 1] = reinterpret_cast<double2 (*)[kRT + 1]>(smem);
  double2 (*sC)[kRT + 1] = reinterpret_cast<double2 (*)[kRT + 1]>(smem + kRK * (kRT + 1));
  double2 (*sD)[kRT + 1] = reinterpret_cast<double2 (*)[kRT + 1]>(smem);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t j0 = (int64_t)blockIdx.x * kRT;
  const bool one_chunk = m <= kRK;
  constexpr int kQ = (kRT * kRK) / 256;  // staged elements per thread and operand

  // staging coordinates of this thread: row r (of the 64), basis index kk
  int sr[kQ], sk[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int idx = tid + 256 * q;
    sr[q] = idx % kRT;
    sk[q] = idx / kRT;
  }
  auto load_c = [&](int64_t i0, double2* cv) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int64_t i = i0 + sk[q], j = j0 + sr[q];
      cv[q] = (i < m && j < M) ? Cc[i * cI + j * cJ] : make_double2(0.0, 0.0);
    }
  };
  auto load_e = [&](int64_t n0, int64_t i0, double2* ev) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int64_t i = i0 + sk[q], n = n0 + sr[q];
      ev[q] = (i < m && n < N) ? E[n + i * ldE] : make_double2(0.0, 0.0);
    }
  };
  if (one_chunk) {
    double2 cv[kQ];
    load_c(0, cv);
#pragma unroll
    for (int q = 0; q < kQ; ++q) sC1[sk[q]][sr[q]] = cv[q];
  }

  // per-lane sums of |w|^2 for the columns this wave finishes (plain FP64:
  // the anchored norms only need to be accurate relative to themselves)
  double nacc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) nacc[c] = 0.0;

  const int64_t nchunks = (m + kRK - 1) / kRK;
  double2 ev[kQ], cv[kQ];
  if (m > 0) {
    load_e(0, 0, ev);
    if (!one_chunk) load_c(0, cv);
  }
  for (int64_t n0 = 0; n0 < N; n0 += kRT) {
    d4v accr[2][2], acci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        accr[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
        acci[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
      }
    for (int64_t c = 0; c < nchunks; ++c) {
      // registers -> LDS, then prefetch the next chunk (or the next row
      // tile's first chunk) while the matrix cores work
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        sE[sk[q]][sr[q]] = ev[q];
        if (!one_chunk) sC[sk[q]][sr[q]] = cv[q];
      }
      __syncthreads();
      {
        int64_t nn = n0, ci = c + 1;
        if (ci == nchunks) {
          ci = 0;
          nn = n0 + kRT;
        }
        if (nn < N) {
          load_e(nn, ci * kRK, ev);
          if (!one_chunk) load_c(ci * kRK, cv);
        }
      }
      double2 (*sCk)[kRT + 1] = one_chunk ? sC1 : sC;
      // basis vectors present in this chunk: the steps of 4 beyond them
      // would only add zero products
      const int64_t kval = m - c * kRK;
#pragma unroll
      for (int kk = 0; kk < kRK; kk += 4) {
        if (kk >= kval) break;
        const int r = kk + (lane >> 4);
        double2 a[2], b[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          a[t] = sE[r][wr * 32 + 16 * t + (lane & 15)];
          b[t] = sCk[r][wc * 32 + 16 * t + (lane & 15)];
        }
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
          for (int tb = 0; tb < 2; ++tb) {
            accr[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, b[tb].x, accr[ta][tb], 0, 0, 0);
            accr[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[ta].y, b[tb].y, accr[ta][tb], 0, 0, 0);
            acci[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, b[tb].y, acci[ta][tb], 0, 0, 0);
            acci[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].y, b[tb].x, acci[ta][tb], 0, 0, 0);
          }
      }
      __syncthreads();
    }
    // epilogue in two column halves through LDS: W = X - E C, column-wise
    // (lane = row) so every load/store of a wave is one contiguous run
    const int64_t n = n0 + lane;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (wc == h) {
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
          for (int tb = 0; tb < 2; ++tb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              sD[16 * tb + (lane & 15)][wr * 32 + 16 * ta + (lane >> 4) + 4 * r] =
                  make_double2(accr[ta][tb][r], acci[ta][tb][r]);
      }
      __syncthreads();
      if constexpr (kVec) {
        // lanes 0-31 and 32-63 take two different columns; each lane two
        // consecutive rows (one 16-byte access of X and of W)
        const int rp = 2 * (lane & 31), cs = lane >> 5;
        const int64_t nv = n0 + rp;
        f4v xv[4];
#pragma unroll
        for (int c2 = 0; c2 < 4; ++c2) {
          const int64_t j = j0 + 32 * h + 8 * wave + 2 * c2 + cs;
          xv[c2] = (f4v){0.0f, 0.0f, 0.0f, 0.0f};
          if (j < M) {
            const float* px = reinterpret_cast<const float*>(X + nv + j * ldX);
            if (nv + 1 < N) {
              xv[c2] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(px));
            } else if (nv < N) {
              xv[c2].x = px[0];
              xv[c2].y = px[1];
            }
          }
        }
#pragma unroll
        for (int c2 = 0; c2 < 4; ++c2) {
          const int cl = 8 * wave + 2 * c2 + cs;
          const int64_t j = j0 + 32 * h + cl;
          if (j < M && nv < N) {
            const double2 d0 = sD[cl][rp], d1 = sD[cl][rp + 1];
            double w0r = (double)xv[c2].x - d0.x, w0i = (double)xv[c2].y - d0.y;
            double w1r = (double)xv[c2].z - d1.x, w1i = (double)xv[c2].w - d1.y;
            const bool two = nv + 1 < N;
            if (W) {
              const f4v wv = (f4v){(float)w0r, (float)w0i, (float)w1r, (float)w1i};
              float* pw = reinterpret_cast<float*>(W + nv + j * ldW);
              if (two) {
                *reinterpret_cast<f4v*>(pw) = wv;
              } else {
                pw[0] = wv.x;
                pw[1] = wv.y;
              }
              w0r = wv.x;
              w0i = wv.y;
              w1r = wv.z;
              w1i = wv.w;
            }
            nacc[4 * h + c2] += w0r * w0r + w0i * w0i + (two ? w1r * w1r + w1i * w1i : 0.0);
          }
        }
        __syncthreads();
        continue;
      }
      double2 x[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int64_t j = j0 + 32 * h + 8 * wave + c;
        x[c] = (j < M && n < N) ? ld_x(X + n + j * ldX) : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int cl = 8 * wave + c;
        const int64_t j = j0 + 32 * h + cl;
        if (j < M && n < N) {
          const double2 d = sD[cl][lane];
          double2 w = make_double2(x[c].x - d.x, x[c].y - d.y);
          if (W) w = st_w(W + n + j * ldW, w.x, w.y);  // W == NULL: norms only
          nacc[8 * h + c] += w.x * w.x + w.y * w.y;
        }
      }
      __syncthreads();
    }
  }
  if constexpr (kVec) {
    // nacc[4 h + c2] holds rows of column 8 wave + 2 c2 + (lane >> 5) of
    // half h: sum within each 32-lane half
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c2 = 0; c2 < 4; ++c2) {
        double t = nacc[4 * h + c2];
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) t += __shfl_xor(t, off);
        const int64_t j = j0 + 32 * h + 8 * wave + 2 * c2 + (lane >> 5);
        if ((lane & 31) == 0 && j < M) {
          nrm[j] = t;
          if (!__builtin_isfinite(t)) *bad = 1;
        }
      }
    return;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double t = wave_sum(nacc[8 * h + c]);
      const int64_t j = j0 + 32 * h + 8 * wave + c;
      if (lane == 0 && j < M) {
        nrm[j] = t;
        if (!__builtin_isfinite(t)) *bad = 1;  // same value from every writer
      }
    }
}

}  // namespace

template <int kTA>
hipError_t launch_project_t(const double2* E, int64_t N, int64_t k, int64_t ldE, const double2* S, int64_t M,
                            int64_t ldS, double2* C, int64_t ldC, hipStream_t s) {
  dim3 grid((unsigned)((M + kPJ - 1) / kPJ), (unsigned)((k + 32 * kTA - 1) / (32 * kTA)));
  if (grid.y > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_project_z<kTA>, grid, dim3(256), 0, s, E, N, k, ldE, S, M, ldS, C, ldC);
  return hipGetLastError();
}

hipError_t launch_project_z(const double2* E, int64_t N, int64_t k, int64_t ldE, const double2* S, int64_t M,
                            int64_t ldS, double2* C, int64_t ldC, hipStream_t s) {
  if (k <= 0 || M <= 0) return hipSuccess;
  // fewest passes over S with blocks of at most 224 basis vectors, k split
  // evenly between them; block height 32 kTA
  const int64_t passes = (k + 223) / 224;
  const int64_t per = (k + passes - 1) / passes;
  switch ((int)((per + 31) / 32)) {
    case 1: return launch_project_t<1>(E, N, k, ldE, S, M, ldS, C, ldC, s);
    case 2: return launch_project_t<2>(E, N, k, ldE, S, M, ldS, C, ldC, s);
    case 3: return launch_project_t<3>(E, N, k, ldE, S, M, ldS, C, ldC, s);
    case 4: return launch_project_t<4>(E, N, k, ldE, S, M, ldS, C, ldC, s);
    case 6: return launch_project_t<6>(E, N, k, ldE, S, M, ldS, C, ldC, s);
    case 7: return launch_project_t<7>(E, N, k, ldE, S, M, ldS, C, ldC, s);
    default: return launch_project_t<5>(E, N, k, ldE, S, M, ldS, C, ldC, s);
  }
}

template <class XT, class WT>
hipError_t launch_resid_t(const XT* X, int64_t ldX, WT* W, int64_t ldW, int64_t N, int64_t M, const double2* E,
                          int64_t ldE, int64_t m, const double2* C, int64_t cI, int64_t cJ, double* nrm, int* bad,
                          hipStream_t s) {
  if (M <= 0) return hipSuccess;
  dim3 grid((unsigned)((M + kRT - 1) / kRT));
  bool vec = false;
  if constexpr (sizeof(XT) == 8 && sizeof(WT) == 8) {
    vec = (ldX % 2 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0) &&
          (!W || ((ldW % 2 == 0) && (reinterpret_cast<uintptr_t>(W) % 16 == 0)));
  }
  if (vec)
    hipLaunchKernelGGL((k_resid<XT, WT, true>), grid, dim3(256), 0, s, X, ldX, W, ldW, N, M, E, ldE, m, C, cI, cJ,
                       nrm, bad);
  else
    hipLaunchKernelGGL((k_resid<XT, WT, false>), grid, dim3(256), 0, s, X, ldX, W, ldW, N, M, E, ldE, m, C, cI, cJ,
                       nrm, bad);
  return hipGetLastError();
}

hipError_t launch_resid(const double2* X, int64_t ldX, double2* W, int64_t ldW, int64_t N, int64_t M,
                        const double2* E, int64_t ldE, int64_t m, const double2* C, int64_t cI, int64_t cJ,
                        double* nrm, int* bad, hipStream_t s) {
  return launch_resid_t(X, ldX, W, ldW, N, M, E, ldE, m, C, cI, cJ, nrm, bad, s);
}
hipError_t launch_resid(const double2* X, int64_t ldX, float2* W, int64_t ldW, int64_t N, int64_t M,
                        const double2* E, int64_t ldE, int64_t m, const double2* C, int64_t cI, int64_t cJ,
                        double* nrm, int* bad, hipStream_t s) {
  return launch_resid_t(X, ldX, W, ldW, N, M, E, ldE, m, C, cI, cJ, nrm, bad, s);
}
hipError_t launch_resid(const float2* X, int64_t ldX, float2* W, int64_t ldW, int64_t N, int64_t M,
                        const double2* E, int64_t ldE, int64_t m, const double2* C, int64_t cI, int64_t cJ,
                        double* nrm, int* bad, hipStream_t s) {
  return launch_resid_t(X, ldX, W, ldW, N, M, E, ldE, m, C, cI, cJ, nrm, bad, s);
}

}  // namespace rb

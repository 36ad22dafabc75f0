// Dense complex FP64 products of the greedy:
//   project : C = E^H S  (k x M), the coefficients of every snapshot on the
//             basis (the projection E E^H s of Sec. 4), on FP64 matrix cores
//             (v_mfma_f64_16x16x4f64);
//   deflate : W = X - E C (N x M), an explicit re-anchoring of the working
//             columns onto their residuals against a panel of m basis
//             vectors, i.e. the stored-residual form of the greedy (the
//             residual matrix V of Alg. 2; Remark 5.5).
#include "rb_internal.h"

namespace rb {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------- project --
// Block tile 64 (basis index i) x 64 (column j), 4 waves as 2 x 2, each wave
// 32 x 32 = 2 x 2 MFMA tiles.  The reduction runs over rows n in chunks of
// kKB staged through LDS (E and S chunks, both as complex128 row-major
// [n][col] so that MFMA operand reads are contiguous).
//
// v_mfma_f64_16x16x4f64 operand layout (64 lanes): A(16x4) lane l holds
// A[l%16][l/16]; B(4x16) lane l holds B[l/16][l%16]; the 16x16 result
// lane l, register r holds D[l/16 + 4r][l%16].
constexpr int kPT = 64;  // tile edge (i and j)
constexpr int kKB = 32;  // rows per LDS chunk

__global__ __launch_bounds__(256) void k_project_z(const double2* __restrict__ E, int64_t N, int64_t k, int64_t ldE,
                                                   const double2* __restrict__ S, int64_t M, int64_t ldS,
                                                   double2* __restrict__ C, int64_t ldC) {
  // +1 column of padding: the staging writes walk down rows (stride 1 row)
  __shared__ double2 sE[kKB][kPT + 1];
  __shared__ double2 sS[kKB][kPT + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * kPT;
  const int64_t i0 = (int64_t)blockIdx.y * kPT;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;

  d4v accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
      acci[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
    }

  for (int64_t n0 = 0; n0 < N; n0 += kKB) {
    // stage: thread t loads rows (t % kKB) of columns (t / kKB) + 8 q
#pragma unroll
    for (int q = 0; q < (kKB * kPT) / 256; ++q) {
      const int idx = tid + 256 * q;
      const int c = idx / kKB, r = idx % kKB;
      const int64_t n = n0 + r;
      double2 ev = make_double2(0.0, 0.0), sv = make_double2(0.0, 0.0);
      if (n < N) {
        if (i0 + c < k) ev = E[n + (i0 + c) * ldE];
        if (j0 + c < M) sv = ld_stream(S + n + (j0 + c) * ldS);
      }
      sE[r][c] = ev;
      sS[r][c] = sv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKB; kk += 4) {
      const int r = kk + (lane >> 4);
      double2 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sE[r][wi + 16 * t + (lane & 15)];
        b[t] = sS[r][wj + 16 * t + (lane & 15)];
      }
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
          // conj(e) * s:  re = er sr + ei si,  im = er si - ei sr
          accr[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, b[tb].x, accr[ta][tb], 0, 0, 0);
          accr[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].y, b[tb].y, accr[ta][tb], 0, 0, 0);
          acci[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, b[tb].y, acci[ta][tb], 0, 0, 0);
          acci[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[ta].y, b[tb].x, acci[ta][tb], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi + 16 * ta + (lane >> 4) + 4 * r;
        const int64_t j = j0 + wj + 16 * tb + (lane & 15);
        if (i < k && j < M) C[i + j * ldC] = make_double2(accr[ta][tb][r], acci[ta][tb][r]);
      }
}

// ------------------------------------------------------------- deflate --
// W[n, j] = X[n, j] - sum_{i<m} E[n, i] C(i, j), C(i, j) = C[i*cI + j*cJ].
// One thread per row n, kDefCols columns per workgroup; the coefficients of
// a column are uniform over the workgroup.
constexpr int kDefCols = 16;

// X and W may alias (in-place re-anchoring): each element is read and then
// written by the same thread.
__global__ __launch_bounds__(256) void k_deflate_z(const double2* X, int64_t ldX,
                                                   double2* W, int64_t ldW, int64_t N, int64_t M,
                                                   const double2* __restrict__ E, int64_t ldE, int64_t m,
                                                   const double2* __restrict__ Cc, int64_t cI, int64_t cJ) {
  const int64_t n = (int64_t)blockIdx.y * 256 + threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kDefCols;
  if (n >= N) return;
  double re[kDefCols], im[kDefCols];
#pragma unroll
  for (int c = 0; c < kDefCols; ++c) re[c] = im[c] = 0.0;
  int64_t jc[kDefCols];
#pragma unroll
  for (int c = 0; c < kDefCols; ++c) jc[c] = (j0 + c < M) ? j0 + c : M - 1;
  for (int64_t i = 0; i < m; ++i) {
    const double2 a = E[n + i * ldE];
#pragma unroll
    for (int c = 0; c < kDefCols; ++c) {
      const double2 g = Cc[i * cI + jc[c] * cJ];
      re[c] += a.x * g.x - a.y * g.y;
      im[c] += a.x * g.y + a.y * g.x;
    }
  }
#pragma unroll
  for (int c = 0; c < kDefCols; ++c) {
    if (j0 + c < M) {
      const double2 x = X[n + (j0 + c) * ldX];
      W[n + (j0 + c) * ldW] = make_double2(x.x - re[c], x.y - im[c]);
    }
  }
}

}  // namespace

hipError_t launch_project_z(const double2* E, int64_t N, int64_t k, int64_t ldE, const double2* S, int64_t M,
                            int64_t ldS, double2* C, int64_t ldC, hipStream_t s) {
  if (k <= 0 || M <= 0) return hipSuccess;
  dim3 grid((unsigned)((M + kPT - 1) / kPT), (unsigned)((k + kPT - 1) / kPT));
  if (grid.y > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_project_z, grid, dim3(256), 0, s, E, N, k, ldE, S, M, ldS, C, ldC);
  return hipGetLastError();
}

hipError_t launch_deflate_z(const double2* X, int64_t ldX, double2* W, int64_t ldW, int64_t N, int64_t M,
                            const double2* E, int64_t ldE, int64_t m, const double2* C, int64_t cI, int64_t cJ,
                            hipStream_t s) {
  dim3 grid((unsigned)((M + kDefCols - 1) / kDefCols), (unsigned)((N + 255) / 256));
  if (grid.y > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_deflate_z, grid, dim3(256), 0, s, X, ldX, W, ldW, N, M, E, ldE, m, C, cI, cJ);
  return hipGetLastError();
}

}  // namespace rb

// Re-anchoring fused with the next sweep (FP64 working matrix).
//
// When the Eq. (6.3) estimate is about to lose resolution, the working
// columns' residual norms against the m panel vectors swept since the last
// written anchoring are recomputed explicitly (the stored-residual form of
// the greedy, Remark 5.5), and the newest basis vector's coefficients are
// formed in the same read of X:
//   r_j    = x_j - E_p c_j           (c_j: the panel coefficients, stored
//                                     by earlier sweeps)
//   nrm_j  = ||r_j||^2               (explicit, no cancellation)
//   c'_j   = e^H x_j                 (the sweep's coefficient, stored as the
//                                     panel's next row)
//   acc_j  = |c'_j|^2, est_j = nrm_j - acc_j, masked argmax (and the
//                                     largest unmasked nrm_j)
// X is not written (a norms-only anchoring: the panel keeps growing).  With
// e orthogonal to E_p, e^H x_j = e^H r_j up to rounding, so est_j is the
// residual^2 after the new vector with a one-term cancellation only.
//
// Work decomposition: a workgroup of 4 waves owns 16 columns (4 per wave in
// the epilogue); lane = row inside 64-row tiles, so every load of X is one
// contiguous 1 KiB run per wave instruction (as in the sweep).  The panel
// coefficients of the 16 columns stay in registers as matrix-core operands
// for the whole pass; each row tile of E_p (64 x m) is staged through LDS.
// The product E_p c (8 m flops per element) runs on the FP64 matrix cores,
// beside the vector work of the epilogue: at m <= kFuseMaxM it stays below
// the time of the HBM read it overlaps.
#include "rb_internal.h"

namespace rb {

namespace {

constexpr int kFWaves = 4;
constexpr int kFCols = 4;                        // columns per wave
constexpr int kFColsPerBlock = kFWaves * kFCols;  // 16
constexpr int kFRows = 64;                       // rows per tile

// kM: the panel size (a template parameter, so the product over the panel
// is straight-line code and the compiler's waits for the pipelined loads
// stay exact)
typedef double d4v __attribute__((ext_vector_type(4)));

// kM: the panel size (a template parameter, so the loops over the panel are
// straight-line code and the compiler's waits for the pipelined loads stay
// exact).
//
// Per 64-row tile: the E_p rows are staged in LDS (vector-major); wave w
// forms D = E_p c for rows 16w..16w+15 of the tile and all 16 columns on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64: A(16x4) lane l holds
// A[l%16][l/16], B(4x16) lane l holds B[l/16][l%16], D lane l register r
// holds D[l/16 + 4r][l%16]); D goes through LDS (column-major) to the
// epilogue, where wave w finishes columns 4w..4w+3 with lane = row.
template <int kM>
__global__ __launch_bounds__(kFWaves * 64, 2) void k_anchor_sweep(
    const double2* __restrict__ X, int64_t ldX, int64_t N, int64_t M, const double2* __restrict__ E,
    int64_t ldE, const double2* __restrict__ Cp, int64_t ldCp, const double2* __restrict__ e,
    double* __restrict__ nrm, double* __restrict__ acc, const uint8_t* __restrict__ mask,
    double2* __restrict__ c_out, ArgMax* __restrict__ partial, int* __restrict__ bad) {
  constexpr int kS = (kM + 3) / 4;                  // k-steps of 4 vectors
  __shared__ double2 sE[kFuseMaxM][kFRows];         // E_p tile, vector-major
  __shared__ double2 sD[kFColsPerBlock][kFRows];    // D = E_p c, column-major
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: column addresses stay scalar
  const int64_t j0 = (int64_t)blockIdx.x * kFColsPerBlock;

  // B operands: lane l holds C(4 s + l / 16, j0 + l % 16) for k-step s
  // (vectors past m: zero; columns past M: column M - 1's)
  double2 bk[kS > 0 ? kS : 1];
  {
    const int64_t jc = j0 + (lane & 15) < M ? j0 + (lane & 15) : M - 1;
#pragma unroll
    for (int q = 0; q < kS; ++q) {
      const int i = 4 * q + (lane >> 4);
      bk[q] = i < kM ? Cp[(int64_t)i * ldCp + jc] : make_double2(0.0, 0.0);
    }
  }

  // the wave's epilogue columns; those past M are clamped onto column M - 1
  // for the loads and neither stored nor counted
  const int64_t jw = j0 + (int64_t)wave * kFCols;
  const double2* x0 = X + (jw + 0 < M ? jw + 0 : M - 1) * ldX;
  const double2* x1 = X + (jw + 1 < M ? jw + 1 : M - 1) * ldX;
  const double2* x2 = X + (jw + 2 < M ? jw + 2 : M - 1) * ldX;
  const double2* x3 = X + (jw + 3 < M ? jw + 3 : M - 1) * ldX;

  // Software pipeline over 64-row tiles.  While tile t is computed, the E_p
  // rows and the X rows of tile t+1 are in flight; every thread issues its
  // E loads (a fixed count, clamped addresses) before its X loads, so the
  // wait for the E rows of a tile never waits for that tile's X rows.  The
  // loop body handles two tiles with alternating register sets (a and b),
  // so no register copy waits on loads still in flight; an odd tile count
  // gets one extra tile of clamped rows with zero weight.
  // Staging: thread t holds row t % 64 of vectors t / 64 + 4 q (q < 4).
  // (kFuseMaxM = 16: four staged vectors per thread; four columns per wave;
  // the staged values and the rows of X are named registers, not arrays,
  // so none of them is placed in scratch memory)
  static_assert(kFuseMaxM == 16 && kFCols == 4, "the tile body below is written out for 16 vectors, 4 columns");
  constexpr int mm = kM > 0 ? kM : 1;
  const int er = tid % kFRows, ei0 = tid / kFRows;
  const int64_t eo0 = (int64_t)(ei0 + 0 < mm ? ei0 + 0 : mm - 1) * ldE;
  const int64_t eo1 = (int64_t)(ei0 + 4 < mm ? ei0 + 4 : mm - 1) * ldE;
  const int64_t eo2 = (int64_t)(ei0 + 8 < mm ? ei0 + 8 : mm - 1) * ldE;
  const int64_t eo3 = (int64_t)(ei0 + 12 < mm ? ei0 + 12 : mm - 1) * ldE;
  double2 sa0, sa1, sa2, sa3, sb0, sb1, sb2, sb3;  // staged E rows (ping, pong)
  double2 xa0, xa1, xa2, xa3, xb0, xb1, xb2, xb3;  // X rows of the wave's columns
  double2 ea, eb;                                  // e rows
  double n0s = 0.0, n1s = 0.0, n2s = 0.0, n3s = 0.0;  // |r|^2 partial sums
  double c0r = 0.0, c0i = 0.0, c1r = 0.0, c1i = 0.0, c2r = 0.0, c2i = 0.0, c3r = 0.0, c3i = 0.0;  // e^H x
  // A operand position of this lane in the wave's 16-row block
  const int ar = 16 * wave + (lane & 15), ak = lane >> 4;

#define RB_LOAD_TILE(N0, S, XV, EV)                         \
  {                                                        \
    const int64_t nr_ = (N0) + er < N ? (N0) + er : N - 1; \
    S##0 = E[nr_ + eo0];                                   \
    S##1 = E[nr_ + eo1];                                   \
    S##2 = E[nr_ + eo2];                                   \
    S##3 = E[nr_ + eo3];                                   \
    const int64_t n_ = (N0) + lane;                        \
    const int64_t nc_ = n_ < N ? n_ : N - 1;               \
    XV##0 = ld_stream(x0 + nc_);                           \
    XV##1 = ld_stream(x1 + nc_);                           \
    XV##2 = ld_stream(x2 + nc_);                           \
    XV##3 = ld_stream(x3 + nc_);                           \
    EV = e[nc_];                                           \
  }

// one column's share of a tile: r = x - (E c), ||r||^2, conj(e) x
#define RB_COL(C, XC)                                               \
  {                                                                 \
    const double2 d_ = sD[4 * wave + C][lane];                      \
    const double rr = XC.x - d_.x, ri = XC.y - d_.y;                \
    n##C##s += wgt * (rr * rr + ri * ri);                           \
    c##C##r += wgt * (ev_.x * XC.x + ev_.y * XC.y);                 \
    c##C##i += wgt * (ev_.x * XC.y - ev_.y * XC.x);                 \
  }

#define RB_TILE(N0, S, XV, EV, SN, XVN, EVN)                                                       \
  {                                                                                              \
    __syncthreads(); /* the previous tile's sE and sD reads are done */                          \
    /* vectors i >= m of sE receive clamped copies; their B operands are zero */                 \
    sE[ei0][er] = S##0;                                                                          \
    sE[ei0 + 4][er] = S##1;                                                                      \
    sE[ei0 + 8][er] = S##2;                                                                      \
    sE[ei0 + 12][er] = S##3;                                                                     \
    __syncthreads();                                                                             \
    RB_LOAD_TILE((N0) + kFRows, SN, XVN, EVN) /* past the end: clamped rows, not used */         \
    d4v dr = {0.0, 0.0, 0.0, 0.0}, di = {0.0, 0.0, 0.0, 0.0};                                    \
    _Pragma("unroll") for (int q = 0; q < kS; ++q) {                                             \
      const double2 av = sE[4 * q + ak][ar];                                                     \
      /* E c:  re = Er cr - Ei ci,  im = Er ci + Ei cr */                                        \
      dr = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bk[q].x, dr, 0, 0, 0);                     \
      dr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bk[q].y, dr, 0, 0, 0);                    \
      di = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bk[q].y, di, 0, 0, 0);                     \
      di = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bk[q].x, di, 0, 0, 0);                     \
    }                                                                                            \
    _Pragma("unroll") for (int r = 0; r < 4; ++r)                                                \
      sD[lane & 15][16 * wave + (lane >> 4) + 4 * r] = make_double2(dr[r], di[r]);               \
    __syncthreads();                                                                             \
    const int64_t n = (N0) + lane;                                                               \
    const double wgt = n < N ? 1.0 : 0.0; /* rows past N count for nothing */                    \
    const double2 ev_ = EV;                                                                      \
    RB_COL(0, XV##0)                                                                             \
    RB_COL(1, XV##1)                                                                             \
    RB_COL(2, XV##2)                                                                             \
    RB_COL(3, XV##3)                                                                             \
  }

  RB_LOAD_TILE(0, sa, xa, ea)
  // two tiles per iteration with alternating registers; an odd tile count
  // gets one extra tile of clamped rows with zero weight
  const int64_t ntile = (N + kFRows - 1) / kFRows;
  for (int64_t t = 0; t < ntile; t += 2) {
    RB_TILE(t * kFRows, sa, xa, ea, sb, xb, eb)
    RB_TILE((t + 1) * kFRows, sb, xb, eb, sa, xa, ea)
  }
#undef RB_TILE
#undef RB_COL
#undef RB_LOAD_TILE
  const double nacc[kFCols] = {n0s, n1s, n2s, n3s};
  const double cre[kFCols] = {c0r, c1r, c2r, c3r}, cim[kFCols] = {c0i, c1i, c2i, c3i};

  // est argmax and the largest fresh norm (the new resolution scale), both
  // over unmasked columns
  vi best = {0.0, -1}, bestn = {0.0, -1};
#pragma unroll
  for (int c = 0; c < kFCols; ++c) {
    const double t = wave_sum(nacc[c]);
    const double cr = wave_sum(cre[c]), ci = wave_sum(cim[c]);
    const int64_t j = jw + c;
    if (j < M && lane == c) {
      nrm[j] = t;
      if (!__builtin_isfinite(t)) *bad = 1;
      const double a2 = cr * cr + ci * ci;
      acc[j] = a2;
      c_out[j] = make_double2(cr, ci);
      if (!(mask && mask[j])) {
        best = vi_max(best, vi{t - a2, j});
        bestn = vi_max(bestn, vi{t, j});
      }
    }
  }
  best = wave_vi_max(best);
  bestn = wave_vi_max(bestn);
  __shared__ vi sbest[2][kFWaves];
  if (lane == 0) {
    sbest[0][wave] = best;
    sbest[1][wave] = bestn;
  }
  __syncthreads();
  if (tid < 2) {
    vi b = sbest[tid][0];
#pragma unroll
    for (int w = 1; w < kFWaves; ++w) b = vi_max(b, sbest[tid][w]);
    ArgMax* out = partial + (int64_t)tid * gridDim.x + blockIdx.x;
    out->v = b.v;
    out->i = b.i;
  }
}

__global__ __launch_bounds__(1024) void k_argmax_n(const ArgMax* __restrict__ partial, int64_t n,
                                                   ArgMax* __restrict__ result) {
  vi best = {0.0, -1};
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) best = vi_max(best, vi{partial[t].v, partial[t].i});
  best = wave_vi_max(best);
  __shared__ vi sbest[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sbest[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    vi b = sbest[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) b = vi_max(b, sbest[w]);
    result->v = (b.i < 0) ? -__builtin_inf() : b.v;
    result->i = b.i;
  }
}

}  // namespace

int64_t anchor_sweep_partials(int64_t M) { return (M + kFColsPerBlock - 1) / kFColsPerBlock; }

hipError_t launch_anchor_sweep(const double2* X, int64_t ldX, int64_t N, int64_t M,
                               const double2* E, int64_t ldE, int64_t m, const double2* Cp, int64_t ldCp,
                               const double2* e, double* nrm, double* acc, const uint8_t* mask, double2* c_out,
                               ArgMax* partial, int64_t npartial_cap, ArgMax* result, int* bad, hipStream_t s) {
  if (m < 0 || m > kFuseMaxM || M <= 0 || N <= 0) return hipErrorInvalidValue;
  const int64_t grid = anchor_sweep_partials(M);
  if (2 * grid > npartial_cap || grid > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (m) {
#define RB_FUSE_CASE(MM)                                                                                   \
  case MM:                                                                                                 \
    hipLaunchKernelGGL(k_anchor_sweep<MM>, dim3((unsigned)grid), dim3(kFWaves * 64), 0, s, X, ldX, N, M, E, \
                       ldE, Cp, ldCp, e, nrm, acc, mask, c_out, partial, bad);                             \
    break;
    RB_FUSE_CASE(0) RB_FUSE_CASE(1) RB_FUSE_CASE(2) RB_FUSE_CASE(3) RB_FUSE_CASE(4) RB_FUSE_CASE(5)
    RB_FUSE_CASE(6) RB_FUSE_CASE(7) RB_FUSE_CASE(8) RB_FUSE_CASE(9) RB_FUSE_CASE(10) RB_FUSE_CASE(11)
    RB_FUSE_CASE(12) RB_FUSE_CASE(13) RB_FUSE_CASE(14) RB_FUSE_CASE(15) RB_FUSE_CASE(16)
#undef RB_FUSE_CASE
    default: return hipErrorInvalidValue;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !result) return err;
  hipLaunchKernelGGL(k_argmax_n, dim3(1), dim3(1024), 0, s, partial, grid, result);
  hipLaunchKernelGGL(k_argmax_n, dim3(1), dim3(1024), 0, s, partial + grid, grid, result + 1);
  return hipGetLastError();
}

}  // namespace rb

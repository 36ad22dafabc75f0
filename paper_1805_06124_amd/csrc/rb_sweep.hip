// Pivot search of the RB-greedy (Sec. 6.1.2): exact column norms, the fused
// Eq. (6.3) sweep with its masked argmax, and the argmax of stored estimates.
//
// Work decomposition (all kernels here are HBM-bound, no matrix cores):
// a wavefront owns kCols consecutive columns and walks down their rows with
// lane n%64 reading row n, so every load instruction of a wave fetches one
// contiguous 1 KiB run of a column (16 B per lane, complex128).  kUnroll row
// blocks are issued before any arithmetic to keep kCols*kUnroll independent
// 16 B loads in flight per lane.  The basis vector e is re-read by every wave
// from L2 (one e element per kCols column elements).
#include "rb_internal.h"

namespace rb {

namespace {

constexpr int kSweepWaves = 4;     // waves per workgroup
constexpr int kSweepCols = 4;      // columns per wave
constexpr int kSweepUnroll = 4;    // 64-row blocks in flight per column
constexpr int kColsPerBlock = kSweepWaves * kSweepCols;
static_assert(kColsPerBlock == kPivotGroup, "one partial argmax per pivot group");


// --------------------------------------------------------------------------
// Exact squared column norms.  One wave per column; every lane accumulates a
// double-double sum of its rows, then the wave combines the 64 partial sums.
__device__ __forceinline__ double2 ld_c(const double2* p) { return ld_stream(p); }
__device__ __forceinline__ double2 ld_c(const float2* p) {
  const float2 v = ld_stream(p);
  return make_double2((double)v.x, (double)v.y);
}

template <class T>
__global__ __launch_bounds__(256) void k_colnorms(const T* __restrict__ S, int64_t N, int64_t M, int64_t ldS,
                                                  double* __restrict__ nrm, int* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (j >= M) return;
  const T* col = S + j * ldS;
  dd acc = {0.0, 0.0};
  for (int64_t n = lane; n < N; n += 64) {
    const double2 v = ld_c(col + n);
    dd_add_sq(acc, v.x);
    dd_add_sq(acc, v.y);
  }
  acc = wave_dd_sum(acc);
  if (lane == 0) {
    double r = acc.hi + acc.lo;
    nrm[j] = r;
    if (!__builtin_isfinite(r)) *bad = 1;  // same value from every writer
  }
}

// --------------------------------------------------------------------------
// Fused sweep: c_j = e^H s_j, acc_j += |c_j|^2, est_j = nrm_j - acc_j and a
// per-workgroup masked (est, index) argmax.
template <bool kStoreC>
__global__ __launch_bounds__(kSweepWaves * 64) void k_sweep_z(
    const double2* __restrict__ S, int64_t N, int64_t M, int64_t ldS, const double2* __restrict__ e,
    const double* __restrict__ nrm, double* __restrict__ acc, const uint8_t* __restrict__ mask,
    double2* __restrict__ c_out, int64_t ldc, ArgMax* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t col0 = (int64_t)blockIdx.x * kColsPerBlock + (int64_t)wave * kSweepCols;

  // columns past M are clamped onto the last column (loads stay in bounds,
  // results are discarded)
  const double2* cp[kSweepCols];
#pragma unroll
  for (int c = 0; c < kSweepCols; ++c) {
    int64_t j = col0 + c;
    if (j > M - 1) j = M - 1;
    cp[c] = S + j * ldS;
  }
  double re[kSweepCols], im[kSweepCols];
#pragma unroll
  for (int c = 0; c < kSweepCols; ++c) re[c] = im[c] = 0.0;

  constexpr int kStep = 64 * kSweepUnroll;
  const int64_t nfull = (N / kStep) * kStep;
  for (int64_t base = 0; base < nfull; base += kStep) {
    double2 ev[kSweepUnroll];
    double2 sv[kSweepCols][kSweepUnroll];
#pragma unroll
    for (int u = 0; u < kSweepUnroll; ++u) ev[u] = e[base + 64 * u + lane];
#pragma unroll
    for (int c = 0; c < kSweepCols; ++c)
#pragma unroll
      for (int u = 0; u < kSweepUnroll; ++u) sv[c][u] = ld_stream(cp[c] + base + 64 * u + lane);
#pragma unroll
    for (int c = 0; c < kSweepCols; ++c)
#pragma unroll
      for (int u = 0; u < kSweepUnroll; ++u) sweep_cmac(ev[u], sv[c][u], re[c], im[c]);
  }
  // ragged tail (N not a multiple of 64 * kSweepUnroll)
  for (int64_t n = nfull + lane; n < N; n += 64) {
    double2 ev = e[n];
#pragma unroll
    for (int c = 0; c < kSweepCols; ++c) sweep_cmac(ev, ld_stream(cp[c] + n), re[c], im[c]);
  }

  vi best = {0.0, -1};
#pragma unroll
  for (int c = 0; c < kSweepCols; ++c) {
    double cr = wave_sum(re[c]);
    double ci = wave_sum(im[c]);
    const int64_t j = col0 + c;
    if (j < M) {
      // lane c finishes column c (spreads the epilogue's loads over lanes)
      if (lane == c) {
        double a = sweep_acc_add(acc[j], cr, ci);
        acc[j] = a;
        if (kStoreC) c_out[j * ldc] = make_double2(cr, ci);
        if (!(mask && mask[j])) {
          vi cand = {nrm[j] - a, j};
          best = vi_max(best, cand);
        }
      }
    }
  }
  best = wave_vi_max(best);
  __shared__ vi sbest[kSweepWaves];
  if (lane == 0) sbest[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    vi b = sbest[0];
#pragma unroll
    for (int w = 1; w < kSweepWaves; ++w) b = vi_max(b, sbest[w]);
    partial[blockIdx.x].v = b.v;
    partial[blockIdx.x].i = b.i;
  }
}

// est_j = nrm_j - acc_j (acc may be NULL = 0) argmax over unmasked columns,
// per-workgroup partials.
__global__ __launch_bounds__(256) void k_est_argmax(const double* __restrict__ nrm, const double* __restrict__ acc,
                                                    const uint8_t* __restrict__ mask, int64_t M,
                                                    ArgMax* __restrict__ partial) {
  vi best = {0.0, -1};
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += (int64_t)gridDim.x * blockDim.x) {
    if (mask && mask[j]) continue;
    vi cand = {nrm[j] - (acc ? acc[j] : 0.0), j};
    best = vi_max(best, cand);
  }
  best = wave_vi_max(best);
  __shared__ vi sbest[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sbest[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    vi b = sbest[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) b = vi_max(b, sbest[w]);
    partial[blockIdx.x].v = b.v;
    partial[blockIdx.x].i = b.i;
  }
}

// Final reduction of n partial argmax records into *result (one workgroup).
__global__ __launch_bounds__(1024) void k_argmax_final(const ArgMax* __restrict__ partial, int64_t n,
                                                       ArgMax* __restrict__ result) {
  // eight records per thread in flight (vi_max is a total order, so the
  // grouping does not change the result)
  constexpr int kU = 8;
  const int64_t step = blockDim.x;
  vi best = {0.0, -1};
  int64_t t = threadIdx.x;
  for (; t + (kU - 1) * step < n; t += kU * step) {
    vi c[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) c[u] = vi{partial[t + u * step].v, partial[t + u * step].i};
#pragma unroll
    for (int u = 0; u < kU; ++u) best = vi_max(best, c[u]);
  }
  for (; t < n; t += step) best = vi_max(best, vi{partial[t].v, partial[t].i});
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

template <class T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

template <class T>
hipError_t launch_fill_t(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t grid = (n + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)grid), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t s) { return launch_fill_t(p, v, n, s); }
hipError_t launch_fill(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) { return launch_fill_t(p, v, n, s); }
hipError_t launch_fill(int* p, int v, int64_t n, hipStream_t s) { return launch_fill_t(p, v, n, s); }

int64_t sweep_partials_needed(int64_t M) {
  int64_t a = (M + kColsPerBlock - 1) / kColsPerBlock;
  int64_t b = 2048;  // k_est_argmax grid cap
  return a > b ? a : b;
}

template <class T>
hipError_t launch_colnorms_t(const T* S, int64_t N, int64_t M, int64_t ldS, double* nrm, int* bad, hipStream_t s) {
  const int waves = 4;
  int64_t grid = (M + waves - 1) / waves;
  hipLaunchKernelGGL(k_colnorms<T>, dim3((unsigned)grid), dim3(64 * waves), 0, s, S, N, M, ldS, nrm, bad);
  return hipGetLastError();
}
hipError_t launch_colnorms_z(const double2* S, int64_t N, int64_t M, int64_t ldS, double* nrm, int* bad,
                             hipStream_t s) {
  return launch_colnorms_t(S, N, M, ldS, nrm, bad, s);
}
hipError_t launch_colnorms_c(const float2* S, int64_t N, int64_t M, int64_t ldS, double* nrm, int* bad,
                             hipStream_t s) {
  return launch_colnorms_t(S, N, M, ldS, nrm, bad, s);
}

hipError_t launch_sweep_z(const double2* S, int64_t N, int64_t M, int64_t ldS, const double2* e,
                          const double* nrm, double* acc, const uint8_t* mask, double2* c_out, int64_t ldc,
                          ArgMax* partial, int64_t npartial_cap, ArgMax* result, hipStream_t s) {
  int64_t grid = (M + kColsPerBlock - 1) / kColsPerBlock;
  if (grid > npartial_cap) return hipErrorInvalidValue;
  if (c_out)
    hipLaunchKernelGGL(k_sweep_z<true>, dim3((unsigned)grid), dim3(kSweepWaves * 64), 0, s, S, N, M, ldS, e,
                       nrm, acc, mask, c_out, ldc, partial);
  else
    hipLaunchKernelGGL(k_sweep_z<false>, dim3((unsigned)grid), dim3(kSweepWaves * 64), 0, s, S, N, M, ldS, e,
                       nrm, acc, mask, c_out, ldc, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !result) return err;
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(1024), 0, s, partial, grid, result);
  return hipGetLastError();
}

hipError_t launch_sweep_final(int64_t M, const ArgMax* partial, ArgMax* result, hipStream_t s) {
  const int64_t grid = (M + kColsPerBlock - 1) / kColsPerBlock;
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(1024), 0, s, partial, grid, result);
  return hipGetLastError();
}

hipError_t launch_argmax_records(const ArgMax* partial, int64_t n, ArgMax* result, hipStream_t s) {
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(1024), 0, s, partial, n, result);
  return hipGetLastError();
}

hipError_t launch_est_argmax(const double* nrm, const double* acc, const uint8_t* mask, int64_t M,
                             ArgMax* partial, int64_t npartial_cap, ArgMax* result, hipStream_t s) {
  int64_t grid = (M + 255) / 256;
  if (grid > 2048) grid = 2048;
  if (grid > npartial_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_est_argmax, dim3((unsigned)grid), dim3(256), 0, s, nrm, acc, mask, M, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(1024), 0, s, partial, grid, result);
  return hipGetLastError();
}

}  // namespace rb

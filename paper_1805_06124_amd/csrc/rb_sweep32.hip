// Mixed-precision pivot search: the Eq. (6.3) sweep over complex64 columns
// with an FP32 copy of the basis vector, FP32 products accumulated in FP32
// over each row tile and promoted to FP64 between tiles; acc, est and the
// coefficients stay FP64.  Instead of one argmax it keeps the kTop best
// (est, index) candidates, which the host confirms in FP64.
//
// Same work decomposition as the FP64 sweep: a wave owns 4 columns and walks
// down their rows; with 16-byte aligned columns each lane loads two
// consecutive complex64 values per instruction (1 KiB contiguous per wave
// instruction), 4 such loads in flight per column.
#include "rb_internal.h"

namespace rb {

namespace {

constexpr int kS32Waves = 4;
constexpr int kS32Cols = 4;
constexpr int kS32Unroll = 8;
constexpr int kS32ColsPerBlock = kS32Waves * kS32Cols;

// candidate order (the order of vi_max): NaN first, then larger value, then
// lower index; index < 0 = empty
__device__ __forceinline__ bool better(double av, int64_t ai, double bv, int64_t bi) {
  if (ai < 0) return false;
  if (bi < 0) return true;
  const bool an = av != av, bn = bv != bv;
  if (an != bn) return an;
  if (!an && av != bv) return av > bv;
  return ai < bi;
}

// sorted (descending) list of kTop candidates kept in registers
struct TopList {
  double v[kTop];
  int64_t i[kTop];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int r = 0; r < kTop; ++r) {
      v[r] = 0.0;
      i[r] = -1;
    }
  }
  __device__ __forceinline__ void insert(double cv, int64_t ci) {
    if (!better(cv, ci, v[kTop - 1], i[kTop - 1])) return;
    // bubble the new entry up from the bottom
    v[kTop - 1] = cv;
    i[kTop - 1] = ci;
#pragma unroll
    for (int r = kTop - 1; r > 0; --r) {
      if (better(v[r], i[r], v[r - 1], i[r - 1])) {
        double tv = v[r];
        v[r] = v[r - 1];
        v[r - 1] = tv;
        int64_t ti = i[r];
        i[r] = i[r - 1];
        i[r - 1] = ti;
      }
    }
  }
  __device__ __forceinline__ void pop() {
#pragma unroll
    for (int r = 0; r < kTop - 1; ++r) {
      v[r] = v[r + 1];
      i[r] = i[r + 1];
    }
    v[kTop - 1] = 0.0;
    i[kTop - 1] = -1;
  }
};

// Merge the lists of all threads of a workgroup into its kTop best, written
// to out[0..kTop).  kTop rounds of a workgroup argmax over list heads; the
// owner of each winner pops it (indices are unique).
__device__ void block_top_merge(TopList& L, ArgMax* __restrict__ out) {
  __shared__ vi sw[16];
  __shared__ vi win;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x / 64);
  for (int r = 0; r < kTop; ++r) {
    vi h = {L.v[0], L.i[0]};
    h = wave_vi_max(h);
    if (lane == 0) sw[wave] = h;
    __syncthreads();
    if (threadIdx.x == 0) {
      vi b = sw[0];
      for (int w = 1; w < nw; ++w) b = vi_max(b, sw[w]);
      win = b;
      out[r].v = b.v;
      out[r].i = b.i;
    }
    __syncthreads();
    if (win.i >= 0 && L.i[0] == win.i) L.pop();
    __syncthreads();
  }
}

__device__ __forceinline__ void cmac_conj32(const float2 e, const float2 s, float& re, float& im) {
  re += e.x * s.x + e.y * s.y;
  im += e.x * s.y - e.y * s.x;
}

typedef float f4v __attribute__((ext_vector_type(4)));

// kVec: every lane loads two consecutive complex64 values (16 bytes) per
// instruction (columns 16-byte aligned); otherwise one (8 bytes).  Either way
// a row tile is 512 rows, summed in FP32 and added to the FP64 totals.
template <bool kStoreC, bool kVec>
__global__ __launch_bounds__(kS32Waves * 64) void k_sweep_c(
    const float2* __restrict__ S, int64_t N, int64_t M, int64_t ldS, const float2* __restrict__ e,
    const double* __restrict__ nrm, double* __restrict__ acc, const uint8_t* __restrict__ mask,
    double2* __restrict__ c_out, int64_t ldc, ArgMax* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t col0 = (int64_t)blockIdx.x * kS32ColsPerBlock + (int64_t)wave * kS32Cols;
  const float2* cp[kS32Cols];
#pragma unroll
  for (int c = 0; c < kS32Cols; ++c) {
    int64_t j = col0 + c;
    if (j > M - 1) j = M - 1;
    cp[c] = S + j * ldS;
  }
  double re[kS32Cols], im[kS32Cols];
#pragma unroll
  for (int c = 0; c < kS32Cols; ++c) re[c] = im[c] = 0.0;

  constexpr int kU = kVec ? kS32Unroll / 2 : kS32Unroll;  // load instructions per column per tile
  constexpr int kStep = 64 * kS32Unroll;                  // rows per tile (512)
  const int64_t nfull = (N / kStep) * kStep;
  for (int64_t base = 0; base < nfull; base += kStep) {
    if (kVec) {
      f4v ev[kU], sv[kS32Cols][kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) ev[u] = *reinterpret_cast<const f4v*>(e + base + 2 * (64 * u + lane));
#pragma unroll
      for (int c = 0; c < kS32Cols; ++c)
#pragma unroll
        for (int u = 0; u < kU; ++u)
          sv[c][u] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(cp[c] + base + 2 * (64 * u + lane)));
#pragma unroll
      for (int c = 0; c < kS32Cols; ++c) {
        float r32 = 0.f, i32 = 0.f;  // FP32 accumulation over this row tile
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          cmac_conj32(make_float2(ev[u].x, ev[u].y), make_float2(sv[c][u].x, sv[c][u].y), r32, i32);
          cmac_conj32(make_float2(ev[u].z, ev[u].w), make_float2(sv[c][u].z, sv[c][u].w), r32, i32);
        }
        re[c] += (double)r32;
        im[c] += (double)i32;
      }
    } else {
      float2 ev[kU];
      float2 sv[kS32Cols][kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) ev[u] = e[base + 64 * u + lane];
#pragma unroll
      for (int c = 0; c < kS32Cols; ++c)
#pragma unroll
        for (int u = 0; u < kU; ++u) sv[c][u] = ld_stream(cp[c] + base + 64 * u + lane);
#pragma unroll
      for (int c = 0; c < kS32Cols; ++c) {
        float r32 = 0.f, i32 = 0.f;  // FP32 accumulation over this row tile
#pragma unroll
        for (int u = 0; u < kU; ++u) cmac_conj32(ev[u], sv[c][u], r32, i32);
        re[c] += (double)r32;
        im[c] += (double)i32;
      }
    }
  }
  {
    float r32[kS32Cols], i32[kS32Cols];
#pragma unroll
    for (int c = 0; c < kS32Cols; ++c) r32[c] = i32[c] = 0.f;
    for (int64_t n = nfull + lane; n < N; n += 64) {
      const float2 ev = e[n];
#pragma unroll
      for (int c = 0; c < kS32Cols; ++c) cmac_conj32(ev, ld_stream(cp[c] + n), r32[c], i32[c]);
    }
#pragma unroll
    for (int c = 0; c < kS32Cols; ++c) {
      re[c] += (double)r32[c];
      im[c] += (double)i32[c];
    }
  }

  __shared__ vi scand[kS32ColsPerBlock];
#pragma unroll
  for (int c = 0; c < kS32Cols; ++c) {
    const double cr = wave_sum(re[c]);
    const double ci = wave_sum(im[c]);
    const int64_t j = col0 + c;
    if (lane == c) {
      vi cand = {0.0, -1};
      if (j < M) {
        const double a = acc[j] + (cr * cr + ci * ci);
        acc[j] = a;
        if (kStoreC) c_out[j * ldc] = make_double2(cr, ci);
        if (!(mask && mask[j])) cand = {nrm[j] - a, j};
      }
      scand[wave * kS32Cols + c] = cand;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    TopList L;
    L.clear();
    for (int t = 0; t < kS32ColsPerBlock; ++t) L.insert(scand[t].v, scand[t].i);
#pragma unroll
    for (int r = 0; r < kTop; ++r) {
      partial[blockIdx.x * kTop + r].v = L.v[r];
      partial[blockIdx.x * kTop + r].i = L.i[r];
    }
  }
}

// kTop best of in[0..n) per workgroup chunk -> out[blockIdx.x * kTop ..]
__global__ __launch_bounds__(256) void k_topk_reduce(const ArgMax* __restrict__ in, int64_t n, int64_t chunk,
                                                     ArgMax* __restrict__ out) {
  TopList L;
  L.clear();
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = (lo + chunk < n) ? lo + chunk : n;
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) L.insert(in[t].v, in[t].i);
  block_top_merge(L, out + (int64_t)blockIdx.x * kTop);
}

// kTop best unmasked est_j = nrm_j - acc_j (acc may be NULL) per workgroup
__global__ __launch_bounds__(256) void k_est_topk(const double* __restrict__ nrm, const double* __restrict__ acc,
                                                  const uint8_t* __restrict__ mask, int64_t M,
                                                  ArgMax* __restrict__ out) {
  TopList L;
  L.clear();
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += (int64_t)gridDim.x * blockDim.x) {
    if (mask && mask[j]) continue;
    L.insert(nrm[j] - (acc ? acc[j] : 0.0), j);
  }
  block_top_merge(L, out + (int64_t)blockIdx.x * kTop);
}

__global__ __launch_bounds__(256) void k_round32(const double2* __restrict__ x, int64_t N, float2* __restrict__ y) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n < N) {
    const double2 v = x[n];
    y[n] = make_float2((float)v.x, (float)v.y);
  }
}

__global__ __launch_bounds__(256) void k_iota(int64_t* __restrict__ cols, int64_t start, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) cols[t] = start + t;
}

// two-level reduction of n candidates in `in` to kTop in `out`; tmp holds
// at least kTop * 256 entries
hipError_t topk_final(const ArgMax* in, int64_t n, ArgMax* tmp, ArgMax* out, hipStream_t s) {
  int64_t blocks = (n + 4095) / 4096;
  if (blocks > 256) blocks = 256;
  if (blocks < 1) blocks = 1;
  const int64_t chunk = (n + blocks - 1) / blocks;
  hipLaunchKernelGGL(k_topk_reduce, dim3((unsigned)blocks), dim3(256), 0, s, in, n, chunk, tmp);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_topk_reduce, dim3(1), dim3(256), 0, s, tmp, blocks * kTop, blocks * kTop, out);
  return hipGetLastError();
}

}  // namespace

int64_t sweep32_partials_needed(int64_t M) {
  int64_t a = kTop * ((M + kS32ColsPerBlock - 1) / kS32ColsPerBlock);
  int64_t b = kTop * 2048;  // k_est_topk
  return (a > b ? a : b) + kTop * 256;
}

hipError_t launch_sweep_c(const float2* S, int64_t N, int64_t M, int64_t ldS, const float2* e, const double* nrm,
                          double* acc, const uint8_t* mask, double2* c_out, int64_t ldc, ArgMax* partial,
                          int64_t cap, ArgMax* top, hipStream_t s) {
  const int64_t grid = (M + kS32ColsPerBlock - 1) / kS32ColsPerBlock;
  if (grid * kTop + kTop * 256 > cap) return hipErrorInvalidValue;
  const bool vec = (ldS % 2 == 0) && (reinterpret_cast<uintptr_t>(S) % 16 == 0) &&
                   (reinterpret_cast<uintptr_t>(e) % 16 == 0);
  const dim3 g((unsigned)grid), b(kS32Waves * 64);
  if (c_out) {
    if (vec)
      hipLaunchKernelGGL((k_sweep_c<true, true>), g, b, 0, s, S, N, M, ldS, e, nrm, acc, mask, c_out, ldc, partial);
    else
      hipLaunchKernelGGL((k_sweep_c<true, false>), g, b, 0, s, S, N, M, ldS, e, nrm, acc, mask, c_out, ldc, partial);
  } else {
    if (vec)
      hipLaunchKernelGGL((k_sweep_c<false, true>), g, b, 0, s, S, N, M, ldS, e, nrm, acc, mask, c_out, ldc, partial);
    else
      hipLaunchKernelGGL((k_sweep_c<false, false>), g, b, 0, s, S, N, M, ldS, e, nrm, acc, mask, c_out, ldc,
                         partial);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !top) return err;
  return topk_final(partial, grid * kTop, partial + grid * kTop, top, s);
}

hipError_t launch_sweep_c_final(int64_t M, ArgMax* partial, ArgMax* top, hipStream_t s) {
  const int64_t grid = (M + kS32ColsPerBlock - 1) / kS32ColsPerBlock;
  return topk_final(partial, grid * kTop, partial + grid * kTop, top, s);
}

hipError_t launch_est_topk(const double* nrm, const double* acc, const uint8_t* mask, int64_t M, ArgMax* partial,
                           int64_t cap, ArgMax* top, hipStream_t s) {
  int64_t grid = (M + 255) / 256;
  if (grid > 2048) grid = 2048;
  if (grid * kTop + kTop * 256 > cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_est_topk, dim3((unsigned)grid), dim3(256), 0, s, nrm, acc, mask, M, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return topk_final(partial, grid * kTop, partial + grid * kTop, top, s);
}

hipError_t launch_iota(int64_t* cols, int64_t start, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cols, start, n);
  return hipGetLastError();
}

hipError_t launch_round32(const double2* x, int64_t N, float2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_round32, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, x, N, y);
  return hipGetLastError();
}

}  // namespace rb

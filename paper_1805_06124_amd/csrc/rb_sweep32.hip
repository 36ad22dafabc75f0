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

// conj(e) s added to an FP32 row-tile sum with explicit fused multiply-adds:
// every kernel that forms a complex64 sweep coefficient (the sweep, the
// sweep with predicted vectors, the reranking of a candidate list) rounds
// it the same way, rows in the same order per lane.
__device__ __forceinline__ void cmac_conj32(const float2 e, const float2 s, float& re, float& im) {
  re = __builtin_fmaf(e.y, s.y, __builtin_fmaf(e.x, s.x, re));
  im = __builtin_fmaf(-e.y, s.x, __builtin_fmaf(e.x, s.y, im));
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
        const double a = sweep_acc_add(acc[j], cr, ci);
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

// ---- pivot lookahead for the mixed greedy (see rb_look.hip for the FP64
// form).  All three kernels follow k_sweep_c<true, true>'s arithmetic for a
// column: per lane, FP32 sums over each 512-row tile (rows base + 2 (64 u +
// lane) + {0, 1}, u = 0..3, in that order) added to FP64 totals, the rows past
// the last full tile (n = nfull + lane + 64 t) summed in FP32 and added once,
// then wave_sum and sweep_acc_add.  So a coefficient, an estimate and the
// top-8 set come out the same whichever of them forms it. ----

typedef __attribute__((address_space(3))) void lds_void32_t;
typedef __attribute__((address_space(1))) const void global_void32_t;

// c_v(j) = e_v^H x_j for the V complex64 vectors e[v * ldv ..], every column j
// (16-byte aligned columns and vectors, even ldS); vector 0 advances acc and
// gives the per-workgroup top-8 (the partial layout of k_sweep_c), vector v
// its coefficients c_out[v * M + j].  The vectors' rows of each 512-row tile
// are shared by the workgroup's waves through LDS, copied by direct
// global-to-LDS loads one tile ahead into one of two buffers, as in the FP64
// k_sweep_look.  From four vectors on the workgroup's 16 columns are spread
// over eight waves of two columns each (half the accumulator registers per
// lane, twice the waves per SIMD: 25.7 ms against 27.6 ms with six vectors on
// 10,000 x 1,638,400); each column's arithmetic is the same either way.
template <int V>
constexpr int look32_waves() { return V >= 4 ? 8 : kS32Waves; }
template <int V>
__global__ __launch_bounds__(look32_waves<V>() * 64) void k_sweep_c_look(
    const float2* __restrict__ S, int64_t N, int64_t M, int64_t ldS, const float2* __restrict__ e, int64_t ldv,
    const double* __restrict__ nrm, double* __restrict__ acc, const uint8_t* __restrict__ mask,
    double2* __restrict__ c_out, ArgMax* __restrict__ partial) {
  constexpr int kLW = look32_waves<V>(), kLC = kS32ColsPerBlock / kLW;  // waves, columns per wave
  constexpr int kU = kS32Unroll / 2;
  constexpr int kRows = 64 * kS32Unroll;
  __shared__ __align__(16) float2 sbuf[2][V][kRows];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t col0 = (int64_t)blockIdx.x * kS32ColsPerBlock + (int64_t)wave * kLC;
  const float2* cp[kLC];
#pragma unroll
  for (int c = 0; c < kLC; ++c) {
    int64_t j = col0 + c;
    if (j > M - 1) j = M - 1;
    cp[c] = S + j * ldS;
  }
  double re[V][kLC], im[V][kLC];
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int c = 0; c < kLC; ++c) re[v][c] = im[v][c] = 0.0;
  const int64_t nch = N / kRows;
  // rows [ch kRows, (ch + 1) kRows) of every vector: 64 lanes x 16 B per load
  auto fill = [&](int64_t ch, float2 (*dst)[kRows]) {
    for (int p = wave; p < V * kU; p += kLW) {
      const int v = p / kU, u = p % kU;
      const float2* src = e + v * ldv + ch * kRows + 2 * (64 * u + lane);
      __builtin_amdgcn_global_load_lds((global_void32_t*)src, (lds_void32_t*)&dst[v][2 * 64 * u], 16, 0, 0);
    }
  };
  auto tile = [&](int64_t ch, float2 (*cur)[kRows]) {
    const int64_t base = ch * kRows;
    f4v sv[kLC][kU];
#pragma unroll
    for (int c = 0; c < kLC; ++c)
#pragma unroll
      for (int u = 0; u < kU; ++u)
        sv[c][u] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(cp[c] + base + 2 * (64 * u + lane)));
#pragma unroll
    for (int v = 0; v < V; ++v) {
      f4v ev[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) ev[u] = *reinterpret_cast<const f4v*>(&cur[v][2 * (64 * u + lane)]);
#pragma unroll
      for (int c = 0; c < kLC; ++c) {
        float r32 = 0.f, i32 = 0.f;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          cmac_conj32(make_float2(ev[u].x, ev[u].y), make_float2(sv[c][u].x, sv[c][u].y), r32, i32);
          cmac_conj32(make_float2(ev[u].z, ev[u].w), make_float2(sv[c][u].z, sv[c][u].w), r32, i32);
        }
        re[v][c] += (double)r32;
        im[v][c] += (double)i32;
      }
      // one vector's rows in registers at a time
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  if (nch > 0) fill(0, sbuf[0]);
  __syncthreads();
  for (int64_t ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) fill(ch + 1, sbuf[(ch + 1) & 1]);
    tile(ch, sbuf[ch & 1]);
    __syncthreads();
  }
  const int64_t nfull = nch * kRows;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    float r32[kLC], i32[kLC];
#pragma unroll
    for (int c = 0; c < kLC; ++c) r32[c] = i32[c] = 0.f;
    for (int64_t n = nfull + lane; n < N; n += 64) {
      const float2 ev = e[v * ldv + n];
#pragma unroll
      for (int c = 0; c < kLC; ++c) cmac_conj32(ev, ld_stream(cp[c] + n), r32[c], i32[c]);
    }
#pragma unroll
    for (int c = 0; c < kLC; ++c) {
      re[v][c] += (double)r32[c];
      im[v][c] += (double)i32[c];
    }
  }
  __shared__ vi scand[kS32ColsPerBlock];
#pragma unroll
  for (int c = 0; c < kLC; ++c) {
    const int64_t j = col0 + c;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double cr = wave_sum(re[v][c]);
      const double ci = wave_sum(im[v][c]);
      if (v == 0) {
        if (lane == c) {
          vi cand = {0.0, -1};
          if (j < M) {
            const double a = sweep_acc_add(acc[j], cr, ci);
            acc[j] = a;
            c_out[j] = make_double2(cr, ci);
            if (!(mask && mask[j])) cand = {nrm[j] - a, j};
          }
          scand[wave * kLC + c] = cand;
        }
      } else if (j < M && lane == c + kLC * v) {
        c_out[v * M + j] = make_double2(cr, ci);
      }
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

// A step taken from a prediction: acc_j += |c_j|^2 (c == NULL: none) and the
// top-8 of nrm_j - acc_j per group of kS32ColsPerBlock columns (the partial
// layout of k_sweep_c).
__global__ __launch_bounds__(256) void k_est_apply32(const double* __restrict__ nrm, double* __restrict__ acc,
                                                     const uint8_t* __restrict__ mask, const double2* __restrict__ c,
                                                     int64_t M, ArgMax* __restrict__ partial) {
  __shared__ vi sc[256];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  vi cand = {0.0, -1};
  if (j < M) {
    double a = acc[j];
    if (c) {
      const double2 cj = c[j];
      a = sweep_acc_add(a, cj.x, cj.y);
      acc[j] = a;
    }
    if (!(mask && mask[j])) cand = {nrm[j] - a, j};
  }
  sc[threadIdx.x] = cand;
  __syncthreads();
  constexpr int kGroups = 256 / kS32ColsPerBlock;
  if (threadIdx.x < kGroups) {
    const int64_t g = (int64_t)blockIdx.x * kGroups + threadIdx.x;
    if (g * kS32ColsPerBlock < M) {
      TopList L;
      L.clear();
      for (int t = 0; t < kS32ColsPerBlock; ++t) L.insert(sc[threadIdx.x * kS32ColsPerBlock + t].v,
                                                          sc[threadIdx.x * kS32ColsPerBlock + t].i);
#pragma unroll
      for (int r = 0; r < kTop; ++r) {
        partial[g * kTop + r].v = L.v[r];
        partial[g * kTop + r].i = L.i[r];
      }
    }
  }
}

// One wave per listed column q of the complex64 matrix: its coefficient with
// e and a = acc + |c|^2 (acc_g[q] when first, else the column's slot of
// acc_l; a -> acc_l), and the top-8 of nrm_q - a per workgroup over listed
// columns neither masked nor among the ex.n pivots predicted before.
struct Excl32 {
  int64_t j[kLookMax];
  int n;
};
constexpr int kRerank32Waves = 4;
__global__ __launch_bounds__(kRerank32Waves * 64) void k_rerank32(
    const float2* __restrict__ X, int64_t N, int64_t ldX, const float2* __restrict__ e,
    const ArgMax* __restrict__ list, int K, const double* __restrict__ nrm, const double* __restrict__ acc_g,
    double* __restrict__ acc_l, int first, const uint8_t* __restrict__ mask, Excl32 ex,
    ArgMax* __restrict__ partial) {
  __shared__ vi scand[kRerank32Waves];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot = blockIdx.x * kRerank32Waves + wave;
  const int64_t q = slot < K ? list[slot].i : -1;
  vi cand = {0.0, -1};
  if (q >= 0) {
    const float2* x = X + q * ldX;
    constexpr int kU = kS32Unroll / 2;
    constexpr int kStep = 64 * kS32Unroll;
    const int64_t nfull = (N / kStep) * kStep;
    double re = 0.0, im = 0.0;
    for (int64_t base = 0; base < nfull; base += kStep) {
      f4v ev[kU], sv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        ev[u] = *reinterpret_cast<const f4v*>(e + base + 2 * (64 * u + lane));
        sv[u] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(x + base + 2 * (64 * u + lane)));
      }
      float r32 = 0.f, i32 = 0.f;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        cmac_conj32(make_float2(ev[u].x, ev[u].y), make_float2(sv[u].x, sv[u].y), r32, i32);
        cmac_conj32(make_float2(ev[u].z, ev[u].w), make_float2(sv[u].z, sv[u].w), r32, i32);
      }
      re += (double)r32;
      im += (double)i32;
    }
    float r32 = 0.f, i32 = 0.f;
    for (int64_t n = nfull + lane; n < N; n += 64) cmac_conj32(e[n], ld_stream(x + n), r32, i32);
    re += (double)r32;
    im += (double)i32;
    const double cr = wave_sum(re);
    const double ci = wave_sum(im);
    const double a = sweep_acc_add(first ? acc_g[q] : acc_l[slot], cr, ci);
    if (lane == 0) acc_l[slot] = a;
    bool skip = mask && mask[q];
    for (int t = 0; t < ex.n; ++t) skip = skip || (ex.j[t] == q);
    if (!skip) cand = vi{nrm[q] - a, q};
  }
  if (lane == 0) scand[wave] = cand;
  __syncthreads();
  if (threadIdx.x == 0) {
    TopList L;
    L.clear();
    for (int t = 0; t < kRerank32Waves; ++t) L.insert(scand[t].v, scand[t].i);
#pragma unroll
    for (int r = 0; r < kTop; ++r) {
      partial[blockIdx.x * kTop + r].v = L.v[r];
      partial[blockIdx.x * kTop + r].i = L.i[r];
    }
  }
}

template <int V>
hipError_t launch_sweep_c_look_t(const float2* S, int64_t N, int64_t M, int64_t ldS, const float2* e, int64_t ldv,
                                 const double* nrm, double* acc, const uint8_t* mask, double2* c_out,
                                 ArgMax* partial, hipStream_t s) {
  const int64_t grid = (M + kS32ColsPerBlock - 1) / kS32ColsPerBlock;
  hipLaunchKernelGGL(k_sweep_c_look<V>, dim3((unsigned)grid), dim3(look32_waves<V>() * 64), 0, s, S, N, M, ldS, e,
                     ldv, nrm,
                     acc, mask, c_out, partial);
  return hipGetLastError();
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

bool sweep_c_look_ok(const float2* S, int64_t ldS, const float2* e, int64_t ldv) {
  return (ldS % 2 == 0) && (reinterpret_cast<uintptr_t>(S) % 16 == 0) && (reinterpret_cast<uintptr_t>(e) % 16 == 0) &&
         (ldv % 2 == 0);
}

hipError_t launch_sweep_c_look(const float2* S, int64_t N, int64_t M, int64_t ldS, const float2* e, int64_t ldv, int V,
                               const double* nrm, double* acc, const uint8_t* mask, double2* c_out, ArgMax* partial,
                               int64_t cap, ArgMax* top, hipStream_t s) {
  const int64_t grid = (M + kS32ColsPerBlock - 1) / kS32ColsPerBlock;
  if (grid * kTop + kTop * 256 > cap || !sweep_c_look_ok(S, ldS, e, ldv)) return hipErrorInvalidValue;
  hipError_t err;
  switch (V) {
    case 2: err = launch_sweep_c_look_t<2>(S, N, M, ldS, e, ldv, nrm, acc, mask, c_out, partial, s); break;
    case 3: err = launch_sweep_c_look_t<3>(S, N, M, ldS, e, ldv, nrm, acc, mask, c_out, partial, s); break;
    case 4: err = launch_sweep_c_look_t<4>(S, N, M, ldS, e, ldv, nrm, acc, mask, c_out, partial, s); break;
    case 5: err = launch_sweep_c_look_t<5>(S, N, M, ldS, e, ldv, nrm, acc, mask, c_out, partial, s); break;
    case 6: err = launch_sweep_c_look_t<6>(S, N, M, ldS, e, ldv, nrm, acc, mask, c_out, partial, s); break;
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess || !top) return err;
  return topk_final(partial, grid * kTop, partial + grid * kTop, top, s);
}

hipError_t launch_est_apply32(const double* nrm, double* acc, const uint8_t* mask, const double2* c, int64_t M,
                              ArgMax* partial, int64_t cap, ArgMax* top, hipStream_t s) {
  const int64_t groups = (M + kS32ColsPerBlock - 1) / kS32ColsPerBlock;
  if (groups * kTop + kTop * 256 > cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_est_apply32, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, nrm, acc, mask, c, M, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return topk_final(partial, groups * kTop, partial + groups * kTop, top, s);
}

int64_t rerank32_partials(int K) { return kTop * ((K + kRerank32Waves - 1) / kRerank32Waves) + kTop * 256; }

hipError_t launch_rerank32(const float2* X, int64_t N, int64_t ldX, const float2* e, const ArgMax* list, int K,
                           const double* nrm, const double* acc_g, double* acc_l, int first, const uint8_t* mask,
                           const int64_t* excl, int nexcl, ArgMax* partial, ArgMax* top, hipStream_t s) {
  if (K < 1 || nexcl < 0 || nexcl > kLookMax || !sweep_c_look_ok(X, ldX, e, 2)) return hipErrorInvalidValue;
  Excl32 ex;
  ex.n = nexcl;
  for (int t = 0; t < kLookMax; ++t) ex.j[t] = t < nexcl ? excl[t] : -1;
  const int64_t grid = (K + kRerank32Waves - 1) / kRerank32Waves;
  hipLaunchKernelGGL(k_rerank32, dim3((unsigned)grid), dim3(kRerank32Waves * 64), 0, s, X, N, ldX, e, list, K, nrm,
                     acc_g, acc_l, first, mask, ex, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return topk_final(partial, grid * kTop, partial + grid * kTop, top, s);
}

}  // namespace rb

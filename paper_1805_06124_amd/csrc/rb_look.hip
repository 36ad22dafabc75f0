// Pivot lookahead for the FP64 greedy (Alg. 3, Sec. 6.1.2): one read of the
// working columns serves several greedy steps when the next pivots can be
// named before the read.
//
// At a sweep with the newest basis vector e_0 the host predicts the next
// pivots from a short list of columns (the best estimates before the
// sweep): for each listed column it forms the coefficients and the Eq. (6.3)
// estimates that the coming sweeps would give it (k_rerank), takes the
// largest, orthogonalises that column as the next step would (e_1), and so
// on for e_2, e_3, ...  The sweep then reads X once for all of them
// (k_sweep_look): e_0's coefficients advance the estimates and give the true
// next pivot; the others are only stored.  When the true pivot is the
// predicted one, the next step takes e_1 and its stored coefficients
// (k_est_apply) instead of orthogonalising and sweeping again.
//
// Every coefficient and estimate here is formed with the plain sweep's
// arithmetic (sweep_cmac over rows in increasing order per lane, wave_sum,
// sweep_acc_add), and the predicted vectors are orthogonalised by the same
// code as a regular step, so a greedy with lookahead returns the same bits
// as one without: a wrong prediction costs time, never accuracy.
#include "rb_internal.h"

namespace rb {

namespace {

constexpr int kLookWaves = 4;
constexpr int kLookCols = 4;    // columns per wave
constexpr int kLookUnroll = 2;  // 64-row blocks per chunk
static_assert(kLookWaves * kLookCols == kPivotGroup, "one partial argmax per pivot group");

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void global_void_t;

// c_v(j) = e_v^H x_j for the V vectors E[:, 0..V-1] and every column j.
// Vector 0 advances the running sums (acc_j += |c_0(j)|^2) and gives the
// masked argmax of est_j = nrm_j - acc_j per workgroup; the coefficients of
// vector v go to c_out[v * M + j].
//
// The vectors' rows are shared by the workgroup's four waves through LDS:
// each chunk of kRows rows of all V vectors is copied by direct
// global-to-LDS loads (no registers), one chunk ahead, into one of two
// buffers while the waves read the other; a barrier per chunk hands the
// buffers over.  Loading them per wave instead costs L2-to-L1 traffic and
// registers (one read of X took 10.7 ms against 9.6 ms with V = 5 on
// 10,000 x 409,600).  The two buffers are separate arrays and the loop is
// unrolled by two, so the compiler sees that the rows being read are not
// the ones in flight and keeps the column loads of X in flight together.
template <int V>
__global__ __launch_bounds__(kLookWaves * 64) void k_sweep_look(
    const double2* __restrict__ S, int64_t N, int64_t M, int64_t ldS, const double2* __restrict__ E, int64_t ldE,
    const double* __restrict__ nrm, double* __restrict__ acc, const uint8_t* __restrict__ mask,
    double2* __restrict__ c_out, ArgMax* __restrict__ partial) {
  constexpr int kRows = 64 * kLookUnroll;
  __shared__ double2 sa[V][kRows];
  __shared__ double2 sb[V][kRows];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t col0 = (int64_t)blockIdx.x * kPivotGroup + (int64_t)wave * kLookCols;
  // columns past M read the last column (results discarded)
  const double2* cp[kLookCols];
#pragma unroll
  for (int c = 0; c < kLookCols; ++c) {
    int64_t j = col0 + c;
    if (j > M - 1) j = M - 1;
    cp[c] = S + j * ldS;
  }
  double re[V][kLookCols], im[V][kLookCols];
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int c = 0; c < kLookCols; ++c) re[v][c] = im[v][c] = 0.0;

  const int64_t nch = N / kRows;  // full chunks; the rows past them are read directly
  // rows [ch kRows, (ch + 1) kRows) of every vector into dst: 64 lanes x 16 B per load
  auto fill = [&](int64_t ch, double2 (*dst)[kRows]) {
    for (int p = wave; p < V * kLookUnroll; p += kLookWaves) {
      const int v = p / kLookUnroll, u = p % kLookUnroll;
      const double2* src = E + v * ldE + ch * kRows + 64 * u + lane;
      __builtin_amdgcn_global_load_lds((global_void_t*)src, (lds_void_t*)&dst[v][64 * u], 16, 0, 0);
    }
  };
  auto chunk = [&](int64_t ch, double2 (*cur)[kRows]) {
    const int64_t base = ch * kRows;
    double2 sv[kLookCols][kLookUnroll];
#pragma unroll
    for (int c = 0; c < kLookCols; ++c)
#pragma unroll
      for (int u = 0; u < kLookUnroll; ++u) sv[c][u] = ld_stream(cp[c] + base + 64 * u + lane);
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int u = 0; u < kLookUnroll; ++u) {
        const double2 e = cur[v][64 * u + lane];
#pragma unroll
        for (int c = 0; c < kLookCols; ++c) sweep_cmac(e, sv[c][u], re[v][c], im[v][c]);
      }
  };
  if (nch > 0) fill(0, sa);
  __syncthreads();
  int64_t ch = 0;
  for (; ch + 1 < nch; ch += 2) {
    fill(ch + 1, sb);
    chunk(ch, sa);
    __syncthreads();
    if (ch + 2 < nch) fill(ch + 2, sa);
    chunk(ch + 1, sb);
    __syncthreads();
  }
  if (ch < nch) chunk(ch, sa);
  for (int64_t n = nch * kRows + lane; n < N; n += 64) {
    double2 sv[kLookCols];
#pragma unroll
    for (int c = 0; c < kLookCols; ++c) sv[c] = ld_stream(cp[c] + n);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double2 e = E[v * ldE + n];
#pragma unroll
      for (int c = 0; c < kLookCols; ++c) sweep_cmac(e, sv[c], re[v][c], im[v][c]);
    }
  }

  vi best = {0.0, -1};
#pragma unroll
  for (int c = 0; c < kLookCols; ++c) {
    const int64_t j = col0 + c;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double cr = wave_sum(re[v][c]);
      const double ci = wave_sum(im[v][c]);
      // lane c + 4 v stores (spreads the epilogue over lanes)
      if (j < M && lane == c + kLookCols * v) {
        if (v == 0) {
          const double a = sweep_acc_add(acc[j], cr, ci);
          acc[j] = a;
          c_out[j] = make_double2(cr, ci);
          if (!(mask && mask[j])) best = vi_max(best, vi{nrm[j] - a, j});
        } else {
          c_out[v * M + j] = make_double2(cr, ci);
        }
      }
    }
  }
  best = wave_vi_max(best);
  __shared__ vi sbest[kLookWaves];
  if (lane == 0) sbest[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    vi b = sbest[0];
#pragma unroll
    for (int w = 1; w < kLookWaves; ++w) b = vi_max(b, sbest[w]);
    partial[blockIdx.x].v = b.v;
    partial[blockIdx.x].i = b.i;
  }
}

// A step taken from a lookahead: acc_j += |c_j|^2 with the stored
// coefficients (c == NULL: acc unchanged), and the masked argmax of
// nrm_j - acc_j per group of kPivotGroup columns, the sweep's layout.
__global__ __launch_bounds__(256) void k_est_apply(const double* __restrict__ nrm, double* __restrict__ acc,
                                                   const uint8_t* __restrict__ mask, const double2* __restrict__ c,
                                                   int64_t M, ArgMax* __restrict__ partial) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  vi best = {0.0, -1};
  if (j < M) {
    double a = acc[j];
    if (c) {
      const double2 cj = c[j];
      a = sweep_acc_add(a, cj.x, cj.y);
      acc[j] = a;
    }
    if (!(mask && mask[j])) best = vi{nrm[j] - a, j};
  }
#pragma unroll
  for (int o = 1; o < kPivotGroup; o <<= 1) {
    vi y;
    y.v = __shfl_xor(best.v, o, kWave);
    y.i = __shfl_xor(best.i, o, kWave);
    best = vi_max(best, y);
  }
  if ((threadIdx.x % kPivotGroup) == 0 && j < M) {
    partial[j / kPivotGroup].v = best.v;
    partial[j / kPivotGroup].i = best.i;
  }
}

// The candidate list: the best K of n partial records (index < 0: none),
// best in the vi order (larger value, NaN above numbers, ties to the lower
// index).  One workgroup selects by radix on an order-preserving 64-bit
// key: eight rounds of 8-bit histograms find the K-th record's key; records
// above it all enter the list, records equal to it fill the remaining places
// in index order.  (Fewer rounds would not do: early in a run the best
// thousands of estimates agree to 1e-4.)  Each wave counts into its own
// histogram (most keys share their leading bytes, so one shared histogram
// would serialise the atomics), and one wave sums them and finds the K-th
// key's bin with a prefix sum over lanes.  The keys are read once, thread t
// taking records t, t + 1024, ..., and kept in registers.  The list's order
// is free (the reranking is order-independent), so records above the K-th
// key take places from an LDS counter; only when the records equal to it
// do not all fit are they placed in index order.  Any list gives the same
// greedy; only the number of correct predictions depends on it.
constexpr int kSelThreads = 1024;
constexpr int kSelRounds = 8;
constexpr int kSelPer = 32;  // records per thread kept in registers (n <= 32768)
__device__ __forceinline__ uint64_t order_key(double v, int64_t i) {
  if (i < 0) return 0;  // no record
  if (v != v) return ~0ull;
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}
// exclusive prefix sum over the workgroup (thread order); *total = the sum
__device__ __forceinline__ int block_exscan(int x, int* swave, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == 63) swave[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < kSelThreads / 64; ++w) {
      const int s = swave[w];
      swave[w] = run;
      run += s;
    }
    swave[kSelThreads / 64] = run;
  }
  __syncthreads();
  const int r = swave[wave] + inc - x;
  *total = swave[kSelThreads / 64];
  __syncthreads();
  return r;
}
__global__ __launch_bounds__(kSelThreads) void k_look_list(const ArgMax* __restrict__ in, int64_t n, int K,
                                                            ArgMax* __restrict__ list) {
  __shared__ unsigned hist[kSelThreads / 64][256];  // one histogram per wave (fewer colliding atomics)
  __shared__ uint64_t s_prefix;
  __shared__ int s_above, s_all, s_na, s_nb;
  __shared__ int swave[kSelThreads / 64 + 1];
  uint64_t key[kSelPer];
#pragma unroll
  for (int q = 0; q < kSelPer; ++q) {
    const int64_t t = threadIdx.x + (int64_t)kSelThreads * q;
    key[q] = t < n ? order_key(in[t].v, in[t].i) : 0;
  }
  uint64_t prefix = 0;
  int shift = 64, above = 0, all = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < kSelRounds; ++r) {
    shift -= 8;
#pragma unroll
    for (int b = lane; b < 256; b += 64) hist[wave][b] = 0;  // the wave's own copy: no barrier needed
#pragma unroll
    for (int q = 0; q < kSelPer; ++q) {
      const uint64_t k = key[q];
      if (k == 0) continue;
      if (r > 0 && (k >> (shift + 8)) != (prefix >> (shift + 8))) continue;
      atomicAdd(&hist[wave][(k >> shift) & 255], 1u);
    }
    __syncthreads();
    if (wave == 0) {
      // lane l holds bins 255 - 4 l .. 252 - 4 l (descending); the K-th key's
      // bin is the first, from the top, at which the running count reaches K
      int c[4], sum = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = 255 - 4 * lane - u;
        int t = 0;
#pragma unroll
        for (int w = 0; w < kSelThreads / 64; ++w) t += (int)hist[w][b];
        c[u] = t;
        sum += t;
      }
      int inc = sum;  // inclusive count over lanes 0..lane
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += y;
      }
      const uint64_t hit = __ballot(above + inc >= K);
      if (lane == 0) s_all = hit == 0;
      if (hit != 0 && lane == __builtin_ctzll(hit)) {
        int cum = above + inc - sum, u = 0;
        for (; u < 3; ++u) {
          if (cum + c[u] >= K) break;
          cum += c[u];
        }
        s_prefix = prefix | ((uint64_t)(255 - 4 * lane - u) << shift);
        s_above = cum;
      }
    }
    __syncthreads();
    all = s_all;
    if (all) break;
    prefix = s_prefix;
    above = s_above;
  }
  // records above the K-th key (or all, when fewer than K exist)
  if (threadIdx.x == 0) {
    s_na = 0;
    s_nb = 0;
  }
  __syncthreads();
  int nb_mine = 0;
#pragma unroll
  for (int q = 0; q < kSelPer; ++q) {
    const uint64_t k = key[q];
    if (k == 0) continue;
    if (all || k > prefix) {
      const int64_t t = threadIdx.x + (int64_t)kSelThreads * q;
      list[atomicAdd(&s_na, 1)] = in[t];
    } else if (k == prefix) {
      ++nb_mine;
    }
  }
  int tb;
  (void)block_exscan(nb_mine, swave, &tb);  // also orders the counter updates above
  const int ta = all ? s_na : above;
  if (!all && ta + tb <= K) {
    // every record equal to the K-th key fits
#pragma unroll
    for (int q = 0; q < kSelPer; ++q) {
      if (key[q] != 0 && key[q] == prefix) {
        const int64_t t = threadIdx.x + (int64_t)kSelThreads * q;
        list[ta + atomicAdd(&s_nb, 1)] = in[t];
      }
    }
  } else if (!all) {
    // ties at the K-th key: the lowest indices first, one block of records at a time
    int placed = ta;
#pragma unroll
    for (int q = 0; q < kSelPer; ++q) {
      const int mine = (key[q] != 0 && key[q] == prefix) ? 1 : 0;
      int tot;
      const int off = block_exscan(mine, swave, &tot);
      if (mine && placed + off < K) list[placed + off] = in[threadIdx.x + (int64_t)kSelThreads * q];
      placed += tot;
    }
  }
  const int filled = all ? ta : (ta + tb < K ? ta + tb : K);
  for (int r = filled + threadIdx.x; r < K; r += kSelThreads) {
    list[r].v = 0.0;
    list[r].i = -1;
  }
}

// out[i] = the best of in[i f .. i f + f - 1] (vi order), i < nout
__global__ __launch_bounds__(256) void k_coarsen(const ArgMax* __restrict__ in, int64_t n, int64_t f,
                                                 ArgMax* __restrict__ out, int64_t nout) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nout) return;
  vi best = {0.0, -1};
  const int64_t j1 = (i + 1) * f < n ? (i + 1) * f : n;
  for (int64_t j = i * f; j < j1; ++j) best = vi_max(best, vi{in[j].v, in[j].i});
  out[i].v = best.v;
  out[i].i = best.i;
}

// One wave per listed column q: c = e^H x_q (the sweep's order), a = acc + |c|^2
// (acc from acc_g[q] when first, else this column's slot of acc_l; a goes to
// acc_l), and the workgroup's argmax of nrm_q - a over listed columns that are
// neither masked nor among the pivots predicted before (chain[0..nprev)).
// If the last of those was not accepted the chain has ended: no candidate.
constexpr int kRerankWaves = 4;
constexpr int kRerankUnroll = 8;
__global__ __launch_bounds__(kRerankWaves * 64) void k_rerank(
    const double2* __restrict__ X, int64_t N, int64_t ldX, const double2* __restrict__ e,
    const ArgMax* __restrict__ list, int K, const double* __restrict__ nrm, const double* __restrict__ acc_g,
    double* __restrict__ acc_l, int first, const uint8_t* __restrict__ mask, const GsState* __restrict__ chain,
    int nprev, ArgMax* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot = blockIdx.x * kRerankWaves + wave;
  const bool alive = nprev == 0 || chain[nprev - 1].accept != 0;
  vi best = {0.0, -1};
  const int64_t q = (alive && slot < K) ? list[slot].i : -1;
  if (q >= 0) {
    const double2* x = X + q * ldX;
    double re = 0.0, im = 0.0;
    for (int64_t n0 = lane; n0 < N; n0 += 64 * kRerankUnroll) {
      double2 xv[kRerankUnroll], ev[kRerankUnroll];
#pragma unroll
      for (int u = 0; u < kRerankUnroll; ++u) {
        const int64_t n = n0 + 64 * u;
        xv[u] = n < N ? ld_stream(x + n) : make_double2(0.0, 0.0);
        ev[u] = n < N ? e[n] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < kRerankUnroll; ++u)
        if (n0 + 64 * u < N) sweep_cmac(ev[u], xv[u], re, im);
    }
    const double cr = wave_sum(re);
    const double ci = wave_sum(im);
    const double a = sweep_acc_add(first ? acc_g[q] : acc_l[slot], cr, ci);
    if (lane == 0) acc_l[slot] = a;
    bool skip = mask && mask[q];
    for (int t = 0; t < nprev; ++t) skip = skip || (chain[t].J == q);
    if (!skip) best = vi{nrm[q] - a, q};
  }
  // every lane of a wave holds the same record
  __shared__ vi sbest[kRerankWaves];
  if (lane == 0) sbest[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    vi b = sbest[0];
#pragma unroll
    for (int w = 1; w < kRerankWaves; ++w) b = vi_max(b, sbest[w]);
    partial[blockIdx.x].v = b.v;
    partial[blockIdx.x].i = b.i;
  }
}

template <int V>
hipError_t launch_sweep_look_t(const double2* S, int64_t N, int64_t M, int64_t ldS, const double2* E, int64_t ldE,
                               const double* nrm, double* acc, const uint8_t* mask, double2* c_out,
                               ArgMax* partial, hipStream_t s) {
  const int64_t grid = (M + kPivotGroup - 1) / kPivotGroup;
  hipLaunchKernelGGL(k_sweep_look<V>, dim3((unsigned)grid), dim3(kLookWaves * 64), 0, s, S, N, M, ldS, E, ldE, nrm,
                     acc, mask, c_out, partial);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep_look(const double2* S, int64_t N, int64_t M, int64_t ldS, const double2* E, int64_t ldE,
                             int V, const double* nrm, double* acc, const uint8_t* mask, double2* c_out,
                             ArgMax* partial, int64_t npartial_cap, hipStream_t s) {
  if ((M + kPivotGroup - 1) / kPivotGroup > npartial_cap || (M + kPivotGroup - 1) / kPivotGroup > 0x7fffffff)
    return hipErrorInvalidValue;
  switch (V) {
    case 2: return launch_sweep_look_t<2>(S, N, M, ldS, E, ldE, nrm, acc, mask, c_out, partial, s);
    case 3: return launch_sweep_look_t<3>(S, N, M, ldS, E, ldE, nrm, acc, mask, c_out, partial, s);
    case 4: return launch_sweep_look_t<4>(S, N, M, ldS, E, ldE, nrm, acc, mask, c_out, partial, s);
    case 5: return launch_sweep_look_t<5>(S, N, M, ldS, E, ldE, nrm, acc, mask, c_out, partial, s);
    case 6: return launch_sweep_look_t<6>(S, N, M, ldS, E, ldE, nrm, acc, mask, c_out, partial, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_est_apply(const double* nrm, double* acc, const uint8_t* mask, const double2* c, int64_t M,
                            ArgMax* partial, int64_t npartial_cap, hipStream_t s) {
  if ((M + kPivotGroup - 1) / kPivotGroup > npartial_cap) return hipErrorInvalidValue;
  const int64_t grid = (M + 255) / 256;
  hipLaunchKernelGGL(k_est_apply, dim3((unsigned)grid), dim3(256), 0, s, nrm, acc, mask, c, M, partial);
  return hipGetLastError();
}

int64_t look_list_scratch(int64_t n) { return n > (int64_t)kSelThreads * kSelPer ? (int64_t)kSelThreads * kSelPer : 0; }

hipError_t launch_look_list(const ArgMax* partial, int64_t n, int K, ArgMax* list, ArgMax* scratch, hipStream_t s) {
  constexpr int64_t kMaxRec = (int64_t)kSelThreads * kSelPer;
  if (K < 1 || K > kLookListMax || n < 1) return hipErrorInvalidValue;
  const ArgMax* src = partial;
  if (n > kMaxRec) {
    // more records than one selection holds: the maxima of f consecutive ones
    if (!scratch) return hipErrorInvalidValue;
    const int64_t f = (n + kMaxRec - 1) / kMaxRec;
    const int64_t nout = (n + f - 1) / f;
    hipLaunchKernelGGL(k_coarsen, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, partial, n, f, scratch, nout);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    src = scratch;
    n = nout;
  }
  hipLaunchKernelGGL(k_look_list, dim3(1), dim3(kSelThreads), 0, s, src, n, K, list);
  return hipGetLastError();
}

int64_t rerank_partials(int K) { return (K + kRerankWaves - 1) / kRerankWaves; }

hipError_t launch_rerank(const double2* X, int64_t N, int64_t ldX, const double2* e, const ArgMax* list, int K,
                         const double* nrm, const double* acc_g, double* acc_l, int first, const uint8_t* mask,
                         const GsState* chain, int nprev, ArgMax* partial, ArgMax* result, hipStream_t s) {
  if (K < 1 || nprev < 0 || nprev > kLookMax || (nprev > 0 && !chain)) return hipErrorInvalidValue;
  const int64_t grid = rerank_partials(K);
  hipLaunchKernelGGL(k_rerank, dim3((unsigned)grid), dim3(kRerankWaves * 64), 0, s, X, N, ldX, e, list, K, nrm,
                     acc_g, acc_l, first, mask, chain, nprev, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_argmax_records(partial, grid, result, s);
}

}  // namespace rb

// Learned coefficient surrogate: an MLP (snapshot parameters and features
// of them) -> [Re c; Im c] with layers din -> hidden -> hidden -> hidden ->
// dout, tanh hidden activations, BF16 weights and activations, FP32
// accumulation and FP32 master weights.  The hidden and output layers run on
// BF16 matrix cores (v_mfma_f32_16x16x32_bf16), their bias gradients ride
// along in the weight-gradient products.  A first layer with din <= 4
// inputs and its gradients are vector kernels; a wider one (up to
// kMaxDin inputs) takes the same matrix-core products as the others, on a
// BF16 copy of the inputs.
//
// Parameter layout (FP32 master and BF16 copy share offsets), row-major
// [in][out]:  W1 (din x h), b1 (h), W2 (h x h), b2, W3 (h x h), b3,
// W4 (h x dout), b4 (dout).  Activations are row-major [batch][feature].
#include <cmath>

#include "rb_host.h"

namespace rb {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// The element-wise arithmetic shared by the layer-by-layer kernels and the
// fused training step (one definition, so both round identically).
__device__ __forceinline__ uint16_t act_tanh(float acc, float bias) { return f2bf(tanhf(acc + bias)); }
__device__ __forceinline__ uint16_t act_dtanh(float acc, float h) { return f2bf(acc * (1.f - h * h)); }
__device__ __forceinline__ uint16_t mse_grad(float d, float scale) { return f2bf(2.f * d * scale); }
__device__ __forceinline__ void adam_update(float& w, float& m, float& v, float g, float lr, float b1, float b2,
                                            float eps, float c1, float c2) {
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  w = w - lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ---------------------------------------------------------------- GEMM --
// C(m, n) = sum_k A(m, k) B(k, n), A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn], BF16 operands, FP32 accumulation.
// Block tile 64 x 64, 4 waves as 2 x 2 (32 x 32 each = 2 x 2 MFMA tiles).
// K is staged in LDS as [row][k], so that each lane's 8 operand values are
// one 16-byte read, kStage chunks of 32 at a time.  For the common layouts
// the loads of a stage carry no branch: a thread issues all of them before
// the first is stored, so one memory latency covers the stage rather than
// one per chunk.
// v_mfma_f32_16x16x32_bf16: A lane l holds A[l%16][8(l/16) .. +7],
// B lane l holds B[8(l/16) .. +7][l%16], result lane l register r holds
// D[4(l/16) + r][l%16].
enum Epi { kEpiStore = 0, kEpiBiasTanh = 1, kEpiBias = 2, kEpiDTanh = 3 };

constexpr int kGT = 64, kGK = 32, kStage = 2, kGKP = kStage * kGK + 8;

// Operand layouts X(r, k) = X[r*sr + k*sk] for staging a 64 x 32 chunk
// X(r0 + r, k0 + kk) into LDS as dst[r][kk]; each thread moves 8 values.
// kK16, kK4: K contiguous (sk == 1) with 16- or 4-byte aligned rows; thread
// t holds X(r0 + t/4, k0 + 8(t%4) + i).  kR16, kR4: R contiguous (sr == 1);
// thread t holds X(r0 + 8(t%8) + i, k0 + t/8), i < 8.  kGen: any strides,
// scalar loads.  Values outside the matrix are zero.
enum Lay { kGen = 0, kK16 = 1, kR16 = 2, kK4 = 3, kR4 = 4 };

// Guarded load of a chunk for a layout chosen at run time.
__device__ __forceinline__ uint4 load_tile(const uint16_t* __restrict__ X, int64_t sr, int64_t sk, int64_t R,
                                           int64_t K, int64_t r0, int64_t k0, int vec, int tid) {
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  if (vec == kK16 || vec == kK4) {
    const int64_t gr = r0 + (tid >> 2), gk = k0 + (tid & 3) * 8;
    if (gr < R && gk + 7 < K) {
      if (vec == kK16) {
        return *reinterpret_cast<const uint4*>(X + gr * sr + gk);
      } else {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(X + gr * sr + gk);
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = src[i];
      }
    } else if (gr < R) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t lo = (gk + 2 * i < K) ? X[gr * sr + gk + 2 * i] : 0u;
        const uint32_t hi = (gk + 2 * i + 1 < K) ? X[gr * sr + gk + 2 * i + 1] : 0u;
        w[i] = lo | (hi << 16);
      }
    }
  } else if (vec == kR16 || vec == kR4) {
    const int64_t gk = k0 + (tid >> 3), gr = r0 + (tid & 7) * 8;
    if (gk < K && gr + 7 < R) {
      if (vec == kR16) {
        return *reinterpret_cast<const uint4*>(X + gk * sk + gr);
      } else {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(X + gk * sk + gr);
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = src[i];
      }
    } else if (gk < K) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t lo = (gr + 2 * i < R) ? X[gk * sk + gr + 2 * i] : 0u;
        const uint32_t hi = (gr + 2 * i + 1 < R) ? X[gk * sk + gr + 2 * i + 1] : 0u;
        w[i] = lo | (hi << 16);
      }
    }
  } else {
    const int64_t gr = r0 + (tid >> 2), gk = k0 + (tid & 3) * 8;
    if (gr < R) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t lo = (gk + 2 * i < K) ? X[gr * sr + (gk + 2 * i) * sk] : 0u;
        const uint32_t hi = (gk + 2 * i + 1 < K) ? X[gr * sr + (gk + 2 * i + 1) * sk] : 0u;
        w[i] = lo | (hi << 16);
      }
    }
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 to_uint4(u32x4 v) { return make_uint4(v[0], v[1], v[2], v[3]); }

// Branch-free load of a chunk for a layout fixed at compile time: the
// address is clamped into the matrix and a value outside it replaced by zero
// with a select (on whole 4-word vectors: a select of one loaded word on a
// scalar condition is turned into a branch around the load by the compiler).  A thread's 8 values (kK16, kR16) or each pair of them
// (kK4, kR4) lie wholly inside or wholly outside the matrix when the extent
// along the contiguous direction is a multiple of 8 (K for kK16, R for kR16)
// or of 2 (K for kK4, R for kR4); the host launches these layouts only then.
template <int L>
__device__ __forceinline__ uint4 load_fast(const uint16_t* __restrict__ X, int64_t sr, int64_t sk, int64_t R,
                                           int64_t K, int64_t r0, int64_t k0, int tid) {
  const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
  if (L == kK16 || L == kK4) {
    const int64_t gr = r0 + (tid >> 2), gk = k0 + (tid & 3) * 8;
    const bool rok = gr < R;
    const uint16_t* row = X + (rok ? gr : R - 1) * sr;
    if (L == kK16) {
      const bool ok = rok && gk < K;
      const uint4 v = *reinterpret_cast<const uint4*>(row + (gk < K ? gk : K - 8));
      return ok ? v : zero;
    } else {
      u32x4 x, keep;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t k = gk + 2 * i;
        x[i] = *reinterpret_cast<const uint32_t*>(row + (k < K ? k : K - 2));
        keep[i] = (rok && k < K) ? ~0u : 0u;
      }
      return to_uint4(x & keep);
    }
  } else {
    const int64_t gk = k0 + (tid >> 3), gr = r0 + (tid & 7) * 8;
    const bool kok = gk < K;
    const uint16_t* col = X + (kok ? gk : K - 1) * sk;
    if (L == kR16) {
      const bool ok = kok && gr < R;
      const uint4 v = *reinterpret_cast<const uint4*>(col + (gr < R ? gr : R - 8));
      return ok ? v : zero;
    } else {
      u32x4 x, keep;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = gr + 2 * i;
        x[i] = *reinterpret_cast<const uint32_t*>(col + (r < R ? r : R - 2));
        keep[i] = (kok && r < R) ? ~0u : 0u;
      }
      return to_uint4(x & keep);
    }
  }
}

// LDS placement of tile element (r, c): the 8-wide column group is XORed
// with (r / 8) % 8, so that the rows 8 apart written by one store
// instruction of the R-contiguous layouts fall in different banks (with
// 16-byte aligned rows they would share one); the row pad keeps adjacent
// rows in different banks for the operand reads.  Needs an even kStage.
static_assert(kStage % 2 == 0, "the swizzle permutes groups within blocks of 8");
__device__ __forceinline__ int swz(int r, int c) { return (((c >> 3) ^ ((r >> 3) & 7)) << 3) | (c & 7); }

// writes a thread's values of a chunk to column koff of dst; rowwise says
// whether they run along R (kR16, kR4) or along K (the other layouts)
__device__ __forceinline__ void store_tile(uint4 v, bool rowwise, uint16_t (*dst)[kGKP], int koff, int tid) {
  if (rowwise) {
    const int kk = koff + (tid >> 3), r = (tid & 7) * 8;
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dst[r + 2 * i][swz(r, kk)] = (uint16_t)(w[i] & 0xffffu);
      dst[r + 2 * i + 1][swz(r, kk)] = (uint16_t)(w[i] >> 16);
    }
  } else {
    *reinterpret_cast<uint4*>(&dst[tid >> 2][swz(tid >> 2, koff + (tid & 3) * 8)]) = v;
  }
}

// one K chunk of 32 at column ko of the staged tiles: 2 x 2 MFMA tiles per wave
__device__ __forceinline__ void mma_chunk(const uint16_t (*sA)[kGKP], const uint16_t (*sB)[kGKP], int ko, int lane,
                                          int wm, int wn, f4v (&acc)[2][2]) {
  bf16x8 a[2], b[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int ra = wm * 32 + 16 * t + (lane & 15), rb = wn * 32 + 16 * t + (lane & 15);
    a[t] = *reinterpret_cast<const bf16x8*>(&sA[ra][swz(ra, ko + 8 * (lane >> 4))]);
    b[t] = *reinterpret_cast<const bf16x8*>(&sB[rb][swz(rb, ko + 8 * (lane >> 4))]);
  }
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
      acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
}

// thread (n = tid / 4, q = tid % 4) adds sB[n][ko + 8q .. ko + 8q + 7]
__device__ __forceinline__ void colsum_chunk(const uint16_t (*sB)[kGKP], int ko, int tid, float& cs) {
  const uint4 w = *reinterpret_cast<const uint4*>(&sB[tid >> 2][swz(tid >> 2, ko + 8 * (tid & 3))]);
  const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    cs += __uint_as_float(u[i] << 16);
    cs += __uint_as_float(u[i] & 0xffff0000u);
  }
}

// LA, LB: the layouts of A (as X(m, k)) and B (as X(n, k)), or kGen for
// layouts passed at run time in vecA, vecB (guarded loads, one chunk at a
// time).  Split over K (kEpiStore only): workgroup z reduces k in
// [z kc, (z+1) kc) and stores its partial product at C + z cz; one split is
// kc = K, cz = 0.  With csum set (kEpiStore only), the workgroups of the
// first row of tiles also add up the columns of B over their K range, from
// the staged tiles, and store them as row M of C: C(M, n) = sum_k B(k, n).
// That is the bias gradient beside a weight gradient dW = H^T dZ.
template <int kEpi, int LA, int LB>
__device__ __forceinline__ void gemm_tile(int64_t M, int64_t N, int64_t K, const uint16_t* __restrict__ A,
                                          int64_t sam, int64_t sak, const uint16_t* __restrict__ B, int64_t sbk,
                                          int64_t sbn, float* __restrict__ C, int64_t ldc,
                                          const float* __restrict__ bias, uint16_t* __restrict__ Cb, int64_t ldcb,
                                          const uint16_t* __restrict__ H, int64_t ldh, int vecA, int vecB,
                                          int64_t kc, int64_t cz, int csum, int64_t bx, int64_t by, int64_t bz,
                                          uint16_t (*sA)[kGKP], uint16_t (*sB)[kGKP]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = by * kGT, n0 = bx * kGT;
  f4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (f4v){0.f, 0.f, 0.f, 0.f};

  const int64_t kb = bz * kc;
  const int64_t ke = (kb + kc < K) ? kb + kc : K;
  if (kEpi == kEpiStore) C += bz * cz;
  const bool do_csum = kEpi == kEpiStore && csum && by == 0;
  float cs = 0.f;
  // the epilogue's operands (bias, or the activations for the tanh
  // derivative) do not depend on the product: load them first, from clamped
  // addresses, so that their latency overlaps the main loop's
  float bv[2] = {0.f, 0.f};
  float hv[2][2][4];
#pragma unroll
  for (int tb = 0; tb < 2; ++tb) {
    const int64_t n = n0 + wn * 32 + 16 * tb + (lane & 15);
    const int64_t nc = n < N ? n : N - 1;
    if (kEpi == kEpiBiasTanh || kEpi == kEpiBias) bv[tb] = bias[nc];
#pragma unroll
    for (int ta = 0; ta < 2; ++ta)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 32 + 16 * ta + 4 * (lane >> 4) + r;
        hv[ta][tb][r] = kEpi == kEpiDTanh ? bf2f(H[(m < M ? m : M - 1) * ldh + nc]) : 0.f;
      }
  }
  for (int64_t k0 = kb; k0 < ke; k0 += kStage * kGK) {
    const int64_t left = (ke - k0 + kGK - 1) / kGK;
    const int nsub = left < kStage ? (int)left : kStage;
    if (LA != kGen && LB != kGen) {
      // chunks past ke load clamped addresses and hold zeros
      uint4 ra[kStage], rb[kStage];
#pragma unroll
      for (int c = 0; c < kStage; ++c) {
        ra[c] = load_fast<LA>(A, sam, sak, M, ke, m0, k0 + c * kGK, tid);
        rb[c] = load_fast<LB>(B, sbn, sbk, N, ke, n0, k0 + c * kGK, tid);
      }
#pragma unroll
      for (int c = 0; c < kStage; ++c) {
        store_tile(ra[c], LA == kR16 || LA == kR4, sA, c * kGK, tid);
        store_tile(rb[c], LB == kR16 || LB == kR4, sB, c * kGK, tid);
      }
    } else {
      for (int c = 0; c < nsub; ++c) {
        store_tile(load_tile(A, sam, sak, M, ke, m0, k0 + c * kGK, vecA, tid), vecA == kR16 || vecA == kR4, sA,
                   c * kGK, tid);
        store_tile(load_tile(B, sbn, sbk, N, ke, n0, k0 + c * kGK, vecB, tid), vecB == kR16 || vecB == kR4, sB,
                   c * kGK, tid);
      }
    }
    __syncthreads();
    if (nsub == kStage) {
#pragma unroll
      for (int c = 0; c < kStage; ++c) {
        if (do_csum) colsum_chunk(sB, c * kGK, tid, cs);
        mma_chunk(sA, sB, c * kGK, lane, wm, wn, acc);
      }
    } else {
      for (int c = 0; c < nsub; ++c) {
        if (do_csum) colsum_chunk(sB, c * kGK, tid, cs);
        mma_chunk(sA, sB, c * kGK, lane, wm, wn, acc);
      }
    }
    __syncthreads();
  }
  if (do_csum) {
    // the four partial sums of a column sit in adjacent lanes; (q0 + q1) + (q2 + q3)
    cs += __shfl_xor(cs, 1, 64);
    cs += __shfl_xor(cs, 2, 64);
    const int64_t n = n0 + (tid >> 2);
    if ((tid & 3) == 0 && n < N) C[M * ldc + n] = cs;
  }
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 32 + 16 * ta + 4 * (lane >> 4) + r;
        const int64_t n = n0 + wn * 32 + 16 * tb + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[ta][tb][r];
        if (kEpi == kEpiStore) {
          C[m * ldc + n] = v;
        } else if (kEpi == kEpiBiasTanh) {
          Cb[m * ldcb + n] = act_tanh(v, bv[tb]);
        } else if (kEpi == kEpiBias) {
          C[m * ldc + n] = v + bv[tb];
        } else {
          Cb[m * ldcb + n] = act_dtanh(v, hv[ta][tb][r]);
        }
      }
}


template <int kEpi, int LA, int LB>
__global__ __launch_bounds__(256) void k_gemm_bf16(int64_t M, int64_t N, int64_t K, const uint16_t* __restrict__ A,
                                                   int64_t sam, int64_t sak, const uint16_t* __restrict__ B,
                                                   int64_t sbk, int64_t sbn, float* __restrict__ C, int64_t ldc,
                                                   const float* __restrict__ bias, uint16_t* __restrict__ Cb,
                                                   int64_t ldcb, const uint16_t* __restrict__ H, int64_t ldh,
                                                   int vecA, int vecB, int64_t kc, int64_t cz, int csum) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[kGT][kGKP];
  __shared__ __attribute__((aligned(16))) uint16_t sB[kGT][kGKP];
  gemm_tile<kEpi, LA, LB>(M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, Cb, ldcb, H, ldh, vecA, vecB, kc, cz, csum,
                          blockIdx.x, blockIdx.y, blockIdx.z, sA, sB);
}

// Up to four split-K weight-gradient products (kEpiStore, with the bias row)
// in one launch: workgroup b belongs to the product p with start[p] <= b <
// start[p + 1] and takes the tile and split that k_gemm_bf16 would give it
// with that product's grid (gx, gy, splits).  lay[p] selects the staging:
// 0 both R16, 1 A R16 B R4, 2 A R4 B R16, 3 both R4, 4 guarded.
struct GemmGroup {
  int64_t M[4], N[4], K[4];
  const uint16_t* A[4];
  int64_t sam[4], sak[4];
  const uint16_t* B[4];
  int64_t sbk[4], sbn[4];
  float* C[4];
  int64_t ldc[4], kc[4], cz[4];
  int vecA[4], vecB[4], lay[4], gx[4], gy[4], splits[4];
  int start[5];
  // every product has a multiple of 8 splits: the 8 XCDs (which take the
  // workgroups in turn) each get a contiguous eighth of the batch, the rows
  // the row kernel wrote on the same XCD
  int xcd;
};

__global__ __launch_bounds__(256) void k_gemm_group(GemmGroup g) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[kGT][kGKP];
  __shared__ __attribute__((aligned(16))) uint16_t sB[kGT][kGKP];
  const int b = blockIdx.x;
  int p = 0;
  while (p < 3 && b >= g.start[p + 1]) ++p;
  const int loc = b - g.start[p];
  int64_t bx, by, bz;
  if (g.xcd) {
    const int spx = g.splits[p] / 8, j = loc / 8, tile = j / spx;
    bz = (loc % 8) * spx + j % spx;
    bx = tile % g.gx[p];
    by = tile / g.gx[p];
  } else {
    bx = loc % g.gx[p];
    by = (loc / g.gx[p]) % g.gy[p];
    bz = loc / (g.gx[p] * g.gy[p]);
  }
#define RB_GEMM_CASE(LA, LB)                                                                                       \
  gemm_tile<kEpiStore, LA, LB>(g.M[p], g.N[p], g.K[p], g.A[p], g.sam[p], g.sak[p], g.B[p], g.sbk[p], g.sbn[p],      \
                               g.C[p], g.ldc[p], nullptr, nullptr, 0, nullptr, 0, g.vecA[p], g.vecB[p], g.kc[p],   \
                               g.cz[p], 1, bx, by, bz, sA, sB)
  switch (g.lay[p]) {
    case 0: RB_GEMM_CASE(kR16, kR16); break;
    case 1: RB_GEMM_CASE(kR16, kR4); break;
    case 2: RB_GEMM_CASE(kR4, kR16); break;
    case 3: RB_GEMM_CASE(kR4, kR4); break;
    default: RB_GEMM_CASE(kGen, kGen); break;
  }
#undef RB_GEMM_CASE
}

// BF16 copy of the FP32 inputs (a wide first layer's matrix-core operand)
__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ X, int64_t n, uint16_t* __restrict__ Xb) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) Xb[t] = f2bf(X[t]);
}

// first layer (din inputs, FP32 in): H1 = bf16(tanh(X W1 + b1))
__global__ __launch_bounds__(256) void k_layer1_fwd(const float* __restrict__ X, int64_t B, int din,
                                                    const uint16_t* __restrict__ W1, const float* __restrict__ b1,
                                                    int h, uint16_t* __restrict__ H1) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= B * h) return;
  const int64_t b = t / h;
  const int o = (int)(t % h);
  float z = b1[o];
  for (int i = 0; i < din; ++i) z += X[b * din + i] * bf2f(W1[(int64_t)i * h + o]);
  H1[t] = f2bf(tanhf(z));
}

// column sums over the batch of a BF16 matrix D (B x d): db[o] = sum_b D[b][o]
// and, if X is given, dW[i][o] = sum_b X[b][i] D[b][o] (i < din <= 4).
// Partial sums per workgroup row chunk go to part[(chunk)(din+1) d], reduced
// by k_colsum_final in a fixed order.  The row loads of a chunk carry no
// branch (clamped row, zero by select), so they are all in flight together.
constexpr int kColRows = 32;
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* __restrict__ D, int64_t B, int d,
                                                const float* __restrict__ X, int din, float* __restrict__ part) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= d) return;
  const int64_t b0 = (int64_t)blockIdx.y * kColRows;
  const int nb = (B - b0 < kColRows) ? (int)(B - b0) : kColRows;
  float v[kColRows];
#pragma unroll
  for (int r = 0; r < kColRows; ++r) {
    const float x = bf2f(D[(b0 + (r < nb ? r : nb - 1)) * d + o]);
    v[r] = r < nb ? x : 0.f;
  }
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < kColRows; ++r) s += v[r];
  float* p = part + (int64_t)blockIdx.y * ((X ? din : 0) + 1) * d;
  p[o] = s;
  if (!X) return;
  for (int i = 0; i < din; ++i) {
    float xv[kColRows];
#pragma unroll
    for (int r = 0; r < kColRows; ++r) xv[r] = X[(b0 + (r < nb ? r : nb - 1)) * din + i];
    float sx = 0.f;
#pragma unroll
    for (int r = 0; r < kColRows; ++r) sx += xv[r] * v[r];
    p[(int64_t)(i + 1) * d + o] = sx;
  }
}
// the partial sums of k_colsum added per output: 16 outputs per workgroup,
// 16 lanes per output each adding every 16th chunk, the 16 sums then added
// in a fixed butterfly order (every lane ends with the same value)
__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ part, int64_t chunks, int64_t len,
                                                      float* __restrict__ db, float* __restrict__ dW, int d) {
  const int q = threadIdx.x & 15;
  const int64_t t = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  float s = 0.f;
  if (t < len) {
#pragma unroll 8
    for (int64_t c = q; c < chunks; c += 16) s += part[c * len + t];
  }
  s += __shfl_xor(s, 8, 64);
  s += __shfl_xor(s, 4, 64);
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 1, 64);
  if (q == 0 && t < len) {
    if (t < d)
      db[t] = s;
    else
      dW[t - d] = s;
  }
}

// C[t] = sum over z of P[z len + t], in order of z
__global__ __launch_bounds__(256) void k_splitk_reduce(const float* __restrict__ P, int splits, int64_t len,
                                                       float* __restrict__ C) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= len) return;
  float s = 0.f;
#pragma unroll 16
  for (int z = 0; z < splits; ++z) s += P[(int64_t)z * len + t];
  C[t] = s;
}

// MSE loss and its gradient: dY = bf16(2 (Y - T) / (B d)); per-block
// partial sums of (Y - T)^2 into part[blockIdx.x]
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int64_t n,
                                             float scale, uint16_t* __restrict__ dY, float* __restrict__ part) {
  float s = 0.f;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
    const float d = Y[t] - T[t];
    s += d * d;
    dY[t] = mse_grad(d, scale);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ float sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}
__global__ __launch_bounds__(256) void k_sum_final(const float* __restrict__ part, int64_t n, float scale,
                                                   float* __restrict__ out) {
  float s = 0.f;
  for (int64_t t = threadIdx.x; t < n; t += 256) s += part[t];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ float sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (sh[0] + sh[1] + sh[2] + sh[3]) * scale;
}

// Adam with bias correction on the FP32 master copy; refreshes the BF16 copy
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, uint16_t* __restrict__ w16,
                                              const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  float wt = w[t], mt = m[t], vt = v[t];
  adam_update(wt, mt, vt, g[t], lr, b1, b2, eps, c1, c2);
  m[t] = mt;
  v[t] = vt;
  w[t] = wt;
  w16[t] = f2bf(wt);
}

// batch gather: X[b] = affine map of params[idx[b]] onto [-1, 1]^2,
// T[b] = targets[idx[b]] (dout floats)
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ params, const float* __restrict__ targets,
                                                const int64_t* __restrict__ idx, int64_t B, int dout, double lo0,
                                                double hi0, double lo1, double hi1, float* __restrict__ X,
                                                float* __restrict__ T) {
  const int64_t b = blockIdx.x;
  const int64_t j = idx[b];
  if (threadIdx.x == 0) {
    X[2 * b] = (float)(2.0 * (params[2 * j] - lo0) / (hi0 - lo0) - 1.0);
    X[2 * b + 1] = (float)(2.0 * (params[2 * j + 1] - lo1) / (hi1 - lo1) - 1.0);
  }
  if (targets)
    for (int o = threadIdx.x; o < dout; o += 256) T[b * dout + o] = targets[j * dout + o];
}

// complex128 coefficients C (sample-major: C[j*ldc + i], i < k) -> FP32
// targets T[j][i] = Re, T[j][k + i] = Im
__global__ __launch_bounds__(256) void k_coef_targets(const double2* __restrict__ C, int64_t ldc, int64_t Mn, int k,
                                                      float* __restrict__ T) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= Mn * k) return;
  const int64_t j = t / k;
  const int i = (int)(t % k);
  const double2 c = C[j * ldc + i];
  T[j * 2 * k + i] = (float)c.x;
  T[j * 2 * k + k + i] = (float)c.y;
}

// per-sample relative error ||c_hat - c|| / ||c|| (FP64 sums), one wave per
// sample; c complex128 (C[j*ldc + i]), c_hat FP32 [Re; Im]
__global__ __launch_bounds__(256) void k_coef_relerr(const float* __restrict__ Yh, const double2* __restrict__ C,
                                                     int64_t ldc, int64_t Mn, int k, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= Mn) return;
  double num = 0.0, den = 0.0;
  for (int i = lane; i < k; i += 64) {
    const double2 c = C[j * ldc + i];
    const double dr = (double)Yh[j * 2 * k + i] - c.x;
    const double di = (double)Yh[j * 2 * k + k + i] - c.y;
    num += dr * dr + di * di;
    den += c.x * c.x + c.y * c.y;
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane == 0) out[j] = den > 0.0 ? sqrt(num / den) : sqrt(num);
}

// layout of an operand X(r, k) = X[r*sr + k*sk] (see Lay)
int vec_mode(const uint16_t* X, int64_t sr, int64_t sk) {
  const bool al = (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  if (al && sk == 1 && (sr * 2) % 16 == 0) return kK16;
  if (al && sr == 1 && (sk * 2) % 16 == 0) return kR16;
  const bool al4 = (reinterpret_cast<uintptr_t>(X) & 3) == 0;
  if (al4 && sk == 1 && sr % 2 == 0) return kK4;
  if (al4 && sr == 1 && sk % 2 == 0) return kR4;
  return kGen;
}

// the layout load_fast may use for an operand of layout vec with R rows and
// reduction length K (see load_fast), else kGen
int fast_layout(int vec, int64_t R, int64_t K) {
  switch (vec) {
    case kK16: return K % 8 == 0 ? kK16 : (K % 2 == 0 ? kK4 : kGen);
    case kK4: return K % 2 == 0 ? kK4 : kGen;
    case kR16: return R % 8 == 0 ? kR16 : (R % 2 == 0 ? kR4 : kGen);
    case kR4: return R % 2 == 0 ? kR4 : kGen;
    default: return kGen;
  }
}

struct GemmArgs {
  int64_t M, N, K;
  const uint16_t* A;
  int64_t sam, sak;
  const uint16_t* B;
  int64_t sbk, sbn;
  float* C;
  int64_t ldc;
  const float* bias;
  uint16_t* Cb;
  int64_t ldcb;
  const uint16_t* H;
  int64_t ldh;
  int64_t kc, cz;
  int csum;
};

template <int kEpi, int LA, int LB>
void launch_gemm(dim3 grid, const GemmArgs& g, int vecA, int vecB, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_bf16<kEpi, LA, LB>), grid, dim3(256), 0, s, g.M, g.N, g.K, g.A, g.sam, g.sak, g.B, g.sbk,
                     g.sbn, g.C, g.ldc, g.bias, g.Cb, g.ldcb, g.H, g.ldh, vecA, vecB, g.kc, g.cz, g.csum);
}

// Launches the instantiation for the operands' layouts.  Each product of the
// MLP has a fixed orientation: the forward products read A along K and B
// along R, the products with transposed weights read both along K, the
// weight gradients both along R; other layouts take the guarded kernel.
template <int kEpi>
hipError_t launch_layouts(dim3 grid, const GemmArgs& g, hipStream_t s) {
  const int vecA = vec_mode(g.A, g.sam, g.sak), vecB = vec_mode(g.B, g.sbn, g.sbk);
  const int la = fast_layout(vecA, g.M, g.K), lb = fast_layout(vecB, g.N, g.K);
  constexpr bool kRA = kEpi == kEpiStore, kRB = kEpi != kEpiDTanh;
  constexpr int a16 = kRA ? kR16 : kK16, a4 = kRA ? kR4 : kK4;
  constexpr int b16 = kRB ? kR16 : kK16, b4 = kRB ? kR4 : kK4;
  if (la == a16 && lb == b16)
    launch_gemm<kEpi, a16, b16>(grid, g, vecA, vecB, s);
  else if (la == a16 && lb == b4)
    launch_gemm<kEpi, a16, b4>(grid, g, vecA, vecB, s);
  else if (la == a4 && lb == b16)
    launch_gemm<kEpi, a4, b16>(grid, g, vecA, vecB, s);
  else if (la == a4 && lb == b4)
    launch_gemm<kEpi, a4, b4>(grid, g, vecA, vecB, s);
  else
    launch_gemm<kEpi, kGen, kGen>(grid, g, vecA, vecB, s);
  return hipGetLastError();
}

template <int kEpi>
hipError_t gemm(int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
                int64_t sbk, int64_t sbn, float* C, int64_t ldc, const float* bias, uint16_t* Cb, int64_t ldcb,
                const uint16_t* H, int64_t ldh, hipStream_t s) {
  dim3 grid((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT));
  if (grid.y > 65535) return hipErrorInvalidValue;
  const GemmArgs g{M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, Cb, ldcb, H, ldh, K, 0, 0};
  return launch_layouts<kEpi>(grid, g, s);
}

// Weight gradients with a long reduction K (the batch): kSplitK workgroups
// per output tile each reduce a K range of at least kSplitMin (whole staging
// chunks); the partial sums of split z of every product go to P + z cz, and
// one k_splitk_reduce adds the splits of all of them in a fixed order.
constexpr int kSplitK = 8;
constexpr int64_t kSplitMin = 128;
int64_t splitk_chunk(int64_t K, int* splits_out) {
  int splits = kSplitK;
  while (splits > 1 && (K + splits - 1) / splits < kSplitMin) splits /= 2;
  int64_t kc = (K + splits - 1) / splits;
  kc = (kc + kGK - 1) / kGK * kGK;
  *splits_out = (int)((K + kc - 1) / kc);
  return kc;
}

// Partial products of C (M x N, row-major) = A B over each split of K, and
// below them the bias gradient C(M, n) = sum_k B(k, n): split z writes the
// (M + 1) x N block at P + z cz.
hipError_t gemm_splitk_partial(int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t sam, int64_t sak,
                               const uint16_t* B, int64_t sbk, int64_t sbn, float* P, int64_t cz, hipStream_t s) {
  int splits;
  const int64_t kc = splitk_chunk(K, &splits);
  dim3 grid((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT), (unsigned)splits);
  if (grid.y > 65535) return hipErrorInvalidValue;
  const GemmArgs g{M, N, K, A, sam, sak, B, sbk, sbn, P, N, nullptr, nullptr, 0, nullptr, 0, kc, cz, 1};
  return launch_layouts<kEpiStore>(grid, g, s);
}

// Product p of a grouped split-K launch, set up as gemm_splitk_partial would
// launch it on its own; returns the workgroups it takes.
int group_add(GemmGroup& g, int p, int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t sam, int64_t sak,
              const uint16_t* B, int64_t sbk, int64_t sbn, float* P, int64_t cz) {
  int splits;
  const int64_t kc = splitk_chunk(K, &splits);
  const int vecA = vec_mode(A, sam, sak), vecB = vec_mode(B, sbn, sbk);
  const int la = fast_layout(vecA, M, K), lb = fast_layout(vecB, N, K);
  g.M[p] = M;
  g.N[p] = N;
  g.K[p] = K;
  g.A[p] = A;
  g.sam[p] = sam;
  g.sak[p] = sak;
  g.B[p] = B;
  g.sbk[p] = sbk;
  g.sbn[p] = sbn;
  g.C[p] = P;
  g.ldc[p] = N;
  g.kc[p] = kc;
  g.cz[p] = cz;
  g.vecA[p] = vecA;
  g.vecB[p] = vecB;
  g.lay[p] = (la == kR16 && lb == kR16) ? 0 : (la == kR16 && lb == kR4) ? 1 : (la == kR4 && lb == kR16) ? 2
             : (la == kR4 && lb == kR4) ? 3 : 4;
  g.gx[p] = (int)((N + kGT - 1) / kGT);
  g.gy[p] = (int)((M + kGT - 1) / kGT);
  g.splits[p] = splits;
  return g.gx[p] * g.gy[p] * splits;
}

// inputs up to kNarrowDin: vector first layer; wider ones: matrix cores
constexpr int kNarrowDin = 4;
constexpr int kMaxDin = 1024;

hipError_t to_bf16(const float* X, int64_t n, uint16_t* Xb, hipStream_t s) {
  int64_t grid = (n + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)grid), dim3(256), 0, s, X, n, Xb);
  return hipGetLastError();
}

struct Layout {
  int64_t W1, b1, W2, b2, W3, b3, W4, b4, total;
  Layout(int din, int h, int dout) {
    W1 = 0;
    b1 = W1 + (int64_t)din * h;
    W2 = b1 + h;
    b2 = W2 + (int64_t)h * h;
    W3 = b2 + h;
    b3 = W3 + (int64_t)h * h;
    W4 = b3 + h;
    b4 = W4 + (int64_t)h * dout;
    total = b4 + dout;
  }
};

hipError_t colsum(const uint16_t* D, int64_t B, int d, const float* X, int din, float* part, float* db, float* dW,
                  hipStream_t s) {
  const int64_t chunks = (B + kColRows - 1) / kColRows;
  dim3 grid((unsigned)((d + 255) / 256), (unsigned)chunks);
  hipLaunchKernelGGL(k_colsum, grid, dim3(256), 0, s, D, B, d, X, din, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t len = (int64_t)((X ? din : 0) + 1) * d;
  hipLaunchKernelGGL(k_colsum_final, dim3((unsigned)((len + 15) / 16)), dim3(256), 0, s, part, chunks, len, db, dW,
                     d);
  return hipGetLastError();
}

// ------------------------------------------------------- fused training --
// rb_mlp_train runs whole Adam steps, four launches each (inputs aside):
//   k_mlp_rows   forward, loss gradient and the backward dZ products for
//                kRB samples per workgroup, activations kept in LDS;
//   split-K      the weight-gradient products (as rb_mlp_backward);
//   k_adam_fused the split reduction, Adam and the BF16 weight copies.
// The row kernel forms every value the layer-by-layer kernels form, from the
// same operands, with the same MFMA sequence over k and the same element
// arithmetic, so a fused step reproduces their bits (the loss value aside,
// whose partial sums run in another order).  Its B operands come straight
// from L2 into registers: each wave's share of a layer is loaded kFKC
// k-steps at a time, so a hidden layer costs one memory latency.  For that
// they need 8 consecutive k per output, which for the forward products is a
// transposed copy of the weights ([out][in]); the backward products read the
// weights as stored (W4 with its rows padded to a multiple of 8).
constexpr int kRB = 16;        // samples per row-kernel workgroup
constexpr int kMT = kRB / 16;  // MFMA row tiles per workgroup
constexpr int kRowW = 16;      // waves per row-kernel workgroup
constexpr int kRowT = 64 * kRowW;
constexpr int kFMaxIn = 512;   // din rounded up to 32
constexpr int kFMaxOut = 320;  // dout rounded up to 32
constexpr int kFMaxH = 256;    // hidden: a multiple of 64
constexpr int kFKC = 9;        // k-steps (of 32) whose operands are loaded together (din, dout <= 288 in one)
constexpr int kFMaxT = (kFMaxOut / 16 + kRowW - 1) / kRowW;  // output tiles of 16 columns per wave

struct RowArgs {
  // inputs of the step's samples idx[0 .. batch): the parameters mapped onto
  // [-1, 1]^2 and the phase factors at the F grid rows `rows` (table `tab`);
  // targets gathered from `targets` (dout floats per sample)
  const double* params;
  const float* targets;
  const int64_t* idx;
  const int64_t* rows;
  const double* tab;
  int64_t F;
  double mlo, mhi, qlo, qhi;
  int64_t batch;
  int din, hid, dout, kin, kout;
  const uint16_t *W1t, *W2t, *W3t, *W4t;  // [out][in]; row strides kin, hid, hid, hid
  const uint16_t *W2, *W3, *W4b;          // [in][out]; row strides hid, hid, kout
  const float *b1, *b2, *b3, *b4;
  uint16_t *Xb, *H1, *H2, *H3, *dY, *dZ3, *dZ2, *dZ1;
  float scale;
  float* loss_part;
};

// acc[m][j] = sum over k < 32 ks of A(16 m + row, k) B(k, n) for this wave's
// output tiles t = wave + kRowW j < ntile: A from LDS (row stride lda), B
// lane l reads the 8 values k = 32 s + 8 (l / 16) .. + 7 of output
// n = 16 t + l % 16 at Bp + n ldb + k, each used for all kMT row tiles.
// Each workgroup reads every weight once per layer, so the samples per
// workgroup set the weight traffic through L2.
__device__ __forceinline__ void rows_mma(const uint16_t* sA, int lda, int ks, const uint16_t* __restrict__ Bp,
                                         int ldb, int ntile, int wave, int lane, f4v (&acc)[kMT][kFMaxT]) {
#pragma unroll
  for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
    for (int j = 0; j < kFMaxT; ++j) acc[mt][j] = (f4v){0.f, 0.f, 0.f, 0.f};
  const uint16_t* arow = sA + (lane & 15) * lda + 8 * (lane >> 4);
  const uint16_t* brow = Bp + (int64_t)(lane & 15) * ldb + 8 * (lane >> 4);
  for (int s0 = 0; s0 < ks; s0 += kFKC) {
    bf16x8 b[kFKC][kFMaxT];
#pragma unroll
    for (int c = 0; c < kFKC; ++c)
#pragma unroll
      for (int j = 0; j < kFMaxT; ++j) {
        const int s = s0 + c, t = wave + kRowW * j;
        b[c][j] = (s < ks && t < ntile) ? *reinterpret_cast<const bf16x8*>(brow + (int64_t)16 * t * ldb + 32 * s)
                                        : (bf16x8){};
      }
#pragma unroll
    for (int c = 0; c < kFKC; ++c) {
      const int s = s0 + c;
      if (s >= ks) break;
#pragma unroll
      for (int mt = 0; mt < kMT; ++mt) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(arow + 16 * mt * lda + 32 * s);
#pragma unroll
        for (int j = 0; j < kFMaxT; ++j)
          if (wave + kRowW * j < ntile)
            acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[c][j], acc[mt][j], 0, 0, 0);
      }
    }
  }
}

// Everything the epilogues read from global memory (inputs, targets, biases)
// is loaded at the start, all in flight together, so that only the weight
// operands of each layer cost a memory latency.
__global__ __launch_bounds__(kRowT) void k_mlp_rows(RowArgs a) {
  constexpr int kLX = kFMaxIn + 8, kLH = kFMaxH + 8, kLD = kFMaxOut + 8;  // LDS row strides (values)
  __shared__ __attribute__((aligned(16))) uint16_t sX[kRB * kLX];
  __shared__ __attribute__((aligned(16))) uint16_t sH[3][kRB * kLH];
  __shared__ __attribute__((aligned(16))) uint16_t sD[kRB * kLD];
  __shared__ __attribute__((aligned(16))) uint16_t sZ[2][kRB * kLH];
  __shared__ float sl[kRowW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // With a multiple of 8 workgroups, the XCDs (which take the workgroups in
  // turn) each process a contiguous eighth of the batch, which the
  // weight-gradient launch then reads on the same XCD.
  const int nb = gridDim.x;
  const int rb = nb % 8 == 0 ? (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
  const int64_t r0 = (int64_t)rb * kRB;
  const int th = a.hid / 16, to = (a.dout + 15) / 16;
  const int rbase = 4 * (lane >> 4);  // the rows of this lane in an MFMA result
  // inputs: the samples' parameter coefficients first (one thread per
  // sample), then the phase factors, written to LDS as BF16 (zero past din
  // and past the batch)
  __shared__ double sA[kRB], sB[kRB];
  __shared__ int64_t spj[kRB];
  if (tid < kRB) {
    const int64_t g = r0 + tid;
    double A = 0.0, B = 0.0;
    int64_t pj = -1;
    uint16_t x0 = 0, x1 = 0;
    if (g < a.batch) {
      pj = a.idx[g];
      const double m = a.params[2 * pj], q = a.params[2 * pj + 1];
      chirp_phase_coeffs(m, q, A, B);
      x0 = f2bf(box_map(m, a.mlo, a.mhi));
      x1 = f2bf(box_map(q, a.qlo, a.qhi));
    }
    sA[tid] = A;
    sB[tid] = B;
    spj[tid] = pj;
    sX[tid * kLX] = x0;
    sX[tid * kLX + 1] = x1;
  }
  for (int e = tid; e < kRB * (a.kin - a.din); e += kRowT) {
    const int r = e / (a.kin - a.din), c = a.din + (e - r * (a.kin - a.din));
    sX[r * kLX + c] = 0;
  }
  for (int e = tid; e < kRB * a.kout; e += kRowT) {
    const int r = e / a.kout, c = e - r * a.kout;
    if (c >= a.dout) sD[r * kLD + c] = 0;
  }
  __syncthreads();
  for (int64_t e = tid; e < kRB * a.F; e += kRowT) {
    const int r = (int)(e / a.F);
    const int64_t f = e - (int64_t)r * a.F;
    uint16_t cs = 0, sn = 0;
    if (spj[r] >= 0) {
      double s, c;
      sincos(chirp_phase(sA[r], sB[r], a.tab, a.rows[f]), &s, &c);
      cs = f2bf((float)c);
      sn = f2bf((float)(-s));
    }
    sX[r * kLX + 2 + 2 * f] = cs;
    sX[r * kLX + 3 + 2 * f] = sn;
  }
  // biases and targets of this lane's output columns
  float bh[3][kFMaxT], b4v[kFMaxT], tv[kMT][kFMaxT][4];
#pragma unroll
  for (int j = 0; j < kFMaxT; ++j) {
    const int t = wave + kRowW * j, col = 16 * t + (lane & 15);
    const bool okh = t < th, oko = t < to && col < a.dout;
    bh[0][j] = okh ? a.b1[col] : 0.f;
    bh[1][j] = okh ? a.b2[col] : 0.f;
    bh[2][j] = okh ? a.b3[col] : 0.f;
    b4v[j] = oko ? a.b4[col] : 0.f;
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t pj = spj[16 * mt + rbase + r];
        tv[mt][j][r] = (oko && pj >= 0) ? a.targets[pj * a.dout + col] : 0.f;
      }
  }
  __syncthreads();
  f4v acc[kMT][kFMaxT];
  // hidden layer: O = bf16(tanh(A W + b)) into LDS and global
  auto hidden_out = [&](const float (&bias)[kFMaxT], uint16_t* sO) {
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
      for (int j = 0; j < kFMaxT; ++j) {
        const int t = wave + kRowW * j;
        if (t >= th) continue;
        const int col = 16 * t + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) sO[(16 * mt + rbase + r) * kLH + col] = act_tanh(acc[mt][j][r], bias[j]);
      }
  };
  // backward: O = bf16(acc (1 - h^2)) with h the layer's activations
  auto dtanh_out = [&](const uint16_t* sHl, uint16_t* sO) {
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
      for (int j = 0; j < kFMaxT; ++j) {
        const int t = wave + kRowW * j;
        if (t >= th) continue;
        const int col = 16 * t + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * mt + rbase + r;
          sO[row * kLH + col] = act_dtanh(acc[mt][j][r], bf2f(sHl[row * kLH + col]));
        }
      }
  };
  // an LDS block of the layer outputs (kRB rows, n values each, row stride
  // ld) to its rows of the global [batch][n] array: 16-byte pieces when the
  // rows allow, else 4-byte or single values
  auto copy_out = [&](const uint16_t* sO, int ld, uint16_t* __restrict__ gO, int n) {
    const int w = n % 8 == 0 ? 8 : n % 2 == 0 ? 2 : 1;
    const int per = n / w;
    for (int e = tid; e < kRB * per; e += kRowT) {
      const int r = e / per, c = (e - r * per) * w;
      if (r0 + r >= a.batch) continue;
      uint16_t* dst = gO + (r0 + r) * n + c;
      const uint16_t* src = sO + r * ld + c;
      if (w == 8)
        *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(src);
      else if (w == 2)
        *reinterpret_cast<uint32_t*>(dst) = *reinterpret_cast<const uint32_t*>(src);
      else
        *dst = *src;
    }
  };
  copy_out(sX, kLX, a.Xb, a.din);
  rows_mma(sX, kLX, a.kin / 32, a.W1t, a.kin, th, wave, lane, acc);
  hidden_out(bh[0], sH[0]);
  __syncthreads();
  copy_out(sH[0], kLH, a.H1, a.hid);
  rows_mma(sH[0], kLH, a.hid / 32, a.W2t, a.hid, th, wave, lane, acc);
  hidden_out(bh[1], sH[1]);
  __syncthreads();
  copy_out(sH[1], kLH, a.H2, a.hid);
  rows_mma(sH[1], kLH, a.hid / 32, a.W3t, a.hid, th, wave, lane, acc);
  hidden_out(bh[2], sH[2]);
  __syncthreads();
  copy_out(sH[2], kLH, a.H3, a.hid);
  // output layer, loss and dY = bf16(2 (Y - T) / (batch dout))
  rows_mma(sH[2], kLH, a.hid / 32, a.W4t, a.hid, to, wave, lane, acc);
  float ls = 0.f;
#pragma unroll
  for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
    for (int j = 0; j < kFMaxT; ++j) {
      const int t = wave + kRowW * j;
      if (t >= to) continue;
      const int col = 16 * t + (lane & 15);
      if (col >= a.dout) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * mt + rbase + r;
        uint16_t dy = 0;
        if (r0 + row < a.batch) {
          const float d = (acc[mt][j][r] + b4v[j]) - tv[mt][j][r];
          ls += d * d;
          dy = mse_grad(d, a.scale);
        }
        sD[row * kLD + col] = dy;
      }
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ls += __shfl_xor(ls, o, 64);
  if (lane == 0) sl[wave] = ls;
  __syncthreads();
  copy_out(sD, kLD, a.dY, a.dout);
  if (tid == 0) {
    float t = 0.f;
    for (int w = 0; w < kRowW; ++w) t += sl[w];
    a.loss_part[rb] = t;
  }
  // dZ3 = (dY W4^T)(1 - H3^2), dZ2 = (dZ3 W3^T)(1 - H2^2), dZ1 = (dZ2 W2^T)(1 - H1^2)
  rows_mma(sD, kLD, a.kout / 32, a.W4b, a.kout, th, wave, lane, acc);
  dtanh_out(sH[2], sZ[0]);
  __syncthreads();
  copy_out(sZ[0], kLH, a.dZ3, a.hid);
  rows_mma(sZ[0], kLH, a.hid / 32, a.W3, a.hid, th, wave, lane, acc);
  dtanh_out(sH[1], sZ[1]);
  __syncthreads();
  copy_out(sZ[1], kLH, a.dZ2, a.hid);
  rows_mma(sZ[1], kLH, a.hid / 32, a.W2, a.hid, th, wave, lane, acc);
  dtanh_out(sH[0], sZ[0]);  // sZ[0] was last read before the barrier above
  __syncthreads();
  copy_out(sZ[0], kLH, a.dZ1, a.hid);
}

// The row kernel's weight copies from the BF16 weights: W1t (hid x kin),
// W2t, W3t (hid x hid), W4t (kout x hid) transposed, W4b (hid x kout) as
// stored; the padding is zero.
__global__ __launch_bounds__(256) void k_fused_copies(const uint16_t* __restrict__ p16, int din, int hid, int dout,
                                                      int kin, int kout, int64_t oW1, int64_t oW2, int64_t oW3,
                                                      int64_t oW4, uint16_t* __restrict__ W1t,
                                                      uint16_t* __restrict__ W2t, uint16_t* __restrict__ W3t,
                                                      uint16_t* __restrict__ W4t, uint16_t* __restrict__ W4b) {
  const int64_t n1 = (int64_t)hid * kin, n2 = (int64_t)hid * hid, n4 = (int64_t)kout * hid;
  const int64_t total = n1 + 2 * n2 + 2 * n4;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int64_t f = e;
    if (f < n1) {  // W1t[o][i] = W1[i][o]
      const int64_t o = f / kin, i = f % kin;
      W1t[f] = i < din ? p16[oW1 + i * hid + o] : 0;
      continue;
    }
    f -= n1;
    if (f < 2 * n2) {  // W2t, W3t
      const bool three = f >= n2;
      if (three) f -= n2;
      const int64_t o = f / hid, i = f % hid;
      (three ? W3t : W2t)[f] = p16[(three ? oW3 : oW2) + i * hid + o];
      continue;
    }
    f -= 2 * n2;
    if (f < n4) {  // W4t[o][i] = W4[i][o]
      const int64_t o = f / hid, i = f % hid;
      W4t[f] = o < dout ? p16[oW4 + i * dout + o] : 0;
      continue;
    }
    f -= n4;  // W4b[i][o] = W4[i][o]
    const int64_t i = f / kout, o = f % kout;
    W4b[f] = o < dout ? p16[oW4 + i * dout + o] : 0;
  }
}

// Split reduction, Adam and the BF16 copies for one step.  Workgroups
// [0, tw[4]) take 32 x 32 tiles of W1..W4 (tile ranges tw[0..4]), the next
// ceil((3 hidden + dout) / kAdamT) the biases b1 b2 b3 b4, the last one the
// loss; one parameter a thread.  Every parameter's gradient is the sum over the
// splits in order, as k_splitk_reduce forms it; a thread loads all the
// splits and moments of its parameters before it updates any of them.
struct AdamArgs {
  float *p32, *m, *v;
  uint16_t* p16;
  const float* split1;  // [dW1; db1] partials, split stride len1
  const float* splitp;  // [dW2 db2 dW3 db3 dW4 db4] partials, split stride lenW
  int64_t len1, lenW;
  int splits;
  int din, hid, dout, kin, kout;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3, oW4, ob4;
  uint16_t *W1t, *W2t, *W3t, *W4t, *W4b;
  int tw[5];
  int nbias_blocks;
  float lr, beta1, beta2, eps, c1, c2;
  const float* loss_part;
  int nparts;
  float scale;
  float* loss_out;
};

// Adam on parameters i[q] (ok[q]); returns the updated weights in w.  All
// loads are issued unconditionally, so that they are in flight together:
// the partial buffers hold kSplitK blocks whatever the split count, and a
// thread without a parameter reads index 0; what is not used is discarded.
template <int Q>
__device__ __forceinline__ void adam_params(const AdamArgs& a, const int64_t (&i)[Q], const bool (&ok)[Q],
                                            float (&w)[Q]) {
  float g[Q][kSplitK], m[Q], v[Q];
  // 32-bit offsets: the row kernel's limits bound the kSplitK blocks by
  // (kFMaxIn + 1) x kFMaxH and (kFMaxH + 1) x (2 kFMaxH + kFMaxOut) values
  const int l1 = (int)a.len1, lw = (int)a.lenW;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const bool first = i[q] < a.oW2;  // W1, b1
    // both candidate addresses, then the choice (a per-lane choice between
    // two argument fields would become a per-lane load of the arguments)
    const int p1 = ok[q] ? (int)(i[q] - a.oW1) : 0, pw = ok[q] ? (int)(i[q] - a.oW2) : 0;
    const int64_t ii = ok[q] ? i[q] : 0;
#pragma unroll
    for (int z = 0; z < kSplitK; ++z) {
      const float* e1 = a.split1 + (z * l1 + p1);
      const float* ew = a.splitp + (z * lw + pw);
      g[q][z] = *(first ? e1 : ew);
    }
    w[q] = a.p32[ii];
    m[q] = a.m[ii];
    v[q] = a.v[ii];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (!ok[q]) {
      w[q] = 0.f;
      continue;
    }
    // gs never holds -0 (it starts at +0), so adding +0 for the splits past
    // the count leaves it as the in-order sum of the used ones
    float gs = 0.f;
#pragma unroll
    for (int z = 0; z < kSplitK; ++z) gs += z < a.splits ? g[q][z] : 0.f;
    adam_update(w[q], m[q], v[q], gs, a.lr, a.beta1, a.beta2, a.eps, a.c1, a.c2);
    a.m[i[q]] = m[q];
    a.v[i[q]] = v[q];
    a.p32[i[q]] = w[q];
    a.p16[i[q]] = f2bf(w[q]);
  }
}

constexpr int kAdamT = 1024;  // one parameter per thread: a 32 x 32 tile per workgroup

__global__ __launch_bounds__(kAdamT) void k_adam_fused(AdamArgs a) {
  __shared__ uint16_t tile[32][33];
  __shared__ float sh[kAdamT / 64];
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  const int blk = blockIdx.x;
  if (blk >= a.tw[4] + a.nbias_blocks) {  // the loss
    if (a.loss_out) {
      float s = 0.f;
      for (int t = tid; t < a.nparts; t += kAdamT) s += a.loss_part[t];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if ((tid & 63) == 0) sh[tid >> 6] = s;
      __syncthreads();
      if (tid == 0) {
        float t = 0.f;
        for (int w = 0; w < kAdamT / 64; ++w) t += sh[w];
        *a.loss_out = t * a.scale;
      }
    }
    return;
  }
  int64_t i[1];
  bool ok[1];
  float w[1];
  if (blk >= a.tw[4]) {  // biases
    const int e = (blk - a.tw[4]) * kAdamT + tid;
    ok[0] = e < 3 * a.hid + a.dout;
    i[0] = e < a.hid ? a.ob1 + e : e < 2 * a.hid ? a.ob2 + (e - a.hid) : e < 3 * a.hid ? a.ob3 + (e - 2 * a.hid)
                                                                                         : a.ob4 + (e - 3 * a.hid);
    adam_params<1>(a, i, ok, w);
    return;
  }
  int l = 0;
  while (blk >= a.tw[l + 1]) ++l;
  const int nin = l == 0 ? a.din : a.hid, nout = l == 3 ? a.dout : a.hid;
  const int64_t oW = l == 0 ? a.oW1 : l == 1 ? a.oW2 : l == 2 ? a.oW3 : a.oW4;
  uint16_t* Wt = l == 0 ? a.W1t : l == 1 ? a.W2t : l == 2 ? a.W3t : a.W4t;
  const int ldt = l == 0 ? a.kin : a.hid;
  const int tcols = (nout + 31) / 32;
  const int t = blk - a.tw[l];
  const int i0 = (t / tcols) * 32, o0 = (t % tcols) * 32;
  ok[0] = i0 + ty < nin && o0 + tx < nout;
  i[0] = oW + (int64_t)(i0 + ty) * nout + o0 + tx;
  adam_params<1>(a, i, ok, w);
  const uint16_t h = ok[0] ? f2bf(w[0]) : (uint16_t)0;
  if (l == 3 && ok[0]) a.W4b[(int64_t)(i0 + ty) * a.kout + o0 + tx] = h;
  tile[ty][tx] = h;
  __syncthreads();
  const int oo = o0 + ty, ii = i0 + tx;
  if (oo < nout && ii < nin) Wt[(int64_t)oo * ldt + ii] = tile[tx][ty];
}

}  // namespace

}  // namespace rb

using namespace rb;

extern "C" {

int64_t rb_mlp_param_count(int din, int hidden, int dout) {
  if (din <= 0 || din > kMaxDin || hidden <= 0 || dout <= 0) return -1;
  return Layout(din, hidden, dout).total;
}

// column-sum partials (the vector first layer's gradients use din + 1 rows
// of them; the loss uses one)
static int64_t colsum_floats(int64_t batch, int din, int hidden, int dout) {
  const int64_t chunks = (batch + kColRows - 1) / kColRows;
  const int dn = din <= kNarrowDin ? din : 0;
  return chunks * (int64_t)(dn + 1) * (hidden > dout ? hidden : dout);
}

size_t rb_mlp_workspace_bytes(int64_t batch, int din, int hidden, int dout) {
  if (batch <= 0 || din <= 0 || din > kMaxDin || hidden <= 0 || dout <= 0) return 0;
  const int64_t part = colsum_floats(batch, din, hidden, dout);
  // split-K partials of [dW2 db2 dW3 db3 dW4 db4], one contiguous block,
  // and of [dW1 db1] for a wide first layer
  const int64_t splitk = (int64_t)kSplitK * ((int64_t)(hidden + 1) * (2 * hidden + dout));
  const int64_t split1 = din > kNarrowDin ? (int64_t)kSplitK * (int64_t)(din + 1) * hidden : 0;
  const int64_t xb = din > kNarrowDin ? batch * (int64_t)din : 0;  // BF16 inputs
  // H1..H3 and dZ (bf16), dY (bf16), X (bf16), Y (fp32), partial sums
  // (column sums, then the split-K partials of the weight gradients)
  return (size_t)(3 * batch * hidden + 2 * batch * hidden + batch * dout + xb) * 2 + (size_t)batch * dout * 4 +
         (size_t)(part + 4096 + splitk + split1) * 4 + 2048;
}

// Workspace carve-up (byte offsets) shared by forward and backward.
static void carve(void* ws, int64_t batch, int din, int hidden, int dout, uint16_t** H, uint16_t** dz,
                  uint16_t** dY, float** Y, float** part, float** splitp = nullptr, uint16_t** Xb = nullptr,
                  float** split1 = nullptr) {
  char* p = static_cast<char*>(ws);
  for (int l = 0; l < 3; ++l) {
    H[l] = reinterpret_cast<uint16_t*>(p);
    p += (size_t)batch * hidden * 2;
  }
  dz[0] = reinterpret_cast<uint16_t*>(p);
  p += (size_t)batch * hidden * 2;
  dz[1] = reinterpret_cast<uint16_t*>(p);
  p += (size_t)batch * hidden * 2;
  *dY = reinterpret_cast<uint16_t*>(p);
  p += (size_t)batch * dout * 2;
  p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 255) & ~(uintptr_t)255);
  if (Xb) *Xb = reinterpret_cast<uint16_t*>(p);
  if (din > kNarrowDin) p += (size_t)batch * din * 2;
  p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 255) & ~(uintptr_t)255);
  *Y = reinterpret_cast<float*>(p);
  p += (size_t)batch * dout * 4;
  *part = reinterpret_cast<float*>(p);
  float* sp = *part + colsum_floats(batch, din, hidden, dout) + 4096;
  if (splitp) *splitp = sp;
  if (split1) *split1 = sp + (int64_t)kSplitK * ((int64_t)(hidden + 1) * (2 * hidden + dout));
}

int rb_mlp_forward(const float* p32, const uint16_t* p16, int din, int hidden, int dout, const float* X,
                   int64_t batch, float* Y, void* ws, hipStream_t stream) {
  last_error().clear();
  if (!p32 || !p16 || !X || !ws || batch <= 0 || din <= 0 || din > kMaxDin || hidden <= 0 || dout <= 0)
    return set_error(RB_EINVAL, "rb_mlp_forward: bad arguments");
  const Layout L(din, hidden, dout);
  uint16_t *H[3], *dz[2], *dY, *Xb;
  float *Yw, *part;
  carve(ws, batch, din, hidden, dout, H, dz, &dY, &Yw, &part, nullptr, &Xb);
  if (!Y) Y = Yw;
  if (din <= kNarrowDin) {
    const int64_t n1 = batch * hidden;
    hipLaunchKernelGGL(k_layer1_fwd, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, stream, X, batch, din,
                       p16 + L.W1, p32 + L.b1, hidden, H[0]);
    RB_HIP(hipGetLastError());
  } else {
    RB_HIP(to_bf16(X, batch * (int64_t)din, Xb, stream));
    RB_HIP(gemm<kEpiBiasTanh>(batch, hidden, din, Xb, din, 1, p16 + L.W1, hidden, 1, nullptr, 0, p32 + L.b1, H[0],
                              hidden, nullptr, 0, stream));
  }
  RB_HIP(gemm<kEpiBiasTanh>(batch, hidden, hidden, H[0], hidden, 1, p16 + L.W2, hidden, 1, nullptr, 0, p32 + L.b2,
                            H[1], hidden, nullptr, 0, stream));
  RB_HIP(gemm<kEpiBiasTanh>(batch, hidden, hidden, H[1], hidden, 1, p16 + L.W3, hidden, 1, nullptr, 0, p32 + L.b3,
                            H[2], hidden, nullptr, 0, stream));
  RB_HIP(gemm<kEpiBias>(batch, dout, hidden, H[2], hidden, 1, p16 + L.W4, dout, 1, Y, dout, p32 + L.b4, nullptr, 0,
                        nullptr, 0, stream));
  return RB_OK;
}

int rb_mlp_loss(const float* Y, const float* T, int64_t batch, int dout, uint16_t* dY_out, float* loss,
                void* ws, int din, int hidden, hipStream_t stream) {
  last_error().clear();
  if (!T || !loss || !ws || batch <= 0 || dout <= 0 || din <= 0 || din > kMaxDin || hidden <= 0)
    return set_error(RB_EINVAL, "rb_mlp_loss: bad arguments");
  uint16_t *H[3], *dz[2], *dY;
  float *Yw, *part;
  carve(ws, batch, din, hidden, dout, H, dz, &dY, &Yw, &part);
  if (!Y) Y = Yw;
  if (!dY_out) dY_out = dY;
  const int64_t n = batch * (int64_t)dout;
  int64_t grid = (n + 255) / 256;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(k_mse, dim3((unsigned)grid), dim3(256), 0, stream, Y, T, n, 1.f / (float)n, dY_out, part);
  RB_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, stream, part, grid, 1.f / (float)n, loss);
  RB_HIP(hipGetLastError());
  return RB_OK;
}

int rb_mlp_backward(const float* p32, const uint16_t* p16, int din, int hidden, int dout, const float* X,
                    int64_t batch, const uint16_t* dY_in, float* grad, void* ws, hipStream_t stream) {
  last_error().clear();
  if (!p32 || !p16 || !X || !grad || !ws || batch <= 0 || din <= 0 || din > kMaxDin || hidden <= 0 || dout <= 0)
    return set_error(RB_EINVAL, "rb_mlp_backward: bad arguments");
  const Layout L(din, hidden, dout);
  uint16_t *H[3], *dz[2], *dY, *Xb;
  float *Yw, *part, *splitp, *split1;
  carve(ws, batch, din, hidden, dout, H, dz, &dY, &Yw, &part, &splitp, &Xb, &split1);
  if (dY_in) dY = const_cast<uint16_t*>(dY_in);
  // Each bias directly follows its weight matrix in the layout (b_l = W_l +
  // rows x cols), and W2 b2 W3 b3 W4 b4 are one contiguous range: the three
  // split-K products write their partials (dW_l with db_l = colsum(dZ_l)
  // below it) into one block laid out like that range, and one reduction
  // adds the splits of all three into grad.
  const int64_t lenW = L.b4 + dout - L.W2;
  int splits;
  (void)splitk_chunk(batch, &splits);
  // output layer: dW4 = H3^T dY, db4 = colsum(dY), dZ3 = (dY W4^T) * (1 - H3^2)
  RB_HIP(gemm_splitk_partial(hidden, dout, batch, H[2], 1, hidden, dY, dout, 1, splitp + (L.W4 - L.W2), lenW,
                             stream));
  RB_HIP(gemm<kEpiDTanh>(batch, hidden, dout, dY, dout, 1, p16 + L.W4, 1, dout, nullptr, 0, nullptr, dz[0], hidden,
                         H[2], hidden, stream));
  // hidden layer 3: dW3 = H2^T dZ3, db3, dZ2 = (dZ3 W3^T) * (1 - H2^2)
  RB_HIP(gemm_splitk_partial(hidden, hidden, batch, H[1], 1, hidden, dz[0], hidden, 1, splitp + (L.W3 - L.W2), lenW,
                             stream));
  RB_HIP(gemm<kEpiDTanh>(batch, hidden, hidden, dz[0], hidden, 1, p16 + L.W3, 1, hidden, nullptr, 0, nullptr, dz[1],
                         hidden, H[1], hidden, stream));
  // hidden layer 2: dW2 = H1^T dZ2, db2, dZ1 = (dZ2 W2^T) * (1 - H1^2)
  RB_HIP(gemm_splitk_partial(hidden, hidden, batch, H[0], 1, hidden, dz[1], hidden, 1, splitp, lenW, stream));
  RB_HIP(gemm<kEpiDTanh>(batch, hidden, hidden, dz[1], hidden, 1, p16 + L.W2, 1, hidden, nullptr, 0, nullptr, dz[0],
                         hidden, H[0], hidden, stream));
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((lenW + 255) / 256)), dim3(256), 0, stream, splitp, splits,
                     lenW, grad + L.W2);
  RB_HIP(hipGetLastError());
  // first layer: dW1 = X^T dZ1, db1 = colsum(dZ1)
  if (din <= kNarrowDin) {
    RB_HIP(colsum(dz[0], batch, hidden, X, din, part, grad + L.b1, grad + L.W1, stream));
  } else {
    // the BF16 inputs of the forward pass on the same X, refreshed here
    RB_HIP(to_bf16(X, batch * (int64_t)din, Xb, stream));
    const int64_t len1 = (int64_t)(din + 1) * hidden;  // [dW1; db1], laid out like W1 b1
    RB_HIP(gemm_splitk_partial(din, hidden, batch, Xb, 1, din, dz[0], hidden, 1, split1, len1, stream));
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((len1 + 255) / 256)), dim3(256), 0, stream, split1, splits,
                       len1, grad + L.W1);
    RB_HIP(hipGetLastError());
  }
  return RB_OK;
}

int rb_mlp_adam(float* p32, uint16_t* p16, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                float beta2, float eps, int64_t step, hipStream_t stream) {
  last_error().clear();
  if (!p32 || !p16 || !grad || !m || !v || n <= 0 || step < 1 || !(lr >= 0.f))
    return set_error(RB_EINVAL, "rb_mlp_adam: bad arguments");
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p32, p16, grad, m, v, n, lr,
                     beta1, beta2, eps, c1, c2);
  RB_HIP(hipGetLastError());
  return RB_OK;
}

int rb_mlp_gather(const double* params, const float* targets, const int64_t* idx, int64_t batch, int dout,
                  const double* ranges, float* X, float* T, hipStream_t stream) {
  last_error().clear();
  if (!params || !idx || !ranges || !X || batch <= 0 || (targets && (!T || dout <= 0)))
    return set_error(RB_EINVAL, "rb_mlp_gather: bad arguments");
  if (!(ranges[1] > ranges[0]) || !(ranges[3] > ranges[2])) return set_error(RB_EINVAL, "rb_mlp_gather: bad ranges");
  hipLaunchKernelGGL(k_gather, dim3((unsigned)batch), dim3(256), 0, stream, params, targets, idx, batch, dout,
                     ranges[0], ranges[1], ranges[2], ranges[3], X, T);
  RB_HIP(hipGetLastError());
  return RB_OK;
}

int rb_mlp_phase_features(const double* params, const float* targets, const int64_t* idx, int64_t batch, int dout,
                          const double* ranges, const int64_t* rows, int64_t F, const double* table, float* X,
                          float* T, hipStream_t stream) {
  last_error().clear();
  if (!params || !idx || !ranges || !rows || !table || !X || batch <= 0 || F < 1 || 2 + 2 * F > kMaxDin ||
      (targets && (!T || dout <= 0)))
    return set_error(RB_EINVAL, "rb_mlp_phase_features: bad arguments");
  if (!(ranges[1] > ranges[0]) || !(ranges[3] > ranges[2]))
    return set_error(RB_EINVAL, "rb_mlp_phase_features: bad ranges");
  RB_HIP(launch_phase_features(params, targets, idx, batch, dout, ranges, rows, F, table, X, T, stream));
  return RB_OK;
}

int rb_coef_targets(const void* C, int64_t ldc, int64_t Mn, int k, float* T, hipStream_t stream) {
  last_error().clear();
  if (!C || !T || Mn <= 0 || k <= 0 || ldc < k) return set_error(RB_EINVAL, "rb_coef_targets: bad arguments");
  const int64_t n = Mn * k;
  hipLaunchKernelGGL(k_coef_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                     static_cast<const double2*>(C), ldc, Mn, k, T);
  RB_HIP(hipGetLastError());
  return RB_OK;
}

int rb_coef_relerr(const float* Yh, const void* C, int64_t ldc, int64_t Mn, int k, double* out, hipStream_t stream) {
  last_error().clear();
  if (!Yh || !C || !out || Mn <= 0 || k <= 0 || ldc < k) return set_error(RB_EINVAL, "rb_coef_relerr: bad arguments");
  hipLaunchKernelGGL(k_coef_relerr, dim3((unsigned)((Mn + 3) / 4)), dim3(256), 0, stream, Yh,
                     static_cast<const double2*>(C), ldc, Mn, k, out);
  RB_HIP(hipGetLastError());
  return RB_OK;
}

// ---- whole training runs ----

namespace {

struct TrainCarve {
  uint16_t *dZ3, *W1t, *W2t, *W3t, *W4t, *W4b;
  float *X, *T, *grad, *lpart, *lscratch;
  void* mws;
};

// the layer-by-layer workspace first, then the fused step's buffers
size_t train_carve(void* base, int64_t batch, int din, int hid, int dout, TrainCarve* c) {
  const int kin = (din + 31) / 32 * 32, kout = (dout + 31) / 32 * 32;
  const int64_t n = rb_mlp_param_count(din, hid, dout);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? static_cast<char*>(base) + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  char* mws = take(rb_mlp_workspace_bytes(batch, din, hid, dout));
  char* dZ3 = take((size_t)batch * hid * 2);
  char* X = take((size_t)batch * din * 4);
  char* T = take((size_t)batch * dout * 4);
  char* grad = take((size_t)n * 4);
  char* W1t = take((size_t)hid * kin * 2);
  char* W2t = take((size_t)hid * hid * 2);
  char* W3t = take((size_t)hid * hid * 2);
  char* W4t = take((size_t)kout * hid * 2);
  char* W4b = take((size_t)hid * kout * 2);
  char* lpart = take((size_t)((batch + kRB - 1) / kRB) * 4);
  char* ls = take(4);
  if (c) {
    c->mws = mws;
    c->dZ3 = reinterpret_cast<uint16_t*>(dZ3);
    c->X = reinterpret_cast<float*>(X);
    c->T = reinterpret_cast<float*>(T);
    c->grad = reinterpret_cast<float*>(grad);
    c->W1t = reinterpret_cast<uint16_t*>(W1t);
    c->W2t = reinterpret_cast<uint16_t*>(W2t);
    c->W3t = reinterpret_cast<uint16_t*>(W3t);
    c->W4t = reinterpret_cast<uint16_t*>(W4t);
    c->W4b = reinterpret_cast<uint16_t*>(W4b);
    c->lpart = reinterpret_cast<float*>(lpart);
    c->lscratch = reinterpret_cast<float*>(ls);
  }
  return off;
}

bool fused_ok(int din, int hid, int dout, const uint16_t* p16) {
  const int kin = (din + 31) / 32 * 32, kout = (dout + 31) / 32 * 32;
  if (din <= kNarrowDin || kin > kFMaxIn || hid % 64 != 0 || hid > kFMaxH || kout > kFMaxOut) return false;
  const Layout L(din, hid, dout);
  // the backward products read W2 and W3 in place, 16 bytes at a time
  return (reinterpret_cast<uintptr_t>(p16 + L.W2) % 16 == 0) && (reinterpret_cast<uintptr_t>(p16 + L.W3) % 16 == 0);
}

}  // namespace

size_t rb_mlp_train_workspace_bytes(int64_t batch, int din, int hidden, int dout) {
  if (batch <= 0 || din <= 0 || din > kMaxDin || hidden <= 0 || dout <= 0) return 0;
  return train_carve(nullptr, batch, din, hidden, dout, nullptr);
}

int rb_mlp_train(float* p32, uint16_t* p16, float* m, float* v, int din, int hidden, int dout, const double* params,
                 const float* targets, const int64_t* idx, int64_t batch, int64_t steps, int64_t step0,
                 const float* lr, float beta1, float beta2, float eps, const double* ranges, const int64_t* rows,
                 int64_t F, const double* table, float* loss, void* ws, size_t ws_bytes, hipStream_t stream) {
  last_error().clear();
  if (!p32 || !p16 || !m || !v || !params || !targets || !idx || !lr || !ranges || !ws || batch <= 0 || steps < 0 ||
      step0 < 0 || din <= 0 || din > kMaxDin || hidden <= 0 || dout <= 0 || (rows && (!table || F < 1)))
    return set_error(RB_EINVAL, "rb_mlp_train: bad arguments");
  if (rows ? din != 2 + 2 * F : din != 2)
    return set_error(RB_EINVAL, "rb_mlp_train: din must be 2 + 2F with phase features, else 2");
  if (!(ranges[1] > ranges[0]) || !(ranges[3] > ranges[2])) return set_error(RB_EINVAL, "rb_mlp_train: bad ranges");
  TrainCarve c;
  const size_t need = train_carve(nullptr, batch, din, hidden, dout, nullptr);
  if (ws_bytes < need)
    return set_error(RB_ENOMEM, "rb_mlp_train: workspace of %zu bytes, %zu needed", ws_bytes, need);
  train_carve(ws, batch, din, hidden, dout, &c);
  const Layout L(din, hidden, dout);
  const int64_t n = L.total;
  const bool fused = rows && fused_ok(din, hidden, dout, p16);
  const int kin = (din + 31) / 32 * 32, kout = (dout + 31) / 32 * 32;
  uint16_t *H[3], *dz[2], *dY, *Xb;
  float *Yw, *part, *splitp, *split1;
  carve(c.mws, batch, din, hidden, dout, H, dz, &dY, &Yw, &part, &splitp, &Xb, &split1);
  if (fused && steps > 0) {
    const int64_t total = (int64_t)hidden * kin + 2 * (int64_t)hidden * hidden + 2 * (int64_t)kout * hidden;
    int64_t grid = (total + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_fused_copies, dim3((unsigned)grid), dim3(256), 0, stream, p16, din, hidden, dout, kin, kout,
                       L.W1, L.W2, L.W3, L.W4, c.W1t, c.W2t, c.W3t, c.W4t, c.W4b);
    RB_HIP(hipGetLastError());
  }
  const int64_t nrb = (batch + kRB - 1) / kRB;
  const int64_t lenW = L.b4 + dout - L.W2, len1 = (int64_t)(din + 1) * hidden;
  int splits;
  (void)splitk_chunk(batch, &splits);
  for (int64_t s = 0; s < steps; ++s) {
    const int64_t* ix = idx + s * batch;
    if (!fused) {
      if (rows)
        RB_HIP(launch_phase_features(params, targets, ix, batch, dout, ranges, rows, F, table, c.X, c.T, stream));
      else
        hipLaunchKernelGGL(k_gather, dim3((unsigned)batch), dim3(256), 0, stream, params, targets, ix, batch, dout,
                           ranges[0], ranges[1], ranges[2], ranges[3], c.X, c.T);
      RB_HIP(hipGetLastError());
    }
    const int64_t st = step0 + s + 1;
    const float c1 = 1.f - powf(beta1, (float)st), c2 = 1.f - powf(beta2, (float)st);
    if (!fused) {
      float* lo = loss ? loss + s : c.lscratch;
      int rc = rb_mlp_forward(p32, p16, din, hidden, dout, c.X, batch, nullptr, c.mws, stream);
      if (rc == RB_OK) rc = rb_mlp_loss(nullptr, c.T, batch, dout, nullptr, lo, c.mws, din, hidden, stream);
      if (rc == RB_OK) rc = rb_mlp_backward(p32, p16, din, hidden, dout, c.X, batch, nullptr, c.grad, c.mws, stream);
      if (rc == RB_OK) rc = rb_mlp_adam(p32, p16, c.grad, m, v, n, lr[s], beta1, beta2, eps, st, stream);
      if (rc != RB_OK) return rc;
      continue;
    }
    RowArgs ra;
    ra.params = params;
    ra.targets = targets;
    ra.idx = ix;
    ra.rows = rows;
    ra.tab = table;
    ra.F = F;
    ra.mlo = ranges[0];
    ra.mhi = ranges[1];
    ra.qlo = ranges[2];
    ra.qhi = ranges[3];
    ra.batch = batch;
    ra.din = din;
    ra.hid = hidden;
    ra.dout = dout;
    ra.kin = kin;
    ra.kout = kout;
    ra.W1t = c.W1t;
    ra.W2t = c.W2t;
    ra.W3t = c.W3t;
    ra.W4t = c.W4t;
    ra.W2 = p16 + L.W2;
    ra.W3 = p16 + L.W3;
    ra.W4b = c.W4b;
    ra.b1 = p32 + L.b1;
    ra.b2 = p32 + L.b2;
    ra.b3 = p32 + L.b3;
    ra.b4 = p32 + L.b4;
    ra.Xb = Xb;
    ra.H1 = H[0];
    ra.H2 = H[1];
    ra.H3 = H[2];
    ra.dY = dY;
    ra.dZ3 = c.dZ3;
    ra.dZ2 = dz[1];
    ra.dZ1 = dz[0];
    ra.scale = 1.f / (float)(batch * (int64_t)dout);
    ra.loss_part = c.lpart;
    hipLaunchKernelGGL(k_mlp_rows, dim3((unsigned)nrb), dim3(kRowT), 0, stream, ra);
    RB_HIP(hipGetLastError());
    // the four weight-gradient products (each with its bias gradient as an
    // extra row, as rb_mlp_backward forms them) in one launch
    GemmGroup gg;
    gg.start[0] = 0;
    gg.start[1] = gg.start[0] + group_add(gg, 0, hidden, dout, batch, H[2], 1, hidden, dY, dout, 1,
                                          splitp + (L.W4 - L.W2), lenW);
    gg.start[2] = gg.start[1] + group_add(gg, 1, hidden, hidden, batch, H[1], 1, hidden, c.dZ3, hidden, 1,
                                          splitp + (L.W3 - L.W2), lenW);
    gg.start[3] = gg.start[2] + group_add(gg, 2, hidden, hidden, batch, H[0], 1, hidden, dz[1], hidden, 1, splitp,
                                          lenW);
    gg.start[4] = gg.start[3] + group_add(gg, 3, din, hidden, batch, Xb, 1, din, dz[0], hidden, 1, split1, len1);
    gg.xcd = 1;
    for (int q = 0; q < 4; ++q) gg.xcd &= gg.splits[q] % 8 == 0;
    hipLaunchKernelGGL(k_gemm_group, dim3((unsigned)gg.start[4]), dim3(256), 0, stream, gg);
    RB_HIP(hipGetLastError());
    AdamArgs aa;
    aa.p32 = p32;
    aa.m = m;
    aa.v = v;
    aa.p16 = p16;
    aa.split1 = split1;
    aa.splitp = splitp;
    aa.len1 = len1;
    aa.lenW = lenW;
    aa.splits = splits;
    aa.din = din;
    aa.hid = hidden;
    aa.dout = dout;
    aa.kin = kin;
    aa.kout = kout;
    aa.oW1 = L.W1;
    aa.ob1 = L.b1;
    aa.oW2 = L.W2;
    aa.ob2 = L.b2;
    aa.oW3 = L.W3;
    aa.ob3 = L.b3;
    aa.oW4 = L.W4;
    aa.ob4 = L.b4;
    aa.W1t = c.W1t;
    aa.W2t = c.W2t;
    aa.W3t = c.W3t;
    aa.W4t = c.W4t;
    aa.W4b = c.W4b;
    const int th = (hidden + 31) / 32, ti = (din + 31) / 32, tob = (dout + 31) / 32;
    aa.tw[0] = 0;
    aa.tw[1] = ti * th;
    aa.tw[2] = aa.tw[1] + th * th;
    aa.tw[3] = aa.tw[2] + th * th;
    aa.tw[4] = aa.tw[3] + th * tob;
    aa.nbias_blocks = (3 * hidden + dout + kAdamT - 1) / kAdamT;
    aa.lr = lr[s];
    aa.beta1 = beta1;
    aa.beta2 = beta2;
    aa.eps = eps;
    aa.c1 = c1;
    aa.c2 = c2;
    aa.loss_part = c.lpart;
    aa.nparts = (int)nrb;
    aa.scale = ra.scale;
    aa.loss_out = loss ? loss + s : nullptr;
    hipLaunchKernelGGL(k_adam_fused, dim3((unsigned)(aa.tw[4] + aa.nbias_blocks + 1)), dim3(kAdamT), 0, stream,
                       aa);
    RB_HIP(hipGetLastError());
  }
  return RB_OK;
}

}  // extern "C"

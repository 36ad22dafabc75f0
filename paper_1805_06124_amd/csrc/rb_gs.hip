// Orthogonalisation of a pivot column against the basis (Sec. 6.1.2): the
// building blocks of one Gram-Schmidt pass in matrix-vector form,
//   G = E^H V   (k x nv),   V -= E G,   ||v_r||^2,
// plus the final scaling e = v / ||v||.  E holds k basis vectors of length N
// (column-major, ldE); V holds nv vectors (ldV).  These kernels touch
// O(k N) data per pass, far below one sweep of S.
#include "rb_internal.h"

namespace rb {

namespace {

constexpr int kGsThreads = 256;
constexpr int kChThreads = 1024;  // k_gemv_ch: rows per thread few enough for one or two rounds of loads

// One workgroup per basis vector i: G[i + r*k] = e_i^H v_r for r < nv.
__global__ __launch_bounds__(kChThreads) void k_gemv_ch(const double2* __restrict__ E, int64_t ldE, int64_t k,
                                                        const double2* __restrict__ V, int64_t ldV, int64_t nv,
                                                        int64_t N, double2* __restrict__ G,
                                                        const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = blockIdx.x;
  const double2* e = E + i * ldE;
  __shared__ double sre[kChThreads / 64], sim[kChThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (nv > 1) {
    // several vectors (at most kMaxV): e_i is read once for all of them;
    // each vector's sum is formed in the same order as below
    constexpr int kMaxV = 8;
    __shared__ double mre[kChThreads / 64][kMaxV], mim[kChThreads / 64][kMaxV];
    double re[kMaxV], im[kMaxV];
#pragma unroll
    for (int r = 0; r < kMaxV; ++r) re[r] = im[r] = 0.0;
    for (int64_t n = threadIdx.x; n < N; n += kChThreads) {
      const double2 a = e[n];
      double2 b[kMaxV];
      // vectors past nv read the last one (valid memory) and are not added
#pragma unroll
      for (int r = 0; r < kMaxV; ++r) b[r] = V[n + (r < nv ? r : nv - 1) * ldV];
#pragma unroll
      for (int r = 0; r < kMaxV; ++r) {
        if (r < nv) {
          re[r] += a.x * b[r].x + a.y * b[r].y;
          im[r] += a.x * b[r].y - a.y * b[r].x;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kMaxV; ++r) {
      const double wr = wave_sum(re[r]), wi = wave_sum(im[r]);
      if (lane == 0) {
        mre[wave][r] = wr;
        mim[wave][r] = wi;
      }
    }
    __syncthreads();
    if (threadIdx.x < nv) {
      const int r = threadIdx.x;
      double tr = 0.0, ti = 0.0;
      for (int w = 0; w < kChThreads / 64; ++w) {
        tr += mre[w][r];
        ti += mim[w][r];
      }
      G[i + r * k] = make_double2(tr, ti);
    }
    return;
  }
  for (int64_t r = 0; r < nv; ++r) {
    const double2* v = V + r * ldV;
    double re = 0.0, im = 0.0;
    // eight rows per thread in flight, added in the order of n
    int64_t n = threadIdx.x;
    for (; n + 7 * kChThreads < N; n += 8 * kChThreads) {
      double2 a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] = e[n + u * kChThreads];
        b[u] = v[n + u * kChThreads];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        re += a[u].x * b[u].x + a[u].y * b[u].y;
        im += a[u].x * b[u].y - a[u].y * b[u].x;
      }
    }
    for (; n < N; n += kChThreads) {
      double2 a = e[n], b = v[n];
      re += a.x * b.x + a.y * b.y;
      im += a.x * b.y - a.y * b.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
      sre[wave] = re;
      sim[wave] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double tr = 0.0, ti = 0.0;
      for (int w = 0; w < kChThreads / 64; ++w) {
        tr += sre[w];
        ti += sim[w];
      }
      G[i + r * k] = make_double2(tr, ti);
    }
    __syncthreads();
  }
}

// V[n + r*ldV] -= sum_i E[n + i*ldE] G[i + r*k].  A workgroup owns 64 rows;
// its kSubWaves waves split the basis vectors into contiguous ranges, each
// lane sums its row over its range in the order of i (eight vectors in
// flight), and the range sums are added in wave order through LDS.
constexpr int kSubWaves = 16;  // a wave per ~k/16 basis vectors: one or two rounds of loads
constexpr int kMaxNv = 8;
__global__ __launch_bounds__(kSubWaves * 64) void k_gemv_n_sub(const double2* __restrict__ E, int64_t ldE, int64_t k,
                                                               const double2* __restrict__ G, double2* __restrict__ V,
                                                               int64_t ldV, int64_t nv, int64_t N,
                                                               const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double sre[kSubWaves][kMaxNv][64], sim[kSubWaves][kMaxNv][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 64 + lane;
  const int64_t per = (k + kSubWaves - 1) / kSubWaves;
  const int64_t i0 = wave * per;
  const int64_t i1 = i0 + per < k ? i0 + per : k;
  double re[kMaxNv], im[kMaxNv];
#pragma unroll
  for (int r = 0; r < kMaxNv; ++r) re[r] = im[r] = 0.0;
  auto add = [&](const double2 a, int64_t i) {
#pragma unroll
    for (int r = 0; r < kMaxNv; ++r) {
      if (r < nv) {
        double2 g = G[i + r * k];
        re[r] += a.x * g.x - a.y * g.y;
        im[r] += a.x * g.y + a.y * g.x;
      }
    }
  };
  if (n < N && nv == 1) {
    // one vector (the orthogonalisation): the coefficients' loads go with
    // the basis loads, all in flight together (a load under r < nv would
    // wait for the one before it); the same products in the same order
    int64_t i = i0;
    for (; i + 8 <= i1; i += 8) {
      double2 a[8], g[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] = E[n + (i + u) * ldE];
        g[u] = G[i + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        re[0] += a[u].x * g[u].x - a[u].y * g[u].y;
        im[0] += a[u].x * g[u].y + a[u].y * g[u].x;
      }
    }
    for (; i < i1; ++i) {
      const double2 a = E[n + i * ldE], g = G[i];
      re[0] += a.x * g.x - a.y * g.y;
      im[0] += a.x * g.y + a.y * g.x;
    }
  } else if (n < N) {
    int64_t i = i0;
    for (; i + 8 <= i1; i += 8) {
      double2 a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = E[n + (i + u) * ldE];
#pragma unroll
      for (int u = 0; u < 8; ++u) add(a[u], i + u);
    }
    for (; i < i1; ++i) add(E[n + i * ldE], i);
  }
#pragma unroll
  for (int r = 0; r < kMaxNv; ++r) {
    sre[wave][r][lane] = re[r];
    sim[wave][r][lane] = im[r];
  }
  __syncthreads();
  if (wave == 0 && n < N) {
#pragma unroll
    for (int r = 0; r < kMaxNv; ++r) {
      if (r < nv) {
        double tr = sre[0][r][lane], ti = sim[0][r][lane];
#pragma unroll
        for (int w = 1; w < kSubWaves; ++w) {
          tr += sre[w][r][lane];
          ti += sim[w][r][lane];
        }
        const double2 v = V[n + r * ldV];
        V[n + r * ldV] = make_double2(v.x - tr, v.y - ti);
      }
    }
  }
}

// out[r] = ||v_r||^2, accumulated exactly (double-double) and rounded once;
// one workgroup per vector.
__global__ __launch_bounds__(1024) void k_sqnorms_small(const double2* __restrict__ V, int64_t ldV, int64_t N,
                                                        double* __restrict__ out, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const double2* v = V + (int64_t)blockIdx.x * ldV;
  dd s = {0.0, 0.0};
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x) {
    double2 a = v[n];
    dd_add_sq(s, a.x);
    dd_add_sq(s, a.y);
  }
  s = wave_dd_sum(s);
  __shared__ dd sh[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    dd t = sh[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) t = dd_add(t, sh[w]);
    out[blockIdx.x] = t.hi + t.lo;
  }
}

// out = v / sqrt(sq[0])
__global__ __launch_bounds__(kGsThreads) void k_scale_into(const double2* __restrict__ v, int64_t N,
                                                           const double* __restrict__ sq, double2* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * kGsThreads + threadIdx.x;
  if (n >= N) return;
  const double r = sqrt(sq[0]);
  double2 a = v[n];
  out[n] = make_double2(a.x / r, a.y / r);
}

// ---- Gram-Schmidt driven from the device (GsState, see rb_internal.h) ----
// Start: column J (from *jsrc, else jhost) of X into v, the state reset.
// The orthogonalisation is live if J >= 0 and the previous one in a chain
// (prev) was accepted.
__global__ __launch_bounds__(kGsThreads) void k_gs_begin(const double2* __restrict__ X, int64_t ldX, int64_t N,
                                                         const ArgMax* __restrict__ jsrc, int64_t jhost,
                                                         const GsState* __restrict__ prev,
                                                         const double* __restrict__ nrm0, double2* __restrict__ v,
                                                         GsState* __restrict__ st) {
  const int64_t J = jsrc ? jsrc->i : jhost;
  const bool live = (prev ? prev->accept != 0 : true) && J >= 0;
  const int64_t n = (int64_t)blockIdx.x * kGsThreads + threadIdx.x;
  if (live && n < N) v[n] = X[J * ldX + n];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->J = J;
    st->live = live;
    st->done = !live;
    st->passes = 0;
    st->settled = 0;
    st->accept = 0;
    st->finite = 1;
    st->in_span = 0;
    st->s_norm2 = live ? nrm0[J] : 0.0;
    st->before = st->after = 0.0;
  }
}
// ||v||^2 into sq[0] (k_sqnorms_small's sum, one vector) and, from it, the
// state: with check == 0 the norm before the first pass; otherwise the
// outcome of a pass, Hoffmann's criterion deciding whether another pass
// is due (Sec. 6.1.2), exactly as a host loop over the passes would.
// Nothing happens once the orthogonalisation is done (or was never live).
__global__ __launch_bounds__(1024) void k_gs_norm(const double2* __restrict__ v, int64_t N, double* __restrict__ sq,
                                                  GsState* __restrict__ st, int check, int nu_min, int nu_max,
                                                  double kappa) {
  if (st->done) return;
  dd s = {0.0, 0.0};
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x) {
    double2 a = v[n];
    dd_add_sq(s, a.x);
    dd_add_sq(s, a.y);
  }
  s = wave_dd_sum(s);
  __shared__ dd sh[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    dd t = sh[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) t = dd_add(t, sh[w]);
    const double q = t.hi + t.lo;
    sq[0] = q;
    const double r = sqrt(q);
    if (!check) {
      st->before = st->after = r;
      return;
    }
    st->passes += 1;
    st->after = r;
    if (st->passes >= nu_min && r > st->before / kappa) {
      st->settled = 1;
      st->done = 1;
    } else {
      st->before = r;
      if (st->passes >= nu_max) st->done = 1;
    }
  }
}
// The outcome: finite, numerically in span(E) (||v|| <= 64 u ||s_J||), and
// accepted (live, finished, finite, not in the span, settled unless
// ||v|| < tol); an accepted vector is written as e = v / ||v|| into out.
// "Finished": settled, or nu_max passes run; a chain queued with fewer
// passes than nu_max is not accepted when it still needed more.
__global__ __launch_bounds__(kGsThreads) void k_gs_finish(GsState* __restrict__ st, double tol,
                                                          const double* __restrict__ sq,
                                                          const double2* __restrict__ v, int64_t N,
                                                          double2* __restrict__ out) {
  const double r = st->after;
  const bool finite = __builtin_isfinite(r);
  const bool in_span = !(r > 64.0 * 0x1p-53 * sqrt(st->s_norm2));
  const bool ok = st->live && st->done && finite && !in_span && (st->settled || r < tol);
  const int64_t n = (int64_t)blockIdx.x * kGsThreads + threadIdx.x;
  if (ok && n < N) {
    const double rr = sqrt(sq[0]);
    const double2 a = v[n];
    out[n] = make_double2(a.x / rr, a.y / rr);
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->finite = finite;
    st->in_span = in_span;
    st->accept = ok;
  }
}

}  // namespace

hipError_t launch_gs_begin(const double2* X, int64_t ldX, int64_t N, const ArgMax* jsrc, int64_t jhost,
                           const GsState* prev, const double* nrm0, double2* v, double* sq1, GsState* st,
                           hipStream_t s) {
  const int64_t grid = (N + kGsThreads - 1) / kGsThreads;
  hipLaunchKernelGGL(k_gs_begin, dim3((unsigned)grid), dim3(kGsThreads), 0, s, X, ldX, N, jsrc, jhost, prev, nrm0, v,
                     st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gs_norm, dim3(1), dim3(1024), 0, s, v, N, sq1, st, 0, 0, 0, 0.0);
  return hipGetLastError();
}

hipError_t launch_gs_pass(const double2* E, int64_t ldE, int64_t kk, double2* v, int64_t N, double2* G, double* sq,
                          GsState* st, int nu_min, int nu_max, double kappa, hipStream_t s) {
  if (kk <= 0) return hipErrorInvalidValue;
  const int32_t* skip = &st->done;
  hipLaunchKernelGGL(k_gemv_ch, dim3((unsigned)kk), dim3(kChThreads), 0, s, E, ldE, kk, v, N, 1, N, G, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gemv_n_sub, dim3((unsigned)((N + 63) / 64)), dim3(kSubWaves * 64), 0, s, E, ldE, kk, G, v, N,
                     1, N, skip);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gs_norm, dim3(1), dim3(1024), 0, s, v, N, sq, st, 1, nu_min, nu_max, kappa);
  return hipGetLastError();
}

hipError_t launch_gs_finish(GsState* st, double tol, const double* sq, const double2* v, int64_t N, double2* out,
                            hipStream_t s) {
  const int64_t grid = (N + kGsThreads - 1) / kGsThreads;
  hipLaunchKernelGGL(k_gs_finish, dim3((unsigned)grid), dim3(kGsThreads), 0, s, st, tol, sq, v, N, out);
  return hipGetLastError();
}

hipError_t launch_gemv_ch(const double2* E, int64_t ldE, int64_t k, const double2* V, int64_t ldV, int64_t nv,
                          int64_t N, double2* G, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (nv > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemv_ch, dim3((unsigned)k), dim3(kChThreads), 0, s, E, ldE, k, V, ldV, nv, N, G,
                     static_cast<const int32_t*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_gemv_n_sub(const double2* E, int64_t ldE, int64_t k, const double2* G, double2* V, int64_t ldV,
                             int64_t nv, int64_t N, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (nv > 8) return hipErrorInvalidValue;
  int64_t grid = (N + 63) / 64;
  hipLaunchKernelGGL(k_gemv_n_sub, dim3((unsigned)grid), dim3(kSubWaves * 64), 0, s, E, ldE, k, G, V, ldV, nv, N,
                     static_cast<const int32_t*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_sqnorms_small(const double2* V, int64_t ldV, int64_t nv, int64_t N, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sqnorms_small, dim3((unsigned)nv), dim3(1024), 0, s, V, ldV, N, out,
                     static_cast<const int32_t*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_scale_into(const double2* v, int64_t N, const double* sq, double2* out, hipStream_t s) {
  int64_t grid = (N + kGsThreads - 1) / kGsThreads;
  hipLaunchKernelGGL(k_scale_into, dim3((unsigned)grid), dim3(kGsThreads), 0, s, v, N, sq, out);
  return hipGetLastError();
}

}  // namespace rb

// Learned warm start for the centroid update (include/d2.h, d2_ws_*): a
// deep-sets network maps the members of a cluster to a proposed initial
// centroid.  The network is not part of the paper; it only chooses the
// starting point of the B-ADMM centroid update of Sec. 3.2, and a gate keeps
// the plain initial centroid whenever the proposal's product-coupling bound
// on the barycenter objective (Eq. (badmm_prob) evaluated at the feasible
// plan w_i w_j) is not at least as good.
//
// All network arithmetic runs here: per-cluster standardisation, BF16 MFMA
// products with FP32 accumulation (__builtin_amdgcn_mfma_f32_32x32x16_bf16,
// 64-lane wavefronts, 32x32 output tiles), pooling, the Chamfer +
// cross-entropy loss and its gradient, weight-gradient products with a
// deterministic two-level reduction, and Adam on FP32 master weights.
//
// This file also holds d2_objective_feasible: the barycenter objective of
// the current centroids under the last plans rounded to exactly feasible
// couplings (an upper bound used to measure time to objective).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/d2.h"
#include "d2_ctx.hpp"

namespace ws {

typedef uint16_t u16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// FP32 -> BF16, round to nearest, ties to even.
__device__ __forceinline__ u16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) {
  return __uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ bf16x8 ld8(const u16* p) {
  return __builtin_bit_cast(bf16x8, *(const uint4*)p);
}
__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// ---------------------------------------------------------------- products

// C[M x N] = A[M x K] * B[K x N] with A row-major and B supplied transposed
// (Bt, N x K, K contiguous), so that both MFMA operands are 16-byte loads of
// 8 consecutive K values.  Epilogue: + bias[n], ReLU, multiply by the
// indicator mask[r][n] > 0, store BF16 and/or FP32.  K % 16 == 0,
// N % 32 == 0, rows and leading dimensions 16-byte aligned.  Each
// wavefront owns 32 rows x up to 128 columns (four accumulators); rows past
// M are clamped on load and dropped on store.
struct GemmArgs {
  const u16* A;
  const u16* Bt;
  const float* bias;
  const u16* mask;
  u16* c16;
  float* c32;
  int M, N, K, lda, ldb, ldm, ldc, ldc32, relu;
};

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = blockIdx.x * 128 + 32 * w;
  if (r0 >= g.M) return;  // no barriers below: whole wavefronts may leave
  const int nb = blockIdx.y * 128;
  const int nt = min(4, (g.N - nb) / 32);
  const int lr = l & 31, lh = l >> 5;
  const u16* ap = g.A + (size_t)min(r0 + lr, g.M - 1) * g.lda + 8 * lh;
  const u16* bp[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
    bp[t] = g.Bt + (size_t)(nb + 32 * min(t, nt - 1) + lr) * g.ldb + 8 * lh;
  f32x16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.0f;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    const bf16x8 a = ld8(ap + k0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < nt)
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, ld8(bp[t] + k0),
                                                        acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= nt) continue;
    const int col = nb + 32 * t + lr;
    const float bv = g.bias ? g.bias[col] : 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = r0 + 8 * (v >> 2) + 4 * lh + (v & 3);
      if (r >= g.M) continue;
      float x = acc[t][v] + bv;
      if (g.relu) x = fmaxf(x, 0.0f);
      if (g.mask && !(bf2f(g.mask[(size_t)r * g.ldm + col]) > 0.0f)) x = 0.0f;
      if (g.c16) g.c16[(size_t)r * g.ldc + col] = f2bf(x);
      if (g.c32) g.c32[(size_t)r * g.ldc32 + col] = x;
    }
  }
}

// Weight gradient dW[i][j] = sum_r X[r][i] Y[r][j] and column sums
// sum_r Y[r][j], per chunk of `rc` rows (grid.x) and 128-column block of Y
// (grid.y).  Each 64-row stage is written to LDS transposed (row index
// contiguous) so that both MFMA operands are 16-byte LDS reads.  Partial
// results go to part[chunk * pstride + ...] (Kx x Ny matrix, then Ny column
// sums) and are summed over chunks in a fixed order by k_wgrad_reduce.
struct WgArgs {
  const u16* X;
  const u16* Y;
  float* part;
  int ldx, ldy, R, Kx, Ny, rc;
  long pstride;
};

constexpr int kLdsStride = 72;  // 64 rows + 8 pad (keeps 16-byte alignment)

__global__ __launch_bounds__(256) void k_wgrad(WgArgs g) {
  __shared__ u16 Xs[128 * kLdsStride];
  __shared__ u16 Ys[128 * kLdsStride];
  __shared__ float cs[16 * 128];
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int lr = l & 31, lh = l >> 5;
  const int ch = blockIdx.x, jb = blockIdx.y * 128;
  const int nj = min(128, g.Ny - jb);
  const int kxp = (g.Kx + 31) / 32 * 32;
  const int nti = kxp / 32, ntj = (nj + 31) / 32, ntile = nti * ntj;
  const int rb = ch * g.rc, re = min(g.R, rb + g.rc);
  f32x16 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[u][v] = 0.0f;
  float csum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int xg = kxp / 8;
  for (int r0 = rb; r0 < re; r0 += 64) {
    for (int q = tid; q < 64 * xg; q += 256) {
      const int rr = q / xg, cg = q % xg, r = r0 + rr;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (r < re && 8 * cg < g.Kx) v = *(const uint4*)(g.X + (size_t)r * g.ldx + 8 * cg);
      const u16* e = (const u16*)&v;
#pragma unroll
      for (int t = 0; t < 8; ++t) Xs[(8 * cg + t) * kLdsStride + rr] = e[t];
    }
    for (int q = tid; q < 64 * 16; q += 256) {
      const int rr = q / 16, cg = q % 16, r = r0 + rr;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (r < re && 8 * cg < nj)
        v = *(const uint4*)(g.Y + (size_t)r * g.ldy + jb + 8 * cg);
      const u16* e = (const u16*)&v;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        Ys[(8 * cg + t) * kLdsStride + rr] = e[t];
        csum[t] += bf2f(e[t]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int tile = w + 4 * u;
        if (tile < ntile) {
          const int ti = tile / ntj, tj = tile % ntj;
          const bf16x8 a = __builtin_bit_cast(
              bf16x8, *(const uint4*)&Xs[(32 * ti + lr) * kLdsStride + 16 * s + 8 * lh]);
          const bf16x8 b = __builtin_bit_cast(
              bf16x8, *(const uint4*)&Ys[(32 * tj + lr) * kLdsStride + 16 * s + 8 * lh]);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[u], 0, 0, 0);
        }
      }
    __syncthreads();
  }
  float* out = g.part + (size_t)ch * g.pstride;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int tile = w + 4 * u;
    if (tile >= ntile) continue;
    const int ti = tile / ntj, tj = tile % ntj;
    const int j = 32 * tj + lr;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 32 * ti + 8 * (v >> 2) + 4 * lh + (v & 3);
      if (i < g.Kx && j < nj) out[(size_t)i * g.Ny + jb + j] = acc[u][v];
    }
  }
  // column sums: the 16 threads with the same column group share columns
  {
    const int cg = tid % 16, rg = tid / 16;
#pragma unroll
    for (int t = 0; t < 8; ++t) cs[rg * 128 + 8 * cg + t] = csum[t];
  }
  __syncthreads();
  if (tid < nj) {
    float s = 0.0f;
    for (int rg = 0; rg < 16; ++rg) s += cs[rg * 128 + tid];
    out[(size_t)g.Kx * g.Ny + jb + tid] = s;
  }
}

// grad[woff + i*Ny + j] = sum over chunks (in order) of the partial matrix;
// grad[boff + j] likewise for the column sums (boff < 0: not wanted).
__global__ void k_wgrad_reduce(const float* part, long pstride, int nch,
                               int Kx, int Ny, float* grad, long woff,
                               long boff) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nw = (long)Kx * Ny;
  if (q >= nw + Ny) return;
  if (q >= nw && boff < 0) return;
  float s = 0.0f;
  for (int c = 0; c < nch; ++c) s += part[(size_t)c * pstride + q];
  if (q < nw)
    grad[woff + q] = s;
  else
    grad[boff + (q - nw)] = s;
}

// out[j] = sum_r A[r][j] (FP32 rows, fixed order)
__global__ void k_colsum(const float* A, int R, int ncol, int lda,
                         float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  float s = 0.0f;
  for (int r = 0; r < R; ++r) s += A[(size_t)r * lda + j];
  out[j] = s;
}

// ------------------------------------------------------- per-cluster input

// Batch description: segment b (cluster bid[b]) owns rows [rs[b], rs[b+1])
// of the batch, which are the points plist[pstart[bid[b]] + (r - rs[b])].
struct Batch {
  const int32_t* bid;
  const int32_t* rs;
  const float* nmem;       // members per segment
  const int32_t* plist;    // points sorted by cluster
  const float* pmk;        // m_k of the member owning each listed point
  const int64_t* pstart;   // K + 1
  int B;
};

// Weighted mean mu and RMS radius s of each segment's points (weights w_j,
// so every member weighs 1), accumulated in FP64.  One workgroup per
// segment; thread (tx, ty) sums coordinate tx over every (256/DP)-th point.
template <typename T>
__global__ __launch_bounds__(256) void k_stats(const T* X, const T* W, int xs,
                                               int d, Batch bt, float* mu,
                                               float* sc, double* mud,
                                               double* sd, double* Sdev,
                                               double* wsum) {
  __shared__ double sh[256];
  __shared__ double mean[64];
  __shared__ double tot;
  const int b = blockIdx.x, tid = threadIdx.x;
  int DP = 1;
  while (DP < d) DP <<= 1;
  const int RP = 256 / DP, tx = tid % DP, ty = tid / DP;
  const int c = bt.bid[b];
  const int64_t p0 = bt.pstart[c], np = bt.pstart[c + 1] - p0;
  // pass 1: sum w, sum w y
  double ay = 0.0, aw = 0.0;
  for (int64_t q = ty; q < np; q += RP) {
    const int64_t p = bt.plist[p0 + q];
    const double wj = (double)W[p];
    aw += wj;
    if (tx < d) ay += wj * (double)X[(size_t)p * xs + tx];
  }
  sh[tid] = aw;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int q = 0; q < RP; ++q) s += sh[q * DP];
    tot = s;
  }
  __syncthreads();
  sh[tid] = ay;
  __syncthreads();
  if (tid < d) {
    double s = 0.0;
    for (int q = 0; q < RP; ++q) s += sh[q * DP + tid];
    mean[tid] = s / tot;
  }
  __syncthreads();
  // pass 2: sum w |y - mu|^2 per coordinate
  double av = 0.0;
  if (tx < d) {
    const double mt = mean[tx];
    for (int64_t q = ty; q < np; q += RP) {
      const int64_t p = bt.plist[p0 + q];
      const double df = (double)X[(size_t)p * xs + tx] - mt;
      av += (double)W[p] * df * df;
    }
  }
  __syncthreads();
  sh[tid] = av;
  __syncthreads();
  if (tid == 0) {
    double S = 0.0;
    for (int t = 0; t < d; ++t) {
      double s = 0.0;
      for (int q = 0; q < RP; ++q) s += sh[q * DP + t];
      S += s;
    }
    const double s2 = std::max(std::sqrt(S / tot), 1e-12);
    sd[b] = s2;
    sc[b] = (float)s2;
    Sdev[b] = S;
    wsum[b] = tot;
  }
  if (tid < d) {
    mud[(size_t)b * d + tid] = mean[tid];
    mu[(size_t)b * d + tid] = (float)mean[tid];
  }
}

__device__ __forceinline__ int find_seg(const int32_t* rs, int B, int r) {
  int lo = 0, hi = B;  // rs[lo] <= r < rs[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rs[mid] <= r) lo = mid; else hi = mid;
  }
  return lo;
}

// Per point: f = [(y - mu)/s, m_k w_j, 0...] (BF16, din wide), the pooling
// weight w_j / N_c and the row's segment.
template <typename T>
__global__ void k_feat(const T* X, const T* W, int xs, int d, int din,
                       Batch bt, const float* mu, const float* sc, int P,
                       u16* F, float* pw, int32_t* seg) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= P) return;
  const int b = find_seg(bt.rs, bt.B, r);
  const int c = bt.bid[b];
  const int64_t q = bt.pstart[c] + (r - bt.rs[b]);
  const int64_t p = bt.plist[q];
  const float inv = 1.0f / sc[b];
  const float wj = (float)W[p];
  u16* fr = F + (size_t)r * din;
  for (int t0 = 0; t0 < din; t0 += 8) {
    u16 e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u;
      float v = 0.0f;
      if (t < d) v = ((float)X[(size_t)p * xs + t] - mu[(size_t)b * d + t]) * inv;
      else if (t == d) v = bt.pmk[q] * wj;
      e[u] = f2bf(v);
    }
    *(uint4*)(fr + t0) = *(const uint4*)e;
  }
  pw[r] = wj / bt.nmem[b];
  seg[r] = b;
}

// Pooling: part[chunk][h] = sum_{rows of chunk} pw[r] H2[r][h]; a chunk lies
// inside one segment.  Then G[b] = sum of the segment's chunks, in order.
__global__ void k_pool_part(const u16* H2, const float* pw, int H,
                            const int32_t* chunks /* 3 per chunk */,
                            float* part) {
  const int ch = blockIdx.x, h = threadIdx.x;
  if (h >= H) return;
  const int r0 = chunks[3 * ch + 1], r1 = chunks[3 * ch + 2];
  float s = 0.0f;
  for (int r = r0; r < r1; ++r) s += pw[r] * bf2f(H2[(size_t)r * H + h]);
  part[(size_t)ch * H + h] = s;
}

__global__ void k_pool_fin(const float* part, const int32_t* cstart, int H,
                           float* G, u16* Gq) {
  const int b = blockIdx.x, h = threadIdx.x;
  if (h >= H) return;
  float s = 0.0f;
  for (int c = cstart[b]; c < cstart[b + 1]; ++c) s += part[(size_t)c * H + h];
  G[(size_t)b * H + h] = s;
  Gq[(size_t)b * H + h] = f2bf(s);
}

// ------------------------------------------------------------------ loss

// Per cluster (one wavefront): predictions Delta_i = O[i d ..], logits
// O[m d + i], targets t_j = (x*_j - mu)/s.  Loss = sum_j w*_j D(nn(j), j) +
// sum_i w_i D(i, nn(i)) - sum_i q_i log w_i with D the squared distance,
// nn by first minimum, q_i the target mass routed to prediction i.
// Writes the batch-mean gradient dO (FP32 and BF16, padding zeroed) and the
// cluster's loss.
__global__ __launch_bounds__(64) void k_loss(const float* O, int outp, int m,
                                             int d, const int32_t* bid,
                                             const float* tx, const float* tw,
                                             const float* mu, const float* sc,
                                             float invB, float* dO32,
                                             u16* dO16, double* loss) {
  __shared__ float Dl[64 * 65];
  __shared__ float del[64 * 65];
  __shared__ float tt[64 * 65];
  __shared__ int nnt[64];
  __shared__ float wts[64];
  const int b = blockIdx.x, l = threadIdx.x;
  const int c = bid[b];
  const float* o = O + (size_t)b * outp;
  const float inv = 1.0f / sc[b];
  for (int q = l; q < m * d; q += 64) {
    const int i = q / d, t = q % d;
    del[i * 65 + t] = o[q];
    tt[i * 65 + t] = (tx[(size_t)c * m * d + q] - mu[(size_t)b * d + t]) * inv;
  }
  if (l < m) wts[l] = tw[(size_t)c * m + l];
  __syncthreads();
  const bool act = l < m;
  // softmax of the logits
  const float lg = act ? o[m * d + l] : -INFINITY;
  const float mx = wave_max(lg);
  const float ex = act ? __expf(lg - mx) : 0.0f;
  const float se = wave_sum(ex);
  const float wh = ex / se;
  const float logw = act ? (lg - mx) - __logf(se) : 0.0f;
  // distances, nearest target of prediction l
  int nnp = 0;
  float a = INFINITY;
  if (act) {
    for (int j = 0; j < m; ++j) {
      float s = 0.0f;
      for (int t = 0; t < d; ++t) {
        const float df = del[l * 65 + t] - tt[j * 65 + t];
        s += df * df;
      }
      Dl[l * 65 + j] = s;
      if (s < a) { a = s; nnp = j; }
    }
  }
  __syncthreads();
  // nearest prediction of target l
  float dj = 0.0f;
  if (act) {
    int best = 0;
    float bv = INFINITY;
    for (int i = 0; i < m; ++i) {
      const float v = Dl[i * 65 + l];
      if (v < bv) { bv = v; best = i; }
    }
    nnt[l] = best;
    dj = bv;
  }
  __syncthreads();
  float q = 0.0f;
  if (act)
    for (int j = 0; j < m; ++j)
      if (nnt[j] == l) q += wts[j];
  const float Q = wave_sum(q);
  const float wa = wave_sum(act ? wh * a : 0.0f);
  const double lx = wave_sum_d(act ? (double)wts[l] * dj : 0.0) +
                    wave_sum_d(act ? (double)wh * a : 0.0);
  const double lw = -wave_sum_d(act ? (double)q * logw : 0.0);
  if (l == 0) loss[b] = lx + lw;
  float* g32 = dO32 + (size_t)b * outp;
  u16* g16 = dO16 + (size_t)b * outp;
  if (act) {
    for (int t = 0; t < d; ++t) {
      const float di = del[l * 65 + t];
      float g = wh * (di - tt[nnp * 65 + t]);
      for (int j = 0; j < m; ++j)
        if (nnt[j] == l) g += wts[j] * (di - tt[j * 65 + t]);
      g *= 2.0f * invB;
      g32[l * d + t] = g;
      g16[l * d + t] = f2bf(g);
    }
    const float gl = (wh * Q - q + wh * (a - wa)) * invB;
    g32[m * d + l] = gl;
    g16[m * d + l] = f2bf(gl);
  }
  for (int t = m * (d + 1) + l; t < outp; t += 64) {
    g32[t] = 0.0f;
    g16[t] = 0;
  }
}

// dZ2[r][h] = bf16(pw[r] dG[seg r][h]) where H2[r][h] > 0, else 0
__global__ void k_dz2(const float* dG, const float* pw, const int32_t* seg,
                      const u16* H2, int H, long n, u16* dZ) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const long r = q / H;
  const int h = (int)(q % H);
  const float v = bf2f(H2[q]) > 0.0f ? pw[r] * dG[(size_t)seg[r] * H + h] : 0.0f;
  dZ[q] = f2bf(v);
}

// ------------------------------------------------------------- optimizer

__global__ void k_sqnorm(const float* g, long n, float* part) {
  __shared__ float sh[256];
  float s = 0.0f;
  for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < n;
       q += (long)gridDim.x * 256)
    s += g[q] * g[q];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

struct AdamArgs {
  float* th;
  float* m1;
  float* m2;
  const float* g;
  const float* norm_part;
  int nparts;
  long n;
  float lr, b1, b2, eps, c1, c2, clip;  // c1, c2: 1 - beta^t
};

__global__ void k_adam(AdamArgs a) {
  __shared__ float scale;
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int q = 0; q < a.nparts; ++q) s += a.norm_part[q];
    const float nrm = sqrtf(s);
    scale = (a.clip > 0.0f && nrm > a.clip) ? a.clip / nrm : 1.0f;
  }
  __syncthreads();
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.n) return;
  const float g = a.g[q] * scale;
  const float m1 = a.b1 * a.m1[q] + (1.0f - a.b1) * g;
  const float m2 = a.b2 * a.m2[q] + (1.0f - a.b2) * g * g;
  a.m1[q] = m1;
  a.m2[q] = m2;
  a.th[q] -= a.lr * (m1 / a.c1) / (sqrtf(m2 / a.c2) + a.eps);
}

// BF16 copies of a master matrix W[in][out]: row-major and transposed
__global__ void k_refresh(const float* W, int nin, int nout, u16* rm,
                          u16* tr) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long)nin * nout) return;
  const int i = (int)(q / nout), o = (int)(q % nout);
  const u16 v = f2bf(W[q]);
  if (rm) rm[q] = v;
  tr[(size_t)o * nin + i] = v;
}

// ------------------------------------------------------- proposal + gate

// Product-coupling bound of centroid (x, w) for a cluster with weighted
// mean mu, total weight Wt and S = sum w |y - mu|^2:
//   sum_k sum_ij w_i w_j^(k) |x_i - y_j^(k)|^2
//     = Wt (sum_i w_i |x_i - xbar|^2 + |xbar - mu|^2) + S.
// One wavefront per segment: x_i = mu + s Delta_i, w = softmax(logits);
// accepted (finite and, if gated, bound <= the current centroid's bound)
// proposals overwrite the context's centroid.
__device__ double product_bound(const double* x, const double* w, int m,
                                int d, const double* mu, double Wt, double S,
                                int l) {
  double V = 0.0, dm = 0.0;
  for (int t = 0; t < d; ++t) {
    double xb = 0.0;
    for (int i = 0; i < m; ++i) xb += w[i] * x[i * d + t];
    double v = 0.0;
    for (int i = l; i < m; i += 64) {
      const double e = x[i * d + t] - xb;
      v += w[i] * e * e;
    }
    V += wave_sum_d(v);
    dm += (xb - mu[t]) * (xb - mu[t]);
  }
  return Wt * (V + dm) + S;
}

__global__ __launch_bounds__(64) void k_propose(
    const float* O, int outp, int m, int d, const int32_t* bid,
    const double* mud, const double* sd, const double* Sdev,
    const double* wsum, int MP, double* xc, double* wc, int gate,
    int32_t* accepted, double* bprop, double* bplain) {
  __shared__ double xp[2048];
  __shared__ double wp[64];
  __shared__ double xq[2048];
  __shared__ double wq[64];
  const int b = blockIdx.x, l = threadIdx.x;
  const int c = bid[b];
  const float* o = O + (size_t)b * outp;
  const double* mu = mud + (size_t)b * d;
  const double s = sd[b];
  for (int q = l; q < m * d; q += 64) {
    xp[q] = mu[q % d] + s * (double)o[q];
    xq[q] = xc[((size_t)c * MP + q / d) * d + q % d];
  }
  const bool act = l < m;
  const float lg = act ? o[m * d + l] : -INFINITY;
  const float mx = wave_max(lg);
  const double ex = act ? exp((double)lg - (double)mx) : 0.0;
  const double se = wave_sum_d(ex);
  if (act) {
    wp[l] = ex / se;
    wq[l] = wc[(size_t)c * MP + l];
  }
  __syncthreads();
  const double bp = product_bound(xp, wp, m, d, mu, wsum[b], Sdev[b], l);
  const double bq = product_bound(xq, wq, m, d, mu, wsum[b], Sdev[b], l);
  bool ok = std::isfinite(bp) && std::isfinite(se);
  for (int q = 0; q < m * d && ok; ++q) ok = std::isfinite(xp[q]);
  if (gate) ok = ok && bp <= bq;
  if (ok) {
    for (int q = l; q < m * d; q += 64)
      xc[((size_t)c * MP + q / d) * d + q % d] = xp[q];
    if (act) wc[(size_t)c * MP + l] = wp[l];
  }
  if (l == 0) {
    accepted[c] = ok ? 1 : 0;
    bprop[c] = bp;
    bplain[c] = bq;
  }
}

// targets from the context's centroids (double, rows padded to MP)
__global__ void k_targets(const double* xc, const double* wc, int K, int m,
                          int d, int MP, float* tx, float* tw) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nx = (long)K * m * d;
  if (q < nx) {
    const long c = q / ((long)m * d), r = q % ((long)m * d);
    tx[q] = (float)xc[((size_t)c * MP + r / d) * d + r % d];
  } else if (q < nx + (long)K * m) {
    const long e = q - nx, c = e / m, i = e % m;
    tw[e] = (float)wc[(size_t)c * MP + i];
  }
}

// ------------------------------------------------ rounded-plan objective

// For instance k in cluster c (one wavefront): the plan Pi (m x m_k,
// column-major at pofs[k]) is rounded to a coupling with row sums w_c and
// column sums w^(k) exactly (scale rows down to at most w_c, then columns
// down to at most w^(k), then add the rank-one correction
// err_r err_c^T / |err_r|_1), and its cost sum_ij Pi_ij |x_i - y_j|^2 is
// written to val[k].  All arithmetic in FP64.
template <typename T>
__global__ __launch_bounds__(64) void k_feasible(
    const T* P, const int64_t* pofs, const int64_t* off, const T* X,
    const T* W, int xs, int d, const int32_t* labels, const double* xc,
    const double* wc, int m, int MP, double* val) {
  __shared__ double xr[64], yc[64], er[64], ec[64];
  const int64_t k = blockIdx.x;
  const int l = threadIdx.x;
  const int c = labels[k];
  const int64_t o0 = off[k];
  const int mk = (int)(off[k + 1] - o0);
  const T* pk = P + pofs[k];
  // row scaling
  if (l < m) {
    double r = 0.0;
    for (int j = 0; j < mk; ++j) r += (double)pk[(size_t)j * m + l];
    const double a = wc[(size_t)c * MP + l];
    xr[l] = r > a ? a / r : 1.0;
  }
  __syncthreads();
  // column scaling
  if (l < mk) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += xr[i] * (double)pk[(size_t)l * m + i];
    const double bj = (double)W[o0 + l];
    yc[l] = s > bj ? bj / s : 1.0;
  }
  __syncthreads();
  if (l < m) {
    double r = 0.0;
    for (int j = 0; j < mk; ++j) r += xr[l] * (double)pk[(size_t)j * m + l] * yc[j];
    er[l] = wc[(size_t)c * MP + l] - r;
  }
  if (l < mk) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += xr[i] * (double)pk[(size_t)l * m + i] * yc[l];
    ec[l] = (double)W[o0 + l] - s;
  }
  __syncthreads();
  double E = 0.0;
  for (int i = 0; i < m; ++i) E += er[i];
  double v = 0.0;
  if (l < mk) {
    const double* xcc = xc + (size_t)c * MP * d;
    for (int i = 0; i < m; ++i) {
      double cij = 0.0;
      for (int t = 0; t < d; ++t) {
        const double df = xcc[i * d + t] - (double)X[(size_t)(o0 + l) * xs + t];
        cij += df * df;
      }
      double pij = xr[i] * (double)pk[(size_t)l * m + i] * yc[l];
      if (E > 0.0) pij += er[i] * ec[l] / E;
      v += pij * cij;
    }
  }
  v = wave_sum_d(v);
  if (l == 0) val[k] = v;
}

}  // namespace ws

// ======================================================================
using ws::u16;

struct d2_ws {
  int device = 0;
  int m = 0, d = 0, H = 0, din = 0, out = 0, outp = 0;
  int64_t np = 0;
  std::string err;
  // parameter block offsets (flat FP32 vector)
  int64_t oW1, ob1, oW2, ob2, oV1, oe1, oV2, oe2, oV3, oe3;
  float* th = nullptr;
  float* gr = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* npart = nullptr;  // gradient-norm partials
  int64_t step = 0;
  // BF16 weights: transposed (forward) and row-major (backward)
  u16 *W1t = nullptr, *W2t = nullptr, *V1t = nullptr, *V2t = nullptr,
      *V3t = nullptr;
  u16 *W2r = nullptr, *V1r = nullptr, *V2r = nullptr, *V3r = nullptr;
  // training targets (K x m x d, K x m)
  float* tx = nullptr;
  float* tw = nullptr;
  int Kt = 0;
  // per-context point lists
  const d2_ctx* lctx = nullptr;
  uint64_t lgen = ~0ull;
  int lK = 0;
  std::vector<int64_t> h_pstart;
  std::vector<int32_t> h_nmem;
  int32_t* plist = nullptr;
  float* pmk = nullptr;
  int64_t* pstart = nullptr;
  int64_t plist_cap = 0, pstart_cap = 0;
  // batch workspace
  int64_t Pcap = 0;
  int Bcap = 0, CHcap = 0;
  u16 *F = nullptr, *H1 = nullptr, *H2 = nullptr, *DZ2 = nullptr,
      *DZ1 = nullptr;
  float* pw = nullptr;
  int32_t* seg = nullptr;
  int32_t* meta = nullptr;  // bid | rs | cstart | chunks
  float* nmemf = nullptr;
  float *mu = nullptr, *sc = nullptr;
  double *mud = nullptr, *sd = nullptr, *Sdev = nullptr, *wsum = nullptr;
  float *G = nullptr, *O = nullptr, *dO32 = nullptr, *dG = nullptr;
  u16 *Gq = nullptr, *U1 = nullptr, *U2 = nullptr, *dO16 = nullptr,
      *dA1 = nullptr, *dA2 = nullptr;
  double* loss = nullptr;
  float* poolp = nullptr;
  float* wpart = nullptr;
  size_t wpart_cap = 0;
  // proposal outputs (per cluster of the context)
  int32_t* acc = nullptr;
  double *bp = nullptr, *bq = nullptr;
  int accK = 0;
  // rounded-plan objective
  double* fval = nullptr;
  int64_t fcap = 0;

  d2_status fail(d2_status s, const std::string& msg) {
    err = msg;
    return s;
  }
};

namespace {

constexpr int kNormParts = 256;
constexpr size_t kWpartBytes = (size_t)64 << 20;

#define WSCHK(w, call)                                                    \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess)                                                 \
      return (w)->fail(D2_EDEVICE, std::string(#call) + ": " +            \
                                       hipGetErrorString(e_));            \
  } while (0)

template <typename P> void wfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

template <typename P>
d2_status walloc(d2_ws* w, P*& p, size_t count) {
  wfree(p);
  if (count == 0) count = 1;
  if (hipMalloc((void**)&p, sizeof(P) * count) != hipSuccess) {
    p = nullptr;
    return w->fail(D2_ENOMEM, "device allocation of " +
                                  std::to_string(sizeof(P) * count) +
                                  " bytes failed");
  }
  return D2_OK;
}

void layout(d2_ws* w) {
  const int64_t H = w->H;
  int64_t o = 0;
  w->oW1 = o; o += (int64_t)w->din * H;
  w->ob1 = o; o += H;
  w->oW2 = o; o += H * H;
  w->ob2 = o; o += H;
  w->oV1 = o; o += H * H;
  w->oe1 = o; o += H;
  w->oV2 = o; o += H * H;
  w->oe2 = o; o += H;
  w->oV3 = o; o += H * w->outp;
  w->oe3 = o; o += w->outp;
  w->np = o;
}

d2_status refresh(d2_ws* w, hipStream_t st) {
  struct M { int64_t o; int nin, nout; u16 *rm, *tr; };
  const M mats[5] = {{w->oW1, w->din, w->H, nullptr, w->W1t},
                     {w->oW2, w->H, w->H, w->W2r, w->W2t},
                     {w->oV1, w->H, w->H, w->V1r, w->V1t},
                     {w->oV2, w->H, w->H, w->V2r, w->V2t},
                     {w->oV3, w->H, w->outp, w->V3r, w->V3t}};
  for (const M& x : mats) {
    const long n = (long)x.nin * x.nout;
    ws::k_refresh<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
        w->th + x.o, x.nin, x.nout, x.rm, x.tr);
  }
  WSCHK(w, hipGetLastError());
  return D2_OK;
}

// point lists of the context's current labels, sorted by cluster
d2_status ensure_lists(d2_ws* w, d2_ctx* c) {
  if (w->lctx == c && w->lgen == c->label_gen && w->lK == c->K)
    return D2_OK;
  WSCHK(w, hipStreamSynchronize(c->stream));
  WSCHK(w, c->sync_labels());
  const int K = c->K;
  std::vector<int64_t> cnt(K + 1, 0);
  std::vector<int32_t> nmem(K, 0);
  for (int64_t k = 0; k < c->N; ++k) {
    const int l = c->h_labels[k];
    cnt[l + 1] += c->h_off[k + 1] - c->h_off[k];
    ++nmem[l];
  }
  for (int q = 0; q < K; ++q) cnt[q + 1] += cnt[q];
  std::vector<int32_t> pl(c->n);
  std::vector<float> mk(c->n);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t k = 0; k < c->N; ++k) {
    const int l = c->h_labels[k];
    const int64_t a = c->h_off[k], e = c->h_off[k + 1];
    for (int64_t p = a; p < e; ++p) {
      pl[pos[l]] = (int32_t)p;
      mk[pos[l]] = (float)(e - a);
      ++pos[l];
    }
  }
  d2_status s;
  if (w->plist_cap < c->n) {
    if ((s = walloc(w, w->plist, c->n))) return s;
    if ((s = walloc(w, w->pmk, c->n))) return s;
    w->plist_cap = c->n;
  }
  if (w->pstart_cap < K + 1) {
    if ((s = walloc(w, w->pstart, K + 1))) return s;
    w->pstart_cap = K + 1;
  }
  WSCHK(w, hipMemcpy(w->plist, pl.data(), sizeof(int32_t) * c->n,
                     hipMemcpyHostToDevice));
  WSCHK(w, hipMemcpy(w->pmk, mk.data(), sizeof(float) * c->n,
                     hipMemcpyHostToDevice));
  WSCHK(w, hipMemcpy(w->pstart, cnt.data(), sizeof(int64_t) * (K + 1),
                     hipMemcpyHostToDevice));
  w->h_pstart.swap(cnt);
  w->h_nmem.swap(nmem);
  w->lctx = c;
  w->lgen = c->label_gen;
  w->lK = K;
  return D2_OK;
}

constexpr int kPoolRows = 256;

d2_status ensure_work(d2_ws* w, int64_t P, int B, int nchunk) {
  d2_status s;
  const int H = w->H;
  if (P > w->Pcap) {
    const int64_t cap = std::max<int64_t>(P, 4096);
    if ((s = walloc(w, w->F, (size_t)cap * w->din))) return s;
    if ((s = walloc(w, w->H1, (size_t)cap * H))) return s;
    if ((s = walloc(w, w->H2, (size_t)cap * H))) return s;
    if ((s = walloc(w, w->DZ2, (size_t)cap * H))) return s;
    if ((s = walloc(w, w->DZ1, (size_t)cap * H))) return s;
    if ((s = walloc(w, w->pw, cap))) return s;
    if ((s = walloc(w, w->seg, cap))) return s;
    w->Pcap = cap;
  }
  if (B > w->Bcap || nchunk > w->CHcap) {
    const int bc = std::max(B, std::max(w->Bcap, 64));
    const int cc = std::max(nchunk, std::max(w->CHcap, 256));
    const int d = w->d, op = w->outp;
    if ((s = walloc(w, w->meta, (size_t)2 * bc + 2 + 3 * (size_t)cc + bc + 1)))
      return s;
    if ((s = walloc(w, w->nmemf, bc))) return s;
    if ((s = walloc(w, w->mu, (size_t)bc * d))) return s;
    if ((s = walloc(w, w->sc, bc))) return s;
    if ((s = walloc(w, w->mud, (size_t)bc * d))) return s;
    if ((s = walloc(w, w->sd, bc))) return s;
    if ((s = walloc(w, w->Sdev, bc))) return s;
    if ((s = walloc(w, w->wsum, bc))) return s;
    if ((s = walloc(w, w->G, (size_t)bc * H))) return s;
    if ((s = walloc(w, w->Gq, (size_t)bc * H))) return s;
    if ((s = walloc(w, w->U1, (size_t)bc * H))) return s;
    if ((s = walloc(w, w->U2, (size_t)bc * H))) return s;
    if ((s = walloc(w, w->O, (size_t)bc * op))) return s;
    if ((s = walloc(w, w->dO32, (size_t)bc * op))) return s;
    if ((s = walloc(w, w->dO16, (size_t)bc * op))) return s;
    if ((s = walloc(w, w->dA1, (size_t)bc * H))) return s;
    if ((s = walloc(w, w->dA2, (size_t)bc * H))) return s;
    if ((s = walloc(w, w->dG, (size_t)bc * H))) return s;
    if ((s = walloc(w, w->loss, bc))) return s;
    if ((s = walloc(w, w->poolp, (size_t)cc * H))) return s;
    w->Bcap = bc;
    w->CHcap = cc;
  }
  return D2_OK;
}

struct HostBatch {
  std::vector<int32_t> ids;
  std::vector<int32_t> rs, cstart, chunks;
  std::vector<float> nm;
  int64_t P = 0;
  int nchunk = 0;
};

d2_status make_batch(d2_ws* w, const int32_t* ids, int B, HostBatch& hb) {
  hb.ids.assign(ids, ids + B);
  hb.rs.assign(B + 1, 0);
  hb.cstart.assign(B + 1, 0);
  hb.chunks.clear();
  hb.nm.resize(B);
  int64_t P = 0;
  for (int b = 0; b < B; ++b) {
    const int c = ids[b];
    if (c < 0 || c >= w->lK) return w->fail(D2_EINVAL, "cluster id out of range");
    if (w->h_nmem[c] == 0)
      return w->fail(D2_EINVAL, "cluster " + std::to_string(c) + " is empty");
    const int64_t np = w->h_pstart[c + 1] - w->h_pstart[c];
    hb.rs[b] = (int32_t)P;
    for (int64_t r = 0; r < np; r += kPoolRows) {
      hb.chunks.push_back(b);
      hb.chunks.push_back((int32_t)(P + r));
      hb.chunks.push_back((int32_t)(P + std::min<int64_t>(np, r + kPoolRows)));
    }
    hb.cstart[b + 1] = (int32_t)(hb.chunks.size() / 3);
    hb.nm[b] = (float)w->h_nmem[c];
    P += np;
    if (P > INT32_MAX / 2) return w->fail(D2_EINVAL, "batch too large");
  }
  hb.rs[B] = (int32_t)P;
  hb.P = P;
  hb.nchunk = (int)(hb.chunks.size() / 3);
  return D2_OK;
}

// upload the batch tables; returns the device Batch view
d2_status upload_batch(d2_ws* w, hipStream_t st, const HostBatch& hb,
                       ws::Batch& bt, int32_t*& d_cstart,
                       int32_t*& d_chunks) {
  const int B = (int)hb.ids.size();
  std::vector<int32_t> meta;
  meta.insert(meta.end(), hb.ids.begin(), hb.ids.end());
  meta.insert(meta.end(), hb.rs.begin(), hb.rs.end());
  meta.insert(meta.end(), hb.cstart.begin(), hb.cstart.end());
  meta.insert(meta.end(), hb.chunks.begin(), hb.chunks.end());
  WSCHK(w, hipMemcpyAsync(w->meta, meta.data(), sizeof(int32_t) * meta.size(),
                          hipMemcpyHostToDevice, st));
  WSCHK(w, hipMemcpyAsync(w->nmemf, hb.nm.data(), sizeof(float) * B,
                          hipMemcpyHostToDevice, st));
  WSCHK(w, hipStreamSynchronize(st));  // host vectors are freed on return
  bt.bid = w->meta;
  bt.rs = w->meta + B;
  bt.nmem = w->nmemf;
  bt.plist = w->plist;
  bt.pmk = w->pmk;
  bt.pstart = w->pstart;
  bt.B = B;
  d_cstart = w->meta + 2 * B + 1;
  d_chunks = w->meta + 3 * B + 2;
  return D2_OK;
}

void gemm(hipStream_t st, const u16* A, int lda, const u16* Bt, int ldb,
          int M, int N, int K, const float* bias, int relu, const u16* mask,
          int ldm, u16* c16, int ldc, float* c32, int ldc32) {
  ws::GemmArgs g{A, Bt, bias, mask, c16, c32, M, N, K, lda, ldb, ldm, ldc,
                 ldc32, relu};
  dim3 grid((unsigned)((M + 127) / 128), (unsigned)((N + 127) / 128));
  ws::k_gemm<<<grid, 256, 0, st>>>(g);
}

d2_status wgrad(d2_ws* w, hipStream_t st, const u16* X, int ldx,
                const u16* Y, int ldy, int R, int Kx, int Ny, int64_t woff,
                int64_t boff) {
  const long pstride = (long)Kx * Ny + Ny;
  if (!w->wpart) {
    d2_status s = walloc(w, w->wpart, kWpartBytes / sizeof(float));
    if (s) return s;
    w->wpart_cap = kWpartBytes / sizeof(float);
  }
  int nch_max = (int)std::max<long>(1, (long)(w->wpart_cap / pstride));
  int rc = 64;
  while ((R + rc - 1) / rc > std::min(nch_max, 512)) rc += 64;
  const int nch = std::max(1, (R + rc - 1) / rc);
  ws::WgArgs g{X, Y, w->wpart, ldx, ldy, R, Kx, Ny, rc, pstride};
  dim3 grid((unsigned)nch, (unsigned)((Ny + 127) / 128));
  ws::k_wgrad<<<grid, 256, 0, st>>>(g);
  const long tot = pstride;
  ws::k_wgrad_reduce<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(
      w->wpart, pstride, nch, Kx, Ny, w->gr, (long)woff, (long)boff);
  return D2_OK;
}

// network forward over one batch: stats, features, point MLP, pooling, head
template <typename T>
d2_status forward(d2_ws* w, d2_ctx* c, const HostBatch& hb, ws::Batch& bt,
                  int32_t* d_cstart, int32_t* d_chunks) {
  hipStream_t st = c->stream;
  const int B = bt.B, H = w->H;
  const int P = (int)hb.P;
  const float* th = w->th;
  ws::k_stats<T><<<B, 256, 0, st>>>((const T*)c->d_X, (const T*)c->d_W,
                                    c->xs, c->d, bt, w->mu, w->sc, w->mud,
                                    w->sd, w->Sdev, w->wsum);
  ws::k_feat<T><<<(P + 255) / 256, 256, 0, st>>>(
      (const T*)c->d_X, (const T*)c->d_W, c->xs, c->d, w->din, bt, w->mu,
      w->sc, P, w->F, w->pw, w->seg);
  gemm(st, w->F, w->din, w->W1t, w->din, P, H, w->din, th + w->ob1, 1,
       nullptr, 0, w->H1, H, nullptr, 0);
  gemm(st, w->H1, H, w->W2t, H, P, H, H, th + w->ob2, 1, nullptr, 0, w->H2,
       H, nullptr, 0);
  ws::k_pool_part<<<hb.nchunk, H, 0, st>>>(w->H2, w->pw, H, d_chunks,
                                            w->poolp);
  ws::k_pool_fin<<<B, H, 0, st>>>(w->poolp, d_cstart, H, w->G, w->Gq);
  gemm(st, w->Gq, H, w->V1t, H, B, H, H, th + w->oe1, 1, nullptr, 0, w->U1,
       H, nullptr, 0);
  gemm(st, w->U1, H, w->V2t, H, B, H, H, th + w->oe2, 1, nullptr, 0, w->U2,
       H, nullptr, 0);
  gemm(st, w->U2, H, w->V3t, H, B, w->outp, H, th + w->oe3, 0, nullptr, 0,
       nullptr, 0, w->O, w->outp);
  WSCHK(w, hipGetLastError());
  return D2_OK;
}

d2_status backward(d2_ws* w, d2_ctx* c, const HostBatch& hb,
                   const ws::Batch& bt) {
  hipStream_t st = c->stream;
  const int B = bt.B, H = w->H, op = w->outp;
  const int P = (int)hb.P;
  d2_status s;
  ws::k_loss<<<B, 64, 0, st>>>(w->O, op, w->m, w->d, bt.bid, w->tx, w->tw,
                               w->mu, w->sc, 1.0f / (float)B, w->dO32,
                               w->dO16, w->loss);
  // head
  gemm(st, w->dO16, op, w->V3r, op, B, H, op, nullptr, 0, w->U2, H, w->dA2,
       H, nullptr, 0);
  if ((s = wgrad(w, st, w->U2, H, w->dO16, op, B, H, op, w->oV3, -1))) return s;
  ws::k_colsum<<<(op + 127) / 128, 128, 0, st>>>(w->dO32, B, op, op,
                                                  w->gr + w->oe3);
  gemm(st, w->dA2, H, w->V2r, H, B, H, H, nullptr, 0, w->U1, H, w->dA1, H,
       nullptr, 0);
  if ((s = wgrad(w, st, w->U1, H, w->dA2, H, B, H, H, w->oV2, w->oe2)))
    return s;
  gemm(st, w->dA1, H, w->V1r, H, B, H, H, nullptr, 0, nullptr, 0, nullptr, 0,
       w->dG, H);
  if ((s = wgrad(w, st, w->Gq, H, w->dA1, H, B, H, H, w->oV1, w->oe1)))
    return s;
  // point MLP
  const long n = (long)P * H;
  ws::k_dz2<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(w->dG, w->pw, w->seg,
                                                         w->H2, H, n, w->DZ2);
  if ((s = wgrad(w, st, w->H1, H, w->DZ2, H, P, H, H, w->oW2, w->ob2)))
    return s;
  gemm(st, w->DZ2, H, w->W2r, H, P, H, H, nullptr, 0, w->H1, H, w->DZ1, H,
       nullptr, 0);
  if ((s = wgrad(w, st, w->F, w->din, w->DZ1, H, P, w->din, H, w->oW1,
                 w->ob1)))
    return s;
  WSCHK(w, hipGetLastError());
  return D2_OK;
}

d2_status check_pair(d2_ws* w, d2_ctx* c) {
  if (!w || !c) return D2_EINVAL;
  if (c->device != w->device)
    return w->fail(D2_EINVAL, "context and warm start on different devices");
  if (!c->N || !c->K || !c->have_labels)
    return w->fail(D2_ESTATE, "context needs instances, centroids, labels");
  if (c->sym)
    return w->fail(D2_EINVAL, "symbolic supports have no coordinates");
  if (c->m != w->m || c->d != w->d)
    return w->fail(D2_EINVAL, "context m / d differ from the network's");
  return D2_OK;
}

d2_status grad_batch(d2_ws* w, d2_ctx* c, const int32_t* ids, int B,
                     double* loss_out) {
  d2_status s;
  if (B < 1 || !ids) return w->fail(D2_EINVAL, "empty batch");
  if (!w->tx) return w->fail(D2_ESTATE, "no training targets");
  if (c->K != w->Kt)
    return w->fail(D2_ESTATE, "targets were taken from a different K");
  if ((s = ensure_lists(w, c))) return s;
  HostBatch hb;
  if ((s = make_batch(w, ids, B, hb))) return s;
  if ((s = ensure_work(w, hb.P, B, hb.nchunk))) return s;
  ws::Batch bt;
  int32_t *dcs, *dch;
  if ((s = upload_batch(w, c->stream, hb, bt, dcs, dch))) return s;
  s = c->dt == D2_F64 ? forward<double>(w, c, hb, bt, dcs, dch)
                      : forward<float>(w, c, hb, bt, dcs, dch);
  if (s) return s;
  if ((s = backward(w, c, hb, bt))) return s;
  if (loss_out) {
    std::vector<double> lv(B);
    WSCHK(w, hipMemcpyAsync(lv.data(), w->loss, sizeof(double) * B,
                            hipMemcpyDeviceToHost, c->stream));
    WSCHK(w, hipStreamSynchronize(c->stream));
    double t = 0.0;
    for (double v : lv) t += v;
    *loss_out = t / B;
  }
  return D2_OK;
}

}  // namespace

extern "C" {

int64_t d2_ws_param_count(int32_t m, int32_t d, int32_t hidden) {
  if (m < 1 || m > 64 || d < 1 || d > 64 || m * d > 2048 || hidden < 32 ||
      hidden > 128 || hidden % 32)
    return -1;
  d2_ws w;
  w.m = m;
  w.d = d;
  w.H = hidden;
  w.din = (d + 1 + 15) / 16 * 16;
  w.out = m * (d + 1);
  w.outp = (w.out + 31) / 32 * 32;
  layout(&w);
  return w.np;
}

d2_status d2_ws_create(d2_ws** out, int32_t device, int32_t m, int32_t d,
                       int32_t hidden, const float* theta) {
  if (!out) return D2_EINVAL;
  *out = nullptr;
  if (d2_ws_param_count(m, d, hidden) < 0 || !theta) return D2_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return D2_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return D2_EDEVICE;
  d2_ws* w = new d2_ws;
  w->device = device;
  w->m = m;
  w->d = d;
  w->H = hidden;
  w->din = (d + 1 + 15) / 16 * 16;
  w->out = m * (d + 1);
  w->outp = (w->out + 31) / 32 * 32;
  layout(w);
  d2_status s = D2_OK;
  const int H = hidden;
  if (!s) s = walloc(w, w->th, w->np);
  if (!s) s = walloc(w, w->gr, w->np);
  if (!s) s = walloc(w, w->m1, w->np);
  if (!s) s = walloc(w, w->m2, w->np);
  if (!s) s = walloc(w, w->npart, kNormParts);
  if (!s) s = walloc(w, w->W1t, (size_t)w->din * H);
  if (!s) s = walloc(w, w->W2t, (size_t)H * H);
  if (!s) s = walloc(w, w->V1t, (size_t)H * H);
  if (!s) s = walloc(w, w->V2t, (size_t)H * H);
  if (!s) s = walloc(w, w->V3t, (size_t)H * w->outp);
  if (!s) s = walloc(w, w->W2r, (size_t)H * H);
  if (!s) s = walloc(w, w->V1r, (size_t)H * H);
  if (!s) s = walloc(w, w->V2r, (size_t)H * H);
  if (!s) s = walloc(w, w->V3r, (size_t)H * w->outp);
  if (!s) s = d2_ws_params_set(w, theta);
  if (s) {
    d2_ws_destroy(w);
    return s;
  }
  *out = w;
  return D2_OK;
}

void d2_ws_destroy(d2_ws* w) {
  if (!w) return;
  (void)hipSetDevice(w->device);
  (void)hipDeviceSynchronize();
  wfree(w->th); wfree(w->gr); wfree(w->m1); wfree(w->m2); wfree(w->npart);
  wfree(w->W1t); wfree(w->W2t); wfree(w->V1t); wfree(w->V2t); wfree(w->V3t);
  wfree(w->W2r); wfree(w->V1r); wfree(w->V2r); wfree(w->V3r);
  wfree(w->tx); wfree(w->tw);
  wfree(w->plist); wfree(w->pmk); wfree(w->pstart);
  wfree(w->F); wfree(w->H1); wfree(w->H2); wfree(w->DZ2); wfree(w->DZ1);
  wfree(w->pw); wfree(w->seg); wfree(w->meta); wfree(w->nmemf);
  wfree(w->mu); wfree(w->sc); wfree(w->mud); wfree(w->sd); wfree(w->Sdev);
  wfree(w->wsum); wfree(w->G); wfree(w->O); wfree(w->dO32); wfree(w->dG);
  wfree(w->Gq); wfree(w->U1); wfree(w->U2); wfree(w->dO16); wfree(w->dA1);
  wfree(w->dA2); wfree(w->loss); wfree(w->poolp); wfree(w->wpart);
  wfree(w->acc); wfree(w->bp); wfree(w->bq); wfree(w->fval);
  delete w;
}

const char* d2_ws_last_error(const d2_ws* w) {
  return w ? w->err.c_str() : "null warm-start handle";
}

d2_status d2_ws_params_set(d2_ws* w, const float* theta) {
  if (!w || !theta) return D2_EINVAL;
  for (int64_t q = 0; q < w->np; ++q)
    if (!std::isfinite(theta[q]))
      return w->fail(D2_EINVAL, "non-finite parameter at " + std::to_string(q));
  WSCHK(w, hipSetDevice(w->device));
  WSCHK(w, hipMemcpy(w->th, theta, sizeof(float) * w->np,
                     hipMemcpyHostToDevice));
  WSCHK(w, hipMemset(w->m1, 0, sizeof(float) * w->np));
  WSCHK(w, hipMemset(w->m2, 0, sizeof(float) * w->np));
  WSCHK(w, hipMemset(w->gr, 0, sizeof(float) * w->np));
  w->step = 0;
  d2_status s = refresh(w, nullptr);
  if (s) return s;
  WSCHK(w, hipDeviceSynchronize());
  return D2_OK;
}

d2_status d2_ws_params_get(d2_ws* w, float* theta) {
  if (!w || !theta) return D2_EINVAL;
  WSCHK(w, hipSetDevice(w->device));
  WSCHK(w, hipDeviceSynchronize());
  WSCHK(w, hipMemcpy(theta, w->th, sizeof(float) * w->np,
                     hipMemcpyDeviceToHost));
  return D2_OK;
}

namespace {
constexpr char kWsMagic[8] = {'D', '2', 'W', 'S', 'N', 'E', 'T', 1};
struct WsHeader {
  char magic[8];
  int32_t m, d, H, pad;
  int64_t np, step;
};
uint64_t fnv(const void* p, size_t n, uint64_t h) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t q = 0; q < n; ++q) h = (h ^ b[q]) * 1099511628211ull;
  return h;
}
}  // namespace

d2_status d2_ws_save(d2_ws* w, const char* path) {
  if (!w) return D2_EINVAL;
  if (!path) return w->fail(D2_EINVAL, "null path");
  WSCHK(w, hipSetDevice(w->device));
  WSCHK(w, hipDeviceSynchronize());
  std::vector<float> buf((size_t)3 * w->np);
  WSCHK(w, hipMemcpy(buf.data(), w->th, sizeof(float) * w->np,
                     hipMemcpyDeviceToHost));
  WSCHK(w, hipMemcpy(buf.data() + w->np, w->m1, sizeof(float) * w->np,
                     hipMemcpyDeviceToHost));
  WSCHK(w, hipMemcpy(buf.data() + 2 * w->np, w->m2, sizeof(float) * w->np,
                     hipMemcpyDeviceToHost));
  WsHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kWsMagic, 8);
  h.m = w->m;
  h.d = w->d;
  h.H = w->H;
  h.np = w->np;
  h.step = w->step;
  uint64_t sum = fnv(&h, sizeof(h), 1469598103934665603ull);
  sum = fnv(buf.data(), sizeof(float) * buf.size(), sum);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return w->fail(D2_EINVAL, "cannot open " + tmp + " for writing");
  bool ok = fwrite(&h, sizeof(h), 1, f) == 1 &&
            fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size() &&
            fwrite(&sum, 8, 1, f) == 1;
  ok = (fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return w->fail(D2_EINVAL, std::string("writing ") + path + " failed");
  }
  return D2_OK;
}

d2_status d2_ws_load(d2_ws* w, const char* path) {
  if (!w) return D2_EINVAL;
  if (!path) return w->fail(D2_EINVAL, "null path");
  FILE* f = fopen(path, "rb");
  if (!f) return w->fail(D2_EINVAL, std::string("cannot open ") + path);
  WsHeader h;
  std::vector<float> buf((size_t)3 * w->np);
  uint64_t sum = 0;
  bool ok = fread(&h, sizeof(h), 1, f) == 1;
  const bool same = ok && std::memcmp(h.magic, kWsMagic, 8) == 0 &&
                    h.m == w->m && h.d == w->d && h.H == w->H &&
                    h.np == w->np && h.step >= 0;
  ok = same && fread(buf.data(), sizeof(float), buf.size(), f) == buf.size() &&
       fread(&sum, 8, 1, f) == 1;
  fclose(f);
  if (!same)
    return w->fail(D2_EINVAL, std::string(path) +
                                  ": not a network of this shape (m, d, H)");
  if (!ok) return w->fail(D2_EINVAL, std::string(path) + ": truncated");
  uint64_t want = fnv(&h, sizeof(h), 1469598103934665603ull);
  want = fnv(buf.data(), sizeof(float) * buf.size(), want);
  if (want != sum)
    return w->fail(D2_EINVAL, std::string(path) + ": checksum mismatch");
  for (size_t q = 0; q < buf.size(); ++q)
    if (!std::isfinite(buf[q]))
      return w->fail(D2_EINVAL, std::string(path) + ": non-finite values");
  WSCHK(w, hipSetDevice(w->device));
  WSCHK(w, hipDeviceSynchronize());
  WSCHK(w, hipMemcpy(w->th, buf.data(), sizeof(float) * w->np,
                     hipMemcpyHostToDevice));
  WSCHK(w, hipMemcpy(w->m1, buf.data() + w->np, sizeof(float) * w->np,
                     hipMemcpyHostToDevice));
  WSCHK(w, hipMemcpy(w->m2, buf.data() + 2 * w->np, sizeof(float) * w->np,
                     hipMemcpyHostToDevice));
  w->step = h.step;
  d2_status s = refresh(w, nullptr);
  if (s) return s;
  WSCHK(w, hipDeviceSynchronize());
  return D2_OK;
}

d2_status d2_ws_targets_from(d2_ws* w, d2_ctx* c) {
  d2_status s = check_pair(w, c);
  if (s) return s;
  WSCHK(w, hipSetDevice(w->device));
  const int K = c->K, m = w->m, d = w->d;
  if ((s = walloc(w, w->tx, (size_t)K * m * d))) return s;
  if ((s = walloc(w, w->tw, (size_t)K * m))) return s;
  const long n = (long)K * m * (d + 1);
  ws::k_targets<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(
      c->d_xc, c->d_wc, K, m, d, c->MP, w->tx, w->tw);
  WSCHK(w, hipGetLastError());
  WSCHK(w, hipStreamSynchronize(c->stream));
  w->Kt = K;
  return D2_OK;
}

d2_status d2_ws_grad(d2_ws* w, d2_ctx* c, const int32_t* clusters,
                     int32_t nb, double* loss, float* grad) {
  d2_status s = check_pair(w, c);
  if (s) return s;
  WSCHK(w, hipSetDevice(w->device));
  if ((s = grad_batch(w, c, clusters, nb, loss))) return s;
  if (grad) {
    WSCHK(w, hipMemcpyAsync(grad, w->gr, sizeof(float) * w->np,
                            hipMemcpyDeviceToHost, c->stream));
    WSCHK(w, hipStreamSynchronize(c->stream));
  }
  return D2_OK;
}

d2_status d2_ws_train_step(d2_ws* w, d2_ctx* c, const int32_t* clusters,
                           int32_t nb, const d2_ws_opt* opt, double* loss) {
  d2_status s = check_pair(w, c);
  if (s) return s;
  if (!opt || !(opt->lr > 0.0) || !(opt->beta1 >= 0.0 && opt->beta1 < 1.0) ||
      !(opt->beta2 >= 0.0 && opt->beta2 < 1.0) || !(opt->eps > 0.0) ||
      !(opt->clip >= 0.0))
    return w->fail(D2_EINVAL, "bad optimizer settings");
  WSCHK(w, hipSetDevice(w->device));
  if ((s = grad_batch(w, c, clusters, nb, loss))) return s;
  hipStream_t st = c->stream;
  ++w->step;
  ws::k_sqnorm<<<kNormParts, 256, 0, st>>>(w->gr, (long)w->np, w->npart);
  ws::AdamArgs a;
  a.th = w->th;
  a.m1 = w->m1;
  a.m2 = w->m2;
  a.g = w->gr;
  a.norm_part = w->npart;
  a.nparts = kNormParts;
  a.n = (long)w->np;
  a.lr = (float)opt->lr;
  a.b1 = (float)opt->beta1;
  a.b2 = (float)opt->beta2;
  a.eps = (float)opt->eps;
  a.c1 = (float)(1.0 - std::pow(opt->beta1, (double)w->step));
  a.c2 = (float)(1.0 - std::pow(opt->beta2, (double)w->step));
  a.clip = (float)opt->clip;
  ws::k_adam<<<(unsigned)((w->np + 255) / 256), 256, 0, st>>>(a);
  if ((s = refresh(w, st))) return s;
  WSCHK(w, hipGetLastError());
  if (!loss) WSCHK(w, hipStreamSynchronize(st));
  return D2_OK;
}

d2_status d2_ws_propose(d2_ws* w, d2_ctx* c, int32_t gate, int32_t* accepted,
                        double* bound_prop, double* bound_plain) {
  d2_status s = check_pair(w, c);
  if (s) return s;
  WSCHK(w, hipSetDevice(w->device));
  if ((s = ensure_lists(w, c))) return s;
  const int K = c->K;
  if (w->accK < K) {
    if ((s = walloc(w, w->acc, K))) return s;
    if ((s = walloc(w, w->bp, K))) return s;
    if ((s = walloc(w, w->bq, K))) return s;
    w->accK = K;
  }
  hipStream_t st = c->stream;
  // -1 marks empty clusters (nothing proposed)
  std::vector<int32_t> init(K, -1);
  WSCHK(w, hipMemcpyAsync(w->acc, init.data(), sizeof(int32_t) * K,
                          hipMemcpyHostToDevice, st));
  // batches of whole clusters, about 2^20 rows each
  std::vector<int32_t> ids;
  int64_t rows = 0;
  auto flush = [&]() -> d2_status {
    if (ids.empty()) return D2_OK;
    HostBatch hb;
    d2_status e;
    if ((e = make_batch(w, ids.data(), (int)ids.size(), hb))) return e;
    if ((e = ensure_work(w, hb.P, (int)ids.size(), hb.nchunk))) return e;
    ws::Batch bt;
    int32_t *dcs, *dch;
    if ((e = upload_batch(w, st, hb, bt, dcs, dch))) return e;
    e = c->dt == D2_F64 ? forward<double>(w, c, hb, bt, dcs, dch)
                        : forward<float>(w, c, hb, bt, dcs, dch);
    if (e) return e;
    ws::k_propose<<<bt.B, 64, 0, st>>>(w->O, w->outp, w->m, w->d, bt.bid,
                                       w->mud, w->sd, w->Sdev, w->wsum,
                                       c->MP, c->d_xc, c->d_wc, gate ? 1 : 0,
                                       w->acc, w->bp, w->bq);
    WSCHK(w, hipGetLastError());
    ids.clear();
    rows = 0;
    return D2_OK;
  };
  for (int q = 0; q < K; ++q) {
    if (w->h_nmem[q] == 0) continue;
    const int64_t np = w->h_pstart[q + 1] - w->h_pstart[q];
    if (!ids.empty() && (rows + np > (1 << 20) || ids.size() >= 1024))
      if ((s = flush())) return s;
    ids.push_back(q);
    rows += np;
  }
  if ((s = flush())) return s;
  std::vector<double> bpv(K), bqv(K);
  std::vector<int32_t> av(K);
  WSCHK(w, hipMemcpyAsync(av.data(), w->acc, sizeof(int32_t) * K,
                          hipMemcpyDeviceToHost, st));
  WSCHK(w, hipMemcpyAsync(bpv.data(), w->bp, sizeof(double) * K,
                          hipMemcpyDeviceToHost, st));
  WSCHK(w, hipMemcpyAsync(bqv.data(), w->bq, sizeof(double) * K,
                          hipMemcpyDeviceToHost, st));
  WSCHK(w, hipStreamSynchronize(st));
  bool any = false;
  for (int q = 0; q < K; ++q) {
    if (accepted) accepted[q] = av[q];
    if (bound_prop) bound_prop[q] = av[q] < 0 ? NAN : bpv[q];
    if (bound_plain) bound_plain[q] = av[q] < 0 ? NAN : bqv[q];
    any = any || av[q] == 1;
  }
  // the cached plans belong to the replaced centroids: a following
  // D2_INIT_CACHED call starts from the product coupling
  if (any) c->have_cache = false;
  return D2_OK;
}

d2_status d2_objective_feasible(d2_ctx* c, double* per_instance,
                                double* per_cluster) {
  if (!c) return D2_EINVAL;
  if (!c->d_P1 || !c->have_cache || !c->have_labels)
    return c->fail(D2_ESTATE, "no plans yet");
  if (c->cache_gen != c->label_gen)
    return c->fail(D2_ESTATE, "labels changed since the last barycenter");
  if (c->sym)
    return c->fail(D2_EINVAL, "not available for symbolic supports");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, c->sync_labels());
  std::vector<double> val(c->N);
  double* dv = nullptr;
  if (hipMalloc((void**)&dv, sizeof(double) * c->N) != hipSuccess)
    return c->fail(D2_ENOMEM, "device allocation failed");
  if (c->dt == D2_F64)
    ws::k_feasible<double><<<(unsigned)c->N, 64, 0, c->stream>>>(
        (const double*)c->d_P1, c->d_pofs, c->d_off, (const double*)c->d_X,
        (const double*)c->d_W, c->xs, c->d, c->d_labels, c->d_xc, c->d_wc,
        c->m, c->MP, dv);
  else
    ws::k_feasible<float><<<(unsigned)c->N, 64, 0, c->stream>>>(
        (const float*)c->d_P1, c->d_pofs, c->d_off, (const float*)c->d_X,
        (const float*)c->d_W, c->xs, c->d, c->d_labels, c->d_xc, c->d_wc,
        c->m, c->MP, dv);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(val.data(), dv, sizeof(double) * c->N,
                       hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(dv);
  if (e != hipSuccess)
    return c->fail(D2_EDEVICE, std::string("feasible objective: ") +
                                   hipGetErrorString(e));
  if (per_instance) std::copy(val.begin(), val.end(), per_instance);
  if (per_cluster) {
    std::vector<int64_t> cnt(c->K, 0);
    std::fill(per_cluster, per_cluster + c->K, 0.0);
    for (int64_t k = 0; k < c->N; ++k) {
      per_cluster[c->h_labels[k]] += val[k];
      ++cnt[c->h_labels[k]];
    }
    for (int q = 0; q < c->K; ++q)
      per_cluster[q] = cnt[q] ? per_cluster[q] / (double)cnt[q] : 0.0;
  }
  return D2_OK;
}

}  // extern "C"

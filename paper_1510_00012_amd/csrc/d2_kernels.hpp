// HIP kernels (gfx950, wave64) for batched B-ADMM Wasserstein barycenters.
//
// Paper: Ye, Wu, Wang, Li, "Fast Discrete Distribution Clustering Using
// Wasserstein Barycenter with Sparse Support".  Sec. 3.2 gives the updates:
//   Pi1  = col-normalise( Pi2 * exp(-(C + Lambda)/rho) + eps ) * w^(k)_j
//                                                   Eq. (badmmc0b), (badmmc0)
//   Pi1~ = Pi1 * exp(Lambda/rho) + eps               Eq. (badmmc1b)
//   w    = R1 / R2 consensus of the row-normalised Pi1~   Eq. (badmmw/badmmw2)
//   Pi2  = row-normalise(Pi1~) * w_i                 Eq. (badmmc1)
//   Lambda += rho (Pi1 - Pi2)                        Eq. (badmm2)
//   x_i  = sum Pi2_ij x^(k)_j / sum Pi2_ij           Eq. (updatex)
//
// Work decomposition.  One wavefront owns one instance's m x m_k plan tile
// at a time.  Lane l holds row i = l % MP (MP = m padded to a power of two)
// of column j = l / MP + (64/MP) r for register slot r < R, so a slot is
// 64/MP whole columns and each load of a slot is a contiguous, coalesced
// 64-entry run of the column-major tile.  Column sums reduce over the MP
// lanes of a column group, row sums over the slots in-lane and then across
// column groups (xor shuffles).  A workgroup processes one "chunk": a run of
// instances of a single cluster from the cluster-sorted work list.  The
// cluster-wide quantities (weight consensus, objective, support numerators,
// rho) are reduced per chunk into a double record; the last workgroup of a
// cluster to finish (atomic ticket) sums the records in chunk order and
// writes the cluster result, so every reduction has a fixed order and runs
// are bitwise reproducible.
//
// Iteration schedule (carried state = Pi1 and Lambda between launches):
//   A0            Pi2^0 (product or cached), Lambda = 0 -> Pi1^1, w^1
//   BA (hot)      [Pi2^{n+1}, Lambda^{n+1} from Pi1^{n+1}, Lambda^n, w^{n+1};
//                  then Pi1^{n+2}, w^{n+2}]      (one launch per iteration)
//   BX / BF       phase B only: store Pi2, Lambda; support numerators
//   AP            phase A from stored Pi2, Lambda (after a support update)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d2k {

constexpr int kWave = 64;

template <typename T> __device__ __forceinline__ T dexp(T v);
template <> __device__ __forceinline__ float dexp<float>(float v) {
  return expf(v);
}
template <> __device__ __forceinline__ double dexp<double>(double v) {
  return exp(v);
}
template <typename T> __device__ __forceinline__ T dsqrt(T v);
template <> __device__ __forceinline__ float dsqrt<float>(float v) {
  return sqrtf(v);
}
template <> __device__ __forceinline__ double dsqrt<double>(double v) {
  return sqrt(v);
}

// Sum over the MP lanes of one column group (same lane / MP).
template <int MP, typename T> __device__ __forceinline__ T sum_col(T v) {
#pragma unroll
  for (int s = 1; s < MP; s <<= 1) v += __shfl_xor(v, s, kWave);
  return v;
}
// Sum over the column groups (lanes with the same lane % MP).
template <int MP, typename T> __device__ __forceinline__ T sum_row(T v) {
#pragma unroll
  for (int s = MP; s < kWave; s <<= 1) v += __shfl_xor(v, s, kWave);
  return v;
}
template <typename T> __device__ __forceinline__ T sum_wave(T v) {
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

// Kernel modes (a uniform runtime switch of the auxiliary kernel).
enum Mode : int {
  kRho = 0,  // cost at the initial support (stored if cached), rho per cluster
  kA0 = 1,   // phase A from Pi2^0 (product / cached), Lambda := 0
  kAP = 2,   // phase A from stored Pi2 and Lambda; recompute + store cost
  kBX = 3,   // phase B, store Pi2 and Lambda, support numerators
  kBF = 4,   // phase B, store Pi2 and Lambda (last iteration, no x update)
  kXO = 5,   // support numerators from stored Pi2 only
};

struct Chunk {
  int32_t cluster, begin, end, pad;
};

template <typename T> struct Args {
  const int64_t* off;   // N+1 instance offsets
  const T* X;           // n x d supports
  const T* W;           // n weights
  const int32_t* work;  // instance ids sorted by cluster
  const Chunk* chunks;  // per workgroup
  const int2* ctab;     // per cluster {first chunk, number of chunks}
  const double* ninv;   // per cluster 1 / N_c
  const double* cinv;   // per cluster 1 / (m * sum_k m_k)
  T* P1;
  T* P2;
  T* L;
  T* Cc;                // cost cache (m x n) or nullptr when computed on the fly
  const uint8_t* warm;  // per instance: start from cached Pi2
  double* xc;           // K x MP x d centroid support
  const double* w_in;   // K x MP weights used by phase B
  double* w_out;        // K x MP weights produced by phase A
  double* rho;          // K
  double* part;         // chunk records, stride ps
  double* partx;        // chunk support numerators, stride MP*(d+1)
  int* cnt;             // per cluster tickets (zero between launches)
  double* trace;        // K objective values of this iteration, or nullptr
  double rho0, eps;
  int m, d, rule, ps, onfly, nchunks;
};

// ---------------------------------------------------------------------------
// Per-cluster finalisation by the last workgroup (fixed-order sums).
// ---------------------------------------------------------------------------
template <typename T>
__device__ bool take_ticket(const Args<T>& a, int c, int nch, int* s_flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int prev = atomicAdd(&a.cnt[c], 1);
    *s_flag = (prev == nch - 1);
  }
  __syncthreads();
  bool last = *s_flag != 0;
  if (last) __threadfence();
  return last;
}

template <typename T>
__device__ void release_ticket(const Args<T>& a, int c) {
  if (threadIdx.x == 0) atomicExch(&a.cnt[c], 0);
}

// Sums columns [0, ncol) of the records of chunks first .. first+nch-1
// (stride `stride`) into out[ncol] (LDS), in a fixed order.
__device__ inline void sum_records(const double* part, int stride, int first,
                                   int nch, int ncol, double* red,
                                   double* out) {
  const int nt = blockDim.x;
  const int groups = nt / ncol;  // >= 1 (ncol <= nt)
  const int tid = threadIdx.x;
  const int col = tid % ncol, grp = tid / ncol;
  double s = 0.0;
  if (grp < groups) {
    for (int q = grp; q < nch; q += groups)
      s += part[(int64_t)(first + q) * stride + col];
    red[grp * ncol + col] = s;
  }
  __syncthreads();
  if (tid < ncol) {
    double t = 0.0;
    for (int gI = 0; gI < groups; ++gI) t += red[gI * ncol + tid];
    out[tid] = t;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Tile helpers
// ---------------------------------------------------------------------------
template <typename T, int MP, int R> struct Tile {
  static constexpr int CPS = kWave / MP;
  int lane, i, g, k, mk, nsl, c;
  int64_t o, base;
  bool rowok;

  __device__ __forceinline__ void setup(const Args<T>& a, int kk, int cc) {
    lane = threadIdx.x & (kWave - 1);
    i = lane % MP;
    g = lane / MP;
    k = kk;
    c = cc;
    o = a.off[k];
    mk = (int)(a.off[k + 1] - o);
    nsl = (mk + CPS - 1) / CPS;
    base = (int64_t)a.m * o;
    rowok = i < a.m;
  }
  __device__ __forceinline__ int col(int r) const { return g + CPS * r; }
  __device__ __forceinline__ bool valid(int r) const {
    return rowok && col(r) < mk;
  }
  __device__ __forceinline__ int64_t idx(int r, int m) const {
    return base + (int64_t)col(r) * m + i;
  }
};

// cost C_ij = sum_t (x_i,t - y_j,t)^2 in T, explicit fma chain
template <typename T>
__device__ __forceinline__ T cost_generic(const double* xrow, const T* yrow,
                                          int d) {
  T s = T(0);
  for (int t = 0; t < d; ++t) {
    T df = (T)xrow[t] - yrow[t];
    s = fma(df, df, s);
  }
  return s;
}

// ---------------------------------------------------------------------------
// Phase B: Pi1~ = Pi1 exp(Lambda/rho) + eps, row sums, Pi2 = Pi1~ w_i / r_i,
// Lambda += rho (Pi1 - Pi2).  On entry p = Pi1, on exit p = Pi2.
// ---------------------------------------------------------------------------
template <typename T, int MP, int R>
__device__ __forceinline__ void phase_b(const Tile<T, MP, R>& tl, T (&p)[R],
                                        T (&l)[R], T wi, T rho, T irho,
                                        T eps) {
  T bv[R];
  T rs = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    bv[r] = T(0);
    if (r < tl.nsl && tl.valid(r)) bv[r] = p[r] * dexp(l[r] * irho) + eps;
    rs += bv[r];
  }
  rs = sum_row<MP>(rs);
  T coef = rs > T(0) ? wi / rs : T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < tl.nsl) {
      T p2 = bv[r] * coef;
      l[r] = l[r] + rho * (p[r] - p2);
      p[r] = p2;
    }
  }
}

// Phase A: given p = Pi2, l = Lambda, cost cs and instance weights wk:
// p <- Pi1 (column KL projection), returns the row sum r_i of Pi1~ through
// rr, and accumulates <C, Pi1> in f.
template <typename T, int MP, int R>
__device__ __forceinline__ void phase_a(const Tile<T, MP, R>& tl, T (&p)[R],
                                        const T (&l)[R], const T (&cs)[R],
                                        const T (&wk)[R], T irho, T eps,
                                        T& rr, T& f) {
  rr = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < tl.nsl) {
      bool v = tl.valid(r);
      T av = v ? p[r] * dexp(-(cs[r] + l[r]) * irho) + eps : T(0);
      T s = sum_col<MP>(av);
      T p1 = (v && s > T(0)) ? av * (wk[r] / s) : T(0);
      f = fma(cs[r], p1, f);
      T b = v ? p1 * dexp(l[r] * irho) + eps : T(0);
      rr += b;
      p[r] = p1;
    }
  }
  rr = sum_row<MP>(rr);
}

// ---------------------------------------------------------------------------
// Hot kernel: one launch per B-ADMM iteration (phase B of n, phase A of n+1)
// ---------------------------------------------------------------------------
template <typename T, int MP, int R>
__global__ void __launch_bounds__(256) k_iter_ba(Args<T> a) {
  __shared__ double s_w[4][MP + 1];
  __shared__ double s_red[256];
  __shared__ double s_out[MP + 1];
  __shared__ int s_flag;
  const int ch = blockIdx.x;
  if (ch >= a.nchunks) return;
  const Chunk cj = a.chunks[ch];
  const int c = cj.cluster;
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  const T rho = (T)a.rho[c];
  const T irho = T(1) / rho;
  const T eps = (T)a.eps;
  const int lane = threadIdx.x & (kWave - 1);
  const int i = lane % MP;
  const T wi = i < a.m ? (T)a.w_in[c * MP + i] : T(0);
  double accw = 0.0, accf = 0.0;
  // on-the-fly cost for d <= 4: centroid row held in registers
  T xr[4] = {T(0), T(0), T(0), T(0)};
  if (a.onfly) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < a.d && i < a.m) xr[t] = (T)a.xc[((int64_t)c * MP + i) * a.d + t];
  }
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<T, MP, R> tl;
    tl.setup(a, a.work[pos], c);
    T p[R], l[R], cs[R], wk[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      p[r] = T(0);
      l[r] = T(0);
      cs[r] = T(0);
      wk[r] = T(0);
      if (r < tl.nsl && tl.valid(r)) {
        int64_t e = tl.idx(r, a.m);
        p[r] = a.P1[e];
        l[r] = a.L[e];
        int j = tl.col(r);
        wk[r] = a.W[tl.o + j];
        if (a.onfly) {
          const T* y = a.X + (tl.o + j) * a.d;
          T s = T(0);
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (t < a.d) {
              T df = xr[t] - y[t];
              s = fma(df, df, s);
            }
          cs[r] = s;
        } else {
          cs[r] = a.Cc[e];
        }
      }
    }
    phase_b<T, MP, R>(tl, p, l, wi, rho, irho, eps);
    T rr, f = T(0);
    phase_a<T, MP, R>(tl, p, l, cs, wk, irho, eps, rr, f);
    T tot = sum_col<MP>(tl.rowok ? rr : T(0));
    T wt = tot > T(0) ? rr / tot : T(0);
    accw += (double)(a.rule == 2 ? dsqrt(wt) : wt);
    accf += (double)f;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < tl.nsl && tl.valid(r)) {
        int64_t e = tl.idx(r, a.m);
        a.P1[e] = p[r];
        a.L[e] = l[r];
      }
  }
  // chunk record: weight sums (rows) + objective
  accf = sum_wave(accf);
  if (lane < MP) s_w[wave][lane] = accw;
  if (lane == 0) s_w[wave][MP] = accf;
  __syncthreads();
  if (threadIdx.x <= MP) {
    double s = 0.0;
    for (int q = 0; q < nwaves; ++q) s += s_w[q][threadIdx.x];
    a.part[(int64_t)ch * a.ps + threadIdx.x] = s;
  }
  const int2 ct = a.ctab[c];
  if (!take_ticket(a, c, ct.y, &s_flag)) return;
  sum_records(a.part, a.ps, ct.x, ct.y, MP + 1, s_red, s_out);
  if (threadIdx.x == 0) {
    double ni = a.ninv[c];
    double vs = 0.0;
    double v[MP];
    for (int q = 0; q < MP; ++q) {
      double t = q < a.m ? s_out[q] * ni : 0.0;
      v[q] = a.rule == 2 ? t * t : t;
      vs += v[q];
    }
    for (int q = 0; q < MP; ++q) a.w_out[c * MP + q] = v[q] / vs;
    if (a.trace) a.trace[c] = s_out[MP] * ni;
  }
  release_ticket(a, c);
}

// ---------------------------------------------------------------------------
// Auxiliary kernel: rho / init phase A / phase B variants / support update
// ---------------------------------------------------------------------------
template <typename T, int MP, int R>
__global__ void __launch_bounds__(256) k_aux(Args<T> a, int mode) {
  extern __shared__ double s_dyn[];  // [nwaves][MP][d+1] support numerators
  __shared__ double s_w[4][MP + 1];
  __shared__ double s_red[256];
  __shared__ double s_out[MP + 1];
  __shared__ int s_flag;
  const int ch = blockIdx.x;
  if (ch >= a.nchunks) return;
  const Chunk cj = a.chunks[ch];
  const int c = cj.cluster;
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int i = lane % MP;
  const int d = a.d;
  const bool xnum = (mode == kBX || mode == kXO);
  const T eps = (T)a.eps;
  T rho = T(1), irho = T(1), wi = T(0);
  if (mode != kRho) {
    rho = (T)a.rho[c];
    irho = T(1) / rho;
  }
  if (mode == kBX || mode == kBF) wi = i < a.m ? (T)a.w_in[c * MP + i] : T(0);
  if (mode == kA0) wi = i < a.m ? (T)a.w_in[c * MP + i] : T(0);
  const double* xrow = a.xc + ((int64_t)c * MP + i) * d;
  double* accx = s_dyn + (int64_t)wave * MP * (d + 1);
  if (xnum) {
    for (int q = lane; q < MP * (d + 1); q += kWave) accx[q] = 0.0;
  }
  double accw = 0.0, accf = 0.0;
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<T, MP, R> tl;
    tl.setup(a, a.work[pos], c);
    T p[R], l[R], cs[R], wk[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      p[r] = T(0);
      l[r] = T(0);
      cs[r] = T(0);
      wk[r] = T(0);
    }
    if (mode == kRho) {
      T s = T(0);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < tl.nsl && tl.valid(r)) {
          int j = tl.col(r);
          T cv = cost_generic<T>(xrow, a.X + (tl.o + j) * d, d);
          if (a.Cc) a.Cc[tl.idx(r, a.m)] = cv;
          s += cv;
        }
      accf += (double)s;  // lane partial; reduced over the wave below
      continue;
    }
    if (mode == kA0 || mode == kAP) {
      const bool cached = (mode == kAP) || (a.warm && a.warm[tl.k]);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < tl.nsl && tl.valid(r)) {
          int64_t e = tl.idx(r, a.m);
          int j = tl.col(r);
          wk[r] = a.W[tl.o + j];
          T cv = cost_generic<T>(xrow, a.X + (tl.o + j) * d, d);
          if (mode == kAP && a.Cc) a.Cc[e] = cv;
          cs[r] = (mode == kA0 && a.Cc) ? a.Cc[e] : cv;
          if (mode == kAP) {
            p[r] = a.P2[e];
            l[r] = a.L[e];
          } else {
            p[r] = cached ? a.P2[e] : wi * wk[r];
          }
        }
      T rr, f = T(0);
      phase_a<T, MP, R>(tl, p, l, cs, wk, irho, eps, rr, f);
      T tot = sum_col<MP>(tl.rowok ? rr : T(0));
      T wt = tot > T(0) ? rr / tot : T(0);
      accw += (double)(a.rule == 2 ? dsqrt(wt) : wt);
      accf += (double)f;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < tl.nsl && tl.valid(r)) {
          int64_t e = tl.idx(r, a.m);
          a.P1[e] = p[r];
          a.L[e] = l[r];
        }
      continue;
    }
    // phase-B modes and the support-only mode
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < tl.nsl && tl.valid(r)) {
        int64_t e = tl.idx(r, a.m);
        if (mode == kXO) {
          p[r] = a.P2[e];
        } else {
          p[r] = a.P1[e];
          l[r] = a.L[e];
        }
      }
    if (mode != kXO) {
      phase_b<T, MP, R>(tl, p, l, wi, rho, irho, eps);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < tl.nsl && tl.valid(r)) {
          int64_t e = tl.idx(r, a.m);
          a.P2[e] = p[r];
          a.L[e] = l[r];
        }
    }
    if (xnum) {
      // numerators sum_j Pi2_ij y_j,t and denominators sum_j Pi2_ij
      for (int t = 0; t <= d; ++t) {
        T v = T(0);
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (r < tl.nsl && tl.valid(r)) {
            T yv = t < d ? a.X[(tl.o + tl.col(r)) * d + t] : T(1);
            v = fma(p[r], yv, v);
          }
        v = sum_row<MP>(v);
        if (lane < MP) accx[lane * (d + 1) + t] += (double)v;
      }
    }
  }
  const int2 ct = a.ctab[c];
  if (mode == kRho) {
    accf = sum_wave(accf);
    if (lane == 0) s_w[wave][0] = accf;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int q = 0; q < nwaves; ++q) s += s_w[q][0];
      a.part[(int64_t)ch * a.ps] = s;
    }
    if (!take_ticket(a, c, ct.y, &s_flag)) return;
    sum_records(a.part, a.ps, ct.x, ct.y, 1, s_red, s_out);
    if (threadIdx.x == 0) a.rho[c] = a.rho0 * s_out[0] * a.cinv[c];
    release_ticket(a, c);
    return;
  }
  if (mode == kA0 || mode == kAP) {
    accf = sum_wave(accf);
    if (lane < MP) s_w[wave][lane] = accw;
    if (lane == 0) s_w[wave][MP] = accf;
    __syncthreads();
    if (threadIdx.x <= MP) {
      double s = 0.0;
      for (int q = 0; q < nwaves; ++q) s += s_w[q][threadIdx.x];
      a.part[(int64_t)ch * a.ps + threadIdx.x] = s;
    }
    if (!take_ticket(a, c, ct.y, &s_flag)) return;
    sum_records(a.part, a.ps, ct.x, ct.y, MP + 1, s_red, s_out);
    if (threadIdx.x == 0) {
      double ni = a.ninv[c];
      double vs = 0.0;
      double v[MP];
      for (int q = 0; q < MP; ++q) {
        double t = q < a.m ? s_out[q] * ni : 0.0;
        v[q] = a.rule == 2 ? t * t : t;
        vs += v[q];
      }
      for (int q = 0; q < MP; ++q) a.w_out[c * MP + q] = v[q] / vs;
      if (a.trace) a.trace[c] = s_out[MP] * ni;
    }
    release_ticket(a, c);
    return;
  }
  if (!xnum) return;
  // support numerators: chunk record = sum over waves (fixed order)
  __syncthreads();
  const int nrec = MP * (d + 1);
  const int64_t xs = (int64_t)nrec;
  for (int q = threadIdx.x; q < nrec; q += blockDim.x) {
    double s = 0.0;
    for (int wv = 0; wv < nwaves; ++wv) s += s_dyn[(int64_t)wv * nrec + q];
    a.partx[(int64_t)ch * xs + q] = s;
  }
  if (!take_ticket(a, c, ct.y, &s_flag)) return;
  for (int q = threadIdx.x; q < nrec; q += blockDim.x) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int nq = ct.y;
    int u = 0;
    for (; u + 3 < nq; u += 4) {
      s0 += a.partx[(int64_t)(ct.x + u) * xs + q];
      s1 += a.partx[(int64_t)(ct.x + u + 1) * xs + q];
      s2 += a.partx[(int64_t)(ct.x + u + 2) * xs + q];
      s3 += a.partx[(int64_t)(ct.x + u + 3) * xs + q];
    }
    for (; u < nq; ++u) s0 += a.partx[(int64_t)(ct.x + u) * xs + q];
    s_dyn[q] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < MP * d; q += blockDim.x) {
    int ii = q / d, t = q % d;
    double den = s_dyn[ii * (d + 1) + d];
    if (ii < a.m && den > 1e-300)
      a.xc[((int64_t)c * MP + ii) * d + t] = s_dyn[ii * (d + 1) + t] / den;
  }
  release_ticket(a, c);
}

// ---------------------------------------------------------------------------
// Assignment: one wavefront per instance, B-ADMM transport against every
// centroid with both marginals fixed; argmin with ties to the lowest index.
// ---------------------------------------------------------------------------
template <typename T> struct AssignArgs {
  const int64_t* off;
  const T* X;
  const T* W;
  const double* xc;  // K x MP x d
  const double* wc;  // K x MP
  int32_t* labels;
  double* best;
  int64_t N;
  double rho0, eps;
  int m, d, K, iters;
};

template <typename T, int MP, int R>
__global__ void __launch_bounds__(256) k_assign(AssignArgs<T> a) {
  constexpr int CPS = kWave / MP;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t k = (int64_t)blockIdx.x * (blockDim.x / kWave) +
                    threadIdx.x / kWave;
  if (k >= a.N) return;  // whole wavefront exits together
  const int i = lane % MP, g = lane / MP;
  const int64_t o = a.off[k];
  const int mk = (int)(a.off[k + 1] - o);
  const int nsl = (mk + CPS - 1) / CPS;
  const bool rowok = i < a.m;
  const T eps = (T)a.eps;
  T wk[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int j = g + CPS * r;
    wk[r] = (r < nsl && rowok && j < mk) ? a.W[o + j] : T(0);
  }
  double bestv = 0.0;
  int bestc = -1;
  for (int c = 0; c < a.K; ++c) {
    const double* xrow = a.xc + ((int64_t)c * MP + i) * a.d;
    T cs[R], p1[R], p2[R], l[R];
    T csum = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int j = g + CPS * r;
      bool v = r < nsl && rowok && j < mk;
      cs[r] = v ? cost_generic<T>(xrow, a.X + (o + j) * a.d, a.d) : T(0);
      csum += cs[r];
    }
    double tot = sum_wave((double)csum);
    const T rho = (T)(a.rho0 * tot / ((double)a.m * mk));
    const T irho = T(1) / rho;
    const T wi = rowok ? (T)a.wc[c * MP + i] : T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      p2[r] = wi * wk[r];
      l[r] = T(0);
      p1[r] = T(0);
    }
    for (int it = 0; it < a.iters; ++it) {
      T rr = T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r < nsl) {
          int j = g + CPS * r;
          bool v = rowok && j < mk;
          T av = v ? p2[r] * dexp(-(cs[r] + l[r]) * irho) + eps : T(0);
          T s = sum_col<MP>(av);
          T q = (v && s > T(0)) ? av * (wk[r] / s) : T(0);
          p1[r] = q;
          T b = v ? q * dexp(l[r] * irho) + eps : T(0);
          p2[r] = b;
          rr += b;
        }
      }
      rr = sum_row<MP>(rr);
      T coef = rr > T(0) ? wi / rr : T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r < nsl) {
          T q = p2[r] * coef;
          l[r] = l[r] + rho * (p1[r] - q);
          p2[r] = q;
        }
      }
    }
    T fv = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) fv = fma(cs[r], p1[r], fv);
    double val = sum_wave((double)fv);
    if (bestc < 0 || val < bestv) {
      bestv = val;
      bestc = c;
    }
  }
  if (lane == 0) {
    a.labels[k] = bestc;
    a.best[k] = bestv;
  }
}

}  // namespace d2k

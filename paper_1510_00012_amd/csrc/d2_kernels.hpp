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
// lanes of a column group with DPP row operations; row sums add the slots
// in-lane and then combine column groups (DPP row_ror / ds_swizzle /
// bpermute).  Loads of a tile are issued unconditionally (inactive lanes read
// a clamped in-bounds element and are masked afterwards) so that all of a
// tile's loads are in flight together.
//
// A workgroup processes one "chunk": a run of instances of one cluster from
// the cluster-sorted work list, and writes one double record per chunk
// (weight-consensus sums, objective, support numerators, cost sums).  A
// second small launch (k_fin, one workgroup per cluster) sums the records of
// each cluster in chunk order and writes the cluster result.  Every
// reduction has a fixed order, so runs are bitwise reproducible, and no
// cross-workgroup synchronisation happens inside a kernel.
//
// Iteration schedule (carried state = Pi1 and Lambda between launches):
//   A0       Pi2^0 (product or cached), Lambda = 0 -> Pi1^1, records for w^1
//   BA (hot) [Pi2^{n+1}, Lambda^{n+1} from Pi1^{n+1}, Lambda^n, w^{n+1};
//             then Pi1^{n+2}, records for w^{n+2}]   (one launch/iteration)
//   BX / BF  phase B only: store Pi2, Lambda; support numerators (BX)
//   AP       phase A from stored Pi2, Lambda (after a support update)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d2k {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// arithmetic helpers
// ---------------------------------------------------------------------------
// exp(x) for FP32: 2^(x log2 e) by the hardware base-2 exponential, with a
// first-order correction for the rounding error of the product x*log2(e)
// (its exact residual r gives exp(x) = 2^t * 2^r ~ 2^t (1 + r ln 2)).
__device__ __forceinline__ float dexp(float x) {
  const float kL2E = 1.44269502162933349609375f;       // log2(e) rounded
  const float kL2ELo = 1.925963033500011079e-08f;     // log2(e) - kL2E
  const float kLn2 = 0.693147180559945309f;
  float t = x * kL2E;
  float r = fmaf(x, kL2E, -t) + x * kL2ELo;
  float e = __builtin_amdgcn_exp2f(t);
  return fmaf(e, r * kLn2, e);
}
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float drcp(float x) {
  return __builtin_amdgcn_rcpf(x);
}
__device__ __forceinline__ double drcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float dsqrt(float v) { return sqrtf(v); }
__device__ __forceinline__ double dsqrt(double v) { return sqrt(v); }

// ---------------------------------------------------------------------------
// lane exchange: DPP within 16-lane rows, ds_swizzle across 16, bpermute 32
// ---------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ float xdpp(float v) {
  return __int_as_float(
      __builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double xdpp(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF,
                                    false);
  int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float xswz16(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}
__device__ __forceinline__ double xswz16(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffLL), 0x401F);
  int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T> __device__ __forceinline__ T x32(T v) {
  return __shfl_xor(v, 32, kWave);
}

// All-reduce over the MP lanes of a column group (lanes sharing lane / MP).
// Every lane ends with bitwise the same sum.
template <int MP, typename T> __device__ __forceinline__ T sum_col(T v) {
  if constexpr (MP >= 2) v += xdpp<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (MP >= 4) v += xdpp<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (MP >= 8) v += xdpp<0x141>(v);  // row_half_mirror
  if constexpr (MP >= 16) v += xdpp<0x140>(v); // row_mirror
  if constexpr (MP >= 32) v += xswz16(v);
  if constexpr (MP >= 64) v += x32(v);
  return v;
}
// All-reduce over the column groups (lanes sharing lane % MP).
template <int MP, typename T> __device__ __forceinline__ T sum_row(T v) {
  if constexpr (MP <= 8) v += xdpp<0x128>(v);  // row_ror:8
  if constexpr (MP <= 16) v += xswz16(v);
  if constexpr (MP <= 32) v += x32(v);
  return v;
}
template <typename T> __device__ __forceinline__ T sum_wave(T v) {
  return sum_col<64>(v);
}

// support point of a column for the on-the-fly cost (d <= 4, stride 4)
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Kernel modes of the auxiliary kernel (uniform runtime switch).
enum Mode : int {
  kRho = 0,  // cost at the initial support (stored if cached): cost sums
  kA0 = 1,   // phase A from Pi2^0 (product / cached), Lambda := 0
  kAP = 2,   // phase A from stored Pi2 and Lambda; recompute (+store) cost
  kBX = 3,   // phase B, store Pi2 and Lambda, support numerators
  kBF = 4,   // phase B, store Pi2 and Lambda (last iteration, no x update)
  kXO = 5,   // support numerators from stored Pi2 only
};
// Finalisation modes.
enum FinMode : int { kFinW = 0, kFinRho = 1, kFinX = 2 };

struct Chunk {
  int32_t cluster, begin, end, pad;
};

template <typename T> struct Args {
  const int64_t* off;   // N+1 instance offsets
  const T* X;           // n x xs supports (xs = 4 when d <= 4, zero padded)
  const T* W;           // n weights
  const int32_t* work;  // instance ids sorted by cluster
  const Chunk* chunks;  // per workgroup
  T* P1;
  T* P2;
  T* L;
  T* Cc;                // cost cache (m x n) or nullptr when computed on the fly
  const uint8_t* warm;  // per instance: start from cached Pi2
  const double* xc;     // K x MP x d centroid support
  const double* w_in;   // K x MP weights used by phase B / the product init
  const double* rho;    // K
  double* part;         // chunk records, stride ps
  double* partx;        // chunk support numerators, stride MP*(d+1)
  double eps;
  int m, d, xs, rule, ps, nchunks;
};

struct FinArgs {
  const int2* ctab;     // per cluster {first chunk, number of chunks}
  const double* ninv;   // per cluster 1 / N_c
  const double* cinv;   // per cluster 1 / (m * sum_k m_k)
  const double* part;
  const double* partx;
  double* w_out;        // K x MP
  double* rho;          // K
  double* xc;           // K x MP x d
  double* trace;        // K or nullptr
  double rho0;
  int m, d, rule, ps;
};

// ---------------------------------------------------------------------------
// tile loads / phases
// ---------------------------------------------------------------------------
template <typename T, int MP, int R> struct Tile {
  static constexpr int CPS = kWave / MP;
  int64_t o, base;
  int mk, i, g, ic;
  bool rowok;
  __device__ __forceinline__ void setup(const Args<T>& a, int k) {
    const int lane = threadIdx.x & (kWave - 1);
    i = lane % MP;
    g = lane / MP;
    rowok = i < a.m;
    ic = rowok ? i : 0;
    o = a.off[k];
    mk = (int)(a.off[k + 1] - o);
    base = (int64_t)a.m * o;
  }
  __device__ __forceinline__ int col(int r) const { return g + CPS * r; }
  __device__ __forceinline__ bool valid(int r) const {
    return rowok && col(r) < mk;
  }
  // in-bounds element index for every lane (inactive lanes clamp)
  __device__ __forceinline__ int colc(int r) const {
    int j = col(r);
    return j < mk ? j : mk - 1;
  }
  __device__ __forceinline__ int64_t eidx(int r, int m) const {
    return base + (int64_t)colc(r) * m + ic;
  }
};

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

template <typename T>
__device__ __forceinline__ T cost4(const T (&xr)[4],
                                   const typename Vec4<T>::type& y) {
  T s = T(0);
  T df = xr[0] - y.x;
  s = fma(df, df, s);
  df = xr[1] - y.y;
  s = fma(df, df, s);
  df = xr[2] - y.z;
  s = fma(df, df, s);
  df = xr[3] - y.w;
  s = fma(df, df, s);
  return s;
}

// Phase B: Pi1~ = Pi1 exp(Lambda/rho) + eps, row sums r_i,
// Pi2 = Pi1~ w_i / r_i, Lambda += rho (Pi1 - Pi2).  In: p = Pi1; out: p = Pi2.
template <typename T, int MP, int R>
__device__ __forceinline__ void phase_b(const bool (&v)[R], T (&p)[R],
                                        T (&l)[R], T wi, T rho, T irho,
                                        T eps) {
  T bv[R];
  T rs = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    bv[r] = v[r] ? p[r] * dexp(l[r] * irho) + eps : T(0);
    rs += bv[r];
  }
  rs = sum_row<MP>(rs);
  const T coef = rs > T(0) ? wi * drcp(rs) : T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T p2 = bv[r] * coef;
    l[r] = l[r] + rho * (p[r] - p2);
    p[r] = p2;
  }
}

// Phase A: in p = Pi2, l = Lambda, cost cs, instance weights wk; out
// p = Pi1 (column KL projection).  Returns the row sum r_i of Pi1~ in rr and
// adds <C, Pi1> to f.
template <typename T, int MP, int R>
__device__ __forceinline__ void phase_a(const bool (&v)[R], T (&p)[R],
                                        const T (&l)[R], const T (&cs)[R],
                                        const T (&wk)[R], T irho, T eps, T& rr,
                                        T& f) {
  rr = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T av = v[r] ? p[r] * dexp(-(cs[r] + l[r]) * irho) + eps : T(0);
    T s = sum_col<MP>(av);
    T p1 = (v[r] && s > T(0)) ? av * (wk[r] * drcp(s)) : T(0);
    f = fma(cs[r], p1, f);
    T b = v[r] ? p1 * dexp(l[r] * irho) + eps : T(0);
    rr += b;
    p[r] = p1;
  }
  rr = sum_row<MP>(rr);
}

// weight-consensus contribution w~_i (R1) or sqrt(w~_i) (R2) of one tile
template <typename T, int MP>
__device__ __forceinline__ double consensus_term(T rr, bool rowok, int rule) {
  T tot = sum_col<MP>(rowok ? rr : T(0));
  T wt = tot > T(0) ? rr / tot : T(0);
  return (double)(rule == 2 ? dsqrt(wt) : wt);
}

// chunk record: per-row weight sums (lanes < MP of each wave) + objective
template <int MP>
__device__ __forceinline__ void write_w_record(double accw, double accf,
                                               double* part, int ps, int ch) {
  __shared__ double s_w[4][MP + 1];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  accf = sum_wave(accf);
  if (lane < MP) s_w[wave][lane] = accw;
  if (lane == 0) s_w[wave][MP] = accf;
  __syncthreads();
  if (threadIdx.x <= MP) {
    double s = 0.0;
    for (int q = 0; q < nwaves; ++q) s += s_w[q][threadIdx.x];
    part[(int64_t)ch * ps + threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Hot kernel: one launch per B-ADMM iteration (phase B of n, phase A of n+1)
// ---------------------------------------------------------------------------
template <typename T, int MP, int R, bool ONFLY>
__global__ void __launch_bounds__(256) k_iter_ba(Args<T> a) {
  using V4 = typename Vec4<T>::type;
  const int ch = blockIdx.x;
  if (ch >= a.nchunks) return;
  const Chunk cj = a.chunks[ch];
  const int c = cj.cluster;
  const int wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int i = lane % MP;
  const bool rowok = i < a.m;
  const T rho = (T)a.rho[c];
  const T irho = T(1) / rho;
  const T eps = (T)a.eps;
  const T wi = rowok ? (T)a.w_in[c * MP + i] : T(0);
  T xr[4] = {T(0), T(0), T(0), T(0)};
  if constexpr (ONFLY) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < a.d && rowok) xr[t] = (T)a.xc[((int64_t)c * MP + i) * a.d + t];
  }
  double accw = 0.0, accf = 0.0;
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<T, MP, R> tl;
    tl.setup(a, a.work[pos]);
    T p[R], l[R], cs[R], wk[R];
    bool v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t e = tl.eidx(r, a.m);
      const int jc = tl.colc(r);
      v[r] = tl.valid(r);
      p[r] = a.P1[e];
      l[r] = a.L[e];
      wk[r] = a.W[tl.o + jc];
      if constexpr (ONFLY) {
        const V4 y = reinterpret_cast<const V4*>(a.X)[tl.o + jc];
        cs[r] = cost4<T>(xr, y);
      } else {
        cs[r] = a.Cc[e];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      p[r] = v[r] ? p[r] : T(0);
      l[r] = v[r] ? l[r] : T(0);
    }
    phase_b<T, MP, R>(v, p, l, wi, rho, irho, eps);
    T rr, f = T(0);
    phase_a<T, MP, R>(v, p, l, cs, wk, irho, eps, rr, f);
    accw += consensus_term<T, MP>(rr, rowok, a.rule);
    accf += (double)f;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (v[r]) {
        const int64_t e = tl.eidx(r, a.m);
        a.P1[e] = p[r];
        a.L[e] = l[r];
      }
  }
  write_w_record<MP>(accw, accf, a.part, a.ps, ch);
}

// ---------------------------------------------------------------------------
// Auxiliary kernel: cost sums / init phase A / phase-B variants / numerators
// ---------------------------------------------------------------------------
template <typename T, int MP, int R>
__global__ void __launch_bounds__(256) k_aux(Args<T> a, int mode) {
  extern __shared__ double s_dyn[];  // [nwaves][MP][d+1] support numerators
  const int ch = blockIdx.x;
  if (ch >= a.nchunks) return;
  const Chunk cj = a.chunks[ch];
  const int c = cj.cluster;
  const int wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int i = lane % MP;
  const int d = a.d;
  const bool rowok = i < a.m;
  const bool xnum = (mode == kBX || mode == kXO);
  const T eps = (T)a.eps;
  const T rho = mode == kRho ? T(1) : (T)a.rho[c];
  const T irho = T(1) / rho;
  const T wi = rowok ? (T)a.w_in[c * MP + i] : T(0);
  const double* xrow = a.xc + ((int64_t)c * MP + (rowok ? i : 0)) * d;
  double* accx = s_dyn + (int64_t)wave * MP * (d + 1);
  if (xnum)
    for (int q = lane; q < MP * (d + 1); q += kWave) accx[q] = 0.0;
  double accw = 0.0, accf = 0.0;
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<T, MP, R> tl;
    const int k = a.work[pos];
    tl.setup(a, k);
    T p[R], l[R], cs[R], wk[R];
    bool v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = tl.valid(r);
      p[r] = l[r] = cs[r] = wk[r] = T(0);
    }
    if (mode == kRho) {
      T s = T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        T cv = cost_generic<T>(xrow, a.X + (tl.o + tl.colc(r)) * a.xs, d);
        if (v[r]) {
          if (a.Cc) a.Cc[tl.eidx(r, a.m)] = cv;
          s += cv;
        }
      }
      accf += (double)s;  // lane partial, reduced over the wave at the end
      continue;
    }
    if (mode == kA0 || mode == kAP) {
      const bool cached = (mode == kAP) || (a.warm && a.warm[k]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t e = tl.eidx(r, a.m);
        const int jc = tl.colc(r);
        wk[r] = a.W[tl.o + jc];
        T cv = cost_generic<T>(xrow, a.X + (tl.o + jc) * a.xs, d);
        if (mode == kAP && a.Cc && v[r]) a.Cc[e] = cv;
        cs[r] = (mode == kA0 && a.Cc) ? a.Cc[e] : cv;
        if (mode == kAP) {
          p[r] = a.P2[e];
          l[r] = a.L[e];
        } else {
          p[r] = cached ? a.P2[e] : wi * wk[r];
        }
        p[r] = v[r] ? p[r] : T(0);
        l[r] = v[r] ? l[r] : T(0);
      }
      T rr, f = T(0);
      phase_a<T, MP, R>(v, p, l, cs, wk, irho, eps, rr, f);
      accw += consensus_term<T, MP>(rr, rowok, a.rule);
      accf += (double)f;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (v[r]) {
          const int64_t e = tl.eidx(r, a.m);
          a.P1[e] = p[r];
          a.L[e] = l[r];
        }
      continue;
    }
    // phase-B modes and the support-only mode
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t e = tl.eidx(r, a.m);
      if (mode == kXO) {
        p[r] = a.P2[e];
      } else {
        p[r] = a.P1[e];
        l[r] = a.L[e];
      }
      p[r] = v[r] ? p[r] : T(0);
      l[r] = v[r] ? l[r] : T(0);
    }
    if (mode != kXO) {
      phase_b<T, MP, R>(v, p, l, wi, rho, irho, eps);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (v[r]) {
          const int64_t e = tl.eidx(r, a.m);
          a.P2[e] = p[r];
          a.L[e] = l[r];
        }
    }
    if (xnum) {
      // numerators sum_j Pi2_ij y_j,t (t < d) and denominators sum_j Pi2_ij
      for (int t = 0; t <= d; ++t) {
        T s = T(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          T yv = t < d ? a.X[(tl.o + tl.colc(r)) * a.xs + t] : T(1);
          s = fma(p[r], yv, s);
        }
        s = sum_row<MP>(s);
        if (lane < MP) accx[lane * (d + 1) + t] += (double)s;
      }
    }
  }
  const int nrec = MP * (d + 1);
  if (mode == kRho) {
    accf = sum_wave(accf);
    __shared__ double s_r[4];
    if (lane == 0) s_r[wave] = accf;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int q = 0; q < nwaves; ++q) s += s_r[q];
      a.part[(int64_t)ch * a.ps] = s;
    }
  } else if (mode == kA0 || mode == kAP) {
    write_w_record<MP>(accw, accf, a.part, a.ps, ch);
  } else if (xnum) {
    __syncthreads();
    for (int q = threadIdx.x; q < nrec; q += blockDim.x) {
      double s = 0.0;
      for (int wv = 0; wv < nwaves; ++wv) s += s_dyn[(int64_t)wv * nrec + q];
      a.partx[(int64_t)ch * nrec + q] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Per-cluster finalisation: sums the chunk records of a cluster in chunk
// order.  One workgroup per cluster.
// ---------------------------------------------------------------------------
template <int MP>
__global__ void __launch_bounds__(256) k_fin(FinArgs f, int mode) {
  extern __shared__ double s_x[];  // kFinX: MP*(d+1) sums
  __shared__ double s_red[256];
  __shared__ double s_out[MP + 1];
  __shared__ double s_v[MP];
  const int c = blockIdx.x;
  const int2 ct = f.ctab[c];
  if (ct.y == 0) return;  // empty cluster: keep everything
  const int tid = threadIdx.x, nt = blockDim.x;
  if (mode == kFinX) {
    const int nrec = MP * (f.d + 1);
    for (int q = tid; q < nrec; q += nt) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int u = 0;
      for (; u + 3 < ct.y; u += 4) {
        s0 += f.partx[(int64_t)(ct.x + u) * nrec + q];
        s1 += f.partx[(int64_t)(ct.x + u + 1) * nrec + q];
        s2 += f.partx[(int64_t)(ct.x + u + 2) * nrec + q];
        s3 += f.partx[(int64_t)(ct.x + u + 3) * nrec + q];
      }
      for (; u < ct.y; ++u) s0 += f.partx[(int64_t)(ct.x + u) * nrec + q];
      s_x[q] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    for (int q = tid; q < MP * f.d; q += nt) {
      const int ii = q / f.d, t = q % f.d;
      const double den = s_x[ii * (f.d + 1) + f.d];
      if (ii < f.m && den > 1e-300)
        f.xc[((int64_t)c * MP + ii) * f.d + t] = s_x[ii * (f.d + 1) + t] / den;
    }
    return;
  }
  const int ncol = mode == kFinRho ? 1 : MP + 1;
  const int groups = nt / ncol;
  const int col = tid % ncol, grp = tid / ncol;
  if (grp < groups) {
    double s = 0.0;
    for (int q = grp; q < ct.y; q += groups)
      s += f.part[(int64_t)(ct.x + q) * f.ps + col];
    s_red[grp * ncol + col] = s;
  }
  __syncthreads();
  if (tid < ncol) {
    double t = 0.0;
    for (int gI = 0; gI < groups; ++gI) t += s_red[gI * ncol + tid];
    s_out[tid] = t;
  }
  __syncthreads();
  if (mode == kFinRho) {
    if (tid == 0) f.rho[c] = f.rho0 * s_out[0] * f.cinv[c];
    return;
  }
  const double ni = f.ninv[c];
  __shared__ double s_vs;
  if (tid < MP) {
    double t = tid < f.m ? s_out[tid] * ni : 0.0;
    s_v[tid] = f.rule == 2 ? t * t : t;
  }
  __syncthreads();
  if (tid == 0) {
    double vs = 0.0;
    for (int q = 0; q < MP; ++q) vs += s_v[q];
    s_vs = vs;
    if (f.trace) f.trace[c] = s_out[MP] * ni;
  }
  __syncthreads();
  if (tid < MP) f.w_out[c * MP + tid] = s_v[tid] / s_vs;
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
  int m, d, xs, K, iters;
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
  const bool rowok = i < a.m;
  const T eps = (T)a.eps;
  T wk[R];
  bool v[R];
  int jc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = g + CPS * r;
    v[r] = rowok && j < mk;
    jc[r] = j < mk ? j : mk - 1;
    wk[r] = a.W[o + jc[r]];
    wk[r] = v[r] ? wk[r] : T(0);
  }
  double bestv = 0.0;
  int bestc = -1;
  for (int c = 0; c < a.K; ++c) {
    const double* xrow = a.xc + ((int64_t)c * MP + (rowok ? i : 0)) * a.d;
    T cs[R], p1[R], p2[R], l[R];
    T csum = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T cv = cost_generic<T>(xrow, a.X + (o + jc[r]) * a.xs, a.d);
      cs[r] = v[r] ? cv : T(0);
      csum += cs[r];
    }
    const double tot = sum_wave((double)csum);
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
        T av = v[r] ? p2[r] * dexp(-(cs[r] + l[r]) * irho) + eps : T(0);
        T s = sum_col<MP>(av);
        T q = (v[r] && s > T(0)) ? av * (wk[r] * drcp(s)) : T(0);
        p1[r] = q;
        T b = v[r] ? q * dexp(l[r] * irho) + eps : T(0);
        p2[r] = b;
        rr += b;
      }
      rr = sum_row<MP>(rr);
      const T coef = rr > T(0) ? wi * drcp(rr) : T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        T q = p2[r] * coef;
        l[r] = l[r] + rho * (p1[r] - q);
        p2[r] = q;
      }
    }
    T fv = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) fv = fma(cs[r], p1[r], fv);
    const double val = sum_wave((double)fv);
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

// ---------------------------------------------------------------------------
// kernel tables indexed by [log2(MP) - 3][log2(R)]
// ---------------------------------------------------------------------------
template <typename T> struct KernTable {
  using BA = void (*)(Args<T>);
  using AX = void (*)(Args<T>, int);
  using AS = void (*)(AssignArgs<T>);
  BA ba[2][4][6] = {};  // [onfly][mp][r]
  AX aux[4][6] = {};
  AS asg[4][6] = {};
};
using FinFn = void (*)(FinArgs, int);

}  // namespace d2k

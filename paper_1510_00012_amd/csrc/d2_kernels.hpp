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
// bpermute).  The hot kernel reads and writes a tile through buffer
// resources that cover exactly the tile, so lanes outside it read zeros and
// drop their stores without clamps or branches, and all of a tile's loads
// are in flight together (other kernels clamp to an in-bounds element and
// mask).  For d > 4 the support-update sums of a tile run on the matrix
// cores (FP32 MFMA), the tile layout being the A operand.
//
// A workgroup processes one "chunk": a run of instances of one cluster from
// the cluster-sorted work list, and writes double records per chunk
// (weight-consensus sums and objective; support-update numerators).  The
// next launch's workgroups sum their cluster's records in a fixed chunk
// order in a short prologue, so every workgroup of a cluster obtains the
// same bits; no cross-workgroup synchronisation happens inside a kernel and
// runs are bitwise reproducible.  Plan tiles start on 128-byte boundaries.
//
// Support update without an extra pass over the plans: Pi2 = Pi1~ w_i/r_i,
// so x_i = sum_k sum_j Pi2_ij y_j / sum_k sum_j Pi2_ij
//        = (sum_k u_i^(k)) / #{k : r_i^(k) > 0},  u_i^(k) = sum_j Pi1~_ij y_j / r_i
// which phase A has in registers when it builds Pi1~ and r.
//
// Iteration schedule (carried state = Pi1 and Lambda between launches):
//   A0       Pi2^0 (product or cached), Lambda = 0 -> Pi1^1, records of A_0
//   BA (hot) prologue: w^{n+1} (and x after iteration n) from the records of
//            A_n; B_n: Pi2^{n+1}, Lambda^{n+1}; A_{n+1}: Pi1^{n+2}, records
//   BF       last launch: prologue, B_{T-1}, store Pi2 (the warm-start cache)
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>
#include <stdint.h>

namespace d2k {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// arithmetic helpers
// ---------------------------------------------------------------------------
// Exponentials are evaluated as 2^t with t = x * log2(e): the caller folds
// log2(e) into its 1/rho scale, so exp costs one multiply-add plus the
// hardware base-2 exponential (FP32) or exp2 (FP64).
constexpr double kLog2e = 1.4426950408889634074;
__device__ __forceinline__ float dexp2(float t) {
  return __builtin_amdgcn_exp2f(t);
}
__device__ __forceinline__ double dexp2(double t) { return exp2(t); }
__device__ __forceinline__ float drcp(float x) {
  return __builtin_amdgcn_rcpf(x);
}
__device__ __forceinline__ double drcp(double x) { return 1.0 / x; }
// reciprocal of a column / row sum; an all-inactive column has sum 0 and
// only zero numerators, so clamping keeps 0 * (1/sum) finite
template <typename T> __device__ __forceinline__ T rcp_sum(T s) {
  return drcp(s > T(1e-30) ? s : T(1e-30));
}
__device__ __forceinline__ float dsqrt(float v) { return sqrtf(v); }
__device__ __forceinline__ double dsqrt(double v) { return sqrt(v); }

// ---------------------------------------------------------------------------
// lane exchange: DPP within 16-lane rows, ds_swizzle across 16, bpermute 32
// ---------------------------------------------------------------------------
// (bound_ctrl set: every exchange below reads an in-row lane of a fully
// active wavefront, and it lets the compiler fold the move into the add)
template <int CTRL> __device__ __forceinline__ float xdpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL,
                                                    0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double xdpp(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF,
                                    false);
  int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL> __device__ __forceinline__ float xdpp_raw(float v) {
  return __int_as_float(
      __builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double xdpp_raw(double v) {
  return xdpp<CTRL>(v);
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
// sum_col of NS independent values, stage by stage so that the exchanges of
// different slots interleave (no idle cycles between dependent DPP adds)
template <int MP, int NS, typename T>
__device__ __forceinline__ void sum_col_n(T (&v)[NS]) {
  if constexpr (MP >= 2) {
#pragma unroll
    for (int r = 0; r < NS; ++r) v[r] += xdpp<0xB1>(v[r]);
  }
  if constexpr (MP >= 4) {
#pragma unroll
    for (int r = 0; r < NS; ++r) v[r] += xdpp<0x4E>(v[r]);
  }
  if constexpr (MP >= 8) {
#pragma unroll
    for (int r = 0; r < NS; ++r) v[r] += xdpp<0x141>(v[r]);
  }
  if constexpr (MP >= 16) {
#pragma unroll
    for (int r = 0; r < NS; ++r) v[r] += xdpp<0x140>(v[r]);
  }
  if constexpr (MP >= 32) {
#pragma unroll
    for (int r = 0; r < NS; ++r) v[r] += xswz16(v[r]);
  }
  if constexpr (MP >= 64) {
#pragma unroll
    for (int r = 0; r < NS; ++r) v[r] += x32(v[r]);
  }
}

// Column sums by reduce-scatter (column groups of MP >= 8 lanes).  A
// lane's NS slots go in chunks of C = 8, 4, 2 or 1 slots, and register t of
// a chunk holds slot t ^ mask(lane & 3).  An exchange with the quad lane of
// the other parity adds, for the half of the chunk a lane keeps, the
// partner's values of the same slots; an exchange with the other pair of
// the quad halves the kept part again.  Each quad lane so ends with the
// quad sums of max(1, C/4) slots, which are then summed over the quads of
// the column group (row rotations by 8 and by 4, then across rows; for
// MP = 8 one swizzle with lane ^ 4).  The
// mask places what a lane sends at the register index its partner keeps,
// so the exchanges need no selects.  Each sum is formed in one lane per
// quad and is bitwise the same in every quad of the group: the exchanges
// pair lanes symmetrically (xor 1, 2, 8 or 4), and the rotation by 4 adds
// two values that are already equal across lanes 8 apart.
constexpr int rs_chunk_size(int left) {
  return left >= 8 ? 8 : (left >= 4 ? 4 : (left >= 2 ? 2 : 1));
}
template <int C> struct RsChunk {
  static constexpr int kept = C >= 8 ? 2 : 1;
  static constexpr int mask(int ql) {
    return C >= 4 ? (ql & 1) * (C / 2) + ((ql >> 1) & 1) * (C / 4)
                  : (C == 2 ? (ql & 1) : 0);
  }
  // quad_perm control by which each lane reads, for its chunk register t,
  // the value of that register's slot from the quad lane holding its sum
  // (at that lane's register t & (kept - 1))
  static constexpr int bcast(int t) {
    int ctrl = 0;
    for (int j = 0; j < 4; ++j) {
      const int want = (t ^ mask(j)) & ~(kept - 1);
      int o = j;
      if (C > 1)
        for (int ql = 3; ql >= 0; --ql)
          if (mask(ql) == want && (C != 2 || ((ql ^ j) & 2) == 0)) o = ql;
      ctrl |= o << (2 * j);
    }
    return ctrl;
  }
};
// kept registers of the chunks before slot c0 (c0 a chunk start; c0 = NS:
// all of them)
constexpr int rs_kept_before(int c0) {
  int n = 0;
  for (int c = 0; c < c0;) {
    const int C = rs_chunk_size(c0 - c);
    n += C >= 8 ? 2 : 1;
    c += C;
  }
  return n;
}
// f.template operator()<C0, C>() for every chunk, in slot order
template <int NS, int C0 = 0, typename F>
__device__ __forceinline__ void rs_chunks(F&& f) {
  if constexpr (C0 < NS) {
    constexpr int C = rs_chunk_size(NS - C0);
    f.template operator()<C0, C>();
    rs_chunks<NS, C0 + C>(f);
  }
}
// Per-lane select written as one v_cndmask_b32 (lanes whose bit in m is set
// take b): as plain code, a select between elements of an array is folded
// into a lane-dependent index into the array, which then lives in scratch.
__device__ __forceinline__ float lane_sel(float a, float b,
                                          unsigned long long m) {
  float r;
  asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(m));
  return r;
}
__device__ __forceinline__ double lane_sel(double a, double b,
                                           unsigned long long m) {
  const long long ab = __double_as_longlong(a), bb = __double_as_longlong(b);
  const float lo = lane_sel(__int_as_float((int)ab), __int_as_float((int)bb), m);
  const float hi = lane_sel(__int_as_float((int)(ab >> 32)),
                            __int_as_float((int)(bb >> 32)), m);
  return __longlong_as_double(((long long)__float_as_int(hi) << 32) |
                              (unsigned int)__float_as_int(lo));
}
// exchange with lane ^ 4 (ds_swizzle, bit mode)
__device__ __forceinline__ float xswz4(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x101F));
}
__device__ __forceinline__ double xswz4(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffLL), 0x101F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x101F);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Slot value x[C0 + (t ^ mask(lane & 3))] of chunk register t, from a
// lane's values in slot order (Q0: those of the first lane of its quad).
template <int C0, int C, int t, bool Q0 = false, int NS, typename T>
__device__ __forceinline__ T rs_pick(const T (&x)[NS]) {
  constexpr unsigned long long kOdd = 0xAAAAAAAAAAAAAAAAull;   // lane & 1
  constexpr unsigned long long kPair = 0xCCCCCCCCCCCCCCCCull;  // lane & 2
  auto val = [&](int r) { return Q0 ? xdpp<0x00>(x[r]) : x[r]; };
  if constexpr (C == 1) {
    return val(C0 + t);
  } else if constexpr (C == 2) {
    return lane_sel(val(C0 + t), val(C0 + (t ^ 1)), kOdd);
  } else {
    const T lo = lane_sel(val(C0 + t), val(C0 + (t ^ (C / 2))), kOdd);
    const T hi = lane_sel(val(C0 + (t ^ (C / 4))),
                          val(C0 + (t ^ (C / 4) ^ (C / 2))), kOdd);
    return lane_sel(lo, hi, kPair);
  }
}
// Sums over the column group of the chunk's C values s[0, C): on return
// s[0, kept) hold the sums of the slots of this lane's first kept
// registers.
template <int MP, int C, typename T>
__device__ __forceinline__ void rs_sum(T (&s)[C]) {
  static_assert(MP >= 8, "reduce-scatter needs two quads per column");
  constexpr int K = RsChunk<C>::kept;
  if constexpr (C >= 2) {
#pragma unroll
    for (int k = 0; k < C / 2; ++k) s[k] += xdpp<0xB1>(s[k + C / 2]);
  }
  if constexpr (C >= 4) {
#pragma unroll
    for (int k = 0; k < C / 4; ++k) s[k] += xdpp<0x4E>(s[k + C / 4]);
  }
  if constexpr (C == 1) s[0] += xdpp<0xB1>(s[0]);
  if constexpr (C <= 2) s[0] += xdpp<0x4E>(s[0]);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if constexpr (MP == 8) {
      // lane ^ 4 (a rotation by 4 would leave the 8-lane column group)
      s[k] += xswz4(s[k]);
    } else {
      s[k] += xdpp<0x128>(s[k]);  // row_ror:8 (lane ^ 8)
      s[k] += xdpp<0x124>(s[k]);  // row_ror:4
    }
    if constexpr (MP >= 32) s[k] += xswz16(s[k]);
    if constexpr (MP >= 64) s[k] += x32(s[k]);
  }
}
// value of chunk register t's slot from the quad lane that holds it
template <int C, int T_, typename T>
__device__ __forceinline__ T rs_get(const T (&f)[RsChunk<C>::kept]) {
  constexpr int ctrl = RsChunk<C>::bcast(T_);
  const T v = f[T_ & (RsChunk<C>::kept - 1)];
  if constexpr (ctrl == 0xE4) return v;  // quad_perm [0,1,2,3]
  else return xdpp<ctrl>(v);
}

// support point of a column for the on-the-fly cost (d <= 4, stride 4)
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Kernel modes of the auxiliary kernel (uniform runtime switch).
enum Mode : int {
  kRho = 0,  // cost at the initial support (stored if cached): cost sums
  kA0 = 1,   // phase A from Pi2^0 (product / cached), Lambda := 0
  kBF = 4,   // phase B of the last iteration: store Pi2 and Lambda
  kXO = 5,   // support records from the stored Pi2 only
};
// Finalisation modes (per-cluster launches).
enum FinMode : int { kFinRho = 1, kFinX = 2, kFinRes = 3 };

struct Chunk {
  int32_t cluster, begin, end, pad;
};

template <typename T> struct Args {
  const int64_t* off;   // N+1 instance offsets
  const int64_t* pofs;  // N plan tile offsets (elements, 128-byte aligned)
  const T* X;           // n x xs supports (xs = 4 when d <= 4, zero padded)
  const T* W;           // n weights
  const int32_t* work;  // instance ids sorted by cluster
  const Chunk* chunks;  // per workgroup
  const int* nch;       // number of chunks (the grid may be larger)
  const int32_t* blist; // hot kernel: chunk ids of its slot bucket, or null
  const int* bcnt;      // per bucket: number of chunk ids
  int bidx, boff;       // this launch's bucket and its offset in blist
  const int2* ctab;     // per cluster {first chunk, number of chunks}
  const double* ninv;   // per cluster 1 / N_c
  T* P1;
  T* P2;
  T* L;
  T* Cc;                // cost cache (plan layout) or nullptr (on the fly)
  const uint8_t* warm;  // per instance: start from cached Pi2
  double* xc;           // K x MP x d centroid support
  double* wc;           // K x MP centroid weights (initial / published)
  const double* rho;    // K
  const double* part_in;  // weight records of the previous phase A
  double* part;           // weight records written by this launch, stride ps
  const double* xin;      // support records of the previous phase A or null
  double* xout;           // support records of this launch's phase A or null
  double* trace;          // K objective values of the previous phase A
  double* rtrace;         // K residuals of the previous launch's phase B
  int rlast;              // kBF: write this launch's residual records
  double eps;
  int m, d, xs, rule, ps;
  int recost;             // cached cost: recompute from xc and store
  int xstage;             // centroid support staged in LDS for cost work
  // Symbolic supports (Sec. 5): when dsym is set, support points are
  // symbols and the cost of centroid row i against support point j is
  // dsym[csym[c * MP + i] * S + isym[j]] (S x S table, device dtype); the
  // rho pass gathers it into the cost cache, which every later launch
  // reads.
  const T* dsym;
  const int32_t* isym;    // n instance symbols
  const int32_t* csym;    // K x MP centroid symbols
  int S;
};

struct FinArgs {
  const int2* ctab;     // per cluster {first chunk, number of chunks}
  const double* ninv;   // per cluster 1 / N_c
  double* rtr;          // kFinRes: K residuals of the last phase B
  const double* cinv;   // per cluster 1 / (m * sum_k m_k)
  const double* part;
  const double* xrec;
  double* rho;          // K
  double* xc;           // K x MP x d
  double rho0;
  int m, d, ps;
};

// fixed-order strided sum of double records, loads issued 8 at a time
__device__ __forceinline__ double sum_strided(const double* base, int64_t st,
                                              int q0, int qn, int step) {
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int q = q0;
  for (; q + 7 * step < qn; q += 8 * step) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += base[(int64_t)(q + u * step) * st];
  }
  for (int u = 0; q < qn; q += step, ++u) acc[u] += base[(int64_t)q * st];
  return ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
         ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// Sums columns [0, ncol) of a cluster's chunk records (stride `st`) into
// out[] (LDS) in a fixed order; every workgroup that calls it with the same
// arguments obtains the same bits.
__device__ __forceinline__ void sum_cluster_records(const double* base,
                                                    int64_t st, int nch,
                                                    int ncol, double* red,
                                                    double* out) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int groups = nt / ncol;
  if (groups >= 2) {
    const int col = tid % ncol, grp = tid / ncol;
    if (grp < groups)
      red[grp * ncol + col] = sum_strided(base + col, st, grp, nch, groups);
    __syncthreads();
    for (int q = tid; q < ncol; q += nt) {
      double t = 0.0;
      for (int gI = 0; gI < groups; ++gI) t += red[gI * ncol + q];
      out[q] = t;
    }
  } else {
    for (int q = tid; q < ncol; q += nt)
      out[q] = sum_strided(base + q, st, 0, nch, 1);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------
// Per-wavefront scalars are made explicitly uniform (readfirstlane) so that
// per-instance control flow is scalar and the instance's offsets come from
// scalar loads.
__device__ __forceinline__ int uni(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

template <typename T, int MP> struct Tile {
  static constexpr int CPS = kWave / MP;
  int64_t o, base;
  int mk, nsl, i, g, ic;
  bool rowok;
  __device__ __forceinline__ void setup(const int64_t* off,
                                        const int64_t* pofs, int m, int k) {
    set(m, off[k], off[k + 1], pofs ? pofs[k] : 0);
  }
  // from instance offsets o0 .. o1 and plan offset pb (all uniform)
  __device__ __forceinline__ void set(int m, int64_t o0, int64_t o1,
                                      int64_t pb) {
    const int lane = threadIdx.x & (kWave - 1);
    i = lane % MP;
    g = lane / MP;
    rowok = i < m;
    ic = rowok ? i : 0;
    o = o0;
    mk = (int)(o1 - o0);
    nsl = (mk + CPS - 1) / CPS;
    base = pb;
  }
  __device__ __forceinline__ int col(int r) const { return g + CPS * r; }
  __device__ __forceinline__ bool valid(int r) const {
    return rowok && col(r) < mk;
  }
  // in-bounds column for every lane (inactive lanes clamp to the last)
  __device__ __forceinline__ int colc(int r) const {
    int j = col(r);
    return j < mk ? j : mk - 1;
  }
  __device__ __forceinline__ int64_t eidx(int r, int m) const {
    return base + (int64_t)colc(r) * m + ic;
  }
  // A copy whose column group the compiler cannot see through: the
  // per-slot columns, masks and addresses derived from it are formed again
  // where they are used instead of being hoisted out of a loop and held in
  // registers across it.
  __device__ __forceinline__ Tile fresh() const {
    Tile t = *this;
    asm volatile("" : "+v"(t.g));
    return t;
  }
};

// Calls f.template operator()<NS>() with the smallest specialised slot
// count NS >= nsl (exact up to 8, then 12, 16, 24, 32; NS <= R).  Each
// specialisation is straight-line code over exactly NS register slots.
template <int R, typename F>
__device__ __forceinline__ void with_slots(int nsl, F&& f) {
#define D2_NS(NSV)                           \
  if constexpr (NSV <= R) {                  \
    if (nsl <= NSV) {                        \
      f.template operator()<NSV>();          \
      return;                                \
    }                                        \
  }
  D2_NS(1) D2_NS(2) D2_NS(3) D2_NS(4) D2_NS(5) D2_NS(6) D2_NS(7) D2_NS(8)
  D2_NS(12) D2_NS(16) D2_NS(24) D2_NS(32)
#undef D2_NS
}

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

// ---------------------------------------------------------------------------
// prologue: cluster quantities from the previous launch's records
// ---------------------------------------------------------------------------
// Weights w^{n+1} (R1: normalised mean of w~^(k); R2: normalised square of
// the mean of sqrt(w~^(k))).  The cluster's first chunk also publishes w and
// the objective of the phase A that wrote the records.
template <typename T, int MP>
__device__ __forceinline__ void cluster_weights(const Args<T>& a, int c,
                                                int2 ct, bool publish,
                                                double* s_w) {
  __shared__ double s_red[256];
  __shared__ double s_out[MP + 2];
  __shared__ double s_vs;
  const int tid = threadIdx.x, nt = blockDim.x;
  sum_cluster_records(a.part_in + (int64_t)ct.x * a.ps, a.ps, ct.y, MP + 2,
                      s_red, s_out);
  const double ni = a.ninv[c];
  for (int q = tid; q < MP; q += nt) {
    double t = q < a.m ? s_out[q] * ni : 0.0;
    s_w[q] = a.rule == 2 ? t * t : t;
  }
  __syncthreads();
  if (tid == 0) {
    double vs = 0.0;
    for (int q = 0; q < MP; ++q) vs += s_w[q];
    s_vs = vs;
    if (publish && a.trace) a.trace[c] = s_out[MP] * ni;
    if (publish && a.rtrace) a.rtrace[c] = s_out[MP + 1] * ni;
  }
  __syncthreads();
  for (int q = tid; q < MP; q += nt) {
    s_w[q] = s_w[q] / s_vs;
    if (publish) a.wc[c * MP + q] = s_w[q];
  }
  __syncthreads();
}

// Updated support (d <= 4) from support records: x_i = sum u / sum den;
// a row no member carries mass on keeps its point.  Result in s_x[MP][4].
template <typename T, int MP>
__device__ __forceinline__ void cluster_support(const Args<T>& a, int c,
                                                int2 ct, bool publish,
                                                double* s_x) {
  __shared__ double s_red[256];
  __shared__ double s_out[MP * 5];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int d = a.d, ncol = MP * (d + 1);
  sum_cluster_records(a.xin + (int64_t)ct.x * ncol, ncol, ct.y, ncol, s_red,
                      s_out);
  for (int q = tid; q < MP * 4; q += nt) {
    const int ii = q / 4, t = q % 4;
    double v = 0.0;
    if (ii < a.m && t < d) {
      const double den = s_out[ii * (d + 1) + d];
      const int64_t xi = ((int64_t)c * MP + ii) * d + t;
      v = den > 0.0 ? s_out[ii * (d + 1) + t] / den : a.xc[xi];
    }
    s_x[q] = v;
  }
  __syncthreads();
  if (publish)
    for (int q = tid; q < MP * d; q += nt) {
      const int ii = q / d, t = q % d;
      if (ii < a.m) a.xc[((int64_t)c * MP + ii) * d + t] = s_x[ii * 4 + t];
    }
}

// ---------------------------------------------------------------------------
// phases of one tile
// ---------------------------------------------------------------------------
// Scales of one cluster: rho, a2 = log2(e)/rho.  Inactive lanes carry
// zero plan, zero weight and a zero eps (el), so every product, column and
// row sum below is exact without per-lane selects.

// Phase B: Pi1~ = Pi1 exp(Lambda/rho) + eps, row sums r_i,
// Pi2 = Pi1~ w_i / r_i, Lambda += rho (Pi1 - Pi2).  In: p = Pi1; out: p = Pi2.
template <typename T, int MP, int NS>
__device__ __forceinline__ void phase_b(const T (&el)[NS], T (&p)[NS],
                                        T (&l)[NS], T wi, T rho, T a2,
                                        T& res) {
  T bv[NS];
  T rs = T(0);
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    bv[r] = fma(p[r], dexp2(l[r] * a2), el[r]);
    rs += bv[r];
  }
  rs = sum_row<MP>(rs);
  const T coef = wi * rcp_sum(rs);
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    T p2 = bv[r] * coef;
    const T dp = p[r] - p2;
    l[r] = fma(rho, dp, l[r]);
    res += fabs(dp);
    p[r] = p2;
  }
}

// Phase A: in p = Pi2, l = Lambda, cost cs, instance weights wk; out
// p = Pi1 (column KL projection) and, with KEEPB, b = Pi1~.  Returns the row
// sum r_i of Pi1~ in rr and adds <C, Pi1> to f.  The column sums are formed
// for a chunk of slots at a time (same adds in the same order per column).
template <typename T, int MP, int NS, bool KEEPB>
__device__ __forceinline__ void phase_a(const T (&el)[NS], T (&p)[NS],
                                        const T (&l)[NS], const T (&cs)[NS],
                                        const T (&wk)[NS], T a2, T (&b)[NS],
                                        T& rr, T& f) {
  constexpr int CH = NS <= 8 ? NS : (NS % 8 == 0 ? 8 : 4);
  rr = T(0);
#pragma unroll
  for (int r0 = 0; r0 < NS; r0 += CH) {
    T av[CH], s[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int r = r0 + u;
      av[u] = fma(p[r], dexp2(-(cs[r] + l[r]) * a2), el[r]);
      s[u] = av[u];
    }
    sum_col_n<MP, CH>(s);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int r = r0 + u;
      T p1 = av[u] * (wk[r] * rcp_sum(s[u]));
      f = fma(cs[r], p1, f);
      const T bt = fma(p1, dexp2(l[r] * a2), el[r]);
      if constexpr (KEEPB) b[r] = bt;
      rr += bt;
      p[r] = p1;
    }
  }
  rr = sum_row<MP>(rr);
}

// weight-consensus contribution w~_i (R1) or sqrt(w~_i) (R2) of one tile
template <typename T, int MP>
__device__ __forceinline__ double consensus_term(T rr, bool rowok, int rule) {
  T tot = sum_col<MP>(rowok ? rr : T(0));
  T wt = rowok ? rr * rcp_sum(tot) : T(0);
  // R2 takes the square root (hardware sqrt for FP32, about 1 ulp: a
  // select over the IEEE-rounded expansion would run on every tile)
  if constexpr (sizeof(T) == 4)
    return (double)(rule == 2 ? __builtin_amdgcn_sqrtf(wt) : wt);
  else
    return (double)(rule == 2 ? dsqrt(wt) : wt);
}

// chunk record: per-row weight sums (lanes < MP of each wave) + objective
template <int MP>
__device__ __forceinline__ void write_w_record(double accw, double accf,
                                               double accr, double* part,
                                               int ps, int ch) {
  __shared__ double s_w[4][MP + 2];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  accf = sum_wave(accf);
  accr = sum_wave(accr);
  if (lane < MP) s_w[wave][lane] = accw;
  if (lane == 0) {
    s_w[wave][MP] = accf;
    s_w[wave][MP + 1] = accr;
  }
  __syncthreads();
  if (threadIdx.x <= MP + 1) {
    double s = 0.0;
    for (int q = 0; q < nwaves; ++q) s += s_w[q][threadIdx.x];
    part[(int64_t)ch * ps + threadIdx.x] = s;
  }
}

// Support record of one tile: u_i,t = sum_j b_ij y_j,t / r_i for t < d and
// the indicator r_i > 0, added (lanes < MP) to acc[MP][d+1] in LDS.
template <typename T, int MP, int NS>
__device__ __forceinline__ void add_support_terms(const Args<T>& a,
                                                  const Tile<T, MP>& tl,
                                                  const T (&b)[NS], T rr,
                                                  double* acc) {
  using V4 = typename Vec4<T>::type;
  const int lane = threadIdx.x & (kWave - 1);
  const int d = a.d;
  const T ir = rcp_sum(rr);
  const V4* yv[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r)
    yv[r] = reinterpret_cast<const V4*>(a.X + (tl.o + tl.colc(r)) * a.xs);
  // four coordinates per step (rows of X are xs = roundup(d, 4) long)
  for (int q = 0; q < (a.xs >> 2); ++q) {
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const V4 y = yv[r][q];
      s0 = fma(b[r], y.x, s0);
      s1 = fma(b[r], y.y, s1);
      s2 = fma(b[r], y.z, s2);
      s3 = fma(b[r], y.w, s3);
    }
    s0 = sum_row<MP>(s0);
    s1 = sum_row<MP>(s1);
    s2 = sum_row<MP>(s2);
    s3 = sum_row<MP>(s3);
    if (lane < MP) {
      double* ap = acc + lane * (d + 1) + 4 * q;
      const int t = 4 * q;
      ap[0] += (double)(s0 * ir);
      if (t + 1 < d) ap[1] += (double)(s1 * ir);
      if (t + 2 < d) ap[2] += (double)(s2 * ir);
      if (t + 3 < d) ap[3] += (double)(s3 * ir);
    }
  }
  if (lane < MP && rr > T(0)) acc[lane * (d + 1) + d] += 1.0;
}

// The same support record for d <= 4 (stride 4) accumulated in registers:
// each lane adds its own partial sum_j b_ij y_j,t / r_i (its columns only)
// and the indicator r_i > 0 in FP64 across the wavefront's tiles; the sums
// over the lanes of a row are formed once, by flush_support4.
struct XAcc4 {
  double u[4] = {0.0, 0.0, 0.0, 0.0};
  double n = 0.0;
};
template <typename T, int MP, int NS>
__device__ __forceinline__ void add_support_terms4(const Args<T>& a,
                                                   const Tile<T, MP>& tl,
                                                   const T (&b)[NS], T rr,
                                                   XAcc4& xa) {
  using V4 = typename Vec4<T>::type;
  const T ir = rcp_sum(rr);
  T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const V4 y = reinterpret_cast<const V4*>(a.X + (tl.o + tl.colc(r)) * 4)[0];
    s0 = fma(b[r], y.x, s0);
    s1 = fma(b[r], y.y, s1);
    s2 = fma(b[r], y.z, s2);
    s3 = fma(b[r], y.w, s3);
  }
  xa.u[0] += (double)(s0 * ir);
  xa.u[1] += (double)(s1 * ir);
  xa.u[2] += (double)(s2 * ir);
  xa.u[3] += (double)(s3 * ir);
  if (tl.g == 0 && rr > T(0)) xa.n += 1.0;
}
// Row sums of the register accumulators into the wavefront's record
// acc[MP][d+1] (lanes < MP hold row lane).
template <int MP>
__device__ __forceinline__ void flush_support4(const XAcc4& xa, int d,
                                               double* acc) {
  const int lane = threadIdx.x & (kWave - 1);
  double u[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) u[t] = sum_row<MP>(xa.u[t]);
  if (lane < MP) {
    double* ap = acc + lane * (d + 1);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < d) ap[t] += u[t];
    ap[d] += xa.n;
  }
}

// The cluster's support rows in LDS as T, row stride xs + 4 (zero padded
// past d), for the cost work of a launch (one cluster per workgroup).
template <typename T, int MP>
__device__ __forceinline__ void stage_support(const Args<T>& a, int c, T* xl) {
  const int xsl = a.xs + 4, d = a.d;
  for (int q = threadIdx.x; q < MP * xsl; q += blockDim.x) {
    const int i = q / xsl, t = q % xsl;
    xl[q] = t < d ? (T)a.xc[((int64_t)c * MP + i) * d + t] : T(0);
  }
  __syncthreads();
}

// C_ij = sum_t (x_it - y_jt)^2 for the lane's row and every slot, with x
// from the LDS stage and y as 4-wide loads (the same sequential sum over t
// as cost_generic; the zero padding adds exact zeros).
template <typename T, int MP, int NS>
__device__ __forceinline__ void cost_tile(const Args<T>& a,
                                          const Tile<T, MP>& tl, const T* xl,
                                          T (&cs)[NS]) {
  using V4 = typename Vec4<T>::type;
  const V4* xv = reinterpret_cast<const V4*>(xl + tl.ic * (a.xs + 4));
  const V4* yv[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    yv[r] = reinterpret_cast<const V4*>(a.X + (tl.o + tl.colc(r)) * a.xs);
    cs[r] = T(0);
  }
  for (int q = 0; q < (a.xs >> 2); ++q) {
    const V4 x = xv[q];
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const V4 y = yv[r][q];
      T df = x.x - y.x;
      cs[r] = fma(df, df, cs[r]);
      df = x.y - y.y;
      cs[r] = fma(df, df, cs[r]);
      df = x.z - y.z;
      cs[r] = fma(df, df, cs[r]);
      df = x.w - y.w;
      cs[r] = fma(df, df, cs[r]);
    }
  }
}

// Sum the per-wave support accumulators into this chunk's record.
__device__ __forceinline__ void write_x_record(const double* acc, int nrec,
                                               double* xout, int ch) {
  const int nwaves = blockDim.x / kWave;
  __syncthreads();
  for (int q = threadIdx.x; q < nrec; q += blockDim.x) {
    double s = 0.0;
    for (int wv = 0; wv < nwaves; ++wv) s += acc[(int64_t)wv * nrec + q];
    xout[(int64_t)ch * nrec + q] = s;
  }
}

// ---------------------------------------------------------------------------
// Hot kernel: one launch per B-ADMM iteration (phase B of n, phase A of n+1)
// ---------------------------------------------------------------------------
// Raw buffer access (range-checked by the hardware: an offset at or past
// the resource's size reads 0 and drops a store).  A resource covers one
// tile, so lanes outside the tile need no clamping, masking or branches.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // 32-bit data format, raw access
constexpr uint32_t kOob = 0x80000000u;  // an offset past every tile

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0,
                                           (int)bytes, kRsrcWord3);
}
// 32-byte loads (double4) as two 16-byte loads
template <typename T>
__device__ __forceinline__ T bload_wide(Rsrc r, uint32_t o) {
  const double2 lo = __builtin_bit_cast(
      double2, __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0));
  const double2 hi = __builtin_bit_cast(
      double2, __builtin_amdgcn_raw_buffer_load_b128(r, o + 16u, 0, 0));
  return make_double4(lo.x, lo.y, hi.x, hi.y);
}

// Cache policy bits of buffer instructions: 0 = the default policy,
// kCpolStream = non-temporal (the line is not kept for reuse).  The hot
// kernel streams its plan state (Pi1, Lambda, cost cache) this way when the
// state is far larger than the last-level cache, so that it does not
// displace what is reused (supports, weights, records).
constexpr int kCpolStream = 2;
template <typename T, int CP = 0>
__device__ __forceinline__ T bload(Rsrc r, uint32_t o) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, CP));
  else if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, CP));
  else if constexpr (sizeof(T) == 16)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, CP));
  else
    return bload_wide<T>(r, o);
}
template <int CP = 0>
__device__ __forceinline__ void bstore(float v, Rsrc r, uint32_t o) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, o, 0, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bstore(double v, Rsrc r, uint32_t o) {
  __builtin_amdgcn_raw_buffer_store_b64(
      __builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v), r, o,
      0, CP);
}

// Support-update sums on the matrix cores (FP32 MFMA, d <= 64, MP = 32 or
// 16, cost cached): u_i = sum_j Pi1~_ij y_j / r_i for all rows of a tile
// is the product (MP x m_k) . (m_k x d).  The register layout of the tile
// is already the A operand: lane l holds row l % MP of column
// (l / MP) + (64 / MP) r in slot r, i.e. A[i][k] of a K = 64 / MP step.
// The B operand is each lane's own column's coordinates, so one slot is one
// MFMA per 32 (or 16) coordinates.  The tile's sums are added to the
// wavefront's FP64 accumulators in LDS.
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaMaxD = 64;
constexpr int kVarNone = 0, kVarPlain = 3;

// Per-wavefront FP32 accumulators of the support sums (MFMA layout) and of
// the row indicators, added to the wavefront's FP64 LDS record once after
// its last tile.
template <int MP> struct SupAcc {
  static constexpr int NT = kMfmaMaxD / MP;
  static constexpr int NV = MP == 32 ? 16 : 4;
  using V = typename std::conditional<MP == 32, f32x16, f32x4>::type;
  V s[NT];
  float den;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < NV; ++v) s[q][v] = 0.0f;
    den = 0.0f;
  }
  __device__ __forceinline__ void flush(int d, double* acc) const {
    const int lane = threadIdx.x & (kWave - 1);
    const int tn = lane % MP;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int t = q * MP + tn;
      if (q * MP < d && t < d) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int i = MP == 32 ? 8 * (v / 4) + 4 * (lane / 32) + (v % 4)
                                 : 4 * (lane / 16) + v;
          acc[i * (d + 1) + t] += (double)s[q][v];
        }
      }
    }
    if (lane < MP) acc[lane * (d + 1) + d] += (double)den;
  }
};

// The support coordinates of the B operands of slots r0 .. r0 + G - 1 of a
// tile, all loaded before their products (one 256-byte row pair per slot
// and block of coordinates), so that the loads are in flight together
// instead of one per product.
template <int MP, int G>
__device__ __forceinline__ void support_operands(
    const Args<float>& a, const Tile<float, MP>& tl, Rsrc rX, int r0,
    float (&yv)[G][SupAcc<MP>::NT]) {
  constexpr int NT = SupAcc<MP>::NT;
  const int tn = (threadIdx.x & (kWave - 1)) % MP;
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const uint32_t j = (uint32_t)tl.col(r0 + r);
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int t = q * MP + tn;
      yv[r][q] = 0.0f;
      if (q * MP < a.d)
        yv[r][q] = bload<float>(
            rX, t < a.d ? (j * (uint32_t)a.xs + (uint32_t)t) * 4u : kOob);
    }
  }
}

// The products of slots r0 .. r0 + G - 1: u_i += sum_j (Pi1~_ij / r_i) y_j
// (ir = 1 / r_i).
template <int MP, int G, int NS>
__device__ __forceinline__ void support_mfma(
    const Args<float>& a, const float (&b)[NS], int r0, float ir,
    const float (&yv)[G][SupAcc<MP>::NT], SupAcc<MP>& sa) {
  static_assert(MP == 16 || MP == 32, "MFMA support sums: MP 16 or 32");
  constexpr int NT = SupAcc<MP>::NT;
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const float av = b[r0 + r] * ir;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      if (q * MP < a.d) {
        if constexpr (MP == 32)
          sa.s[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, yv[r][q], sa.s[q],
                                                         0, 0, 0);
        else
          sa.s[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, yv[r][q], sa.s[q],
                                                         0, 0, 0);
      }
    }
  }
}

// Cost recomputation on the matrix cores (FP32 MFMA 32x32x2, MP = 32,
// d <= 64) for one 32-column block of a tile: C_ij = |x_i|^2 + |y_j|^2 -
// 2 x_i . y_j as D^T = Y' X^T with Y' = the block's points in a permuted
// order, chosen so that the accumulator layout (lane: row i = l % 32;
// register v: column 8 (v/4) + 4 (l/32) + v % 4 of the block) is the
// tile's slot layout (register v holds slot 16 b + v, column 32 b + l / 32
// + 2 v).  The block's points sit in LDS (yl, rows of xsl floats, staged
// with coalesced loads); the two lane halves h take the coordinates
// [h H, h H + H) (H = xs / 2 rounded up to 4; the row padding is zero), so
// each lane reads its operands as 16-byte LDS words.  xh holds the lane's
// half of x_i, i = l % 32, in registers.  The squared norms of the points
// are summed from the same operands; one more MFMA step with K = (|y|^2,
// 1) x (1, |x|^2) adds the norms.  Negative rounding residue is clamped to
// 0.
__device__ __forceinline__ f32x16 cost_block_mfma(const float* yl, int xsl,
                                                  int H, const float (&xh)[32],
                                                  float xnorm) {
  const int lane = threadIdx.x & (kWave - 1);
  const int n = lane & 31, h = lane >> 5;
  // A operand row n: column g + 8 q + 2 s of the block
  const int jl = ((n >> 2) & 1) + 8 * (n >> 3) + 2 * (n & 3);
  const float* yrow = yl + jl * xsl + h * H;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  float yy = 0.0f;
#pragma unroll
  for (int s4 = 0; s4 < 8; ++s4) {
    if (4 * s4 < H) {
      const f32x4 y4 = *reinterpret_cast<const f32x4*>(yrow + 4 * s4);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        yy = fmaf(y4[u], y4[u], yy);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(-2.0f * y4[u],
                                                   xh[4 * s4 + u], acc, 0, 0,
                                                   0);
      }
    }
  }
  yy += __shfl_xor(yy, 32);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(h == 0 ? yy : 1.0f,
                                             h == 0 ? 1.0f : xnorm, acc, 0, 0,
                                             0);
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = fmaxf(acc[v], 0.0f);
  return acc;
}

template <typename T, int MP, int NS, bool ONFLY, int VAR, int CP>
__device__ __forceinline__ void ba_tile(const Args<T>& a, const Tile<T, MP>& tl,
                                        const T (&xr)[4], const double* xrow,
                                        const T* xl, T wi, T rho,
                                        T a2, T eps, double& accw,
                                        double& accf, double& accr,
                                        double* accx, XAcc4& xa4) {
  using V4 = typename Vec4<T>::type;
  constexpr uint32_t es = sizeof(T);
  // one resource per array over this tile (uniform), 32-bit lane offsets;
  // lanes on rows >= m and columns >= m_k get offsets past the tile
  const uint32_t tb = (uint32_t)(a.m * tl.mk) * es;
  const Rsrc rP = make_rsrc(a.P1 + tl.base, tb);
  const Rsrc rL = make_rsrc(a.L + tl.base, tb);
  const Rsrc rW = make_rsrc(a.W + tl.o, (uint32_t)tl.mk * es);
  const Rsrc rX = make_rsrc(a.X + tl.o * a.xs, (uint32_t)(tl.mk * a.xs) * es);
  Rsrc rC = rP;
  if constexpr (!ONFLY) rC = make_rsrc(a.Cc + tl.base, tb);
  T p[NS], l[NS], cs[NS], wk[NS], el[NS], b[NS];
  uint32_t eo[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const uint32_t j = (uint32_t)tl.col(r);
    eo[r] = tl.rowok ? (j * (uint32_t)a.m + (uint32_t)tl.i) * es : kOob;
    el[r] = tl.valid(r) ? eps : T(0);
    p[r] = bload<T, CP>(rP, eo[r]);
    l[r] = bload<T, CP>(rL, eo[r]);
    wk[r] = bload<T>(rW, j * es);
    if constexpr (ONFLY) {
      cs[r] = cost4<T>(xr, bload<V4>(rX, j * (uint32_t)sizeof(V4)));
    } else if constexpr (VAR == kVarPlain) {
      // plain launches never recompute
      cs[r] = bload<T, CP>(rC, eo[r]);
    } else {
      if (!a.recost)
        cs[r] = bload<T, CP>(rC, eo[r]);
      else if (!xl)
        cs[r] = cost_generic<T>(xrow, a.X + (tl.o + tl.colc(r)) * a.xs, a.d);
    }
  }
  if constexpr (!ONFLY && VAR != kVarPlain) {
    if (a.recost && xl) cost_tile<T, MP, NS>(a, tl, xl, cs);
  }
  T res = T(0);
  phase_b<T, MP, NS>(el, p, l, wi, rho, a2, res);
  accr += (double)res;
  T rr, f = T(0);
  phase_a<T, MP, NS, VAR != kVarPlain>(el, p, l, cs, wk, a2, b, rr, f);
  accw += consensus_term<T, MP>(rr, tl.rowok, a.rule);
  accf += (double)f;
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    bstore<CP>(p[r], rP, eo[r]);
    bstore<CP>(l[r], rL, eo[r]);
  }
  if constexpr (!ONFLY && VAR != kVarPlain) {
    if (a.recost) {
#pragma unroll
      for (int r = 0; r < NS; ++r) bstore<CP>(cs[r], rC, eo[r]);
    }
  }
  if constexpr (VAR != kVarPlain) {
    if (a.xout) {
      if constexpr (ONFLY)
        add_support_terms4<T, MP, NS>(a, tl, b, rr, xa4);
      else
        add_support_terms<T, MP, NS>(a, tl, b, rr, accx);
    }
  }
}

// VAR: kVarPlain kernels leave out the support terms and the cost
// recomputation altogether and serve the launches that do neither (most of
// them), so that the registers of the rarer launches do not lower their
// occupancy.  (FP32 contexts with 32 <= d <= 64 form the support sums and
// the new cost in passes of their own on the matrix cores, k_sup_mfma and
// k_cost_mfma below, beside plain launches.)
template <typename T, int MP, int R, bool ONFLY, int VAR = kVarNone,
          int CP = 0>
__global__ void __launch_bounds__(256) k_iter_ba(Args<T> a) {
  extern __shared__ double s_dyn[];  // [nwaves][MP][d+1] support terms
  __shared__ double s_w[MP];
  __shared__ double s_x[MP * 4];
  int ch = blockIdx.x;
  if (a.blist) {
    if (ch >= a.bcnt[a.bidx]) return;
    ch = uni(a.blist[a.boff + ch]);
  } else if (ch >= *a.nch) {
    return;
  }
  const Chunk cj = a.chunks[ch];
  const int c = cj.cluster;
  const int2 ct = a.ctab[c];
  cluster_weights<T, MP>(a, c, ct, ch == ct.x, s_w);
  const int wave = uni(threadIdx.x / kWave), nwaves = blockDim.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int i = lane % MP;
  const bool rowok = i < a.m;
  const T rho = (T)a.rho[c];
  const T a2 = (T)(kLog2e / a.rho[c]);
  const T eps = (T)a.eps;
  const T wi = rowok ? (T)s_w[i] : T(0);
  const int nrec = MP * (a.d + 1);
  double* accx = s_dyn + (int64_t)wave * nrec;
  if (a.xout)
    for (int q = lane; q < nrec; q += kWave) accx[q] = 0.0;
  T xr[4] = {T(0), T(0), T(0), T(0)};
  if constexpr (ONFLY) {
    if (a.xin) {
      cluster_support<T, MP>(a, c, ct, ch == ct.x, s_x);
#pragma unroll
      for (int t = 0; t < 4; ++t) xr[t] = (T)s_x[i * 4 + t];
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < a.d && rowok)
          xr[t] = (T)a.xc[((int64_t)c * MP + i) * a.d + t];
    }
  }
  const double* xrow = a.xc + ((int64_t)c * MP + (rowok ? i : 0)) * a.d;
  T* xl = nullptr;
  if constexpr (!ONFLY && VAR != kVarPlain) {
    if (a.recost && a.xstage) {
      xl = reinterpret_cast<T*>(s_dyn + (a.xout ? nwaves * nrec : 0));
      stage_support<T, MP>(a, c, xl);
    }
  }
  double accw = 0.0, accf = 0.0, accr = 0.0;
  XAcc4 xa4;  // support terms of d <= 4 launches, in registers
  // (fetching the next tile's offsets one pass ahead measured no faster)
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<T, MP> tl;
    {
      const int k = uni(a.work[pos]);
      tl.set(a.m, a.off[k], a.off[k + 1], a.pofs[k]);
    }
    with_slots<R>(tl.nsl, [&]<int NS>() {
      ba_tile<T, MP, NS, ONFLY, VAR, CP>(a, tl, xr, xrow, xl, wi, rho, a2,
                                         eps, accw, accf, accr, accx, xa4);
    });
  }
  if constexpr (ONFLY && VAR != kVarPlain)
    if (a.xout) flush_support4<MP>(xa4, a.d, accx);
  write_w_record<MP>(accw, accf, accr, a.part, a.ps, ch);
  if (a.xout) write_x_record(s_dyn, nrec, a.xout, ch);
}

// ---------------------------------------------------------------------------
// Matrix-core passes of FP32 contexts with 32 <= d <= 64, launched per slot
// bucket beside a plain plan-update launch, over the same chunks and work
// list (one wavefront per tile, as there):
//   k_cost_mfma (MP = 32): the cost cache at a new support, written before
//     the launch that first reads it (Eq. (updatex) moved the support);
//   k_sup_mfma (MP = 16 or 32): the support-update sums of the launch just
//     made, from its stored Pi1 and Lambda.  Pi1~ = Pi1 exp(Lambda / rho) +
//     eps and its row sums r_i are formed again with the operations of
//     phase A in the same order (Pi1 and Lambda are stored as computed), so
//     the sums are those of phase A.
// Kept out of the plan-update kernel so that neither the accumulators nor
// the support loads share its registers: with them it held one wavefront
// per SIMD for the widest tiles instead of two.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool chunk_of(const Args<T>& a, int& ch) {
  ch = blockIdx.x;
  if (a.blist) {
    if (ch >= a.bcnt[a.bidx]) return false;
    ch = uni(a.blist[a.boff + ch]);
    return true;
  }
  return ch < *a.nch;
}

// LDS floats of k_cost_mfma: the cluster's support, then one staged block
// of 32 support points per wavefront, rows of xs + 4 floats
__host__ __device__ inline size_t cost_mfma_lds_bytes(int xs, int nwaves) {
  return sizeof(float) * 32 * (size_t)(xs + 4) * (size_t)(1 + nwaves);
}

// LDS writes of a wavefront visible to its other lanes (and its earlier
// LDS reads complete) before it goes on
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

template <int R>
__global__ void __launch_bounds__(256) k_cost_mfma(Args<float> a) {
  extern __shared__ f32x4 s_cost[];  // 16-byte aligned rows
  int ch;
  if (!chunk_of(a, ch)) return;
  const Chunk cj = a.chunks[ch];
  const int wave = uni(threadIdx.x / kWave), nwaves = blockDim.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int n = lane & 31, h = lane >> 5;
  const int xsl = a.xs + 4;
  float* xl = reinterpret_cast<float*>(s_cost);
  float* yl = xl + (1 + wave) * 32 * xsl;
  // the block rows' padding [xs, xs + 4) stays zero
  for (int q = lane; q < 32 * 4; q += kWave) yl[(q >> 2) * xsl + a.xs + (q & 3)] = 0.0f;
  stage_support<float, 32>(a, cj.cluster, xl);
  // |x_i|^2 of the lane's row, in index order, and the lane's half of x_i
  float xnorm = 0.0f;
  for (int t = 0; t < a.d; ++t) {
    const float v = xl[n * xsl + t];
    xnorm = fmaf(v, v, xnorm);
  }
  const int H = ((a.xs >> 1) + 3) & ~3;
  float xh[32];
#pragma unroll
  for (int s4 = 0; s4 < 32; ++s4) xh[s4] = s4 < H ? xl[n * xsl + h * H + s4] : 0.0f;
  const int n16 = 8 * a.xs;  // 16-byte words of one block (<= 8 per lane)
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<float, 32> tl;
    {
      const int k = uni(a.work[pos]);
      tl.set(a.m, a.off[k], a.off[k + 1], a.pofs[k]);
    }
    with_slots<R>(tl.nsl, [&]<int NS>() {
      const uint32_t tb = (uint32_t)(a.m * tl.mk) * 4u;
      const Rsrc rC = make_rsrc(a.Cc + tl.base, tb);
      const Rsrc rX =
          make_rsrc(a.X + tl.o * a.xs, (uint32_t)(tl.mk * a.xs) * 4u);
      constexpr int NB = (NS + 15) / 16;
#pragma unroll
      for (int bk = 0; bk < NB; ++bk) {
        // stage points 32 bk .. 32 bk + 31 (zero past the tile): the block
        // is contiguous, 32 xs floats, read as 16-byte words
        const uint32_t b0 = (uint32_t)(32 * bk * a.xs) * 4u;
        f32x4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (u * kWave + lane < n16)
            v[u] = bload<f32x4>(rX, b0 + (uint32_t)((u * kWave + lane) * 16));
        wave_lds_sync();  // the previous block's operand reads are done
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (u * kWave + lane < n16) {
            const int f = (u * kWave + lane) * 4;
            const int row = f / a.xs;
            *reinterpret_cast<f32x4*>(yl + row * xsl + (f - row * a.xs)) = v[u];
          }
        }
        wave_lds_sync();
        const f32x16 acc = cost_block_mfma(yl, xsl, H, xh, xnorm);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int r = 16 * bk + u;
          if (r < NS) {
            const uint32_t j = (uint32_t)tl.col(r);
            bstore(acc[u], rC,
                   tl.rowok ? (j * (uint32_t)a.m + (uint32_t)tl.i) * 4u
                            : kOob);
          }
        }
      }
    });
  }
}

// Cost recomputation pass on the VALU (FP32, cost cached, where the
// matrix-core pass does not apply): the cost of every tile at the new
// support, by cost_tile from the support staged in LDS (the arithmetic of
// the plan-update kernel's own recomputation), written to the cost cache
// before the plain launch that first reads it.  Few registers, so that many
// wavefronts hide the support loads.
template <int MP, int R>
__global__ void __launch_bounds__(256) k_cost_valu(Args<float> a) {
  extern __shared__ double s_dyn[];  // the cluster's support, [MP][xs + 4]
  int ch;
  if (!chunk_of(a, ch)) return;
  const Chunk cj = a.chunks[ch];
  const int wave = uni(threadIdx.x / kWave), nwaves = blockDim.x / kWave;
  float* xl = reinterpret_cast<float*>(s_dyn);
  stage_support<float, MP>(a, cj.cluster, xl);
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<float, MP> tl;
    {
      const int k = uni(a.work[pos]);
      tl.set(a.m, a.off[k], a.off[k + 1], a.pofs[k]);
    }
    with_slots<R>(tl.nsl, [&]<int NS>() {
      float cs[NS];
      cost_tile<float, MP, NS>(a, tl, xl, cs);
      const Rsrc rC =
          make_rsrc(a.Cc + tl.base, (uint32_t)(a.m * tl.mk) * 4u);
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const uint32_t j = (uint32_t)tl.col(r);
        bstore(cs[r], rC,
               tl.rowok ? (j * (uint32_t)a.m + (uint32_t)tl.i) * 4u : kOob);
      }
    });
  }
}

template <int MP, int R, int CP>
__global__ void __launch_bounds__(256, 2) k_sup_mfma(Args<float> a) {
  extern __shared__ double s_dyn[];  // [nwaves][MP][d+1] support terms
  constexpr int NT = SupAcc<MP>::NT;
  int ch;
  if (!chunk_of(a, ch)) return;
  const Chunk cj = a.chunks[ch];
  const int c = cj.cluster;
  const int wave = uni(threadIdx.x / kWave), nwaves = blockDim.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const float a2 = (float)(kLog2e / a.rho[c]);
  const float eps = (float)a.eps;
  const int nrec = MP * (a.d + 1);
  double* accx = s_dyn + (int64_t)wave * nrec;
  for (int q = lane; q < nrec; q += kWave) accx[q] = 0.0;
  SupAcc<MP> sacc;
  sacc.zero();
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<float, MP> tl;
    {
      const int k = uni(a.work[pos]);
      tl.set(a.m, a.off[k], a.off[k + 1], a.pofs[k]);
    }
    with_slots<R>(tl.nsl, [&]<int NS>() {
      const uint32_t tb = (uint32_t)(a.m * tl.mk) * 4u;
      const Rsrc rP = make_rsrc(a.P1 + tl.base, tb);
      const Rsrc rL = make_rsrc(a.L + tl.base, tb);
      const Rsrc rX =
          make_rsrc(a.X + tl.o * a.xs, (uint32_t)(tl.mk * a.xs) * 4u);
      // slots in groups of G: the operands of group g + 1 load while the
      // products of group g run
      constexpr int G = NS <= 16 ? NS : 4, NG = NS / G;
      static_assert(NS % G == 0, "slot groups");
      float p[NS], l[NS], b[NS], yv[2][G][NT];
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const uint32_t j = (uint32_t)tl.col(r);
        const uint32_t eo =
            tl.rowok ? (j * (uint32_t)a.m + (uint32_t)tl.i) * 4u : kOob;
        p[r] = bload<float, CP>(rP, eo);
        l[r] = bload<float, CP>(rL, eo);
      }
      support_operands<MP, G>(a, tl, rX, 0, yv[0]);
      float rr = 0.0f;
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        b[r] = fmaf(p[r], dexp2(l[r] * a2), tl.valid(r) ? eps : 0.0f);
        rr += b[r];
      }
      rr = sum_row<MP>(rr);
      const float ir = rcp_sum(rr);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG)
          support_operands<MP, G>(a, tl, rX, (g + 1) * G, yv[(g + 1) & 1]);
        support_mfma<MP, G, NS>(a, b, g * G, ir, yv[g & 1], sacc);
      }
      if ((threadIdx.x & (kWave - 1)) < MP && rr > 0.0f) sacc.den += 1.0f;
    });
  }
  sacc.flush(a.d, accx);
  write_x_record(s_dyn, nrec, a.xout, ch);
}

// ---------------------------------------------------------------------------
// Auxiliary kernel: cost sums / first phase A / last phase B / support only
// ---------------------------------------------------------------------------
template <typename T, int MP, int NS, int MODE>
__device__ __forceinline__ void aux_tile(const Args<T>& a, const Tile<T, MP>& tl,
                                         int k, int mode_arg, const double* xrow,
                                         int64_t srow,
                                         const T (&xr)[4], const T* xl, T wi,
                                         T rho, T a2, T eps, double& accw,
                                         double& accf, double& accr,
                                         double* accx) {
  using V4 = typename Vec4<T>::type;
  const int mode = MODE >= 0 ? MODE : mode_arg;
  const int d = a.d;
  const int lane = threadIdx.x & (kWave - 1);
  // cost of slot r: for d <= 4 (stride 4, zero padded) one 4-wide load of
  // the support point against the centroid row in registers, the same
  // arithmetic in the same order as the direct difference over t < d
  auto cost_of = [&](int r) -> T {
    const int jc = tl.colc(r);
    if (a.xs == 4)
      return cost4<T>(xr, reinterpret_cast<const V4*>(a.X + (tl.o + jc) * 4)[0]);
    return cost_generic<T>(xrow, a.X + (tl.o + jc) * a.xs, d);
  };
  T p[NS], l[NS], cs[NS], wk[NS], el[NS], b[NS];
  bool v[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    v[r] = tl.valid(r);
    p[r] = l[r] = cs[r] = wk[r] = T(0);
    el[r] = v[r] ? eps : T(0);
  }
  if (mode == kRho) {
    T s = T(0);
    if (xl) cost_tile<T, MP, NS>(a, tl, xl, cs);
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const T cv = a.dsym ? a.dsym[srow + a.isym[tl.o + tl.colc(r)]]
                          : (xl ? cs[r] : cost_of(r));
      if (v[r]) {
        if (a.Cc) a.Cc[tl.eidx(r, a.m)] = cv;
        s += cv;
      }
    }
    accf += (double)s;  // lane partial, reduced over the wave at the end
    return;
  }
  if (mode == kA0) {
    const bool cached = a.warm && a.warm[k];
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int64_t e = tl.eidx(r, a.m);
      const int jc = tl.colc(r);
      wk[r] = a.W[tl.o + jc];
      cs[r] = a.Cc ? a.Cc[e] : cost_of(r);
      p[r] = cached ? a.P2[e] : wi * wk[r];
      p[r] = v[r] ? p[r] : T(0);
      wk[r] = v[r] ? wk[r] : T(0);
    }
    T rr, f = T(0);
    phase_a<T, MP, NS, true>(el, p, l, cs, wk, a2, b, rr, f);
    accw += consensus_term<T, MP>(rr, tl.rowok, a.rule);
    accf += (double)f;
    if (a.xout) add_support_terms<T, MP, NS>(a, tl, b, rr, accx);
#pragma unroll
    for (int r = 0; r < NS; ++r)
      if (v[r]) {
        const int64_t e = tl.eidx(r, a.m);
        a.P1[e] = p[r];
        a.L[e] = l[r];
      }
    return;
  }
  if (mode == kBF) {
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int64_t e = tl.eidx(r, a.m);
      p[r] = a.P1[e];
      l[r] = a.L[e];
      p[r] = v[r] ? p[r] : T(0);
      l[r] = v[r] ? l[r] : T(0);
    }
    T res = T(0);
    phase_b<T, MP, NS>(el, p, l, wi, rho, a2, res);
    accr += (double)res;
#pragma unroll
    for (int r = 0; r < NS; ++r)
      if (v[r]) {
        const int64_t e = tl.eidx(r, a.m);
        a.P2[e] = p[r];
        a.L[e] = l[r];
      }
    return;
  }
  // kXO: support terms from the stored Pi2 (u = sum_j Pi2 y / sum_j Pi2)
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const T pv = a.P2[tl.eidx(r, a.m)];
    p[r] = v[r] ? pv : T(0);
  }
  T rr = T(0);
#pragma unroll
  for (int r = 0; r < NS; ++r) rr += p[r];
  rr = sum_row<MP>(rr);
  add_support_terms<T, MP, NS>(a, tl, p, rr, accx);
  (void)lane;
}

// MODE >= 0: a kernel fixed to that mode (the other modes' paths and their
// registers compiled out); MODE < 0: the mode from the argument
template <typename T, int MP, int R, int MODE = -1>
__global__ void __launch_bounds__(256) k_aux(Args<T> a, int mode_arg) {
  const int mode = MODE >= 0 ? MODE : mode_arg;
  extern __shared__ double s_dyn[];  // [nwaves][MP][d+1] support terms
  __shared__ double s_w[MP];
  __shared__ double s_x[MP * 4];
  const int ch = blockIdx.x;
  if (ch >= *a.nch) return;
  const Chunk cj = a.chunks[ch];
  const int c = cj.cluster;
  const int2 ct = a.ctab[c];
  if (mode == kBF) {
    cluster_weights<T, MP>(a, c, ct, ch == ct.x, s_w);
    // the support update after the last iteration (small d)
    if (a.xin && a.d <= 4) cluster_support<T, MP>(a, c, ct, ch == ct.x, s_x);
  } else if (mode == kA0) {
    for (int q = threadIdx.x; q < MP; q += blockDim.x) s_w[q] = a.wc[c * MP + q];
    __syncthreads();
  }
  const int wave = uni(threadIdx.x / kWave), nwaves = blockDim.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int i = lane % MP;
  const int d = a.d;
  const bool rowok = i < a.m;
  const bool xrecs = (mode == kXO) || (mode == kA0 && a.xout);
  const T eps = (T)a.eps;
  const double rhod = mode == kRho ? 1.0 : a.rho[c];
  const T rho = (T)rhod;
  const T a2 = (T)(kLog2e / rhod);
  const T wi = (rowok && (mode == kBF || mode == kA0)) ? (T)s_w[i] : T(0);
  const double* xrow = a.xc + ((int64_t)c * MP + (rowok ? i : 0)) * d;
  T xr[4] = {T(0), T(0), T(0), T(0)};
  if (a.xs == 4) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < d && rowok) xr[t] = (T)xrow[t];
  }
  // symbolic supports: this row's offset into the symbol table
  const int64_t srow =
      a.dsym ? (int64_t)a.csym[(int64_t)c * MP + (rowok ? i : 0)] * a.S : 0;
  const int nrec = MP * (d + 1);
  double* accx = s_dyn + (int64_t)wave * nrec;
  if (xrecs)
    for (int q = lane; q < nrec; q += kWave) accx[q] = 0.0;
  T* xl = nullptr;
  if (mode == kRho && a.xstage) {
    xl = reinterpret_cast<T*>(s_dyn);
    stage_support<T, MP>(a, c, xl);
  }
  double accw = 0.0, accf = 0.0, accr = 0.0;
  for (int pos = cj.begin + wave; pos < cj.end; pos += nwaves) {
    Tile<T, MP> tl;
    const int k = uni(a.work[pos]);
    tl.setup(a.off, a.pofs, a.m, k);
    with_slots<R>(tl.nsl, [&]<int NS>() {
      aux_tile<T, MP, NS, MODE>(a, tl, k, mode, xrow, srow, xr, xl, wi, rho,
                                a2, eps, accw, accf, accr, accx);
    });
  }
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
  } else if (mode == kA0) {
    write_w_record<MP>(accw, accf, 0.0, a.part, a.ps, ch);
  } else if (mode == kBF && a.rlast) {
    // residual of the last phase B (summed per cluster by k_fin kFinRes)
    write_w_record<MP>(0.0, 0.0, accr, a.part, a.ps, ch);
  }
  if (xrecs) write_x_record(s_dyn, nrec, a.xout, ch);
}

// ---------------------------------------------------------------------------
// Per-cluster finalisation launches (one workgroup per cluster): rho from
// the cost records; the support update from support records (used when the
// support dimension is too large for the prologue).
// ---------------------------------------------------------------------------
template <int MP>
__global__ void __launch_bounds__(256) k_fin(FinArgs f, int mode) {
  extern __shared__ double s_x[];  // kFinX: MP*(d+1) sums
  __shared__ double s_red[256];
  const int c = blockIdx.x;
  const int2 ct = f.ctab[c];
  if (ct.y == 0) return;  // empty cluster: keep everything
  const int tid = threadIdx.x, nt = blockDim.x;
  if (mode == kFinX) {
    const int nrec = MP * (f.d + 1);
    sum_cluster_records(f.xrec + (int64_t)ct.x * nrec, nrec, ct.y, nrec, s_red,
                        s_x);
    for (int q = tid; q < MP * f.d; q += nt) {
      const int ii = q / f.d, t = q % f.d;
      const double den = s_x[ii * (f.d + 1) + f.d];
      if (ii < f.m && den > 0.0)
        f.xc[((int64_t)c * MP + ii) * f.d + t] = s_x[ii * (f.d + 1) + t] / den;
    }
    return;
  }
  if (mode == kFinRes) {
    // residual of the last phase B: column MP + 1 of its records
    s_red[tid] = sum_strided(f.part + (int64_t)ct.x * f.ps + MP + 1, f.ps, tid,
                             ct.y, nt);
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int gI = 0; gI < nt; ++gI) t += s_red[gI];
      f.rtr[c] = t * f.ninv[c];
    }
    return;
  }
  // kFinRho: sum of the cost records
  s_red[tid] = sum_strided(f.part + (int64_t)ct.x * f.ps, f.ps, tid, ct.y, nt);
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int gI = 0; gI < nt; ++gI) t += s_red[gI];
    f.rho[c] = f.rho0 * t * f.cinv[c];
  }
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
  int32_t* labels;      // out; with prev_valid also the previous labels
  double* best;
  int32_t* counts;      // N x 2 per instance: pairs run through the
                        // iterations, pairs whose cost block was formed
                        // (null: not counted)
  const T* cmu;         // d x K weighted mean of each centroid's support
  const T* crad;        // K  radius of the support around that mean
  const T* xct;         // K x MP x xs centroid supports in the device dtype
  const int32_t* list;  // instance ids of this launch (one slot class);
                        // null: instances 0 .. N-1
  // Cross-round bounds (pruning only): lbs[k * K + c] holds a lower bound
  // on sqrt(LB(k, c)), LB the column-relaxed bound below, valid for the
  // centroid supports of the last pruned assignment; dlt[c] bounds how far
  // any support point of centroid c moved since then.  lbs_in: the stored
  // values may be read (else they are written only).  lbs null: no bounds.
  float* lbs;
  const float* dlt;
  int lbs_in;
  // symbolic supports (as in Args; null dsym: squared Euclidean costs)
  const T* dsym;
  const int32_t* isym;
  const int32_t* csym;
  int S;
  // every pair's distance added to dall[k * K + c] (exhaustive launches of
  // multi-modal instances, whose combined distance sums the modalities);
  // null: not stored
  double* dall;
  int64_t N;            // instances in this launch
  double rho0, eps;
  int m, d, xs, K, iters, prune, prev_valid;
  // 1: the exact column bounds of up to 64 candidate centroids at a time,
  // one per lane (FP32, d <= 16, no symbols, kernels for pad(m) <= 16 whose
  // tiles have at most 32 columns); 0: one candidate at a time across the
  // wavefront
  int batch;
};

// LDS of one assignment wavefront (byte offsets): the instance mean (d
// values), |y_j - mu_P| and w_j per column (2 CPS R values), then for the
// batched bounds a candidate list (128 ints), the instance's points
// centred on mu_P (CPS R rows of xs floats), their squared norms (CPS R)
// and mu_P padded to xs.
struct AssignLds {
  int list, ys, bytes;
};
__host__ __device__ inline AssignLds assign_lds(int d, int MP, int R, int xs,
                                                int esz, int batch) {
  AssignLds L;
  L.list = ((d + 2 * (64 / MP) * R) * esz + 15) & ~15;
  L.ys = L.list + (batch ? 128 * 4 : 0);
  L.bytes = L.ys + (batch ? ((64 / MP) * R * (xs + 1) + xs) * 4 : 0);
  return L;
}

// value of v in lane `src` (src uniform), for 32- and 64-bit types
__device__ __forceinline__ float lane_value(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_value(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Any coupling whose column sums are the instance weights w_j (as Pi1's are,
// Eq. (badmmc0)) has cost sum_j w_j sum_i (Pi1_ij / w_j) C_ij >=
// sum_j w_j min_i C_ij.  This lower bound of the assignment distance lets a
// centroid be skipped when it exceeds the best distance found so far.
template <typename T, int MP, int NS>
__device__ __forceinline__ double cost_lower_bound(const Tile<T, MP>& tl0,
                                                   const T (&cs)[NS],
                                                   const T (&wk)[NS]) {
  const Tile<T, MP> tl = tl0.fresh();
  const T big = T(3.0e38);
  T mn[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) mn[r] = tl.valid(r) ? cs[r] : big;
  // column minimum over the MP lanes of each column group
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    if constexpr (MP >= 2) mn[r] = fmin(mn[r], xdpp_raw<0xB1>(mn[r]));
    if constexpr (MP >= 4) mn[r] = fmin(mn[r], xdpp_raw<0x4E>(mn[r]));
    if constexpr (MP >= 8) mn[r] = fmin(mn[r], xdpp_raw<0x141>(mn[r]));
    if constexpr (MP >= 16) mn[r] = fmin(mn[r], xdpp_raw<0x140>(mn[r]));
    if constexpr (MP >= 32) mn[r] = fmin(mn[r], xswz16(mn[r]));
    if constexpr (MP >= 64) mn[r] = fmin(mn[r], x32(mn[r]));
  }
  // per lane at most NS non-negative terms: the FP32 sum is within a few
  // ulps, far inside the pruning margin
  T lb = T(0);
#pragma unroll
  for (int r = 0; r < NS; ++r) lb = fma(wk[r] > T(0) ? wk[r] : T(0), mn[r] < big ? mn[r] : T(0), lb);
  return sum_wave((double)(tl.i == 0 ? lb : T(0)));
}

// Costs of one (instance, centroid) tile with 4-wide loads: supports and
// centroid rows share the zero-padded stride xs (a multiple of 4).  Slots
// go in chunks, each over all coordinates, so that only one chunk's loads
// are in flight; columns past m_k read 0 through the buffer bounds, and
// entries outside the tile are 0.
template <typename T, int MP, int NS>
__device__ __forceinline__ void pair_costs(const AssignArgs<T>& a,
                                           const Tile<T, MP>& tl0, int c,
                                           T (&cs)[NS]) {
  using V4 = typename Vec4<T>::type;
  const Tile<T, MP> tl = tl0.fresh();
  if (a.dsym) {
    // symbolic supports: the costs are gathered from the symbol table
    const int64_t srow = (int64_t)a.csym[(int64_t)c * MP + tl.ic] * a.S;
#pragma unroll
    for (int r = 0; r < NS; ++r)
      cs[r] = tl.valid(r) ? a.dsym[srow + a.isym[tl.o + tl.colc(r)]] : T(0);
    return;
  }
  const uint32_t rowb = (uint32_t)a.xs * (uint32_t)sizeof(T);
  const Rsrc rY = make_rsrc(a.X + tl.o * a.xs, (uint32_t)tl.mk * rowb);
  const Rsrc rC = make_rsrc(a.xct + (int64_t)c * MP * a.xs, MP * rowb);
  const uint32_t xo = (uint32_t)tl.ic * rowb;
  const int n4 = a.xs / 4;
  constexpr int CH = NS <= 8 ? NS : (NS % 8 == 0 ? 8 : 4);
#pragma unroll
  for (int r0 = 0; r0 < NS; r0 += CH) {
    T acc[CH];
    uint32_t yo[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      acc[u] = T(0);
      yo[u] = (uint32_t)tl.col(r0 + u) * rowb;
    }
    for (int t4 = 0; t4 < n4; ++t4) {
      const uint32_t tb = (uint32_t)t4 * (uint32_t)sizeof(V4);
      const V4 xv = bload<V4>(rC, xo + tb);
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const V4 y = bload<V4>(rY, yo[u] + tb);
        T df = xv.x - y.x;
        acc[u] = fma(df, df, acc[u]);
        df = xv.y - y.y;
        acc[u] = fma(df, df, acc[u]);
        df = xv.z - y.z;
        acc[u] = fma(df, df, acc[u]);
        df = xv.w - y.w;
        acc[u] = fma(df, df, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u)
      cs[r0 + u] = tl.valid(r0 + u) ? acc[u] : T(0);
  }
}

// B-ADMM transport value <C, Pi1> of one (instance, centroid) pair after
// `iters` iterations with both marginals fixed (Eqs. (badmmc0b)-(badmm2)
// with the centroid's weights held).  Carried per entry: Pi2, Lambda and
// the scaled cost C/rho (in base-2 units), from which exp(-(C + Lambda)/rho)
// is one exponential; Pi1 lives only within an iteration, and the last
// one's value is the transport value.  Padded columns of a row carry the
// smoothing eps in Pi2 with no other effect; their share of the row sum,
// eps times the padded column count, is taken out again.
template <typename T, int MP, int NS>
__device__ __forceinline__ double pair_value(const AssignArgs<T>& a,
                                             const Tile<T, MP>& tl0, int c,
                                             const T (&cs)[NS],
                                             const T (&wk)[NS]) {
  const Tile<T, MP> tl = tl0.fresh();
  T csum = T(0);
#pragma unroll
  for (int r = 0; r < NS; ++r) csum += cs[r];
  const double tot = sum_wave((double)csum);
  const double rhod = a.rho0 * tot / ((double)a.m * tl.mk);
  const T rho = (T)rhod;
  const T a2 = (T)(kLog2e / rhod);
  const T wi = tl.rowok ? (T)a.wc[c * MP + tl.i] : T(0);
  const T elr = tl.rowok ? (T)a.eps : T(0);
  const T pad = elr * (T)(NS * Tile<T, MP>::CPS - tl.mk);
  T ca[NS], p2[NS], l[NS], q[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    l[r] = T(0);
    q[r] = T(0);
  }
  // exp2(-1e30) = 0: an entry outside the tile never takes mass
  if constexpr (sizeof(T) == 4 ? MP >= 8 && NS <= (MP >= 32 ? 32 : 8)
                                : MP >= 16 && NS <= 4) {
    // Column normalisation by reduce-scatter: the column sums and the
    // factors w_j / sum are formed once per quad instead of in every lane
    // (about a quarter fewer instructions per entry and iteration; in FP64
    // one division per column and quad instead of one per entry).  Tiles of
    // 8 and 16 rows use it up to 8 slots only: the 16-slot kernel of the
    // 16-row padding would need 20 more registers and lose a wavefront per
    // SIMD.  FP64 uses it for tiles of 16 rows or more up to 4 slots (its
    // 8-row 8-slot kernel would lose a wavefront, its wider-slot kernels
    // spill more, and with 5-8 slots the later rounds on d = 16 measured
    // slower).
    const int ql = threadIdx.x & 3;
    // weights of the slots whose sums this lane holds (the chunks' kept
    // registers), in chunk order, taken from the first lane of the quad:
    // rows past m hold zero weights, and a quad with any row below m has
    // its first row below m
    T wr[rs_kept_before(NS)];
    rs_chunks<NS>([&]<int C0, int C>() {
      constexpr int n = rs_kept_before(C0);
      wr[n] = rs_pick<C0, C, 0, true>(wk);
      if constexpr (RsChunk<C>::kept == 2)
        wr[n + 1] = rs_pick<C0, C, 1, true>(wk);
    });
    // scaled costs and Pi2 of the slots in this lane's register order
    rs_chunks<NS>([&]<int C0, int C>() {
      [&]<int... U>(std::integer_sequence<int, U...>) {
        ((ca[C0 + U] =
              tl.rowok && tl.g + Tile<T, MP>::CPS *
                                     (C0 + (U ^ RsChunk<C>::mask(ql))) <
                              tl.mk
                  ? rs_pick<C0, C, U>(cs) * a2
                  : T(1.0e30),
          p2[C0 + U] = wi * rs_pick<C0, C, U>(wk)),
         ...);
      }(std::make_integer_sequence<int, C>{});
    });
    // For 16-row tiles (and 8-row ones) l holds Lambda / rho in base-2
    // units (Lambda * a2):
    // its update rho * (Pi1 - Pi2) becomes log2(e) * (Pi1 - Pi2), and the
    // exponents need no multiply (measured 2-5 % faster there, 2 % slower
    // for 32-row tiles, which keep Lambda itself)
    constexpr bool SL = MP <= 16;
    const T lu = SL ? T(kLog2e) : rho;
    for (int it = 0; it < a.iters; ++it) {
      T rr = T(0);
      rs_chunks<NS>([&]<int C0, int C>() {
        constexpr int K = RsChunk<C>::kept;
        T E[C], s[C];
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const int r = C0 + u;
          E[u] = dexp2(SL ? l[r] : l[r] * a2);
          q[r] = fma(p2[r],
                     dexp2(SL ? -(l[r] + ca[r]) : -fma(l[r], a2, ca[r])),
                     elr);
          s[u] = q[r];
        }
        rs_sum<MP, C>(s);
        T f[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
          f[k] = wr[rs_kept_before(C0) + k] * rcp_sum(s[k]);
        [&]<int... U>(std::integer_sequence<int, U...>) {
          ((q[C0 + U] *= rs_get<C, U>(f),
            p2[C0 + U] = fma(q[C0 + U], E[U], elr), rr += p2[C0 + U]),
           ...);
        }(std::make_integer_sequence<int, C>{});
      });
      rr = sum_row<MP>(rr) - pad;
      const T coef = wi * rcp_sum(rr);
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const T u = p2[r] * coef;
        l[r] = fma(lu, q[r] - u, l[r]);
        p2[r] = u;
      }
    }
    T fv = T(0);
#pragma unroll
    for (int r = 0; r < NS; ++r) fv = fma(ca[r], q[r], fv);
    return sum_wave((double)fv) * (rhod / kLog2e);
  }
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    ca[r] = tl.valid(r) ? cs[r] * a2 : T(1.0e30);
    p2[r] = wi * wk[r];
  }
  // slots in chunks of CH: exp(Lambda/rho) and the column sums are held
  // for one chunk at a time
  constexpr int CH = NS <= 8 ? NS : (NS % 8 == 0 ? 8 : 4);
  for (int it = 0; it < a.iters; ++it) {
    T rr = T(0);
#pragma unroll
    for (int r0 = 0; r0 < NS; r0 += CH) {
      T E[CH], s[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int r = r0 + u;
        E[u] = dexp2(l[r] * a2);
        q[r] = fma(p2[r], dexp2(-fma(l[r], a2, ca[r])), elr);
        s[u] = q[r];
      }
      sum_col_n<MP, CH>(s);
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int r = r0 + u;
        q[r] *= wk[r] * rcp_sum(s[u]);
        p2[r] = fma(q[r], E[u], elr);
        rr += p2[r];
      }
    }
    rr = sum_row<MP>(rr) - pad;
    const T coef = wi * rcp_sum(rr);
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const T u = p2[r] * coef;
      l[r] = fma(rho, q[r] - u, l[r]);
      p2[r] = u;
    }
  }
  T fv = T(0);
#pragma unroll
  for (int r = 0; r < NS; ++r) fv = fma(ca[r], q[r], fv);
  return sum_wave((double)fv) * (rhod / kLog2e);
}

// Exact lower bound of the distance from the triangle inequality around the
// centroid mean mu_c (support radius rad_c) and the instance mean mu_P:
//   sum_j w_j max(0, |dist(mu_P, mu_c) - |y_j - mu_P|| - rad_c)^2,
// for centroid c of this lane.  smu holds mu_P, srj / swj the instance's
// |y_j - mu_P| and w_j.  A small relative slack keeps it below the true
// bound under FP32 rounding.
template <typename T>
__device__ __forceinline__ T cheap_bound(const AssignArgs<T>& a, int c,
                                         const T* smu, const T* srj,
                                         const T* swj, int mk) {
  T sq = T(0);
  for (int t = 0; t < a.d; ++t) {
    const T df = smu[t] - a.cmu[(int64_t)t * a.K + c];
    sq = fma(df, df, sq);
  }
  const T dl = dsqrt(sq);
  const T rad = a.crad[c];
  T acc = T(0);
  for (int j = 0; j < mk; ++j) {
    const T rj = srj[j];
    T gap = fabs(dl - rj) - rad - T(1e-5) * (dl + rj + rad);
    gap = gap > T(0) ? gap : T(0);
    acc = fma(swj[j] * gap, gap, acc);
  }
  return acc;
}

// Column-relaxed lower bound sum_j w_j min_i C_ij of the pair (this
// wavefront's instance, centroid c), one centroid per lane, from the Gram
// form of the cost over points centred on the instance mean mu:
// C_ij = |x'_i|^2 + |y'_j|^2 - 2 x'_i . y'_j with x' = x - mu, y' = y - mu;
// the column's own term |y'_j|^2 is constant over i and added after the
// minimum.  Every FP32 step (centring, the three sums of at most 16
// products, the last additions) errs by well under 64 u (|x'_i|^2 +
// |y'_j|^2) in total (u = 2^-24); both squared norms are scaled by
// 1 - 1e-5, a margin of about 168 u, so each entry stays below the exact
// cost and the result a lower bound of the sum of exact minima.  The centred points y', their squared norms and mu are
// in the wavefront's LDS (the same words for every lane); the centroid
// rows are the lane's own.  d <= 16, m_k <= MK.
template <int MP, int MK>
__device__ __forceinline__ float lane_column_bound(const AssignArgs<float>& a,
                                                   const float* ys,
                                                   const float* yy,
                                                   const float* mu,
                                                   const float* swj, int mk,
                                                   int c) {
  const float big = 3.0e38f;
  const int n4 = a.xs >> 2;
  float mn[MK];
#pragma unroll
  for (int j = 0; j < MK; ++j) mn[j] = big;
  for (int i = 0; i < a.m; ++i) {
    const float4* xp =
        reinterpret_cast<const float4*>(a.xct + ((int64_t)c * MP + i) * a.xs);
    float4 xv[4];
    float xx = 0.0f;
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4) {
      if (t4 < n4) {
        const float4 x = xp[t4];
        const float4 u = reinterpret_cast<const float4*>(mu)[t4];
        xv[t4] = make_float4(x.x - u.x, x.y - u.y, x.z - u.z, x.w - u.w);
        xx = fmaf(xv[t4].x, xv[t4].x, xx);
        xx = fmaf(xv[t4].y, xv[t4].y, xx);
        xx = fmaf(xv[t4].z, xv[t4].z, xx);
        xx = fmaf(xv[t4].w, xv[t4].w, xx);
      }
    }
    const float xxm = xx * (1.0f - 1.0e-5f);
#pragma unroll
    for (int j = 0; j < MK; ++j) {
      if (j < mk) {
        const float4* yp = reinterpret_cast<const float4*>(ys + j * a.xs);
        float dot = 0.0f;
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
          if (t4 < n4) {
            const float4 y = yp[t4];
            dot = fmaf(xv[t4].x, y.x, dot);
            dot = fmaf(xv[t4].y, y.y, dot);
            dot = fmaf(xv[t4].z, y.z, dot);
            dot = fmaf(xv[t4].w, y.w, dot);
          }
        }
        mn[j] = fminf(mn[j], fmaf(-2.0f, dot, xxm));
      }
    }
  }
  float lb = 0.0f;
#pragma unroll
  for (int j = 0; j < MK; ++j) {
    if (j < mk) {
      // the column's own term, constant over i, after the minimum
      const float v = mn[j] < big ? mn[j] + yy[j] * (1.0f - 1.0e-5f) : 0.0f;
      lb = fmaf(swj[j] > 0.0f ? swj[j] : 0.0f, v > 0.0f ? v : 0.0f, lb);
    }
  }
  return lb * (1.0f - 4.0e-6f);  // at most 32 terms: FP32 sum within 32 u
}

template <typename T, int MP, int NS>
__device__ __forceinline__ void assign_tile(const AssignArgs<T>& a,
                                            const Tile<T, MP>& tl,
                                            int64_t kinst, T* sw, int* slist,
                                            float* sys, int prev,
                                            double& bestv, int& bestc,
                                            int& nevals, int& ncost) {
  const int d = a.d;
  const int lane = threadIdx.x & (kWave - 1);
  T wk[NS], cs[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r)
    wk[r] = tl.valid(r) ? a.W[tl.o + tl.colc(r)] : T(0);
  auto consider = [&](int c) {
    const double val = pair_value<T, MP, NS>(a, tl, c, cs, wk);
    if (a.dall && lane == 0) a.dall[kinst * a.K + c] += val;
    ++nevals;
    if (bestc < 0 || val < bestv || (val == bestv && c < bestc)) {
      bestv = val;
      bestc = c;
    }
  };
  if (!a.prune) {
    for (int c = 0; c < a.K; ++c) {
      pair_costs<T, MP, NS>(a, tl, c, cs);
      ++ncost;
      consider(c);
    }
    return;
  }
  // instance mean mu_P (dimensions split over the MP lanes of a column
  // group), then |y_j - mu_P| and w_j per column into the wave's LDS
  T* smu = sw;
  T* srj = sw + d;
  T* swj = srj + tl.mk;
  for (int t = tl.i; t < d; t += MP) {
    T sm = T(0);
#pragma unroll
    for (int r = 0; r < NS; ++r)
      sm = fma(wk[r], a.X[(tl.o + tl.colc(r)) * a.xs + t], sm);
    sm = sum_row<MP>(sm);
    if (tl.g == 0) smu[t] = sm;
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    T sq = T(0);
    for (int t = tl.i; t < d; t += MP) {
      const T df = a.X[(tl.o + tl.colc(r)) * a.xs + t] - smu[t];
      sq = fma(df, df, sq);
    }
    const T rj = dsqrt(sum_col<MP>(sq));
    if (tl.i == 0 && tl.col(r) < tl.mk) {
      srj[tl.col(r)] = rj;
      swj[tl.col(r)] = wk[r];
    }
  }
  __builtin_amdgcn_wave_barrier();
  const T big = T(3.0e38);
  // 1) first candidate: the previous label, else the smallest bound
  int c0 = prev;
  if (c0 < 0 || c0 >= a.K) {
    T lbm = big;
    int cm = a.K;
    for (int b0 = 0; b0 < a.K; b0 += kWave) {
      const int c = b0 + lane;
      const T lb = c < a.K ? cheap_bound(a, c, smu, srj, swj, tl.mk) : big;
      if (lb < lbm) {
        lbm = lb;
        cm = c;
      }
    }
    // wave argmin, ties to the lowest index
    for (int o = 1; o < kWave; o <<= 1) {
      const T ov = __shfl_xor(lbm, o, kWave);
      const int oc = __shfl_xor(cm, o, kWave);
      if (ov < lbm || (ov == lbm && oc < cm)) {
        lbm = ov;
        cm = oc;
      }
    }
    c0 = uni(cm);
  }
  pair_costs<T, MP, NS>(a, tl, c0, cs);
  ++ncost;
  const double lb0 = a.lbs ? cost_lower_bound<T, MP, NS>(tl, cs, wk) : 0.0;
  consider(c0);
  // stored bound of a formed cost block: sqrt(LB) rounded down by far more
  // than the FP32 rounding of the block, so it stays a lower bound
  auto stored = [](double lbv) -> float {
    return (float)(sqrt(lbv > 0.0 ? lbv : 0.0) * (1.0 - 1e-6));
  };
  const int64_t lrow = kinst * (int64_t)a.K;  // this instance's bounds
  // 2) every other centroid unless a bound clears the best value by a
  // margin far above FP32 rounding of the column sums, so a skipped
  // centroid can never be the argmin (ties go to the lowest index).  The
  // bounds of 64 centroids at a time, one per lane: the stored bound of the
  // last pruned assignment decayed by the centroid's support drift (if
  // sqrt(LB) was at least u and no support point moved further than dlt,
  // sqrt(LB) is at least u - dlt: every min_i |y_j - x_i| falls by at most
  // dlt and the w-weighted 2-norm over j by at most dlt), else the cheap
  // bound; the survivors in index order, each checked again against the
  // best value at its turn.
  if constexpr (sizeof(T) == 4 && MP <= 16 && NS * Tile<T, MP>::CPS <= 32) {
    if (a.batch) {
      // Batched: the candidates of each group of 64 centroids (those whose
      // stored / cheap bound does not clear the best value) join a list;
      // every 64 of them (and at the end) their exact column bounds are
      // formed one per lane, then taken in index order: the cost block and
      // transport where the bound does not clear the best value at its turn
      // (the same decisions as one candidate at a time, on bounds formed
      // from the same cost entries).
      constexpr int MK = NS * Tile<T, MP>::CPS;
      // the instance's points centred on mu_P, their squared norms and mu_P
      // (padded with zeros to xs) into the wavefront's LDS
      float* syy = sys + MK * a.xs;
      float* smp = syy + MK;
      for (int t = lane; t < a.xs; t += kWave) smp[t] = t < d ? smu[t] : 0.0f;
      wave_lds_sync();
      for (int f = 4 * lane; f < tl.mk * a.xs; f += 4 * kWave) {
        const float4 y = *reinterpret_cast<const float4*>(a.X + tl.o * a.xs + f);
        const float4 u = *reinterpret_cast<const float4*>(smp + f % a.xs);
        *reinterpret_cast<float4*>(sys + f) =
            make_float4(y.x - u.x, y.y - u.y, y.z - u.z, y.w - u.w);
      }
      wave_lds_sync();
      for (int j = lane; j < tl.mk; j += kWave) {
        float q = 0.0f;
        for (int t = 0; t < a.xs; ++t) q = fmaf(sys[j * a.xs + t], sys[j * a.xs + t], q);
        syy[j] = q;
      }
      int nb = 0;
      for (int b0 = 0; b0 < a.K; b0 += kWave) {
        const int c = b0 + lane;
        const double cut0 = bestv * (1.0 + 1e-4);
        T lb = big;
        float nu = 0.0f;
        if (c < a.K) {
          T sb = T(0);
          if (a.lbs && a.lbs_in) {
            const T u = (T)a.lbs[lrow + c] - (T)a.dlt[c];
            sb = u > T(0) ? u : T(0);
          }
          lb = sb * sb;
          if ((double)lb <= cut0) {
            const T cb = cheap_bound(a, c, smu, srj, swj, tl.mk);
            lb = cb > lb ? cb : lb;
          }
          nu = (float)dsqrt(lb) * (1.0f - 1e-6f);
          if (c == c0) nu = stored(lb0);
        }
        const bool lv = c < a.K && c != c0 && (double)lb <= cut0;
        const unsigned long long live = __ballot(lv);
        // bounds of the centroids that are no candidates are final
        if (a.lbs && c < a.K && !lv) a.lbs[lrow + c] = nu;
        const int rank = __builtin_amdgcn_mbcnt_hi(
            (unsigned)(live >> 32),
            __builtin_amdgcn_mbcnt_lo((unsigned)live, 0u));
        wave_lds_sync();
        if (lv) slist[nb + rank] = c;
        nb += __builtin_popcountll(live);
        wave_lds_sync();
        const bool last = b0 + kWave >= a.K;
        while (nb >= kWave || (last && nb > 0)) {
          const int nq = nb < kWave ? nb : kWave;
          const int cq = lane < nq ? slist[lane] : -1;
          const double lbq =
              cq >= 0 ? (double)lane_column_bound<MP, MK>(
                            a, sys, syy, smp,
                            reinterpret_cast<const float*>(swj), tl.mk, cq)
                      : 0.0;
          if (a.lbs && cq >= 0) a.lbs[lrow + cq] = stored(lbq);
          ncost += nq;
          // in increasing order of the bound (ties: list order, i.e.
          // centroid index), so that the best value falls early; once the
          // smallest bound left clears the best value, so do all the rest
          double open = cq >= 0 ? lbq : 1.0e300;
          for (int it = 0; it < nq; ++it) {
            double mv = open;
            int ml = lane;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
              const double ov = __shfl_xor(mv, o, kWave);
              const int ol = __shfl_xor(ml, o, kWave);
              if (ov < mv || (ov == mv && ol < ml)) {
                mv = ov;
                ml = ol;
              }
            }
            ml = uni(ml);
            if (!(lane_value(mv, 0) <= bestv * (1.0 + 1e-4))) break;
            const int cc = __builtin_amdgcn_readlane(cq, ml);
            if (lane == ml) open = 1.0e300;
            pair_costs<T, MP, NS>(a, tl, cc, cs);
            consider(cc);
          }
          // the unprocessed rest moves to the front of the list
          const int rest = nb - nq;
          const int mv = lane < rest ? slist[nq + lane] : 0;
          wave_lds_sync();
          if (lane < rest) slist[lane] = mv;
          wave_lds_sync();
          nb = rest;
        }
      }
      return;
    }
  }
  for (int b0 = 0; b0 < a.K; b0 += kWave) {
    const int c = b0 + lane;
    const double cut0 = bestv * (1.0 + 1e-4);
    T lb = big;
    float nu = 0.0f;  // new stored bound of pair (k, c)
    if (c < a.K) {
      T sb = T(0);
      if (a.lbs && a.lbs_in) {
        const T u = (T)a.lbs[lrow + c] - (T)a.dlt[c];
        sb = u > T(0) ? u : T(0);
      }
      lb = sb * sb;
      if ((double)lb <= cut0) {
        const T cb = cheap_bound(a, c, smu, srj, swj, tl.mk);
        lb = cb > lb ? cb : lb;
      }
      nu = (float)dsqrt(lb) * (1.0f - 1e-6f);
      if (c == c0) nu = stored(lb0);
    }
    unsigned long long live =
        __ballot(c < a.K && c != c0 && (double)lb <= cut0);
    while (live) {
      const int bit = __builtin_ctzll(live);
      live &= live - 1;
      const double cut = bestv * (1.0 + 1e-4);
      if ((double)lane_value(lb, bit) > cut) continue;
      const int cc = b0 + bit;
      pair_costs<T, MP, NS>(a, tl, cc, cs);
      ++ncost;
      const double lbx = cost_lower_bound<T, MP, NS>(tl, cs, wk);
      if (lane == bit) nu = stored(lbx);
      if (lbx > cut) continue;
      consider(cc);
    }
    if (a.lbs && c < a.K) a.lbs[lrow + c] = nu;
  }
}

// (pad(m) = 16, 4 slots: five wavefronts per SIMD instead of four, a few
// registers spilled outside the transport loop; measured 2.5-3 % faster)
template <typename T, int MP, int R>
__global__ void __launch_bounds__(256, MP == 16 && R == 4 ? 5 : 1)
    k_assign(AssignArgs<T> a) {
  // per wave: d values (mu_P), then |y_j - mu_P| and w_j per column
  extern __shared__ __attribute__((aligned(16))) unsigned char s_raw[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uni(threadIdx.x / kWave);
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
  if (q >= a.N) return;  // whole wavefront exits together
  const int64_t k = a.list ? uni(a.list[q]) : q;
  const AssignLds L = assign_lds(a.d, MP, R, a.xs, (int)sizeof(T), a.batch);
  unsigned char* wl = s_raw + (int64_t)wave * L.bytes;
  T* sw = reinterpret_cast<T*>(wl);
  Tile<T, MP> tl;
  tl.setup(a.off, nullptr, a.m, (int)k);
  if (tl.mk < 1 || tl.nsl > R) {
    // outside this kernel's tile shapes (only reachable through callers
    // that hand over unchecked offsets): no support point is read
    if (lane == 0) {
      a.labels[k] = -1;
      a.best[k] = __builtin_nan("");
    }
    return;
  }
  const int prev = a.prev_valid ? uni(a.labels[k]) : -1;
  double bestv = 0.0;
  int bestc = -1, nevals = 0, ncost = 0;
  with_slots<R>(tl.nsl, [&]<int NS>() {
    assign_tile<T, MP, NS>(a, tl, k, sw, reinterpret_cast<int*>(wl + L.list),
                           reinterpret_cast<float*>(wl + L.ys), prev, bestv,
                           bestc, nevals, ncost);
  });
  if (lane == 0) {
    a.labels[k] = bestc;
    a.best[k] = bestv;
    // per-instance counts (plain stores: a counter shared by all
    // wavefronts serialises its atomic updates)
    if (a.counts)
      reinterpret_cast<int2*>(a.counts)[k] = make_int2(nevals, ncost);
  }
}

// Per-centroid quantities of the assignment's lower bounds: the weighted
// mean of the support, the largest distance of a support point from it
// (inflated by 1e-6 relative so that rounding cannot make a bound
// invalid), and the support in the device dtype with row stride xs.  One
// wavefront per centroid, FP64 sums in index order.
template <typename T>
__global__ void __launch_bounds__(64)
    k_cstats(const double* xc, const double* wc, int m, int MP, int d,
             int xs, int K, T* cmu, T* crad, T* xct, const double* xref,
             float* dlt) {
  extern __shared__ double s_mu[];  // d
  const int q = blockIdx.x, l = threadIdx.x;
  const double* xq = xc + (size_t)q * MP * d;
  const double* wq = wc + (size_t)q * MP;
  for (int e = l; e < MP * xs; e += 64) {
    const int i = e / xs, t = e % xs;
    xct[(size_t)q * MP * xs + e] = t < d ? (T)xq[(size_t)i * d + t] : T(0);
  }
  double ws = 0.0;
  for (int i = 0; i < m; ++i) ws += wq[i];
  const double div = ws > 0 ? ws : 1.0;
  for (int t = l; t < d; t += 64) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += wq[i] * xq[(size_t)i * d + t] / div;
    s_mu[t] = s;
    cmu[(size_t)t * K + q] = (T)s;
  }
  __syncthreads();
  double r = 0.0;
  for (int i = l; i < m; i += 64) {
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
      const double df = xq[(size_t)i * d + t] - s_mu[t];
      s += df * df;
    }
    r = fmax(r, sqrt(s));
  }
  for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o));
  if (l == 0) crad[q] = (T)(r * (1.0 + 1e-6) + 1e-30);
  if (xref) {
    // drift: the largest distance a support point moved since xref
    const double* xo = xref + (size_t)q * MP * d;
    double g = 0.0;
    for (int i = l; i < m; i += 64) {
      double s = 0.0;
      for (int t = 0; t < d; ++t) {
        const double df = xq[(size_t)i * d + t] - xo[(size_t)i * d + t];
        s += df * df;
      }
      g = fmax(g, sqrt(s));
    }
    for (int o = 32; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o));
    if (l == 0) dlt[q] = (float)(g * (1.0 + 1e-6) + 1e-30);
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
  BA bap[2][4][6] = {}; // the same without support terms
  BA bapn[2][4][6] = {}; // bap streaming its plan state (FP32)
  BA ban[4][6] = {};    // ba streaming its plan state (FP32, d > 4)
  BA sup[2][4][6] = {}; // k_sup_mfma [stream][mp][r], FP32, MP 16 / 32
  BA cst[6] = {};       // k_cost_mfma, FP32, MP 32
  BA cstv[4][6] = {};   // k_cost_valu [mp][r], FP32
  AX aux[4][6] = {};
  AX auxm[3][4][6] = {};  // fixed to kRho, kA0, kBF
  AS asg[4][6] = {};
};
using FinFn = void (*)(FinArgs, int);

}  // namespace d2k

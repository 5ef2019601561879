// Exact transport problems and the subgradient-descent centroid update
// (Appendix A, Algorithm "Centroid Update with Subgradient Descent").
//
// k_lp_transport solves, for every instance, the transport LP Eq. (primal)
// between its cluster's centroid (rows, supplies w_i) and the instance
// (columns, demands w^(k)_j) exactly, by the network simplex of the
// transportation problem in FP64, one wavefront per instance:
//   * initial basis: the north-west corner rule (m + m_k - 1 basic cells,
//     degenerate zero flows where a row and a column run out together);
//   * potentials u_i + v_j = C_ij on the basic cells (u_0 = 0) and the
//     basis tree rooted at row 0 (parent, parent arc, depth of every node):
//     once, spread from the root by parallel relaxation over the arcs;
//   * pricing: the cell of most negative reduced cost C_ij - u_i - v_j
//     (ties to the lowest cell) enters, until none is below -1e-12 max C;
//   * the cycle it closes in the basis tree (the tree paths of its row and
//     column up to their common ancestor) alternates -/+ from the entering
//     cell; the "-" cell of least flow (first along the column's path, then
//     the row's, each from the entering cell) leaves;
//   * the tree is then kept instead of rebuilt: with ancestor tables
//     (binary lifting, 7 levels for at most 128 nodes) every node finds in
//     a fixed number of steps whether it lies on the cycle and whether it
//     hangs below the leaving arc; that subtree is re-hung from the
//     entering cell (the tree path from its endpoint up to the leaving arc
//     reverses, depths follow from the common ancestors), and its
//     potentials shift by the entering cell's reduced cost (+ on its
//     endpoint's side, - on the other), so that every basic cell keeps a
//     zero reduced cost.
// The cost block lives in LDS (m x m_k doubles), the basis (cells, flows,
// costs) and the tree (parent arc, depth) too.  Outputs per instance: the
// optimal plan (in the plan layout of the context), the LP value, and the
// row duals u_i minus their mean -- the projected subgradient of
// W^2(w) with respect to the centroid weights, Eq. (dualvar).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "d2_kernels.hpp"

namespace d2s {

constexpr int kArcs = 128;  // basis size m + m_k - 1 <= 127
constexpr int kLevels = 7;  // ancestor table levels: depth < 128

struct LpArgs {
  const int64_t* off;
  const int64_t* pofs;
  const int32_t* labels;
  const double* xc;   // K x MP x d
  const double* wc;   // K x MP
  const void* X;      // n x xs, device dtype
  const void* W;      // n
  // symbolic supports (Sec. 5): cost = D[csym[c * MP + i] * S + isym[j]]
  const void* dsym;
  const int32_t* isym;
  const int32_t* csym;
  int S;
  void* P1;           // plan outputs (device dtype), may coincide
  void* P2;
  double* U;          // N x MP projected row duals
  double* val;        // N LP values
  int* fail;          // instances whose LP hit the pivot cap
  unsigned long long* pivots;  // total pivots
  int64_t N;
  int m, MP, d, xs, mkmax, max_pivots, f64;
};

struct LpLds {
  double u[64];
  double v[64];
  double af[kArcs];   // arc flow
  double ac[kArcs];   // arc cost
  int16_t ai[kArcs];  // arc row
  int16_t aj[kArcs];  // arc column
  int16_t parc[kArcs];  // tree: arc to the parent (-1 at the root)
  int16_t par[kArcs];   // tree: parent node (-1 at the root)
  int16_t dep[kArcs];   // tree depth
  int8_t known[kArcs];
  int16_t anc[kLevels][kArcs];  // ancestor 2^k levels up (root: itself)
};

// Order this wavefront's LDS accesses across lanes (the wavefront's LDS
// operations complete in issue order; this keeps the compiler from caching
// values across the exchange).
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// LDS bytes of one wavefront: the fixed part, then the cost block
__host__ __device__ inline size_t lp_lds_bytes(int MP, int mkmax) {
  return (sizeof(LpLds) + 15) / 16 * 16 + sizeof(double) * MP * mkmax;
}

template <typename T>
__device__ __forceinline__ double ld(const void* p, int64_t i) {
  return (double)reinterpret_cast<const T*>(p)[i];
}

__global__ void __launch_bounds__(256) k_lp_transport(LpArgs a) {
  extern __shared__ unsigned char s_raw[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * nw + wave;
  if (k >= a.N) return;  // whole wavefront leaves together
  const size_t per = lp_lds_bytes(a.MP, a.mkmax);
  LpLds& s = *reinterpret_cast<LpLds*>(s_raw + per * wave);
  double* C = reinterpret_cast<double*>(s_raw + per * wave +
                                        (sizeof(LpLds) + 15) / 16 * 16);
  const int m = a.m;
  const int64_t o = a.off[k];
  const int mk = (int)(a.off[k + 1] - o);
  const int c = a.labels[k];
  const int nn = m + mk;  // nodes: rows 0..m-1, columns m..m+mk-1
  const int na = nn - 1;  // basic cells
  const double* xq = a.xc + (int64_t)c * a.MP * a.d;
  const double* wq = a.wc + (int64_t)c * a.MP;
  // cost block, column-major (cell e = j * m + i)
  double cmax = 0.0;
  for (int e = lane; e < m * mk; e += 64) {
    const int i = e % m, j = e / m;
    double cv;
    if (a.dsym) {
      const int64_t q = (int64_t)a.csym[(int64_t)c * a.MP + i] * a.S +
                        a.isym[o + j];
      cv = a.f64 ? ld<double>(a.dsym, q) : ld<float>(a.dsym, q);
    } else {
      cv = 0.0;
      for (int t = 0; t < a.d; ++t) {
        const int64_t q = (o + j) * a.xs + t;
        const double y = a.f64 ? ld<double>(a.X, q) : ld<float>(a.X, q);
        const double df = xq[(int64_t)i * a.d + t] - y;
        cv = fma(df, df, cv);
      }
    }
    C[e] = cv;
    cmax = fmax(cmax, cv);
  }
  for (int off2 = 32; off2 > 0; off2 >>= 1)
    cmax = fmax(cmax, __shfl_xor(cmax, off2));
  const double tol = -1e-12 * (cmax > 0.0 ? cmax : 1.0);
  wsync();
  // north-west corner basis
  if (lane == 0) {
    int i = 0, j = 0, n = 0;
    double ra = wq[0];
    double rb = a.f64 ? ld<double>(a.W, o) : ld<float>(a.W, o);
    for (;;) {
      const double f = fmin(ra, rb);
      s.ai[n] = (int16_t)i;
      s.aj[n] = (int16_t)j;
      s.af[n] = f > 0.0 ? f : 0.0;
      s.ac[n] = C[j * m + i];
      ++n;
      ra -= f;
      rb -= f;
      if (i == m - 1 && j == mk - 1) break;
      if (j == mk - 1 || (i < m - 1 && ra <= rb)) {
        ++i;
        ra = wq[i];
      } else {
        ++j;
        rb = a.f64 ? ld<double>(a.W, o + j) : ld<float>(a.W, o + j);
      }
    }
  }
  wsync();
  int piv = 0;
  bool capped = false;
  // potentials and the basis tree, spread from the root (row 0), once
  for (int q = lane; q < nn; q += 64) {
    s.known[q] = (int8_t)(q == 0);
    s.dep[q] = 0;
    s.parc[q] = -1;
    s.par[q] = -1;
  }
  if (lane == 0) s.u[0] = 0.0;
  wsync();
  for (int pass = 0; pass < nn; ++pass) {
    bool ch = false;
    for (int e = lane; e < na; e += 64) {
      const int i = s.ai[e], j = s.aj[e], cj = m + j;
      const bool ki = s.known[i] != 0, kj = s.known[cj] != 0;
      if (ki && !kj) {
        s.v[j] = s.ac[e] - s.u[i];
        s.parc[cj] = (int16_t)e;
        s.par[cj] = (int16_t)i;
        s.dep[cj] = (int16_t)(s.dep[i] + 1);
        s.known[cj] = 1;
        ch = true;
      } else if (kj && !ki) {
        s.u[i] = s.ac[e] - s.v[j];
        s.parc[i] = (int16_t)e;
        s.par[i] = (int16_t)cj;
        s.dep[i] = (int16_t)(s.dep[cj] + 1);
        s.known[i] = 1;
        ch = true;
      }
    }
    wsync();
    if (!__any(ch)) break;
  }
  // the ancestor of q `up` levels above (0 <= up < 128), by the tables
  auto lift = [&](int q, int up) {
#pragma unroll
    for (int k = 0; k < kLevels; ++k)
      if ((up >> k) & 1) q = s.anc[k][q];
    return q;
  };
  // the common ancestor of a and b
  auto lca = [&](int x, int y) {
    if (s.dep[x] < s.dep[y]) {
      const int t = x;
      x = y;
      y = t;
    }
    x = lift(x, s.dep[x] - s.dep[y]);
    if (x == y) return x;
#pragma unroll
    for (int k = kLevels - 1; k >= 0; --k) {
      const int ax = s.anc[k][x], ay = s.anc[k][y];
      if (ax != ay) {
        x = ax;
        y = ay;
      }
    }
    return (int)s.anc[0][x];
  };
  for (;;) {
    // pricing: most negative reduced cost, ties to the lowest cell
    double best = 0.0;
    int bc = 0x7fffffff;
    for (int e = lane; e < m * mk; e += 64) {
      const int i = e % m, j = e / m;
      const double rc = C[e] - s.u[i] - s.v[j];
      if (rc < best || (rc == best && e < bc)) {
        best = rc;
        bc = e;
      }
    }
    for (int off2 = 32; off2 > 0; off2 >>= 1) {
      const double ob = __shfl_xor(best, off2);
      const int oc = __shfl_xor(bc, off2);
      if (ob < best || (ob == best && oc < bc)) {
        best = ob;
        bc = oc;
      }
    }
    if (!(best < tol)) break;  // optimal
    if (piv >= a.max_pivots) {
      capped = true;
      break;
    }
    ++piv;
    const int ie = bc % m, je = bc / m;
    // ancestor tables of the current tree
    for (int q = lane; q < nn; q += 64)
      s.anc[0][q] = s.par[q] < 0 ? (int16_t)q : s.par[q];
    wsync();
#pragma unroll
    for (int k = 1; k < kLevels; ++k) {
      for (int q = lane; q < nn; q += 64) s.anc[k][q] = s.anc[k - 1][s.anc[k - 1][q]];
      wsync();
    }
    // the cycle: nodes strictly below the common ancestor on the paths from
    // the entering cell's column (side 0) and row (side 1); a node's arc to
    // its parent is on the cycle, "-" at even positions from the cell
    const int nA = m + je, nB = ie;
    const int top = lca(nA, nB);
    const int dtop = s.dep[top];
    int side[2] = {-1, -1}, pos[2] = {0, 0};
    double lf = 1e300;
    int lkey = 0x7fffffff, lnode = -1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = lane + 64 * h;
      if (q >= nn) continue;
      const int dq = s.dep[q];
      if (dq > dtop) {
        if (dq <= s.dep[nA] && lift(nA, s.dep[nA] - dq) == q) {
          side[h] = 0;
          pos[h] = s.dep[nA] - dq;
        } else if (dq <= s.dep[nB] && lift(nB, s.dep[nB] - dq) == q) {
          side[h] = 1;
          pos[h] = s.dep[nB] - dq;
        }
      }
      if (side[h] >= 0 && (pos[h] & 1) == 0) {
        const double f = s.af[s.parc[q]];
        const int key = side[h] * 256 + pos[h];
        if (f < lf || (f == lf && key < lkey)) {
          lf = f;
          lkey = key;
          lnode = q;
        }
      }
    }
    // leaving cell: least flow among the "-" cells, first along the paths
    for (int off2 = 32; off2 > 0; off2 >>= 1) {
      const double of = __shfl_xor(lf, off2);
      const int ok = __shfl_xor(lkey, off2);
      const int on = __shfl_xor(lnode, off2);
      if (of < lf || (of == lf && ok < lkey)) {
        lf = of;
        lkey = ok;
        lnode = on;
      }
    }
    if (lnode < 0) {  // no "-" cell: the basis is not a spanning tree
      capped = true;
      break;
    }
    const double th = lf;
    const int cl = lnode;                 // the leaving arc's lower node
    const int lside = lkey >> 8, lpos = lkey & 255;
    const int lv = s.parc[cl];
    const int es = lside == 0 ? nA : nB;  // entering endpoint below it
    const int other = lside == 0 ? nB : nA;
    const int dcl = s.dep[cl], des = s.dep[es], dot = s.dep[other];
    // phase 1 (reads of the old tree): flows, subtree, new depths, the
    // re-hung path
    int wpar[2] = {-1, -1}, wparc[2] = {-1, -1}, ndep[2] = {-1, -1};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = lane + 64 * h;
      if (q >= nn) continue;
      const int dq = s.dep[q];
      if (dq >= dcl && lift(q, dq - dcl) == cl)
        ndep[h] = dot + 1 + dq + des - 2 * s.dep[lca(q, es)];
      if (side[h] == lside && pos[h] <= lpos && q != cl) {
        wpar[h] = s.par[q];
        wparc[h] = s.parc[q];
      }
    }
    wsync();
    // phase 2 (writes): flows on the cycle, potentials and depths of the
    // subtree, parents along the re-hung path, then the entering cell in
    // the leaving cell's slot
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = lane + 64 * h;
      if (q >= nn) continue;
      if (side[h] >= 0) {
        const int e = s.parc[q];
        const double f = s.af[e] + ((pos[h] & 1) ? th : -th);
        s.af[e] = f > 0.0 ? f : 0.0;
      }
      if (ndep[h] >= 0) {
        // the entering endpoint's side moves by +best, the other by -best
        const bool rowq = q < m;
        const double sh = (rowq == (es < m)) ? best : -best;
        if (rowq)
          s.u[q] += sh;
        else
          s.v[q - m] += sh;
        s.dep[q] = (int16_t)ndep[h];
      }
    }
    wsync();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (wpar[h] >= 0) {
        const int q = lane + 64 * h;
        s.par[wpar[h]] = (int16_t)q;
        s.parc[wpar[h]] = (int16_t)wparc[h];
      }
    }
    if (lane == 0) {
      s.par[es] = (int16_t)other;
      s.parc[es] = (int16_t)lv;
      s.ai[lv] = (int16_t)ie;
      s.aj[lv] = (int16_t)je;
      s.af[lv] = th;
      s.ac[lv] = C[bc];
    }
    wsync();
  }
  // plan (basic cells carry their flow), value and projected row duals
  const int64_t pb0 = a.pofs[k];
  double vsum = 0.0;
  for (int e = lane; e < m * mk; e += 64) {
    double f = 0.0;
    for (int q = 0; q < na; ++q)
      if (s.ai[q] == e % m && s.aj[q] == e / m) f = s.af[q];
    vsum = fma(f, C[e], vsum);
    if (a.f64) {
      reinterpret_cast<double*>(a.P1)[pb0 + e] = f;
      reinterpret_cast<double*>(a.P2)[pb0 + e] = f;
    } else {
      reinterpret_cast<float*>(a.P1)[pb0 + e] = (float)f;
      reinterpret_cast<float*>(a.P2)[pb0 + e] = (float)f;
    }
  }
  for (int off2 = 32; off2 > 0; off2 >>= 1) vsum += __shfl_xor(vsum, off2);
  double um = 0.0;
  for (int i = 0; i < m; ++i) um += s.u[i];
  um /= (double)m;
  for (int i = lane; i < a.MP; i += 64)
    a.U[k * a.MP + i] = i < m ? s.u[i] - um : 0.0;
  if (lane == 0) {
    a.val[k] = vsum;
    if (capped) atomicAdd(a.fail, 1);
    atomicAdd(a.pivots, (unsigned long long)piv);
  }
}

struct StepArgs {
  const int32_t* work;     // instances sorted by cluster
  const d2k::Chunk* chunks;
  const int2* ctab;        // per cluster {first chunk, chunks}
  const double* U;         // N x MP
  const double* val;       // N
  double* s;               // K x MP log-weights (centred)
  double* wc;              // K x MP weights (out)
  double* trace;           // K objective values of this iteration
  double alpha, zeta;
  int m, MP;
};

// One subgradient step per cluster (one workgroup each): the mean over the
// members of the projected duals (Eq. (dualvar)), the softmax chain rule,
// the step of Eq. (stepsize), the rescaling to zero mean and the new
// weights; the members' mean LP value goes to the objective trace.  Member
// sums in a fixed order (strided per thread, then a tree in LDS).
__global__ void __launch_bounds__(256) k_sg_step(StepArgs a) {
  __shared__ double s_red[256];
  __shared__ double s_g[64];
  const int c = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int2 ct = a.ctab[c];
  if (ct.y == 0) return;  // empty cluster: the centroid stays
  const int b0 = a.chunks[ct.x].begin;
  const int b1 = a.chunks[ct.x + ct.y - 1].end;
  const double inv = 1.0 / (double)(b1 - b0);
  auto reduce = [&](double v) {
    s_red[tid] = v;
    __syncthreads();
    for (int h = nt / 2; h > 0; h >>= 1) {
      if (tid < h) s_red[tid] += s_red[tid + h];
      __syncthreads();
    }
    const double r = s_red[0];
    __syncthreads();
    return r;
  };
  for (int i = 0; i < a.m; ++i) {
    double acc = 0.0;
    for (int p = b0 + tid; p < b1; p += nt)
      acc += a.U[(int64_t)a.work[p] * a.MP + i];
    const double g = reduce(acc) * inv;
    if (tid == 0) s_g[i] = g;
  }
  double fv = 0.0;
  for (int p = b0 + tid; p < b1; p += nt) fv += a.val[a.work[p]];
  const double F = reduce(fv) * inv;
  if (tid == 0) {
    double* sq = a.s + (int64_t)c * a.MP;
    double* wq = a.wc + (int64_t)c * a.MP;
    a.trace[c] = F;
    double wg = 0.0;
    for (int i = 0; i < a.m; ++i) wg += wq[i] * s_g[i];
    double gs[64];
    double nrm = 0.0;
    for (int i = 0; i < a.m; ++i) {
      gs[i] = wq[i] * (s_g[i] - wg);
      nrm += gs[i] * gs[i];
    }
    nrm = sqrt(nrm);
    const double sig = nrm > 0.0 ? fmin(a.alpha / nrm, a.zeta) : 0.0;
    double mean = 0.0;
    for (int i = 0; i < a.m; ++i) {
      sq[i] -= sig * gs[i];
      mean += sq[i];
    }
    mean /= (double)a.m;
    double mx = -1e300;
    for (int i = 0; i < a.m; ++i) {
      sq[i] -= mean;
      mx = fmax(mx, sq[i]);
    }
    double z = 0.0;
    for (int i = 0; i < a.m; ++i) z += exp(sq[i] - mx);
    for (int i = 0; i < a.m; ++i) wq[i] = exp(sq[i] - mx) / z;
  }
}

// s = log w - mean(log w) and w = softmax(s) for every cluster (the start of
// a subgradient run; empty clusters too, whose weights stay a softmax of
// themselves).
__global__ void __launch_bounds__(64)
    k_sg_init(double* s, double* wc, int K, int m, int MP) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  double* sq = s + (int64_t)c * MP;
  double* wq = wc + (int64_t)c * MP;
  double mean = 0.0;
  for (int i = 0; i < m; ++i) {
    sq[i] = log(fmax(wq[i], 1e-300));
    mean += sq[i];
  }
  mean /= (double)m;
  double mx = -1e300;
  for (int i = 0; i < m; ++i) {
    sq[i] -= mean;
    mx = fmax(mx, sq[i]);
  }
  double z = 0.0;
  for (int i = 0; i < m; ++i) z += exp(sq[i] - mx);
  for (int i = 0; i < m; ++i) wq[i] = exp(sq[i] - mx) / z;
}

}  // namespace d2s

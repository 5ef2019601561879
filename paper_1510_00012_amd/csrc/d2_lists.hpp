// Device construction of a round's work list (the cluster-sorted instance
// order, the workgroup chunks and the per-cluster tables the B-ADMM
// kernels read), so that the labels written by the assignment never travel
// to the host between the assignment and the centroid update.
//
// Key of instance k: g = label[k] * nbk + bucket[k] (bucket = the slot
// bucket of its support size).  The list is a stable counting sort by key:
// instances of one key keep their index order.  Tiles of kTile instances,
// one wavefront each:
//   k_list_count   per-tile key histograms (instances and support points)
//                  in LDS, written as row t of tcnt / tsum; warm flags.
//   k_list_tiles   per key, exclusive scan of the tile counts over tiles
//                  (in place: row t becomes the tile's offset within the
//                  key), key totals.
//   k_list_layout  one workgroup: key starts, chunk counts and first chunk
//                  per key, per-bucket chunk offsets, per-cluster tables
//                  (first chunk / chunk count, 1 / N_c, 1 / (m sum m_k)),
//                  the chunk total and the per-bucket chunk counts.
//   k_list_scatter per tile, the instances placed in index order: a
//                  wavefront ranks its 64 lanes within their keys (ballot
//                  groups) and advances an LDS running offset per key.
//   k_list_chunks  one thread per chunk: cluster, range and bucket, and
//                  its entry in its bucket's chunk list.
// The result equals the host construction entry for entry.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "d2_kernels.hpp"

namespace d2l {

constexpr int kTile = 4096;     // instances per tile (one wavefront)
constexpr int kMaxKeys = 4096;  // keys handled on the device (LDS limit)

__global__ void __launch_bounds__(64)
    k_list_count(const int32_t* __restrict__ labels,
                 const uint8_t* __restrict__ bkt,
                 const int64_t* __restrict__ off, int64_t N, int nbk, int G,
                 int32_t* __restrict__ tcnt, int32_t* __restrict__ tsum,
                 const int32_t* __restrict__ cache_labels,
                 uint8_t* __restrict__ warm) {
  __shared__ int s_c[kMaxKeys];
  __shared__ int s_s[kMaxKeys];
  const int t = blockIdx.x, l = threadIdx.x;
  for (int g = l; g < G; g += 64) s_c[g] = s_s[g] = 0;
  __syncthreads();
  const int64_t k0 = (int64_t)t * kTile;
  const int64_t k1 = k0 + kTile < N ? k0 + kTile : N;
  for (int64_t k = k0 + l; k < k1; k += 64) {
    const int q = labels[k];
    const int g = q * nbk + bkt[k];
    atomicAdd(&s_c[g], 1);
    atomicAdd(&s_s[g], (int)(off[k + 1] - off[k]));
    warm[k] = cache_labels ? (uint8_t)(cache_labels[k] == q) : (uint8_t)0;
  }
  __syncthreads();
  for (int g = l; g < G; g += 64) {
    tcnt[(int64_t)t * G + g] = s_c[g];
    tsum[(int64_t)t * G + g] = s_s[g];
  }
}

__global__ void __launch_bounds__(256)
    k_list_tiles(int32_t* __restrict__ tcnt, const int32_t* __restrict__ tsum,
                 int ntiles, int G, int64_t* __restrict__ kcnt,
                 int64_t* __restrict__ ksum) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  int64_t run = 0, s = 0;
  for (int t = 0; t < ntiles; ++t) {
    const int64_t e = (int64_t)t * G + g;
    const int c = tcnt[e];
    tcnt[e] = (int32_t)run;
    run += c;
    s += tsum[e];
  }
  kcnt[g] = run;
  ksum[g] = s;
}

// Exclusive scan of v[0..n) in place by one workgroup (blockDim.x threads,
// s_tmp of blockDim.x entries); returns the total on every thread.
__device__ inline int64_t block_scan(int64_t* v, int n, int64_t* s_tmp) {
  const int tid = threadIdx.x, nt = blockDim.x;
  // each thread scans a contiguous run of ceil(n / nt) entries
  const int per = (n + nt - 1) / nt;
  const int a = tid * per < n ? tid * per : n;
  const int b = a + per < n ? a + per : n;
  int64_t loc = 0;
  for (int i = a; i < b; ++i) loc += v[i];
  s_tmp[tid] = loc;
  __syncthreads();
  if (tid == 0) {
    int64_t run = 0;
    for (int i = 0; i < nt; ++i) {
      const int64_t x = s_tmp[i];
      s_tmp[i] = run;
      run += x;
    }
    s_tmp[nt] = run;
  }
  __syncthreads();
  int64_t run = s_tmp[tid];
  for (int i = a; i < b; ++i) {
    const int64_t x = v[i];
    v[i] = run;
    run += x;
  }
  const int64_t total = s_tmp[nt];
  __syncthreads();
  return total;
}

struct LayoutArgs {
  const int64_t* kcnt;  // G instances per key
  const int64_t* ksum;  // G support points per key
  int64_t* kstart;      // G out: first list position of each key
  int64_t* kchunk;      // G out: first chunk of each key
  int64_t* kbofs;       // G out: position in its bucket's chunk list
  int2* ctab;           // K out: {first chunk, chunks}
  double* ninv;         // K out
  double* cinv;         // K out
  int* nch;             // out: total chunks
  int* bcnt;            // 6 out: chunks per bucket
  int K, nbk, G, chunk, m;
};

__global__ void __launch_bounds__(1024) k_list_layout(LayoutArgs a) {
  __shared__ int64_t s_tmp[1025];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int g = tid; g < a.G; g += nt) {
    a.kstart[g] = a.kcnt[g];
    a.kchunk[g] = (a.kcnt[g] + a.chunk - 1) / a.chunk;
  }
  __syncthreads();
  block_scan(a.kstart, a.G, s_tmp);
  // chunks per key, then per bucket in cluster order
  for (int g = tid; g < a.G; g += nt) a.kbofs[g] = a.kchunk[g];
  __syncthreads();
  const int64_t total = block_scan(a.kchunk, a.G, s_tmp);
  if (tid < a.nbk) {
    int64_t run = 0;
    for (int q = 0; q < a.K; ++q) {
      const int g = q * a.nbk + tid;
      const int64_t x = a.kbofs[g];
      a.kbofs[g] = run;
      run += x;
    }
    a.bcnt[tid] = (int)run;
  } else if (tid < 6) {
    a.bcnt[tid] = 0;
  }
  if (tid == 0) *a.nch = (int)total;
  for (int q = tid; q < a.K; q += nt) {
    int64_t n = 0, cols = 0;
    for (int b = 0; b < a.nbk; ++b) {
      n += a.kcnt[q * a.nbk + b];
      cols += a.ksum[q * a.nbk + b];
    }
    const int64_t first = a.kchunk[q * a.nbk];
    const int64_t next = q + 1 < a.K ? a.kchunk[(q + 1) * a.nbk] : total;
    a.ctab[q] = make_int2((int)first, (int)(next - first));
    a.ninv[q] = n > 0 ? 1.0 / (double)n : 0.0;
    a.cinv[q] = n > 0 ? 1.0 / ((double)a.m * (double)cols) : 0.0;
  }
}

__global__ void __launch_bounds__(64)
    k_list_scatter(const int32_t* __restrict__ labels,
                   const uint8_t* __restrict__ bkt, int64_t N, int nbk, int G,
                   const int32_t* __restrict__ tbase,
                   const int64_t* __restrict__ kstart,
                   int32_t* __restrict__ work) {
  __shared__ int64_t s_run[kMaxKeys];
  const int t = blockIdx.x, l = threadIdx.x;
  for (int g = l; g < G; g += 64)
    s_run[g] = kstart[g] + tbase[(int64_t)t * G + g];
  __syncthreads();
  const int64_t k0 = (int64_t)t * kTile;
  const int64_t k1 = k0 + kTile < N ? k0 + kTile : N;
  const unsigned long long below = (1ull << l) - 1ull;
  for (int64_t base = k0; base < k1; base += 64) {
    const int64_t k = base + l;
    const bool valid = k < k1;
    const int g = valid ? labels[k] * nbk + bkt[k] : -1;
    // rank among the lanes of the same key below this lane
    unsigned long long todo = __ballot(valid);
    int rank = 0, size = 0;
    while (todo) {
      const int lead = __builtin_ctzll(todo);
      const int gl = __shfl(g, lead);
      const unsigned long long grp = __ballot(valid && g == gl);
      if (valid && g == gl) {
        rank = __popcll(grp & below);
        size = __popcll(grp);
      }
      todo &= ~grp;
    }
    int64_t dst = 0;
    if (valid) dst = s_run[g] + rank;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) s_run[g] += size;
    __builtin_amdgcn_wave_barrier();
    if (valid) work[dst] = (int32_t)k;
  }
}

struct ChunkArgs {
  const int64_t* kcnt;
  const int64_t* kstart;
  const int64_t* kchunk;
  const int64_t* kbofs;
  const int* nch;
  d2k::Chunk* chunks;
  int32_t* blist;
  int boff[6];
  int G, nbk, chunk, cap;
};

__global__ void __launch_bounds__(256) k_list_chunks(ChunkArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.cap || c >= *a.nch) return;
  // the key of chunk c: the largest g with kchunk[g] <= c (keys without
  // chunks share the next key's first chunk and are skipped this way)
  int lo = 0, hi = a.G - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (a.kchunk[mid] <= c)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int g = lo;
  const int64_t i = c - a.kchunk[g];
  const int b = g % a.nbk;
  d2k::Chunk ck;
  ck.cluster = g / a.nbk;
  const int64_t begin = a.kstart[g] + i * a.chunk;
  const int64_t end = a.kstart[g] + a.kcnt[g];
  ck.begin = (int32_t)begin;
  ck.end = (int32_t)(begin + a.chunk < end ? begin + a.chunk : end);
  ck.pad = b;
  a.chunks[c] = ck;
  a.blist[a.boff[b] + a.kbofs[g] + i] = c;
}

}  // namespace d2l

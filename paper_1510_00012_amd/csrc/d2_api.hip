// C ABI implementation (include/d2.h): context, validation, work lists, the
// B-ADMM launch schedule, centroid initialisation and the clustering loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/d2.h"
#include "d2_ctx.hpp"
#include "d2_kernels.hpp"
#include "d2_lists.hpp"
#include "d2_lp.hpp"

static const char* kKindNames[kKinds] = {"rho_cost", "init_a", "iter_ba",
                                         "b_final", "xnum_only", "assign",
                                         "finalize"};

namespace {

int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}
int pad_rows(int m) { return 1 << std::max(3, ilog2(m)); }

}  // namespace

// kernel tables, filled by the per-type translation units
void d2k_fill_f32(d2k::KernTable<float>* t);
void d2k_fill_f32w(d2k::KernTable<float>* t);
void d2k_fill_f32p(d2k::KernTable<float>* t);
void d2k_fill_f64(d2k::KernTable<double>* t);
void d2k_fill_f64w(d2k::KernTable<double>* t);
void d2k_fill_f64p(d2k::KernTable<double>* t);
void d2k_fill_fin(d2k::FinFn* f);

namespace {

template <typename T> const d2k::KernTable<T>& kern();
template <> const d2k::KernTable<float>& kern<float>() {
  static const d2k::KernTable<float> t = [] {
    d2k::KernTable<float> x;
    d2k_fill_f32(&x);
    d2k_fill_f32w(&x);
    d2k_fill_f32p(&x);
    return x;
  }();
  return t;
}
template <> const d2k::KernTable<double>& kern<double>() {
  static const d2k::KernTable<double> t = [] {
    d2k::KernTable<double> x;
    d2k_fill_f64(&x);
    d2k_fill_f64w(&x);
    d2k_fill_f64p(&x);
    return x;
  }();
  return t;
}
const d2k::FinFn* fin_table() {
  static d2k::FinFn f[4] = {};
  static bool init = false;
  if (!init) {
    d2k_fill_fin(f);
    init = true;
  }
  return f;
}

}  // namespace

namespace {

bool finite_all(const double* p, size_t n) {
  for (size_t q = 0; q < n; ++q)
    if (!std::isfinite(p[q])) return false;
  return true;
}

template <typename P> void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

d2_status dalloc(d2_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return c->fail(D2_ENOMEM, "hipMalloc(" + std::to_string(bytes) +
                                  "): " + hipGetErrorString(e));
  }
  return D2_OK;
}

void drop_graph(d2_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->graph_key.clear();
}

void free_plans(d2_ctx* c) {
  drop_graph(c);
  dfree(c->d_P1);
  dfree(c->d_P2);
  dfree(c->d_L);
  dfree(c->d_C);
  c->have_cache = false;
}

void free_lists(d2_ctx* c) {
  dfree(c->d_work);
  dfree(c->d_chunks);
  dfree(c->d_ctab);
  dfree(c->d_ninv);
  dfree(c->d_cinv);
  dfree(c->d_warm);
  dfree(c->d_part);
  dfree(c->d_partx);
  dfree(c->d_nch);
  dfree(c->d_blist);
  dfree(c->d_bcnt);
  c->nch_cap = 0;
  c->blist_cap = 0;
  c->nbk = 0;
  c->lists_valid = false;
  drop_graph(c);
}

void free_bounds(d2_ctx* c) {
  dfree(c->d_lbs);
  dfree(c->d_xref);
  dfree(c->d_dlt);
  c->lbs_valid = false;
}

void free_centroids(d2_ctx* c) {
  drop_graph(c);
  free_bounds(c);
  dfree(c->d_csym);
  c->h_csym.clear();
  dfree(c->d_rho_fix);
  c->rho_fix_K = 0;
  c->rho_fixed = false;
  dfree(c->d_cmu);
  dfree(c->d_crad);
  dfree(c->d_xct);
  dfree(c->d_xc);
  dfree(c->d_wc);
  dfree(c->d_xsave);
  dfree(c->d_wsave);
  dfree(c->d_rho);
  dfree(c->d_cnt);
  c->K = c->m = c->MP = 0;
}

void free_instances(d2_ctx* c) {
  free_bounds(c);
  dfree(c->d_off);
  dfree(c->d_pofs);
  if (c->borrowed) {
    c->d_X = c->d_W = nullptr;
    c->borrowed = false;
  }
  dfree(c->d_X);
  dfree(c->d_W);
  dfree(c->d_isym);
  dfree(c->d_D);
  c->sym = false;
  c->S = 0;
  dfree(c->d_cache_labels);
  dfree(c->d_prev_labels);
  dfree(c->d_nchg);
  dfree(c->d_bkt);
  c->bkt_MP = 0;
  c->bkt_pct = -1;
  dfree(c->d_tcnt);
  dfree(c->d_tsum);
  c->tcnt_cap = 0;
  dfree(c->d_keys);
  c->keys_cap = 0;
  dfree(c->d_dall);
  c->dall_cap = 0;
  dfree(c->d_sgU);
  dfree(c->d_sgval);
  dfree(c->d_sgs);
  dfree(c->d_sgfail);
  dfree(c->d_sgpiv);
  c->sg_N = 0;
  c->sg_KMP = 0;
  c->hlab_ok = c->hcache_ok = true;
  c->cache_gen = ~0ull;
  dfree(c->d_labels);
  dfree(c->d_best);
  dfree(c->d_pairs);
  c->last_pairs = 0;
  dfree(c->d_alist);
  c->alist_MP = 0;
  c->cls_MP = 0;
  dfree(c->d_trace);
  dfree(c->d_rtrace);
  c->trace_cap = 0;
  c->N = c->n = 0;
  c->have_labels = false;
  free_plans(c);
  free_lists(c);
}

template <typename T>
d2_status upload_conv(d2_ctx* c, void* dst, const double* src, size_t count) {
  std::vector<T> tmp(count);
  for (size_t q = 0; q < count; ++q) tmp[q] = (T)src[q];
  HIPCHK(c, hipMemcpy(dst, tmp.data(), count * sizeof(T),
                      hipMemcpyHostToDevice));
  return D2_OK;
}

template <typename T>
d2_status download_conv(d2_ctx* c, double* dst, const void* src,
                        size_t count) {
  std::vector<T> tmp(count);
  HIPCHK(c, hipMemcpy(tmp.data(), src, count * sizeof(T),
                      hipMemcpyDeviceToHost));
  for (size_t q = 0; q < count; ++q) dst[q] = (double)tmp[q];
  return D2_OK;
}

// Sec. 5, Eq. (merge): pairwise merge down to m points.  Ties go to the
// lexicographically smallest pair; the merged point keeps the first slot.
void merge_support(int mk, int d, const double* y, const double* wy, int m,
                   double* x, double* w) {
  std::vector<double> px(y, y + (size_t)mk * d), pw(wy, wy + mk);
  int cnt = mk;
  while (cnt > m) {
    int ba = 0, bb = 1;
    double best = INFINITY;
    for (int p = 0; p < cnt; ++p)
      for (int q = p + 1; q < cnt; ++q) {
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
          double df = px[(size_t)p * d + t] - px[(size_t)q * d + t];
          s += df * df;
        }
        double ws = pw[p] + pw[q];
        double cr = ws > 0.0 ? pw[p] * pw[q] * s / ws : 0.0;
        if (cr < best) {
          best = cr;
          ba = p;
          bb = q;
        }
      }
    double ws = pw[ba] + pw[bb];
    for (int t = 0; t < d; ++t) {
      double v = ws > 0.0 ? (pw[ba] * px[(size_t)ba * d + t] +
                             pw[bb] * px[(size_t)bb * d + t]) /
                                ws
                          : px[(size_t)ba * d + t];
      px[(size_t)ba * d + t] = v;
    }
    pw[ba] = ws;
    px.erase(px.begin() + (size_t)bb * d, px.begin() + (size_t)(bb + 1) * d);
    pw.erase(pw.begin() + bb);
    --cnt;
  }
  std::copy(px.begin(), px.begin() + (size_t)m * d, x);
  std::copy(pw.begin(), pw.begin() + m, w);
}

d2_status ensure_centroid_bufs(d2_ctx* c, int K, int m) {
  if (c->K == K && c->m == m && c->d_xc) return D2_OK;
  free_centroids(c);
  free_plans(c);
  free_lists(c);
  c->K = K;
  c->m = m;
  c->MP = pad_rows(m);
  d2_status s;
  if ((s = dalloc(c, (void**)&c->d_xc, sizeof(double) * K * c->MP * c->d)))
    return s;
  if ((s = dalloc(c, (void**)&c->d_wc, sizeof(double) * K * c->MP))) return s;
  if ((s = dalloc(c, (void**)&c->d_xsave,
                  sizeof(double) * K * c->MP * c->d)))
    return s;
  if ((s = dalloc(c, (void**)&c->d_wsave, sizeof(double) * K * c->MP)))
    return s;
  if ((s = dalloc(c, (void**)&c->d_rho, sizeof(double) * K))) return s;
  if ((s = dalloc(c, (void**)&c->d_cnt, sizeof(int) * K))) return s;
  HIPCHK(c, hipMemset(c->d_cnt, 0, sizeof(int) * K));
  HIPCHK(c, hipMemset(c->d_xc, 0, sizeof(double) * K * c->MP * c->d));
  HIPCHK(c, hipMemset(c->d_wc, 0, sizeof(double) * K * c->MP));
  return D2_OK;
}

d2_status check_limits(d2_ctx* c, int m) {
  if (m < 1 || m > 64) return c->fail(D2_EINVAL, "m must be in [1, 64]");
  int MP = pad_rows(m);
  int cps = 64 / MP;
  int slots = (c->mk_max + cps - 1) / cps;
  if (slots > 32)
    return c->fail(D2_EINVAL, "m_k * pad(m) exceeds 2048 entries (m_k max " +
                                  std::to_string(c->mk_max) + ")");
  if ((int64_t)MP * (c->d + 1) > 8192)
    return c->fail(D2_EINVAL, "pad(m) * (d + 1) exceeds 8192");
  return D2_OK;
}

d2_status set_centroids_host(d2_ctx* c, int K, int m, const double* Xc,
                             const double* Wc) {
  d2_status s = ensure_centroid_bufs(c, K, m);
  if (s) return s;
  const int MP = c->MP, d = c->d;
  std::vector<double> hx((size_t)K * MP * d, 0.0), hw((size_t)K * MP, 0.0);
  for (int q = 0; q < K; ++q) {
    double sum = 0.0;
    for (int i = 0; i < m; ++i) sum += Wc[(size_t)q * m + i];
    for (int i = 0; i < m; ++i) {
      hw[(size_t)q * MP + i] = Wc[(size_t)q * m + i] / sum;
      for (int t = 0; t < d; ++t)
        hx[((size_t)q * MP + i) * d + t] = Xc[((size_t)q * m + i) * d + t];
    }
  }
  HIPCHK(c, hipMemcpy(c->d_xc, hx.data(), hx.size() * 8,
                      hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_wc, hw.data(), hw.size() * 8,
                      hipMemcpyHostToDevice));
  return D2_OK;
}

struct Upload {
  void* dst;
  const void* src;
  size_t bytes;
};

// Copy the sources into pinned staging memory and issue the transfers on
// the context's stream without waiting (later launches on the stream see
// the data).  The staging memory is reused once the previous batch ended.
d2_status stage_uploads(d2_ctx* c, const std::vector<Upload>& ups) {
  size_t total = 0;
  for (const Upload& u : ups) total += (u.bytes + 255) / 256 * 256;
  if (c->stage_ev) HIPCHK(c, hipEventSynchronize(c->stage_ev));
  if (total > c->stage_cap) {
    if (c->h_stage) HIPCHK(c, hipHostFree(c->h_stage));
    c->h_stage = nullptr;
    c->stage_cap = 0;
    HIPCHK(c, hipHostMalloc((void**)&c->h_stage, total));
    c->stage_cap = total;
  }
  if (!c->stage_ev) HIPCHK(c, hipEventCreateWithFlags(&c->stage_ev,
                                                      hipEventDisableTiming));
  size_t o = 0;
  for (const Upload& u : ups) {
    std::memcpy(c->h_stage + o, u.src, u.bytes);
    HIPCHK(c, hipMemcpyAsync(u.dst, c->h_stage + o, u.bytes,
                             hipMemcpyHostToDevice, c->stream));
    o += (u.bytes + 255) / 256 * 256;
  }
  HIPCHK(c, hipEventRecord(c->stage_ev, c->stream));
  return D2_OK;
}

// Slot class of an instance: log2 of the register slots (columns per lane)
// its tile needs, i.e. the hot-kernel specialisation R = 1 << class.
int slot_class(const d2_ctx* c, int64_t k) {
  const int cps = 64 / c->MP;
  const int mk = (int)(c->h_off[k + 1] - c->h_off[k]);
  return ilog2(std::max(1, (mk + cps - 1) / cps));
}

// Bucket launch capacities that hold for any labels: bucket b never has
// more than ceil(instances of b / chunk) + K chunks (one partial chunk per
// cluster), and the chunk total never exceeds ceil(N / chunk) + 6 K.  A
// captured launch sequence therefore stays valid across rounds.  Also
// (re)allocates the list buffers for those capacities.
d2_status list_capacities(d2_ctx* c, int nbk, const std::vector<int>& bR,
                          const int64_t* inst_b) {
  const int K = c->K;
  const int64_t N = c->N;
  const int CH = c->chunk_inst;
  const int cap = (int)((N + CH - 1) / CH) + K * 6;
  if (cap > c->nch_cap || !c->d_work) {
    free_lists(c);
    d2_status s;
    c->nch_cap = cap;
    if ((s = dalloc(c, (void**)&c->d_work, sizeof(int32_t) * N))) return s;
    if ((s = dalloc(c, (void**)&c->d_chunks, sizeof(d2k::Chunk) * cap)))
      return s;
    if ((s = dalloc(c, (void**)&c->d_ctab, sizeof(int2) * K))) return s;
    if ((s = dalloc(c, (void**)&c->d_ninv, sizeof(double) * K))) return s;
    if ((s = dalloc(c, (void**)&c->d_cinv, sizeof(double) * K))) return s;
    if ((s = dalloc(c, (void**)&c->d_warm, N))) return s;
    if ((s = dalloc(c, (void**)&c->d_part,
                    sizeof(double) * 2 * cap * (c->MP + 2))))
      return s;
    if ((s = dalloc(c, (void**)&c->d_nch, sizeof(int)))) return s;
    if ((s = dalloc(c, (void**)&c->d_bcnt, sizeof(int) * 6))) return s;
    if ((s = dalloc(c, (void**)&c->d_partx,
                    sizeof(double) * 2 * cap * c->MP * (c->d + 1))))
      return s;
  }
  int want[6] = {0, 0, 0, 0, 0, 0};
  for (int b = 0; b < nbk; ++b)
    want[b] = (int)((inst_b[b] + CH - 1) / CH) + K;
  bool same = nbk == c->nbk;
  for (int b = 0; same && b < 6; ++b)
    same = (b < nbk ? bR[b] : 0) == c->bk_R[b] && want[b] == c->bk_cap[b];
  if (!same) {
    drop_graph(c);
    int total = 0;
    for (int b = 0; b < 6; ++b) {
      c->bk_R[b] = b < nbk ? bR[b] : 0;
      c->bk_cap[b] = want[b];
      c->bk_off[b] = total;
      total += want[b];
    }
    c->nbk = nbk;
    if (total > c->blist_cap) {
      dfree(c->d_blist);
      d2_status s = dalloc(c, (void**)&c->d_blist, sizeof(int32_t) * total);
      if (s) return s;
      c->blist_cap = total;
    }
  }
  return D2_OK;
}

// The work list built on the device from the device labels (d2_lists.hpp):
// the same lists as the host construction below, entry for entry.
d2_status build_lists_device(d2_ctx* c, bool warm_start, int nbk,
                             const std::vector<int>& bR, const int* bidx_of) {
  const int K = c->K;
  const int64_t N = c->N;
  const int G = K * nbk;
  d2_status s;
  // per-instance bucket, for this pad(m) and merge threshold
  if (c->bkt_MP != c->MP || c->bkt_pct != c->bucket_min_pct || !c->d_bkt) {
    std::vector<uint8_t> hb(N);
    for (int64_t k = 0; k < N; ++k) hb[k] = (uint8_t)bidx_of[c->h_cls[k]];
    if (!c->d_bkt && (s = dalloc(c, (void**)&c->d_bkt, N))) return s;
    HIPCHK(c, hipMemcpy(c->d_bkt, hb.data(), N, hipMemcpyHostToDevice));
    c->bkt_MP = c->MP;
    c->bkt_pct = c->bucket_min_pct;
  }
  int64_t inst_b[6] = {0, 0, 0, 0, 0, 0};
  for (int q = 0; q < 6; ++q) inst_b[bidx_of[q]] += c->cls_cnt[q];
  if ((s = list_capacities(c, nbk, bR, inst_b))) return s;
  const int ntiles = (int)((N + d2l::kTile - 1) / d2l::kTile);
  if ((int64_t)ntiles * G > c->tcnt_cap) {
    dfree(c->d_tcnt);
    dfree(c->d_tsum);
    c->tcnt_cap = 0;
    const size_t b = sizeof(int32_t) * (size_t)ntiles * G;
    if ((s = dalloc(c, (void**)&c->d_tcnt, b))) return s;
    if ((s = dalloc(c, (void**)&c->d_tsum, b))) return s;
    c->tcnt_cap = (int64_t)ntiles * G;
  }
  if (G > c->keys_cap) {
    dfree(c->d_keys);
    c->keys_cap = 0;
    if ((s = dalloc(c, (void**)&c->d_keys, sizeof(int64_t) * 5 * G)))
      return s;
    c->keys_cap = G;
  }
  int64_t* kcnt = c->d_keys;
  int64_t* ksum = kcnt + G;
  int64_t* kstart = ksum + G;
  int64_t* kchunk = kstart + G;
  int64_t* kbofs = kchunk + G;
  const bool any_warm = warm_start && c->have_cache;
  hipLaunchKernelGGL(d2l::k_list_count, dim3(ntiles), dim3(64), 0, c->stream,
                     c->d_labels, c->d_bkt, c->d_off, N, nbk, G, c->d_tcnt,
                     c->d_tsum, any_warm ? c->d_cache_labels : nullptr,
                     c->d_warm);
  HIPCHK(c, hipGetLastError());
  hipLaunchKernelGGL(d2l::k_list_tiles, dim3((G + 255) / 256), dim3(256), 0,
                     c->stream, c->d_tcnt, c->d_tsum, ntiles, G, kcnt, ksum);
  HIPCHK(c, hipGetLastError());
  d2l::LayoutArgs la;
  la.kcnt = kcnt;
  la.ksum = ksum;
  la.kstart = kstart;
  la.kchunk = kchunk;
  la.kbofs = kbofs;
  la.ctab = c->d_ctab;
  la.ninv = c->d_ninv;
  la.cinv = c->d_cinv;
  la.nch = c->d_nch;
  la.bcnt = c->d_bcnt;
  la.K = K;
  la.nbk = nbk;
  la.G = G;
  la.chunk = c->chunk_inst;
  la.m = c->m;
  hipLaunchKernelGGL(d2l::k_list_layout, dim3(1), dim3(1024), 0, c->stream,
                     la);
  HIPCHK(c, hipGetLastError());
  hipLaunchKernelGGL(d2l::k_list_scatter, dim3(ntiles), dim3(64), 0,
                     c->stream, c->d_labels, c->d_bkt, N, nbk, G, c->d_tcnt,
                     kstart, c->d_work);
  HIPCHK(c, hipGetLastError());
  d2l::ChunkArgs ca;
  ca.kcnt = kcnt;
  ca.kstart = kstart;
  ca.kchunk = kchunk;
  ca.kbofs = kbofs;
  ca.nch = c->d_nch;
  ca.chunks = c->d_chunks;
  ca.blist = c->d_blist;
  for (int b = 0; b < 6; ++b) ca.boff[b] = c->bk_off[b];
  ca.G = G;
  ca.nbk = nbk;
  ca.chunk = c->chunk_inst;
  ca.cap = c->nch_cap;
  hipLaunchKernelGGL(d2l::k_list_chunks, dim3((c->nch_cap + 255) / 256),
                     dim3(256), 0, c->stream, ca);
  HIPCHK(c, hipGetLastError());
  c->host_ctab = false;
  c->lists_valid = true;
  return D2_OK;
}

// Cluster-sorted work list, chunks and per-cluster tables for the labels.
// Inside a cluster, instances are ordered by slot bucket and every chunk
// holds one bucket, so a cluster's chunks stay contiguous (the per-cluster
// record sums are unchanged) while each bucket runs in a kernel sized for
// its own slot count.
d2_status build_lists(d2_ctx* c, bool warm_start) {
  const int K = c->K;
  const int64_t N = c->N;
  if (c->cls_MP != c->MP) {
    // slot class of every instance and the plan entries per class
    c->h_cls.resize(N);
    for (int q = 0; q < 6; ++q) {
      c->cls_ent[q] = 0.0;
      c->cls_cnt[q] = 0;
    }
    for (int64_t k = 0; k < N; ++k) {
      c->h_cls[k] = (uint8_t)slot_class(c, k);
      c->cls_ent[c->h_cls[k]] += (double)(c->h_off[k + 1] - c->h_off[k]);
      c->cls_cnt[c->h_cls[k]]++;
    }
    c->cls_MP = c->MP;
  }
  const uint8_t* cls = c->h_cls.data();
  // buckets: slot classes present, a class with fewer than
  // bucket_min_pct % of the entries joins the next larger bucket
  const double* ent = c->cls_ent;
  double tot = 0.0;
  for (int q = 0; q < 6; ++q) tot += ent[q];
  int bmap[6];
  std::vector<int> bR;
  {
    int cur = -1;
    for (int q = 5; q >= 0; --q) {
      if (ent[q] > 0 &&
          (cur < 0 || ent[q] * 100.0 >= c->bucket_min_pct * tot)) {
        cur = q;
        bR.insert(bR.begin(), 1 << q);
      }
      bmap[q] = cur;
    }
  }
  const int nbk = std::max<int>(1, (int)bR.size());
  if (bR.empty()) bR.push_back(1);
  int bidx_of[6] = {0, 0, 0, 0, 0, 0};
  for (int q = 0; q < 6; ++q)
    for (int b = 0; b < nbk; ++b)
      if (bmap[q] >= 0 && (1 << bmap[q]) == bR[b]) bidx_of[q] = b;
  if ((int64_t)K * nbk <= d2l::kMaxKeys)
    return build_lists_device(c, warm_start, nbk, bR, bidx_of);
  // many clusters: the list is built on the host from the host labels
  HIPCHK(c, c->sync_labels());
  if (warm_start && c->have_cache) HIPCHK(c, c->sync_cache_labels());
  // one pass: (cluster, bucket) key per instance and the counts
  std::vector<int64_t> cnt(K, 0), ncols(K, 0);
  std::vector<int64_t> kcnt((size_t)K * nbk, 0);
  c->h_key.resize(N);
  uint32_t* key = c->h_key.data();
  const int32_t* lab = c->h_labels.data();
  const int64_t* off = c->h_off.data();
  for (int64_t k = 0; k < N; ++k) {
    const int l = lab[k];
    const uint32_t g = (uint32_t)l * nbk + bidx_of[cls[k]];
    key[k] = g;
    cnt[l]++;
    ncols[l] += off[k + 1] - off[k];
    kcnt[g]++;
  }
  std::vector<int64_t> start((size_t)K * nbk + 1, 0);
  for (size_t q = 0; q < (size_t)K * nbk; ++q) start[q + 1] = start[q] + kcnt[q];
  c->h_work.resize(N);
  int32_t* work = c->h_work.data();
  {
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (int64_t k = 0; k < N; ++k) work[pos[key[k]]++] = (int32_t)k;
  }
  std::vector<d2k::Chunk> chunks;
  std::vector<std::vector<int32_t>> blists(nbk);
  c->h_ctab.assign(K, make_int2(0, 0));
  std::vector<double> ninv(K, 0.0), cinv(K, 0.0);
  const int CH = c->chunk_inst;
  for (int q = 0; q < K; ++q) {
    c->h_ctab[q].x = (int)chunks.size();
    for (int b = 0; b < nbk; ++b) {
      const size_t g = (size_t)q * nbk + b;
      for (int64_t e = start[g]; e < start[g + 1]; e += CH) {
        d2k::Chunk ck;
        ck.cluster = q;
        ck.begin = (int32_t)e;
        ck.end = (int32_t)std::min<int64_t>(e + CH, start[g + 1]);
        ck.pad = b;
        blists[b].push_back((int32_t)chunks.size());
        chunks.push_back(ck);
      }
    }
    c->h_ctab[q].y = (int)chunks.size() - c->h_ctab[q].x;
    if (cnt[q] > 0) {
      ninv[q] = 1.0 / (double)cnt[q];
      cinv[q] = 1.0 / ((double)c->m * (double)ncols[q]);
    }
  }
  c->nchunks = (int)chunks.size();
  {
    int64_t inst_b[6] = {0, 0, 0, 0, 0, 0};
    for (int q = 0; q < 6; ++q) inst_b[bidx_of[q]] += c->cls_cnt[q];
    d2_status s = list_capacities(c, nbk, bR, inst_b);
    if (s) return s;
  }
  for (int b = 0; b < nbk; ++b) c->bk_cnt[b] = (int)blists[b].size();
  for (int b = nbk; b < 6; ++b) c->bk_cnt[b] = 0;
  const bool any_warm = warm_start && c->have_cache;
  if (any_warm) {
    c->h_warm.resize(N);
    for (int64_t k = 0; k < N; ++k)
      c->h_warm[k] = lab[k] == c->h_cache_labels[k];
  } else {
    HIPCHK(c, hipMemsetAsync(c->d_warm, 0, N, c->stream));
  }
  std::vector<Upload> ups = {
      {c->d_work, work, sizeof(int32_t) * N},
      {c->d_chunks, chunks.data(),
       sizeof(d2k::Chunk) * std::max<size_t>(1, chunks.size())},
      {c->d_ctab, c->h_ctab.data(), sizeof(int2) * K},
      {c->d_ninv, ninv.data(), sizeof(double) * K},
      {c->d_cinv, cinv.data(), sizeof(double) * K},
      {c->d_nch, &c->nchunks, sizeof(int)},
      {c->d_bcnt, c->bk_cnt, sizeof(int) * 6}};
  if (any_warm) ups.push_back({c->d_warm, c->h_warm.data(), (size_t)N});
  for (int b = 0; b < nbk; ++b)
    if (!blists[b].empty())
      ups.push_back({c->d_blist + c->bk_off[b], blists[b].data(),
                     sizeof(int32_t) * blists[b].size()});
  d2_status su = stage_uploads(c, ups);
  if (su) return su;
  c->host_ctab = true;
  c->lists_valid = true;
  return D2_OK;
}

d2_status ensure_plans(d2_ctx* c) {
  if (c->d_P1) return D2_OK;
  // plan tile of instance k starts at pofs[k], a multiple of 32 elements
  c->h_pofs.assign(c->N + 1, 0);
  for (int64_t k = 0; k < c->N; ++k) {
    int64_t sz = (int64_t)c->m * (c->h_off[k + 1] - c->h_off[k]);
    c->h_pofs[k + 1] = c->h_pofs[k] + (sz + 31) / 32 * 32;
  }
  dfree(c->d_pofs);
  d2_status s0 = dalloc(c, (void**)&c->d_pofs, sizeof(int64_t) * (c->N + 1));
  if (s0) return s0;
  HIPCHK(c, hipMemcpy(c->d_pofs, c->h_pofs.data(),
                      sizeof(int64_t) * (c->N + 1), hipMemcpyHostToDevice));
  size_t bytes = (size_t)c->h_pofs[c->N] * c->esz();
  d2_status s;
  if ((s = dalloc(c, &c->d_P1, bytes))) return s;
  if ((s = dalloc(c, &c->d_P2, bytes))) return s;
  if ((s = dalloc(c, &c->d_L, bytes))) return s;
  c->onfly = c->d <= 4 && !c->sym;
  if (!c->onfly && (s = dalloc(c, &c->d_C, bytes))) return s;
  return D2_OK;
}

hipEvent_t take_event(d2_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket a launch with events when profiling (start before, stop after).
hipEvent_t prof_begin(d2_ctx* c) {
  if (!c->prof) return nullptr;
  hipEvent_t a = take_event(c);
  if (a) (void)hipEventRecord(a, c->stream);
  return a;
}

void prof_end(d2_ctx* c, int kind, hipEvent_t a) {
  if (!c->prof || !a) return;
  hipEvent_t b = take_event(c);
  if (!b) return;
  (void)hipEventRecord(b, c->stream);
  c->pending.push_back({kind, a, b});
}

// Called after the stream has been synchronised.
void prof_collect(d2_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof_launches[p.kind] += 1;
      c->prof_ms[p.kind] += ms;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

int aux_kind(int mode) {
  switch (mode) {
    case d2k::kRho: return kKRho;
    case d2k::kA0: return kKInitA;
    case d2k::kBF: return kKBF;
    default: return kKXO;
  }
}

template <typename T>
d2k::Args<T> make_args(d2_ctx* c, const d2_badmm_params* p) {
  d2k::Args<T> a;
  a.off = c->d_off;
  a.pofs = c->d_pofs;
  a.X = (const T*)c->d_X;
  a.W = (const T*)c->d_W;
  a.work = c->d_work;
  a.chunks = c->d_chunks;
  a.nch = c->d_nch;
  a.blist = nullptr;
  a.bcnt = c->d_bcnt;
  a.bidx = 0;
  a.boff = 0;
  a.ctab = c->d_ctab;
  a.ninv = c->d_ninv;
  a.P1 = (T*)c->d_P1;
  a.P2 = (T*)c->d_P2;
  a.L = (T*)c->d_L;
  a.Cc = (T*)c->d_C;
  a.warm = c->d_warm;
  a.xc = c->d_xc;
  a.wc = c->d_wc;
  a.rho = c->d_rho;
  a.part_in = c->d_part;
  a.part = c->d_part;
  a.xin = nullptr;
  a.xout = nullptr;
  a.trace = nullptr;
  a.rtrace = nullptr;
  a.rlast = 0;
  a.recost = 0;
  a.xstage = 0;
  a.eps = p ? p->eps : 1e-16;
  a.m = c->m;
  a.d = c->d;
  a.xs = c->xs;
  a.rule = p ? p->rule : 1;
  a.ps = c->MP + 2;
  a.dsym = c->sym ? (const T*)c->d_D : nullptr;
  a.isym = c->d_isym;
  a.csym = c->d_csym;
  a.S = c->S;
  return a;
}

d2k::FinArgs make_fin(d2_ctx* c, const d2_badmm_params* p) {
  d2k::FinArgs f;
  f.ctab = c->d_ctab;
  f.ninv = c->d_ninv;
  f.rtr = nullptr;
  f.cinv = c->d_cinv;
  f.part = c->d_part;
  f.xrec = c->d_partx;
  f.rho = c->d_rho;
  f.xc = c->d_xc;
  f.rho0 = p ? p->rho0 : 2.0;
  f.m = c->m;
  f.d = c->d;
  f.ps = c->MP + 2;
  return f;
}

d2_status launch_fin(d2_ctx* c, const d2k::FinArgs& f, int mode, int& nl) {
  d2k::FinFn fn = fin_table()[ilog2(c->MP) - 3];
  size_t shm =
      mode == d2k::kFinX ? sizeof(double) * c->MP * (c->d + 1) : 0;
  hipEvent_t pe = prof_begin(c);
  hipLaunchKernelGGL(fn, dim3(c->K), dim3(256), shm, c->stream, f, mode);
  HIPCHK(c, hipGetLastError());
  prof_end(c, kKFin, pe);
  ++nl;
  return D2_OK;
}

template <typename T>
d2_status launch_aux(d2_ctx* c, const d2k::Args<T>& a0, int mode, int& nl) {
  const auto& kt = kern<T>();
  const int ma = ilog2(c->MP) - 3, mr = ilog2(c->R);
  auto fn = mode == d2k::kRho ? kt.auxm[0][ma][mr]
            : mode == d2k::kA0 ? kt.auxm[1][ma][mr]
            : mode == d2k::kBF ? kt.auxm[2][ma][mr]
                               : kt.aux[ma][mr];
  if (!fn) return c->fail(D2_EINVAL, "no kernel for this tile shape");
  d2k::Args<T> a = a0;
  int waves = c->waves;
  size_t per_wave = sizeof(double) * c->MP * (c->d + 1);
  bool xnum = (mode == d2k::kXO) || (mode == d2k::kA0 && a.xout);
  if (xnum)
    while (waves > 1 && per_wave * waves > 64 * 1024) --waves;
  size_t shm = xnum ? per_wave * waves : 0;
  // large d: the cost pass reads the centroid support from LDS
  const size_t stage = (size_t)c->MP * (c->xs + 4) * sizeof(T);
  a.xstage = 0;
  if (mode == d2k::kRho && !c->onfly && !c->sym && stage <= 64 * 1024) {
    a.xstage = 1;
    shm = stage;
  }
  hipEvent_t pe = prof_begin(c);
  hipLaunchKernelGGL(fn, dim3(c->nch_cap), dim3(64 * waves), shm, c->stream,
                     a, mode);
  HIPCHK(c, hipGetLastError());
  prof_end(c, aux_kind(mode), pe);
  ++nl;
  return D2_OK;
}

// Launch q of a group of independent launches goes to stream_of(c, q):
// launch 0 to the context stream, the others to side streams that wait for
// the work issued before the group (fork) and that the context stream waits
// for after it (join).  Under graph capture the group becomes parallel
// branches.
hipStream_t stream_of(const d2_ctx* c, int q) {
  return q == 0 ? c->stream : c->side[(q - 1) % d2_ctx::kSide];
}
d2_status fork_side(d2_ctx* c, int n) {
  if (n <= 1) return D2_OK;
  HIPCHK(c, hipEventRecord(c->fork_ev, c->stream));
  for (int q = 1; q < n && q <= d2_ctx::kSide; ++q)
    HIPCHK(c, hipStreamWaitEvent(c->side[q - 1], c->fork_ev, 0));
  return D2_OK;
}
d2_status join_side(d2_ctx* c, int n) {
  for (int q = 1; q < n && q <= d2_ctx::kSide; ++q) {
    HIPCHK(c, hipEventRecord(c->join_ev[q - 1], c->side[q - 1]));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->join_ev[q - 1], 0));
  }
  return D2_OK;
}

// Whether the hot kernel streams the plan state: per iteration it reads and
// writes Pi1 and Lambda (and reads the cost cache for d > 4); beyond the
// 256 MiB last-level cache the default policy only displaces lines that are
// reused (measured: the d = 16, 2,000,000-instance workload 171.5 -> 146.8
// ms per update, the d = 3, 65,536-instance one, whose state fits, 30 %
// slower when streamed).
bool stream_state(const d2_ctx* c) {
  if (c->cache_policy == 1) return false;
  if (c->cache_policy == 2) return true;
  const double bytes = (double)c->h_pofs[c->N] * (double)c->esz() *
                       (c->onfly ? 2.0 : 3.0);
  return bytes > 256.0 * 1024.0 * 1024.0;
}

// One B-ADMM iteration: a launch per slot bucket, each kernel specialised
// for its bucket's register slots (profiled as one "iter_ba" unit).
template <typename T>
d2_status launch_ba(d2_ctx* c, const d2k::Args<T>& a, int& nl) {
  const auto& kt = kern<T>();
  const int mi = ilog2(c->MP) - 3;
  const size_t per_wave = sizeof(double) * c->MP * (c->d + 1);
  // FP32: the support sums (MP 16 / 32, 16 <= d <= 64) and the cost at a
  // new support (MP 32, 32 <= d <= 64) come from matrix-core passes of
  // their own beside a plain launch (k_sup_mfma after it, k_cost_mfma
  // before it)
  const bool xo = a.xout && !a.recost && !c->onfly && c->d >= 16 &&
                  c->d <= 64 && kt.sup[0][mi][0] != nullptr;
  const bool cx = a.recost && !a.xout && !c->onfly && c->d >= 32 &&
                  c->d <= 64 && c->MP == 32 && kt.cst[0] != nullptr;
  // otherwise (FP32, cost cached) the cost at a new support comes from a
  // VALU pass before the plain launch
  const bool cv = a.recost && !a.xout && !c->onfly && !cx &&
                  kt.cstv[mi][0] != nullptr;
  // large d, first launch after a support update: the cost is recomputed
  // from the centroid support staged in LDS after the support records
  const bool want_stage = a.recost && !c->onfly;
  const size_t stage =
      want_stage ? (size_t)c->MP * (c->xs + 4) * sizeof(T) : 0;
  auto fits = [](size_t b) { return b <= 64 * 1024; };
  // the full kernel forms what the passes do not; waves per workgroup are
  // lowered until its (or k_sup_mfma's) support records fit in LDS
  const bool full = (a.xout && !xo) || (a.recost && !cx && !cv);
  auto lds = [&](int wv) { return (a.xout ? per_wave * wv : 0) + stage; };
  int waves = c->waves;
  if (full)
    while (waves > 1 && !fits(lds(waves))) --waves;
  const int xstage = (full && want_stage && fits(lds(waves))) ? 1 : 0;
  size_t shm = full && a.xout ? per_wave * waves : 0;
  if (xstage) shm += stage;
  int wsup = c->waves;
  while (wsup > 1 && !fits(per_wave * wsup)) --wsup;
  hipEvent_t pe = prof_begin(c);
  // plan state far beyond the last-level cache (256 MiB on this part):
  // the launches stream it (non-temporal)
  const bool nt = stream_state(c) && kt.bapn[c->onfly ? 1 : 0][0][0] != nullptr;
  // the buckets' launches write disjoint chunk records: side by side
  {
    d2_status s = fork_side(c, c->nbk);
    if (s) return s;
  }
  // widest slot class first: its launch has the fewest wavefronts per SIMD
  // and the longest tiles, so it sets the end of the group
  for (int bi = 0; bi < c->nbk; ++bi) {
    const int b = c->nbk - 1 - bi;
    const int rb = ilog2(c->bk_R[b]);
    const int oi = c->onfly ? 1 : 0;
    auto fn = full ? (nt && !c->onfly && kt.ban[mi][rb] ? kt.ban[mi][rb]
                                                        : kt.ba[oi][mi][rb])
              : nt ? kt.bapn[oi][mi][rb]
                   : kt.bap[oi][mi][rb];
    if (!fn) return c->fail(D2_EINVAL, "no kernel for this tile shape");
    d2k::Args<T> ab = a;
    ab.blist = c->d_blist;
    ab.xstage = xstage;
    ab.bidx = b;
    ab.boff = c->bk_off[b];
    hipStream_t st = stream_of(c, bi);
    if (cx) {
      hipLaunchKernelGGL(kt.cst[rb], dim3(c->bk_cap[b]), dim3(64 * c->waves),
                         d2k::cost_mfma_lds_bytes(c->xs, c->waves), st, ab);
      HIPCHK(c, hipGetLastError());
      ++nl;
      ab.recost = 0;
    } else if (cv) {
      hipLaunchKernelGGL(kt.cstv[mi][rb], dim3(c->bk_cap[b]),
                         dim3(64 * c->waves),
                         (size_t)c->MP * (c->xs + 4) * sizeof(float), st, ab);
      HIPCHK(c, hipGetLastError());
      ++nl;
      ab.recost = 0;
    }
    if (xo) ab.xout = nullptr;
    hipLaunchKernelGGL(fn, dim3(c->bk_cap[b]), dim3(64 * waves), shm, st,
                       ab);
    HIPCHK(c, hipGetLastError());
    ++nl;
    if (xo) {
      auto fs = kt.sup[nt ? 1 : 0][mi][rb];
      if (!fs) return c->fail(D2_EINVAL, "no kernel for this tile shape");
      ab.xout = a.xout;
      hipLaunchKernelGGL(fs, dim3(c->bk_cap[b]), dim3(64 * wsup),
                         per_wave * wsup, st, ab);
      HIPCHK(c, hipGetLastError());
      ++nl;
    }
  }
  {
    d2_status s = join_side(c, c->nbk);
    if (s) return s;
  }
  prof_end(c, kKIterBA, pe);
  return D2_OK;
}

// The launch sequence of one B-ADMM call (all clusters): issued eagerly or
// captured once into a HIP graph and replayed.  It contains kernel launches
// only.
template <typename T>
d2_status issue_barycenter(d2_ctx* c, const d2_badmm_params* p, int& nl) {
  const int K = c->K, T_ = p->iters, tau = p->tau;
  const int64_t ps = c->MP + 2;
  const int64_t xs = (int64_t)c->MP * (c->d + 1);
  d2k::Args<T> a = make_args<T>(c, p);
  d2k::FinArgs f = make_fin(c, p);
  double* rec[2] = {c->d_part, c->d_part + (int64_t)c->nch_cap * ps};
  double* xrec[2] = {c->d_partx, c->d_partx + (int64_t)c->nch_cap * xs};
  // support update after iteration n (0-based): (n + 1) % tau == 0
  auto xupd = [&](int n) {
    return !p->fixed_support && n < T_ && ((n + 1) % tau == 0);
  };
  d2_status s;
  // rho from the cost at the initial support
  a.part = rec[1];
  f.part = rec[1];
  if ((s = launch_aux<T>(c, a, d2k::kRho, nl))) return s;
  if ((s = launch_fin(c, f, d2k::kFinRho, nl))) return s;
  if (c->rho_fixed && c->rho_fix_K == c->K) {
    // rho held at the caller's values (d2_set_rho)
    HIPCHK(c, hipMemcpyAsync(c->d_rho, c->d_rho_fix, sizeof(double) * K,
                             hipMemcpyDeviceToDevice, c->stream));
  }
  // A_0 from the initial plans and weights
  a.part = rec[0];
  a.xout = xupd(0) ? xrec[0] : nullptr;
  if ((s = launch_aux<T>(c, a, d2k::kA0, nl))) return s;
  for (int n = 0; n < T_; ++n) {
    a.part_in = rec[n & 1];      // records of A_n -> w^{n+1}, F(n)
    a.part = rec[(n + 1) & 1];   // records of A_{n+1}
    a.trace = c->d_trace + (size_t)n * K;
    // residual of phase B_{n-1} (computed by the previous launch)
    a.rtrace = n > 0 ? c->d_rtrace + (size_t)(n - 1) * K : nullptr;
    // support records of A_n (support update after iteration n)
    const bool xin = xupd(n);
    a.xin = (xin && c->onfly) ? xrec[n & 1] : nullptr;
    a.xout = xupd(n + 1) ? xrec[(n + 1) & 1] : nullptr;
    a.recost = 0;
    if (xin && !c->onfly) {
      // large d: a per-cluster launch updates x, then the next phase A
      // recomputes (and re-caches) the cost
      f.xrec = xrec[n & 1];
      if ((s = launch_fin(c, f, d2k::kFinX, nl))) return s;
      a.recost = 1;
    }
    if (n == T_ - 1) {
      a.rlast = 1;
      if ((s = launch_aux<T>(c, a, d2k::kBF, nl))) return s;
      a.rlast = 0;
      f.part = a.part;
      f.rtr = c->d_rtrace + (size_t)n * K;
      if ((s = launch_fin(c, f, d2k::kFinRes, nl))) return s;
    } else {
      if ((s = launch_ba<T>(c, a, nl))) return s;
    }
  }
  return D2_OK;
}

std::vector<double> graph_key(const d2_ctx* c, const d2_badmm_params* p) {
  return {(double)c->rho_fixed, (double)stream_state(c), (double)p->iters,
          (double)p->tau,
          (double)p->fixed_support,
          (double)p->rule, p->eps, p->rho0, (double)c->waves,
          (double)c->nch_cap, (double)c->MP, (double)c->R, (double)c->onfly,
          (double)c->dt, (double)c->K, (double)c->nbk,
          (double)c->bk_R[0], (double)c->bk_R[1], (double)c->bk_R[2],
          (double)c->bk_R[3], (double)c->bk_R[4], (double)c->bk_R[5],
          (double)c->bk_cap[0], (double)c->bk_cap[1], (double)c->bk_cap[2],
          (double)c->bk_cap[3], (double)c->bk_cap[4], (double)c->bk_cap[5]};
}

template <typename T>
d2_status run_barycenter(d2_ctx* c, const d2_badmm_params* p,
                         d2_badmm_stats* st) {
  const int K = c->K, MP = c->MP, T_ = p->iters;
  if (T_ > c->trace_cap) {
    drop_graph(c);
    dfree(c->d_trace);
    dfree(c->d_rtrace);
    d2_status s = dalloc(c, (void**)&c->d_trace, sizeof(double) * T_ * K);
    if (s) return s;
    if ((s = dalloc(c, (void**)&c->d_rtrace, sizeof(double) * T_ * K)))
      return s;
    c->trace_cap = T_;
  }
  HIPCHK(c, hipMemsetAsync(c->d_trace, 0, sizeof(double) * T_ * K,
                           c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_rtrace, 0, sizeof(double) * T_ * K,
                           c->stream));
  const size_t xbytes = sizeof(double) * (size_t)K * MP * c->d;
  const size_t wbytes = sizeof(double) * (size_t)K * MP;
  HIPCHK(c, hipMemcpyAsync(c->d_xsave, c->d_xc, xbytes,
                           hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_wsave, c->d_wc, wbytes,
                           hipMemcpyDeviceToDevice, c->stream));
  int nl = 0;
  bool graphed = false;
  d2_status s;
  // per-kernel event timing needs eager launches
  const bool want_graph = c->use_graph && !c->prof;
  if (want_graph) {
    std::vector<double> key = graph_key(c, p);
    if (!c->gexec || key != c->graph_key) {
      drop_graph(c);
      HIPCHK(c, hipStreamBeginCapture(c->stream,
                                      hipStreamCaptureModeThreadLocal));
      int cnt = 0;
      s = issue_barycenter<T>(c, p, cnt);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->stream, &g);
      if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
      }
      if (e != hipSuccess)
        return c->fail(D2_EDEVICE, std::string("hipStreamEndCapture: ") +
                                       hipGetErrorString(e));
      c->graph = g;
      HIPCHK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
      c->graph_key = key;
      c->graph_launches = cnt;
    }
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    nl = c->graph_launches;
    graphed = true;
  } else {
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    if ((s = issue_barycenter<T>(c, p, nl))) return s;
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  // non-finite guard on the new centroids: on failure the centroids of the
  // call's start are restored and the (non-finite) plans are not a cache
  std::vector<double> hx((size_t)K * MP * c->d), hw((size_t)K * MP);
  HIPCHK(c, hipMemcpy(hx.data(), c->d_xc, hx.size() * 8,
                      hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hw.data(), c->d_wc, hw.size() * 8,
                      hipMemcpyDeviceToHost));
  if (!finite_all(hx.data(), hx.size()) || !finite_all(hw.data(), hw.size())) {
    HIPCHK(c, hipMemcpy(c->d_xc, c->d_xsave, xbytes,
                        hipMemcpyDeviceToDevice));
    HIPCHK(c, hipMemcpy(c->d_wc, c->d_wsave, wbytes,
                        hipMemcpyDeviceToDevice));
    c->have_cache = false;
    c->trace_rows = 0;
    return c->fail(D2_ENUMERIC, "non-finite centroid support or weights "
                                "(centroids restored)");
  }
  c->trace_rows = T_;
  // the labels of this update are those of the cached plans
  HIPCHK(c, hipMemcpyAsync(c->d_cache_labels, c->d_labels,
                           sizeof(int32_t) * c->N, hipMemcpyDeviceToDevice,
                           c->stream));
  c->cache_gen = c->label_gen;
  c->hcache_ok = c->hlab_ok;
  if (c->hlab_ok) c->h_cache_labels = c->h_labels;
  c->have_cache = true;
  if (st) {
    st->iters = T_;
    if (!c->host_ctab) {
      c->h_ctab.resize(K);
      HIPCHK(c, hipMemcpy(c->h_ctab.data(), c->d_ctab, sizeof(int2) * K,
                          hipMemcpyDeviceToHost));
      c->host_ctab = true;
    }
    int ne = 0;
    for (int q = 0; q < K; ++q) ne += c->h_ctab[q].y == 0;
    st->n_empty = ne;
    st->launches = nl;
    st->graph = graphed ? 1 : 0;
    st->ms = ms;
  }
  return D2_OK;
}

int slots_for(const d2_ctx* c) {
  int cps = 64 / c->MP;
  int need = (c->mk_max + cps - 1) / cps;
  return 1 << ilog2(std::max(1, need));
}

template <typename T>
d2_status centroid_stats(d2_ctx* c) {
  const int K = c->K, MP = c->MP, d = c->d;
  if (!c->d_cmu) {
    d2_status s;
    if ((s = dalloc(c, &c->d_cmu, sizeof(T) * (size_t)K * d))) return s;
    if ((s = dalloc(c, &c->d_crad, sizeof(T) * (size_t)K))) return s;
    if ((s = dalloc(c, &c->d_xct, sizeof(T) * (size_t)K * MP * c->xs)))
      return s;
  }
  hipLaunchKernelGGL(d2k::k_cstats<T>, dim3(K), dim3(64), sizeof(double) * d,
                     c->stream, c->d_xc, c->d_wc, c->m, MP, d, c->xs, K,
                     (T*)c->d_cmu, (T*)c->d_crad, (T*)c->d_xct,
                     c->lbs_valid ? (const double*)c->d_xref : nullptr,
                     c->d_dlt);
  HIPCHK(c, hipGetLastError());
  return D2_OK;
}

// Buffers of the cross-round assignment bounds (N x K floats); without
// them (switched off, or no memory) the assignment prunes within the round
// only.
bool ensure_bounds(d2_ctx* c) {
  if (!c->use_lbs) return false;
  if (c->d_lbs) return true;
  const size_t nb = sizeof(float) * (size_t)c->N * c->K;
  if (hipMalloc((void**)&c->d_lbs, nb) != hipSuccess ||
      hipMalloc((void**)&c->d_xref,
                sizeof(double) * (size_t)c->K * c->MP * c->d) != hipSuccess ||
      hipMalloc((void**)&c->d_dlt, sizeof(float) * c->K) != hipSuccess) {
    (void)hipGetLastError();
    free_bounds(c);
    c->use_lbs = false;
    return false;
  }
  c->lbs_valid = false;
  return true;
}

template <typename T>
d2_status run_assign(d2_ctx* c, const d2_ot_params* p, float* ms_out,
                     double* dall = nullptr) {
  const auto& kt = kern<T>();
  auto fn = kt.asg[ilog2(c->MP) - 3][ilog2(c->R)];
  if (!fn) return c->fail(D2_EINVAL, "no kernel for this tile shape");
  d2k::AssignArgs<T> a{};
  a.dall = dall;
  a.off = c->d_off;
  a.X = (const T*)c->d_X;
  a.W = (const T*)c->d_W;
  a.xc = c->d_xc;
  a.wc = c->d_wc;
  a.labels = c->d_labels;
  a.best = c->d_best;
  a.counts = c->d_pairs;
  a.prune = p->prune ? 1 : 0;
  a.prev_valid = c->have_labels ? 1 : 0;
  const bool bounds = a.prune && ensure_bounds(c);
  {
    d2_status s = centroid_stats<T>(c);
    if (s) return s;
  }
  a.lbs = bounds ? c->d_lbs : nullptr;
  a.dlt = c->d_dlt;
  a.dsym = c->sym ? (const T*)c->d_D : nullptr;
  a.isym = c->d_isym;
  a.csym = c->d_csym;
  a.S = c->S;
  a.lbs_in = bounds && c->lbs_valid ? 1 : 0;
  a.cmu = (const T*)c->d_cmu;
  a.crad = (const T*)c->d_crad;
  a.xct = (const T*)c->d_xct;
  a.N = c->N;
  a.rho0 = p->rho0;
  a.eps = p->eps;
  a.m = c->m;
  a.d = c->d;
  a.xs = c->xs;
  a.K = c->K;
  a.iters = p->iters;
  // candidate bounds one per lane where a centroid row fits in registers
  // and the centroids fill the lanes (FP32 vectors, d <= 16, K >= 32)
  const bool batch = sizeof(T) == 4 && a.prune && !c->sym && c->d <= 16 &&
                     c->K >= 32;
  if (c->alist_MP != c->MP) {
    // Instance ids grouped by slot class (stable).  The classes run as
    // separate launches only when the largest needs 8 or more slots (its
    // kernel holds few wavefronts per SIMD); a class with under 10 % of
    // the instances then joins the next larger one.  Otherwise one launch.
    std::vector<uint8_t> cls(c->N);
    int64_t hist[6] = {0, 0, 0, 0, 0, 0};
    int top = 0;
    for (int64_t k = 0; k < c->N; ++k) {
      cls[k] = (uint8_t)slot_class(c, k);
      hist[cls[k]]++;
      top = std::max(top, (int)cls[k]);
    }
    int map[6];
    for (int q = 5, cur = top; q >= 0; --q) {
      if ((1 << top) >= 8 && hist[q] > 0 && q < top &&
          hist[q] * 10 >= c->N)
        cur = q;
      map[q] = std::min(cur, top);
    }
    std::vector<int64_t> cnt(7, 0);
    for (int64_t k = 0; k < c->N; ++k) {
      cls[k] = (uint8_t)map[cls[k]];
      cnt[cls[k] + 1]++;
    }
    for (int q = 0; q < 6; ++q) {
      c->acnt[q] = cnt[q + 1];
      cnt[q + 1] += cnt[q];
      c->aofs[q] = cnt[q];
    }
    std::vector<int32_t> lst(c->N);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t k = 0; k < c->N; ++k) lst[pos[cls[k]]++] = (int32_t)k;
    if (!c->d_alist) {
      d2_status s = dalloc(c, (void**)&c->d_alist, sizeof(int32_t) * c->N);
      if (s) return s;
    }
    HIPCHK(c, hipMemcpy(c->d_alist, lst.data(), sizeof(int32_t) * c->N,
                        hipMemcpyHostToDevice));
    c->alist_MP = c->MP;
  }
  const int wpb = 4;
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  hipEvent_t pe = prof_begin(c);
  // one launch per slot class, each kernel sized for its class; the
  // classes hold disjoint instances and run side by side
  int nact = 0;
  for (int q = 0; q < 6; ++q) nact += c->acnt[q] ? 1 : 0;
  {
    d2_status s = fork_side(c, nact);
    if (s) return s;
  }
  int qi = 0;
  for (int q = 0; q < 6; ++q) {
    if (!c->acnt[q]) continue;
    auto fq = kt.asg[ilog2(c->MP) - 3][q];
    if (!fq) return c->fail(D2_EINVAL, "no kernel for this tile shape");
    d2k::AssignArgs<T> aq = a;
    aq.list = c->d_alist + c->aofs[q];
    aq.N = c->acnt[q];
    aq.batch = batch && c->MP <= 16 && (64 / c->MP) * (1 << q) <= 32 ? 1 : 0;
    const int64_t blocks = (aq.N + wpb - 1) / wpb;
    const size_t lds = (size_t)wpb * d2k::assign_lds(c->d, c->MP, 1 << q,
                                                     c->xs, (int)sizeof(T),
                                                     aq.batch).bytes;
    hipLaunchKernelGGL(fq, dim3((unsigned)blocks), dim3(64 * wpb), lds,
                       stream_of(c, qi++), aq);
    HIPCHK(c, hipGetLastError());
  }
  {
    d2_status s = join_side(c, nact);
    if (s) return s;
  }
  prof_end(c, kKAssign, pe);
  if (bounds) {
    // the stored bounds now refer to the current centroid supports
    HIPCHK(c, hipMemcpyAsync(c->d_xref, c->d_xc,
                             sizeof(double) * (size_t)c->K * c->MP * c->d,
                             hipMemcpyDeviceToDevice, c->stream));
    c->lbs_valid = true;
  }
  HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (ms_out) *ms_out = ms;
  c->last_pairs = c->N * (int64_t)c->K;
  return D2_OK;
}

// Number of instances whose label differs from the previous one (integer
// sums, so the count does not depend on the order of the atomic adds).
__global__ void __launch_bounds__(256)
    k_count_changes(const int32_t* __restrict__ a,
                    const int32_t* __restrict__ b, int64_t N,
                    int64_t* __restrict__ out) {
  int64_t n = 0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N;
       k += st)
    n += a[k] != b[k];
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd((unsigned long long*)out,
                                              (unsigned long long)n);
}

// Multi-modal assignment (Sec. 5): label = argmin over centroids of the
// summed per-modality distances dall (N x K), ties to the lowest index.
__global__ void __launch_bounds__(256)
    k_argmin_rows(const double* __restrict__ dall, int64_t N, int K,
                  int32_t* __restrict__ labels, double* __restrict__ best) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double* r = dall + k * K;
  int bc = 0;
  double bv = r[0];
  for (int c = 1; c < K; ++c)
    if (r[c] < bv) {
      bv = r[c];
      bc = c;
    }
  labels[k] = bc;
  best[k] = bv;
}

// Device-copy probe: each thread moves 4 x 16 bytes per step (all four
// loads issued before the stores), grid-stride over the buffer.
__global__ void __launch_bounds__(256)
    k_copy_probe(const float4* __restrict__ src, float4* __restrict__ dst,
                 int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                 d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n4; i += stride) dst[i] = src[i];
}


}  // namespace

extern "C" {

d2_status d2_create(d2_ctx** out, int device, d2_dtype dtype,
                    void* hip_stream) {
  if (!out) return D2_EINVAL;
  *out = nullptr;
  if (dtype != D2_F32 && dtype != D2_F64) return D2_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 ||
      device >= ndev) {
    (void)hipGetLastError();
    return D2_EDEVICE;
  }
  d2_ctx* c = new d2_ctx();
  c->device = device;
  c->dt = dtype;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return D2_EDEVICE;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) !=
        hipSuccess) {
      delete c;
      return D2_EDEVICE;
    }
    c->own_stream = true;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess ||
      hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) !=
          hipSuccess) {
    d2_destroy(c);
    return D2_EDEVICE;
  }
  for (int i = 0; i < d2_ctx::kSide; ++i)
    if (hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) !=
            hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming) !=
            hipSuccess) {
      d2_destroy(c);
      return D2_EDEVICE;
    }
  *out = c;
  return D2_OK;
}

void d2_destroy(d2_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_instances(c);
  free_centroids(c);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (int i = 0; i < d2_ctx::kSide; ++i) {
    if (c->side[i]) {
      (void)hipStreamSynchronize(c->side[i]);
      (void)hipStreamDestroy(c->side[i]);
    }
    if (c->join_ev[i]) (void)hipEventDestroy(c->join_ev[i]);
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* d2_last_error(const d2_ctx* c) {
  return c ? c->err.c_str() : "null context";
}

}  // extern "C"

namespace {

// Validate the instance offsets (Sec. 2 layout): offsets[0] = 0, 1 <= m_k
// <= 64, n < 2^31.  Returns the largest m_k through mkmax.
d2_status check_offsets(d2_ctx* c, int64_t N, int32_t d,
                        const int64_t* offsets, int& mkmax) {
  if (N < 1 || d < 1 || !offsets)
    return c->fail(D2_EINVAL, "need N >= 1, d >= 1 and non-null arrays");
  if (offsets[0] != 0) return c->fail(D2_EINVAL, "offsets[0] must be 0");
  mkmax = 0;
  for (int64_t k = 0; k < N; ++k) {
    int64_t mk = offsets[k + 1] - offsets[k];
    if (mk < 1 || mk > 64)
      return c->fail(D2_EINVAL, "instance " + std::to_string(k) +
                                    ": support size must be in [1, 64]");
    mkmax = std::max<int>(mkmax, (int)mk);
  }
  if (offsets[N] > INT32_MAX)
    return c->fail(D2_EINVAL, "n exceeds 2^31 - 1");
  return D2_OK;
}

// Drop the previous instances, centroids and plans and take over the new
// offsets; allocates the per-instance device arrays except X and W.
d2_status adopt_offsets(d2_ctx* c, int64_t N, int32_t d,
                        const int64_t* offsets, int mkmax) {
  free_instances(c);
  free_centroids(c);
  c->N = N;
  c->n = offsets[N];
  c->d = d;
  c->xs = (d + 3) / 4 * 4;  // zero-padded stride, a multiple of 4
  c->mk_max = mkmax;
  c->h_off.assign(offsets, offsets + N + 1);
  c->inst_hash = 0;
  d2_status s;
  if ((s = dalloc(c, (void**)&c->d_off, sizeof(int64_t) * (N + 1)))) return s;
  if ((s = dalloc(c, (void**)&c->d_labels, sizeof(int32_t) * N))) return s;
  if ((s = dalloc(c, (void**)&c->d_cache_labels, sizeof(int32_t) * N)))
    return s;
  if ((s = dalloc(c, (void**)&c->d_prev_labels, sizeof(int32_t) * N)))
    return s;
  if ((s = dalloc(c, (void**)&c->d_nchg, sizeof(int64_t)))) return s;
  if ((s = dalloc(c, (void**)&c->d_best, sizeof(double) * N))) return s;
  if ((s = dalloc(c, (void**)&c->d_pairs, 2 * sizeof(int32_t) * N)))
    return s;
  HIPCHK(c, hipMemcpy(c->d_off, offsets, sizeof(int64_t) * (N + 1),
                      hipMemcpyHostToDevice));
  c->h_labels.assign(N, 0);
  c->hlab_ok = true;
  ++c->label_gen;
  return D2_OK;
}

// Validation of borrowed device instances, one thread per instance: finite
// coordinates, zero padding columns, finite non-negative weights summing
// to 1 within 1e-6 (in double).  bad gets min over failing instances of
// (k << 2 | reason): reason 1 coordinates, 2 weights, 3 weight sum.
template <typename T>
__global__ void __launch_bounds__(256)
    k_check_instances(const int64_t* off, const T* X, const T* W, int64_t N,
                      int d, int xs, unsigned long long* bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  int reason = 0;
  double s = 0.0;
  for (int64_t j = off[k]; j < off[k + 1] && !reason; ++j) {
    for (int t = 0; t < xs; ++t) {
      const T v = X[j * xs + t];
      if (t < d ? !isfinite((double)v) : v != T(0)) reason = 1;
    }
    const T w = W[j];
    if (!(w >= T(0)) || !isfinite((double)w)) reason = 2;
    s += (double)w;
  }
  if (!reason && !(fabs(s - 1.0) <= 1e-6)) reason = 3;
  if (reason)
    atomicMin(bad, ((unsigned long long)k << 2) | (unsigned long long)reason);
}

// Order-independent 64-bit fingerprint of 32-bit words: the wrapping sum of
// a mix of (index, word) for every word, so that any change of a word or of
// its position changes it (with high probability) and the result does not
// depend on the summation order.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void __launch_bounds__(256)
    k_fingerprint(const uint32_t* w, int64_t nw, unsigned long long salt,
                  unsigned long long* out) {
  unsigned long long acc = 0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nw;
       q += st)
    acc += mix64(salt ^ mix64((unsigned long long)q * 0x100000001B3ull ^
                              (unsigned long long)w[q]));
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

// Fingerprint of the loaded instances (offsets, and the device copies of
// X and W in the device dtype), computed on first use.
d2_status instance_hash(d2_ctx* c, uint64_t* out) {
  if (c->inst_hash) {
    *out = c->inst_hash;
    return D2_OK;
  }
  unsigned long long* d = nullptr;
  // symbolic instances: also their symbols and the symbol table
  const void* src[5] = {c->d_off, c->d_X, c->d_W, c->d_isym, c->d_D};
  const int64_t words[5] = {2 * (c->N + 1),
                            (int64_t)(c->esz() / 4) * c->n * c->xs,
                            (int64_t)(c->esz() / 4) * c->n, c->n,
                            (int64_t)(c->esz() / 4) * c->S * c->S};
  const int nsrc = c->sym ? 5 : 3;
  d2_status s0 = dalloc(c, (void**)&d, sizeof(unsigned long long) * 5);
  if (s0) return s0;
  d2_status st = D2_OK;
  if (hipMemsetAsync(d, 0, sizeof(unsigned long long) * 5, c->stream) !=
      hipSuccess)
    st = c->fail(D2_EDEVICE, "hipMemsetAsync");
  for (int q = 0; q < nsrc && !st; ++q) {
    hipLaunchKernelGGL(k_fingerprint, dim3(1024), dim3(256), 0, c->stream,
                       (const uint32_t*)src[q], words[q],
                       (unsigned long long)(q + 1), d + q);
    if (hipGetLastError() != hipSuccess)
      st = c->fail(D2_EDEVICE, "k_fingerprint launch");
  }
  unsigned long long h[5] = {0, 0, 0, 0, 0};
  if (!st && hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost,
                            c->stream) != hipSuccess)
    st = c->fail(D2_EDEVICE, "hipMemcpyAsync");
  if (!st && hipStreamSynchronize(c->stream) != hipSuccess)
    st = c->fail(D2_EDEVICE, "hipStreamSynchronize");
  dfree(d);
  if (st) return st;
  c->inst_hash = (((h[0] * 31 + h[1]) * 31 + h[2]) * 31 + h[3]) * 31 + h[4] +
                 (uint64_t)c->dt;
  if (!c->inst_hash) c->inst_hash = 1;
  *out = c->inst_hash;
  return D2_OK;
}

}  // namespace

extern "C" {

d2_status d2_load_instances(d2_ctx* c, int64_t N, int32_t d,
                            const int64_t* offsets, const double* X,
                            const double* W) {
  if (!c) return D2_EINVAL;
  int mkmax = 0;
  d2_status s = check_offsets(c, N, d, offsets, mkmax);
  if (s) return s;
  if (!X || !W) return c->fail(D2_EINVAL, "null X or W");
  const int64_t n = offsets[N];
  std::vector<double> Wn(W, W + n);
  for (int64_t k = 0; k < N; ++k) {
    double sum = 0.0;
    for (int64_t j = offsets[k]; j < offsets[k + 1]; ++j) {
      if (!(W[j] >= 0.0) || !std::isfinite(W[j]))
        return c->fail(D2_EINVAL, "instance " + std::to_string(k) +
                                      ": weights must be finite and >= 0");
      for (int t = 0; t < d; ++t)
        if (!std::isfinite(X[j * d + t]))
          return c->fail(D2_EINVAL, "instance " + std::to_string(k) +
                                        ": non-finite support point");
      sum += W[j];
    }
    if (!(std::fabs(sum - 1.0) <= 1e-6))
      return c->fail(D2_EINVAL, "instance " + std::to_string(k) +
                                    ": weights do not sum to 1");
    for (int64_t j = offsets[k]; j < offsets[k + 1]; ++j) Wn[j] = W[j] / sum;
  }
  HIPCHK(c, hipSetDevice(c->device));
  if ((s = adopt_offsets(c, N, d, offsets, mkmax))) return s;
  if ((s = dalloc(c, &c->d_X, c->esz() * n * c->xs))) return s;
  if ((s = dalloc(c, &c->d_W, c->esz() * n))) return s;
  // supports with row stride xs (zero padding for d <= 4)
  std::vector<double> Xp((size_t)n * c->xs, 0.0);
  for (int64_t j = 0; j < n; ++j)
    for (int t = 0; t < d; ++t) Xp[(size_t)j * c->xs + t] = X[j * d + t];
  if (c->dt == D2_F64) {
    if ((s = upload_conv<double>(c, c->d_X, Xp.data(), Xp.size()))) return s;
    if ((s = upload_conv<double>(c, c->d_W, Wn.data(), n))) return s;
  } else {
    if ((s = upload_conv<float>(c, c->d_X, Xp.data(), Xp.size()))) return s;
    if ((s = upload_conv<float>(c, c->d_W, Wn.data(), n))) return s;
  }
  return D2_OK;
}

d2_status d2_load_instances_device(d2_ctx* c, int64_t N, int32_t d,
                                   const int64_t* offsets, const void* dX,
                                   const void* dW) {
  if (!c) return D2_EINVAL;
  int mkmax = 0;
  d2_status s = check_offsets(c, N, d, offsets, mkmax);
  if (s) return s;
  if (!dX || !dW) return c->fail(D2_EINVAL, "null X or W");
  HIPCHK(c, hipSetDevice(c->device));
  // the device data are checked before anything of the context changes
  const int xs = (d + 3) / 4 * 4;
  int64_t* doff = nullptr;
  unsigned long long* dbad = nullptr;
  if ((s = dalloc(c, (void**)&doff, sizeof(int64_t) * (N + 1)))) return s;
  if ((s = dalloc(c, (void**)&dbad, sizeof(unsigned long long)))) {
    dfree(doff);
    return s;
  }
  unsigned long long bad = ~0ull;
  hipError_t e = hipMemcpy(doff, offsets, sizeof(int64_t) * (N + 1),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(dbad, &bad, sizeof(bad), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const unsigned blocks = (unsigned)((N + 255) / 256);
    if (c->dt == D2_F64)
      hipLaunchKernelGGL(k_check_instances<double>, dim3(blocks), dim3(256),
                         0, c->stream, doff, (const double*)dX,
                         (const double*)dW, N, d, xs, dbad);
    else
      hipLaunchKernelGGL(k_check_instances<float>, dim3(blocks), dim3(256), 0,
                         c->stream, doff, (const float*)dX, (const float*)dW,
                         N, d, xs, dbad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess)
    e = hipMemcpy(&bad, dbad, sizeof(bad), hipMemcpyDeviceToHost);
  dfree(doff);
  dfree(dbad);
  if (e != hipSuccess)
    return c->fail(D2_EDEVICE, std::string("instance check: ") +
                                   hipGetErrorString(e));
  if (bad != ~0ull) {
    static const char* why[4] = {"", "non-finite coordinate or non-zero "
                                     "padding", "weights must be finite and "
                                     ">= 0", "weights do not sum to 1"};
    return c->fail(D2_EINVAL, "instance " + std::to_string(bad >> 2) + ": " +
                                  why[bad & 3]);
  }
  if ((s = adopt_offsets(c, N, d, offsets, mkmax))) return s;
  c->d_X = const_cast<void*>(dX);
  c->d_W = const_cast<void*>(dW);
  c->borrowed = true;
  return D2_OK;
}

d2_status d2_load_instances_symbolic(d2_ctx* c, int64_t N,
                                     const int64_t* offsets,
                                     const int32_t* sym, const double* W,
                                     int32_t S, const double* D) {
  if (!c) return D2_EINVAL;
  int mkmax = 0;
  d2_status s = check_offsets(c, N, 1, offsets, mkmax);
  if (s) return s;
  if (!sym || !W || !D) return c->fail(D2_EINVAL, "null symbols, W or D");
  if (S < 1 || S > 16384)
    return c->fail(D2_EINVAL, "the symbol count S must be in [1, 16384]");
  const int64_t n = offsets[N];
  for (int64_t k = 0; k < N; ++k)
    for (int64_t j = offsets[k]; j < offsets[k + 1]; ++j)
      if (sym[j] < 0 || sym[j] >= S)
        return c->fail(D2_EINVAL, "instance " + std::to_string(k) +
                                      ": symbol out of range");
  for (int64_t q = 0; q < (int64_t)S * S; ++q)
    if (!(D[q] >= 0.0) || !std::isfinite(D[q]))
      return c->fail(D2_EINVAL, "the symbol table must be finite and >= 0");
  // the weights are checked and renormalised as for vector supports; the
  // support coordinates are a zero column (d = 1)
  std::vector<double> zx((size_t)n, 0.0);
  if ((s = d2_load_instances(c, N, 1, offsets, zx.data(), W))) return s;
  if ((s = dalloc(c, (void**)&c->d_isym, sizeof(int32_t) * n))) return s;
  HIPCHK(c, hipMemcpy(c->d_isym, sym, sizeof(int32_t) * n,
                      hipMemcpyHostToDevice));
  if ((s = dalloc(c, &c->d_D, c->esz() * (size_t)S * S))) return s;
  if (c->dt == D2_F64) {
    if ((s = upload_conv<double>(c, c->d_D, D, (size_t)S * S))) return s;
  } else {
    if ((s = upload_conv<float>(c, c->d_D, D, (size_t)S * S))) return s;
  }
  c->sym = true;
  c->S = S;
  c->inst_hash = 0;
  return D2_OK;
}

static d2_status centroids_set_impl(d2_ctx* c, int32_t K, int32_t m,
                             const double* Xc, const double* Wc) {
  if (!c->N) return c->fail(D2_ESTATE, "load instances first");
  if (K < 1 || !Xc || !Wc) return c->fail(D2_EINVAL, "bad centroid arguments");
  d2_status s = check_limits(c, m);
  if (s) return s;
  if (!finite_all(Xc, (size_t)K * m * c->d))
    return c->fail(D2_EINVAL, "non-finite centroid support");
  for (int q = 0; q < K; ++q) {
    double sum = 0.0;
    for (int i = 0; i < m; ++i) {
      double v = Wc[(size_t)q * m + i];
      if (!(v >= 0.0) || !std::isfinite(v))
        return c->fail(D2_EINVAL, "centroid weights must be finite, >= 0");
      sum += v;
    }
    if (!(std::fabs(sum - 1.0) <= 1e-6))
      return c->fail(D2_EINVAL, "centroid " + std::to_string(q) +
                                    ": weights do not sum to 1");
  }
  HIPCHK(c, hipSetDevice(c->device));
  bool reshape = (K != c->K || m != c->m);
  if ((s = set_centroids_host(c, K, m, Xc, Wc))) return s;
  c->R = slots_for(c);
  if (reshape) {
    c->have_labels = false;
    c->have_cache = false;
  }
  return D2_OK;
}

d2_status d2_centroids_set(d2_ctx* c, int32_t K, int32_t m, const double* Xc,
                           const double* Wc) {
  if (!c) return D2_EINVAL;
  if (c->sym)
    return c->fail(D2_EINVAL, "symbolic instances: set the centroids with "
                              "d2_centroids_set_symbolic");
  return centroids_set_impl(c, K, m, Xc, Wc);
}

d2_status d2_centroids_set_symbolic(d2_ctx* c, int32_t K, int32_t m,
                                    const int32_t* csym, const double* Wc) {
  if (!c) return D2_EINVAL;
  if (!c->sym)
    return c->fail(D2_ESTATE, "load symbolic instances first");
  if (K < 1 || m < 1 || !csym || !Wc)
    return c->fail(D2_EINVAL, "bad centroid arguments");
  for (int64_t q = 0; q < (int64_t)K * m; ++q)
    if (csym[q] < 0 || csym[q] >= c->S)
      return c->fail(D2_EINVAL, "centroid symbol out of range at " +
                                    std::to_string(q));
  std::vector<double> zx((size_t)K * m, 0.0);
  d2_status s = centroids_set_impl(c, K, m, zx.data(), Wc);
  if (s) return s;
  const int MP = c->MP;
  std::vector<int32_t> hs((size_t)K * MP, 0);
  for (int q = 0; q < K; ++q)
    for (int i = 0; i < m; ++i)
      hs[(size_t)q * MP + i] = csym[(size_t)q * m + i];
  if (!c->d_csym || c->h_csym.size() != (size_t)K * m) {
    dfree(c->d_csym);
    drop_graph(c);
    if ((s = dalloc(c, (void**)&c->d_csym, sizeof(int32_t) * hs.size())))
      return s;
  }
  HIPCHK(c, hipMemcpy(c->d_csym, hs.data(), sizeof(int32_t) * hs.size(),
                      hipMemcpyHostToDevice));
  // the stored assignment bounds refer to the previous symbols
  if (c->h_csym.size() != (size_t)K * m ||
      !std::equal(c->h_csym.begin(), c->h_csym.end(), csym))
    c->lbs_valid = false;
  c->h_csym.assign(csym, csym + (size_t)K * m);
  return D2_OK;
}

d2_status d2_centroids_get(d2_ctx* c, double* Xc, double* Wc) {
  if (!c) return D2_EINVAL;
  if (!c->d_xc) return c->fail(D2_ESTATE, "no centroids");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int K = c->K, m = c->m, MP = c->MP, d = c->d;
  std::vector<double> hx((size_t)K * MP * d), hw((size_t)K * MP);
  HIPCHK(c, hipMemcpy(hx.data(), c->d_xc, hx.size() * 8,
                      hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hw.data(), c->d_wc, hw.size() * 8,
                      hipMemcpyDeviceToHost));
  for (int q = 0; q < K; ++q)
    for (int i = 0; i < m; ++i) {
      if (Wc) Wc[(size_t)q * m + i] = hw[(size_t)q * MP + i];
      if (Xc && c->sym)
        Xc[(size_t)q * m + i] = (double)c->h_csym[(size_t)q * m + i];
      else if (Xc)
        for (int t = 0; t < d; ++t)
          Xc[((size_t)q * m + i) * d + t] = hx[((size_t)q * MP + i) * d + t];
    }
  return D2_OK;
}

d2_status d2_centroids_init(d2_ctx* c, int32_t K, int32_t m,
                            const int64_t* members) {
  if (!c) return D2_EINVAL;
  if (!c->N) return c->fail(D2_ESTATE, "load instances first");
  if (K < 1 || !members) return c->fail(D2_EINVAL, "bad init arguments");
  if (c->sym)
    return c->fail(D2_EINVAL, "symbolic instances: the merge initialisation "
                              "needs vector supports");
  d2_status s = check_limits(c, m);
  if (s) return s;
  const int d = c->d;
  // instance data back from the device is not needed: keep a host copy
  // of the chosen members only
  std::vector<double> Xc((size_t)K * m * d), Wc((size_t)K * m);
  for (int q = 0; q < K; ++q) {
    int64_t k = members[q];
    if (k < 0 || k >= c->N)
      return c->fail(D2_EINVAL, "member index out of range");
    int mk = (int)(c->h_off[k + 1] - c->h_off[k]);
    if (mk < m)
      return c->fail(D2_EINVAL, "member " + std::to_string(k) +
                                    " has fewer than m support points");
    std::vector<double> yp((size_t)mk * c->xs), y((size_t)mk * d), wy(mk);
    const size_t xo = (size_t)c->h_off[k] * c->xs;
    if (c->dt == D2_F64) {
      if ((s = download_conv<double>(c, yp.data(), (const double*)c->d_X + xo,
                                     yp.size())))
        return s;
      if ((s = download_conv<double>(c, wy.data(),
                                     (const double*)c->d_W + c->h_off[k], mk)))
        return s;
    } else {
      if ((s = download_conv<float>(c, yp.data(), (const float*)c->d_X + xo,
                                    yp.size())))
        return s;
      if ((s = download_conv<float>(c, wy.data(),
                                    (const float*)c->d_W + c->h_off[k], mk)))
        return s;
    }
    for (int j = 0; j < mk; ++j)
      for (int t = 0; t < d; ++t)
        y[(size_t)j * d + t] = yp[(size_t)j * c->xs + t];
    merge_support(mk, d, y.data(), wy.data(), m, &Xc[(size_t)q * m * d],
                  &Wc[(size_t)q * m]);
  }
  if ((s = d2_centroids_set(c, K, m, Xc.data(), Wc.data()))) return s;
  // fresh centroids: cached plans of earlier ones are not a warm start
  c->have_cache = false;
  return D2_OK;
}

d2_status d2_labels_set(d2_ctx* c, const int32_t* labels) {
  if (!c) return D2_EINVAL;
  if (!c->N || !c->K) return c->fail(D2_ESTATE, "need instances, centroids");
  if (!labels) return c->fail(D2_EINVAL, "null labels");
  for (int64_t k = 0; k < c->N; ++k)
    if (labels[k] < 0 || labels[k] >= c->K)
      return c->fail(D2_EINVAL, "label out of range at " + std::to_string(k));
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, c->sync_labels());
  const bool same =
      c->have_labels && std::equal(c->h_labels.begin(), c->h_labels.end(),
                                   labels);
  c->h_labels.assign(labels, labels + c->N);
  c->hlab_ok = true;
  if (!same) ++c->label_gen;
  HIPCHK(c, hipMemcpy(c->d_labels, labels, sizeof(int32_t) * c->N,
                      hipMemcpyHostToDevice));
  c->have_labels = true;
  c->lists_valid = false;
  return D2_OK;
}

d2_status d2_labels_get(d2_ctx* c, int32_t* labels) {
  if (!c) return D2_EINVAL;
  if (!c->have_labels) return c->fail(D2_ESTATE, "no labels");
  if (!labels) return c->fail(D2_EINVAL, "null labels");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, c->sync_labels());
  std::copy(c->h_labels.begin(), c->h_labels.end(), labels);
  return D2_OK;
}

d2_status d2_assign(d2_ctx* c, const d2_ot_params* p, int32_t* labels_out,
                    double* dist_out, int64_t* n_changed) {
  if (!c) return D2_EINVAL;
  if (!c->N || !c->K) return c->fail(D2_ESTATE, "need instances, centroids");
  if (!p || p->iters < 1 || !(p->rho0 > 0) || !(p->eps >= 0))
    return c->fail(D2_EINVAL, "bad transport parameters");
  HIPCHK(c, hipSetDevice(c->device));
  // the labels before the assignment, for the count of changes
  if (c->have_labels)
    HIPCHK(c, hipMemcpyAsync(c->d_prev_labels, c->d_labels,
                             sizeof(int32_t) * c->N, hipMemcpyDeviceToDevice,
                             c->stream));
  d2_status s = c->dt == D2_F64 ? run_assign<double>(c, p, nullptr)
                                : run_assign<float>(c, p, nullptr);
  if (s) return s;
  int64_t changed = c->N;
  if (c->have_labels) {
    HIPCHK(c, hipMemsetAsync(c->d_nchg, 0, sizeof(int64_t), c->stream));
    hipLaunchKernelGGL(k_count_changes, dim3(512), dim3(256), 0, c->stream,
                       c->d_labels, c->d_prev_labels, c->N, c->d_nchg);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&changed, c->d_nchg, sizeof(int64_t),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (changed > 0) {
    ++c->label_gen;
    c->hlab_ok = false;
    c->lists_valid = false;
  }
  c->have_labels = true;
  if (labels_out) {
    HIPCHK(c, c->sync_labels());
    std::copy(c->h_labels.begin(), c->h_labels.end(), labels_out);
  }
  if (dist_out)
    HIPCHK(c, hipMemcpy(dist_out, c->d_best, sizeof(double) * c->N,
                        hipMemcpyDeviceToHost));
  if (n_changed) *n_changed = changed;
  return D2_OK;
}

d2_status d2_assign_pairs(const d2_ctx* c, int64_t* evaluated,
                          int64_t* costed, int64_t* total) {
  if (!c) return D2_EINVAL;
  // sums of the per-instance counts of the last assignment
  int64_t ev = 0, co = 0;
  if (c->last_pairs > 0) {
    std::vector<int32_t> cnt(2 * (size_t)c->N);
    if (hipSetDevice(c->device) != hipSuccess ||
        hipMemcpy(cnt.data(), c->d_pairs, sizeof(int32_t) * cnt.size(),
                  hipMemcpyDeviceToHost) != hipSuccess)
      return D2_EDEVICE;
    for (size_t q = 0; q < cnt.size(); q += 2) {
      ev += cnt[q];
      co += cnt[q + 1];
    }
  }
  if (evaluated) *evaluated = ev;
  if (costed) *costed = co;
  if (total) *total = c->last_pairs;
  return D2_OK;
}

// Probe gate of the learned warm start: a short B-ADMM run (ws_gate
// iterations, product start) from the current centroid and from the
// network's proposal; per cluster the start whose rounded-plan objective
// (an upper bound on Eq. (centroid), see d2_objective_feasible) is lower
// after the probe is kept (ties keep the current centroid).  Leaves the
// chosen starting centroids set and no plan cache.
static d2_status probe_gate(d2_ctx* c, const d2_badmm_params* p) {
  const int K = c->K, m = c->m, d = c->d;
  d2_status s;
  std::vector<double> X0((size_t)K * m * d), W0((size_t)K * m);
  std::vector<double> X1(X0.size()), W1(W0.size()), F0(K), F1(K);
  if ((s = d2_centroids_get(c, X0.data(), W0.data()))) return s;
  d2_badmm_params q = *p;
  q.iters = c->ws_gate;
  q.init = D2_INIT_PRODUCT;
  if ((s = d2_ws_propose(c->ws, c, 0, nullptr, nullptr, nullptr))) {
    const char* e = d2_ws_last_error(c->ws);
    return c->fail(s, std::string("warm-start proposal: ") + (e ? e : ""));
  }
  if ((s = d2_centroids_get(c, X1.data(), W1.data()))) return s;
  if ((s = d2_barycenter(c, &q, nullptr))) return s;
  if ((s = d2_objective_feasible(c, nullptr, F1.data()))) return s;
  if ((s = centroids_set_impl(c, K, m, X0.data(), W0.data()))) return s;
  if ((s = d2_barycenter(c, &q, nullptr))) return s;
  if ((s = d2_objective_feasible(c, nullptr, F0.data()))) return s;
  for (int q2 = 0; q2 < K; ++q2)
    if (F1[q2] < F0[q2]) {
      std::copy(&X1[(size_t)q2 * m * d], &X1[(size_t)(q2 + 1) * m * d],
                &X0[(size_t)q2 * m * d]);
      std::copy(&W1[(size_t)q2 * m], &W1[(size_t)(q2 + 1) * m],
                &W0[(size_t)q2 * m]);
    }
  if ((s = centroids_set_impl(c, K, m, X0.data(), W0.data()))) return s;
  c->have_cache = false;
  return D2_OK;
}

d2_status d2_barycenter(d2_ctx* c, const d2_badmm_params* p,
                        d2_badmm_stats* st) {
  if (!c) return D2_EINVAL;
  if (!c->N || !c->K) return c->fail(D2_ESTATE, "need instances, centroids");
  if (!c->have_labels) return c->fail(D2_ESTATE, "need labels");
  if (!p || p->iters < 1 || p->tau < 1 || !(p->rho0 > 0) || !(p->eps >= 0) ||
      (p->rule != 1 && p->rule != 2) || p->xplan != 0 ||
      (p->init != D2_INIT_PRODUCT && p->init != D2_INIT_CACHED &&
       p->init != D2_INIT_LEARNED))
    return c->fail(D2_EINVAL, "bad B-ADMM parameters");
  if (p->init == D2_INIT_LEARNED && !c->ws)
    return c->fail(D2_ESTATE, "D2_INIT_LEARNED needs d2_set_warm_start");
  if (p->init == D2_INIT_LEARNED && c->sym)
    return c->fail(D2_EINVAL, "no learned warm start for symbolic supports");
  HIPCHK(c, hipSetDevice(c->device));
  d2_status s;
  if (p->init == D2_INIT_LEARNED) {
    // the network proposes each cluster's starting centroid from its
    // members (gated against the current centroid); plans start from the
    // product coupling
    if (c->ws_gate >= 2) {
      if ((s = probe_gate(c, p))) return s;
    } else if ((s = d2_ws_propose(c->ws, c, c->ws_gate, nullptr, nullptr,
                                  nullptr))) {
      const char* e = d2_ws_last_error(c->ws);
      return c->fail(s, std::string("warm-start proposal: ") + (e ? e : ""));
    }
  }
  if ((s = ensure_plans(c))) return s;
  if ((s = build_lists(c, p->init == D2_INIT_CACHED))) return s;
  // symbolic supports never move: the support step is skipped (Sec. 5)
  d2_badmm_params q = *p;
  if (c->sym) q.fixed_support = 1;
  return c->dt == D2_F64 ? run_barycenter<double>(c, &q, st)
                         : run_barycenter<float>(c, &q, st);
}

d2_status d2_support_update(d2_ctx* c) {
  if (!c) return D2_EINVAL;
  if (c->sym)
    return c->fail(D2_EINVAL, "symbolic supports are fixed (Sec. 5)");
  if (!c->have_cache || !c->have_labels || c->cache_gen != c->label_gen)
    return c->fail(D2_ESTATE, "need a barycenter on the current labels");
  HIPCHK(c, hipSetDevice(c->device));
  d2_status s;
  if (!c->lists_valid && (s = build_lists(c, false))) return s;
  int nl = 0;
  if (c->dt == D2_F64) {
    auto a = make_args<double>(c, nullptr);
    a.xout = c->d_partx;
    s = launch_aux<double>(c, a, d2k::kXO, nl);
  } else {
    auto a = make_args<float>(c, nullptr);
    a.xout = c->d_partx;
    s = launch_aux<float>(c, a, d2k::kXO, nl);
  }
  if (s) return s;
  if ((s = launch_fin(c, make_fin(c, nullptr), d2k::kFinX, nl))) return s;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  return D2_OK;
}

d2_status d2_cluster(d2_ctx* c, int32_t rounds, const d2_badmm_params* bp,
                     const d2_ot_params* op, d2_round_cb cb, void* user) {
  if (!c) return D2_EINVAL;
  if (rounds < 0 || !bp || !op) return c->fail(D2_EINVAL, "bad arguments");
  for (int r = 0; r < rounds; ++r) {
    d2_round_info info;
    std::memset(&info, 0, sizeof(info));
    info.round = r;
    int64_t changed = 0;
    float msa = 0.f;
    if (!c->N || !c->K) return c->fail(D2_ESTATE, "need instances, centroids");
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<double> best(c->N);
    d2_status s = d2_assign(c, op, nullptr, best.data(), &changed);
    if (s) return s;
    (void)msa;
    double sum = 0.0;
    for (double v : best) sum += v;
    info.n_changed = changed;
    info.assign_obj = sum / (double)c->N;
    d2_badmm_params q = *bp;
    q.init = (r == 0 && !c->have_cache) ? D2_INIT_PRODUCT : bp->init;
    d2_badmm_stats st;
    if ((s = d2_barycenter(c, &q, &st))) return s;
    info.ms_barycenter = st.ms;
    if (cb) cb(&info, user);
  }
  return D2_OK;
}

d2_status d2_assign_multi(int32_t n_modal, d2_ctx* const* ctxs,
                          const d2_ot_params* p, int32_t* labels_out,
                          double* dist_out, int64_t* n_changed) {
  if (n_modal < 1 || !ctxs || !ctxs[0]) return D2_EINVAL;
  d2_ctx* c0 = ctxs[0];
  if (!p || p->iters < 1 || !(p->rho0 > 0) || !(p->eps >= 0))
    return c0->fail(D2_EINVAL, "bad transport parameters");
  for (int i = 0; i < n_modal; ++i) {
    d2_ctx* c = ctxs[i];
    if (!c) return c0->fail(D2_EINVAL, "null context");
    if (!c->N || !c->K)
      return c0->fail(D2_ESTATE, "modality " + std::to_string(i) +
                                     ": need instances, centroids");
    if (c->device != c0->device || c->N != c0->N || c->K != c0->K)
      return c0->fail(D2_EINVAL, "modality " + std::to_string(i) +
                                     ": device, N or K differ");
  }
  HIPCHK(c0, hipSetDevice(c0->device));
  const int64_t N = c0->N;
  const int K = c0->K;
  const size_t need = (size_t)N * K;
  if (need > c0->dall_cap) {
    dfree(c0->d_dall);
    c0->dall_cap = 0;
    d2_status s = dalloc(c0, (void**)&c0->d_dall, sizeof(double) * need);
    if (s) return s;
    c0->dall_cap = need;
  }
  // every modality's distances, all pairs, summed in modality order
  for (int i = 0; i < n_modal; ++i)
    HIPCHK(c0, hipStreamSynchronize(ctxs[i]->stream));
  HIPCHK(c0, hipMemsetAsync(c0->d_dall, 0, sizeof(double) * need,
                            c0->stream));
  HIPCHK(c0, hipStreamSynchronize(c0->stream));
  d2_ot_params q = *p;
  q.prune = 0;
  for (int i = 0; i < n_modal; ++i) {
    d2_ctx* c = ctxs[i];
    if (c->have_labels)
      HIPCHK(c0, hipMemcpyAsync(c->d_prev_labels, c->d_labels,
                                sizeof(int32_t) * N, hipMemcpyDeviceToDevice,
                                c->stream));
    d2_status s = c->dt == D2_F64
                      ? run_assign<double>(c, &q, nullptr, c0->d_dall)
                      : run_assign<float>(c, &q, nullptr, c0->d_dall);
    if (s) {
      if (c != c0) c0->fail(s, "modality " + std::to_string(i) + ": " + c->err);
      return s;
    }
  }
  hipLaunchKernelGGL(k_argmin_rows, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, c0->stream, c0->d_dall, N, K, c0->d_labels,
                     c0->d_best);
  HIPCHK(c0, hipGetLastError());
  HIPCHK(c0, hipStreamSynchronize(c0->stream));
  int64_t ch0 = N;
  for (int i = 0; i < n_modal; ++i) {
    d2_ctx* c = ctxs[i];
    if (c != c0) {
      HIPCHK(c0, hipMemcpyAsync(c->d_labels, c0->d_labels,
                                sizeof(int32_t) * N, hipMemcpyDeviceToDevice,
                                c->stream));
      HIPCHK(c0, hipMemcpyAsync(c->d_best, c0->d_best, sizeof(double) * N,
                                hipMemcpyDeviceToDevice, c->stream));
    }
    int64_t changed = N;
    if (c->have_labels) {
      HIPCHK(c0, hipMemsetAsync(c->d_nchg, 0, sizeof(int64_t), c->stream));
      hipLaunchKernelGGL(k_count_changes, dim3(512), dim3(256), 0, c->stream,
                         c->d_labels, c->d_prev_labels, N, c->d_nchg);
      HIPCHK(c0, hipGetLastError());
      HIPCHK(c0, hipMemcpyAsync(&changed, c->d_nchg, sizeof(int64_t),
                                hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c0, hipStreamSynchronize(c->stream));
    if (changed > 0) {
      ++c->label_gen;
      c->hlab_ok = false;
      c->lists_valid = false;
    }
    c->have_labels = true;
    if (i == 0) ch0 = changed;
  }
  if (labels_out) {
    HIPCHK(c0, c0->sync_labels());
    std::copy(c0->h_labels.begin(), c0->h_labels.end(), labels_out);
  }
  if (dist_out)
    HIPCHK(c0, hipMemcpy(dist_out, c0->d_best, sizeof(double) * N,
                         hipMemcpyDeviceToHost));
  if (n_changed) *n_changed = ch0;
  return D2_OK;
}

d2_status d2_cluster_multi(int32_t n_modal, d2_ctx* const* ctxs,
                           int32_t rounds, const d2_badmm_params* bp,
                           const d2_ot_params* op, d2_round_cb cb,
                           void* user) {
  if (n_modal < 1 || !ctxs || !ctxs[0]) return D2_EINVAL;
  d2_ctx* c0 = ctxs[0];
  if (rounds < 0 || !bp || !op) return c0->fail(D2_EINVAL, "bad arguments");
  std::vector<double> best(c0->N);
  for (int r = 0; r < rounds; ++r) {
    d2_round_info info;
    std::memset(&info, 0, sizeof(info));
    info.round = r;
    int64_t changed = 0;
    d2_status s = d2_assign_multi(n_modal, ctxs, op, nullptr, best.data(),
                                  &changed);
    if (s) return s;
    double sum = 0.0;
    for (double v : best) sum += v;
    info.n_changed = changed;
    info.assign_obj = sum / (double)c0->N;
    // the modalities' centroids are updated separately (Sec. 5)
    for (int i = 0; i < n_modal; ++i) {
      d2_ctx* c = ctxs[i];
      d2_badmm_params q = *bp;
      q.init = (r == 0 && !c->have_cache) ? D2_INIT_PRODUCT : bp->init;
      d2_badmm_stats st;
      if ((s = d2_barycenter(c, &q, &st))) {
        if (c != c0) c0->fail(s, "modality " + std::to_string(i) + ": " + c->err);
        return s;
      }
      info.ms_barycenter += st.ms;
    }
    if (cb) cb(&info, user);
  }
  return D2_OK;
}

d2_status d2_subgradient(d2_ctx* c, const d2_sg_params* p, d2_sg_stats* st) {
  if (!c) return D2_EINVAL;
  if (!c->N || !c->K) return c->fail(D2_ESTATE, "need instances, centroids");
  if (!c->have_labels) return c->fail(D2_ESTATE, "need labels");
  if (!p || p->iters < 1 || p->tau < 1 || !(p->alpha > 0.0) ||
      !(p->zeta > 0.0) || p->max_pivots < 0)
    return c->fail(D2_EINVAL, "bad subgradient parameters");
  HIPCHK(c, hipSetDevice(c->device));
  d2_status s;
  if ((s = ensure_plans(c))) return s;
  if ((s = build_lists(c, false))) return s;
  const int K = c->K, MP = c->MP, T_ = p->iters;
  const int64_t N = c->N;
  if (c->sg_N != N || c->sg_KMP != K * MP) {
    dfree(c->d_sgU);
    dfree(c->d_sgval);
    dfree(c->d_sgs);
    dfree(c->d_sgfail);
    dfree(c->d_sgpiv);
    c->sg_N = 0;
    if ((s = dalloc(c, (void**)&c->d_sgU, sizeof(double) * N * MP))) return s;
    if ((s = dalloc(c, (void**)&c->d_sgval, sizeof(double) * N))) return s;
    if ((s = dalloc(c, (void**)&c->d_sgs, sizeof(double) * K * MP))) return s;
    if ((s = dalloc(c, (void**)&c->d_sgfail, sizeof(int)))) return s;
    if ((s = dalloc(c, (void**)&c->d_sgpiv, sizeof(unsigned long long))))
      return s;
    c->sg_N = N;
    c->sg_KMP = K * MP;
  }
  if (T_ > c->trace_cap) {
    drop_graph(c);
    dfree(c->d_trace);
    dfree(c->d_rtrace);
    c->trace_cap = 0;
    if ((s = dalloc(c, (void**)&c->d_trace, sizeof(double) * T_ * K)))
      return s;
    if ((s = dalloc(c, (void**)&c->d_rtrace, sizeof(double) * T_ * K)))
      return s;
    c->trace_cap = T_;
  }
  HIPCHK(c, hipMemsetAsync(c->d_trace, 0, sizeof(double) * T_ * K, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_rtrace, 0, sizeof(double) * T_ * K,
                           c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_sgfail, 0, sizeof(int), c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_sgpiv, 0, sizeof(unsigned long long),
                           c->stream));
  const size_t xbytes = sizeof(double) * (size_t)K * MP * c->d;
  const size_t wbytes = sizeof(double) * (size_t)K * MP;
  HIPCHK(c, hipMemcpyAsync(c->d_xsave, c->d_xc, xbytes,
                           hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_wsave, c->d_wc, wbytes,
                           hipMemcpyDeviceToDevice, c->stream));
  d2s::LpArgs la;
  la.off = c->d_off;
  la.pofs = c->d_pofs;
  la.labels = c->d_labels;
  la.xc = c->d_xc;
  la.wc = c->d_wc;
  la.X = c->d_X;
  la.W = c->d_W;
  la.dsym = c->sym ? c->d_D : nullptr;
  la.isym = c->d_isym;
  la.csym = c->d_csym;
  la.S = c->S;
  la.P1 = c->d_P1;
  la.P2 = c->d_P2;
  la.U = c->d_sgU;
  la.val = c->d_sgval;
  la.fail = c->d_sgfail;
  la.pivots = c->d_sgpiv;
  la.N = N;
  la.m = c->m;
  la.MP = MP;
  la.d = c->d;
  la.xs = c->xs;
  la.mkmax = c->mk_max;
  la.max_pivots = p->max_pivots > 0 ? p->max_pivots
                                    : 50 * (c->m + c->mk_max);
  la.f64 = c->dt == D2_F64 ? 1 : 0;
  const size_t per = d2s::lp_lds_bytes(MP, c->mk_max);
  int lw = 4;
  while (lw > 1 && per * lw > 64 * 1024) --lw;
  const unsigned lgrid = (unsigned)((N + lw - 1) / lw);
  d2s::StepArgs sa;
  sa.work = c->d_work;
  sa.chunks = c->d_chunks;
  sa.ctab = c->d_ctab;
  sa.U = c->d_sgU;
  sa.val = c->d_sgval;
  sa.s = c->d_sgs;
  sa.wc = c->d_wc;
  sa.alpha = p->alpha;
  sa.zeta = p->zeta;
  sa.m = c->m;
  sa.MP = MP;
  const bool xupd = !p->fixed_support && !c->sym;
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  hipLaunchKernelGGL(d2s::k_sg_init, dim3((K + 63) / 64), dim3(64), 0,
                     c->stream, c->d_sgs, c->d_wc, K, c->m, MP);
  HIPCHK(c, hipGetLastError());
  int nl = 1;
  for (int n = 0; n < T_; ++n) {
    if (xupd && n > 0 && n % p->tau == 0) {
      // Eq. (updatex) from the previous iteration's exact plans (Pi2)
      if (c->dt == D2_F64) {
        auto a = make_args<double>(c, nullptr);
        a.xout = c->d_partx;
        if ((s = launch_aux<double>(c, a, d2k::kXO, nl))) return s;
      } else {
        auto a = make_args<float>(c, nullptr);
        a.xout = c->d_partx;
        if ((s = launch_aux<float>(c, a, d2k::kXO, nl))) return s;
      }
      if ((s = launch_fin(c, make_fin(c, nullptr), d2k::kFinX, nl))) return s;
    }
    hipLaunchKernelGGL(d2s::k_lp_transport, dim3(lgrid), dim3(64 * lw),
                       per * lw, c->stream, la);
    HIPCHK(c, hipGetLastError());
    sa.trace = c->d_trace + (size_t)n * K;
    hipLaunchKernelGGL(d2s::k_sg_step, dim3(K), dim3(256), 0, c->stream, sa);
    HIPCHK(c, hipGetLastError());
    nl += 2;
  }
  HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  int nfail = 0;
  unsigned long long npiv = 0;
  HIPCHK(c, hipMemcpy(&nfail, c->d_sgfail, sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&npiv, c->d_sgpiv, sizeof(npiv), hipMemcpyDeviceToHost));
  std::vector<double> hx((size_t)K * MP * c->d), hw((size_t)K * MP);
  HIPCHK(c, hipMemcpy(hx.data(), c->d_xc, hx.size() * 8,
                      hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hw.data(), c->d_wc, hw.size() * 8,
                      hipMemcpyDeviceToHost));
  if (!finite_all(hx.data(), hx.size()) || !finite_all(hw.data(), hw.size())) {
    HIPCHK(c, hipMemcpy(c->d_xc, c->d_xsave, xbytes, hipMemcpyDeviceToDevice));
    HIPCHK(c, hipMemcpy(c->d_wc, c->d_wsave, wbytes, hipMemcpyDeviceToDevice));
    c->have_cache = false;
    c->trace_rows = 0;
    return c->fail(D2_ENUMERIC, "non-finite centroid support or weights "
                                "(centroids restored)");
  }
  // the last iteration's exact plans are the plan cache (Pi2 rows sum to
  // the weights used by that iteration); Lambda has no meaning here
  HIPCHK(c, hipMemsetAsync(c->d_L, 0, (size_t)c->h_pofs[N] * c->esz(),
                           c->stream));
  c->trace_rows = T_;
  HIPCHK(c, hipMemcpyAsync(c->d_cache_labels, c->d_labels,
                           sizeof(int32_t) * N, hipMemcpyDeviceToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->cache_gen = c->label_gen;
  c->hcache_ok = c->hlab_ok;
  if (c->hlab_ok) c->h_cache_labels = c->h_labels;
  c->have_cache = true;
  if (st) {
    st->iters = T_;
    st->lp_failed = nfail;
    st->pivots = (int64_t)npiv;
    st->launches = nl;
    st->ms = ms;
  }
  return D2_OK;
}

d2_status d2_objective(d2_ctx* c, double* trace, int32_t max_iters,
                       double* rho) {
  if (!c) return D2_EINVAL;
  if (!c->trace_rows) return c->fail(D2_ESTATE, "no barycenter yet");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int rows = std::min(max_iters, c->trace_rows);
  if (trace && rows > 0)
    HIPCHK(c, hipMemcpy(trace, c->d_trace, sizeof(double) * rows * c->K,
                        hipMemcpyDeviceToHost));
  if (rho)
    HIPCHK(c, hipMemcpy(rho, c->d_rho, sizeof(double) * c->K,
                        hipMemcpyDeviceToHost));
  return D2_OK;
}

d2_status d2_residual(d2_ctx* c, double* residual, int32_t max_iters) {
  if (!c) return D2_EINVAL;
  if (!c->trace_rows) return c->fail(D2_ESTATE, "no barycenter yet");
  if (!residual) return c->fail(D2_EINVAL, "null output");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int rows = std::min(max_iters, c->trace_rows);
  if (rows > 0)
    HIPCHK(c, hipMemcpy(residual, c->d_rtrace, sizeof(double) * rows * c->K,
                        hipMemcpyDeviceToHost));
  return D2_OK;
}

d2_status d2_plans_get(d2_ctx* c, int64_t k, double* P1, double* P2,
                       double* L) {
  if (!c) return D2_EINVAL;
  if (!c->d_P1 || !c->have_cache) return c->fail(D2_ESTATE, "no plans yet");
  if (k < 0 || k >= c->N) return c->fail(D2_EINVAL, "instance out of range");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  size_t cnt = (size_t)c->m * (c->h_off[k + 1] - c->h_off[k]);
  size_t ofs = (size_t)c->h_pofs[k];
  void* src[3] = {c->d_P1, c->d_P2, c->d_L};
  double* dst[3] = {P1, P2, L};
  for (int q = 0; q < 3; ++q) {
    if (!dst[q]) continue;
    d2_status s =
        c->dt == D2_F64
            ? download_conv<double>(c, dst[q], (const double*)src[q] + ofs, cnt)
            : download_conv<float>(c, dst[q], (const float*)src[q] + ofs, cnt);
    if (s) return s;
  }
  return D2_OK;
}

d2_status d2_set_profiling(d2_ctx* c, int32_t on) {
  if (!c) return D2_EINVAL;
  c->prof = on != 0;
  return D2_OK;
}

d2_status d2_kernel_stats(d2_ctx* c, d2_kernel_stat* out, int32_t cap,
                          int32_t* count, int32_t reset) {
  if (!c) return D2_EINVAL;
  int n = 0;
  for (int q = 0; q < kKinds; ++q) {
    if (!c->prof_launches[q]) continue;
    if (out && n < cap) {
      std::memset(out[n].name, 0, sizeof(out[n].name));
      std::strncpy(out[n].name, kKindNames[q], sizeof(out[n].name) - 1);
      out[n].launches = c->prof_launches[q];
      out[n].total_ms = c->prof_ms[q];
    }
    ++n;
  }
  if (count) *count = n;
  if (reset)
    for (int q = 0; q < kKinds; ++q) {
      c->prof_launches[q] = 0;
      c->prof_ms[q] = 0.0;
    }
  return D2_OK;
}

d2_status d2_set_warm_start(d2_ctx* c, d2_ws* ws, int32_t gate) {
  if (!c) return D2_EINVAL;
  if (gate < 0) return c->fail(D2_EINVAL, "gate must be >= 0");
  c->ws = ws;
  c->ws_gate = gate;
  return D2_OK;
}

d2_status d2_set_rho(d2_ctx* c, const double* rho) {
  if (!c) return D2_EINVAL;
  if (!rho) {
    if (c->rho_fixed) drop_graph(c);
    c->rho_fixed = false;
    return D2_OK;
  }
  if (!c->K) return c->fail(D2_ESTATE, "set centroids first");
  for (int q = 0; q < c->K; ++q)
    if (!(rho[q] > 0.0) || !std::isfinite(rho[q]))
      return c->fail(D2_EINVAL, "rho must be finite and > 0");
  HIPCHK(c, hipSetDevice(c->device));
  if (!c->d_rho_fix || c->rho_fix_K != c->K) {
    dfree(c->d_rho_fix);
    drop_graph(c);
    d2_status s = dalloc(c, (void**)&c->d_rho_fix, sizeof(double) * c->K);
    if (s) return s;
    c->rho_fix_K = c->K;
  }
  HIPCHK(c, hipMemcpy(c->d_rho_fix, rho, sizeof(double) * c->K,
                      hipMemcpyHostToDevice));
  if (!c->rho_fixed) drop_graph(c);
  c->rho_fixed = true;
  return D2_OK;
}

d2_status d2_set_assign_bounds(d2_ctx* c, int32_t on) {
  if (!c) return D2_EINVAL;
  if (!on) {
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_bounds(c);
  }
  c->use_lbs = on != 0;
  return D2_OK;
}

d2_status d2_set_cache_policy(d2_ctx* c, int32_t policy) {
  if (!c) return D2_EINVAL;
  if (policy < 0 || policy > 2)
    return c->fail(D2_EINVAL, "cache policy must be 0, 1 or 2");
  c->cache_policy = policy;
  return D2_OK;
}

d2_status d2_set_graph(d2_ctx* c, int32_t on) {
  if (!c) return D2_EINVAL;
  c->use_graph = on != 0;
  if (!c->use_graph) drop_graph(c);
  return D2_OK;
}

d2_status d2_set_schedule(d2_ctx* c, int32_t chunk_instances,
                          int32_t waves_per_group) {
  if (!c) return D2_EINVAL;
  if (chunk_instances < 1 || chunk_instances > 4096 ||
      (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4))
    return c->fail(D2_EINVAL, "bad schedule");
  if (chunk_instances != c->chunk_inst) {
    c->chunk_inst = chunk_instances;
    free_lists(c);
  }
  if (c->waves != waves_per_group) drop_graph(c);
  c->waves = waves_per_group;
  return D2_OK;
}

d2_status d2_set_bucketing(d2_ctx* c, int32_t min_pct) {
  if (!c) return D2_EINVAL;
  if (min_pct < 0 || min_pct > 100)
    return c->fail(D2_EINVAL, "bucketing threshold must be in [0, 100]");
  if (min_pct != c->bucket_min_pct) {
    c->bucket_min_pct = min_pct;
    c->lists_valid = false;
    drop_graph(c);
  }
  return D2_OK;
}

d2_status d2_autotune(d2_ctx* c, const d2_badmm_params* p,
                      int32_t* chunk_out, int32_t* waves_out,
                      int32_t* bucket_out, double* ms_out) {
  if (!c) return D2_EINVAL;
  if (!c->N || !c->K || !c->have_labels)
    return c->fail(D2_ESTATE, "need instances, centroids and labels");
  if (!p) return c->fail(D2_EINVAL, "null parameters");
  HIPCHK(c, hipSetDevice(c->device));
  const size_t nx = (size_t)c->K * c->MP * c->d, nw = (size_t)c->K * c->MP;
  std::vector<double> hx(nx), hw(nw);
  HIPCHK(c, hipMemcpy(hx.data(), c->d_xc, nx * 8, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hw.data(), c->d_wc, nw * 8, hipMemcpyDeviceToHost));
  d2_badmm_params q = *p;
  q.init = D2_INIT_PRODUCT;
  const bool prof = c->prof;
  c->prof = false;
  static const int kChunks[] = {16, 32, 64, 128, 256};
  static const int kWaves[] = {2, 4};
  static const int kBuckets[] = {100, 10};
  double best = INFINITY;
  int bc = c->chunk_inst, bw = c->waves, bb = c->bucket_min_pct;
  d2_status s = D2_OK;
  for (int ch : kChunks)
    for (int wv : kWaves)
      for (int bk : kBuckets) {
      if ((s = d2_set_schedule(c, ch, wv))) break;
      if ((s = d2_set_bucketing(c, bk))) break;
      double tmin = INFINITY;
      for (int rep = 0; rep < 2 && !s; ++rep) {  // first call captures
        d2_badmm_stats st;
        HIPCHK(c, hipMemcpy(c->d_xc, hx.data(), nx * 8,
                            hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->d_wc, hw.data(), nw * 8,
                            hipMemcpyHostToDevice));
        if ((s = d2_barycenter(c, &q, &st))) break;
        if (rep > 0) tmin = std::min(tmin, st.ms);
      }
      if (s) break;
      if (tmin < best) {
        best = tmin;
        bc = ch;
        bw = wv;
        bb = bk;
      }
    }
  c->prof = prof;
  HIPCHK(c, hipMemcpy(c->d_xc, hx.data(), nx * 8, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_wc, hw.data(), nw * 8, hipMemcpyHostToDevice));
  c->have_cache = false;
  if (s) return s;
  if ((s = d2_set_schedule(c, bc, bw))) return s;
  if ((s = d2_set_bucketing(c, bb))) return s;
  if (chunk_out) *chunk_out = bc;
  if (waves_out) *waves_out = bw;
  if (bucket_out) *bucket_out = bb;
  if (ms_out) *ms_out = best;
  return D2_OK;
}

d2_status d2_copy_probe(int device, int64_t bytes, int32_t reps,
                        double* gbs, double* ms) {
  if (bytes < (1 << 20) || reps < 1 || !gbs) return D2_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return D2_EDEVICE;
  const int64_t n4 = bytes / 16;
  void *a = nullptr, *b = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  d2_status st = D2_OK;
  float best = 0.f;
  if (hipMalloc(&a, n4 * 16) != hipSuccess ||
      hipMalloc(&b, n4 * 16) != hipSuccess) {
    st = D2_ENOMEM;
  } else if (hipMemset(a, 0, n4 * 16) != hipSuccess ||
             hipEventCreate(&e0) != hipSuccess ||
             hipEventCreate(&e1) != hipSuccess) {
    st = D2_EDEVICE;
  } else {
    // 256 CUs x 8 workgroups of 256 threads
    for (int r = 0; r <= reps && st == D2_OK; ++r) {
      (void)hipEventRecord(e0, nullptr);
      hipLaunchKernelGGL(k_copy_probe, dim3(2048), dim3(256), 0, nullptr,
                         (const float4*)a, (float4*)b, n4);
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = D2_EDEVICE;
        break;
      }
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      if (r > 0 && (best == 0.f || t < best)) best = t;  // first: warm-up
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  (void)hipGetLastError();
  if (st == D2_OK) {
    *gbs = 2.0 * (double)(n4 * 16) / (best * 1e-3) / 1e9;
    if (ms) *ms = best;
  }
  return st;
}

}  // extern "C"

namespace {

// Checkpoint file: a fixed header, then the sections it announces, then a
// checksum of everything before it.
struct CkptHeader {
  char magic[8];
  int32_t version, dtype, d, K, m, MP;
  int32_t chunk, waves, bucket, have_labels, have_cache;
  int64_t N, n, plan_elems;
  uint64_t inst_hash;
};
constexpr char kCkptMagic[8] = {'D', '2', 'C', 'K', 'P', 'T', 0, 1};

struct Hasher {  // FNV-1a over the bytes written / read
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t q = 0; q < n; ++q) h = (h ^ b[q]) * 1099511628211ull;
  }
};

bool write_all(FILE* f, Hasher& hs, const void* p, size_t n) {
  hs.add(p, n);
  return n == 0 || fwrite(p, 1, n, f) == n;
}
bool read_all(FILE* f, Hasher& hs, void* p, size_t n) {
  if (n && fread(p, 1, n, f) != n) return false;
  hs.add(p, n);
  return true;
}

}  // namespace

extern "C" {

d2_status d2_checkpoint_save(d2_ctx* c, const char* path) {
  if (!c) return D2_EINVAL;
  if (!path) return c->fail(D2_EINVAL, "null path");
  if (!c->N || !c->K) return c->fail(D2_ESTATE, "need instances, centroids");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = 1;
  h.dtype = (int32_t)c->dt;
  h.d = c->d;
  h.K = c->K;
  h.m = c->m;
  h.MP = c->MP;
  h.chunk = c->chunk_inst;
  h.waves = c->waves;
  h.bucket = c->bucket_min_pct;
  h.have_labels = c->have_labels ? 1 : 0;
  h.have_cache = (c->have_cache && c->d_P2) ? 1 : 0;
  h.N = c->N;
  h.n = c->n;
  h.plan_elems = h.have_cache ? c->h_pofs[c->N] : 0;
  d2_status s = instance_hash(c, &h.inst_hash);
  if (s) return s;
  HIPCHK(c, c->sync_labels());
  if (h.have_cache) HIPCHK(c, c->sync_cache_labels());
  std::vector<double> hx((size_t)c->K * c->MP * c->d), hw((size_t)c->K * c->MP);
  HIPCHK(c, hipMemcpy(hx.data(), c->d_xc, hx.size() * 8,
                      hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hw.data(), c->d_wc, hw.size() * 8,
                      hipMemcpyDeviceToHost));
  // symbolic supports (d = 1, zero coordinates): the centroid symbols take
  // the place of the coordinates
  if (c->sym)
    for (int q = 0; q < c->K; ++q)
      for (int i = 0; i < c->m; ++i)
        hx[(size_t)q * c->MP + i] = (double)c->h_csym[(size_t)q * c->m + i];
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return c->fail(D2_EINVAL, "cannot open " + tmp + " for writing");
  Hasher hs;
  bool ok = write_all(f, hs, &h, sizeof(h)) &&
            write_all(f, hs, hx.data(), hx.size() * 8) &&
            write_all(f, hs, hw.data(), hw.size() * 8);
  if (ok && h.have_labels)
    ok = write_all(f, hs, c->h_labels.data(), sizeof(int32_t) * c->N);
  if (ok && h.have_cache) {
    ok = write_all(f, hs, c->h_cache_labels.data(), sizeof(int32_t) * c->N);
    // the cached Pi2 in 64 MB pieces
    std::vector<unsigned char> buf((size_t)64 << 20);
    const size_t total = (size_t)h.plan_elems * c->esz();
    for (size_t o = 0; ok && o < total; o += buf.size()) {
      const size_t nb = std::min(buf.size(), total - o);
      if (hipMemcpy(buf.data(), (const unsigned char*)c->d_P2 + o, nb,
                    hipMemcpyDeviceToHost) != hipSuccess) {
        fclose(f);
        std::remove(tmp.c_str());
        return c->fail(D2_EDEVICE, "reading the plan cache");
      }
      ok = write_all(f, hs, buf.data(), nb);
    }
  }
  const uint64_t sum = hs.h;
  ok = ok && fwrite(&sum, 1, 8, f) == 8;
  ok = (fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return c->fail(D2_EINVAL, std::string("writing ") + path + " failed");
  }
  return D2_OK;
}

d2_status d2_checkpoint_load(d2_ctx* c, const char* path) {
  if (!c) return D2_EINVAL;
  if (!path) return c->fail(D2_EINVAL, "null path");
  if (!c->N) return c->fail(D2_ESTATE, "load the same instances first");
  HIPCHK(c, hipSetDevice(c->device));
  FILE* f = fopen(path, "rb");
  if (!f) return c->fail(D2_EINVAL, std::string("cannot open ") + path);
  // read and check everything before the context changes
  Hasher hs;
  CkptHeader h;
  auto bad = [&](const std::string& why) {
    fclose(f);
    return c->fail(D2_EINVAL, std::string(path) + ": " + why);
  };
  if (!read_all(f, hs, &h, sizeof(h))) return bad("truncated header");
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 1)
    return bad("not a checkpoint of this library");
  if (h.dtype != (int32_t)c->dt) return bad("device dtype differs");
  if (h.N != c->N || h.n != c->n || h.d != c->d)
    return bad("instance sizes differ from the loaded instances");
  if (h.K < 1 || h.m < 1 || h.m > 64 || h.MP != pad_rows(h.m) ||
      h.chunk < 1 || h.chunk > 4096 ||
      (h.waves != 1 && h.waves != 2 && h.waves != 4) || h.bucket < 0 ||
      h.bucket > 100)
    return bad("corrupt header");
  uint64_t ih = 0;
  d2_status s = instance_hash(c, &ih);
  if (s) {
    fclose(f);
    return s;
  }
  if (ih != h.inst_hash) return bad("the loaded instances differ");
  std::vector<double> hx((size_t)h.K * h.MP * h.d), hw((size_t)h.K * h.MP);
  std::vector<int32_t> lab, clab;
  if (!read_all(f, hs, hx.data(), hx.size() * 8) ||
      !read_all(f, hs, hw.data(), hw.size() * 8))
    return bad("truncated centroids");
  if (!finite_all(hx.data(), hx.size()) || !finite_all(hw.data(), hw.size()))
    return bad("non-finite centroids");
  std::vector<int32_t> csym;
  if (c->sym) {
    csym.resize((size_t)h.K * h.m);
    for (int q = 0; q < h.K; ++q)
      for (int i = 0; i < h.m; ++i) {
        const double v = hx[(size_t)q * h.MP + i];
        if (!(v >= 0.0 && v < (double)c->S && v == std::floor(v)))
          return bad("centroid symbol out of range");
        csym[(size_t)q * h.m + i] = (int32_t)v;
      }
    std::fill(hx.begin(), hx.end(), 0.0);
  }
  if (h.have_labels) {
    lab.resize(c->N);
    if (!read_all(f, hs, lab.data(), sizeof(int32_t) * c->N))
      return bad("truncated labels");
  }
  std::vector<unsigned char> plans;
  if (h.have_cache) {
    clab.resize(c->N);
    if (!read_all(f, hs, clab.data(), sizeof(int32_t) * c->N))
      return bad("truncated cache labels");
    int64_t pe = 0;
    for (int64_t k = 0; k < c->N; ++k)
      pe += ((int64_t)h.m * (c->h_off[k + 1] - c->h_off[k]) + 31) / 32 * 32;
    if (pe != h.plan_elems) return bad("plan cache size differs");
    plans.resize((size_t)h.plan_elems * c->esz());
    if (!read_all(f, hs, plans.data(), plans.size()))
      return bad("truncated plan cache");
  }
  for (int32_t v : lab)
    if (v < 0 || v >= h.K) return bad("label out of range");
  for (int32_t v : clab)
    if (v < 0 || v >= h.K) return bad("label out of range");
  uint64_t sum = 0;
  const uint64_t want = hs.h;
  if (fread(&sum, 1, 8, f) != 8 || sum != want) return bad("checksum mismatch");
  fclose(f);
  if ((s = check_limits(c, h.m))) return s;
  // apply
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if ((s = ensure_centroid_bufs(c, h.K, h.m))) return s;
  HIPCHK(c, hipMemcpy(c->d_xc, hx.data(), hx.size() * 8,
                      hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_wc, hw.data(), hw.size() * 8,
                      hipMemcpyHostToDevice));
  c->R = slots_for(c);
  free_bounds(c);
  if (c->sym) {
    std::vector<int32_t> hs((size_t)h.K * h.MP, 0);
    for (int q = 0; q < h.K; ++q)
      for (int i = 0; i < h.m; ++i)
        hs[(size_t)q * h.MP + i] = csym[(size_t)q * h.m + i];
    if (!c->d_csym &&
        (s = dalloc(c, (void**)&c->d_csym, sizeof(int32_t) * hs.size())))
      return s;
    HIPCHK(c, hipMemcpy(c->d_csym, hs.data(), sizeof(int32_t) * hs.size(),
                        hipMemcpyHostToDevice));
    c->h_csym = csym;
  }
  if ((s = d2_set_schedule(c, h.chunk, h.waves))) return s;
  if ((s = d2_set_bucketing(c, h.bucket))) return s;
  c->lists_valid = false;
  drop_graph(c);
  c->have_labels = h.have_labels != 0;
  if (c->have_labels) {
    c->h_labels = lab;
    HIPCHK(c, hipMemcpy(c->d_labels, lab.data(), sizeof(int32_t) * c->N,
                        hipMemcpyHostToDevice));
  } else {
    c->h_labels.assign(c->N, 0);
  }
  c->hlab_ok = true;
  ++c->label_gen;
  c->have_cache = false;
  if (h.have_cache) {
    if ((s = ensure_plans(c))) return s;
    HIPCHK(c, hipMemcpy(c->d_P2, plans.data(), plans.size(),
                        hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_cache_labels, clab.data(),
                        sizeof(int32_t) * c->N, hipMemcpyHostToDevice));
    c->h_cache_labels = clab;
    c->hcache_ok = true;
    c->cache_gen = (c->have_labels && clab == lab) ? c->label_gen
                                                    : c->label_gen - 1;
    c->have_cache = true;
  }
  c->trace_rows = 0;
  return D2_OK;
}

d2_status d2_sizes(const d2_ctx* c, int64_t* N, int64_t* n, int32_t* d,
                   int32_t* K, int32_t* m) {
  if (!c) return D2_EINVAL;
  if (N) *N = c->N;
  if (n) *n = c->n;
  if (d) *d = c->d;
  if (K) *K = c->K;
  if (m) *m = c->m;
  return D2_OK;
}

}  // extern "C"

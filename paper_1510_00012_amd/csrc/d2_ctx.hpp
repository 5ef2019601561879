// Internal state of a d2_ctx, shared by the translation units of the
// library (d2_api.hip: B-ADMM and assignment; d2_ws.hip: warm start).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/d2.h"
#include "d2_kernels.hpp"

enum KernelKind {
  kKRho = 0, kKInitA, kKIterBA, kKBF, kKXO, kKAssign, kKFin, kKinds
};

struct d2_ctx {
  int device = 0;
  d2_dtype dt = D2_F32;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // instances
  int64_t N = 0, n = 0;
  int d = 0, xs = 0, mk_max = 0;  // xs: row stride of X, d rounded up to 4
  std::vector<int64_t> h_off;
  std::vector<int64_t> h_pofs;  // plan tile offsets (128-byte aligned), N+1
  int64_t* d_off = nullptr;
  int64_t* d_pofs = nullptr;
  void* d_X = nullptr;
  void* d_W = nullptr;
  bool borrowed = false;  // d_X, d_W belong to the caller (device load)
  // symbolic supports (d2_load_instances_symbolic): d = 1 with zero X,
  // instance symbols, the S x S table in the device dtype, and the
  // centroids' symbols (K x MP, host copy K x m)
  bool sym = false;
  int S = 0;
  int32_t* d_isym = nullptr;
  void* d_D = nullptr;
  int32_t* d_csym = nullptr;
  std::vector<int32_t> h_csym;
  // learned warm start used by D2_INIT_LEARNED (owned by the caller)
  d2_ws* ws = nullptr;
  int ws_gate = 1;
  uint64_t inst_hash = 0;  // fingerprint of the instances (0: not yet)
  // centroids (double on device, rows padded to MP)
  int K = 0, m = 0, MP = 0, R = 0;
  double* d_xc = nullptr;
  double* d_wc = nullptr;
  double* d_xsave = nullptr;  // centroids at the start of a barycenter call
  double* d_wsave = nullptr;  // (restored if it fails numerically)
  double* d_rho = nullptr;
  // rho held at caller values (d2_set_rho) instead of Eq. (rho)
  double* d_rho_fix = nullptr;
  int rho_fix_K = 0;
  bool rho_fixed = false;
  int* d_cnt = nullptr;
  // labels: d_labels is authoritative; h_labels mirrors it when hlab_ok
  // (the assignment leaves the labels on the device).  d_cache_labels are
  // the labels of the last centroid update (whose Pi2 is cached), mirrored
  // in h_cache_labels when hcache_ok.  label_gen changes whenever the
  // labels do; cache_gen is its value at the last centroid update.
  std::vector<int32_t> h_labels, h_cache_labels;
  bool have_labels = false, have_cache = false;
  bool hlab_ok = true, hcache_ok = true;
  uint64_t label_gen = 0, cache_gen = ~0ull;
  int32_t* d_labels = nullptr;
  int32_t* d_cache_labels = nullptr;
  int32_t* d_prev_labels = nullptr;  // labels before the last assignment
  int64_t* d_nchg = nullptr;         // label changes of the last assignment
  double* d_dall = nullptr;          // N x K summed multi-modal distances
  size_t dall_cap = 0;
  // subgradient refinement: per-instance projected duals (N x MP) and LP
  // values, per-cluster log-weights (K x MP), failure / pivot counters
  double* d_sgU = nullptr;
  double* d_sgval = nullptr;
  double* d_sgs = nullptr;
  int* d_sgfail = nullptr;
  unsigned long long* d_sgpiv = nullptr;
  int64_t sg_N = 0;
  int sg_KMP = 0;
  double* d_best = nullptr;
  int32_t* d_pairs = nullptr;  // N x 2: per instance of the last assignment,
                               // transports run and cost blocks formed
  void* d_cmu = nullptr;   // d x K centroid means (device dtype)
  void* d_crad = nullptr;  // K centroid support radii
  void* d_xct = nullptr;   // K x MP x xs centroid supports (device dtype)
  int64_t last_pairs = 0;  // pairs of the last assignment (0: none yet)
  // cross-round assignment bounds: N x K stored lower bounds, the centroid
  // supports they refer to, and the per-centroid drift since then
  bool use_lbs = true, lbs_valid = false;
  float* d_lbs = nullptr;
  double* d_xref = nullptr;
  float* d_dlt = nullptr;
  // assignment: instance ids grouped by slot class (one launch per class,
  // each kernel specialised for its class), built for the current pad(m)
  int32_t* d_alist = nullptr;
  int alist_MP = 0;
  int64_t acnt[6] = {}, aofs[6] = {};
  // plans
  void* d_P1 = nullptr;
  void* d_P2 = nullptr;
  void* d_L = nullptr;
  void* d_C = nullptr;
  bool onfly = true;
  // work lists
  int chunk_inst = 64;  // instances per chunk
  int waves = 4;        // wavefronts per workgroup
  int nchunks = 0, nch_cap = 0;
  int32_t* d_work = nullptr;
  d2k::Chunk* d_chunks = nullptr;
  int2* d_ctab = nullptr;
  double* d_ninv = nullptr;
  double* d_cinv = nullptr;
  uint8_t* d_warm = nullptr;
  double* d_part = nullptr;   // 2 x cap x ps (double-buffered records)
  double* d_partx = nullptr;  // 2 x cap x MP x (d+1) support records
  int* d_nch = nullptr;       // device copy of nchunks
  // Slot buckets of the hot kernel: chunks hold instances of one bucket;
  // bucket b (register slots bk_R[b]) is one launch over the chunk ids
  // d_blist[bk_off[b] .. bk_off[b] + d_bcnt[b]) with grid bk_cap[b].
  int nbk = 0;
  int bk_R[6] = {}, bk_cap[6] = {}, bk_off[6] = {}, bk_cnt[6] = {};
  int32_t* d_blist = nullptr;
  int* d_bcnt = nullptr;
  int blist_cap = 0;
  int bucket_min_pct = 100;
  // cache policy of the plan state in the hot kernel: 0 automatic
  // (streaming when the state per iteration exceeds the last-level
  // cache), 1 default caching, 2 streaming (non-temporal)
  int cache_policy = 0;
  // pinned staging for the per-call list uploads (one host copy, async
  // transfers; stage_ev marks the end of the last batch of transfers)
  uint8_t* h_stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t stage_ev = nullptr;
  // per-instance slot class for the current pad(m), and reused host lists
  std::vector<uint8_t> h_cls;
  int cls_MP = 0;
  double cls_ent[6] = {};
  int64_t cls_cnt[6] = {};  // instances per slot class
  bool host_ctab = false;   // h_ctab matches d_ctab (host-built lists)
  std::vector<uint32_t> h_key;
  std::vector<int32_t> h_work;
  std::vector<uint8_t> h_warm;  // slot classes under this % of entries merge up
  std::vector<int2> h_ctab;
  bool lists_valid = false;
  // device construction of the work list: per-instance slot bucket (for
  // bkt_MP / bkt_pct), per-tile key histograms and per-key scratch
  uint8_t* d_bkt = nullptr;
  int bkt_MP = 0, bkt_pct = -1;
  int32_t* d_tcnt = nullptr;
  int32_t* d_tsum = nullptr;
  int64_t tcnt_cap = 0;
  int64_t* d_keys = nullptr;  // 5 x G: counts, support sums, starts,
  int keys_cap = 0;           // first chunks, bucket offsets
  // objective trace of the last barycenter
  double* d_trace = nullptr;
  double* d_rtrace = nullptr;  // residual trace, same shape as d_trace
  int trace_cap = 0, trace_rows = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // side streams (default priority) for launches that may run side by side
  // -- the slot buckets of one iteration, the slot classes of the
  // assignment -- forked from `stream` and joined back to it by events
  static constexpr int kSide = 5;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kSide] = {};
  // captured launch sequence of d2_barycenter
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<double> graph_key;
  int graph_launches = 0;
  // per-kernel profiling
  bool prof = false;
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
  int64_t prof_launches[kKinds] = {};
  double prof_ms[kKinds] = {};

  d2_status fail(d2_status s, const std::string& msg) {
    err = msg;
    return s;
  }
  // host mirrors of the device labels, refreshed on demand
  hipError_t sync_labels() {
    if (hlab_ok || !d_labels) return hipSuccess;
    h_labels.resize(N);
    hipError_t e = hipMemcpy(h_labels.data(), d_labels, sizeof(int32_t) * N,
                             hipMemcpyDeviceToHost);
    if (e == hipSuccess) hlab_ok = true;
    return e;
  }
  hipError_t sync_cache_labels() {
    if (hcache_ok || !d_cache_labels) return hipSuccess;
    h_cache_labels.resize(N);
    hipError_t e = hipMemcpy(h_cache_labels.data(), d_cache_labels,
                             sizeof(int32_t) * N, hipMemcpyDeviceToHost);
    if (e == hipSuccess) hcache_ok = true;
    return e;
  }
  size_t esz() const { return dt == D2_F64 ? 8 : 4; }
};

#define HIPCHK(ctx, call)                                                 \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess)                                                 \
      return (ctx)->fail(D2_EDEVICE, std::string(#call) + ": " +          \
                                         hipGetErrorString(e_));          \
  } while (0)


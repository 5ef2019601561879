// Assignment step that allocates nothing (d2_assign_noalloc in d2.h).
//
// The same kernels as d2_assign (the pruned or exhaustive B-ADMM transport
// argmin over the centroids, Algorithm "D2 Clustering"), for callers that
// cannot allocate device memory.  Inputs and outputs are the caller's
// device buffers; the per-centroid data the kernels need besides them (the
// centroids repacked to the padded row layout and normalised, their
// support means, radii and device-dtype copies) lives in `scratch`, a
// file-scope device array of fixed size.  Host code never passes the
// array's name to a kernel: the device address of each GPU's copy comes
// from hipGetSymbolAddress, taken once per device with that device current.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/d2.h"
#include "d2_kernels.hpp"

void d2k_fill_f32(d2k::KernTable<float>* t);
void d2k_fill_f32w(d2k::KernTable<float>* t);
void d2k_fill_f64(d2k::KernTable<double>* t);
void d2k_fill_f64w(d2k::KernTable<double>* t);

namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;  // 8 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// ceil(log2(v)) for v >= 1
int clog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

// Scratch layout for K centroids of MP padded rows in d dimensions (row
// stride xs of the instance supports, element size esz): padded centroid
// supports and weights (double), then the lower-bound data of k_cstats
// (support means d x K, radii K, supports K x MP x xs in the device dtype).
struct Layout {
  size_t xc, wc, cmu, crad, xct, total;
};
Layout layout(int K, int MP, int d, int xs, int esz) {
  Layout L;
  L.xc = 0;
  L.wc = L.xc + up256(sizeof(double) * (size_t)K * MP * d);
  L.cmu = L.wc + up256(sizeof(double) * (size_t)K * MP);
  L.crad = L.cmu + up256((size_t)esz * K * d);
  L.xct = L.crad + up256((size_t)esz * K);
  L.total = L.xct + up256((size_t)esz * K * MP * xs);
  return L;
}

// Centroid c's m rows copied to MP padded rows (zeros beyond m), weights
// divided by their sum taken in index order, as d2_centroids_set does on
// the host, so both entry points hand the kernels the same values.
__global__ void __launch_bounds__(64)
    k_pack_centroids(const double* __restrict__ Xc,
                     const double* __restrict__ Wc, int m, int MP, int d,
                     double* __restrict__ xc, double* __restrict__ wc) {
  const int c = blockIdx.x, l = threadIdx.x;
  double sum = 0.0;
  for (int i = 0; i < m; ++i) sum += Wc[(size_t)c * m + i];
  for (int i = l; i < MP; i += 64)
    wc[(size_t)c * MP + i] = i < m ? Wc[(size_t)c * m + i] / sum : 0.0;
  for (int e = l; e < MP * d; e += 64) {
    const int i = e / d;
    xc[(size_t)c * MP * d + e] =
        i < m ? Xc[(size_t)c * m * d + e] : 0.0;
  }
}

template <typename T>
const d2k::KernTable<T>& table();
template <>
const d2k::KernTable<float>& table<float>() {
  static const d2k::KernTable<float> t = [] {
    d2k::KernTable<float> x;
    d2k_fill_f32(&x);
    d2k_fill_f32w(&x);
    return x;
  }();
  return t;
}
template <>
const d2k::KernTable<double>& table<double>() {
  static const d2k::KernTable<double> t = [] {
    d2k::KernTable<double> x;
    d2k_fill_f64(&x);
    d2k_fill_f64w(&x);
    return x;
  }();
  return t;
}

d2_status say(char* err, int32_t err_len, d2_status s, const char* msg) {
  if (err && err_len > 0) {
    std::strncpy(err, msg, (size_t)err_len - 1);
    err[err_len - 1] = '\0';
  }
  return s;
}

template <typename T>
d2_status launch(hipStream_t st, unsigned char* base, const Layout& L,
                 int64_t N, int d, int xs, const int64_t* off, const void* X,
                 const void* W, int K, int m, int MP, int R,
                 const double* Xc, const double* Wc, const d2_ot_params* p,
                 int32_t* labels, double* dist, char* err, int32_t err_len) {
  auto fn = table<T>().asg[clog2(MP) - 3][clog2(R)];
  if (!fn) return say(err, err_len, D2_EINVAL, "no kernel for this tile shape");
  double* xc = reinterpret_cast<double*>(base + L.xc);
  double* wc = reinterpret_cast<double*>(base + L.wc);
  T* cmu = reinterpret_cast<T*>(base + L.cmu);
  T* crad = reinterpret_cast<T*>(base + L.crad);
  T* xct = reinterpret_cast<T*>(base + L.xct);
  hipLaunchKernelGGL(k_pack_centroids, dim3(K), dim3(64), 0, st, Xc, Wc, m,
                     MP, d, xc, wc);
  hipLaunchKernelGGL(d2k::k_cstats<T>, dim3(K), dim3(64), sizeof(double) * d,
                     st, xc, wc, m, MP, d, xs, K, cmu, crad, xct,
                     (const double*)nullptr, (float*)nullptr);
  d2k::AssignArgs<T> a{};
  a.off = off;
  a.X = (const T*)X;
  a.W = (const T*)W;
  a.xc = xc;
  a.wc = wc;
  a.labels = labels;
  a.best = dist;
  a.counts = nullptr;
  a.cmu = cmu;
  a.crad = crad;
  a.xct = xct;
  a.list = nullptr;
  a.lbs = nullptr;
  a.dlt = nullptr;
  a.lbs_in = 0;
  a.N = N;
  a.rho0 = p->rho0;
  a.eps = p->eps;
  a.m = m;
  a.d = d;
  a.xs = xs;
  a.K = K;
  a.iters = p->iters;
  a.prune = p->prune ? 1 : 0;
  a.prev_valid = 0;
  // candidate bounds one per lane as in d2_assign
  a.batch = sizeof(T) == 4 && a.prune && d <= 16 && K >= 32 && MP <= 16 &&
                    (64 / MP) * R <= 32
                ? 1
                : 0;
  const int wpb = 4;
  const int64_t blocks = (N + wpb - 1) / wpb;
  const size_t lds = (size_t)wpb * d2k::assign_lds(d, MP, R, xs,
                                                   (int)sizeof(T), a.batch)
                                       .bytes;
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return say(err, err_len, D2_EDEVICE, hipGetErrorString(e));
  return D2_OK;
}

}  // namespace

extern "C" d2_status d2_assign_noalloc(
    int32_t device, void* hip_stream, d2_dtype dtype, int64_t N, int32_t d,
    int32_t mk_max, const int64_t* offsets, const void* X, const void* W,
    int32_t K, int32_t m, const double* Xc, const double* Wc,
    const d2_ot_params* p, int32_t* labels, double* dist, char* err,
    int32_t err_len) {
  if (err && err_len > 0) err[0] = '\0';
  // argument checks first: they need no device
  if (dtype != D2_F32 && dtype != D2_F64)
    return say(err, err_len, D2_EINVAL, "dtype must be D2_F32 or D2_F64");
  if (N < 0 || N > INT32_MAX)
    return say(err, err_len, D2_EINVAL, "N must be in [0, 2^31 - 1]");
  if (d < 1) return say(err, err_len, D2_EINVAL, "d must be >= 1");
  if (m < 1 || m > 64) return say(err, err_len, D2_EINVAL, "m must be in [1, 64]");
  if (K < 1) return say(err, err_len, D2_EINVAL, "K must be >= 1");
  if (!p || p->iters < 1 || !(p->rho0 > 0.0) || !(p->eps >= 0.0))
    return say(err, err_len, D2_EINVAL,
               "parameters: iters >= 1, rho0 > 0 and eps >= 0 required");
  const int MP = 1 << (clog2(m) > 3 ? clog2(m) : 3);  // pad(m)
  const int cps = 64 / MP;
  if (mk_max < 1 || (mk_max + cps - 1) / cps > 32)
    return say(err, err_len, D2_EINVAL,
               "mk_max must be >= 1 with mk_max * pad(m) <= 2048");
  if ((int64_t)MP * (d + 1) > 8192)
    return say(err, err_len, D2_EINVAL, "pad(m) * (d + 1) exceeds 8192");
  const int xs = (d + 3) / 4 * 4;
  const int esz = dtype == D2_F32 ? 4 : 8;
  const Layout L = layout(K, MP, d, xs, esz);
  if (L.total > kScratchBytes) {
    char msg[160];
    std::snprintf(msg, sizeof msg,
                  "K x pad(m) x d needs %zu scratch bytes, above the limit "
                  "of %zu",
                  L.total, kScratchBytes);
    return say(err, err_len, D2_EINVAL, msg);
  }
  if (N == 0) return D2_OK;
  if (!offsets || !X || !W || !Xc || !Wc || !labels || !dist)
    return say(err, err_len, D2_EINVAL, "a device pointer is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
      device >= kMaxDevices) {
    (void)hipGetLastError();
    return say(err, err_len, D2_EDEVICE, "no such HIP device");
  }
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return say(err, err_len, D2_EDEVICE, "hipSetDevice failed");
  }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[device]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        (void)hipSetDevice(prev);
        return say(err, err_len, D2_EDEVICE,
                   "hipGetSymbolAddress of the scratch array failed");
      }
      g_scratch[device] = ptr;
    }
    base = g_scratch[device];
  }
  const int R = 1 << clog2((mk_max + cps - 1) / cps);  // register slots
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const d2_status s =
      dtype == D2_F32
          ? launch<float>(st, (unsigned char*)base, L, N, d, xs, offsets, X, W,
                          K, m, MP, R, Xc, Wc, p, labels, dist, err, err_len)
          : launch<double>(st, (unsigned char*)base, L, N, d, xs, offsets, X,
                           W, K, m, MP, R, Xc, Wc, p, labels, dist, err,
                           err_len);
  (void)hipSetDevice(prev);
  return s;
}

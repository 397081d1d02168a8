// Multi-query batch kernels: Q queries of one vertex program (personalized
// PageRank or SSSP) on one graph, iterated together.
//
// Values are vertex-major with a padded query stride Qp (a multiple of 64):
// value(u, q) = X[u * Qp + q]. A wavefront takes a (row, 64-query slice)
// pair: its lanes are queries, so each gathered edge reads one contiguous
// 256-byte run of the source's values and the edge word is read once per
// slice. Every query follows the same synchronous iteration as a
// single-query run over the same edge set (all edges, or the shared sampled
// subset).
#include "gg_internal.h"

namespace ggk {

namespace {

__device__ __forceinline__ uint32_t bld(const uint32_t* p) { return __builtin_nontemporal_load(p); }

template <int APP>
struct BTr;
template <>
struct BTr<kPPR> {
  using T = double;
  static __device__ __forceinline__ T id() { return 0.0; }
  static __device__ __forceinline__ T op(T a, T b) { return a + b; }
  static __device__ __forceinline__ T elem(const BatchSweep& s, uint32_t e, int q) {
    return (double)s.c_in[(int64_t)e * s.qp + q];
  }
};
template <>
struct BTr<kSSSP> {
  using T = uint32_t;
  static __device__ __forceinline__ T id() { return kInf; }
  static __device__ __forceinline__ T op(T a, T b) { return min(a, b); }
  static __device__ __forceinline__ T elem(const BatchSweep& s, uint32_t e, int q) {
    const uint32_t xv = s.x_in[(int64_t)(e & 0xFFFFFFu) * s.qp + q];
    return xv == kInf ? kInf : xv + (e >> 24);
  }
};

template <int APP>
__device__ __forceinline__ void bapply(const BatchSweep& s, int u, int q, typename BTr<APP>::T acc, int& nchanged) {
  const int64_t o = (int64_t)u * s.qp + q;
  if constexpr (APP == kPPR) {
    const bool src = s.src[q] == u;
    const double x = (src ? (1.0 - s.damping) : 0.0) + s.damping * (acc + (src ? s.dang[q] : 0.0));
    const int od = s.outdeg[u];
    s.c_out[o] = od > 0 ? (float)(x / (double)od) : (float)x;
    if (s.x_out) s.x_out[o] = (float)x;
  } else {
    const uint32_t old = s.x_in[o];
    const uint32_t nv = min(old, acc);
    s.x_next[o] = nv;
    nchanged += (nv != old);
  }
}

// Reduce edges [e0, e1) of the edge array for query q, 8 loads in flight.
template <int APP>
__device__ __forceinline__ typename BTr<APP>::T bgather(const BatchSweep& s, int e0, int e1, int q) {
  using R = BTr<APP>;
  typename R::T acc = R::id();
  int k = e0;
  for (; k + 8 <= e1; k += 8) {
    uint32_t w[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) w[j] = bld(s.edges + k + j);
    typename R::T v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = R::elem(s, w[j], q);
#pragma unroll
    for (int j = 0; j < 8; ++j) acc = R::op(acc, v[j]);
  }
  for (; k < e1; ++k) acc = R::op(acc, R::elem(s, bld(s.edges + k), q));
  return acc;
}

__device__ __forceinline__ int brow_len(const BatchSweep& s, int u, int b) {
  return s.cnt ? s.cnt[u] : s.rowptr[u + 1] - b;
}

__device__ __forceinline__ int bfind_hub(const int32_t* hub_start, int n_hub, int ch) {
  int lo = 0, hi = n_hub - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (hub_start[mid] <= ch) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int APP>
__device__ __forceinline__ void bflush(const BatchSweep& s, int nchanged) {
  if constexpr (APP == kSSSP) {
    // Only whether anything changed is used (the captured loop stops on an
    // iteration without change): a wave sets the flag only while it still
    // reads clear, so the flag is written a handful of times per iteration
    // instead of once per (row, slice).
    const bool any = __ballot(nchanged != 0) != 0;
    if (any && __lane_id() == 0 &&
        __hip_atomic_load(s.changed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      atomicOr(s.changed, 1);
  }
}

// Waves [0, nrow_items): (row of the small/wave bins, slice) pairs, slice
// fastest. Waves [nrow_items, ...): (hub chunk, slice) pairs -> partials.
template <int APP>
__global__ __launch_bounds__(kBlock) void k_bgather(BatchSweep s, int64_t nrow_items, int64_t nitems) {
  if (s.done && *s.done) return;
  const int64_t item = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (item >= nitems) return;
  const int lane = __lane_id();
  int nchanged = 0;
  if (item < nrow_items) {
    const int r = (int)(item / s.nslice);
    const int j = (int)(item - (int64_t)r * s.nslice);
    const int q = j * 64 + lane;
    const int u = s.list[r];
    const int b = s.rowptr[u];
    const int len = brow_len(s, u, b);
    const typename BTr<APP>::T acc = bgather<APP>(s, b, b + len, q);
    bapply<APP>(s, u, q, acc, nchanged);
  } else {
    const int64_t hi_item = item - nrow_items;
    const int ch = (int)(hi_item / s.nslice);
    const int j = (int)(hi_item - (int64_t)ch * s.nslice);
    const int q = j * 64 + lane;
    const int h = bfind_hub(s.hub_start, s.n_hub, ch);
    const int u = s.list[s.n_small + s.n_wave + h];
    const int c = ch - s.hub_start[h];
    const int b = s.rowptr[u];
    const int len = brow_len(s, u, b);
    const int e0 = b + c * s.hub_chunk, e1 = b + min(len, (c + 1) * s.hub_chunk);
    const typename BTr<APP>::T acc = bgather<APP>(s, e0, e1, q);
    if constexpr (APP == kPPR) s.part_f[(int64_t)ch * s.qp + q] = acc;
    else s.part_u[(int64_t)ch * s.qp + q] = acc;
  }
  bflush<APP>(s, nchanged);
}

// (hub row, slice) pairs: combine the chunk partials in chunk order, apply.
template <int APP>
__global__ __launch_bounds__(kBlock) void k_bhub_combine(BatchSweep s) {
  if (s.done && *s.done) return;
  const int64_t item = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (item >= (int64_t)s.n_hub * s.nslice) return;
  const int h = (int)(item / s.nslice);
  const int j = (int)(item - (int64_t)h * s.nslice);
  const int q = j * 64 + __lane_id();
  const int c0 = s.hub_start[h], c1 = s.hub_start[h + 1];
  using R = BTr<APP>;
  typename R::T acc = R::id();
  for (int c = c0; c < c1; ++c) {
    if constexpr (APP == kPPR) acc = R::op(acc, s.part_f[(int64_t)c * s.qp + q]);
    else acc = R::op(acc, s.part_u[(int64_t)c * s.qp + q]);
  }
  int nchanged = 0;
  bapply<APP>(s, s.list[s.n_small + s.n_wave + h], q, acc, nchanged);
  bflush<APP>(s, nchanged);
}


// Per-query dangling mass: chunk c of the dangling list, one wave per
// (chunk, slice), then a fixed-order sum over chunks.
__global__ __launch_bounds__(64) void k_bdang_partial(BatchSweep s, const int32_t* dlist, int ndang,
                                                      double* partial) {
  const int c = blockIdx.x / s.nslice;
  const int j = blockIdx.x - c * s.nslice;
  const int q = j * 64 + __lane_id();
  const int per = (ndang + kBDangChunks - 1) / kBDangChunks;
  const int lo = c * per, hi = min(ndang, lo + per);
  double acc = 0.0;
  int i = lo;
  // eight list entries and their values in flight, added in list order
  for (; i + 8 <= hi; i += 8) {
    int d[8];
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) d[k] = dlist[i + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = s.c_in[(int64_t)d[k] * s.qp + q];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += (double)v[k];
  }
  for (; i < hi; ++i) acc += (double)s.c_in[(int64_t)dlist[i] * s.qp + q];
  partial[(int64_t)c * s.qp + q] = acc;
}

// Sum of the chunk partials of a 64-query slice: wave w adds chunks
// w, w+16, ... in order, then the 16 wave sums are added in order.
__global__ __launch_bounds__(1024) void k_bdang_final(BatchSweep s, const double* partial, double* out) {
  __shared__ double red[16][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int q = blockIdx.x * 64 + l;
  double acc = 0.0;
  for (int c = w; c < kBDangChunks; c += 16) acc += partial[(int64_t)c * s.qp + q];
  red[w][l] = acc;
  __syncthreads();
  if (w == 0) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[k][l];
    out[q] = t;
  }
}

// Initial values: PPR contributions e_s / outdeg; SSSP distances 0 at the
// source, INF elsewhere (both buffers). Padded queries have no source.
__global__ void k_binit(int app, int32_t n, int32_t qp, const int32_t* src, const int32_t* outdeg, float* c,
                        uint32_t* x0, uint32_t* x1) {
  const int64_t total = (int64_t)n * qp;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(i / qp);
    const int q = (int)(i - (int64_t)u * qp);
    const bool is_src = src[q] == u;
    if (app == kPPR) {
      const int od = outdeg[u];
      c[i] = is_src ? (od > 0 ? (float)(1.0 / (double)od) : 1.0f) : 0.0f;
    } else {
      x0[i] = is_src ? 0u : kInf;
      x1[i] = is_src ? 0u : kInf;
    }
  }
}

// After an iteration of a captured SSSP loop: no change -> done; else count it.
__global__ void k_bdone(int32_t* changed, int32_t* done, int32_t* iters) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (*done == 0) {
      *iters += 1;
      if (*changed == 0) *done = 1;
    }
    *changed = 0;
  }
}

}  // namespace

hipError_t launch_batch_init(int app, int32_t n, int32_t qp, const int32_t* src, const int32_t* outdeg, float* c,
                             uint32_t* x0, uint32_t* x1, hipStream_t st) {
  const int64_t total = (int64_t)n * qp;
  if (total == 0) return hipSuccess;
  int64_t g = (total + 2047) / 2048;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_binit, dim3((int)g), dim3(256), 0, st, app, n, qp, src, outdeg, c, x0, x1);
  return hipGetLastError();
}

hipError_t launch_batch_dangling(const BatchSweep& s, const int32_t* dlist, int32_t ndang, double* partial,
                                 double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_bdang_partial, dim3(kBDangChunks * s.nslice), dim3(64), 0, st, s, dlist, ndang, partial);
  hipLaunchKernelGGL(k_bdang_final, dim3(s.nslice), dim3(1024), 0, st, s, partial, out);
  return hipGetLastError();
}

hipError_t launch_batch_gather(int app, const BatchSweep& s, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int64_t nrow_items = (int64_t)(s.n_small + s.n_wave) * s.nslice;
  const int64_t nitems = nrow_items + (int64_t)s.n_chunks * s.nslice;
  const int wpb = kBlock / 64;
  if (ev0) (void)hipEventRecord(ev0, st);
  if (nitems > 0) {
    const int64_t g = (nitems + wpb - 1) / wpb;
    if (app == kPPR)
      hipLaunchKernelGGL(k_bgather<kPPR>, dim3((unsigned)g), dim3(kBlock), 0, st, s, nrow_items, nitems);
    else
      hipLaunchKernelGGL(k_bgather<kSSSP>, dim3((unsigned)g), dim3(kBlock), 0, st, s, nrow_items, nitems);
  }
  if (ev1) (void)hipEventRecord(ev1, st);
  const int64_t hitems = (int64_t)s.n_hub * s.nslice;
  if (hitems > 0) {
    const int64_t g = (hitems + wpb - 1) / wpb;
    if (app == kPPR) hipLaunchKernelGGL(k_bhub_combine<kPPR>, dim3((unsigned)g), dim3(kBlock), 0, st, s);
    else hipLaunchKernelGGL(k_bhub_combine<kSSSP>, dim3((unsigned)g), dim3(kBlock), 0, st, s);
  }
  return hipGetLastError();
}

hipError_t launch_batch_done(int32_t* changed, int32_t* done, int32_t* iters, hipStream_t st) {
  hipLaunchKernelGGL(k_bdone, dim3(1), dim3(64), 0, st, changed, done, iters);
  return hipGetLastError();
}

}  // namespace ggk

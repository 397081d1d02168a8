// Dynamic graphs: device side of an update batch (deletions, then
// insertions) applied to the in-CSR, the remapping of the edge flags, and
// the repair of min-type values after deletions. The method is stated to
// apply to changing graphs [Sec. 1]; the paper evaluates none, so the
// update rules are this library's reading (see include/gg.h).
//
// Arcs of a batch are keyed (destination << 32) | source and radix-sorted
// (stable, so equal arcs keep their batch order). Each distinct deletion
// finds its run of matching edges in the sorted row; the surviving edges and
// the sorted insertions of a row are merged by source, old edges first on
// equal sources, so rows stay sorted by source. Out-degrees and the out-CSR
// of the frontier are carried over (survivors compacted, insertions
// appended) instead of being recounted with one atomic per edge.
#include <hipcub/hipcub.hpp>

#include "gg_internal.h"

namespace ggk {

namespace {

constexpr int kUpdBlock = 256;

int grid_of(int64_t work) {
  int64_t b = (work + kUpdBlock - 1) / kUpdBlock;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

__device__ __forceinline__ uint64_t arc_key(int32_t src, int32_t dst) {
  return ((uint64_t)(uint32_t)dst << 32) | (uint32_t)src;
}

// First index in sorted keys[lo, hi) whose key is >= k.
__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* keys, int64_t lo, int64_t hi, uint64_t k) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Whether edge s -> d (weight w) realises d's value: SSSP x_s + w == x_d
// (d not the source, both finite); CC l_s == l_d with l_d not d's own id.
__device__ __forceinline__ bool supports(int app, const uint32_t* x, int32_t source, int32_t s, int32_t d,
                                         uint32_t w) {
  const uint32_t xs = x[s], xd = x[d];
  if (app == kSSSP) {
    if (d == source || xs == kInf || xd == kInf) return false;
    return (uint64_t)xs + (uint64_t)w == (uint64_t)xd;
  }
  return xs == xd && xd != (uint32_t)d;
}

__global__ void k_batch_check(const int32_t* src, const int32_t* dst, const int32_t* w, int64_t k, int32_t n,
                              int32_t* flags) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < k; j += (int64_t)gridDim.x * blockDim.x) {
    if (src[j] < 0 || src[j] >= n || dst[j] < 0 || dst[j] >= n) atomicOr(flags, 1);
    if (w && (w[j] < 0 || w[j] > 255)) atomicOr(flags, 2);
  }
}

__global__ void k_arc_keys(const int32_t* src, const int32_t* dst, int64_t k, uint64_t* keys, int32_t* idx) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < k; j += (int64_t)gridDim.x * blockDim.x) {
    keys[j] = arc_key(src[j], dst[j]);
    if (idx) idx[j] = (int32_t)j;
  }
}

// Row of every edge. A block takes kUpdBlock consecutive rows, whose edges
// are one contiguous range: it stages their starts in LDS, and each thread
// writes the row ids of every kUpdBlock-th edge of the range (coalesced),
// finding the row by binary search over the staged starts (the last row
// starting at or before the edge; empty rows share their successor's start).
__global__ __launch_bounds__(kUpdBlock) void k_row_ids(const int32_t* rowptr, int32_t n, int32_t* dst) {
  __shared__ int32_t s_rp[kUpdBlock + 1];
  for (int64_t u0 = (int64_t)blockIdx.x * kUpdBlock; u0 < n; u0 += (int64_t)gridDim.x * kUpdBlock) {
    const int cnt = (int)min((int64_t)kUpdBlock, (int64_t)n - u0);
    __syncthreads();  // the previous round's searches are done with s_rp
    if ((int)threadIdx.x < cnt) s_rp[threadIdx.x] = rowptr[u0 + threadIdx.x];
    if (threadIdx.x == 0) s_rp[cnt] = rowptr[u0 + cnt];
    __syncthreads();
    const int32_t base = s_rp[0];
    const int32_t total = s_rp[cnt] - base;
    for (int32_t k = threadIdx.x; k < total; k += kUpdBlock) {
      int lo = 0, hi = cnt - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_rp[mid] - base <= k) lo = mid;
        else hi = mid - 1;
      }
      dst[base + k] = (int32_t)(u0 + lo);
    }
  }
}

// One thread per distinct deletion key (s, d): the matching edges, a run of
// equal sources in the sorted row d, get keep[e] = 0 and leave s's
// out-degree. With x set, a deleted edge that supports d's value appends d
// to the taint list (taint[d] guards against duplicates).
__global__ void k_mark_deleted(const int32_t* rowptr, const int32_t* col, const int32_t* weight,
                               const uint64_t* dkeys, int64_t nd, int32_t* keep, int32_t* od_new, uint8_t* rowflag,
                               int app, const uint32_t* x, int32_t source, int32_t* taint, int32_t* list,
                               int32_t* count) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nd; j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = dkeys[j];
    if (j > 0 && dkeys[j - 1] == key) continue;
    const int32_t d = (int32_t)(key >> 32);
    const int32_t s = (int32_t)(uint32_t)key;
    int lo = rowptr[d], hi = rowptr[d + 1];  // first edge of the row with source >= s
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (col[mid] < s) lo = mid + 1;
      else hi = mid;
    }
    int cnt = 0;
    bool seed = false;
    for (int e = lo; e < rowptr[d + 1] && col[e] == s; ++e) {
      keep[e] = 0;
      ++cnt;
      if (x && supports(app, x, source, s, d, weight ? (uint32_t)weight[e] : 0u)) seed = true;
    }
    if (cnt) {
      atomicSub(&od_new[s], cnt);
      rowflag[d] = 1;  // every writer stores the same byte
    }
    if (seed && atomicExch(&taint[d], 1) == 0) list[atomicAdd(count, 1)] = d;
  }
}

// Out-degree and per-source insertion count of the inserted arcs.
__global__ void k_ins_outdeg(const uint64_t* ikeys, int64_t ni, int32_t* od_new, int32_t* ins_cnt) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ni; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = (int32_t)(uint32_t)ikeys[j];
    atomicAdd(&od_new[s], 1);
    if (ins_cnt) atomicAdd(&ins_cnt[s], 1);
  }
}

// ins_rp[u] = first sorted insertion whose destination is >= u, for u in [0, n].
__global__ void k_ins_rows(const uint64_t* ikeys, int64_t ni, int32_t n, int32_t* ins_rp) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u <= n; u += (int64_t)gridDim.x * blockDim.x)
    ins_rp[u] = (int32_t)lower_bound_u64(ikeys, 0, ni, (uint64_t)u << 32);
}

__global__ void k_new_len(const int32_t* rowptr, const int32_t* keep_ex, const int32_t* ins_rp, int32_t n,
                          int32_t* len, uint8_t* rowflag) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t ins = ins_rp[u + 1] - ins_rp[u];
    len[u] = (keep_ex[rowptr[u + 1]] - keep_ex[rowptr[u]]) + ins;
    if (ins > 0) rowflag[u] |= 2;
  }
}

// A surviving old edge goes after the survivors before it in its row and
// after the row's insertions with a smaller source. new_of_old[e] receives
// its new position (-1 when deleted).
__global__ void k_scatter_old(const int32_t* rowptr, const int32_t* row_of_edge, const int32_t* col,
                              const int32_t* weight, int64_t m, const int32_t* keep, const int32_t* keep_ex,
                              const uint64_t* ikeys, const int32_t* ins_rp, const int32_t* new_rp, int32_t* ncol,
                              int32_t* nweight, int32_t* old_of_new, int32_t* new_of_old) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    if (!keep[e]) {
      new_of_old[e] = -1;
      continue;
    }
    const int u = row_of_edge[e];
    const int32_t s = col[e];
    const int64_t rank = keep_ex[e] - keep_ex[rowptr[u]];
    const int32_t i0 = ins_rp[u], i1 = ins_rp[u + 1];
    const int64_t before = i0 == i1 ? 0 : lower_bound_u64(ikeys, i0, i1, arc_key(s, u)) - i0;
    const int64_t pos = new_rp[u] + rank + before;
    ncol[pos] = s;
    if (nweight) nweight[pos] = weight[e];
    old_of_new[pos] = (int32_t)e;
    new_of_old[e] = (int32_t)pos;
  }
}

// An inserted arc goes after the row's earlier insertions and after every
// surviving old edge whose source is not larger.
__global__ void k_scatter_ins(const int32_t* rowptr, const int32_t* col, const int32_t* keep_ex, const uint64_t* ikeys,
                              const int32_t* iidx, int64_t ni, const int32_t* ins_rp, const int32_t* ins_w,
                              const int32_t* new_rp, int32_t* ncol, int32_t* nweight, int32_t* old_of_new,
                              const int32_t* orow_new, const int32_t* ins_cnt, int32_t* icur, int32_t* noedge,
                              int32_t* nodst, int32_t* nosrc) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ni; j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = ikeys[j];
    const int u = (int)(key >> 32);
    const int32_t s = (int32_t)(uint32_t)key;
    int lo = rowptr[u], hi = rowptr[u + 1];  // first old edge of the row with a larger source
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (col[mid] <= s) lo = mid + 1;
      else hi = mid;
    }
    const int64_t kept = keep_ex[lo] - keep_ex[rowptr[u]];
    const int64_t pos = new_rp[u] + (j - ins_rp[u]) + kept;
    ncol[pos] = s;
    if (nweight) nweight[pos] = ins_w[iidx[j]];
    old_of_new[pos] = -1;
    if (noedge) {
      // the inserted arcs of a source follow its surviving out-arcs
      const int32_t q = orow_new[s + 1] - ins_cnt[s] + atomicAdd(&icur[s], 1);
      noedge[q] = (int32_t)pos;
      nodst[q] = u;
      nosrc[q] = s;
    }
  }
}

// Per row: how its old edges move. A row that neither lost nor gained edges
// moves as a whole (new row start minus old); the others are marked
// kMoveByMap and look every edge up in new_of_old.
constexpr int32_t kMoveByMap = INT32_MIN;

__global__ void k_row_move(const int32_t* rp_old, const int32_t* rp_new, const uint8_t* rowflag, int32_t n,
                           int32_t* move) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
    move[u] = rowflag[u] ? kMoveByMap : rp_new[u] - rp_old[u];
}

// Out-CSR after an update: the new in-edge id of out-entry k (in-edge
// oedge[k] of row odst[k]), -1 when deleted, in ne[k], and kout[k] = 1 for
// a survivor. The out-CSR is read in order; the one gather per entry is
// the destination row's move (n entries).
__global__ void k_out_keep(const int32_t* oedge, const int32_t* odst, int64_t m, const int32_t* move,
                           const int32_t* new_of_old, int32_t* ne, int32_t* kout) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = oedge[k];
    const int32_t mv = move[odst[k]];
    const int32_t x = mv == kMoveByMap ? new_of_old[e] : e + mv;
    ne[k] = x;
    kout[k] = x >= 0 ? 1 : 0;
  }
}

// Per source: the new position of its first survivor minus the survivors
// before it.
__global__ void k_out_base(const int32_t* orow_old, const int32_t* orow_new, const int32_t* kout_ex, int32_t n,
                           int32_t* obase) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    obase[v] = orow_new[v] - kout_ex[orow_old[v]];
}

// A surviving out-entry keeps its rank among its source's survivors, now
// pointing at the edge's new position (ne). Streams the out-CSR in order.
__global__ void k_out_compact(const int32_t* ne, const int32_t* odst, const int32_t* osrc, int64_t m,
                              const int32_t* kout, const int32_t* kout_ex, const int32_t* obase, int32_t* noedge,
                              int32_t* nodst, int32_t* nosrc) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    if (!kout[k]) continue;
    const int32_t v = osrc[k];
    const int64_t q = (int64_t)kout_ex[k] + obase[v];
    noedge[q] = ne[k];
    nodst[q] = odst[k];
    nosrc[q] = v;
  }
}

// One new flag word per thread: a continued edge keeps its old flag, an
// inserted one is set.
__global__ void k_remap_bits(const uint32_t* old_bits, const int32_t* old_of_new, int64_t m, uint32_t* new_bits) {
  const int64_t nw = (m + 31) / 32;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw; w += (int64_t)gridDim.x * blockDim.x) {
    uint32_t word = 0;
    const int64_t e0 = w * 32;
    const int cnt = (int)min((int64_t)32, m - e0);
    for (int b = 0; b < cnt; ++b) {
      const int32_t o = old_of_new[e0 + b];
      const uint32_t bit = o < 0 ? 1u : (old_bits[o >> 5] >> (o & 31)) & 1u;
      word |= bit << b;
    }
    new_bits[w] = word;
  }
}

// c = x / outdeg under the new out-degrees, from c = x / outdeg_old (x
// itself for vertices without out-edges).
__global__ void k_rescale_contrib(float* c, const int32_t* od_old, const int32_t* od_new, int32_t n) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int a = od_old[u], b = od_new[u];
    if (a == b) continue;
    const double x = a > 0 ? (double)c[u] * (double)a : (double)c[u];
    c[u] = b > 0 ? (float)(x / (double)b) : (float)x;
  }
}

// Work list of row chunks: for each vertex of list[lo, hi), one entry
// (vertex, chunk) per kTaintChunk edges of its row in offsets (none for an
// empty row), appended at wcount. A wavefront takes one entry, so a hub row
// is spread over many wavefronts.
__device__ __forceinline__ void append_chunks(int32_t v, const int32_t* offsets, int32_t* wv, int32_t* wc,
                                              int32_t* wcount) {
  const int32_t nch = (offsets[v + 1] - offsets[v] + kTaintChunk - 1) / kTaintChunk;
  if (nch == 0) return;
  const int32_t base = atomicAdd(wcount, nch);
  for (int32_t c = 0; c < nch; ++c) {
    wv[base + c] = v;
    wc[base + c] = c;
  }
}

__global__ void k_row_chunks(const int32_t* list, int32_t count, const int32_t* offsets, int32_t* wv, int32_t* wc,
                             int32_t* wcount) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    append_chunks(list[i], offsets, wv, wc, wcount);
}

// One wavefront per work entry (p, chunk) of [lo, hi): every out-edge
// p -> v of the chunk that supports v taints v, which is appended once to
// tlist (tcount) and its out-row's chunks to the work list. The test is that
// of supports(), with the SSSP weight read only when x_v - x_p can be a
// weight.
__global__ __launch_bounds__(kUpdBlock) void k_taint_push(int32_t* wv, int32_t* wc, int32_t lo, int32_t hi,
                                                          const int32_t* orow, const int32_t* oedge,
                                                          const int32_t* odst, const int32_t* weight, int app,
                                                          const uint32_t* x, int32_t source, int32_t* taint,
                                                          int32_t* tlist, int32_t* counts) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = lo + wave; i < hi; i += nwaves) {
    const int32_t p = wv[i];
    const uint32_t xs = x[p];
    const int32_t k0 = orow[p] + wc[i] * kTaintChunk;
    const int32_t k1 = min(orow[p + 1], k0 + kTaintChunk);
    for (int32_t k = k0 + lane; k < k1; k += 64) {
      const int32_t v = odst[k];
      const int32_t tv = taint[v];
      const uint32_t xd = x[v];  // loaded with taint[v], before the test
      if (tv != 0) continue;
      bool sup;
      if (app == kSSSP) {
        sup = v != source && xs != kInf && xd != kInf && xd >= xs && xd - xs <= 255u &&
              (uint32_t)weight[oedge[k]] == xd - xs;
      } else {
        sup = xs == xd && xd != (uint32_t)v;
      }
      if (sup && atomicExch(&taint[v], 1) == 0) {
        tlist[atomicAdd(&counts[0], 1)] = v;
        append_chunks(v, orow, wv, wc, &counts[1]);
      }
    }
  }
}

__global__ void k_taint_reset(const int32_t* list, int32_t count, int app, int32_t source, uint32_t* x0,
                              uint32_t* x1) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = list[i];
    const uint32_t init = app == kSSSP ? (v == source ? 0u : kInf) : (uint32_t)v;
    x0[v] = init;
    x1[v] = init;
  }
}

// chg[src] = 1 for every in-edge src -> v of the work entries (v, chunk)
// (one wavefront per entry).
__global__ __launch_bounds__(kUpdBlock) void k_mark_in_neighbors(const int32_t* wv, const int32_t* wc, int32_t count,
                                                                 const int32_t* rowptr, const int32_t* col,
                                                                 uint8_t* chg) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < count; i += nwaves) {
    const int32_t v = wv[i];
    const int32_t e0 = rowptr[v] + wc[i] * kTaintChunk;
    const int32_t e1 = min(rowptr[v + 1], e0 + kTaintChunk);
    for (int32_t e = e0 + lane; e < e1; e += 64) chg[col[e]] = 1;
  }
}

__global__ void k_mark_sources(const uint64_t* ikeys, int64_t ni, uint8_t* chg) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ni; j += (int64_t)gridDim.x * blockDim.x)
    chg[(int32_t)(uint32_t)ikeys[j]] = 1;
}

}  // namespace

hipError_t launch_batch_check(const int32_t* src, const int32_t* dst, const int32_t* w, int64_t k, int32_t n,
                              int32_t* flags, hipStream_t st) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_check, dim3(grid_of(k)), dim3(kUpdBlock), 0, st, src, dst, w, k, n, flags);
  return hipGetLastError();
}

hipError_t launch_arc_keys(const int32_t* src, const int32_t* dst, int64_t k, uint64_t* keys, int32_t* idx,
                           hipStream_t st) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(k_arc_keys, dim3(grid_of(k)), dim3(kUpdBlock), 0, st, src, dst, k, keys, idx);
  return hipGetLastError();
}

hipError_t sort_keys_bytes(int64_t k, size_t* bytes) {
  *bytes = 0;
  return hipcub::DeviceRadixSort::SortKeys(nullptr, *bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr, (int)k);
}

hipError_t sort_pairs_bytes(int64_t k, size_t* bytes) {
  *bytes = 0;
  return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                            (const int32_t*)nullptr, (int32_t*)nullptr, (int)k);
}

hipError_t launch_sort_keys(const uint64_t* in, uint64_t* out, int64_t k, void* temp, size_t bytes, hipStream_t st) {
  if (k == 0) return hipSuccess;
  return hipcub::DeviceRadixSort::SortKeys(temp, bytes, in, out, (int)k, 0, 64, st);
}

hipError_t launch_sort_pairs(const uint64_t* kin, uint64_t* kout, const int32_t* vin, int32_t* vout, int64_t k,
                             void* temp, size_t bytes, hipStream_t st) {
  if (k == 0) return hipSuccess;
  return hipcub::DeviceRadixSort::SortPairs(temp, bytes, kin, kout, vin, vout, (int)k, 0, 64, st);
}

hipError_t launch_row_ids(const int32_t* rowptr, int32_t n, int32_t* dst, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_ids, dim3(grid_of(n)), dim3(kUpdBlock), 0, st, rowptr, n, dst);
  return hipGetLastError();
}

hipError_t launch_mark_deleted(const int32_t* rowptr, const int32_t* col, const int32_t* weight,
                               const uint64_t* dkeys, int64_t nd, int32_t* keep, int32_t* od_new, uint8_t* rowflag,
                               int app, const uint32_t* x, int32_t source, int32_t* taint, int32_t* list,
                               int32_t* count, hipStream_t st) {
  if (nd == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_deleted, dim3(grid_of(nd)), dim3(kUpdBlock), 0, st, rowptr, col, weight, dkeys, nd, keep,
                     od_new, rowflag, app, x, source, taint, list, count);
  return hipGetLastError();
}

hipError_t launch_ins_outdeg(const uint64_t* ikeys, int64_t ni, int32_t* od_new, int32_t* ins_cnt, hipStream_t st) {
  if (ni == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ins_outdeg, dim3(grid_of(ni)), dim3(kUpdBlock), 0, st, ikeys, ni, od_new, ins_cnt);
  return hipGetLastError();
}

hipError_t launch_ins_rows(const uint64_t* ikeys, int64_t ni, int32_t n, int32_t* ins_rp, hipStream_t st) {
  hipLaunchKernelGGL(k_ins_rows, dim3(grid_of((int64_t)n + 1)), dim3(kUpdBlock), 0, st, ikeys, ni, n, ins_rp);
  return hipGetLastError();
}

hipError_t launch_new_len(const int32_t* rowptr, const int32_t* keep_ex, const int32_t* ins_rp, int32_t n,
                          int32_t* len, uint8_t* rowflag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_new_len, dim3(grid_of(n)), dim3(kUpdBlock), 0, st, rowptr, keep_ex, ins_rp, n, len, rowflag);
  return hipGetLastError();
}

hipError_t launch_scatter_old(const int32_t* rowptr, const int32_t* row_of_edge, const int32_t* col,
                              const int32_t* weight, int64_t m, const int32_t* keep, const int32_t* keep_ex,
                              const uint64_t* ikeys, const int32_t* ins_rp, const int32_t* new_rp, int32_t* ncol,
                              int32_t* nweight, int32_t* old_of_new, int32_t* new_of_old, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_old, dim3(grid_of(m)), dim3(kUpdBlock), 0, st, rowptr, row_of_edge, col, weight, m,
                     keep, keep_ex, ikeys, ins_rp, new_rp, ncol, nweight, old_of_new, new_of_old);
  return hipGetLastError();
}

hipError_t launch_scatter_ins(const int32_t* rowptr, const int32_t* col, const int32_t* keep_ex,
                              const uint64_t* ikeys, const int32_t* iidx, int64_t ni, const int32_t* ins_rp,
                              const int32_t* ins_w, const int32_t* new_rp, int32_t* ncol, int32_t* nweight,
                              int32_t* old_of_new, const int32_t* orow_new, const int32_t* ins_cnt, int32_t* icur,
                              int32_t* noedge, int32_t* nodst, int32_t* nosrc, hipStream_t st) {
  if (ni == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_ins, dim3(grid_of(ni)), dim3(kUpdBlock), 0, st, rowptr, col, keep_ex, ikeys, iidx, ni,
                     ins_rp, ins_w, new_rp, ncol, nweight, old_of_new, orow_new, ins_cnt, icur, noedge, nodst, nosrc);
  return hipGetLastError();
}

hipError_t launch_row_move(const int32_t* rp_old, const int32_t* rp_new, const uint8_t* rowflag, int32_t n,
                           int32_t* move, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_move, dim3(grid_of(n)), dim3(kUpdBlock), 0, st, rp_old, rp_new, rowflag, n, move);
  return hipGetLastError();
}

hipError_t launch_out_keep(const int32_t* oedge, const int32_t* odst, int64_t m, const int32_t* move,
                           const int32_t* new_of_old, int32_t* ne, int32_t* kout, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_out_keep, dim3(grid_of(m)), dim3(kUpdBlock), 0, st, oedge, odst, m, move, new_of_old, ne,
                     kout);
  return hipGetLastError();
}

hipError_t launch_out_base(const int32_t* orow_old, const int32_t* orow_new, const int32_t* kout_ex, int32_t n,
                           int32_t* obase, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_out_base, dim3(grid_of(n)), dim3(kUpdBlock), 0, st, orow_old, orow_new, kout_ex, n, obase);
  return hipGetLastError();
}

hipError_t launch_out_compact(const int32_t* ne, const int32_t* odst, const int32_t* osrc, int64_t m,
                              const int32_t* kout, const int32_t* kout_ex, const int32_t* obase, int32_t* noedge,
                              int32_t* nodst, int32_t* nosrc, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_out_compact, dim3(grid_of(m)), dim3(kUpdBlock), 0, st, ne, odst, osrc, m, kout, kout_ex, obase,
                     noedge, nodst, nosrc);
  return hipGetLastError();
}

hipError_t launch_remap_bits(const uint32_t* old_bits, const int32_t* old_of_new, int64_t m, uint32_t* new_bits,
                             hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_remap_bits, dim3(grid_of((m + 31) / 32)), dim3(kUpdBlock), 0, st, old_bits, old_of_new, m,
                     new_bits);
  return hipGetLastError();
}

hipError_t launch_rescale_contrib(float* c, const int32_t* od_old, const int32_t* od_new, int32_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rescale_contrib, dim3(grid_of(n)), dim3(kUpdBlock), 0, st, c, od_old, od_new, n);
  return hipGetLastError();
}

hipError_t launch_row_chunks(const int32_t* list, int32_t count, const int32_t* offsets, int32_t* wv, int32_t* wc,
                             int32_t* wcount, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_chunks, dim3(grid_of(count)), dim3(kUpdBlock), 0, st, list, count, offsets, wv, wc, wcount);
  return hipGetLastError();
}

hipError_t launch_taint_push(int32_t* wv, int32_t* wc, int32_t lo, int32_t hi, const int32_t* orow,
                             const int32_t* oedge, const int32_t* odst, const int32_t* weight, int app,
                             const uint32_t* x, int32_t source, int32_t* taint, int32_t* tlist, int32_t* counts,
                             hipStream_t st) {
  if (hi <= lo) return hipSuccess;
  const dim3 grid(grid_of((int64_t)(hi - lo) * 64));
  hipLaunchKernelGGL(k_taint_push, grid, dim3(kUpdBlock), 0, st, wv, wc, lo, hi, orow, oedge, odst, weight, app, x,
                     source, taint, tlist, counts);
  return hipGetLastError();
}

hipError_t launch_taint_reset(const int32_t* list, int32_t count, int app, int32_t source, uint32_t* x0,
                              uint32_t* x1, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_taint_reset, dim3(grid_of(count)), dim3(kUpdBlock), 0, st, list, count, app, source, x0, x1);
  return hipGetLastError();
}

hipError_t launch_mark_in_neighbors(const int32_t* wv, const int32_t* wc, int32_t count, const int32_t* rowptr,
                                    const int32_t* col, uint8_t* chg, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_in_neighbors, dim3(grid_of((int64_t)count * 64)), dim3(kUpdBlock), 0, st, wv, wc, count,
                     rowptr, col, chg);
  return hipGetLastError();
}

hipError_t launch_mark_sources(const uint64_t* ikeys, int64_t ni, uint8_t* chg, hipStream_t st) {
  if (ni == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_sources, dim3(grid_of(ni)), dim3(kUpdBlock), 0, st, ikeys, ni, chg);
  return hipGetLastError();
}

}  // namespace ggk

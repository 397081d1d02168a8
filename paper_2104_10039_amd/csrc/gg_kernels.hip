// Device kernels of the GraphGuess sweep for CDNA4 (gfx950, wave64).
//
// The sweep is the pull-based vertex program of the paper [Sec. 3.1, Alg. 2]:
// for every destination row, gather over its in-edges (all of them in
// accurate mode, only the active ones in approximate mode [Sec. 3.3]), then
// apply. A superstep is an accurate iteration that also computes each edge's
// influence and re-selects the active edges against theta [Sec. 3.4].
//
// Work distribution is degree-binned: rows with few edges are handled by
// teams of 4..32 lanes, medium rows by one wavefront, long rows by 256-thread
// workgroups over fixed-size edge chunks whose partial results are combined
// in a fixed order. Every reduction has a fixed shape, so results are
// bitwise reproducible for a fixed tuning.
//
// The active edges of a row are kept packed at the front of the row's own
// slot [rowptr[u], rowptr[u+1]) of a second edge array, with a per-row count;
// the approximate gather streams only that prefix. A bitmap holds the flag of
// every edge (bit e mod 32 of word e/32).
#include "gg_internal.h"

namespace ggk {

// ---------------------------------------------------------------------------
// Wavefront / team primitives
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t ld_stream(const uint32_t* p) { return __builtin_nontemporal_load(p); }

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T x, int m, int w) {
  return __shfl_xor(x, m, w);
}

template <int TEAM>
__device__ __forceinline__ double team_sum(double x) {
#pragma unroll
  for (int o = TEAM / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, TEAM);
  return x;
}

template <int TEAM>
__device__ __forceinline__ uint32_t team_min(uint32_t x) {
#pragma unroll
  for (int o = TEAM / 2; o > 0; o >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, o, TEAM));
  return x;
}

// Inclusive scans inside a team of TEAM lanes (lt = lane index in the team).
template <int TEAM>
__device__ __forceinline__ double team_scan_add(double x, int lt) {
#pragma unroll
  for (int d = 1; d < TEAM; d <<= 1) {
    double y = __shfl_up(x, d, TEAM);
    if (lt >= d) x += y;
  }
  return x;
}

template <int TEAM>
__device__ __forceinline__ uint32_t team_scan_min(uint32_t x, int lt) {
#pragma unroll
  for (int d = 1; d < TEAM; d <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int)x, d, TEAM);
    if (lt >= d) x = min(x, y);
  }
  return x;
}

// Apps whose gather is a sum of binary32 per-vertex contributions (PR, PPR:
// rank over out-degree; BP: message log-ratio).
template <int APP>
constexpr bool kSumApp = APP == kPR || APP == kPPR || APP == kBP;

// Per-app gather element, identity and combine.
template <int APP>
struct Tr;

template <>
struct Tr<kPR> {
  using T = double;
  static __device__ __forceinline__ T id() { return 0.0; }
  static __device__ __forceinline__ T op(T a, T b) { return a + b; }
  static __device__ __forceinline__ T elem(const Sweep& s, uint32_t e) { return (double)s.c_in[e]; }
};
template <>
struct Tr<kPPR> : Tr<kPR> {};
template <>
struct Tr<kBP> : Tr<kPR> {};
template <>
struct Tr<kSSSP> {
  using T = uint32_t;
  static __device__ __forceinline__ T id() { return kInf; }
  static __device__ __forceinline__ T op(T a, T b) { return min(a, b); }
  // packed edge: source in the low 24 bits, weight in the high 8 bits
  static __device__ __forceinline__ T elem(const Sweep& s, uint32_t e) {
    uint32_t xv = s.x_in[e & 0xFFFFFFu];
    return xv == kInf ? kInf : xv + (e >> 24);
  }
};
template <>
struct Tr<kCC> {
  using T = uint32_t;
  static __device__ __forceinline__ T id() { return kInf; }
  static __device__ __forceinline__ T op(T a, T b) { return min(a, b); }
  static __device__ __forceinline__ T elem(const Sweep& s, uint32_t e) { return s.x_in[e]; }
};

template <int TEAM>
__device__ __forceinline__ double team_reduce(double x) { return team_sum<TEAM>(x); }
template <int TEAM>
__device__ __forceinline__ uint32_t team_reduce(uint32_t x) { return team_min<TEAM>(x); }

// Block (256 threads = 4 waves) reductions in a fixed order; result valid in
// every thread. lds must hold 4 elements.
template <int APP>
__device__ __forceinline__ typename Tr<APP>::T block_reduce(typename Tr<APP>::T x, typename Tr<APP>::T* lds) {
  using T = typename Tr<APP>::T;
  x = team_reduce<64>(x);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[wid] = x;
  __syncthreads();
  T r = Tr<APP>::op(Tr<APP>::op(lds[0], lds[1]), Tr<APP>::op(lds[2], lds[3]));
  __syncthreads();
  return r;
}

__device__ __forceinline__ int block_sum_int(int x, int* lds) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[wid] = x;
  __syncthreads();
  int r = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return r;
}

// Exclusive rank of this thread among the block's threads with pred set.
__device__ __forceinline__ int block_rank(bool pred, int* lds, int& total) {
  const uint64_t bal = __ballot(pred);
  const int lane = __lane_id();
  const int wid = threadIdx.x >> 6;
  const int r = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) lds[wid] = __popcll(bal);
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int c = lds[w];
    off += (w < wid) ? c : 0;
    tot += c;
  }
  __syncthreads();
  total = tot;
  return off + r;
}

__device__ __forceinline__ int row_len(const Sweep& s, int u, int b) {
  return s.cnt ? s.cnt[u] : s.rowptr[u + 1] - b;
}

// Index of the hub row that owns chunk ch: the last h with hub_start[h] <= ch.
__device__ __forceinline__ int find_hub(const int32_t* hub_start, int n_hub, int ch) {
  int lo = 0, hi = n_hub - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (hub_start[mid] <= ch) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Apply [Alg. 2, GG-Apply]
// ---------------------------------------------------------------------------

// The per-row word the apply reads (PR/PPR: out-degree; SSSP/CC: the old
// value), so that callers can issue its load before their gather.
template <int APP>
__device__ __forceinline__ uint32_t apply_word(const Sweep& s, int u) {
  if constexpr (APP == kPR || APP == kPPR) return (uint32_t)s.outdeg[u];
  else if constexpr (APP == kBP) return __float_as_uint(s.bp_prior[u]);
  else return s.x_in[u];
}

// BP message log-ratio of a vertex with belief log-odds L under the coupling
// kappa: log(m(1) / m(0)) = 2 atanh(kappa tanh(L / 2)) (the sum over the
// sender's states of the potential times its belief, in closed form).
__device__ __forceinline__ double bp_message(double L, double kappa) {
  return 2.0 * atanh(kappa * tanh(0.5 * L));
}

template <int APP>
__device__ __forceinline__ void apply_with(const Sweep& s, int u, typename Tr<APP>::T acc, uint32_t word,
                                           int& nchanged) {
  if constexpr (APP == kPR || APP == kPPR) {
    const double D = *s.dangling;
    double x;
    if constexpr (APP == kPR) {
      if (s.part_of) {
        // a part of a block-diagonal union: its own vertex count and dangling mass
        const int p = s.part_of[u];
        const double np = (double)(s.part_start[p + 1] - s.part_start[p]);
        x = (1.0 - s.damping) / np + s.damping * (acc + s.part_dang[p] / np);
      } else {
        x = s.base + s.damping * (acc + D / (double)s.n);
      }
    } else {
      const bool src = (u == s.source);
      x = (src ? (1.0 - s.damping) : 0.0) + s.damping * (acc + (src ? D : 0.0));
    }
    const int od = (int)word;
    s.c_out[u] = od > 0 ? (float)(x / (double)od) : (float)x;
    if (s.x_out) s.x_out[u] = (float)x;
    if (s.sum_out) s.sum_out[u] = acc;
    if (s.vact) {
      // GG-VStatus [Alg. 2]: active iff the value moved by more than eps
      const double xo = (double)s.x_prev[u];
      const double bound = s.vs_rel ? s.vs_eps * fabs(xo) : s.vs_eps;
      s.vact[u] = (uint8_t)(fabs(x - xo) > bound);
      s.x_prev[u] = (float)x;
    }
  } else if constexpr (APP == kBP) {
    // belief log-odds: prior plus the gathered messages; the new message is
    // what the next iteration gathers
    const double L = (double)__uint_as_float(word) + acc;
    s.c_out[u] = (float)bp_message(L, s.bp_kappa);
    if (s.x_out) s.x_out[u] = (float)L;
  } else {
    const uint32_t old = word;
    const uint32_t nv = min(old, acc);
    s.x_next[u] = nv;
    nchanged += (nv != old);
    if (s.chg) s.chg[u] = (uint8_t)(nv != old);
  }
}

template <int APP>
__device__ __forceinline__ void apply(const Sweep& s, int u, typename Tr<APP>::T acc, int& nchanged) {
  apply_with<APP>(s, u, acc, apply_word<APP>(s, u), nchanged);
}

// ---------------------------------------------------------------------------
// Plain gather-apply (exact and approximate iterations)
// ---------------------------------------------------------------------------

template <int APP, int TEAM>
__device__ __forceinline__ void gather_team_rows(const Sweep& s, const int32_t* list, int count, int blk, int nblk,
                                                 int& nchanged) {
  using R = Tr<APP>;
  using T = typename R::T;
  const int lt = threadIdx.x & (TEAM - 1);
  constexpr int TPB = kBlock / TEAM;
  const int stride = nblk * TPB;
  for (int t = blk * TPB + (int)threadIdx.x / TEAM; t < count; t += stride) {
    const int u = list[t];
    if (s.skip && s.skip[u]) continue;  // the whole team skips the row
    const int b = s.rowptr[u];
    const int len = row_len(s, u, b);
    const uint32_t* ed = s.edges + b;
    T acc = R::id();
    int k = lt;
    for (; k + 3 * TEAM < len; k += 4 * TEAM) {
      const uint32_t e0 = ld_stream(ed + k), e1 = ld_stream(ed + k + TEAM);
      const uint32_t e2 = ld_stream(ed + k + 2 * TEAM), e3 = ld_stream(ed + k + 3 * TEAM);
      const T v0 = R::elem(s, e0), v1 = R::elem(s, e1), v2 = R::elem(s, e2), v3 = R::elem(s, e3);
      acc = R::op(acc, R::op(R::op(v0, v1), R::op(v2, v3)));
    }
    for (; k < len; k += TEAM) acc = R::op(acc, R::elem(s, ld_stream(ed + k)));
    acc = team_reduce<TEAM>(acc);
    if (lt == 0) apply<APP>(s, u, acc, nchanged);
  }
}

// One 256-thread block reduces one chunk of a hub row. Rows with a single
// chunk are applied directly; otherwise the partial goes to part[ch].
template <int APP>
__device__ __forceinline__ void gather_hub_chunk(const Sweep& s, int ch, bool always_partial, int& nchanged,
                                                 typename Tr<APP>::T* lds) {
  using R = Tr<APP>;
  using T = typename R::T;
  const int h = find_hub(s.hub_start, s.n_hub, ch);
  const int u = s.list[s.n_small + s.n_wave + h];
  if (s.skip && s.skip[u]) return;  // uniform over the block
  const int j = ch - s.hub_start[h];
  const int nch = s.hub_start[h + 1] - s.hub_start[h];
  const int b = s.rowptr[u];
  const int len = row_len(s, u, b);
  const int e0 = j * s.hub_chunk;
  const int e1 = min(len, e0 + s.hub_chunk);
  const uint32_t* ed = s.edges + b;
  T acc = R::id();
  int k = e0 + (int)threadIdx.x;
  for (; k + 3 * kBlock < e1; k += 4 * kBlock) {
    const uint32_t a0 = ld_stream(ed + k), a1 = ld_stream(ed + k + kBlock);
    const uint32_t a2 = ld_stream(ed + k + 2 * kBlock), a3 = ld_stream(ed + k + 3 * kBlock);
    const T v0 = R::elem(s, a0), v1 = R::elem(s, a1), v2 = R::elem(s, a2), v3 = R::elem(s, a3);
    acc = R::op(acc, R::op(R::op(v0, v1), R::op(v2, v3)));
  }
  for (; k < e1; k += kBlock) acc = R::op(acc, R::elem(s, ld_stream(ed + k)));
  acc = block_reduce<APP>(acc, lds);
  if (threadIdx.x == 0) {
    if (nch == 1 && !always_partial) {
      apply<APP>(s, u, acc, nchanged);
    } else {
      if constexpr (kSumApp<APP>) s.part_f[ch] = acc;
      else s.part_u[ch] = acc;
    }
  }
}

template <int APP>
__device__ __forceinline__ void flush_changed(const Sweep& s, int nchanged, int* ilds) {
  if constexpr (APP == kSSSP || APP == kCC) {
    if (!s.changed) return;  // counted elsewhere (the frontier's changed list)
    const int tot = block_sum_int(nchanged, ilds);
    if (threadIdx.x == 0 && tot) atomicAdd(s.changed, tot);
  }
}

// Blocks [0, gs): small rows; [gs, gs+gw): wavefront rows; the rest: one hub
// chunk each.
template <int APP, int TEAM>
__global__ __launch_bounds__(kBlock) void k_gather(Sweep s, int gs, int gw) {
  __shared__ typename Tr<APP>::T lds[4];
  __shared__ int ilds[4];
  int nchanged = 0;
  const int bid = blockIdx.x;
  if (bid < gs) {
    gather_team_rows<APP, TEAM>(s, s.list, s.n_small, bid, gs, nchanged);
  } else if (bid < gs + gw) {
    gather_team_rows<APP, 64>(s, s.list + s.n_small, s.n_wave, bid - gs, gw, nchanged);
  } else {
    gather_hub_chunk<APP>(s, bid - gs - gw, false, nchanged, lds);
  }
  flush_changed<APP>(s, nchanged, ilds);
}

// Combine the chunk partials of multi-chunk hub rows in chunk order.
template <int APP>
__global__ __launch_bounds__(kBlock) void k_hub_combine(Sweep s) {
  using R = Tr<APP>;
  __shared__ int ilds[4];
  int nchanged = 0;
  const int h = blockIdx.x * kBlock + threadIdx.x;
  if (h < s.n_hub) {
    const int c0 = s.hub_start[h], nch = s.hub_start[h + 1] - c0;
    const int u = s.list[s.n_small + s.n_wave + h];
    if (nch > 1 && !(s.skip && s.skip[u])) {
      typename R::T acc = R::id();
      for (int j = 0; j < nch; ++j) {
        if constexpr (kSumApp<APP>) acc = R::op(acc, s.part_f[c0 + j]);
        else acc = R::op(acc, s.part_u[c0 + j]);
      }
      apply<APP>(s, u, acc, nchanged);
    }
  }
  flush_changed<APP>(s, nchanged, ilds);
}

// ---------------------------------------------------------------------------
// Superstep: accurate gather-apply + influence + GG-EStatus + repack
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t edge_bit(const uint32_t* bits, int e) { return (bits[e >> 5] >> (e & 31)) & 1u; }

// Flag of one edge given the running value of its row. PR/PPR: influence =
// c / P with P the inclusive running sum; BP: |c| / |P|. SSSP: relative
// improvement of the running minimum; unreached sources keep their flag.
// CC: the source label lowers the running minimum.

// c / P > theta for c, P >= 0, identical to comparing the rounded quotient:
// away from the threshold (relative margin 1e-12, far above the rounding of
// theta * P) a product decides; only near-ties evaluate the division.
__device__ __forceinline__ bool infl_above(double c, double P, double theta) {
  if (!(P > 0.0)) return false;
  const double tp = theta * P;
  if (c > tp * (1.0 + 1e-12)) return true;
  if (c < tp * (1.0 - 1e-12)) return false;
  return c / P > theta;
}

// Sum-type apps: influence c / P (BP on magnitudes, its messages having
// both signs).
template <int APP>
__device__ __forceinline__ bool sum_flag(const Sweep& s, bool valid, double c, double P, uint32_t oldf) {
  if constexpr (APP == kBP) {
    c = fabs(c);
    P = fabs(P);
  }
  return (valid && infl_above(c, P, s.theta)) || (s.mask_union && oldf);
}

// Start of a superstep row's running value: the gather identity, or for
// SSSP/CC in push order the row's own value.
template <int APP>
__device__ __forceinline__ typename Tr<APP>::T run_init(const Sweep& s, int u) {
  if constexpr (kSumApp<APP>) return Tr<APP>::id();
  else return s.push_infl ? s.x_in[u] : Tr<APP>::id();
}

// Set the new flag bits of TEAM consecutive edges (edge e at team lane lt).
template <int TEAM>
__device__ __forceinline__ void write_bits(uint32_t* bits, uint64_t tm, int lt, int e, int remaining, bool valid) {
  if (valid && (lt == 0 || (e & 31) == 0)) {
    const int off = e & 31;
    const int nb = min(32 - off, min(TEAM - lt, remaining));
    const uint64_t sel = (tm >> lt) & ((1ull << nb) - 1ull);
    const uint32_t word = (uint32_t)(sel << off);
    if (word) atomicOr(&bits[e >> 5], word);
  }
}

template <int APP, int TEAM>
__device__ __forceinline__ void super_team_rows(const Sweep& s, const int32_t* list, int count, int blk, int nblk,
                                                int& nchanged) {
  using R = Tr<APP>;
  using T = typename R::T;
  const int lt = threadIdx.x & (TEAM - 1);
  const int lane = __lane_id();
  const int team_base = lane & ~(TEAM - 1);
  constexpr int TPB = kBlock / TEAM;
  const int stride = nblk * TPB;
  for (int t = blk * TPB + (int)threadIdx.x / TEAM; t < count; t += stride) {
    const int u = list[t];
    const int b = s.rowptr[u];
    const int len = s.rowptr[u + 1] - b;
    // TOTAL influence compares with the row sum, PREFIX with the running sum
    const double rtot = (kSumApp<APP> && s.row_total) ? s.row_total[u] : -1.0;
    T carry = run_init<APP>(s, u);
    int carry_cnt = 0;
    // edge words and values of kPreT consecutive team-wide steps are loaded
    // before the first step's scan
    constexpr int kPreT = 4;
    for (int g0 = 0; g0 < len; g0 += kPreT * TEAM) {
    uint32_t evq[kPreT];
    T vq[kPreT];
#pragma unroll
    for (int q = 0; q < kPreT; ++q) {
      const int k = g0 + q * TEAM + lt;
      evq[q] = k < len ? ld_stream(s.edges + b + k) : 0u;
    }
#pragma unroll
    for (int q = 0; q < kPreT; ++q) {
      const int k = g0 + q * TEAM + lt;
      vq[q] = k < len ? R::elem(s, evq[q]) : R::id();
    }
#pragma unroll
    for (int q = 0; q < kPreT; ++q) {
      const int k0 = g0 + q * TEAM;
      if (k0 >= len) break;  // uniform over the team
      const int k = k0 + lt;
      const bool valid = k < len;
      const int e = b + k;
      const uint32_t ev = evq[q];
      // the old flag matters only for SSSP (unassessable edges) and UNION
      const uint32_t oldf =
          (valid && s.old_bits && (APP == kSSSP || s.mask_union)) ? edge_bit(s.old_bits, e) : 0u;
      bool flag;
      T chunk_total;
      if constexpr (kSumApp<APP>) {
        const double c = vq[q];
        const double incl = team_scan_add<TEAM>(c, lt);
        const double P = carry + incl;
        flag = sum_flag<APP>(s, valid, c, rtot >= 0.0 ? rtot : P, oldf);
        chunk_total = __shfl(incl, TEAM - 1, TEAM);
      } else if constexpr (APP == kSSSP) {
        const uint32_t cand = vq[q];  // INF exactly when the source is unreached
        const uint32_t xv = cand;
        const uint32_t incl = team_scan_min<TEAM>(cand, lt);
        uint32_t excl = (uint32_t)__shfl_up((int)incl, 1, TEAM);
        if (lt == 0) excl = kInf;
        const uint32_t rp = min(carry, excl);
        const uint32_t nw = min(rp, cand);
        const bool dec = (rp == kInf) || ((((uint64_t)(rp - nw)) << 16) > s.theta_q * (uint64_t)rp);
        if (valid && xv != kInf) flag = dec || (s.mask_union && oldf);
        else flag = oldf != 0u;
        chunk_total = __shfl(incl, TEAM - 1, TEAM);
      } else {  // CC
        const uint32_t xv = vq[q];
        const uint32_t incl = team_scan_min<TEAM>(xv, lt);
        uint32_t excl = (uint32_t)__shfl_up((int)incl, 1, TEAM);
        if (lt == 0) excl = kInf;
        const uint32_t rp = min(carry, excl);
        flag = (valid && xv < rp) || (s.mask_union && oldf);
        chunk_total = __shfl(incl, TEAM - 1, TEAM);
      }
      flag = flag && valid;
      const uint64_t bal = __ballot(flag);
      const uint64_t tm = TEAM == 64 ? bal : ((bal >> team_base) & ((1ull << (TEAM & 63)) - 1ull));
      const int rank = __popcll(tm & ((1ull << lt) - 1ull));
      if (flag) s.act_edges[b + carry_cnt + rank] = ev;
      write_bits<TEAM>(s.new_bits, tm, lt, e, len - k, valid);
      carry_cnt += __popcll(tm);
      carry = R::op(carry, chunk_total);
    }
    }
    if (lt == 0) {
      apply<APP>(s, u, carry, nchanged);
      s.act_cnt[u] = carry_cnt;
    }
  }
}

// One 256-edge step of a hub chunk in a superstep: edge b + k (k = sub + thread)
// with gathered value v, the row prefix before the step in carry (advanced by
// the step's total). Writes the new flag bits and returns this thread's flag.
template <int APP>
__device__ __forceinline__ bool hub_step(const Sweep& s, int b, int sub, int e1, typename Tr<APP>::T v,
                                         typename Tr<APP>::T& carry, typename Tr<APP>::T* lds, double rtot) {
  using R = Tr<APP>;
  using T = typename R::T;
  const int lane = __lane_id();
  const int wid = threadIdx.x >> 6;
  const int k = sub + (int)threadIdx.x;
  const bool valid = k < e1;
  const int e = b + k;
  const uint32_t oldf = (valid && s.old_bits && (APP == kSSSP || s.mask_union)) ? edge_bit(s.old_bits, e) : 0u;
  bool flag;
  T sub_total;
  if constexpr (kSumApp<APP>) {
    const double c = v;
    const double incl_w = team_scan_add<64>(c, lane);
    if (lane == 63) lds[wid] = incl_w;
    __syncthreads();
    double before = 0.0;
    for (int w = 0; w < wid; ++w) before += lds[w];
    sub_total = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    const double P = carry + (before + incl_w);
    flag = sum_flag<APP>(s, valid, c, rtot >= 0.0 ? rtot : P, oldf);
  } else {
    const uint32_t val = v;  // SSSP: INF exactly when the source is unreached
    const uint32_t incl_w = team_scan_min<64>(val, lane);
    uint32_t excl_w = (uint32_t)__shfl_up((int)incl_w, 1, 64);
    if (lane == 0) excl_w = kInf;
    if (lane == 63) lds[wid] = incl_w;
    __syncthreads();
    uint32_t before = kInf;
    for (int w = 0; w < wid; ++w) before = min(before, lds[w]);
    sub_total = min(min(lds[0], lds[1]), min(lds[2], lds[3]));
    __syncthreads();
    const uint32_t rp = min(carry, min(before, excl_w));
    if constexpr (APP == kSSSP) {
      const uint32_t nw = min(rp, val);
      const bool dec = (rp == kInf) || ((((uint64_t)(rp - nw)) << 16) > s.theta_q * (uint64_t)rp);
      if (valid && val != kInf) flag = dec || (s.mask_union && oldf);
      else flag = oldf != 0u;
    } else {
      flag = (valid && val < rp) || (s.mask_union && oldf);
    }
  }
  flag = flag && valid;
  const uint64_t bal = __ballot(flag);
  write_bits<64>(s.new_bits, bal, lane, e, e1 - (sub + wid * 64) - lane, valid);
  carry = R::op(carry, sub_total);
  return flag;
}

// Hub chunk of a superstep: prefix carried from the chunk totals computed
// beforehand (part_f / part_u), flags and bits for the chunk, active count
// to part_cnt[ch]. Chunk 0 applies the row with the total of all chunks.
template <int APP>
__device__ __forceinline__ void super_hub_chunk(const Sweep& s, int ch, int& nchanged, typename Tr<APP>::T* lds,
                                                int* ilds) {
  using R = Tr<APP>;
  using T = typename R::T;
  const int h = find_hub(s.hub_start, s.n_hub, ch);
  const int u = s.list[s.n_small + s.n_wave + h];
  const int c0 = s.hub_start[h];
  const int j = ch - c0;
  const int nch = s.hub_start[h + 1] - c0;
  const int b = s.rowptr[u];
  const int len = s.rowptr[u + 1] - b;
  const int e0 = j * s.hub_chunk;
  const int e1 = min(len, e0 + s.hub_chunk);
  const double rtot = (kSumApp<APP> && s.row_total) ? s.row_total[u] : -1.0;

  auto part = [&](int i) -> T {
    if constexpr (kSumApp<APP>) return s.part_f[i];
    else return s.part_u[i];
  };
  T carry = run_init<APP>(s, u);
  for (int i = 0; i < j; ++i) carry = R::op(carry, part(c0 + i));
  int cnt = 0;
  // The edge words and gathered values of kHubPre consecutive 256-edge steps
  // are loaded before the first step's scan, so one round trip to memory
  // serves the whole group.
  for (int g0 = e0; g0 < e1; g0 += kHubPre * kBlock) {
  uint32_t evq[kHubPre];
  T vq[kHubPre];
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) {
    const int k = g0 + q * kBlock + (int)threadIdx.x;
    evq[q] = k < e1 ? ld_stream(s.edges + b + k) : 0u;
  }
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) {
    const int k = g0 + q * kBlock + (int)threadIdx.x;
    vq[q] = k < e1 ? R::elem(s, evq[q]) : R::id();
  }
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) {
    const int sub = g0 + q * kBlock;
    if (sub >= e1) break;  // uniform over the block
    const bool flag = hub_step<APP>(s, b, sub, e1, vq[q], carry, lds, rtot);
    cnt += __popcll(__ballot(flag));
  }
  }
  // cnt is per wave; sum over the block
  const int tot = block_sum_int((__lane_id() == 0) ? cnt : 0, ilds);
  if (threadIdx.x == 0) {
    s.part_cnt[ch] = tot;
    if (j == 0) {
      T all = R::id();
      for (int i = 0; i < nch; ++i) all = R::op(all, part(c0 + i));
      apply<APP>(s, u, all, nchanged);
    }
  }
}

// Chunk totals of the single-pass hub path travel in one 64-bit word that is
// zero until written: PR/PPR/BP the complemented bits of the binary64 total (a
// finite total never complements to zero), SSSP/CC (1 << 32) | minimum.
// Counts travel as count + 1 in a 32-bit word. Both are written and polled
// with relaxed device-scope atomics, which stay coherent across the dies
// without the cache-wide writeback or invalidation that release / acquire
// ordering would cost on every poll.
template <int APP>
__device__ __forceinline__ uint64_t pack_total(typename Tr<APP>::T v) {
  if constexpr (kSumApp<APP>) return ~(uint64_t)__double_as_longlong(v);
  else return (1ull << 32) | (uint64_t)v;
}
template <int APP>
__device__ __forceinline__ typename Tr<APP>::T unpack_total(uint64_t w) {
  if constexpr (kSumApp<APP>) return __longlong_as_double((long long)~w);
  else return (uint32_t)w;
}

// Poll a word until it is non-zero. Past `limit` polls the wait gives up: it
// sets gave_up, raises the error word err (which the host reads back after
// the superstep) and returns 0; the kernel still ends. limit <= 0 gives up
// without polling, which exercises that path on purpose.
template <typename W>
__device__ __forceinline__ W wait_word(W* p, uint32_t* err, int limit, bool& gave_up) {
  W v = 0;
  if (limit > 0) {
    for (int it = 0; (v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0; ++it) {
      if (it >= limit) break;
      __builtin_amdgcn_s_sleep(2);
    }
    if (v != 0) return v;
  }
  atomicOr(err, 1u);
  gave_up = true;
  return 0;
}

// Gathered value in its stored width (defined with the flat batches below).
template <int APP>
struct GV;

// Hub chunk of a superstep in a single pass (hub_chunk <= kHubPre * kBlock).
// Blocks take tickets in dispatch order and process the chunk at that position
// of chunk_order (the natural order when null); the order keeps the chunks of
// a row in row order. A chunk gathers its edges once, publishes its total,
// and takes its row prefix from the totals of the row's earlier chunks,
// summed in a fixed tree order. After its flags it publishes its active
// count, and writes its active edges at the offset that the earlier chunks'
// counts give. The row's last chunk applies the row and writes its active
// count. A chunk waits only on chunks with smaller tickets, whose blocks are
// already resident and publish before they wait, so every wait ends. If a
// wait gives up anyway, the chunk writes no active edge and no active count:
// its offsets would be wrong, and the row keeps the count of its previous
// packing, which still bounds edges written in every packing since.
template <int APP>
__device__ void super_hub_chunk_1p(const Sweep& s, int nchunks, int& nchanged, typename Tr<APP>::T* lds, int* ilds) {
  using R = Tr<APP>;
  using T = typename R::T;
  __shared__ int s_ch, s_cbase, s_bad;
  __shared__ T s_carry;
  __shared__ int s_cnt[kHubPre][4];
  uint32_t* const err = s.hub_sync;
  uint64_t* const tot_w = (uint64_t*)(s.hub_sync + 2);             // [nchunks]
  uint32_t* const cnt_w = s.hub_sync + 2 + 2 * (int64_t)nchunks;   // [nchunks]
  const int lane = __lane_id();
  const int wid = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    const int t = atomicAdd((int*)(s.hub_sync + 1), 1);
    s_ch = s.chunk_order ? s.chunk_order[t] : t;
    s_bad = 0;
  }
  __syncthreads();
  const int ch = s_ch;
  const int h = find_hub(s.hub_start, s.n_hub, ch);
  const int u = s.list[s.n_small + s.n_wave + h];
  const int c0 = s.hub_start[h];
  const int j = ch - c0;
  const int nch = s.hub_start[h + 1] - c0;
  const int b = s.rowptr[u];
  const int len = s.rowptr[u + 1] - b;
  const int e0 = j * s.hub_chunk;
  const int e1 = min(len, e0 + s.hub_chunk);
  const double rtot = (kSumApp<APP> && s.row_total) ? s.row_total[u] : -1.0;
  // gather: every edge of the chunk, all loads in flight together, values
  // held in their stored width (binary32 contributions for PR)
  using V = typename GV<APP>::V;
  uint32_t evq[kHubPre];
  V vq[kHubPre];
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) {
    const int k = e0 + q * kBlock + (int)threadIdx.x;
    evq[q] = k < e1 ? ld_stream(s.edges + b + k) : 0u;
  }
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) {
    const int k = e0 + q * kBlock + (int)threadIdx.x;
    vq[q] = k < e1 ? GV<APP>::get(s, evq[q]) : (V)R::id();
  }
  T acc = R::id();
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) acc = R::op(acc, GV<APP>::widen(vq[q]));
  acc = block_reduce<APP>(acc, lds);
  if (threadIdx.x == 0) __hip_atomic_store(tot_w + ch, pack_total<APP>(acc), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // row prefix: totals of chunks c0 .. ch-1, lane i takes i, i + 64, ...
  if (wid == 0) {
    T p = R::id();
    bool bad = false;
    for (int i = lane; i < j; i += 64) p = R::op(p, unpack_total<APP>(wait_word(tot_w + c0 + i, err, s.hub_spin, bad)));
    p = team_reduce<64>(p);
    if (bad) s_bad = 1;
    if (lane == 0) s_carry = p;
  }
  __syncthreads();
  const T carry0 = R::op(s_carry, run_init<APP>(s, u));
  T carry = carry0;
  bool fq[kHubPre];
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) {
    const int sub = e0 + q * kBlock;
    fq[q] = false;
    if (sub < e1) fq[q] = hub_step<APP>(s, b, sub, e1, GV<APP>::widen(vq[q]), carry, lds, rtot);  // uniform over the block
    const int c = __popcll(__ballot(fq[q]));
    if (lane == 0) s_cnt[q][wid] = c;
  }
  __syncthreads();
  int ctot = 0;
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) ctot += (s_cnt[q][0] + s_cnt[q][1]) + (s_cnt[q][2] + s_cnt[q][3]);
  if (threadIdx.x == 0) __hip_atomic_store(cnt_w + ch, (uint32_t)ctot + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // offset of the chunk's active edges in the row
  if (wid == 0) {
    int cb = 0;
    bool bad = false;
    for (int i = lane; i < j; i += 64) {
      const uint32_t w = wait_word(cnt_w + c0 + i, err, s.hub_spin, bad);
      cb += w != 0u ? (int)w - 1 : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cb += __shfl_xor(cb, o, 64);
    if (bad) s_bad = 1;
    if (lane == 0) s_cbase = cb;
  }
  __syncthreads();
  if (s_bad) {
    // a wait gave up: the carry or the offset is unknown (reported by the
    // error word); write nothing that the offset or count would place
    if (j == nch - 1 && threadIdx.x == 0) apply<APP>(s, u, R::op(carry0, acc), nchanged);
    return;
  }
  int off = s_cbase;
#pragma unroll
  for (int q = 0; q < kHubPre; ++q) {
    int before = 0;
    for (int w = 0; w < wid; ++w) before += s_cnt[q][w];
    const uint64_t bal = __ballot(fq[q]);
    if (fq[q]) s.act_edges[b + off + before + __popcll(bal & ((1ull << lane) - 1ull))] = evq[q];
    off += (s_cnt[q][0] + s_cnt[q][1]) + (s_cnt[q][2] + s_cnt[q][3]);
  }
  if (j == nch - 1 && threadIdx.x == 0) {
    apply<APP>(s, u, R::op(carry0, acc), nchanged);
    s.act_cnt[u] = s_cbase + ctot;
  }
}

template <int APP, int TEAM>
__global__ __launch_bounds__(kBlock) void k_super(Sweep s, int gs, int gw) {
  __shared__ typename Tr<APP>::T lds[4];
  __shared__ int ilds[4];
  int nchanged = 0;
  const int bid = blockIdx.x;
  if (bid < gs) {
    super_team_rows<APP, TEAM>(s, s.list, s.n_small, bid, gs, nchanged);
  } else if (bid < gs + gw) {
    super_team_rows<APP, 64>(s, s.list + s.n_small, s.n_wave, bid - gs, gw, nchanged);
  } else {
    super_hub_chunk<APP>(s, bid - gs - gw, nchanged, lds, ilds);
  }
  flush_changed<APP>(s, nchanged, ilds);
}

// Chunk totals of hub rows before a superstep.
template <int APP>
__global__ __launch_bounds__(kBlock) void k_hub_totals(Sweep s) {
  __shared__ typename Tr<APP>::T lds[4];
  int dummy = 0;
  gather_hub_chunk<APP>(s, s.chunk_order ? s.chunk_order[blockIdx.x] : (int)blockIdx.x, true, dummy, lds);
}

// ---------------------------------------------------------------------------
// Packing of flagged edges (after the initial sampling, and the hub part of
// a superstep)
// ---------------------------------------------------------------------------

template <int TEAM>
__device__ __forceinline__ void pack_team_rows(const Sweep& s, const uint32_t* bits, const int32_t* list, int count,
                                               int blk, int nblk) {
  const int lt = threadIdx.x & (TEAM - 1);
  const int lane = __lane_id();
  const int team_base = lane & ~(TEAM - 1);
  constexpr int TPB = kBlock / TEAM;
  const int stride = nblk * TPB;
  for (int t = blk * TPB + (int)threadIdx.x / TEAM; t < count; t += stride) {
    const int u = list[t];
    const int b = s.rowptr[u];
    const int len = s.rowptr[u + 1] - b;
    int carry_cnt = 0;
    // the flag words and edge words of kPreP team-wide steps are loaded
    // before the first step's ranks
    constexpr int kPreP = 4;
    for (int g0 = 0; g0 < len; g0 += kPreP * TEAM) {
      uint32_t fw[kPreP], ev[kPreP];
#pragma unroll
      for (int q = 0; q < kPreP; ++q) {
        const int k = g0 + q * TEAM + lt;
        fw[q] = k < len ? bits[(b + k) >> 5] : 0u;
        ev[q] = k < len ? ld_stream(s.edges + b + k) : 0u;
      }
#pragma unroll
      for (int q = 0; q < kPreP; ++q) {
        const int k = g0 + q * TEAM + lt;
        const int e = b + k;
        const bool flag = k < len && ((fw[q] >> (e & 31)) & 1u);
        const uint64_t bal = __ballot(flag);
        const uint64_t tm = TEAM == 64 ? bal : ((bal >> team_base) & ((1ull << (TEAM & 63)) - 1ull));
        const int rank = __popcll(tm & ((1ull << lt) - 1ull));
        if (flag) s.act_edges[b + carry_cnt + rank] = ev[q];
        carry_cnt += __popcll(tm);
      }
    }
    if (lt == 0) s.act_cnt[u] = carry_cnt;
  }
}

// Count of flagged edges per hub chunk.
__device__ __forceinline__ void hub_chunk_count(const Sweep& s, const uint32_t* bits, int ch, int* ilds) {
  const int h = find_hub(s.hub_start, s.n_hub, ch);
  const int u = s.list[s.n_small + s.n_wave + h];
  const int j = ch - s.hub_start[h];
  const int b = s.rowptr[u];
  const int len = s.rowptr[u + 1] - b;
  const int e0 = j * s.hub_chunk;
  const int e1 = min(len, e0 + s.hub_chunk);
  // popcount over the flag words covering edges [b + e0, b + e1), the bits
  // outside the range masked off
  int c = 0;
  const int lo = b + e0, hi = b + e1;  // hi > lo
  for (int w = (lo >> 5) + (int)threadIdx.x; w <= ((hi - 1) >> 5); w += kBlock) {
    uint32_t x = bits[w];
    if (w == (lo >> 5)) x &= ~0u << (lo & 31);
    if (w == ((hi - 1) >> 5) && (hi & 31)) x &= (1u << (hi & 31)) - 1u;
    c += __popc(x);
  }
  const int tot = block_sum_int(c, ilds);
  if (threadIdx.x == 0) s.part_cnt[ch] = tot;
}

// Packing of the edges flagged in s.old_bits (the initial sample). Blocks
// [0, gw): wavefront-bin rows, one wavefront per row. [gw, gw + nchunks): the
// flagged-edge count of each hub chunk (k_hub_pack writes their edges next).
// The rest: short rows (degree <= small_max) as flattened batches: a block
// takes kBlock consecutive vertices, stages the edge words of their short
// rows in LDS (every load of a window in flight), then the owner thread of
// each row walks it in CSR order and writes the flagged edges to the front of
// the row's slot.
__global__ __launch_bounds__(kBlock) void k_pack_flat(Sweep s, int gw, int nchunks) {
  __shared__ int ilds[4];
  __shared__ uint32_t s_ev[kFlatWin];
  __shared__ int s_lo[kBlock];
  __shared__ int s_scan[kBlock + 1];
  const int bid = blockIdx.x;
  if (bid < gw) {
    pack_team_rows<64>(s, s.old_bits, s.list + s.n_small, s.n_wave, bid, gw);
    return;
  }
  if (bid < gw + nchunks) {
    hub_chunk_count(s, s.old_bits, bid - gw, ilds);
    return;
  }
  const int tid = threadIdx.x;
  const int u0 = (bid - gw - nchunks) * kBlock;
  const int P = min(kBlock, s.n - u0);
  int u = 0, lo = 0, len = 0;
  bool mine = false;
  if (tid < P) {
    u = u0 + tid;
    lo = s.rowptr[u];
    len = s.rowptr[u + 1] - lo;
    mine = len <= s.small_max;
    if (!mine) len = 0;
  }
  // exclusive scan of the row lengths
  int x = len;
  const int lane = __lane_id(), wid = tid >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) ilds[wid] = x;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wid; ++w) before += ilds[w];
  const int total = ilds[0] + ilds[1] + ilds[2] + ilds[3];
  s_scan[tid] = before + x - len;
  s_lo[tid] = lo;
  __syncthreads();
  const int mine0 = s_scan[tid], mine1 = s_scan[tid] + len;
  int cnt = 0;
  int ow = -1;  // cached flag word
  uint32_t oword = 0;
  for (int base = 0; base < total; base += kFlatWin) {
    const int lim = min(kFlatWin, total - base);
#pragma unroll
    for (int j = 0; j < kFlatWin / kBlock; ++j) {
      const int k = j * kBlock + tid;
      if (k < lim) {
        const int kk = base + k;
        int a = 0, b = P - 1;
        while (a < b) {
          const int mid = (a + b + 1) >> 1;
          if (s_scan[mid] <= kk) a = mid;
          else b = mid - 1;
        }
        s_ev[k] = ld_stream(s.edges + s_lo[a] + (kk - s_scan[a]));
      }
    }
    __syncthreads();
    const int a0 = max(mine0, base), a1 = min(mine1, base + lim);
    for (int k = a0; k < a1; ++k) {
      const int e = lo + (k - mine0);
      if ((e >> 5) != ow) {
        ow = e >> 5;
        oword = s.old_bits[ow];
      }
      if ((oword >> (e & 31)) & 1u) s.act_edges[lo + cnt++] = s_ev[k - base];
    }
    __syncthreads();
  }
  if (mine) s.act_cnt[u] = cnt;
}

// Write the flagged edges of one hub chunk at its rank inside the row; chunk
// 0 writes the row's active count.
__global__ __launch_bounds__(kBlock) void k_hub_pack(Sweep s, const uint32_t* bits) {
  __shared__ int ilds[4];
  const int ch = blockIdx.x;
  const int h = find_hub(s.hub_start, s.n_hub, ch);
  const int u = s.list[s.n_small + s.n_wave + h];
  const int c0 = s.hub_start[h];
  const int j = ch - c0;
  const int nch = s.hub_start[h + 1] - c0;
  const int b = s.rowptr[u];
  const int len = s.rowptr[u + 1] - b;
  const int e0 = j * s.hub_chunk;
  const int e1 = min(len, e0 + s.hub_chunk);
  // counts of the row's earlier chunks (and, for chunk 0, of all chunks),
  // summed by the lanes of wave 0
  __shared__ int s_base[2];
  if (threadIdx.x < 64) {
    int before = 0, all = 0;
    for (int i = (int)threadIdx.x; i < nch; i += 64) {
      const int c = s.part_cnt[c0 + i];
      all += c;
      before += i < j ? c : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      before += __shfl_xor(before, o, 64);
      all += __shfl_xor(all, o, 64);
    }
    if (threadIdx.x == 0) {
      s_base[0] = before;
      s_base[1] = all;
    }
  }
  __syncthreads();
  int carry = s_base[0];
  if (j == 0 && threadIdx.x == 0) s.act_cnt[u] = s_base[1];
  // flag words and edge words of kHubPre steps loaded before the ranks
  for (int g0 = e0; g0 < e1; g0 += kHubPre * kBlock) {
    uint32_t fw[kHubPre], ev[kHubPre];
#pragma unroll
    for (int q = 0; q < kHubPre; ++q) {
      const int k = g0 + q * kBlock + (int)threadIdx.x;
      fw[q] = k < e1 ? bits[(b + k) >> 5] : 0u;
      ev[q] = k < e1 ? ld_stream(s.edges + b + k) : 0u;
    }
#pragma unroll
    for (int q = 0; q < kHubPre; ++q) {
      const int sub = g0 + q * kBlock;
      if (sub >= e1) break;  // uniform over the block
      const int k = sub + (int)threadIdx.x;
      const bool flag = k < e1 && ((fw[q] >> ((b + k) & 31)) & 1u);
      int tot;
      const int rank = block_rank(flag, ilds, tot);
      if (flag) s.act_edges[b + carry + rank] = ev[q];
      carry += tot;
    }
  }
}

// ---------------------------------------------------------------------------
// Degree binning (stable: every list keeps vertex order)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int bin_of(int len, int small_max, int wave_max) {
  return len <= small_max ? 0 : (len <= wave_max ? 1 : 2);
}

__global__ __launch_bounds__(kBlock) void k_bin_count(const int32_t* rowptr, const int32_t* cnt, int n, int small_max,
                                                      int wave_max, int32_t* blk, int64_t* blk_edges, int nblk,
                                                      const uint8_t* rowsel, int selwant) {
  __shared__ int ilds[4];
  __shared__ long long elds[4];
  const int u = blockIdx.x * kBlock + threadIdx.x;
  int len = 0, bin = -1;
  if (u < n && (!rowsel || (rowsel[u] != 0) == (selwant != 0))) {
    len = cnt ? cnt[u] : rowptr[u + 1] - rowptr[u];
    bin = bin_of(len, small_max, wave_max);
  }
  for (int q = 0; q < 3; ++q) {
    int tot;
    block_rank(bin == q, ilds, tot);
    if (threadIdx.x == 0) blk[q * nblk + blockIdx.x] = tot;
  }
  long long e = len;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
  if ((threadIdx.x & 63) == 0) elds[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) blk_edges[blockIdx.x] = elds[0] + elds[1] + elds[2] + elds[3];
}

// Exclusive scan of a[0..count) in place by one 1024-thread block; returns
// the total through *total.
__device__ void block1024_exclusive_scan(int32_t* a, int count, int32_t* total) {
  // wave w owns the contiguous range [w * per, w * per + per), per a multiple
  // of 64; it reads the range in coalesced slices of 16 x 64 with every load
  // of a slice in flight, first to sum it, then to rewrite it through wave
  // scans carried from the range's offset
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = __lane_id(), wid = tid >> 6;
  const int per = ((count + 15) / 16 + 63) & ~63;
  const int b = min(count, wid * per), e = min(count, b + per);
  int sum = 0;
  for (int i0 = b; i0 < e; i0 += 1024) {
    int v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = i0 + k * 64 + lane;
      v[k] = i < e ? a[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += v[k];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (lane == 0) wsum[wid] = sum;
  __syncthreads();
  int carry = 0, all = 0;
  for (int w = 0; w < 16; ++w) {
    carry += (w < wid) ? wsum[w] : 0;
    all += wsum[w];
  }
  for (int i0 = b; i0 < e; i0 += 1024) {
    int v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = i0 + k * 64 + lane;
      v[k] = i < e ? a[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      int x = v[k];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      const int i = i0 + k * 64 + lane;
      if (i < e) a[i] = carry + x - v[k];
      carry += __shfl(x, 63, 64);
    }
  }
  if (tid == 0) *total = all;
  __syncthreads();
}

__global__ __launch_bounds__(1024) void k_bin_scan(int32_t* blk, const int64_t* blk_edges, int nblk, BinCounts* bc) {
  __shared__ int32_t tot[3];
  for (int q = 0; q < 3; ++q) {
    block1024_exclusive_scan(blk + q * nblk, nblk, &tot[q]);
    __syncthreads();
  }
  __shared__ long long es[16];
  long long e = 0;
  for (int i = threadIdx.x; i < nblk; i += 1024) e += blk_edges[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
  if ((threadIdx.x & 63) == 0) es[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < 16; ++w) t += es[w];
    bc->small = tot[0];
    bc->wave = tot[1];
    bc->hub = tot[2];
    bc->edges = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(const int32_t* rowptr, const int32_t* cnt, int n,
                                                        int small_max, int wave_max, const int32_t* blk, int nblk,
                                                        const BinCounts* bc, int32_t* list, const uint8_t* rowsel,
                                                        int selwant) {
  __shared__ int ilds[4];
  const int u = blockIdx.x * kBlock + threadIdx.x;
  int bin = -1;
  if (u < n && (!rowsel || (rowsel[u] != 0) == (selwant != 0))) {
    const int len = cnt ? cnt[u] : rowptr[u + 1] - rowptr[u];
    bin = bin_of(len, small_max, wave_max);
  }
  const int base[3] = {0, bc->small, bc->small + bc->wave};
  for (int q = 0; q < 3; ++q) {
    int tot;
    const int r = block_rank(bin == q, ilds, tot);
    if (bin == q) list[base[q] + blk[q * nblk + blockIdx.x] + r] = u;
  }
}

__global__ __launch_bounds__(kBlock) void k_hub_nchunks(const int32_t* rowptr, const int32_t* cnt, const int32_t* list,
                                                        const BinCounts* bc, int hub_chunk, int32_t* hub_start) {
  const int h = blockIdx.x * kBlock + threadIdx.x;
  if (h < bc->hub) {
    const int u = list[bc->small + bc->wave + h];
    const int len = cnt ? cnt[u] : rowptr[u + 1] - rowptr[u];
    hub_start[h] = (len + hub_chunk - 1) / hub_chunk;
  }
}

__global__ __launch_bounds__(1024) void k_hub_scan(int32_t* hub_start, BinCounts* bc, const uint32_t* hub_err) {
  __shared__ int32_t tot;
  const int nh = bc->hub;
  block1024_exclusive_scan(hub_start, nh, &tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    hub_start[nh] = tot;
    bc->chunks = tot;
    bc->hub_err = hub_err ? *hub_err : 0u;
  }
}

// ---------------------------------------------------------------------------
// Sampling [Sec. 3.4]: Philox4x64-10 (Salmon et al., SC'11)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1, uint64_t out[4]) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// One thread per bitmap word (32 edges = 4 Philox blocks of 8 draws).
__global__ __launch_bounds__(kBlock) void k_sample_bits(int64_t m, uint64_t seed, uint64_t epoch, uint64_t keep,
                                                        uint32_t* bits) {
  const int64_t nw = (m + 31) >> 5;
  for (int64_t w = blockIdx.x * (int64_t)kBlock + threadIdx.x; w < nw; w += (int64_t)gridDim.x * kBlock) {
    uint32_t word = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint64_t o[4];
      philox4x64_10((uint64_t)(w * 4 + q), epoch, 0, 0, seed, 0, o);
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const uint64_t word64 = o[h >> 1];
        const uint32_t d = (h & 1) ? (uint32_t)(word64 >> 32) : (uint32_t)word64;
        const int64_t e = w * 32 + q * 8 + h;
        if (e < m && (uint64_t)d < keep) word |= 1u << (q * 8 + h);
      }
    }
    bits[w] = word;
  }
}

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------

__global__ void k_outdeg(const int32_t* col, int64_t m, int32_t* outdeg) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&outdeg[col[i]], 1);
}

__global__ void k_pack_weights(const int32_t* col, const int32_t* w, int64_t m, uint32_t* packed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    packed[i] = ((uint32_t)w[i] << 24) | (uint32_t)col[i];
}

__global__ void k_fill_u32(uint32_t* p, int64_t count, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_copy_u32(const uint32_t* a, uint32_t* b, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_iota(int32_t* p, int32_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

__global__ void k_pr_init(int app, const int32_t* outdeg, int32_t n, int32_t source, const int32_t* part_of,
                          const int32_t* part_start, float* c) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double x;
    if (app == kPR) {
      // 1/N, with N the vertex count of the vertex's part when parts are set
      double N = (double)n;
      if (part_of) {
        const int p = part_of[i];
        N = (double)(part_start[p + 1] - part_start[p]);
      }
      x = 1.0 / N;
    } else {
      x = (i == source) ? 1.0 : 0.0;
    }
    const int od = outdeg[i];
    c[i] = od > 0 ? (float)(x / (double)od) : (float)x;
  }
}

// BP before iteration 1: every belief is its prior; c[u] is its message.
__global__ void k_bp_init(const float* prior, int32_t n, double kappa, float* c) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c[i] = (float)bp_message((double)prior[i], kappa);
}

__global__ void k_min_init(int app, int32_t n, int32_t source, uint32_t* x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (app == kSSSP) x[i] = (i == source) ? 0u : kInf;
    else x[i] = (uint32_t)i;
  }
}

// Dangling list: stable compaction of the vertices with out-degree 0.
__global__ __launch_bounds__(kBlock) void k_dang_count(const int32_t* outdeg, int n, int32_t* blk) {
  __shared__ int ilds[4];
  const int u = blockIdx.x * kBlock + threadIdx.x;
  int tot;
  block_rank(u < n && outdeg[u] == 0, ilds, tot);
  if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan1(int32_t* a, int count, int32_t* total) {
  __shared__ int32_t tot;
  block1024_exclusive_scan(a, count, &tot);
  __syncthreads();
  if (threadIdx.x == 0) *total = tot;
}

__global__ __launch_bounds__(kBlock) void k_dang_scatter(const int32_t* outdeg, int n, const int32_t* blk,
                                                         int32_t* list) {
  __shared__ int ilds[4];
  const int u = blockIdx.x * kBlock + threadIdx.x;
  const bool d = u < n && outdeg[u] == 0;
  int tot;
  const int r = block_rank(d, ilds, tot);
  if (d) list[blk[blockIdx.x] + r] = u;
}

constexpr int kDangBlocks = 256;

__global__ __launch_bounds__(kBlock) void k_dsum_partial(const float* c, const int32_t* list, int count,
                                                         double* partial) {
  __shared__ double lds[4];
  const int per = (count + kDangBlocks - 1) / kDangBlocks;
  const int lo = blockIdx.x * per, hi = min(count, lo + per);
  double acc = 0.0;
  // 8 index and value loads in flight per thread; added in index order
  int i = lo + (int)threadIdx.x;
  for (; i + 7 * kBlock < hi; i += 8 * kBlock) {
    int id[8];
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) id[k] = list[i + k * kBlock];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = c[id[k]];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += (double)v[k];
  }
  for (; i < hi; i += kBlock) acc += (double)c[list[i]];
  acc = block_reduce<kPR>(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void k_dsum_final(const double* partial, double* out) {
  __shared__ double lds[4];
  double acc = partial[threadIdx.x];
  acc = block_reduce<kPR>(acc, lds);
  if (threadIdx.x == 0) *out = acc;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_outdeg(const int32_t* col, int64_t m, int32_t* outdeg, int32_t n, hipStream_t st) {
  hipError_t e = launch_fill_u32((uint32_t*)outdeg, n, 0u, st);
  if (e != hipSuccess || m == 0) return e;
  hipLaunchKernelGGL(k_outdeg, dim3(grid_for(m, kBlock * 8, 1 << 16)), dim3(kBlock), 0, st, col, m, outdeg);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const int32_t* col, const int32_t* w, int64_t m, uint32_t* packed, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_weights, dim3(grid_for(m, kBlock * 8, 1 << 16)), dim3(kBlock), 0, st, col, w, m, packed);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, kBlock * 8, 1 << 16)), dim3(kBlock), 0, st, p, count, v);
  return hipGetLastError();
}

hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_u32, dim3(grid_for(count, kBlock * 8, 1 << 16)), dim3(kBlock), 0, st, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t* p, int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n, kBlock * 8, 1 << 16)), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_dangling_list(const int32_t* outdeg, int32_t n, int32_t* list, int32_t* count,
                                int32_t* blk_scratch, hipStream_t st) {
  const int nblk = (n + kBlock - 1) / kBlock;
  if (n == 0) return launch_fill_u32((uint32_t*)count, 1, 0u, st);
  hipLaunchKernelGGL(k_dang_count, dim3(nblk), dim3(kBlock), 0, st, outdeg, n, blk_scratch);
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, st, blk_scratch, nblk, count);
  hipLaunchKernelGGL(k_dang_scatter, dim3(nblk), dim3(kBlock), 0, st, outdeg, n, blk_scratch, list);
  return hipGetLastError();
}

hipError_t launch_dangling_sum(const float* c, const int32_t* list, const int32_t* /*count_dev*/, int32_t count,
                               double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dsum_partial, dim3(kDangBlocks), dim3(kBlock), 0, st, c, list, count, partial);
  hipLaunchKernelGGL(k_dsum_final, dim3(1), dim3(kBlock), 0, st, partial, out);
  return hipGetLastError();
}

hipError_t launch_rebin(const int32_t* rowptr, const int32_t* cnt, int32_t n, int32_t small_max, int32_t wave_max,
                        int32_t hub_chunk, Bins& bins, void* blk_scratch, hipStream_t st, const uint8_t* rowsel,
                        int selwant, const uint32_t* hub_err) {
  const int nblk = (n + kBlock - 1) / kBlock;
  int32_t* blk = (int32_t*)blk_scratch;
  int64_t* blk_edges = (int64_t*)(blk + 3 * (int64_t)nblk + ((3 * nblk) & 1));
  if (n == 0) {
    BinCounts z{};
    hipError_t e = hipMemcpyAsync(bins.dcounts, &z, sizeof(z), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return launch_fill_u32((uint32_t*)bins.hub_start, 1, 0u, st);
  }
  hipLaunchKernelGGL(k_bin_count, dim3(nblk), dim3(kBlock), 0, st, rowptr, cnt, n, small_max, wave_max, blk,
                     blk_edges, nblk, rowsel, selwant);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, blk, blk_edges, nblk, bins.dcounts);
  hipLaunchKernelGGL(k_bin_scatter, dim3(nblk), dim3(kBlock), 0, st, rowptr, cnt, n, small_max, wave_max, blk, nblk,
                     bins.dcounts, bins.list, rowsel, selwant);
  hipLaunchKernelGGL(k_hub_nchunks, dim3(nblk), dim3(kBlock), 0, st, rowptr, cnt, bins.list, bins.dcounts, hub_chunk,
                     bins.hub_start);
  hipLaunchKernelGGL(k_hub_scan, dim3(1), dim3(1024), 0, st, bins.hub_start, bins.dcounts, hub_err);
  return hipGetLastError();
}

hipError_t launch_pr_init(int app, const int32_t* outdeg, int32_t n, int32_t source, const int32_t* part_of,
                          const int32_t* part_start, float* c, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pr_init, dim3(grid_for(n, kBlock * 4, 1 << 16)), dim3(kBlock), 0, st, app, outdeg, n, source,
                     part_of, part_start, c);
  return hipGetLastError();
}

__global__ __launch_bounds__(64) void k_post(const uint32_t* src, int32_t words, uint32_t* host, uint32_t seq) {
  const int t = threadIdx.x;
  if (t < words) __hip_atomic_store(host + 1 + t, src[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __syncthreads();
  if (t == 0) {
    __threadfence_system();
    __hip_atomic_store(host, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

hipError_t launch_post(const uint32_t* src, int32_t words, uint32_t* host, uint32_t seq, hipStream_t st) {
  hipLaunchKernelGGL(k_post, dim3(1), dim3(64), 0, st, src, words, host, seq);
  return hipGetLastError();
}

hipError_t launch_bp_init(const float* prior, int32_t n, double kappa, float* c, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bp_init, dim3(grid_for(n, kBlock * 4, 1 << 16)), dim3(kBlock), 0, st, prior, n, kappa, c);
  return hipGetLastError();
}

hipError_t launch_min_init(int app, int32_t n, int32_t source, uint32_t* x, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_min_init, dim3(grid_for(n, kBlock * 4, 1 << 16)), dim3(kBlock), 0, st, app, n, source, x);
  return hipGetLastError();
}

hipError_t launch_sample_bits(int64_t m, uint64_t seed, uint64_t epoch, uint64_t keep, uint32_t* bits,
                              hipStream_t st) {
  const int64_t nw = (m + 31) >> 5;
  if (nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_bits, dim3(grid_for(nw, kBlock, 1 << 16)), dim3(kBlock), 0, st, m, seed, epoch, keep,
                     bits);
  return hipGetLastError();
}

static constexpr int kTeamBlockCap = 16384;

static void section_grids(const Sweep& s, int team, int& gs, int& gw) {
  gs = s.n_small > 0 ? grid_for(s.n_small, kBlock / team, kTeamBlockCap) : 0;
  gw = s.n_wave > 0 ? grid_for(s.n_wave, kBlock / 64, kTeamBlockCap) : 0;
}

static int hub_chunks(const Sweep& s) { return s.n_hub > 0 ? s.n_chunks : 0; }

template <int APP, int TEAM>
static hipError_t gather_t(const Sweep& s, int nchunks, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  int gs, gw;
  section_grids(s, TEAM, gs, gw);
  const int total = gs + gw + nchunks;
  if (ev0) (void)hipEventRecord(ev0, st);
  if (total > 0) hipLaunchKernelGGL((k_gather<APP, TEAM>), dim3(total), dim3(kBlock), 0, st, s, gs, gw);
  if (ev1) (void)hipEventRecord(ev1, st);
  if (s.n_hub > 0) hipLaunchKernelGGL((k_hub_combine<APP>), dim3(grid_for(s.n_hub, kBlock, 1 << 20)), dim3(kBlock), 0,
                                      st, s);
  return hipGetLastError();
}

template <int APP, int TEAM>
static hipError_t super_t(const Sweep& s, int nchunks, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  int gs, gw;
  section_grids(s, TEAM, gs, gw);
  if (nchunks > 0) hipLaunchKernelGGL((k_hub_totals<APP>), dim3(nchunks), dim3(kBlock), 0, st, s);
  const int total = gs + gw + nchunks;
  if (ev0) (void)hipEventRecord(ev0, st);
  if (total > 0) hipLaunchKernelGGL((k_super<APP, TEAM>), dim3(total), dim3(kBlock), 0, st, s, gs, gw);
  if (ev1) (void)hipEventRecord(ev1, st);
  if (nchunks > 0) hipLaunchKernelGGL(k_hub_pack, dim3(nchunks), dim3(kBlock), 0, st, s, (const uint32_t*)s.new_bits);
  return hipGetLastError();
}


#define GG_DISPATCH_TEAM(FN, APP, team, ...)                      \
  switch (team) {                                                 \
    case 4: return FN<APP, 4>(__VA_ARGS__);                       \
    case 8: return FN<APP, 8>(__VA_ARGS__);                       \
    case 16: return FN<APP, 16>(__VA_ARGS__);                     \
    case 32: return FN<APP, 32>(__VA_ARGS__);                     \
    default: return hipErrorInvalidValue;                         \
  }

template <int APP>
static hipError_t gather_app(int team, const Sweep& s, int nchunks, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  GG_DISPATCH_TEAM(gather_t, APP, team, s, nchunks, st, ev0, ev1)
}
template <int APP>
static hipError_t super_app(int team, const Sweep& s, int nchunks, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  GG_DISPATCH_TEAM(super_t, APP, team, s, nchunks, st, ev0, ev1)
}

hipError_t launch_gather(int app, int team, const Sweep& s, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int nchunks = hub_chunks(s);
  switch (app) {
    case kPR: return gather_app<kPR>(team, s, nchunks, st, ev0, ev1);
    case kPPR: return gather_app<kPPR>(team, s, nchunks, st, ev0, ev1);
    case kBP: return gather_app<kBP>(team, s, nchunks, st, ev0, ev1);
    case kSSSP: return gather_app<kSSSP>(team, s, nchunks, st, ev0, ev1);
    case kCC: return gather_app<kCC>(team, s, nchunks, st, ev0, ev1);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_superstep(int app, int team, const Sweep& s, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int nchunks = hub_chunks(s);
  switch (app) {
    case kPR: return super_app<kPR>(team, s, nchunks, st, ev0, ev1);
    case kPPR: return super_app<kPPR>(team, s, nchunks, st, ev0, ev1);
    case kBP: return super_app<kBP>(team, s, nchunks, st, ev0, ev1);
    case kSSSP: return super_app<kSSSP>(team, s, nchunks, st, ev0, ev1);
    case kCC: return super_app<kCC>(team, s, nchunks, st, ev0, ev1);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pack(const Sweep& s, hipStream_t st) {
  const int nchunks = hub_chunks(s);
  const int gw = s.n_wave > 0 ? grid_for(s.n_wave, kBlock / 64, kTeamBlockCap) : 0;
  const int gs = (s.n + kBlock - 1) / kBlock;
  const int total = gw + nchunks + gs;
  if (total > 0) hipLaunchKernelGGL(k_pack_flat, dim3(total), dim3(kBlock), 0, st, s, gw, nchunks);
  if (nchunks > 0) hipLaunchKernelGGL(k_hub_pack, dim3(nchunks), dim3(kBlock), 0, st, s, s.old_bits);
  return hipGetLastError();
}

}  // namespace ggk

namespace ggk {

// Structure check of an in-CSR: bit 0 rowptr ends, bit 1 rowptr decreasing,
// bit 2 column out of range, bit 3 weight outside [0, 255].
__global__ void k_validate(const int32_t* rowptr, const int32_t* col, const int32_t* w, int32_t n, int64_t m,
                           int32_t* flags) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int f = 0;
  if (tid == 0 && (rowptr[0] != 0 || (int64_t)rowptr[n] != m)) f |= 1;
  for (int64_t u = tid; u < n; u += stride)
    if (rowptr[u + 1] < rowptr[u]) f |= 2;
  for (int64_t e = tid; e < m; e += stride) {
    const int32_t v = col[e];
    if (v < 0 || v >= n) f |= 4;
    if (w && (w[e] < 0 || w[e] > 255)) f |= 8;
  }
  if (f) atomicOr(flags, f);
}

// Bit 4: some row lists its sources out of ascending order. One wavefront
// per row (rowptr already checked).
__global__ void k_rows_sorted(const int32_t* rowptr, const int32_t* col, int32_t n, int32_t* flags) {
  const int lane = __lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  bool bad = false;
  for (int64_t u = wave; u < n; u += nwaves) {
    const int b = rowptr[u], e = rowptr[u + 1];
    for (int k = b + 1 + lane; k < e; k += 64) bad |= col[k] < col[k - 1];
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(flags, 16);
}

hipError_t launch_validate(const int32_t* rowptr, const int32_t* col, const int32_t* w, int32_t n, int64_t m,
                           int32_t* flags, hipStream_t st) {
  hipError_t e = launch_fill_u32((uint32_t*)flags, 1, 0u, st);
  if (e != hipSuccess) return e;
  const int64_t work = m > n ? m : n;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(work + 1, kBlock * 8, 1 << 16)), dim3(kBlock), 0, st, rowptr, col, w,
                     n, m, flags);
  return hipGetLastError();
}

hipError_t launch_rows_sorted(const int32_t* rowptr, const int32_t* col, int32_t n, int32_t* flags, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_sorted, dim3(grid_for((int64_t)n * 64, kBlock, 1 << 14)), dim3(kBlock), 0, st, rowptr,
                     col, n, flags);
  return hipGetLastError();
}

}  // namespace ggk

// ===========================================================================
// Source-segmented gather of long rows
//
// Rows longer than the small bin are sorted by source id, so the edges of a
// row whose sources fall in segment s = [s*Z, (s+1)*Z) are contiguous. Each
// (row, segment) piece is reduced separately; all pieces of one segment read
// source values from a Z-vertex window that fits in one die's L2. Consecutive
// block ids are dispatched to the eight dies in turn, so the block->piece map
// keeps each die on one segment at a time. Pieces are combined per row in
// segment order (fixed order: bitwise reproducible).
// ===========================================================================
namespace ggk {

__device__ __forceinline__ void seg_map(int b, int S, int Q, int& seg, int& q) {
  const int xcd = b & 7, k = b >> 3;
  seg = xcd + 8 * (k / Q);
  q = k % Q;
}

__global__ __launch_bounds__(kBlock) void k_seg_offsets(Sweep s, uint32_t src_mask, int32_t* seg_off) {
  const int nl = s.n_wave + s.n_hub;
  const int S = s.seg_s;
  const int64_t total = (int64_t)(S + 1) * nl;
  for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock) {
    const int sg = (int)(t / nl);
    const int i = (int)(t - (int64_t)sg * nl);
    const int u = s.list[s.n_small + i];
    const int b = s.rowptr[u];
    const int len = row_len(s, u, b);
    int off;
    if (sg == 0) {
      off = b;
    } else if (sg == S) {
      off = b + len;
    } else {
      const uint32_t key = (uint32_t)sg * (uint32_t)s.seg_z;
      int lo = 0, hi = len;  // first position with source >= key
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((s.edges[b + mid] & src_mask) < key) lo = mid + 1;
        else hi = mid;
      }
      off = b + lo;
    }
    seg_off[(int64_t)sg * nl + i] = off;
  }
}

template <int APP>
__device__ __forceinline__ void seg_store(const Sweep& s, int64_t idx, typename Tr<APP>::T v) {
  if constexpr (kSumApp<APP>) s.seg_part_f[idx] = v;
  else s.seg_part_u[idx] = v;
}

// Value type a gathered edge contributes before the reduction (what LDS holds).
template <int APP>
struct GV {
  using V = uint32_t;
  static __device__ __forceinline__ V get(const Sweep& s, uint32_t e) { return Tr<APP>::elem(s, e); }
  static __device__ __forceinline__ typename Tr<APP>::T widen(V v) { return v; }
};
template <>
struct GV<kPR> {
  using V = float;
  static __device__ __forceinline__ V get(const Sweep& s, uint32_t e) { return s.c_in[e]; }
  static __device__ __forceinline__ double widen(V v) { return (double)v; }
};
template <>
struct GV<kPPR> : GV<kPR> {};
template <>
struct GV<kBP> : GV<kPR> {};



// One block reduces a batch of P <= kBlock pieces [lo_p, hi_p) of the edge
// array: every edge of the batch is gathered independently (kSegWin per
// round) into LDS, then the owner thread of each piece sums its values in
// edge order. Returns the owner's result. A round runs in phases (positions,
// edge words, values, LDS stores) so that all of a thread's edge-word loads,
// and then all of its value loads, are in flight together.
template <int APP>
__device__ __forceinline__ typename Tr<APP>::T flat_batch(const Sweep& s, int P, int my_lo, int my_len,
                                                          typename GV<APP>::V* s_val, int* s_lo, int* s_scan,
                                                          int* ilds) {
  using R = Tr<APP>;
  const int tid = threadIdx.x;
  // exclusive scan of the piece lengths
  const int len = tid < P ? my_len : 0;
  int x = len;
  const int lane = __lane_id(), wid = tid >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) ilds[wid] = x;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wid; ++w) before += ilds[w];
  const int total = ilds[0] + ilds[1] + ilds[2] + ilds[3];
  s_scan[tid] = before + x - len;
  s_lo[tid] = my_lo;
  if (tid == 0) s_scan[kBlock] = total;
  __syncthreads();
  typename R::T acc = R::id();
  const int mine0 = s_scan[tid], mine1 = tid < P ? s_scan[tid] + len : s_scan[tid];
  for (int base = 0; base < total; base += kSegWin) {
    const int lim = min(kSegWin, total - base);
    constexpr int J = kSegWin / kBlock;
    int pos[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int k = j * kBlock + tid;
      pos[j] = -1;
      if (k < lim) {
        const int kk = base + k;
        int lo = 0, hi = P - 1;  // last piece whose start <= kk
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_scan[mid] <= kk) lo = mid;
          else hi = mid - 1;
        }
        pos[j] = s_lo[lo] + (kk - s_scan[lo]);
      }
    }
    uint32_t ev[J];
#pragma unroll
    for (int j = 0; j < J; ++j) ev[j] = pos[j] >= 0 ? ld_stream(s.edges + pos[j]) : 0u;
    typename GV<APP>::V val[J];
#pragma unroll
    for (int j = 0; j < J; ++j) val[j] = pos[j] >= 0 ? GV<APP>::get(s, ev[j]) : typename GV<APP>::V(0);
#pragma unroll
    for (int j = 0; j < J; ++j)
      if (pos[j] >= 0) s_val[j * kBlock + tid] = val[j];
    __syncthreads();
    const int a = max(mine0, base), b = min(mine1, base + lim);
    for (int k = a; k < b; ++k) acc = R::op(acc, GV<APP>::widen(s_val[k - base]));
    __syncthreads();
  }
  return acc;
}

template <int APP>
__global__ __launch_bounds__(kBlock) void k_gather_seg(Sweep s, int gh, int gw, int gs) {
  using R = Tr<APP>;
  using T = typename R::T;
  __shared__ T lds[4];
  __shared__ int ilds[4];
  __shared__ typename GV<APP>::V s_val[kSegWin];
  __shared__ int s_lo[kBlock];
  __shared__ int s_scan[kBlock + 1];
  int nchanged = 0;
  const int bid = blockIdx.x;
  const int nl = s.n_wave + s.n_hub;
  if (bid < gh) {
    // one block per (hub row, segment) piece
    int sg, h;
    seg_map(bid, s.seg_s, s.n_hub, sg, h);
    const int i = s.n_wave + h;
    const bool skipped = s.skip && s.skip[s.list[s.n_small + i]];  // uniform over the block
    const int lo = s.seg_off[(int64_t)sg * nl + i];
    const int hi = skipped ? lo : s.seg_off[(int64_t)(sg + 1) * nl + i];
    T acc = R::id();
    int k = lo + (int)threadIdx.x;
    for (; k + 3 * kBlock < hi; k += 4 * kBlock) {
      const uint32_t a0 = ld_stream(s.edges + k), a1 = ld_stream(s.edges + k + kBlock);
      const uint32_t a2 = ld_stream(s.edges + k + 2 * kBlock), a3 = ld_stream(s.edges + k + 3 * kBlock);
      const T v0 = R::elem(s, a0), v1 = R::elem(s, a1), v2 = R::elem(s, a2), v3 = R::elem(s, a3);
      acc = R::op(acc, R::op(R::op(v0, v1), R::op(v2, v3)));
    }
    for (; k < hi; k += kBlock) acc = R::op(acc, R::elem(s, ld_stream(s.edges + k)));
    acc = block_reduce<APP>(acc, lds);
    if (threadIdx.x == 0) seg_store<APP>(s, (int64_t)sg * nl + i, acc);
  } else if (bid < gh + gw) {
    // (segment, batch of kSegRowsPerBlock wavefront-bin rows): flattened pieces
    int sg, q;
    seg_map(bid - gh, s.seg_s, s.seg_qw, sg, q);
    const int i0 = q * kSegRowsPerBlock;
    const int P = min(kSegRowsPerBlock, s.n_wave - i0);
    int lo = 0, len = 0;
    if ((int)threadIdx.x < P) {
      const int i = i0 + threadIdx.x;
      lo = s.seg_off[(int64_t)sg * nl + i];
      len = s.seg_off[(int64_t)(sg + 1) * nl + i] - lo;
      if (s.skip && s.skip[s.list[s.n_small + i]]) len = 0;
    }
    const T acc = flat_batch<APP>(s, P, lo, len, s_val, s_lo, s_scan, ilds);
    if ((int)threadIdx.x < P) seg_store<APP>(s, (int64_t)sg * nl + i0 + threadIdx.x, acc);
  } else {
    // kBlock consecutive vertices: the short ones (length <= small_max) are
    // gathered here, unsegmented, and applied; the long ones have length 0
    // here (their pieces are combined by k_seg_combine)
    const int u0 = (bid - gh - gw) * kBlock;
    const int P = min(kBlock, s.n - u0);
    const int u = u0 + (int)threadIdx.x;
    int lo = 0, len = 0;
    bool mine = false;
    uint32_t word = 0;  // the apply's own read, issued before the gather
    if ((int)threadIdx.x < P) {
      lo = s.rowptr[u];
      len = row_len(s, u, lo);
      word = apply_word<APP>(s, u);
      mine = len <= s.small_max && !(s.skip && s.skip[u]);
      if (!mine) len = 0;
    }
    const T acc = flat_batch<APP>(s, P, lo, len, s_val, s_lo, s_scan, ilds);
    if (mine) apply_with<APP>(s, u, acc, word, nchanged);
  }
  flush_changed<APP>(s, nchanged, ilds);
}

// Combine the segment pieces of every long row in segment order and apply.
template <int APP>
__global__ __launch_bounds__(kBlock) void k_seg_combine(Sweep s) {
  using R = Tr<APP>;
  __shared__ int ilds[4];
  int nchanged = 0;
  const int nl = s.n_wave + s.n_hub;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int u = i < nl ? s.list[s.n_small + i] : 0;
  if (i < nl && !(s.skip && s.skip[u])) {
    typename R::T acc = R::id();
    for (int sg = 0; sg < s.seg_s; ++sg) {
      if constexpr (kSumApp<APP>) acc = R::op(acc, s.seg_part_f[(int64_t)sg * nl + i]);
      else acc = R::op(acc, s.seg_part_u[(int64_t)sg * nl + i]);
    }
    apply<APP>(s, u, acc, nchanged);
  }
  flush_changed<APP>(s, nchanged, ilds);
}

hipError_t launch_seg_offsets(const Sweep& s, uint32_t src_mask, int32_t* seg_off, hipStream_t st) {
  const int64_t total = (int64_t)(s.seg_s + 1) * (s.n_wave + s.n_hub);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_offsets, dim3(grid_for(total, kBlock, 1 << 16)), dim3(kBlock), 0, st, s, src_mask,
                     seg_off);
  return hipGetLastError();
}

template <int APP, int TEAM>
static hipError_t gather_seg_t(const Sweep& s, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int gh = s.n_hub > 0 ? s.seg_s * s.n_hub : 0;
  const int gw = s.n_wave > 0 ? s.seg_s * s.seg_qw : 0;
  const int gs = (s.n + kBlock - 1) / kBlock;
  const int total = gh + gw + gs;
  if (ev0) (void)hipEventRecord(ev0, st);
  if (total > 0) hipLaunchKernelGGL((k_gather_seg<APP>), dim3(total), dim3(kBlock), 0, st, s, gh, gw, gs);
  if (ev1) (void)hipEventRecord(ev1, st);
  const int nl = s.n_wave + s.n_hub;
  if (nl > 0) hipLaunchKernelGGL((k_seg_combine<APP>), dim3(grid_for(nl, kBlock, 1 << 20)), dim3(kBlock), 0, st, s);
  return hipGetLastError();
}

template <int APP>
static hipError_t gather_seg_app(int team, const Sweep& s, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  switch (team) {
    case 4: return gather_seg_t<APP, 4>(s, st, ev0, ev1);
    case 8: return gather_seg_t<APP, 8>(s, st, ev0, ev1);
    case 16: return gather_seg_t<APP, 16>(s, st, ev0, ev1);
    case 32: return gather_seg_t<APP, 32>(s, st, ev0, ev1);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gather_seg(int app, int team, const Sweep& s, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  switch (app) {
    case kPR: return gather_seg_app<kPR>(team, s, st, ev0, ev1);
    case kPPR: return gather_seg_app<kPPR>(team, s, st, ev0, ev1);
    case kBP: return gather_seg_app<kBP>(team, s, st, ev0, ev1);
    case kSSSP: return gather_seg_app<kSSSP>(team, s, st, ev0, ev1);
    case kCC: return gather_seg_app<kCC>(team, s, st, ev0, ev1);
  }
  return hipErrorInvalidValue;
}

}  // namespace ggk

// ===========================================================================
// Frontier iterations for SSSP / CC (the active-vertex list of the vertex-
// centric model): only vertices that changed in the previous iteration can
// change their out-neighbours, provided the edge set did not grow. A sparse
// iteration pushes from the changed vertices over their out-edges with
// atomicMin into the next buffer, which reproduces the synchronous pull
// result exactly (min is order-free).
// ===========================================================================
namespace ggk {

// ---- generic multi-block exclusive scan ------------------------------------
__global__ __launch_bounds__(1024) void k_scan_blocks(const int32_t* in, int32_t n, int32_t* blk) {
  __shared__ int ws[16];
  const int i = blockIdx.x * 1024 + threadIdx.x;
  int v = i < n ? in[i] : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < 16; ++w) t += ws[w];
    blk[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(1024) void k_scan_apply(const int32_t* in, int32_t* out, int32_t n, const int32_t* blk) {
  __shared__ int ws[16];
  const int tid = threadIdx.x, lane = __lane_id(), wid = tid >> 6;
  const int i = blockIdx.x * 1024 + tid;
  const int v = i < n ? in[i] : 0;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) ws[wid] = x;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wid; ++w) before += ws[w];
  if (i < n) out[i] = blk[blockIdx.x] + before + x - v;
}

hipError_t launch_scan(const int32_t* in, int32_t* out, int32_t n, int32_t* total, int32_t* scratch,
                       hipStream_t st) {
  const int nb = (n + 1023) / 1024;
  if (n == 0) return launch_fill_u32((uint32_t*)total, 1, 0u, st);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, st, in, n, scratch);
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, st, scratch, nb, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, st, in, out, n, scratch);
  return hipGetLastError();
}

// ---- out-CSR structure -------------------------------------------------------
// Entry pos of source v: in-edge id oedge, destination odst and the source
// itself in osrc (what an update needs to carry an entry over without
// looking up its in-edge).
__global__ void k_out_scatter(const int32_t* rowptr, const int32_t* col, int32_t n, int64_t m, const int32_t* orow,
                              int32_t* cursor, int32_t* oedge, int32_t* odst, int32_t* osrc) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = n - 1;  // the row holding edge e: last u with rowptr[u] <= e
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rowptr[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int v = col[e];
    const int pos = orow[v] + atomicAdd(&cursor[v], 1);
    oedge[pos] = (int32_t)e;
    odst[pos] = lo;
    osrc[pos] = v;
  }
}

hipError_t launch_build_out(const int32_t* rowptr, const int32_t* col, int32_t n, int64_t m, const int32_t* orow,
                            int32_t* cursor, int32_t* oedge, int32_t* odst, int32_t* osrc, hipStream_t st) {
  hipError_t e = launch_fill_u32((uint32_t*)cursor, n, 0u, st);
  if (e != hipSuccess || m == 0 || n == 0) return e;
  hipLaunchKernelGGL(k_out_scatter, dim3(grid_for(m, kBlock * 4, 1 << 16)), dim3(kBlock), 0, st, rowptr, col, n, m,
                     orow, cursor, oedge, odst, osrc);
  return hipGetLastError();
}

// ---- changed list after a dense iteration ----------------------------------
// Per-block counts of changed vertices; block 0 also clears the touched
// counter (the count and the out-degree sum are written by later kernels).
__global__ __launch_bounds__(kBlock) void k_chg_count(const uint8_t* chg, int n, int32_t* blk, FrontCounters* fc) {
  __shared__ int ilds[4];
  const int u = blockIdx.x * kBlock + threadIdx.x;
  int tot;
  block_rank(u < n && chg[u], ilds, tot);
  if (threadIdx.x == 0) blk[blockIdx.x] = tot;
  if (blockIdx.x == 0 && threadIdx.x == 0) fc->touched = 0;
}

// Per-block out-degree sums go to psum[block]; k_sum_i64 adds them.
__global__ __launch_bounds__(kBlock) void k_chg_scatter(const uint8_t* chg, const int32_t* outdeg, int n,
                                                        const int32_t* blk, int32_t* list, int64_t* psum) {
  __shared__ int ilds[4];
  __shared__ long long elds[4];
  const int u = blockIdx.x * kBlock + threadIdx.x;
  const bool c = u < n && chg[u];
  int tot;
  const int r = block_rank(c, ilds, tot);
  if (c) list[blk[blockIdx.x] + r] = u;
  long long d = c ? outdeg[u] : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
  if ((threadIdx.x & 63) == 0) elds[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) psum[blockIdx.x] = elds[0] + elds[1] + elds[2] + elds[3];
}

__global__ __launch_bounds__(1024) void k_sum_i64(const int64_t* psum, int count, int64_t* out) {
  __shared__ long long ws[16];
  long long acc = 0;
  for (int i = threadIdx.x; i < count; i += 1024) acc += psum[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < 16; ++w) t += ws[w];
    *out = t;
  }
}

hipError_t launch_compact_changed(const uint8_t* chg, const int32_t* outdeg, int32_t n, int32_t* list,
                                  FrontCounters* fc, int32_t* blk_scratch, int64_t* psum, hipStream_t st) {
  if (n == 0) return launch_fill_u32((uint32_t*)fc, sizeof(FrontCounters) / 4, 0u, st);
  const int nblk = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_chg_count, dim3(nblk), dim3(kBlock), 0, st, chg, n, blk_scratch, fc);
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, st, blk_scratch, nblk, &fc->count);
  hipLaunchKernelGGL(k_chg_scatter, dim3(nblk), dim3(kBlock), 0, st, chg, outdeg, n, blk_scratch, list, psum);
  hipLaunchKernelGGL(k_sum_i64, dim3(1), dim3(1024), 0, st, psum, nblk, &fc->outdeg_sum);
  return hipGetLastError();
}

// ---- sparse push -----------------------------------------------------------
// Append the block's threads whose pred is set to list (one atomic per block).
__device__ __forceinline__ void block_append(bool pred, int32_t val, int32_t* list, int32_t* counter, int* ilds,
                                             int* base_lds) {
  int tot;
  const int r = block_rank(pred, ilds, tot);
  if (tot == 0) return;  // uniform: every thread sees the same total
  if (threadIdx.x == 0) *base_lds = atomicAdd(counter, tot);
  __syncthreads();
  const int base = *base_lds;
  if (pred) list[base + r] = val;
  __syncthreads();
}

// Frontier vertices: out-degree for the edge-balanced push, and the next
// buffer catches up with the vertex's current value.
__global__ void k_front_prep(Sweep s, const int32_t* front, int32_t nfront, const int32_t* orow, int32_t* fdeg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nfront) {
    const int v = front[i];
    fdeg[i] = orow[v + 1] - orow[v];
    atomicMin(&s.x_next[v], s.x_in[v]);
  }
}

// Frontiers up to this size are prepared and scanned by one 1024-thread
// block (one launch instead of four).
constexpr int kFrontOneBlock = 16384;

// One-block form of the push preparation: clears the counters, writes the
// frontier out-degrees to fscan, lets the next buffer catch up with each
// frontier vertex's current value, and scans fscan in place (fscan[nfront] =
// total).
__global__ __launch_bounds__(1024) void k_front_prep_scan(Sweep s, const int32_t* front, int32_t nfront,
                                                          const int32_t* orow, int32_t* fscan, FrontCounters* fc) {
  if (threadIdx.x == 0) {
    fc->count = 0;
    fc->touched = 0;
    fc->outdeg_sum = 0;
  }
  for (int i = threadIdx.x; i < nfront; i += 1024) {
    const int v = front[i];
    fscan[i] = orow[v + 1] - orow[v];
    atomicMin(&s.x_next[v], s.x_in[v]);
  }
  __syncthreads();
  block1024_exclusive_scan(fscan, nfront, fscan + nfront);
}

constexpr int kPushEdgesPerBlock = 1024;

// Edge-balanced push: block b relaxes flattened out-edges
// [b * kPushEdgesPerBlock, ...) of the whole frontier (fscan: exclusive scan
// of the frontier out-degrees, fscan[nfront] = total).
template <int APP>
__global__ __launch_bounds__(kBlock) void k_push(Sweep s, const int32_t* front, int32_t nfront, const int32_t* fscan,
                                                 const int32_t* orow, const int32_t* oedge, const int32_t* odst,
                                                 const uint32_t* bits, uint32_t* stamp, uint32_t epoch,
                                                 int32_t* touched, FrontCounters* fc) {
  __shared__ int ilds[4];
  __shared__ int base_lds;
  const int total = fscan[nfront];
  for (int64_t b0 = (int64_t)blockIdx.x * kPushEdgesPerBlock; b0 < total;
       b0 += (int64_t)gridDim.x * kPushEdgesPerBlock) {
#pragma unroll
    for (int j = 0; j < kPushEdgesPerBlock / kBlock; ++j) {
      const int64_t k = b0 + j * kBlock + threadIdx.x;
      bool newly = false;
      int u = 0;
      if (k < total) {
        int a = 0, hi = nfront - 1;  // last frontier entry whose first edge <= k
        while (a < hi) {
          const int mid = (a + hi + 1) >> 1;
          if (fscan[mid] <= k) a = mid;
          else hi = mid - 1;
        }
        const int v = front[a];
        const int pos = orow[v] + (int)(k - fscan[a]);
        const int e = oedge[pos];
        u = odst[pos];
        const bool act = bits == nullptr || ((bits[e >> 5] >> (e & 31)) & 1u);
        if (act) {
          const uint32_t xs = s.x_in[v];
          uint32_t cand;
          if constexpr (APP == kSSSP) cand = xs == kInf ? kInf : xs + (s.edges[e] >> 24);
          else cand = xs;
          if (cand != kInf) {
            const uint32_t old = atomicMin(&s.x_next[u], cand);
            if (cand < old) newly = atomicExch(&stamp[u], epoch) != epoch;
          }
        }
      }
      block_append(newly, u, touched, &fc->touched, ilds, &base_lds);
    }
  }
}

// Touched vertices whose value dropped below the previous iteration's form
// the next frontier; per-block out-degree sums go to psum[block].
__global__ __launch_bounds__(kBlock) void k_push_finalize(Sweep s, const int32_t* touched, int32_t* next,
                                                          FrontCounters* fc, int64_t* psum) {
  __shared__ int ilds[4];
  __shared__ int base_lds;
  __shared__ long long elds[4];
  const int nt = fc->touched;
  long long dsum = 0;
  for (int base = blockIdx.x * kBlock; base < nt; base += gridDim.x * kBlock) {
    const int t = base + (int)threadIdx.x;
    bool c = false;
    int u = 0;
    if (t < nt) {
      u = touched[t];
      c = s.x_next[u] < s.x_in[u];
      if (c) dsum += s.outdeg[u];
    }
    block_append(c, u, next, &fc->count, ilds, &base_lds);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dsum += __shfl_xor(dsum, o, 64);
  if ((threadIdx.x & 63) == 0) elds[threadIdx.x >> 6] = dsum;
  __syncthreads();
  if (threadIdx.x == 0) psum[blockIdx.x] = elds[0] + elds[1] + elds[2] + elds[3];
}

constexpr int kFinalizeBlocks = 1024;

// ACTIVE out-degree: odeg[col[e]] += 1 for every edge whose flag is set
// (odeg cleared beforehand).
__global__ void k_odeg_act(const int32_t* col, int64_t m, const uint32_t* bits, int32_t* odeg) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    if ((bits[e >> 5] >> (e & 31)) & 1u) atomicAdd(&odeg[col[e]], 1);
}

// Contributions from binary32 values: c[v] = x[v] / deg[v], or x[v] when deg[v] = 0.
__global__ void k_recontrib(const float* x, const int32_t* deg, int32_t n, float* c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    const int d = deg[v];
    c[v] = d > 0 ? (float)((double)x[v] / (double)d) : x[v];
  }
}

hipError_t launch_active_degree(const int32_t* col, int64_t m, const uint32_t* bits, int32_t n, int32_t* odeg,
                                hipStream_t st) {
  hipError_t e = launch_fill_u32((uint32_t*)odeg, n, 0u, st);
  if (e != hipSuccess || m == 0) return e;
  const int64_t blocks = (m + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_odeg_act, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(kBlock), 0, st, col, m,
                     bits, odeg);
  return hipGetLastError();
}

hipError_t launch_recontrib(const float* x, const int32_t* deg, int32_t n, float* c, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_recontrib, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, x, deg, n, c);
  return hipGetLastError();
}

__global__ void k_vs_deg(const int32_t* front, int32_t nfront, const int32_t* orow, int32_t* fdeg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nfront) {
    const int v = front[i];
    fdeg[i] = orow[v + 1] - orow[v];
  }
}

__global__ __launch_bounds__(kBlock) void k_vs_mark(const int32_t* front, int32_t nfront, const int32_t* fscan,
                                                    const int32_t* orow, const int32_t* oedge, const int32_t* odst,
                                                    const uint32_t* bits, uint8_t* dirty) {
  const int64_t total = fscan[nfront];
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < total; k += (int64_t)gridDim.x * kBlock) {
    int a = 0, hi = nfront - 1;  // last list entry whose first out-edge <= k
    while (a < hi) {
      const int mid = (a + hi + 1) >> 1;
      if (fscan[mid] <= k) a = mid;
      else hi = mid - 1;
    }
    const int v = front[a];
    const int pos = orow[v] + (int)(k - fscan[a]);
    const int e = oedge[pos];
    if ((bits[e >> 5] >> (e & 31)) & 1u) dirty[odst[pos]] = 1;
  }
}

hipError_t launch_vs_mark(const int32_t* front, int32_t nfront, int64_t front_outdeg, const int32_t* orow,
                          const int32_t* oedge, const int32_t* odst, const uint32_t* bits, int32_t* fdeg,
                          int32_t* fscan, int32_t* scan_scratch, uint8_t* dirty, hipStream_t st) {
  if (nfront <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vs_deg, dim3((nfront + kBlock - 1) / kBlock), dim3(kBlock), 0, st, front, nfront, orow, fdeg);
  const hipError_t e = launch_scan(fdeg, fscan, nfront, fscan + nfront, scan_scratch, st);
  if (e != hipSuccess) return e;
  if (front_outdeg <= 0) return hipGetLastError();
  const int64_t blocks = (front_outdeg + kBlock - 1) / kBlock;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(k_vs_mark, dim3(grid), dim3(kBlock), 0, st, front, nfront, fscan, orow, oedge, odst, bits, dirty);
  return hipGetLastError();
}

hipError_t launch_push(int app, const Sweep& s, const int32_t* front, int32_t nfront, int64_t front_outdeg,
                       const int32_t* orow, const int32_t* oedge, const int32_t* odst, const uint32_t* bits,
                       uint32_t* stamp, uint32_t epoch, int32_t* touched, int32_t* next, FrontCounters* fc,
                       int32_t* fdeg, int32_t* fscan, int32_t* scan_scratch, int64_t* psum, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (nfront == 0) return launch_fill_u32((uint32_t*)fc, sizeof(FrontCounters) / 4, 0u, st);
  if (nfront <= kFrontOneBlock) {
    hipLaunchKernelGGL(k_front_prep_scan, dim3(1), dim3(1024), 0, st, s, front, nfront, orow, fscan, fc);
  } else {
    e = launch_fill_u32((uint32_t*)fc, sizeof(FrontCounters) / 4, 0u, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_front_prep, dim3((nfront + kBlock - 1) / kBlock), dim3(kBlock), 0, st, s, front, nfront,
                       orow, fdeg);
    e = launch_scan(fdeg, fscan, nfront, fscan + nfront, scan_scratch, st);
    if (e != hipSuccess) return e;
  }
  const int g = grid_for(front_outdeg > 0 ? front_outdeg : 1, kPushEdgesPerBlock, 1 << 20);
  if (app == kSSSP)
    hipLaunchKernelGGL((k_push<kSSSP>), dim3(g), dim3(kBlock), 0, st, s, front, nfront, fscan, orow, oedge, odst,
                       bits, stamp, epoch, touched, fc);
  else
    hipLaunchKernelGGL((k_push<kCC>), dim3(g), dim3(kBlock), 0, st, s, front, nfront, fscan, orow, oedge, odst,
                       bits, stamp, epoch, touched, fc);
  // at most one touched vertex per pushed edge: a frontier of few out-edges
  // is finalized by one block, which writes the out-degree sum itself
  const int64_t fin = (front_outdeg + kBlock - 1) / kBlock;
  const int gf = (int)std::max<int64_t>(1, std::min<int64_t>(kFinalizeBlocks, fin));
  if (gf == 1) {
    hipLaunchKernelGGL(k_push_finalize, dim3(1), dim3(kBlock), 0, st, s, touched, next, fc,
                       (int64_t*)&fc->outdeg_sum);
  } else {
    hipLaunchKernelGGL(k_push_finalize, dim3(gf), dim3(kBlock), 0, st, s, touched, next, fc, psum);
    hipLaunchKernelGGL(k_sum_i64, dim3(1), dim3(1024), 0, st, psum, gf, &fc->outdeg_sum);
  }
  return hipGetLastError();
}

}  // namespace ggk


// ===========================================================================
// Independent parts: a block-diagonal union of graphs run as one graph
// ===========================================================================
namespace ggk {

__global__ void k_part_of(int32_t n, int32_t np, const int32_t* part_start, int32_t* part_of) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = np - 1;  // last part whose start <= u
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (part_start[mid] <= u) lo = mid;
      else hi = mid - 1;
    }
    part_of[u] = lo;
  }
}

__global__ void k_part_check(const int32_t* rowptr, const int32_t* col, int32_t n, int64_t m, const int32_t* part_of,
                             int32_t* bad) {
  int f = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rowptr[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    if (part_of[lo] != part_of[col[e]]) f = 1;
  }
  if (f) atomicOr(bad, 1);
}

hipError_t launch_parts_setup(const int32_t* rowptr, const int32_t* col, int32_t n, int64_t m, int32_t np,
                              const int32_t* part_start, int32_t* part_of, int32_t* bad, hipStream_t st) {
  hipError_t e = launch_fill_u32((uint32_t*)bad, 1, 0u, st);
  if (e != hipSuccess || n == 0) return e;
  hipLaunchKernelGGL(k_part_of, dim3(grid_for(n, kBlock * 4, 1 << 16)), dim3(kBlock), 0, st, n, np, part_start,
                     part_of);
  if (m > 0)
    hipLaunchKernelGGL(k_part_check, dim3(grid_for(m, kBlock * 4, 1 << 16)), dim3(kBlock), 0, st, rowptr, col, n, m,
                       part_of, bad);
  return hipGetLastError();
}

__global__ void k_part_dranges(const int32_t* dlist, int32_t ndang, int32_t np, const int32_t* part_start,
                               int32_t* dstart) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > np) return;
  const int key = part_start[p];
  int lo = 0, hi = ndang;  // first dangling vertex >= key
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (dlist[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  dstart[p] = lo;
}

hipError_t launch_parts_dangling_ranges(const int32_t* dlist, int32_t ndang, int32_t np, const int32_t* part_start,
                                        int32_t* dstart, hipStream_t st) {
  hipLaunchKernelGGL(k_part_dranges, dim3((np + 1 + kBlock - 1) / kBlock), dim3(kBlock), 0, st, dlist, ndang, np,
                     part_start, dstart);
  return hipGetLastError();
}

// Dangling mass of every part: kPartDangBlocks blocks per part take
// interleaved slices of its dangling list (4 loads in flight per thread),
// then one thread per part adds its partials in block order.
__global__ __launch_bounds__(kBlock) void k_part_dsum(const float* c, const int32_t* dlist, const int32_t* dstart,
                                                      double* partial) {
  __shared__ double lds[4];
  const int p = blockIdx.x / kPartDangBlocks, k = blockIdx.x % kPartDangBlocks;
  const int hi = dstart[p + 1];
  constexpr int kStride = kPartDangBlocks * kBlock;
  double acc = 0.0;
  int i = dstart[p] + k * kBlock + (int)threadIdx.x;
  for (; i + 3 * kStride < hi; i += 4 * kStride) {
    const int a0 = dlist[i], a1 = dlist[i + kStride], a2 = dlist[i + 2 * kStride], a3 = dlist[i + 3 * kStride];
    const float v0 = c[a0], v1 = c[a1], v2 = c[a2], v3 = c[a3];
    acc += (double)v0;
    acc += (double)v1;
    acc += (double)v2;
    acc += (double)v3;
  }
  for (; i < hi; i += kStride) acc += (double)c[dlist[i]];
  acc = block_reduce<kPR>(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ void k_part_dsum_final(const double* partial, int32_t np, double* part_dang) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) {
    double acc = 0.0;
    for (int k = 0; k < kPartDangBlocks; ++k) acc += partial[(int64_t)p * kPartDangBlocks + k];
    part_dang[p] = acc;
  }
}

hipError_t launch_parts_dangling_sum(const float* c, const int32_t* dlist, int32_t np, const int32_t* dstart,
                                     double* part_dang, double* partial, hipStream_t st) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_part_dsum, dim3(np * kPartDangBlocks), dim3(kBlock), 0, st, c, dlist, dstart, partial);
  hipLaunchKernelGGL(k_part_dsum_final, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, st, partial, np,
                     part_dang);
  return hipGetLastError();
}

// One thread per bitmap word; each edge finds its part and draws from the
// Philox block of its part-local index.
__global__ __launch_bounds__(kBlock) void k_sample_bits_parts(int64_t m, uint64_t seed, uint64_t epoch, uint64_t keep,
                                                              int32_t np, const int32_t* part_e0, uint32_t* bits) {
  const int64_t nw = (m + 31) >> 5;
  for (int64_t w = blockIdx.x * (int64_t)kBlock + threadIdx.x; w < nw; w += (int64_t)gridDim.x * kBlock) {
    uint32_t word = 0;
    int64_t cached_block = -1;
    int cached_part = -1;
    uint64_t o[4] = {0, 0, 0, 0};
    for (int h = 0; h < 32; ++h) {
      const int64_t e = w * 32 + h;
      if (e >= m) break;
      int lo = 0, hi = np - 1;  // last part whose first edge <= e
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (part_e0[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      const int64_t local = e - part_e0[lo];
      if (lo != cached_part || (local >> 3) != cached_block) {
        philox4x64_10((uint64_t)(local >> 3), epoch, 0, 0, seed + (uint64_t)lo, 0, o);
        cached_part = lo;
        cached_block = local >> 3;
      }
      const int j = (int)(local & 7);
      const uint64_t w64 = o[j >> 1];
      const uint32_t d = (j & 1) ? (uint32_t)(w64 >> 32) : (uint32_t)w64;
      if ((uint64_t)d < keep) word |= 1u << h;
    }
    bits[w] = word;
  }
}

hipError_t launch_sample_bits_parts(int64_t m, uint64_t seed, uint64_t epoch, uint64_t keep, int32_t np,
                                    const int32_t* part_e0, uint32_t* bits, hipStream_t st) {
  const int64_t nw = (m + 31) >> 5;
  if (nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_bits_parts, dim3(grid_for(nw, kBlock, 1 << 16)), dim3(kBlock), 0, st, m, seed, epoch,
                     keep, np, part_e0, bits);
  return hipGetLastError();
}

__global__ void k_set_sources(const int32_t* src, int32_t count, uint32_t* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) x[src[i]] = 0u;
}

hipError_t launch_set_sources(const int32_t* src, int32_t count, uint32_t* x, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_sources, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, st, src, count, x);
  return hipGetLastError();
}

}  // namespace ggk

namespace ggk {
__global__ void k_gather_i32(const int32_t* src, const int32_t* idx, int32_t count, int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = src[idx[i]];
}
hipError_t launch_gather_i32(const int32_t* src, const int32_t* idx, int32_t count, int32_t* out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_i32, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, st, src, idx, count, out);
  return hipGetLastError();
}
}  // namespace ggk

// ===========================================================================
// Superstep for short rows (degree <= small_max) as flattened batches: a block
// takes kBlock consecutive vertices, gathers every edge of those rows into LDS
// (all loads of a window in flight together), then the owner thread of each
// row walks its values in CSR order: running sum / minimum, edge influence and
// GG-EStatus [Alg. 2], flag bits, packed active edges, apply. Rows up to
// wave_max use one wavefront each with shuffle scans; longer rows the chunked
// hub path (k_hub_totals, super_hub_chunk, k_hub_pack).
// ===========================================================================
namespace ggk {

// Seven waves per SIMD: the hub section otherwise holds the PR instance at six
// (SSSP and CC reach eight).
template <int APP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_super_flat(Sweep s, int nchunks,
                                                                                              int gw) {
  using R = Tr<APP>;
  using T = typename R::T;
  using V = typename GV<APP>::V;
  __shared__ T lds[4];
  __shared__ int ilds[4];
  __shared__ V s_val[kFlatWin];
  __shared__ uint32_t s_ev[kFlatWin];
  __shared__ int s_lo[kBlock];
  __shared__ int s_scan[kBlock + 1];
  int nchanged = 0;
  if ((int)blockIdx.x < nchunks) {
    if (s.hub_sync) super_hub_chunk_1p<APP>(s, nchunks, nchanged, lds, ilds);
    else super_hub_chunk<APP>(s, s.chunk_order ? s.chunk_order[blockIdx.x] : (int)blockIdx.x, nchanged, lds, ilds);
    flush_changed<APP>(s, nchanged, ilds);
    return;
  }
  if ((int)blockIdx.x < nchunks + gw) {
    // wavefront-bin rows: one wavefront per row, shuffle scans
    super_team_rows<APP, 64>(s, s.list + s.n_small, s.n_wave, (int)blockIdx.x - nchunks, gw, nchanged);
    flush_changed<APP>(s, nchanged, ilds);
    return;
  }
  const int tid = threadIdx.x;
  // natural order: every vertex, the short rows taken; listed: the small-bin
  // rows list[0, n_small)
  const int u0 = ((int)blockIdx.x - nchunks - gw) * kBlock;
  const int P = min(kBlock, (s.flat_list ? s.n_small : s.n) - u0);
  int u = 0, lo = 0, len = 0;
  bool mine = false;
  uint32_t word = 0;  // the apply's own read, issued before the gather
  double rtot = -1.0;  // TOTAL influence: the row sum
  if (tid < P) {
    u = s.flat_list ? s.list[u0 + tid] : u0 + tid;
    lo = s.rowptr[u];
    len = s.rowptr[u + 1] - lo;
    word = apply_word<APP>(s, u);
    mine = len <= s.small_max;
    if (!mine) len = 0;
    if (kSumApp<APP> && s.row_total && mine) rtot = s.row_total[u];
  }
  // exclusive scan of the row lengths
  int x = len;
  const int lane = __lane_id(), wid = tid >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) ilds[wid] = x;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wid; ++w) before += ilds[w];
  const int total = ilds[0] + ilds[1] + ilds[2] + ilds[3];
  s_scan[tid] = before + x - len;
  s_lo[tid] = lo;
  __syncthreads();
  // owner state, carried across windows
  const int mine0 = s_scan[tid], mine1 = s_scan[tid] + len;
  double Psum = 0.0;            // PR: running sum of the row's contributions
  uint32_t run = kInf;          // SSSP/CC: running minimum
  if constexpr (!kSumApp<APP>) {
    if (s.push_infl && mine) run = s.x_in[u];  // push order: from the row's own value
  }
  int cnt = 0;                  // active edges written
  int bw = -1;                  // current flag word
  uint32_t bacc = 0;            // new bits of that word
  int ow = -1;                  // cached old-flag word index
  uint32_t oword = 0;
  for (int base = 0; base < total; base += kFlatWin) {
    const int lim = min(kFlatWin, total - base);
#pragma unroll
    for (int j = 0; j < kFlatWin / kBlock; ++j) {
      const int k = j * kBlock + tid;
      if (k < lim) {
        const int kk = base + k;
        int a = 0, b = P - 1;
        while (a < b) {
          const int mid = (a + b + 1) >> 1;
          if (s_scan[mid] <= kk) a = mid;
          else b = mid - 1;
        }
        const int e = s_lo[a] + (kk - s_scan[a]);
        const uint32_t ev = ld_stream(s.edges + e);
        s_ev[k] = ev;
        s_val[k] = GV<APP>::get(s, ev);
      }
    }
    __syncthreads();
    const int a0 = max(mine0, base), a1 = min(mine1, base + lim);
    for (int k = a0; k < a1; ++k) {
      const int e = lo + (k - mine0);
      const V val = s_val[k - base];
      uint32_t oldf = 0;
      if (s.old_bits && (APP == kSSSP || s.mask_union)) {
        if ((e >> 5) != ow) {
          ow = e >> 5;
          oword = s.old_bits[ow];
        }
        oldf = (oword >> (e & 31)) & 1u;
      }
      bool flag;
      if constexpr (kSumApp<APP>) {
        const double c = (double)val;
        Psum += c;
        flag = sum_flag<APP>(s, true, c, rtot >= 0.0 ? rtot : Psum, oldf);
      } else if constexpr (APP == kSSSP) {
        const uint32_t cand = val;  // INF iff the source is unreached
        if (cand == kInf) {
          flag = oldf != 0u;  // not assessable: keeps its flag
        } else {
          const uint32_t nw = min(run, cand);
          const bool dec = (run == kInf) || ((((uint64_t)(run - nw)) << 16) > s.theta_q * (uint64_t)run);
          flag = dec || (s.mask_union && oldf);
          run = nw;
        }
      } else {
        flag = (val < run) || (s.mask_union && oldf);
        run = min(run, (uint32_t)val);
      }
      if ((e >> 5) != bw) {
        if (bacc) atomicOr(&s.new_bits[bw], bacc);
        bw = e >> 5;
        bacc = 0;
      }
      if (flag) {
        bacc |= 1u << (e & 31);
        s.act_edges[lo + cnt] = s_ev[k - base];
        ++cnt;
      }
    }
    __syncthreads();
  }
  if (mine) {
    if (bacc) atomicOr(&s.new_bits[bw], bacc);
    T acc;
    if constexpr (kSumApp<APP>) acc = Psum;
    else acc = run;
    apply_with<APP>(s, u, acc, word, nchanged);
    s.act_cnt[u] = cnt;
  }
  flush_changed<APP>(s, nchanged, ilds);
}

// With s.hub_sync (and hub_chunk <= kHubPre * kBlock) the hub chunks run in a
// single pass inside k_super_flat; otherwise chunk totals come from
// k_hub_totals before it and k_hub_pack writes the hub rows' active edges
// after it. hub_sync[1 .. 2 + 3 * nchunks) (ticket, chunk totals and counts)
// is cleared here.
template <int APP>
static hipError_t super_flat_t(Sweep s, int nchunks, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const bool one_pass = s.hub_sync && nchunks > 0 && s.hub_chunk <= kHubPre * kBlock;
  if (!one_pass) s.hub_sync = nullptr;
  if (one_pass) {
    const hipError_t e = launch_fill_u32(s.hub_sync + 1, 3 * (int64_t)nchunks + 1, 0u, st);
    if (e != hipSuccess) return e;
  } else if (nchunks > 0) {
    hipLaunchKernelGGL((k_hub_totals<APP>), dim3(nchunks), dim3(kBlock), 0, st, s);
  }
  const int gs = ((s.flat_list ? s.n_small : s.n) + kBlock - 1) / kBlock;
  const int gw = s.n_wave > 0 ? grid_for(s.n_wave, kBlock / 64, kTeamBlockCap) : 0;
  const int total = nchunks + gw + gs;
  if (ev0) (void)hipEventRecord(ev0, st);
  if (total > 0) hipLaunchKernelGGL((k_super_flat<APP>), dim3(total), dim3(kBlock), 0, st, s, nchunks, gw);
  if (ev1) (void)hipEventRecord(ev1, st);
  if (nchunks > 0 && !one_pass)
    hipLaunchKernelGGL(k_hub_pack, dim3(nchunks), dim3(kBlock), 0, st, s, (const uint32_t*)s.new_bits);
  return hipGetLastError();
}

// Source segment of the first edge of every hub chunk (rows are sorted by
// source, so a chunk of a long row spans a narrow source range). The host
// orders the chunks by it, stably, for the superstep.
__global__ void k_chunk_seg(Sweep s, const int32_t* col, int32_t z, int32_t nseg, int32_t* seg_of) {
  for (int ch = blockIdx.x * blockDim.x + threadIdx.x; ch < s.n_chunks; ch += gridDim.x * blockDim.x) {
    const int h = find_hub(s.hub_start, s.n_hub, ch);
    const int u = s.list[s.n_small + s.n_wave + h];
    const int j = ch - s.hub_start[h];
    const int64_t e = (int64_t)s.rowptr[u] + (int64_t)j * s.hub_chunk;
    seg_of[ch] = min(col[e] / z, nseg - 1);
  }
}

hipError_t launch_chunk_seg(const Sweep& s, const int32_t* col, int32_t z, int32_t nseg, int32_t* seg_of,
                            hipStream_t st) {
  if (s.n_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_chunk_seg, dim3(grid_for(s.n_chunks, kBlock, 4096)), dim3(kBlock), 0, st, s, col, z, nseg,
                     seg_of);
  return hipGetLastError();
}

hipError_t launch_superstep_flat(int app, const Sweep& s, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int nchunks = s.n_hub > 0 ? s.n_chunks : 0;
  switch (app) {
    case kPR: return super_flat_t<kPR>(s, nchunks, st, ev0, ev1);
    case kPPR: return super_flat_t<kPPR>(s, nchunks, st, ev0, ev1);
    case kBP: return super_flat_t<kBP>(s, nchunks, st, ev0, ev1);
    case kSSSP: return super_flat_t<kSSSP>(s, nchunks, st, ev0, ev1);
    case kCC: return super_flat_t<kCC>(s, nchunks, st, ev0, ev1);
  }
  return hipErrorInvalidValue;
}

}  // namespace ggk

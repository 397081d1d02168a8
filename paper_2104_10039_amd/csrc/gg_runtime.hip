// Host runtime and C ABI of the GraphGuess sweep library (see include/gg.h).
//
// A graph handle owns the device copy (or borrows the caller's device
// arrays) of the in-CSR, its out-degrees, the dangling-vertex list, the
// degree binning of the full rows, and a workspace reused by every run on
// the graph: double-buffered vertex values, the edge-flag bitmaps, the
// active edge array with its per-row counts and binning, and scratch for
// hub partial results.
//
// A run follows the schedule of its correction scheme [Sec. 3.4, Sec. 5.2]:
// iteration i (1-based) is accurate for EXACT always, for SMS from
// i = alpha+1 on, for GG when i is a multiple of alpha+1; SP never. Each
// accurate GG iteration is a superstep that re-selects the active edges.
// LEARNED keeps GG's correction steps but lets a network pick the rows they
// correct (a partial superstep), with GG's full superstep as fallback.
// Updates are synchronous: iteration i reads the values of iteration i-1.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gg.h"
#include "gg_internal.h"

using namespace ggk;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define GG_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      if (e_ == hipErrorOutOfMemory) return fail(GG_E_NOMEM, std::string(#call) + ": out of device memory"); \
      return fail(GG_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));            \
    }                                                                                         \
  } while (0)

#define GG_TRY(x)            \
  do {                       \
    int r_ = (x);            \
    if (r_ != GG_OK) return r_; \
  } while (0)

// Device memory of the library's objects comes from the caller's allocator
// (gg_set_allocator) or, when none is set, from hipMalloc / hipFree. The
// allocator can change only while no graph, network or trace exists, so
// every block is freed by the allocator that made it. Around the caller's
// functions the device is synchronized, as hipMalloc / hipFree do: a block
// handed back is idle on every stream, and a block received carries no
// work still pending from its previous owner.
gg_alloc_fn g_alloc_fn = nullptr;
gg_free_fn g_free_fn = nullptr;
void* g_alloc_ctx = nullptr;
std::atomic<int64_t> g_live_objects{0};

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (g_alloc_fn) {
    void* p = g_alloc_fn(bytes, g_alloc_ctx);
    if (p) (void)hipDeviceSynchronize();
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  if (g_free_fn) {
    (void)hipDeviceSynchronize();
    g_free_fn(p, g_alloc_ctx);
  } else {
    (void)hipFree(p);
  }
}

// Allocates count elements into *p. A block already held there (left by an
// earlier set-up step that failed part way) is freed first, so a retry
// leaks nothing.
template <typename T>
int dalloc(T** p, size_t count) {
  if (*p) dev_free((void*)*p);
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = dev_alloc(count * sizeof(T));
  if (!q) return fail(GG_E_NOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
  *p = (T*)q;
  return GG_OK;
}

template <typename T>
void dfree(T*& p) {
  dev_free((void*)p);
  p = nullptr;
}

// Member of every graph, network and trace: keeps the count of live objects.
struct LiveObject {
  LiveObject() { g_live_objects.fetch_add(1); }
  ~LiveObject() { g_live_objects.fetch_sub(1); }
  LiveObject(const LiveObject&) = delete;
  LiveObject& operator=(const LiveObject&) = delete;
};

}  // namespace

struct gg_graph {
  LiveObject live;
  int32_t n = 0;
  int64_t m = 0;
  hipStream_t stream = nullptr;
  void* pin = nullptr;  // kPinBytes of pinned host memory for small readbacks
  uint32_t* pin_dev = nullptr;  // its device address when mapped and coherent (posted readbacks)
  uint32_t pin_seq = 0;
  bool owns_csr = false;
  int32_t* rowptr = nullptr;
  int32_t* col = nullptr;
  int32_t* weight = nullptr;   // owned copy (host input) or borrowed
  uint32_t* wedges = nullptr;  // (weight << 24) | source, when weights exist
  int32_t* outdeg = nullptr;
  int32_t* dang = nullptr;
  int32_t n_dang = 0;
  int32_t* i32_scratch = nullptr;  // small device scalars: [0] dangling count, [1] validate flags
  int64_t* blk_scratch = nullptr;  // block-level scan scratch (8-byte units)
  gg_tuning tune{32, 4, 1024, 2048, 1, 0, 1, 16};
  int device = 0;  // the device current at load
  int32_t hub_spin = kHubSpinLimit;  // gg_graph_set_wait_limit
  bool rows_sorted = true;  // every row lists its sources in ascending order (else no segmentation)
  // frontier (SSSP / CC): out-CSR structure and lists, built on first use
  bool out_built = false;
  int32_t* orow = nullptr;
  int32_t* oedge = nullptr;
  int32_t* odst = nullptr;
  int32_t* osrc = nullptr;  // source of every out-CSR entry (for updates)
  // buffers of the arrays an update replaced, reused as the next update's
  // destinations when large enough; bytes is what the replaced graph needed
  // (a lower bound of the allocation)
  struct Spare {
    void* p = nullptr;
    size_t bytes = 0;
  } spare[11];
  uint8_t* chg = nullptr;
  uint32_t* stamp = nullptr;
  uint32_t epoch = 0;
  int32_t* flist[2] = {nullptr, nullptr};
  int32_t* touched = nullptr;
  FrontCounters* fc = nullptr;
  int32_t* fdeg = nullptr;   // n
  int32_t* fscan = nullptr;  // n + 1
  int64_t* psum = nullptr;   // max(ceil(n / kBlock), 1024)
  // independent parts (gg_graph_set_parts)
  int32_t n_parts = 0;
  int32_t* part_start = nullptr;  // np+1
  int32_t* part_of = nullptr;     // n
  int32_t* part_e0 = nullptr;     // np+1: first edge of each part
  int32_t* part_dstart = nullptr; // np+1: range of each part in the dangling list
  int32_t* part_src = nullptr;    // np or null
  double* part_dang = nullptr;    // np, then np * kPartDangBlocks partials
  // multi-query batch workspace
  struct Batch {
    int64_t val_cap = 0;  // elements of each value buffer
    uint32_t* buf[3] = {nullptr, nullptr, nullptr};  // 4-byte values
    int64_t part_cap = 0;  // elements (chunks * qp) of the partial array
    double* part = nullptr;
    int32_t qp_cap = 0;
    double* dpart = nullptr;  // kBDangChunks * qp dangling partials
    double* dang = nullptr;   // qp
    int32_t* src = nullptr;   // qp
    int32_t* ctr = nullptr;   // [0] changed, [1] done, [2] iterations
    hipStream_t cs = nullptr; // private capture stream (default priority)
    hipEvent_t ea = nullptr, eb = nullptr, t0 = nullptr, t1 = nullptr;
  } batch;
  // source segmentation of long rows (plain gathers)
  int32_t seg_s = 8, seg_z = 1;
  int32_t* seg_off_full = nullptr;
  int32_t* seg_off_act = nullptr;
  double* seg_part = nullptr;  // 8-byte partials (double for PR, uint32 in the low half otherwise)
  int64_t seg_cap_off = 0;   // int32 entries of each offset array
  int64_t seg_cap_part = 0;  // 8-byte entries of the partial array
  Bins full;         // binning of the full rows by in-degree
  bool full_valid = false;
  int32_t* chunk_order = nullptr;    // hub chunks of `full` in source-segment order
  int32_t* chunk_scratch = nullptr;
  int32_t chunk_cap = 0, chunk_order_n = 0;
  // learned correction and traces (allocated on first use)
  bool lws = false;
  uint16_t* feat = nullptr;        // [n][8] bfloat16 features
  uint8_t* sel = nullptr;          // n: selected rows of the last correction step
  float* logits = nullptr;         // n
  uint8_t* labels = nullptr;       // n: drift labels of the last traced / audited superstep
  uint32_t* shadow = nullptr;      // n: approximate update of that superstep
  int32_t* sel_count = nullptr;    // 4: |S| (int32), pad, in-edges of S (uint64 at +2)
  unsigned long long* audit = nullptr;  // [0] drifted vertices, [1] of which selected, [2] active edges of S
  Bins selb;                       // binning of the selected rows (full rows)
  // workspace (allocated on first run)
  bool ws = false;
  float* c[2] = {nullptr, nullptr};
  float* xout = nullptr;
  uint32_t* xu[2] = {nullptr, nullptr};
  uint32_t* bits[2] = {nullptr, nullptr};
  uint32_t* act_edges = nullptr;
  int32_t* act_cnt = nullptr;
  Bins act;
  double* part_f = nullptr;
  uint32_t* part_u = nullptr;
  int32_t* part_cnt = nullptr;
  uint32_t* hub_sync = nullptr;  // 3 * part_cap + 2: single-pass hub chunk sync (Sweep::hub_sync)
  int64_t part_cap = 0;
  double* dpartial = nullptr;  // 256 dangling partials + [256] = D
  double* row_sum = nullptr;   // n: row sums for TOTAL influence (first use)
  // GG-VStatus (first use): vertex status, rows to recompute, previous values
  uint8_t* vact = nullptr;     // n (+ padding to whole words)
  uint8_t* vdirty = nullptr;   // n (+ padding)
  float* x_prev = nullptr;     // n
  // ACTIVE out-degree (first use): active out-edges per vertex, and the
  // vertices without one
  int32_t* odeg_act = nullptr;
  int32_t* dang_act = nullptr;
  int32_t n_dang_act = 0;
  float* bp_prior = nullptr;  // n: BP prior log-odds of the current run (first use)
  int32_t* changed = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  gg_run* active_run = nullptr;
  // The captured iteration schedule of the last static whole run (EXACT, SP
  // or SMS of PR/PPR/BP: no host decision depends on device data once the
  // run has begun), replayed while its key and the graph's generation match.
  // gen changes whenever a buffer or binning that the schedule refers to is
  // rebuilt or moved.
  uint64_t gen = 1;
  struct RunGraph {
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = nullptr;  // private stream (default priority)
    hipEvent_t ea = nullptr, eb = nullptr;
    uint64_t gen = 0;
    std::vector<unsigned char> key;
    // host state of the run after the schedule
    int32_t iter = 0;
    int cur = 0;
    bool x_valid = false;
    int64_t edges_total = 0, edges_processed = 0;
  } rg;
  bool capture = false;  // gg_graph_set_capture
  // kernel profiling (gg_graph_set_profiling)
  struct ProfRec {
    int kind, app;
    hipEvent_t e0, e1;
    double bytes;
    int64_t edges;
  };
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
};

struct gg_run {
  gg_graph* g = nullptr;
  gg_app_params p{};
  gg_correction_policy pol{};
  double sigma = 1.0;
  int32_t iter = 0;
  bool done = false;
  int cur = 0;   // value buffer holding iteration `iter`
  int bcur = 0;  // bitmap holding the current flags
  bool x_valid = false;  // PR: xout holds the values of iteration `iter`
  bool write_x_each_step = false;
  int32_t supersteps = 0;
  int64_t edges_total = 0;
  int64_t edges_processed = 0;
  int32_t sparse_iters = 0;
  // frontier state: list flist[fcur] holds the vertices changed by iteration
  // `iter` (front_count < 0: unknown, the next iteration runs dense)
  int fcur = 0;
  int64_t front_count = -1;
  int64_t front_outdeg = 0;
  bool timing = false;
  // learned correction
  int32_t corrections = 0;
  int32_t partials = 0;
  int64_t selected_total = 0;
  int64_t audit_selected = 0;
  bool have_feat = false, have_sel = false, have_labels = false;
  // an exact SSSP/CC run that ended on an iteration that changed nothing
  bool converged = false;
};

struct gg_mlp {
  LiveObject live;
  hipStream_t stream = nullptr;
  ggk::MlpDev d{};
  float* grad = nullptr;  // kMlpParams gradient + loss sum
  float* scratch = nullptr;
  int64_t scratch_cap = 0;
  float* loss = nullptr;  // per-epoch loss sums
  int64_t loss_cap = 0;
  int64_t t = 0;          // Adam steps taken
};

struct gg_trace {
  LiveObject live;
  int64_t cap = 0, size = 0, dropped = 0;
  uint16_t* feat = nullptr;  // [cap][8]
  float* label = nullptr;    // cap
  unsigned long long* pos = nullptr;  // positives recorded
};

namespace {

int64_t max_chunks(const gg_graph* g) {
  const int64_t m = g->m;
  return m / g->tune.hub_chunk + m / ((int64_t)g->tune.wave_max + 1) + 2;
}

// Small device-to-host readback that the host waits for: through the graph's
// pinned buffer when it fits (a direct DMA, no staging copy).
constexpr size_t kPinBytes = 256;
static_assert(sizeof(BinCounts) <= kPinBytes - 4 && sizeof(FrontCounters) <= kPinBytes - 4,
              "the per-iteration readbacks fit the pinned buffer behind its sequence word");

// A posted readback: a one-wavefront kernel, queued after the work it must
// follow, writes the words and then a sequence number into mapped coherent
// host memory, and the host polls that number. This wakes the host as soon
// as the data lands instead of after a copy engine transfer and a stream
// synchronization. A poll that has not seen the number after 20 ms
// synchronizes the stream (which reports any earlier device error) before
// trusting the data.
int readback_posted(gg_graph* g, void* dst, const void* src, size_t bytes) {
  uint32_t seq = ++g->pin_seq;
  if (seq == 0) seq = ++g->pin_seq;
  GG_HIP(launch_post((const uint32_t*)src, (int32_t)(bytes / 4), g->pin_dev, seq, g->stream));
  volatile uint32_t* flag = (volatile uint32_t*)g->pin;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t spins = 1; *flag != seq; ++spins) {
    if ((spins & 4095) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
      GG_HIP(hipStreamSynchronize(g->stream));
      if (*flag != seq) return fail(GG_E_DEVICE, "posted readback not seen after its stream completed");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  std::memcpy(dst, (const char*)g->pin + 4, bytes);
  return GG_OK;
}

int readback(gg_graph* g, void* dst, const void* src, size_t bytes) {
  if (g->pin_dev && bytes <= kPinBytes - 4 && bytes % 4 == 0 && ((uintptr_t)src & 3) == 0)
    return readback_posted(g, dst, src, bytes);
  if (g->pin && bytes <= kPinBytes) {
    GG_HIP(hipMemcpyAsync(g->pin, src, bytes, hipMemcpyDeviceToHost, g->stream));
    GG_HIP(hipStreamSynchronize(g->stream));
    std::memcpy(dst, g->pin, bytes);
  } else {
    GG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, g->stream));
    GG_HIP(hipStreamSynchronize(g->stream));
  }
  return GG_OK;
}

int sync_bins(gg_graph* g, Bins& b) { return readback(g, &b.h, b.dcounts, sizeof(BinCounts)); }

int alloc_bins(Bins& b, int32_t n) {
  GG_TRY(dalloc(&b.list, (size_t)n));
  GG_TRY(dalloc(&b.hub_start, (size_t)n + 1));
  GG_TRY(dalloc(&b.dcounts, 1));
  return GG_OK;
}

void free_bins(Bins& b) {
  dfree(b.list);
  dfree(b.hub_start);
  dfree(b.dcounts);
}

int rebin(gg_graph* g, Bins& b, const int32_t* cnt, const uint8_t* rowsel = nullptr, int selwant = 0,
          bool hub_check = false) {
  const uint32_t* err = hub_check ? g->hub_sync : nullptr;
  GG_HIP(launch_rebin(g->rowptr, cnt, g->n, g->tune.small_max, g->tune.wave_max, g->tune.hub_chunk, b,
                      g->blk_scratch, g->stream, rowsel, selwant, err));
  GG_TRY(sync_bins(g, b));
  if (b.h.hub_err != 0) {
    // a hub chunk of the superstep before this rebin gave up waiting: its
    // results are undefined (its memory writes stayed inside its row)
    b.h.hub_err = 0;
    GG_HIP(launch_fill_u32(g->hub_sync, 1, 0u, g->stream));
    return fail(GG_E_DEVICE, "a superstep hub chunk gave up waiting for its row prefix");
  }
  return GG_OK;
}

int ensure_selb(gg_graph* g) {
  if (!g->selb.list) GG_TRY(alloc_bins(g->selb, g->n));
  return GG_OK;
}

int ensure_learned(gg_graph* g) {
  if (g->lws) return GG_OK;
  const size_t n = (size_t)g->n;
  GG_TRY(dalloc(&g->feat, n * 8));
  GG_TRY(dalloc(&g->sel, n));
  GG_TRY(dalloc(&g->logits, n));
  GG_TRY(dalloc(&g->labels, n));
  GG_TRY(dalloc(&g->shadow, n));
  GG_TRY(dalloc(&g->sel_count, 4));
  GG_TRY(dalloc(&g->audit, 3));
  GG_TRY(alloc_bins(g->selb, g->n));
  g->lws = true;
  return GG_OK;
}

// Segment count (a multiple of the 8 dies) and size for the current tuning.
void seg_geometry(gg_graph* g) {
  const int64_t target = g->tune.seg_vertices > 0 ? g->tune.seg_vertices : (int64_t)(2 << 20) / 4;
  int64_t S = (g->n + target - 1) / target;
  if (S < 1) S = 1;
  S = (S + 7) / 8 * 8;
  g->seg_s = (int32_t)S;
  const int64_t z = ((int64_t)g->n + S - 1) / S;
  g->seg_z = (int32_t)(z < 1 ? 1 : z);
}

// The offset arrays hold (S+1) entries and the partial array S entries per
// long row of the full binning (an active binning never has more long rows).
// Both depend on S as well as on the long-row count.
int ensure_seg(gg_graph* g) {
  const int64_t nl = (int64_t)g->full.h.wave + g->full.h.hub;
  const int64_t rows = nl < 1 ? 1 : nl;
  const int64_t need_off = ((int64_t)g->seg_s + 1) * rows;
  const int64_t need_part = (int64_t)g->seg_s * rows;
  if (g->seg_off_full && g->seg_cap_off >= need_off && g->seg_cap_part >= need_part) return GG_OK;
  g->gen++;
  dfree(g->seg_off_full);
  dfree(g->seg_off_act);
  dfree(g->seg_part);
  g->seg_cap_off = g->seg_cap_part = 0;
  GG_TRY(dalloc(&g->seg_off_full, (size_t)need_off));
  GG_TRY(dalloc(&g->seg_off_act, (size_t)need_off));
  GG_TRY(dalloc(&g->seg_part, (size_t)need_part));
  g->seg_cap_off = need_off;
  g->seg_cap_part = need_part;
  return GG_OK;
}

// Host-side capacity checks before launches that index sized scratch.
int check_seg_capacity(const gg_graph* g, const Bins& b) {
  const int64_t nl = (int64_t)b.h.wave + b.h.hub;
  if (((int64_t)g->seg_s + 1) * nl > g->seg_cap_off || (int64_t)g->seg_s * nl > g->seg_cap_part)
    return fail(GG_E_STATE, "segment arrays smaller than the binning requires");
  return GG_OK;
}

int check_part_capacity(const gg_graph* g, const Bins& b) {
  if ((int64_t)b.h.chunks > g->part_cap) return fail(GG_E_STATE, "hub partial array smaller than the chunk count");
  return GG_OK;
}

void set_seg(const gg_graph* g, Sweep& s, const int32_t* off) {
  s.seg_s = g->seg_s;
  s.seg_z = g->seg_z;
  s.seg_qw = (s.n_wave + kSegRowsPerBlock - 1) / kSegRowsPerBlock;
  s.seg_off = off;
  s.seg_part_f = (double*)g->seg_part;
  s.seg_part_u = (uint32_t*)g->seg_part;
}

// Segment offsets of one binned view (edges: its edge array, cnt: active counts or null).
int seg_offsets(gg_graph* g, const Bins& b, const uint32_t* edges, const int32_t* cnt, uint32_t src_mask,
                int32_t* off) {
  GG_TRY(check_seg_capacity(g, b));
  Sweep s;
  std::memset(&s, 0, sizeof(s));
  s.n = g->n;
  s.rowptr = g->rowptr;
  s.cnt = cnt;
  s.edges = edges;
  s.list = b.list;
  s.n_small = b.h.small;
  s.n_wave = b.h.wave;
  s.n_hub = b.h.hub;
  s.seg_s = g->seg_s;
  s.seg_z = g->seg_z;
  GG_HIP(launch_seg_offsets(s, src_mask, off, g->stream));
  return GG_OK;
}

// Binning of the full rows plus, with segmentation, their segment offsets.
void set_bins(Sweep& s, const Bins& b);

int rebin_full(gg_graph* g) {
  g->gen++;
  GG_TRY(rebin(g, g->full, nullptr));
  g->chunk_order_n = 0;
  if (!g->tune.seg_enable) return GG_OK;
  seg_geometry(g);
  GG_TRY(ensure_seg(g));
  GG_TRY(seg_offsets(g, g->full, (const uint32_t*)g->col, nullptr, 0xFFFFFFFFu, g->seg_off_full));
  // superstep hub chunks in source-segment order
  const int32_t nch = g->full.h.hub > 0 ? g->full.h.chunks : 0;
  if (nch == 0) return GG_OK;
  if (g->chunk_cap < nch) {
    dfree(g->chunk_order);
    dfree(g->chunk_scratch);
    g->chunk_cap = 0;
    GG_TRY(dalloc(&g->chunk_order, (size_t)nch));
    GG_TRY(dalloc(&g->chunk_scratch, (size_t)nch));
    g->chunk_cap = nch;
  }
  Sweep s;
  std::memset(&s, 0, sizeof(s));
  s.n = g->n;
  s.rowptr = g->rowptr;
  s.hub_chunk = g->tune.hub_chunk;
  set_bins(s, g->full);
  GG_HIP(launch_chunk_seg(s, g->col, g->seg_z, g->seg_s, g->chunk_scratch, g->stream));
  // stable counting sort by segment: the chunks of a row keep their order,
  // which the single-pass superstep relies on
  std::vector<int32_t> seg_of((size_t)nch), order((size_t)nch), cursor((size_t)g->seg_s + 1, 0);
  GG_HIP(hipMemcpyAsync(seg_of.data(), g->chunk_scratch, sizeof(int32_t) * (size_t)nch, hipMemcpyDeviceToHost,
                        g->stream));
  GG_HIP(hipStreamSynchronize(g->stream));
  for (int32_t c = 0; c < nch; ++c) {
    if (seg_of[c] < 0 || seg_of[c] >= g->seg_s) return fail(GG_E_DEVICE, "hub chunk segment out of range");
    cursor[(size_t)seg_of[c] + 1]++;
  }
  for (int32_t k = 0; k < g->seg_s; ++k) cursor[(size_t)k + 1] += cursor[(size_t)k];
  for (int32_t c = 0; c < nch; ++c) order[(size_t)cursor[(size_t)seg_of[c]]++] = c;
  GG_HIP(hipMemcpyAsync(g->chunk_order, order.data(), sizeof(int32_t) * (size_t)nch, hipMemcpyHostToDevice,
                        g->stream));
  GG_HIP(hipStreamSynchronize(g->stream));
  g->chunk_order_n = nch;
  return GG_OK;
}

// Binning of the active rows plus, with segmentation, their segment offsets.
int rebin_act(gg_graph* g, int app, bool after_superstep = false) {
  GG_TRY(rebin(g, g->act, g->act_cnt, nullptr, 0, after_superstep));
  if (!g->tune.seg_enable) return GG_OK;
  GG_TRY(ensure_seg(g));
  const uint32_t mask = app == GG_APP_SSSP ? 0xFFFFFFu : 0xFFFFFFFFu;
  return seg_offsets(g, g->act, g->act_edges, g->act_cnt, mask, g->seg_off_act);
}

// Out-CSR structure and frontier lists (first SSSP/CC run with the frontier on).
int ensure_out(gg_graph* g) {
  if (g->out_built) {
    if (!g->orow || !g->oedge || !g->odst || !g->osrc || !g->chg || !g->stamp || !g->flist[0] || !g->flist[1] ||
        !g->touched || !g->fc || !g->fdeg || !g->fscan || !g->psum)
      return fail(GG_E_STATE, "frontier arrays missing");
    return GG_OK;
  }
  const size_t n = (size_t)g->n, m = (size_t)g->m;
  GG_TRY(dalloc(&g->orow, n + 1));
  GG_TRY(dalloc(&g->oedge, m));
  GG_TRY(dalloc(&g->odst, m));
  GG_TRY(dalloc(&g->osrc, m));
  GG_TRY(dalloc(&g->chg, (n + 3) / 4 * 4));  // whole words, so that 32-bit fills clear it
  GG_TRY(dalloc(&g->stamp, n));
  GG_TRY(dalloc(&g->flist[0], n));
  GG_TRY(dalloc(&g->flist[1], n));
  GG_TRY(dalloc(&g->touched, n));
  GG_TRY(dalloc(&g->fc, 1));
  GG_TRY(dalloc(&g->fdeg, n));
  GG_TRY(dalloc(&g->fscan, n + 1));
  const size_t nblk = (n + kBlock - 1) / kBlock;
  GG_TRY(dalloc(&g->psum, nblk > 1024 ? nblk : 1024));
  GG_HIP(launch_fill_u32(g->stamp, g->n, 0u, g->stream));
  GG_HIP(launch_scan(g->outdeg, g->orow, g->n, g->orow + g->n, (int32_t*)g->blk_scratch, g->stream));
  // cursor scratch: the touched list is free at this point
  GG_HIP(launch_build_out(g->rowptr, g->col, g->n, g->m, g->orow, g->touched, g->oedge, g->odst, g->osrc,
                          g->stream));
  GG_HIP(hipStreamSynchronize(g->stream));
  g->out_built = true;
  return GG_OK;
}

int ensure_parts(gg_graph* g) {
  const int64_t need = max_chunks(g);
  if (g->part_cap >= need) return GG_OK;
  g->gen++;
  dfree(g->part_f);
  dfree(g->part_u);
  dfree(g->part_cnt);
  dfree(g->hub_sync);
  g->part_cap = 0;
  GG_TRY(dalloc(&g->part_f, (size_t)need));
  GG_TRY(dalloc(&g->part_u, (size_t)need));
  GG_TRY(dalloc(&g->part_cnt, (size_t)need));
  GG_TRY(dalloc(&g->hub_sync, 3 * (size_t)need + 2));
  GG_HIP(launch_fill_u32(g->hub_sync, 3 * need + 2, 0u, g->stream));
  g->part_cap = need;
  return GG_OK;
}

int ensure_workspace(gg_graph* g) {
  if (g->ws) return ensure_parts(g);
  g->gen++;
  const size_t n = (size_t)g->n, m = (size_t)g->m, nw = (m + 31) / 32;
  GG_TRY(dalloc(&g->c[0], n));
  GG_TRY(dalloc(&g->c[1], n));
  GG_TRY(dalloc(&g->xout, n));
  GG_TRY(dalloc(&g->xu[0], n));
  GG_TRY(dalloc(&g->xu[1], n));
  GG_TRY(dalloc(&g->bits[0], nw));
  GG_TRY(dalloc(&g->bits[1], nw));
  GG_TRY(dalloc(&g->act_edges, m));
  GG_TRY(dalloc(&g->act_cnt, n));
  GG_TRY(alloc_bins(g->act, g->n));
  GG_TRY(dalloc(&g->dpartial, 257));
  GG_TRY(dalloc(&g->changed, 1));
  if (!g->ev0) GG_HIP(hipEventCreate(&g->ev0));
  if (!g->ev1) GG_HIP(hipEventCreate(&g->ev1));
  g->ws = true;
  return ensure_parts(g);
}

void free_graph(gg_graph* g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  for (auto& s : g->spare) {
    dev_free(s.p);
    s.p = nullptr;
    s.bytes = 0;
  }
  if (g->owns_csr) {
    dfree(g->rowptr);
    dfree(g->col);
    dfree(g->weight);
  }
  dfree(g->wedges);
  dfree(g->outdeg);
  dfree(g->dang);
  dfree(g->i32_scratch);
  dfree(g->blk_scratch);
  free_bins(g->full);
  dfree(g->chunk_order);
  dfree(g->chunk_scratch);
  for (int i = 0; i < 2; ++i) {
    dfree(g->c[i]);
    dfree(g->xu[i]);
    dfree(g->bits[i]);
  }
  dfree(g->xout);
  dfree(g->act_edges);
  dfree(g->act_cnt);
  free_bins(g->act);
  dfree(g->part_f);
  dfree(g->part_u);
  dfree(g->part_cnt);
  dfree(g->hub_sync);
  dfree(g->dpartial);
  dfree(g->row_sum);
  dfree(g->vact);
  dfree(g->vdirty);
  dfree(g->x_prev);
  dfree(g->odeg_act);
  dfree(g->dang_act);
  dfree(g->bp_prior);
  dfree(g->changed);
  dfree(g->seg_off_full);
  dfree(g->seg_off_act);
  dfree(g->orow);
  dfree(g->oedge);
  dfree(g->odst);
  dfree(g->osrc);
  dfree(g->chg);
  dfree(g->stamp);
  dfree(g->flist[0]);
  dfree(g->flist[1]);
  dfree(g->touched);
  dfree(g->fc);
  dfree(g->fdeg);
  dfree(g->fscan);
  dfree(g->psum);
  dfree(g->part_start);
  dfree(g->part_of);
  dfree(g->part_e0);
  dfree(g->part_dstart);
  dfree(g->part_src);
  dfree(g->part_dang);
  for (int i = 0; i < 3; ++i) dfree(g->batch.buf[i]);
  dfree(g->batch.part);
  dfree(g->batch.dpart);
  dfree(g->batch.dang);
  dfree(g->batch.src);
  dfree(g->batch.ctr);
  if (g->batch.cs) (void)hipStreamDestroy(g->batch.cs);
  if (g->rg.exec) (void)hipGraphExecDestroy(g->rg.exec);
  if (g->rg.cs) (void)hipStreamDestroy(g->rg.cs);
  for (hipEvent_t e : {g->rg.ea, g->rg.eb})
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {g->batch.ea, g->batch.eb, g->batch.t0, g->batch.t1})
    if (e) (void)hipEventDestroy(e);
  dfree(g->seg_part);
  dfree(g->feat);
  dfree(g->sel);
  dfree(g->logits);
  dfree(g->labels);
  dfree(g->shadow);
  dfree(g->sel_count);
  dfree(g->audit);
  free_bins(g->selb);
  for (hipEvent_t e : g->pool) (void)hipEventDestroy(e);
  if (g->ev0) (void)hipEventDestroy(g->ev0);
  if (g->ev1) (void)hipEventDestroy(g->ev1);
  if (g->pin) (void)hipHostFree(g->pin);
  delete g;
}

bool valid_tuning(const gg_tuning& t) {
  const bool team_ok = t.small_team == 4 || t.small_team == 8 || t.small_team == 16 || t.small_team == 32;
  return team_ok && t.small_max >= 0 && t.wave_max >= t.small_max && t.wave_max >= 1 && t.hub_chunk >= kBlock &&
         (t.hub_chunk % kBlock) == 0 && t.hub_chunk <= (1 << 24) && (t.seg_enable == 0 || t.seg_enable == 1) &&
         t.seg_vertices >= 0 && (t.frontier_enable == 0 || t.frontier_enable == 1) && t.frontier_div >= 1;
}

// ---- schedule -------------------------------------------------------------

// Correction step (superstep) of GG and LEARNED at iteration i, 1-based:
// every (alpha+1)-th iteration; with decoupled parameters the first is
// iteration alpha0 + 1 and the later ones recur every alpha+1 iterations
// after it [Sec. 3.4].
bool is_correction(const gg_correction_policy& p, int32_t i) {
  if (!p.decoupled) return (i % (p.alpha + 1)) == 0;
  const int32_t first = p.alpha0 + 1;
  return i == first || (i > first && (i - first) % (p.alpha + 1) == 0);
}

// Influence threshold of the superstep at iteration i.
double theta_at(const gg_correction_policy& p, int32_t i) {
  return (p.decoupled && i == p.alpha0 + 1) ? p.theta0 : p.theta;
}

// Kind of iteration i by the schedule alone (a LEARNED correction step may
// become partial once its selection is known).
int step_kind(const gg_correction_policy& p, int32_t i) {
  switch (p.kind) {
    case GG_POLICY_EXACT: return GG_STEP_ACCURATE;
    case GG_POLICY_SP: return GG_STEP_APPROX;
    case GG_POLICY_SMS: return i >= p.alpha + 1 ? GG_STEP_ACCURATE : GG_STEP_APPROX;
    default: return is_correction(p, i) ? GG_STEP_FULL : GG_STEP_APPROX;
  }
}

bool is_pr(int app) { return app == GG_APP_PR || app == GG_APP_PPR; }
// Apps whose values are binary32 and whose gather sums binary32 per-vertex
// contributions (PR, PPR, BP); they run a fixed number of iterations.
bool is_float(int app) { return is_pr(app) || app == GG_APP_BP; }

int check_params(const gg_graph* g, const gg_app_params* p, double sigma, const gg_correction_policy* pol) {
  if (!p || !pol) return fail(GG_E_INVAL, "null params or policy");
  if (!g->full_valid) return fail(GG_E_STATE, "the graph was left unusable by a failed update");
  if (p->app < GG_APP_PR || p->app > GG_APP_BP) return fail(GG_E_INVAL, "unknown app");
  if (p->app == GG_APP_BP) {
    if (!(p->coupling >= 0.0 && p->coupling < 1.0)) return fail(GG_E_INVAL, "coupling outside [0, 1)");
    if (!p->prior && g->n > 0) return fail(GG_E_INVAL, "BP needs a prior");
    if (pol->kind == GG_POLICY_LEARNED || pol->trace) return fail(GG_E_UNSUPPORTED, "BP with LEARNED or traces");
    if (g->n_parts > 0) return fail(GG_E_UNSUPPORTED, "BP on a graph with parts");
  }
  if (pol->kind < GG_POLICY_EXACT || pol->kind > GG_POLICY_LEARNED) return fail(GG_E_INVAL, "unknown policy kind");
  if (pol->kind == GG_POLICY_LEARNED) {
    if (!pol->mlp) return fail(GG_E_INVAL, "LEARNED needs a network");
    if (!(pol->rho >= 0.0)) return fail(GG_E_INVAL, "rho < 0");
    if (pol->fallback_k < 0) return fail(GG_E_INVAL, "fallback_k < 0");
    if (std::isnan(pol->tau)) return fail(GG_E_INVAL, "tau is NaN");
  }
  if (pol->trace && pol->kind != GG_POLICY_GG && pol->kind != GG_POLICY_LEARNED)
    return fail(GG_E_INVAL, "traces are recorded by GG and LEARNED runs");
  if ((pol->trace || (pol->kind == GG_POLICY_LEARNED && pol->audit)) && is_pr(p->app) && !(pol->label_eps > 0.0f))
    return fail(GG_E_INVAL, "label_eps must be > 0");
  if (!(sigma >= 0.0 && sigma <= 1.0)) return fail(GG_E_INVAL, "sample_ratio outside [0, 1]");
  if (pol->alpha < 0) return fail(GG_E_INVAL, "alpha < 0");
  if (pol->decoupled != 0 && pol->decoupled != 1) return fail(GG_E_INVAL, "decoupled must be 0 or 1");
  if (pol->decoupled) {
    if (pol->kind != GG_POLICY_GG && pol->kind != GG_POLICY_LEARNED)
      return fail(GG_E_INVAL, "decoupled parameters belong to GG and LEARNED");
    if (pol->alpha0 < 0) return fail(GG_E_INVAL, "alpha0 < 0");
    if (!(pol->theta0 >= 0.0 && pol->theta0 < 65536.0)) return fail(GG_E_INVAL, "theta0 outside [0, 65536)");
  }
  if (!(pol->theta >= 0.0 && pol->theta < 65536.0)) return fail(GG_E_INVAL, "theta outside [0, 65536)");
  if (pol->mask_update != GG_MASK_REPLACE && pol->mask_update != GG_MASK_UNION)
    return fail(GG_E_INVAL, "unknown mask_update");
  if (pol->stop != GG_STOP_FIXED_ITERS && pol->stop != GG_STOP_FIXED_POINT) return fail(GG_E_INVAL, "unknown stop");
  if (pol->influence < GG_INFL_PREFIX || pol->influence > GG_INFL_PUSH) return fail(GG_E_INVAL, "unknown influence");
  if (pol->influence == GG_INFL_PUSH && p->app != GG_APP_SSSP && p->app != GG_APP_CC)
    return fail(GG_E_INVAL, "PUSH influence is defined for SSSP and CC (push order is PREFIX for sum-type apps)");
  if (p->pr_degree != GG_DEGREE_FULL && p->pr_degree != GG_DEGREE_ACTIVE) return fail(GG_E_INVAL, "unknown pr_degree");
  if (p->pr_degree == GG_DEGREE_ACTIVE) {
    if (!is_pr(p->app)) return fail(GG_E_INVAL, "the ACTIVE out-degree is defined for PR and PPR");
    if (pol->kind == GG_POLICY_LEARNED || pol->trace || pol->vstatus != GG_VSTATUS_NONE || g->n_parts > 0)
      return fail(GG_E_UNSUPPORTED, "ACTIVE out-degree with LEARNED, traces, vertex status or parts");
  }
  if (pol->vstatus < GG_VSTATUS_NONE || pol->vstatus > GG_VSTATUS_REL) return fail(GG_E_INVAL, "unknown vstatus");
  if (pol->vstatus != GG_VSTATUS_NONE) {
    if (!is_pr(p->app)) return fail(GG_E_INVAL, "vertex status is defined for PR and PPR");
    if (!(pol->eps >= 0.0) || !std::isfinite(pol->eps)) return fail(GG_E_INVAL, "eps must be finite and >= 0");
    if (pol->kind == GG_POLICY_LEARNED || pol->trace) return fail(GG_E_UNSUPPORTED, "vertex status with LEARNED or traces");
    if (g->n_parts > 0) return fail(GG_E_UNSUPPORTED, "vertex status on a graph with parts");
  }
  if (pol->influence == GG_INFL_TOTAL) {
    if (!is_pr(p->app)) return fail(GG_E_INVAL, "TOTAL influence is defined for PR and PPR");
    if (pol->kind == GG_POLICY_LEARNED) return fail(GG_E_UNSUPPORTED, "TOTAL influence with LEARNED");
  }
  if (p->dangling != GG_DANGLING_UNIFORM && p->dangling != GG_DANGLING_NONE) return fail(GG_E_INVAL, "unknown dangling");
  if (is_pr(p->app) && !(p->damping >= 0.0 && p->damping < 1.0)) return fail(GG_E_INVAL, "damping outside [0, 1)");
  if (g->n_parts > 0) {
    if (p->app == GG_APP_PPR) return fail(GG_E_UNSUPPORTED, "PPR on a graph with parts");
    if (p->app == GG_APP_SSSP && !g->part_src) return fail(GG_E_INVAL, "SSSP on parts needs part sources");
  } else if ((p->app == GG_APP_SSSP || p->app == GG_APP_PPR) && (p->source < 0 || p->source >= g->n)) {
    return fail(GG_E_INVAL, "source out of range");
  }
  if (p->app == GG_APP_SSSP && !g->wedges) return fail(GG_E_INVAL, "SSSP needs edge weights");
  const bool fixed_iters = is_float(p->app) || (pol->kind != GG_POLICY_EXACT && pol->stop == GG_STOP_FIXED_ITERS);
  if (fixed_iters && p->iters < 0) return fail(GG_E_INVAL, "iters < 0");
  if (!fixed_iters && p->max_iters <= 0) return fail(GG_E_INVAL, "max_iters must be > 0");
  return GG_OK;
}

Sweep base_sweep(const gg_graph* g, const gg_run* r, int32_t i) {
  Sweep s;
  std::memset(&s, 0, sizeof(s));
  s.n = g->n;
  s.small_max = g->tune.small_max;
  s.wave_max = g->tune.wave_max;
  s.hub_chunk = g->tune.hub_chunk;
  s.rowptr = g->rowptr;
  s.outdeg = g->outdeg;
  s.dangling = g->dpartial + 256;
  s.damping = r->p.damping;
  s.base = g->n > 0 ? (1.0 - r->p.damping) / (double)g->n : 0.0;
  s.source = r->p.source;
  s.changed = g->changed;
  s.part_f = g->part_f;
  s.part_u = g->part_u;
  s.part_cnt = g->part_cnt;
  s.hub_sync = g->hub_sync;
  s.hub_spin = g->hub_spin;
  s.theta = theta_at(r->pol, i);
  s.theta_q = (uint64_t)std::floor(s.theta * 65536.0 + 0.5);
  s.mask_union = r->pol.mask_update == GG_MASK_UNION;
  s.push_infl = r->pol.influence == GG_INFL_PUSH;
  s.act_edges = g->act_edges;
  s.act_cnt = g->act_cnt;
  if (r->p.app == GG_APP_BP) {
    s.bp_prior = g->bp_prior;
    s.bp_kappa = r->p.coupling;
  }
  if (r->pol.vstatus != GG_VSTATUS_NONE) {
    s.vact = g->vact;
    s.x_prev = g->x_prev;
    s.vs_eps = r->pol.eps;
    s.vs_rel = r->pol.vstatus == GG_VSTATUS_REL;
  }
  if (g->n_parts > 0) {
    s.part_of = g->part_of;
    s.part_start = g->part_start;
    s.part_dang = g->part_dang;
  }
  return s;
}

void set_bins(Sweep& s, const Bins& b) {
  s.list = b.list;
  s.hub_start = b.hub_start;
  s.n_small = b.h.small;
  s.n_wave = b.h.wave;
  s.n_hub = b.h.hub;
  s.n_chunks = b.h.chunks;
}

// Two events for one profiled launch (nullptr pair when profiling is off).
int prof_events(gg_graph* g, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (!g->prof) return GG_OK;
  while (g->pool.size() < g->pool_used + 2) {
    hipEvent_t e;
    GG_HIP(hipEventCreate(&e));
    g->pool.push_back(e);
  }
  *e0 = g->pool[g->pool_used++];
  *e1 = g->pool[g->pool_used++];
  return GG_OK;
}

// Algorithmic bytes of one sweep launch: per gathered edge the edge word and
// the gathered source value; per row its list entry, row offset, active count
// (approximate mode), out-degree or own value, and the value written.
double alg_bytes(int kind, int64_t rows, int64_t edges, bool x_out) {
  const double per_row = 16.0 + (kind == 1 ? 4.0 : 0.0) + (kind == 2 ? 4.0 : 0.0) + (x_out ? 4.0 : 0.0);
  return 8.0 * (double)edges + per_row * (double)rows;
}

const uint32_t* full_edges(const gg_graph* g, int app) {
  return app == GG_APP_SSSP ? g->wedges : (const uint32_t*)g->col;
}

int pack_from_bits0(gg_graph* g, int app);

// Initial sample of the edge flags into bits[0], the packed active edges and
// their binning [Sec. 3.4].
int sample_and_pack(gg_graph* g, int app, double sigma, uint64_t seed) {
  const uint64_t keep = (uint64_t)std::floor(sigma * 4294967296.0 + 0.5);
  if (g->n_parts > 0)
    GG_HIP(launch_sample_bits_parts(g->m, seed, 0, keep, g->n_parts, g->part_e0, g->bits[0], g->stream));
  else
    GG_HIP(launch_sample_bits(g->m, seed, 0, keep, g->bits[0], g->stream));
  return pack_from_bits0(g, app);
}

// Packed active edges (flag set in bits[0], CSR order within each row) and
// their binning.
int pack_from_bits0(gg_graph* g, int app) {
  Sweep s;
  std::memset(&s, 0, sizeof(s));
  s.n = g->n;
  s.small_max = g->tune.small_max;
  s.wave_max = g->tune.wave_max;
  s.hub_chunk = g->tune.hub_chunk;
  s.rowptr = g->rowptr;
  s.part_cnt = g->part_cnt;
  s.act_edges = g->act_edges;
  s.act_cnt = g->act_cnt;
  set_bins(s, g->full);
  s.edges = full_edges(g, app);
  s.old_bits = g->bits[0];
  GG_TRY(check_part_capacity(g, g->full));
  GG_HIP(launch_pack(s, g->stream));
  return rebin_act(g, app);
}

// PR with the ACTIVE out-degree: approximate iterations divide by it
bool active_degree_run(const gg_run* r) {
  return is_pr(r->p.app) && r->p.pr_degree == GG_DEGREE_ACTIVE && r->pol.kind != GG_POLICY_EXACT;
}

// Active out-degree of the flags in bits[b] and the list of vertices without
// an active out-edge (the dangling set of the sparsified graph).
int active_degree(gg_graph* g, int b) {
  if (!g->odeg_act) GG_TRY(dalloc(&g->odeg_act, (size_t)g->n));
  if (!g->dang_act) GG_TRY(dalloc(&g->dang_act, (size_t)g->n));
  if (g->n == 0) {
    g->n_dang_act = 0;
    return GG_OK;
  }
  GG_HIP(launch_active_degree(g->col, g->m, g->bits[b], g->n, g->odeg_act, g->stream));
  GG_HIP(launch_dangling_list(g->odeg_act, g->n, g->dang_act, g->i32_scratch + 3, (int32_t*)g->blk_scratch,
                              g->stream));
  return readback(g, &g->n_dang_act, g->i32_scratch + 3, sizeof(int32_t));
}

int run_begin(gg_graph* g, const gg_app_params* p, double sigma, const gg_correction_policy* pol, gg_run** out) {
  GG_TRY(check_params(g, p, sigma, pol));
  if (g->active_run) return fail(GG_E_STATE, "another run is active on this graph");
  GG_TRY(ensure_workspace(g));
  std::unique_ptr<gg_run> owner(new (std::nothrow) gg_run());
  gg_run* r = owner.get();
  if (!r) return fail(GG_E_NOMEM, "host allocation failed");
  r->g = g;
  r->p = *p;
  r->pol = *pol;
  r->sigma = sigma;
  const int app = p->app;
  // initial values
  const bool parts = g->n_parts > 0;
  if (is_pr(app)) {
    GG_HIP(launch_pr_init(app, g->outdeg, g->n, p->source, parts ? g->part_of : nullptr,
                          parts ? g->part_start : nullptr, g->c[0], g->stream));
    if (p->dangling == GG_DANGLING_NONE) {
      GG_HIP(launch_fill_u32((uint32_t*)(g->dpartial + 256), 2, 0u, g->stream));
      if (parts) GG_HIP(launch_fill_u32((uint32_t*)g->part_dang, 2 * (int64_t)g->n_parts, 0u, g->stream));
    }
  } else if (app == GG_APP_BP) {
    // the run keeps its own copy of the prior
    if (g->n > 0) {
      if (!g->bp_prior) GG_TRY(dalloc(&g->bp_prior, (size_t)g->n));
      GG_HIP(hipMemcpyAsync(g->bp_prior, p->prior, sizeof(float) * (size_t)g->n, hipMemcpyDeviceToDevice, g->stream));
      GG_HIP(launch_bp_init(g->bp_prior, g->n, p->coupling, g->c[0], g->stream));
    }
  } else {
    const int32_t src0 = parts ? -1 : p->source;
    GG_HIP(launch_min_init(app, g->n, src0, g->xu[0], g->stream));
    GG_HIP(launch_min_init(app, g->n, src0, g->xu[1], g->stream));
    if (parts && app == GG_APP_SSSP) {
      GG_HIP(launch_set_sources(g->part_src, g->n_parts, g->xu[0], g->stream));
      GG_HIP(launch_set_sources(g->part_src, g->n_parts, g->xu[1], g->stream));
    }
    if (g->tune.frontier_enable) {
      GG_TRY(ensure_out(g));
      if (parts && app == GG_APP_SSSP) {
        // every part's source is new at iteration 0
        GG_HIP(launch_copy_u32((const uint32_t*)g->part_src, (uint32_t*)g->flist[0], g->n_parts, g->stream));
        r->fcur = 0;
        r->front_count = g->n_parts;
        r->front_outdeg = 0;
      } else if (app == GG_APP_SSSP && g->n > 0) {
        // the source is the only vertex whose value is new at iteration 0
        const int32_t src = p->source;
        int32_t od = 0;
        GG_HIP(hipMemcpyAsync(g->flist[0], &src, sizeof(int32_t), hipMemcpyHostToDevice, g->stream));
        GG_TRY(readback(g, &od, g->outdeg + src, sizeof(int32_t)));
        r->fcur = 0;
        r->front_count = 1;
        r->front_outdeg = od;
      } else {
        // every label is new at iteration 0: no list is materialised, the first
        // iteration runs dense (front_count < 0)
        r->front_count = -1;
        r->front_outdeg = 0;
      }
    }
  }
  if (pol->vstatus != GG_VSTATUS_NONE && g->n > 0) {
    // every vertex is active before the first iteration; previous values x0
    const size_t words = ((size_t)g->n + 3) / 4;
    if (!g->vact) GG_TRY(dalloc(&g->vact, words * 4));
    if (!g->vdirty) GG_TRY(dalloc(&g->vdirty, words * 4));
    if (!g->x_prev) GG_TRY(dalloc(&g->x_prev, (size_t)g->n));
    GG_TRY(ensure_out(g));
    GG_HIP(launch_fill_u32((uint32_t*)g->vact, (int64_t)words, 0x01010101u, g->stream));
    float x0 = p->app == GG_APP_PR ? (float)(1.0 / (double)g->n) : 0.0f;
    uint32_t bits0;
    std::memcpy(&bits0, &x0, 4);
    GG_HIP(launch_fill_u32((uint32_t*)g->x_prev, g->n, bits0, g->stream));
    if (p->app == GG_APP_PPR) {
      const float one = 1.0f;
      uint32_t b1;
      std::memcpy(&b1, &one, 4);
      GG_HIP(launch_fill_u32((uint32_t*)g->x_prev + p->source, 1, b1, g->stream));
    }
  }
  // initial sparsification [Sec. 3.4]
  if (pol->kind != GG_POLICY_EXACT) GG_TRY(sample_and_pack(g, app, sigma, pol->seed));
  if (active_degree_run(r)) {
    // the first iteration's contributions divide by the active out-degree
    GG_TRY(active_degree(g, 0));
    if (step_kind(*pol, 1) == GG_STEP_APPROX)
      GG_HIP(launch_pr_init(app, g->odeg_act, g->n, p->source, nullptr, nullptr, g->c[0], g->stream));
  }
  if (pol->kind == GG_POLICY_LEARNED || pol->trace) {
    GG_TRY(ensure_learned(g));
    // the delta features start at 0 (no iteration before iteration 0)
    GG_HIP(launch_fill_u32((uint32_t*)g->feat, (int64_t)g->n * 4, 0u, g->stream));
    GG_HIP(launch_fill_u32((uint32_t*)g->audit, 4, 0u, g->stream));
  }
  const bool fixed_iters = is_float(app) || (pol->kind != GG_POLICY_EXACT && pol->stop == GG_STOP_FIXED_ITERS);
  if (fixed_iters && p->iters == 0) r->done = true;
  g->active_run = owner.release();
  *out = r;
  return GG_OK;
}

// Features and selection of a LEARNED correction step; sets the step kind
// (full when forced by the fallback schedule or when |S| > rho * n).
int learned_select(gg_run* r, int* kind, int64_t* selected) {
  gg_graph* g = r->g;
  const int32_t c = ++r->corrections;
  const bool forced = r->pol.fallback_k > 0 && c % r->pol.fallback_k == 0;
  GG_HIP(launch_feat_base(g->n, g->rowptr, g->outdeg, g->act_cnt, g->feat, g->stream));
  r->have_feat = true;
  *kind = GG_STEP_FULL;
  GG_HIP(launch_fill_u32((uint32_t*)g->sel_count, 4, 0u, g->stream));
  unsigned long long* sel_edges_dev = (unsigned long long*)(g->sel_count + 2);
  GG_HIP(launch_mlp_forward(r->pol.mlp->d, g->feat, g->n, g->logits, g->sel, r->pol.tau, g->sel_count, g->rowptr,
                            sel_edges_dev, g->stream));
  int32_t h[4] = {0, 0, 0, 0};
  GG_HIP(hipMemcpyAsync(h, g->sel_count, sizeof(h), hipMemcpyDeviceToHost, g->stream));
  GG_HIP(hipStreamSynchronize(g->stream));
  const int32_t cnt = h[0];
  unsigned long long sel_edges = 0;
  memcpy(&sel_edges, h + 2, sizeof(sel_edges));
  r->have_sel = true;
  *selected = cnt;
  r->selected_total += cnt;
  // fallback when the selected rows hold more than rho * m in-edges
  if (!forced && !((double)sel_edges > r->pol.rho * (double)g->m)) *kind = GG_STEP_PARTIAL;
  if (*kind == GG_STEP_FULL && r->pol.audit) r->audit_selected += cnt;
  return GG_OK;
}

// One iteration. sync_changed: read the changed count back (needed for
// fixed-point termination and for step info).
int run_step(gg_run* r, gg_step_info* info, bool sync_changed) {
  gg_graph* g = r->g;
  if (r->done) return 0;
  const int32_t i = r->iter + 1;
  const int app = r->p.app;
  const bool pr = is_float(app);  // binary32 values (PR, PPR, BP)
  const bool learned = r->pol.kind == GG_POLICY_LEARNED;
  int kind = step_kind(r->pol, i);
  int64_t selected = -1;
  r->have_sel = false;
  r->have_labels = false;
  // Delta features of the next correction step c: at the start of iterations
  // c-1 and c the buffers hold the states of iterations (c-2, c-3) and then
  // (c-1, c-2); each shift moves f3 to f4 and writes the newer delta to f3.
  if ((learned || r->pol.trace) && i >= 2 && g->n > 0) {
    if (is_correction(r->pol, i) || is_correction(r->pol, i + 1)) {
      const uint32_t* now = pr ? (const uint32_t*)g->c[r->cur] : g->xu[r->cur];
      const uint32_t* before = pr ? (const uint32_t*)g->c[1 - r->cur] : g->xu[1 - r->cur];
      GG_HIP(launch_feat_shift(app, g->n, now, before, g->feat, g->stream));
    }
  }
  if (learned && kind == GG_STEP_FULL) GG_TRY(learned_select(r, &kind, &selected));
  const bool accurate = kind == GG_STEP_ACCURATE || kind == GG_STEP_FULL;
  const bool superstep = kind == GG_STEP_FULL || kind == GG_STEP_PARTIAL;
  // a traced or audited full superstep also computes the approximate update
  // and labels every vertex by the difference
  const bool traced = r->pol.trace != nullptr && kind == GG_STEP_FULL;
  const bool audited = learned && r->pol.audit && kind == GG_STEP_FULL && r->have_sel;
  if (traced && !learned) {
    GG_HIP(launch_feat_base(g->n, g->rowptr, g->outdeg, g->act_cnt, g->feat, g->stream));
    r->have_feat = true;
  }
  const bool last_fixed = (pr || (r->pol.kind != GG_POLICY_EXACT && r->pol.stop == GG_STOP_FIXED_ITERS)) &&
                          i >= r->p.iters;
  Sweep s = base_sweep(g, r, i);
  const bool act_deg = active_degree_run(r);
  if (pr) {
    if (is_pr(app) && r->p.dangling == GG_DANGLING_UNIFORM) {
      // with the ACTIVE out-degree an approximate iteration's dangling set is
      // the vertices without an active out-edge
      const bool ad = act_deg && kind == GG_STEP_APPROX;
      if (g->n_parts > 0)
        GG_HIP(launch_parts_dangling_sum(g->c[r->cur], g->dang, g->n_parts, g->part_dstart, g->part_dang,
                                         g->part_dang + g->n_parts, g->stream));
      else
        GG_HIP(launch_dangling_sum(g->c[r->cur], ad ? g->dang_act : g->dang, nullptr, ad ? g->n_dang_act : g->n_dang,
                                   g->dpartial, g->dpartial + 256, g->stream));
    }
    // the apply writes the contributions the next iteration gathers: over the
    // active out-degree when that iteration is approximate (after a superstep
    // they are recomputed once the new flags are known)
    if (act_deg && !superstep && step_kind(r->pol, i + 1) == GG_STEP_APPROX) s.outdeg = g->odeg_act;
    s.c_in = g->c[r->cur];
    s.c_out = g->c[1 - r->cur];
    s.x_out = (r->write_x_each_step || last_fixed) ? g->xout : nullptr;
    if (act_deg && superstep && step_kind(r->pol, i + 1) == GG_STEP_APPROX) s.x_out = g->xout;
  } else {
    s.x_in = g->xu[r->cur];
    s.x_next = g->xu[1 - r->cur];
  }
  const bool frontier = !pr && g->tune.frontier_enable && g->out_built;
  // with the frontier the changed count comes from the compacted list and
  // the counter is never read
  if (!pr && !frontier) GG_HIP(launch_fill_u32((uint32_t*)g->changed, 1, 0u, g->stream));
  if (frontier) GG_TRY(ensure_out(g));
  // A push from the changed vertices is exact when this iteration's edge set
  // is contained in the previous one's: not at a superstep, not at a switch
  // from approximate to accurate mode.
  const bool grows = accurate && (i == 1 || step_kind(r->pol, i - 1) == GG_STEP_APPROX) && r->pol.kind != GG_POLICY_EXACT;
  // front_count >= 0 only when flist[fcur] was written (source seed, dense
  // compaction or push finalize)
  const bool sparse = frontier && !superstep && !grows && r->front_count >= 0 && r->front_count <= g->n &&
                      (double)r->front_outdeg * (double)g->tune.frontier_div <= (double)g->m;
  // with the frontier, the changed count comes from the compacted changed
  // list, so the dense kernels skip their (contended) counter
  if (frontier) {
    s.chg = g->chg;
    s.changed = nullptr;
  }
  // A push from an empty frontier changes nothing (both value buffers already
  // hold the current values), so such an iteration launches no work at all:
  // an approximate run whose sampled edges have converged idles this way
  // until its next superstep.
  const bool idle = sparse && r->front_count == 0;
  int64_t edges;
  int64_t processed;
  hipEvent_t pe0 = nullptr, pe1 = nullptr;
  if (!idle) GG_TRY(prof_events(g, &pe0, &pe1));
  int pkind;
  if (sparse) {
    pkind = accurate ? 0 : 1;
    if (!idle) {
      s.edges = full_edges(g, app);
      const uint32_t* bits = accurate ? nullptr : g->bits[r->bcur];
      g->epoch++;
      if (pe0) GG_HIP(hipEventRecord(pe0, g->stream));
      GG_HIP(launch_push(app, s, g->flist[r->fcur], (int32_t)r->front_count, r->front_outdeg, g->orow, g->oedge,
                         g->odst, bits, g->stamp, g->epoch, g->touched, g->flist[1 - r->fcur], g->fc, g->fdeg,
                         g->fscan, (int32_t*)g->blk_scratch, g->psum, g->stream));
      if (pe1) GG_HIP(hipEventRecord(pe1, g->stream));
    }
    edges = accurate ? g->m : g->act.h.edges;
    processed = r->front_outdeg;
    r->sparse_iters++;
  } else if (kind == GG_STEP_PARTIAL) {
    // Partial superstep: the selected rows S gather over all in-edges and
    // re-select their flags; the other rows take an approximate iteration and
    // keep theirs. The approximate gather skips the rows of S (selection
    // bytes as its skip mask), so its work scales with the rows outside S;
    // the superstep then computes S from its list.
    pkind = 4;
    GG_TRY(rebin(g, g->selb, nullptr, g->sel, 1));
    const int32_t ns = g->selb.h.small + g->selb.h.wave + g->selb.h.hub;
    GG_HIP(launch_copy_u32(g->bits[r->bcur], g->bits[1 - r->bcur], (g->m + 31) / 32, g->stream));
    GG_HIP(launch_clear_rows(g->selb.list, g->selb.h.small, ns, g->rowptr, g->bits[1 - r->bcur], g->stream));
    GG_HIP(launch_fill_u32((uint32_t*)(g->audit + 2), 2, 0u, g->stream));
    Sweep sa = s;
    set_bins(sa, g->act);
    sa.edges = g->act_edges;
    sa.cnt = g->act_cnt;
    sa.skip = g->sel;
    GG_TRY(check_part_capacity(g, g->act));
    if (g->tune.seg_enable) {
      GG_TRY(check_seg_capacity(g, g->act));
      set_seg(g, sa, g->seg_off_act);
      GG_HIP(launch_gather_seg(app, g->tune.small_team, sa, g->stream, pe0, nullptr));
    } else {
      GG_HIP(launch_gather(app, g->tune.small_team, sa, g->stream, pe0, nullptr));
    }
    // active edges of S, for the edge count
    GG_HIP(launch_sel_active(g->selb.list, ns, g->act_cnt, g->audit + 2, g->stream));
    const int64_t act_all = g->act.h.edges;
    Sweep sc = s;
    set_bins(sc, g->selb);
    sc.edges = full_edges(g, app);
    sc.cnt = nullptr;
    sc.old_bits = g->bits[r->bcur];
    sc.new_bits = g->bits[1 - r->bcur];
    GG_TRY(check_part_capacity(g, g->selb));
    if (g->tune.seg_enable) {
      sc.flat_list = 1;
      GG_HIP(launch_superstep_flat(app, sc, g->stream, nullptr, pe1));
    } else {
      GG_HIP(launch_superstep(app, g->tune.small_team, sc, g->stream, nullptr, pe1));
    }
    unsigned long long act_s = 0;
    GG_HIP(hipMemcpyAsync(&act_s, g->audit + 2, sizeof(act_s), hipMemcpyDeviceToHost, g->stream));
    r->bcur = 1 - r->bcur;
    GG_TRY(rebin_act(g, app, true));  // synchronizes the stream, reads the hub error word
    r->supersteps++;
    r->partials++;
    // S over all in-edges, the other rows over their active ones
    edges = act_all - (int64_t)act_s + g->selb.h.edges;
    processed = edges;
  } else if (superstep) {
    pkind = 2;
    if (traced || audited) {
      // approximate update from the same state, into the shadow buffer
      Sweep sh = s;
      set_bins(sh, g->act);
      sh.edges = g->act_edges;
      sh.cnt = g->act_cnt;
      sh.chg = nullptr;
      sh.x_out = nullptr;
      if (pr) {
        sh.c_out = (float*)g->shadow;
      } else {
        sh.x_next = g->shadow;
        sh.changed = nullptr;  // the shadow pass counts nothing
      }
      GG_TRY(check_part_capacity(g, g->act));
      GG_HIP(launch_gather(app, g->tune.small_team, sh, g->stream));
    }
    GG_HIP(launch_fill_u32(g->bits[1 - r->bcur], (g->m + 31) / 32, 0u, g->stream));
    set_bins(s, g->full);
    s.edges = full_edges(g, app);
    s.cnt = nullptr;
    if (pr && r->pol.influence == GG_INFL_TOTAL) {
      // TOTAL influence [Alg. 2, GG-Gather variant]: each edge's contribution
      // over its row's sum, from an accurate gather before the superstep
      if (!g->row_sum) GG_TRY(dalloc(&g->row_sum, (size_t)g->n));
      Sweep st = s;
      st.sum_out = g->row_sum;
      GG_TRY(check_part_capacity(g, g->full));
      if (g->tune.seg_enable) {
        GG_TRY(check_seg_capacity(g, g->full));
        set_seg(g, st, g->seg_off_full);
        GG_HIP(launch_gather_seg(app, g->tune.small_team, st, g->stream));
      } else {
        GG_HIP(launch_gather(app, g->tune.small_team, st, g->stream));
      }
      s.row_total = g->row_sum;
    }
    s.old_bits = g->bits[r->bcur];
    s.new_bits = g->bits[1 - r->bcur];
    GG_TRY(check_part_capacity(g, g->full));
    if (g->tune.seg_enable && g->chunk_order_n == g->full.h.chunks && g->full.h.hub > 0)
      s.chunk_order = g->chunk_order;
    if (g->tune.seg_enable)
      GG_HIP(launch_superstep_flat(app, s, g->stream, pe0, pe1));
    else
      GG_HIP(launch_superstep(app, g->tune.small_team, s, g->stream, pe0, pe1));
    r->bcur = 1 - r->bcur;
    if (traced || audited) {
      const uint32_t* acc = pr ? (const uint32_t*)s.c_out : s.x_next;
      float* lf = nullptr;
      int32_t nf = 0;
      unsigned long long* tpos = nullptr;
      if (traced) {
        gg_trace* T = r->pol.trace;
        const int64_t room = T->cap - T->size;
        nf = (int32_t)(room < (int64_t)g->n ? room : (int64_t)g->n);
        if (nf > 0) {
          GG_HIP(launch_copy_u32((const uint32_t*)g->feat, (uint32_t*)(T->feat + T->size * 8), (int64_t)nf * 4,
                                 g->stream));
          lf = T->label + T->size;
          tpos = T->pos;
        }
        T->size += nf;
        T->dropped += (int64_t)g->n - nf;
      }
      GG_HIP(launch_labels(app, g->n, acc, g->shadow, r->pol.label_eps, audited ? g->sel : nullptr, g->labels, lf, nf,
                           audited ? g->audit : nullptr, tpos, g->stream));
      r->have_labels = true;
    }
    GG_TRY(rebin_act(g, app, true));  // reads the hub error word too
    if (act_deg && step_kind(r->pol, i + 1) == GG_STEP_APPROX) {
      // the next iteration divides by the active out-degree of the new flags
      GG_TRY(active_degree(g, r->bcur));
      GG_HIP(launch_recontrib(g->xout, g->odeg_act, g->n, g->c[1 - r->cur], g->stream));
    }
    r->supersteps++;
    edges = g->m;
    processed = s.row_total ? 2 * edges : edges;
  } else if (accurate) {
    pkind = 0;
    set_bins(s, g->full);
    s.edges = full_edges(g, app);
    s.cnt = nullptr;
    GG_TRY(check_part_capacity(g, g->full));
    if (g->tune.seg_enable) {
      GG_TRY(check_seg_capacity(g, g->full));
      set_seg(g, s, g->seg_off_full);
      GG_HIP(launch_gather_seg(app, g->tune.small_team, s, g->stream, pe0, pe1));
    } else {
      GG_HIP(launch_gather(app, g->tune.small_team, s, g->stream, pe0, pe1));
    }
    edges = g->m;
    processed = edges;
  } else if (r->pol.vstatus != GG_VSTATUS_NONE && i > 1 && g->n > 0) {
    // GG-VStatus [Alg. 2; Sec. 2.1]: only the rows that an active in-edge from
    // an active vertex reaches are recomputed; the others keep their values
    // (and become inactive)
    pkind = 1;
    GG_HIP(launch_compact_changed(g->vact, g->outdeg, g->n, g->flist[0], g->fc, (int32_t*)g->blk_scratch, g->psum,
                                  g->stream));
    FrontCounters h = {0, 0, 0};
    GG_TRY(readback(g, &h, g->fc, sizeof(h)));
    const int64_t words = ((int64_t)g->n + 3) / 4;
    GG_HIP(launch_fill_u32((uint32_t*)g->vdirty, words, 0u, g->stream));
    GG_HIP(launch_vs_mark(g->flist[0], h.count, h.outdeg_sum, g->orow, g->oedge, g->odst, g->bits[r->bcur], g->fdeg,
                          g->fscan, (int32_t*)g->blk_scratch, g->vdirty, g->stream));
    GG_TRY(ensure_selb(g));
    GG_TRY(rebin(g, g->selb, g->act_cnt, g->vdirty, 1));
    GG_HIP(launch_copy_u32((const uint32_t*)s.c_in, (uint32_t*)s.c_out, g->n, g->stream));
    if (s.x_out) GG_HIP(launch_copy_u32((const uint32_t*)g->x_prev, (uint32_t*)s.x_out, g->n, g->stream));
    GG_HIP(launch_fill_u32((uint32_t*)g->vact, words, 0u, g->stream));
    set_bins(s, g->selb);
    s.edges = g->act_edges;
    s.cnt = g->act_cnt;
    GG_TRY(check_part_capacity(g, g->selb));
    if (pe0) GG_HIP(hipEventRecord(pe0, g->stream));
    GG_HIP(launch_gather(app, g->tune.small_team, s, g->stream));
    if (pe1) GG_HIP(hipEventRecord(pe1, g->stream));
    edges = g->selb.h.edges;
    processed = edges + h.outdeg_sum;
  } else {
    pkind = 1;
    set_bins(s, g->act);
    s.edges = g->act_edges;
    s.cnt = g->act_cnt;
    GG_TRY(check_part_capacity(g, g->act));
    if (g->tune.seg_enable) {
      GG_TRY(check_seg_capacity(g, g->act));
      set_seg(g, s, g->seg_off_act);
      GG_HIP(launch_gather_seg(app, g->tune.small_team, s, g->stream, pe0, pe1));
    } else {
      GG_HIP(launch_gather(app, g->tune.small_team, s, g->stream, pe0, pe1));
    }
    edges = g->act.h.edges;
    processed = edges;
  }
  if (frontier && !sparse)
    GG_HIP(launch_compact_changed(g->chg, g->outdeg, g->n, g->flist[1 - r->fcur], g->fc, (int32_t*)g->blk_scratch,
                                  g->psum, g->stream));
  if (g->prof && !idle) {
    double bytes = alg_bytes(pkind == 4 ? 2 : pkind, g->n, edges, s.x_out != nullptr);
    if (pkind == 2) bytes += 4.0 * (double)g->act.h.edges + (double)((g->m + 31) / 32) * 4.0;
    if (sparse) {
      // per pushed edge: edge id, destination, weight word, flag word (approx), atomic on the target;
      // per frontier vertex: list entry, out-row offsets, value, sync
      pkind = 3;
      bytes = (accurate ? 16.0 : 20.0) * (double)processed + 16.0 * (double)r->front_count;
    }
    g->recs.push_back({pkind, app, pe0, pe1, bytes, processed});
  }
  r->cur = 1 - r->cur;
  r->iter = i;
  r->x_valid = pr && s.x_out != nullptr;
  r->edges_total += edges;
  r->edges_processed += processed;
  int64_t changed = -1;
  if (frontier) {
    // The counters decide whether the next iteration may push. The host need
    // not wait for them when that iteration runs dense anyway (a superstep, or
    // the switch to accurate mode) or when a fixed-count run ends here, unless
    // the caller wants the changed count; the frontier is then left unknown.
    const int nk = step_kind(r->pol, i + 1);
    const bool next_dense = nk == GG_STEP_FULL || (nk == GG_STEP_ACCURATE && step_kind(r->pol, i) == GG_STEP_APPROX &&
                                                   r->pol.kind != GG_POLICY_EXACT);
    const bool known = idle || sync_changed || !(last_fixed || next_dense);
    FrontCounters h = {0, 0, 0};
    if (!idle && known) GG_TRY(readback(g, &h, g->fc, sizeof(h)));
    r->fcur = 1 - r->fcur;
    r->front_count = known ? h.count : -1;
    r->front_outdeg = known ? h.outdeg_sum : 0;
    changed = known ? h.count : -1;
  } else if (!pr && sync_changed) {
    int32_t hc = 0;
    GG_TRY(readback(g, &hc, g->changed, sizeof(int32_t)));
    changed = hc;
  }
  // termination
  if (pr) {
    if (i >= r->p.iters) r->done = true;
  } else if (r->pol.kind == GG_POLICY_EXACT) {
    if (changed == 0) r->converged = true;
    if (changed == 0 || i >= r->p.max_iters) r->done = true;
  } else if (r->pol.stop == GG_STOP_FIXED_ITERS) {
    if (i >= r->p.iters) r->done = true;
  } else {
    const bool final_kind = accurate || r->pol.kind == GG_POLICY_SP;
    if ((changed == 0 && final_kind) || i >= r->p.max_iters) r->done = true;
  }
  if (info) {
    info->iter = i;
    info->accurate = accurate;
    info->superstep = superstep;
    info->edges = edges;
    info->changed = changed;
    info->active_edges = r->pol.kind == GG_POLICY_EXACT ? g->m : g->act.h.edges;
    info->edges_processed = processed;
    info->sparse = sparse ? 1 : 0;
    info->kind = kind;
    info->selected = selected;
  }
  return 1;
}

int copy_out(gg_graph* g, const void* dsrc, void* out, size_t bytes, uint32_t flags) {
  if (flags & GG_OUT_HOST) {
    GG_HIP(hipMemcpyAsync(out, dsrc, bytes, hipMemcpyDeviceToHost, g->stream));
  } else {
    GG_HIP(hipMemcpyAsync(out, dsrc, bytes, hipMemcpyDeviceToDevice, g->stream));
  }
  GG_HIP(hipStreamSynchronize(g->stream));
  return GG_OK;
}

// PR values before any iteration: the initial vector.
int pr_initial_x(gg_run* r) {
  gg_graph* g = r->g;
  if (g->n == 0) return GG_OK;
  float* h = new (std::nothrow) float[(size_t)g->n];
  if (!h) return fail(GG_E_NOMEM, "host allocation failed");
  std::vector<int32_t> ps;
  if (g->n_parts > 0) {
    ps.resize((size_t)g->n_parts + 1);
    hipError_t e = hipMemcpy(ps.data(), g->part_start, sizeof(int32_t) * ps.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      delete[] h;
      return fail(GG_E_DEVICE, std::string("initial values: ") + hipGetErrorString(e));
    }
  }
  for (int32_t p = 0, u = 0; u < g->n; ++u) {
    double N = (double)g->n;
    if (!ps.empty()) {
      while (u >= ps[p + 1]) ++p;
      N = (double)(ps[p + 1] - ps[p]);
    }
    h[u] = r->p.app == GG_APP_PR ? (float)(1.0 / N) : (u == r->p.source ? 1.0f : 0.0f);
  }
  hipError_t e = hipMemcpyAsync(g->xout, h, sizeof(float) * (size_t)g->n, hipMemcpyHostToDevice, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  delete[] h;
  if (e != hipSuccess) return fail(GG_E_DEVICE, std::string("initial values: ") + hipGetErrorString(e));
  r->x_valid = true;
  return GG_OK;
}

// Error word of the single-pass hub chunks: a wait that reached its spin
// limit leaves the results of that superstep undefined.
int check_hub_sync(gg_graph* g) {
  if (!g->hub_sync) return GG_OK;
  uint32_t e = 0;
  GG_TRY(readback(g, &e, g->hub_sync, sizeof(e)));
  if (e == 0) return GG_OK;
  GG_HIP(launch_fill_u32(g->hub_sync, 1, 0u, g->stream));
  return fail(GG_E_DEVICE, "a superstep hub chunk gave up waiting for its row prefix");
}

int run_values(gg_run* r, void* out, uint32_t flags) {
  gg_graph* g = r->g;
  if (!out) return fail(GG_E_INVAL, "null output");
  // only a superstep can raise the hub error word
  if (r->supersteps > 0) GG_TRY(check_hub_sync(g));
  if (r->p.app == GG_APP_BP && r->iter == 0)
    return copy_out(g, g->bp_prior, out, sizeof(float) * (size_t)g->n, flags);  // the beliefs start at the prior
  if (is_float(r->p.app)) {
    if (r->iter == 0) GG_TRY(pr_initial_x(r));
    if (!r->x_valid) return fail(GG_E_STATE, "PR values of this iteration were not materialized");
    return copy_out(g, g->xout, out, sizeof(float) * (size_t)g->n, flags);
  }
  return copy_out(g, g->xu[r->cur], out, sizeof(uint32_t) * (size_t)g->n, flags);
}

// Learned-policy fields of the run statistics (reads the audit counters).
int learned_stats(gg_run* r, gg_run_stats* st) {
  st->partial_supersteps = r->partials;
  st->selected_total = r->selected_total;
  st->audit_positives = st->audit_hits = 0;
  st->audit_selected = r->audit_selected;
  if (r->g->lws && r->pol.kind == GG_POLICY_LEARNED && r->pol.audit) {
    unsigned long long h[2] = {0, 0};
    GG_HIP(hipMemcpyAsync(h, r->g->audit, sizeof(h), hipMemcpyDeviceToHost, r->g->stream));
    GG_HIP(hipStreamSynchronize(r->g->stream));
    st->audit_positives = (int64_t)h[0];
    st->audit_hits = (int64_t)h[1];
  }
  return GG_OK;
}

// ---- run state (checkpoint / resume) --------------------------------------
//
// Blob layout: StateHeader, then the values of iteration `iter` (PR/PPR: the
// binary32 contributions the next iteration gathers, then the binary32
// values when they were materialised; SSSP/CC: the uint32 values), then the
// edge flags as ceil(m/32) words when the scheme has flags. Everything else a
// run carries (packed active edges, bins, frontier lists) is derived from
// these on import; the frontier restarts as unknown, so the first resumed
// SSSP/CC iteration runs dense, which changes no value.
struct StateHeader {
  uint32_t magic, version;
  int32_t app, kind, n, n_parts;
  int64_t m;
  int32_t iter, done, has_x, has_bits;
  double sigma, theta, damping;
  uint64_t seed;
  int32_t alpha, influence, mask_update, stop, iters, max_iters, source, dangling;
  int32_t supersteps, sparse_iters;
  int64_t edges_total, edges_processed;
  int32_t decoupled, alpha0;
  double theta0;
};
constexpr uint32_t kStateMagic = 0x53524747u;  // "GGRS"
constexpr uint32_t kStateVersion = 2;

int state_check_kind(const gg_run* r) {
  if (r->pol.kind == GG_POLICY_LEARNED || r->pol.trace)
    return fail(GG_E_UNSUPPORTED, "run state of LEARNED or traced runs (their delta features span two iterations)");
  if (r->pol.vstatus != GG_VSTATUS_NONE)
    return fail(GG_E_UNSUPPORTED, "run state of runs with vertex status (it spans two iterations)");
  if (active_degree_run(r)) return fail(GG_E_UNSUPPORTED, "run state of runs with the ACTIVE out-degree");
  if (r->p.app == GG_APP_BP) return fail(GG_E_UNSUPPORTED, "run state of BP runs");
  return GG_OK;
}

int64_t state_bytes(const gg_run* r, bool has_x) {
  const gg_graph* g = r->g;
  int64_t b = (int64_t)sizeof(StateHeader) + 4 * (int64_t)g->n;
  if (has_x) b += 4 * (int64_t)g->n;
  if (r->pol.kind != GG_POLICY_EXACT) b += 4 * ((g->m + 31) / 32);
  return b;
}

bool state_has_x(const gg_run* r) { return is_pr(r->p.app) && r->iter > 0 && r->x_valid; }

int run_state_size(gg_run* r, int64_t* bytes) {
  GG_TRY(state_check_kind(r));
  *bytes = state_bytes(r, state_has_x(r));
  return GG_OK;
}

int run_export_state(gg_run* r, void* buf, int64_t bytes) {
  GG_TRY(state_check_kind(r));
  gg_graph* g = r->g;
  const bool has_x = state_has_x(r);
  if (bytes != state_bytes(r, has_x)) return fail(GG_E_INVAL, "state buffer size differs from gg_run_state_size");
  GG_TRY(check_hub_sync(g));
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kStateMagic;
  h.version = kStateVersion;
  h.app = r->p.app;
  h.kind = r->pol.kind;
  h.n = g->n;
  h.n_parts = g->n_parts;
  h.m = g->m;
  h.iter = r->iter;
  h.done = r->done ? 1 : 0;
  h.has_x = has_x ? 1 : 0;
  h.has_bits = r->pol.kind != GG_POLICY_EXACT ? 1 : 0;
  h.sigma = r->sigma;
  h.theta = r->pol.theta;
  h.damping = r->p.damping;
  h.seed = r->pol.seed;
  h.alpha = r->pol.alpha;
  h.influence = r->pol.influence;
  h.mask_update = r->pol.mask_update;
  h.stop = r->pol.stop;
  h.iters = r->p.iters;
  h.max_iters = r->p.max_iters;
  h.source = r->p.source;
  h.dangling = r->p.dangling;
  h.supersteps = r->supersteps;
  h.sparse_iters = r->sparse_iters;
  h.edges_total = r->edges_total;
  h.edges_processed = r->edges_processed;
  h.decoupled = r->pol.decoupled;
  h.alpha0 = r->pol.alpha0;
  h.theta0 = r->pol.theta0;
  char* p = (char*)buf;
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  const size_t vb = 4 * (size_t)g->n;
  const void* vals = is_pr(r->p.app) ? (const void*)g->c[r->cur] : (const void*)g->xu[r->cur];
  if (vb) GG_HIP(hipMemcpyAsync(p, vals, vb, hipMemcpyDeviceToHost, g->stream));
  p += vb;
  if (has_x && vb) GG_HIP(hipMemcpyAsync(p, g->xout, vb, hipMemcpyDeviceToHost, g->stream));
  if (has_x) p += vb;
  const size_t wb = 4 * (size_t)((g->m + 31) / 32);
  if (h.has_bits && wb) GG_HIP(hipMemcpyAsync(p, g->bits[r->bcur], wb, hipMemcpyDeviceToHost, g->stream));
  GG_HIP(hipStreamSynchronize(g->stream));
  return GG_OK;
}

int run_import_state(gg_run* r, const void* buf, int64_t bytes) {
  GG_TRY(state_check_kind(r));
  gg_graph* g = r->g;
  if (r->iter != 0) return fail(GG_E_STATE, "state can only be imported into a run that has executed no iteration");
  if (bytes < (int64_t)sizeof(StateHeader)) return fail(GG_E_INVAL, "state buffer shorter than its header");
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kStateMagic || h.version != kStateVersion) return fail(GG_E_INVAL, "not a run state of this library version");
  const bool same = h.app == r->p.app && h.kind == r->pol.kind && h.n == g->n && h.n_parts == g->n_parts &&
                    h.m == g->m && h.sigma == r->sigma && h.theta == r->pol.theta && h.damping == r->p.damping &&
                    h.seed == r->pol.seed && h.alpha == r->pol.alpha && h.influence == r->pol.influence &&
                    h.mask_update == r->pol.mask_update && h.stop == r->pol.stop && h.iters == r->p.iters &&
                    h.max_iters == r->p.max_iters && h.source == r->p.source && h.dangling == r->p.dangling &&
                    h.decoupled == r->pol.decoupled &&
                    (!h.decoupled || (h.alpha0 == r->pol.alpha0 && h.theta0 == r->pol.theta0));
  if (!same) return fail(GG_E_INVAL, "state was exported from a run with another graph shape, app, parameters or policy");
  const bool has_x = h.has_x != 0;
  if (has_x && !is_pr(r->p.app)) return fail(GG_E_INVAL, "state holds PR values for a min-type app");
  if (h.has_bits != (r->pol.kind != GG_POLICY_EXACT ? 1 : 0)) return fail(GG_E_INVAL, "state flag section mismatch");
  if (bytes != state_bytes(r, has_x)) return fail(GG_E_INVAL, "state buffer size does not match its header");
  if (h.iter < 0 || (h.iter == 0 && has_x)) return fail(GG_E_INVAL, "state iteration out of range");
  const char* p = (const char*)buf + sizeof(h);
  const size_t vb = 4 * (size_t)g->n;
  if (is_pr(r->p.app)) {
    if (vb) GG_HIP(hipMemcpyAsync(g->c[0], p, vb, hipMemcpyHostToDevice, g->stream));
    p += vb;
    if (has_x && vb) GG_HIP(hipMemcpyAsync(g->xout, p, vb, hipMemcpyHostToDevice, g->stream));
    if (has_x) p += vb;
  } else {
    // both buffers hold the values, as at the start of a run
    if (vb) {
      GG_HIP(hipMemcpyAsync(g->xu[0], p, vb, hipMemcpyHostToDevice, g->stream));
      GG_HIP(hipMemcpyAsync(g->xu[1], p, vb, hipMemcpyHostToDevice, g->stream));
    }
    p += vb;
  }
  if (h.has_bits) {
    const size_t wb = 4 * (size_t)((g->m + 31) / 32);
    if (wb) GG_HIP(hipMemcpyAsync(g->bits[0], p, wb, hipMemcpyHostToDevice, g->stream));
    GG_TRY(pack_from_bits0(g, r->p.app));
  }
  GG_HIP(hipStreamSynchronize(g->stream));
  r->cur = 0;
  r->bcur = 0;
  r->iter = h.iter;
  r->done = h.done != 0;
  r->x_valid = has_x;
  r->supersteps = h.supersteps;
  r->sparse_iters = h.sparse_iters;
  r->edges_total = h.edges_total;
  r->edges_processed = h.edges_processed;
  r->fcur = 0;
  r->front_count = -1;
  r->front_outdeg = 0;
  return GG_OK;
}

void end_run(gg_run* r) {
  if (!r) return;
  if (r->g && r->g->active_run == r) r->g->active_run = nullptr;
  delete r;
}

// Whether a whole run's iterations form a static schedule: after run_begin
// no host decision of run_step depends on device data (no superstep, no
// frontier, no readback), so the iterations can be captured once and
// replayed.
bool static_schedule(const gg_graph* g, const gg_app_params* p, const gg_correction_policy* pol) {
  return g->capture && !g->prof && is_float(p->app) &&
         (pol->kind == GG_POLICY_EXACT || pol->kind == GG_POLICY_SP || pol->kind == GG_POLICY_SMS) &&
         pol->vstatus == GG_VSTATUS_NONE && p->pr_degree == GG_DEGREE_FULL && !pol->trace;
}

template <typename T>
void key_add(std::vector<unsigned char>& k, const T& v) {
  const unsigned char* b = (const unsigned char*)&v;
  k.insert(k.end(), b, b + sizeof(T));
}

// Everything the captured kernels' arguments and grids depend on besides
// the graph's buffers (covered by gen): the run's parameters, the scheme,
// the sample (sigma, seed) and the tuning.
std::vector<unsigned char> schedule_key(const gg_graph* g, const gg_app_params* p, double sigma,
                                        const gg_correction_policy* pol) {
  std::vector<unsigned char> k;
  key_add(k, p->app);
  key_add(k, p->damping);
  key_add(k, p->iters);
  key_add(k, p->source);
  key_add(k, p->dangling);
  key_add(k, p->coupling);
  key_add(k, pol->kind);
  key_add(k, pol->alpha);
  key_add(k, pol->seed);
  key_add(k, sigma);
  key_add(k, g->tune);
  return k;
}

// Runs the iterations of a begun static-schedule run: replays the captured
// schedule when it matches, else captures the iterations on the graph's
// private stream, instantiates and launches them. The launch is ordered
// after the work already on the graph's stream and before what follows.
int run_static(gg_graph* g, gg_run* r, const gg_app_params* p, double sigma, const gg_correction_policy* pol) {
  auto& G = g->rg;
  if (!G.cs) GG_HIP(hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking));
  if (!G.ea) GG_HIP(hipEventCreateWithFlags(&G.ea, hipEventDisableTiming));
  if (!G.eb) GG_HIP(hipEventCreateWithFlags(&G.eb, hipEventDisableTiming));
  std::vector<unsigned char> key = schedule_key(g, p, sigma, pol);
  if (!(G.exec && G.gen == g->gen && G.key == key)) {
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
    hipStream_t saved = g->stream;
    g->stream = G.cs;
    int rc = GG_OK;
    hipError_t e = hipStreamBeginCapture(G.cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      g->stream = saved;
      return fail(GG_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    while (!r->done) {
      const int s = run_step(r, nullptr, false);
      if (s < 0) {
        rc = s;
        break;
      }
      if (s == 0) break;
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(G.cs, &graph);
    g->stream = saved;
    if (rc != GG_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(GG_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      G.exec = nullptr;
      return fail(GG_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    G.gen = g->gen;
    G.key = key;
    G.iter = r->iter;
    G.cur = r->cur;
    G.x_valid = r->x_valid;
    G.edges_total = r->edges_total;
    G.edges_processed = r->edges_processed;
  } else {
    r->iter = G.iter;
    r->cur = G.cur;
    r->x_valid = G.x_valid;
    r->edges_total = G.edges_total;
    r->edges_processed = G.edges_processed;
    r->done = true;
  }
  GG_HIP(hipEventRecord(G.ea, g->stream));
  GG_HIP(hipStreamWaitEvent(G.cs, G.ea, 0));
  GG_HIP(hipGraphLaunch(G.exec, G.cs));
  GG_HIP(hipEventRecord(G.eb, G.cs));
  GG_HIP(hipStreamWaitEvent(g->stream, G.eb, 0));
  return GG_OK;
}

int whole_run(gg_graph* g, const gg_app_params* p, double sigma, const gg_correction_policy* pol, void* out,
              uint32_t flags, gg_run_stats* st) {
  if (!g) return fail(GG_E_INVAL, "null graph");
  if (!out) return fail(GG_E_INVAL, "null output");
  gg_run* r = nullptr;
  GG_TRY(ensure_workspace(g));
  GG_HIP(hipEventRecord(g->ev0, g->stream));
  GG_TRY(run_begin(g, p, sigma, pol, &r));
  const bool need_changed = !is_float(p->app) && (pol->kind == GG_POLICY_EXACT || pol->stop == GG_STOP_FIXED_POINT);
  int rc = GG_OK;
  if (static_schedule(g, p, pol) && !r->done) {
    rc = run_static(g, r, p, sigma, pol);
  } else {
    while (!r->done) {
      int s = run_step(r, nullptr, need_changed);
      if (s < 0) {
        rc = s;
        break;
      }
      if (s == 0) break;
    }
  }
  if (rc == GG_OK) {
    hipError_t e = hipEventRecord(g->ev1, g->stream);
    if (e != hipSuccess) rc = fail(GG_E_DEVICE, hipGetErrorString(e));
  }
  if (rc == GG_OK) rc = run_values(r, out, flags);
  if (rc == GG_OK && st) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, g->ev0, g->ev1);
    if (e != hipSuccess) rc = fail(GG_E_DEVICE, hipGetErrorString(e));
    st->iterations = r->iter;
    st->supersteps = r->supersteps;
    st->edges_gathered = r->edges_total;
    st->active_edges = pol->kind == GG_POLICY_EXACT ? g->m : g->act.h.edges;
    st->device_ms = ms;
    st->edges_processed = r->edges_processed;
    st->sparse_iterations = r->sparse_iters;
    if (rc == GG_OK) rc = learned_stats(r, st);
  }
  end_run(r);
  return rc;
}

// ---- exact runs that allocate nothing -----------------------------------------
// Scratch of gg_exact_run_noalloc: the double-buffered vertex values, the
// dangling partial sums, the hub chunk partials and the source-segment
// partials of the gather, in one array per device that the device holds
// until the process ends. In host code the array's name is only a stand-in:
// every use goes through the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(GG_E_RANGE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GG_E_DEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return GG_OK;
}

// Byte offsets of the scratch regions of one run (each 256-byte aligned).
struct NoAllocLayout {
  size_t val[2], dpart, part_f, part_u, part_cnt, seg_part, total;
};

NoAllocLayout noalloc_layout(const gg_graph* g) {
  NoAllocLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += ((bytes > 0 ? bytes : 1) + 255) & ~(size_t)255;
    return at;
  };
  const size_t n = (size_t)g->n;
  const size_t chunks = (size_t)(g->full.h.chunks > 0 ? g->full.h.chunks : 1);
  const size_t nl = (size_t)g->full.h.wave + (size_t)g->full.h.hub;
  L.val[0] = take(n * 4);
  L.val[1] = take(n * 4);
  L.dpart = take(257 * sizeof(double));
  L.part_f = take(chunks * sizeof(double));
  L.part_u = take(chunks * sizeof(uint32_t));
  L.part_cnt = take(chunks * sizeof(int32_t));
  L.seg_part = take(g->tune.seg_enable ? (size_t)g->seg_s * (nl > 0 ? nl : 1) * sizeof(double) : 0);
  L.total = off;
  return L;
}

// Exact run of p->iters iterations over the graph's full binning, its
// per-run state in the scratch array; only enqueues work on the graph's
// stream. Nothing in the scratch needs to start at zero: every region is
// written before it is read, in every iteration.
int exact_noalloc(gg_graph* g, const gg_app_params* p, void* out, gg_run_stats* st) {
  if (!g || !p || !out) return fail(GG_E_INVAL, "null argument");
  const int app = p->app;
  if (app == GG_APP_BP) return fail(GG_E_UNSUPPORTED, "BP runs");
  if (app < GG_APP_PR || app > GG_APP_PPR) return fail(GG_E_INVAL, "unknown app");
  if (p->iters < 1) return fail(GG_E_INVAL, "iters must be >= 1");
  const bool pr = is_pr(app);
  if (pr && !(p->damping >= 0.0 && p->damping < 1.0)) return fail(GG_E_INVAL, "damping outside [0, 1)");
  if (p->dangling != GG_DANGLING_UNIFORM && p->dangling != GG_DANGLING_NONE) return fail(GG_E_INVAL, "unknown dangling");
  if ((app == GG_APP_SSSP || app == GG_APP_PPR) && (p->source < 0 || p->source >= g->n))
    return fail(GG_E_INVAL, "source out of range");
  if (app == GG_APP_SSSP && !g->wedges) return fail(GG_E_INVAL, "SSSP needs edge weights");
  if (g->n_parts > 0) return fail(GG_E_UNSUPPORTED, "graphs with parts");
  if (g->active_run) return fail(GG_E_STATE, "a run is active on this graph");
  if (!g->full_valid) return fail(GG_E_STATE, "the graph has no binning");
  const NoAllocLayout L = noalloc_layout(g);
  if (L.total > kNoAllocScratchBytes)
    return fail(GG_E_RANGE, "the run needs " + std::to_string(L.total) + " bytes of scratch, more than the " +
                                std::to_string(kNoAllocScratchBytes) + " the library holds");
  if (g->tune.seg_enable) GG_TRY(check_seg_capacity(g, g->full));
  int dev = -1;
  GG_HIP(hipGetDevice(&dev));
  if (dev != g->device) return fail(GG_E_STATE, "the current device is not the graph's device");
  unsigned char* sp = nullptr;
  GG_TRY(scratch_address(dev, &sp));
  if (st) std::memset(st, 0, sizeof(*st));
  if (g->n > 0) {
    Sweep s;
    std::memset(&s, 0, sizeof(s));
    s.n = g->n;
    s.small_max = g->tune.small_max;
    s.wave_max = g->tune.wave_max;
    s.hub_chunk = g->tune.hub_chunk;
    s.rowptr = g->rowptr;
    s.outdeg = g->outdeg;
    double* dpart = (double*)(sp + L.dpart);
    s.dangling = dpart + 256;
    s.damping = p->damping;
    s.base = (1.0 - p->damping) / (double)g->n;
    s.source = p->source;
    s.part_f = (double*)(sp + L.part_f);
    s.part_u = (uint32_t*)(sp + L.part_u);
    s.part_cnt = (int32_t*)(sp + L.part_cnt);
    set_bins(s, g->full);
    s.edges = full_edges(g, app);
    if (g->tune.seg_enable) {
      set_seg(g, s, g->seg_off_full);
      s.seg_part_f = (double*)(sp + L.seg_part);
      s.seg_part_u = (uint32_t*)(sp + L.seg_part);
    }
    float* c[2] = {(float*)(sp + L.val[0]), (float*)(sp + L.val[1])};
    uint32_t* x[2] = {(uint32_t*)(sp + L.val[0]), (uint32_t*)(sp + L.val[1])};
    if (pr) {
      GG_HIP(launch_pr_init(app, g->outdeg, g->n, p->source, nullptr, nullptr, c[0], g->stream));
      if (p->dangling == GG_DANGLING_NONE) GG_HIP(launch_fill_u32((uint32_t*)(dpart + 256), 2, 0u, g->stream));
    } else {
      GG_HIP(launch_min_init(app, g->n, p->source, x[0], g->stream));
    }
    for (int32_t i = 1; i <= p->iters; ++i) {
      const int cur = (i - 1) & 1;
      const bool last = i == p->iters;
      if (pr) {
        if (p->dangling == GG_DANGLING_UNIFORM)
          GG_HIP(launch_dangling_sum(c[cur], g->dang, nullptr, g->n_dang, dpart, dpart + 256, g->stream));
        s.c_in = c[cur];
        s.c_out = c[1 - cur];
        s.x_out = last ? (float*)out : nullptr;
      } else {
        s.x_in = x[cur];
        s.x_next = last ? (uint32_t*)out : x[1 - cur];
      }
      if (g->tune.seg_enable)
        GG_HIP(launch_gather_seg(app, g->tune.small_team, s, g->stream));
      else
        GG_HIP(launch_gather(app, g->tune.small_team, s, g->stream));
    }
  }
  if (st) {
    st->iterations = p->iters;
    st->edges_gathered = (int64_t)p->iters * g->m;
    st->edges_processed = st->edges_gathered;
    st->active_edges = g->m;
  }
  return GG_OK;
}

}  // namespace

// ---- multi-query batch --------------------------------------------------------

int ensure_batch(gg_graph* g, int32_t qp) {
  auto& B = g->batch;
  const int64_t need_val = (int64_t)g->n * qp;
  if (B.val_cap < need_val) {
    for (int i = 0; i < 3; ++i) dfree(B.buf[i]);
    B.val_cap = 0;
    for (int i = 0; i < 3; ++i) GG_TRY(dalloc(&B.buf[i], (size_t)(need_val > 0 ? need_val : 1)));
    B.val_cap = need_val;
  }
  const int64_t need_part = max_chunks(g) * (int64_t)qp;
  if (B.part_cap < need_part) {
    dfree(B.part);
    B.part_cap = 0;
    GG_TRY(dalloc(&B.part, (size_t)need_part));
    B.part_cap = need_part;
  }
  if (B.qp_cap < qp) {
    dfree(B.dpart);
    dfree(B.dang);
    dfree(B.src);
    B.qp_cap = 0;
    GG_TRY(dalloc(&B.dpart, (size_t)kBDangChunks * qp));
    GG_TRY(dalloc(&B.dang, (size_t)qp));
    GG_TRY(dalloc(&B.src, (size_t)qp));
    B.qp_cap = qp;
  }
  if (!B.ctr) GG_TRY(dalloc(&B.ctr, 4));
  if (!B.cs) GG_HIP(hipStreamCreateWithFlags(&B.cs, hipStreamNonBlocking));
  for (hipEvent_t* e : {&B.ea, &B.eb, &B.t0, &B.t1})
    if (!*e) GG_HIP(hipEventCreate(e));
  return GG_OK;
}

// Capture `body` on the batch stream into a graph, instantiate and launch it.
template <typename F>
int capture_launch(gg_graph* g, F&& body) {
  auto& B = g->batch;
  GG_HIP(hipStreamBeginCapture(B.cs, hipStreamCaptureModeThreadLocal));
  int rc = body(B.cs);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(B.cs, &graph);
  if (rc != GG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(GG_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess) e = hipGraphLaunch(exec, B.cs);
  // the executable graph is destroyed only after its work has completed
  const hipError_t es = hipStreamSynchronize(B.cs);
  if (e == hipSuccess) e = es;
  if (exec) (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(GG_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  return GG_OK;
}

int batch_run(gg_graph* g, const gg_app_params* p, int32_t nq, const int32_t* sources, double sigma,
              const gg_correction_policy* pol, void* out, uint32_t flags, gg_run_stats* st) {
  if (!g || !p || !pol || !sources || !out) return fail(GG_E_INVAL, "null argument");
  if (p->app != GG_APP_PPR && p->app != GG_APP_SSSP) return fail(GG_E_UNSUPPORTED, "batch runs support PPR and SSSP");
  if (pol->decoupled) return fail(GG_E_INVAL, "decoupled parameters belong to GG and LEARNED");
  if (pol->kind != GG_POLICY_EXACT && pol->kind != GG_POLICY_SP && pol->kind != GG_POLICY_SMS)
    return fail(GG_E_UNSUPPORTED, "batch runs support the EXACT, SP and SMS schemes");
  if (pol->kind == GG_POLICY_SMS && pol->alpha < 0) return fail(GG_E_INVAL, "alpha < 0");
  if (nq < 1 || nq > 4096) return fail(GG_E_INVAL, "n_queries outside [1, 4096]");
  if (g->n_parts > 0) return fail(GG_E_UNSUPPORTED, "batch runs on a graph with parts");
  if (!(sigma >= 0.0 && sigma <= 1.0)) return fail(GG_E_INVAL, "sample_ratio outside [0, 1]");
  if (p->app == GG_APP_SSSP && !g->wedges) return fail(GG_E_INVAL, "SSSP needs edge weights");
  if (p->app == GG_APP_PPR && !(p->damping >= 0.0 && p->damping < 1.0)) return fail(GG_E_INVAL, "bad damping");
  if (p->pr_degree != GG_DEGREE_FULL && p->pr_degree != GG_DEGREE_ACTIVE) return fail(GG_E_INVAL, "unknown pr_degree");
  if (p->pr_degree == GG_DEGREE_ACTIVE && p->app != GG_APP_PPR)
    return fail(GG_E_INVAL, "the ACTIVE out-degree is defined for PPR batches");
  for (int32_t q = 0; q < nq; ++q)
    if (sources[q] < 0 || sources[q] >= g->n) return fail(GG_E_INVAL, "source out of range");
  const bool ppr = p->app == GG_APP_PPR;
  const bool fixed = ppr || pol->kind != GG_POLICY_EXACT;
  const int32_t T = fixed ? p->iters : p->max_iters;
  if (T <= 0) return fail(GG_E_INVAL, "batch runs need at least one iteration");
  if (g->active_run) return fail(GG_E_STATE, "a run is active on this graph");
  const int32_t qp = (nq + 63) / 64 * 64;
  GG_TRY(ensure_workspace(g));
  GG_TRY(ensure_batch(g, qp));
  auto& B = g->batch;
  // stream order: graph stream -> batch stream
  GG_HIP(hipEventRecord(B.ea, g->stream));
  GG_HIP(hipStreamWaitEvent(B.cs, B.ea, 0));
  GG_HIP(hipEventRecord(B.t0, B.cs));
  std::vector<int32_t> hs(qp, -1);
  for (int32_t q = 0; q < nq; ++q) hs[q] = sources[q];
  GG_HIP(hipMemcpyAsync(B.src, hs.data(), sizeof(int32_t) * qp, hipMemcpyHostToDevice, B.cs));
  GG_HIP(hipStreamSynchronize(B.cs));
  const int app = p->app;
  // shared edge set: all edges, or the sample of ratio sigma (one mask for all queries)
  const bool approx = pol->kind != GG_POLICY_EXACT;
  // PPR with the ACTIVE out-degree: approximate iterations divide by the
  // sample's out-degree and spread the mass of the vertices without a
  // sampled out-edge, as single runs do
  const bool act_deg = ppr && approx && p->pr_degree == GG_DEGREE_ACTIVE;
  if (approx) {
    hipStream_t keep = g->stream;
    g->stream = B.cs;
    int rc = sample_and_pack(g, app, sigma, pol->seed);
    if (rc == GG_OK && act_deg) rc = active_degree(g, 0);
    g->stream = keep;
    GG_TRY(rc);
  }
  // SMS: approximate iterations 1..alpha over the sample, accurate ones after
  const bool sms = pol->kind == GG_POLICY_SMS;
  auto approx_iter = [&](int32_t i) { return approx && !(sms && i >= pol->alpha + 1); };
  const Bins& bins = approx ? g->act : g->full;
  if ((int64_t)bins.h.chunks * qp > B.part_cap || (int64_t)g->full.h.chunks * qp > B.part_cap)
    return fail(GG_E_STATE, "batch partial array too small");
  BatchSweep s;
  std::memset(&s, 0, sizeof(s));
  s.n = g->n;
  s.qp = qp;
  s.nslice = qp / 64;
  s.list = bins.list;
  s.hub_start = bins.hub_start;
  s.n_small = bins.h.small;
  s.n_wave = bins.h.wave;
  s.n_hub = bins.h.hub;
  s.n_chunks = bins.h.chunks;
  s.hub_chunk = g->tune.hub_chunk;
  s.rowptr = g->rowptr;
  s.cnt = approx ? g->act_cnt : nullptr;
  s.edges = approx ? g->act_edges : full_edges(g, app);
  s.outdeg = g->outdeg;
  s.dang = B.dang;
  s.damping = p->damping;
  s.src = B.src;
  s.changed = B.ctr;
  s.part_f = B.part;
  s.part_u = (uint32_t*)B.part;
  // the accurate-mode sweep of an SMS run
  BatchSweep sf = s;
  sf.list = g->full.list;
  sf.hub_start = g->full.hub_start;
  sf.n_small = g->full.h.small;
  sf.n_wave = g->full.h.wave;
  sf.n_hub = g->full.h.hub;
  sf.n_chunks = g->full.h.chunks;
  sf.cnt = nullptr;
  sf.edges = full_edges(g, app);
  auto sweep_for = [&](int32_t i) -> const BatchSweep& { return (sms && i >= pol->alpha + 1) ? sf : s; };
  float* C[2] = {(float*)B.buf[0], (float*)B.buf[1]};
  float* X = (float*)B.buf[2];
  uint32_t* U[2] = {(uint32_t*)B.buf[0], (uint32_t*)B.buf[1]};
  GG_HIP(launch_batch_init(app, g->n, qp, B.src, (act_deg && approx_iter(1)) ? g->odeg_act : g->outdeg, C[0], U[0],
                           U[1], B.cs));
  GG_HIP(launch_fill_u32((uint32_t*)B.ctr, 4, 0u, B.cs));
  if (ppr && p->dangling == GG_DANGLING_NONE) GG_HIP(launch_fill_u32((uint32_t*)B.dang, 2 * (int64_t)qp, 0u, B.cs));
  int32_t iters = 0;
  if (ppr) {
    // all T iterations in one captured graph
    GG_TRY(capture_launch(g, [&](hipStream_t cs) -> int {
      for (int32_t i = 1; i <= T; ++i) {
        BatchSweep t = sweep_for(i);
        t.c_in = C[(i - 1) & 1];
        t.c_out = C[i & 1];
        t.x_out = i == T ? X : nullptr;
        // contributions for iteration i + 1 divide by its out-degree
        if (act_deg && approx_iter(i + 1)) t.outdeg = g->odeg_act;
        const bool ad = act_deg && approx_iter(i);
        if (p->dangling == GG_DANGLING_UNIFORM)
          GG_HIP(launch_batch_dangling(t, ad ? g->dang_act : g->dang, ad ? g->n_dang_act : g->n_dang, B.dpart, B.dang,
                                       cs));
        GG_HIP(launch_batch_gather(app, t, cs));
      }
      return GG_OK;
    }));
    iters = T;
  } else {
    // SSSP: chunks of K iterations; without a fixed count, every iteration
    // exits early once an iteration changed nothing (device flag)
    const int K = fixed ? (T > 0 ? T : 0) : 32;
    int32_t done_iters = 0;
    while (K > 0) {
      const int32_t kk = fixed ? T : std::min(K, T - done_iters);
      if (kk <= 0) break;
      GG_TRY(capture_launch(g, [&](hipStream_t cs) -> int {
        for (int32_t i = 0; i < kk; ++i) {
          BatchSweep t = sweep_for(done_iters + i + 1);
          t.x_in = U[(done_iters + i) & 1];
          t.x_next = U[(done_iters + i + 1) & 1];
          t.done = fixed ? nullptr : B.ctr + 1;
          GG_HIP(launch_batch_gather(app, t, cs));
          if (!fixed) GG_HIP(launch_batch_done(B.ctr, B.ctr + 1, B.ctr + 2, cs));
        }
        return GG_OK;
      }));
      if (fixed) {
        iters = T;
        break;
      }
      int32_t h[3];
      GG_HIP(hipMemcpyAsync(h, B.ctr, sizeof(h), hipMemcpyDeviceToHost, B.cs));
      GG_HIP(hipStreamSynchronize(B.cs));
      done_iters += kk;
      iters = h[2];
      if (h[1] || done_iters >= T) break;
    }
  }
  GG_HIP(hipEventRecord(B.t1, B.cs));
  // values out: n rows of nq elements (drop the query padding)
  const void* src_buf = ppr ? (const void*)X : (const void*)U[iters & 1];
  const hipMemcpyKind kind = (flags & GG_OUT_HOST) ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (g->n > 0)
    GG_HIP(hipMemcpy2DAsync(out, (size_t)nq * 4, src_buf, (size_t)qp * 4, (size_t)nq * 4, (size_t)g->n, kind, B.cs));
  GG_HIP(hipEventRecord(B.eb, B.cs));
  GG_HIP(hipStreamWaitEvent(g->stream, B.eb, 0));
  GG_HIP(hipStreamSynchronize(B.cs));
  if (st) {
    float ms = 0.f;
    GG_HIP(hipEventElapsedTime(&ms, B.t0, B.t1));
    const int64_t eset = approx ? bins.h.edges : g->m;
    const int64_t n_approx = sms ? std::min<int64_t>(iters, pol->alpha) : (approx ? iters : 0);
    st->iterations = iters;
    st->supersteps = 0;
    st->edges_gathered = (eset * n_approx + g->m * ((int64_t)iters - n_approx)) * nq;
    st->active_edges = sms && iters > pol->alpha ? g->m : eset;
    st->device_ms = ms;
    st->edges_processed = st->edges_gathered;
    st->sparse_iterations = 0;
  }
  return GG_OK;
}


// ---- dynamic graphs ---------------------------------------------------------

// Device buffers that live for one call.
// Temporaries of one update, carved from one block reserved up front (one
// allocator call instead of one per array); requests beyond the reserve get
// blocks of their own. All are freed when the object goes.
struct TempBufs {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  std::vector<void*> ptrs;
  int reserve(size_t bytes) {
    GG_TRY(dalloc(&base, bytes));
    ptrs.push_back((void*)base);
    cap = bytes;
    return GG_OK;
  }
  template <typename T>
  int get(T** p, size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    if (base && bytes <= cap - used) {
      *p = (T*)(base + used);
      used += bytes;
      return GG_OK;
    }
    *p = nullptr;
    GG_TRY(dalloc(p, count));
    ptrs.push_back((void*)*p);
    return GG_OK;
  }
  ~TempBufs() {
    for (void* q : ptrs) dev_free(q);
  }
};

// Update destinations: the spare of the slot when it holds at least count
// elements, else a new block.
enum SpareSlot { kSpRowptr, kSpCol, kSpWeight, kSpWedges, kSpBits0, kSpBits1, kSpAct, kSpOrow, kSpOedge, kSpOdst,
                 kSpOsrc };

template <typename T>
int take_spare(gg_graph* g, int slot, T** p, size_t count) {
  auto& s = g->spare[slot];
  if (*p) dev_free((void*)*p);
  *p = nullptr;
  if (s.p && s.bytes >= (count ? count : 1) * sizeof(T)) {
    *p = (T*)s.p;
    s.p = nullptr;
    s.bytes = 0;
    return GG_OK;
  }
  return dalloc(p, count);
}

// A replaced array becomes the slot's spare (bytes: what it held).
void retire(gg_graph* g, int slot, void* p, size_t bytes) {
  auto& s = g->spare[slot];
  dev_free(s.p);
  s.p = p;
  s.bytes = p ? bytes : 0;
}

// Device copy of a batch array (or the caller's device pointer).
int batch_array(gg_graph* g, TempBufs& T, const int32_t* a, int64_t k, bool device, const int32_t** out) {
  *out = nullptr;
  if (k == 0 || !a) return GG_OK;
  if (device) {
    *out = a;
    return GG_OK;
  }
  int32_t* d = nullptr;
  GG_TRY(T.get(&d, (size_t)k));
  GG_HIP(hipMemcpyAsync(d, a, sizeof(int32_t) * (size_t)k, hipMemcpyHostToDevice, g->stream));
  *out = d;
  return GG_OK;
}

// Frontier of a converged exact SSSP/CC run after an update: the vertices
// flagged in g->chg, compacted into flist[r->fcur].
int seed_frontier(gg_graph* g, gg_run* r) {
  GG_HIP(launch_compact_changed(g->chg, g->outdeg, g->n, g->flist[r->fcur], g->fc, (int32_t*)g->blk_scratch, g->psum,
                                g->stream));
  FrontCounters h = {0, 0, 0};
  GG_TRY(readback(g, &h, g->fc, sizeof(h)));
  r->front_count = h.count;
  r->front_outdeg = h.outdeg_sum;
  return GG_OK;
}

// Applies an update batch to g (and to the active run r, when given). Every
// check that can fail on the caller's input runs before anything changes.
int update_graph(gg_graph* g, const gg_update_batch* b, gg_run* r, int32_t more, uint8_t* reset_host) {
  if (!b) return fail(GG_E_INVAL, "null batch");
  if (b->n_delete < 0 || b->n_insert < 0) return fail(GG_E_INVAL, "negative batch size");
  if (b->n_delete >= ((int64_t)1 << 31) || b->n_insert >= ((int64_t)1 << 31))
    return fail(GG_E_RANGE, "a batch list holds 2^31 entries or more");
  if (b->n_delete > 0 && (!b->del_src || !b->del_dst)) return fail(GG_E_INVAL, "null deletion arrays");
  if (b->n_insert > 0 && (!b->ins_src || !b->ins_dst)) return fail(GG_E_INVAL, "null insertion arrays");
  const bool weighted = g->weight != nullptr;
  if (b->n_insert > 0 && weighted != (b->ins_weight != nullptr))
    return fail(GG_E_INVAL, weighted ? "the graph has weights: ins_weight is required" : "the graph has no weights");
  if (!weighted && b->ins_weight) return fail(GG_E_INVAL, "the graph has no weights");
  if (!g->rows_sorted) return fail(GG_E_UNSUPPORTED, "updates need rows sorted by source");
  if (g->n_parts > 0) return fail(GG_E_UNSUPPORTED, "updates of a graph with parts");
  if (!g->full_valid) return fail(GG_E_STATE, "the graph was left unusable by a failed update");
  const int app = r ? r->p.app : -1;
  if (r) {
    if (more < 0) return fail(GG_E_INVAL, "more_iters < 0");
    if (r->pol.kind == GG_POLICY_LEARNED || r->pol.trace || r->pol.vstatus != GG_VSTATUS_NONE ||
        active_degree_run(r))
      return fail(GG_E_UNSUPPORTED, "updates of LEARNED, traced, vertex-status or ACTIVE-degree runs");
    if (r->supersteps > 0) GG_TRY(check_hub_sync(g));
  }
  const int32_t n = g->n;
  const int64_t m0 = g->m, nd = b->n_delete, ni = b->n_insert;
  const bool dev = (b->flags & GG_UPDATE_DEVICE_PTRS) != 0;
  size_t sb1 = 0, sb2 = 0;  // radix sort scratch of both key lists
  GG_HIP(sort_keys_bytes(nd, &sb1));
  GG_HIP(sort_pairs_bytes(ni, &sb2));
  TempBufs T;
  {
    // one reserve covering every temporary below, in 4-byte words plus each
    // request's alignment (m0 + ni bounds the new arc count)
    const bool out0 = g->out_built;
    const bool taint0 = r && (app == GG_APP_SSSP || app == GG_APP_CC) && r->pol.kind == GG_POLICY_EXACT &&
                        r->converged && nd > 0;
    const size_t N = (size_t)n, M = (size_t)m0, I = (size_t)ni, D = (size_t)nd;
    size_t w = 0;
    auto add = [&](size_t words) { w += words + 64; };
    if (!dev) {
      add(D);
      add(D);
      add(I);
      add(I);
      add(I);
    }
    add(1);
    add(2 * D);
    add(2 * D);
    add(2 * I);
    add(2 * I);
    add(I);
    add(I);
    add((std::max(sb1, sb2) + 3) / 4);
    if (taint0) {
      add(N);
      add(N);
      add(2);
      add(N + (M + I) / kTaintChunk + 2);
      add(N + (M + I) / kTaintChunk + 2);
    }
    add((N + 3) / 4);
    add(M);
    add(M + 1);
    add(N);
    add(std::max(M, N) / 1024 + 2);
    if (out0) {
      add(N);
      add(N);
    }
    add(N + 1);
    add(N + 1);
    add(M + I);
    add(M);
    add(M);
    if (out0) {
      add(M);
      add(M + 1);
      add(N);
      add(N);
      add(M);
    }
    if (r && is_pr(app)) add(N);
    GG_TRY(T.reserve(w * 4));
  }
  const int32_t *ds, *dd, *is, *id, *iw;
  GG_TRY(batch_array(g, T, b->del_src, nd, dev, &ds));
  GG_TRY(batch_array(g, T, b->del_dst, nd, dev, &dd));
  GG_TRY(batch_array(g, T, b->ins_src, ni, dev, &is));
  GG_TRY(batch_array(g, T, b->ins_dst, ni, dev, &id));
  GG_TRY(batch_array(g, T, weighted ? b->ins_weight : nullptr, ni, dev, &iw));
  int32_t* flags = nullptr;
  GG_TRY(T.get(&flags, 1));
  GG_HIP(launch_fill_u32((uint32_t*)flags, 1, 0u, g->stream));
  GG_HIP(launch_batch_check(ds, dd, nullptr, nd, n, flags, g->stream));
  GG_HIP(launch_batch_check(is, id, iw, ni, n, flags, g->stream));
  int32_t hf = 0;
  GG_TRY(readback(g, &hf, flags, sizeof(hf)));
  if (hf & 1) return fail(GG_E_RANGE, "a batch vertex id is outside [0, n)");
  if (hf & 2) return fail(GG_E_RANGE, "an inserted weight is outside [0, 255]");

  // sorted arc keys of both lists
  uint64_t *dk, *dks, *ik, *iks;
  int32_t *ix, *ixs;
  GG_TRY(T.get(&dk, (size_t)nd));
  GG_TRY(T.get(&dks, (size_t)nd));
  GG_TRY(T.get(&ik, (size_t)ni));
  GG_TRY(T.get(&iks, (size_t)ni));
  GG_TRY(T.get(&ix, (size_t)ni));
  GG_TRY(T.get(&ixs, (size_t)ni));
  GG_HIP(launch_arc_keys(ds, dd, nd, dk, nullptr, g->stream));
  GG_HIP(launch_arc_keys(is, id, ni, ik, ix, g->stream));
  unsigned char* stemp = nullptr;
  GG_TRY(T.get(&stemp, std::max(sb1, sb2)));
  GG_HIP(launch_sort_keys(dk, dks, nd, stemp, sb1, g->stream));
  GG_HIP(launch_sort_pairs(ik, iks, ix, ixs, ni, stemp, sb2, g->stream));

  // survivors (and, for a converged exact SSSP/CC run, the taint seeds)
  const bool min_app = r && (app == GG_APP_SSSP || app == GG_APP_CC);
  const bool taint_mode = min_app && r->pol.kind == GG_POLICY_EXACT && r->converged && nd > 0;
  // taint closure: tainted vertices (tlist, tcounts[0]) and a work list of
  // row chunks (wv, wc, tcounts[1]) of at most n + m1 / kTaintChunk entries
  int32_t *taint = nullptr, *tlist = nullptr, *tcounts = nullptr, *wv = nullptr, *wc = nullptr;
  if (taint_mode) {
    GG_TRY(T.get(&taint, (size_t)n));
    GG_TRY(T.get(&tlist, (size_t)n));
    GG_TRY(T.get(&tcounts, 2));
    const size_t wcap = (size_t)n + (size_t)(m0 + ni) / kTaintChunk + 2;
    GG_TRY(T.get(&wv, wcap));
    GG_TRY(T.get(&wc, wcap));
    GG_HIP(launch_fill_u32((uint32_t*)taint, n, 0u, g->stream));
    GG_HIP(launch_fill_u32((uint32_t*)tcounts, 2, 0u, g->stream));
  }
  int32_t *keep, *keep_ex, *scr, *od_new;
  uint8_t* rowflag = nullptr;  // per row: 1 lost edges, 2 gained edges
  GG_TRY(T.get(&rowflag, ((size_t)n + 3) / 4 * 4));
  GG_HIP(launch_fill_u32((uint32_t*)rowflag, ((int64_t)n + 3) / 4, 0u, g->stream));
  GG_TRY(T.get(&keep, (size_t)m0));
  GG_TRY(T.get(&keep_ex, (size_t)m0 + 1));
  GG_TRY(T.get(&od_new, (size_t)n));
  const int64_t big = std::max<int64_t>(m0, n);
  GG_TRY(T.get(&scr, (size_t)(big / 1024 + 2)));
  GG_HIP(launch_fill_u32((uint32_t*)keep, m0, 1u, g->stream));
  GG_HIP(launch_copy_u32((const uint32_t*)g->outdeg, (uint32_t*)od_new, n, g->stream));
  GG_HIP(launch_mark_deleted(g->rowptr, g->col, g->weight, dks, nd, keep, od_new, rowflag, app,
                             taint_mode ? g->xu[r->cur] : nullptr, r ? r->p.source : 0, taint, tlist, tcounts,
                             g->stream));
  // the out-CSR, when built, is carried over rather than rebuilt
  const bool out = g->out_built;
  int32_t *ins_cnt = nullptr, *icur = nullptr;
  if (out) {
    GG_TRY(T.get(&ins_cnt, (size_t)n));
    GG_TRY(T.get(&icur, (size_t)n));
    GG_HIP(launch_fill_u32((uint32_t*)ins_cnt, n, 0u, g->stream));
    GG_HIP(launch_fill_u32((uint32_t*)icur, n, 0u, g->stream));
  }
  GG_HIP(launch_ins_outdeg(iks, ni, od_new, ins_cnt, g->stream));
  if (m0 > 0) GG_HIP(launch_scan(keep, keep_ex, (int32_t)m0, keep_ex + m0, scr, g->stream));
  else GG_HIP(launch_fill_u32((uint32_t*)keep_ex, 1, 0u, g->stream));
  int32_t kept = 0;
  GG_TRY(readback(g, &kept, keep_ex + m0, sizeof(kept)));
  const int64_t m1 = (int64_t)kept + ni;
  if (m1 >= ((int64_t)1 << 31)) return fail(GG_E_RANGE, "the updated graph would hold 2^31 arcs or more");
  const bool deleted_any = kept < m0;

  // every array the new graph needs, before anything is replaced
  int32_t *ins_rp, *len;
  GG_TRY(T.get(&ins_rp, (size_t)n + 1));
  GG_TRY(T.get(&len, (size_t)n + 1));
  int32_t *oon = nullptr, *rowid = nullptr, *new_of_old = nullptr;
  GG_TRY(T.get(&oon, (size_t)m1));
  GG_TRY(T.get(&rowid, (size_t)m0));
  GG_TRY(T.get(&new_of_old, (size_t)m0));
  struct Owned {
    int32_t *rowptr = nullptr, *col = nullptr, *weight = nullptr, *orow = nullptr, *oedge = nullptr, *odst = nullptr,
            *osrc = nullptr;
    uint32_t *wedges = nullptr, *bits0 = nullptr, *bits1 = nullptr, *act_edges = nullptr;
    ~Owned() {
      dfree(rowptr);
      dfree(col);
      dfree(weight);
      dfree(orow);
      dfree(oedge);
      dfree(odst);
      dfree(osrc);
      dfree(wedges);
      dfree(bits0);
      dfree(bits1);
      dfree(act_edges);
    }
  } nw;
  GG_TRY(take_spare(g, kSpRowptr, &nw.rowptr, (size_t)n + 1));
  GG_TRY(take_spare(g, kSpCol, &nw.col, (size_t)m1));
  if (weighted) {
    GG_TRY(take_spare(g, kSpWeight, &nw.weight, (size_t)m1));
    GG_TRY(take_spare(g, kSpWedges, &nw.wedges, (size_t)m1));
  }
  const size_t nwords = (size_t)((m1 + 31) / 32);
  if (g->ws) {
    GG_TRY(take_spare(g, kSpBits0, &nw.bits0, nwords));
    GG_TRY(take_spare(g, kSpBits1, &nw.bits1, nwords));
    GG_TRY(take_spare(g, kSpAct, &nw.act_edges, (size_t)m1));
  }
  int32_t *kout = nullptr, *kout_ex = nullptr, *obase = nullptr, *omove = nullptr, *one = nullptr;
  if (out) {
    GG_TRY(take_spare(g, kSpOrow, &nw.orow, (size_t)n + 1));
    GG_TRY(take_spare(g, kSpOedge, &nw.oedge, (size_t)m1));
    GG_TRY(take_spare(g, kSpOdst, &nw.odst, (size_t)m1));
    GG_TRY(take_spare(g, kSpOsrc, &nw.osrc, (size_t)m1));
    GG_TRY(T.get(&kout, (size_t)m0));
    GG_TRY(T.get(&kout_ex, (size_t)m0 + 1));
    GG_TRY(T.get(&obase, (size_t)n));
    GG_TRY(T.get(&omove, (size_t)n));
    GG_TRY(T.get(&one, (size_t)m0));
  }
  int32_t* od_old = nullptr;
  if (r && is_pr(app)) {
    GG_TRY(T.get(&od_old, (size_t)n));
    GG_HIP(launch_copy_u32((const uint32_t*)g->outdeg, (uint32_t*)od_old, n, g->stream));
  }

  // the new CSR
  GG_HIP(launch_ins_rows(iks, ni, n, ins_rp, g->stream));
  GG_HIP(launch_new_len(g->rowptr, keep_ex, ins_rp, n, len, rowflag, g->stream));
  if (n > 0) GG_HIP(launch_scan(len, nw.rowptr, n, nw.rowptr + n, scr, g->stream));
  else GG_HIP(launch_fill_u32((uint32_t*)nw.rowptr, 1, 0u, g->stream));
  GG_HIP(launch_row_ids(g->rowptr, n, rowid, g->stream));
  if (out) {
    if (n > 0) GG_HIP(launch_scan(od_new, nw.orow, n, nw.orow + n, scr, g->stream));
    else GG_HIP(launch_fill_u32((uint32_t*)nw.orow, 1, 0u, g->stream));
  }
  GG_HIP(launch_scatter_old(g->rowptr, rowid, g->col, g->weight, m0, keep, keep_ex, iks, ins_rp, nw.rowptr, nw.col,
                            nw.weight, oon, new_of_old, g->stream));
  GG_HIP(launch_scatter_ins(g->rowptr, g->col, keep_ex, iks, ixs, ni, ins_rp, iw, nw.rowptr, nw.col, nw.weight, oon,
                            nw.orow, ins_cnt, icur, out ? nw.oedge : nullptr, nw.odst, nw.osrc, g->stream));
  if (out && m0 > 0) {
    GG_HIP(launch_row_move(g->rowptr, nw.rowptr, rowflag, n, omove, g->stream));
    GG_HIP(launch_out_keep(g->oedge, g->odst, m0, omove, new_of_old, one, kout, g->stream));
    GG_HIP(launch_scan(kout, kout_ex, (int32_t)m0, kout_ex + m0, scr, g->stream));
    GG_HIP(launch_out_base(g->orow, nw.orow, kout_ex, n, obase, g->stream));
    GG_HIP(launch_out_compact(one, g->odst, g->osrc, m0, kout, kout_ex, obase, nw.oedge, nw.odst, nw.osrc,
                              g->stream));
  }
  const bool flags_run = r && r->pol.kind != GG_POLICY_EXACT;
  if (flags_run) GG_HIP(launch_remap_bits(g->bits[r->bcur], oon, m1, nw.bits0, g->stream));
  GG_HIP(hipStreamSynchronize(g->stream));

  // replace the CSR and everything derived from it; a failure from here on
  // leaves the graph unusable (full_valid stays false)
  g->full_valid = false;
  g->gen++;
  // the replaced arrays become the next update's spares (a borrowed CSR
  // stays the caller's)
  const size_t ob = sizeof(int32_t) * (size_t)m0, rb = sizeof(int32_t) * ((size_t)n + 1);
  const size_t bb = sizeof(uint32_t) * (size_t)((m0 + 31) / 32);
  if (g->owns_csr) {
    retire(g, kSpRowptr, g->rowptr, rb);
    retire(g, kSpCol, g->col, ob);
    retire(g, kSpWeight, g->weight, ob);
  }
  g->rowptr = g->col = g->weight = nullptr;
  g->owns_csr = true;
  g->rowptr = nw.rowptr;
  g->col = nw.col;
  g->weight = nw.weight;
  nw.rowptr = nw.col = nw.weight = nullptr;
  g->m = m1;
  if (weighted) {
    retire(g, kSpWedges, g->wedges, ob);
    g->wedges = nw.wedges;
    nw.wedges = nullptr;
    GG_HIP(launch_pack_weights(g->col, g->weight, g->m, g->wedges, g->stream));
  }
  if (g->ws) {
    retire(g, kSpBits0, g->bits[0], bb);
    retire(g, kSpBits1, g->bits[1], bb);
    retire(g, kSpAct, g->act_edges, ob);
    g->bits[0] = nw.bits0;
    g->bits[1] = nw.bits1;
    g->act_edges = nw.act_edges;
    nw.bits0 = nw.bits1 = nw.act_edges = nullptr;
  }
  GG_HIP(launch_copy_u32((const uint32_t*)od_new, (uint32_t*)g->outdeg, n, g->stream));
  GG_HIP(launch_dangling_list(g->outdeg, g->n, g->dang, g->i32_scratch, (int32_t*)g->blk_scratch, g->stream));
  GG_TRY(readback(g, &g->n_dang, g->i32_scratch, sizeof(int32_t)));
  if (out) {
    retire(g, kSpOrow, g->orow, rb);
    retire(g, kSpOedge, g->oedge, ob);
    retire(g, kSpOdst, g->odst, ob);
    retire(g, kSpOsrc, g->osrc, ob);
    g->orow = nw.orow;
    g->oedge = nw.oedge;
    g->odst = nw.odst;
    g->osrc = nw.osrc;
    nw.orow = nw.oedge = nw.odst = nw.osrc = nullptr;
  }
  GG_TRY(rebin_full(g));
  if (g->ws) GG_TRY(ensure_parts(g));
  g->full_valid = true;
  if (!r) return GG_OK;

  // the run continues on the new graph
  if (flags_run) {
    r->bcur = 0;
    GG_TRY(pack_from_bits0(g, app));
  }
  if (is_pr(app)) GG_HIP(launch_rescale_contrib(g->c[r->cur], od_old, g->outdeg, n, g->stream));
  // reset vertices for reset_host, written only once the update has
  // succeeded: the tainted list, or every vertex after a restart
  std::vector<int32_t> reset_list;
  bool reset_all = false;
  if (min_app) {
    const bool frontier = g->tune.frontier_enable != 0;
    r->front_count = -1;
    r->front_outdeg = 0;
    if (deleted_any && taint_mode) {
      // closure of the seeds along supporting out-edges of the new graph,
      // level by level over chunks of the out-rows
      GG_TRY(ensure_out(g));
      int32_t c2[2] = {0, 0};
      GG_TRY(readback(g, c2, tcounts, sizeof(c2)));
      GG_HIP(launch_row_chunks(tlist, c2[0], g->orow, wv, wc, tcounts + 1, g->stream));
      int32_t lo = 0;
      GG_TRY(readback(g, c2, tcounts, sizeof(c2)));
      while (lo < c2[1]) {
        const int32_t hi = c2[1];
        GG_HIP(launch_taint_push(wv, wc, lo, hi, g->orow, g->oedge, g->odst, g->weight, app, g->xu[r->cur],
                                 r->p.source, taint, tlist, tcounts, g->stream));
        lo = hi;
        GG_TRY(readback(g, c2, tcounts, sizeof(c2)));
      }
      const int32_t hi = c2[0];  // tainted vertices
      GG_HIP(launch_taint_reset(tlist, hi, app, r->p.source, g->xu[0], g->xu[1], g->stream));
      if (frontier) {
        GG_HIP(launch_fill_u32((uint32_t*)g->chg, ((int64_t)n + 3) / 4, 0u, g->stream));
        // the in-rows of the reset vertices, again as chunks
        GG_HIP(launch_fill_u32((uint32_t*)(tcounts + 1), 1, 0u, g->stream));
        GG_HIP(launch_row_chunks(tlist, hi, g->rowptr, wv, wc, tcounts + 1, g->stream));
        GG_TRY(readback(g, c2, tcounts, sizeof(c2)));
        GG_HIP(launch_mark_in_neighbors(wv, wc, c2[1], g->rowptr, g->col, g->chg, g->stream));
        GG_HIP(launch_mark_sources(iks, ni, g->chg, g->stream));
        GG_TRY(seed_frontier(g, r));
      }
      if (reset_host && hi > 0) {
        reset_list.resize((size_t)hi);
        GG_HIP(hipMemcpyAsync(reset_list.data(), tlist, sizeof(int32_t) * (size_t)hi, hipMemcpyDeviceToHost,
                              g->stream));
        GG_HIP(hipStreamSynchronize(g->stream));
      }
    } else if (deleted_any) {
      // any other run restarts from its initial values
      GG_HIP(launch_min_init(app, n, r->p.source, g->xu[0], g->stream));
      GG_HIP(launch_min_init(app, n, r->p.source, g->xu[1], g->stream));
      reset_all = true;
    } else if (r->pol.kind == GG_POLICY_EXACT && r->converged && frontier) {
      // insertions only: a push from their sources
      GG_TRY(ensure_out(g));
      GG_HIP(launch_fill_u32((uint32_t*)g->chg, ((int64_t)n + 3) / 4, 0u, g->stream));
      GG_HIP(launch_mark_sources(iks, ni, g->chg, g->stream));
      GG_TRY(seed_frontier(g, r));
    }
  }
  r->converged = false;
  const bool fixed_iters = is_float(app) || (r->pol.kind != GG_POLICY_EXACT && r->pol.stop == GG_STOP_FIXED_ITERS);
  if (fixed_iters) {
    if (r->p.iters < r->iter) r->p.iters = r->iter;
    r->p.iters += more;
    r->done = r->iter >= r->p.iters;
  } else {
    if (r->p.max_iters < r->iter) r->p.max_iters = r->iter;
    r->p.max_iters = (int32_t)std::min<int64_t>((int64_t)r->p.max_iters + more, INT32_MAX);
    r->done = r->iter >= r->p.max_iters;
  }
  GG_HIP(hipStreamSynchronize(g->stream));
  if (reset_host) {
    std::memset(reset_host, reset_all ? 1 : 0, (size_t)n);
    for (int32_t v : reset_list) reset_host[(size_t)v] = 1;
  }
  return GG_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

// Every entry point runs under guard(), so no C++ exception crosses the C
// ABI: a failed host allocation returns GG_E_NOMEM.
int fail_noexcept(int code, const char* msg) noexcept {
  try {
    g_err = msg;
  } catch (...) {
  }
  return code;
}

template <typename F>
int guard(F&& f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail_noexcept(GG_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail_noexcept(GG_E_DEVICE, "unexpected exception inside the library");
  }
}

extern "C" {

int gg_version(void) { return GG_VERSION; }

int gg_set_allocator(gg_alloc_fn alloc, gg_free_fn free_fn, void* ctx) {
  return guard([&]() -> int {
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(GG_E_INVAL, "alloc and free must both be set or both null");
    if (g_live_objects.load() > 0) return fail(GG_E_STATE, "graphs, networks or traces exist");
    g_alloc_fn = alloc;
    g_free_fn = free_fn;
    g_alloc_ctx = ctx;
    return GG_OK;
  });
}

int64_t gg_live_objects(void) { return g_live_objects.load(); }

const char* gg_last_error(void) { return g_err.c_str(); }

int gg_graph_load_csr(const gg_csr_desc* d, void* hip_stream, gg_graph** out) {
  return guard([&]() -> int {
    if (!d || !out) return fail(GG_E_INVAL, "null argument");
    *out = nullptr;
    if (d->n < 0 || d->m < 0) return fail(GG_E_RANGE, "negative n or m");
    if (d->m >= ((int64_t)1 << 31)) return fail(GG_E_RANGE, "m must be < 2^31");
    if (d->n >= INT32_MAX) return fail(GG_E_RANGE, "n must be < 2^31 - 1");
    if (!d->rowptr || (d->m > 0 && !d->col)) return fail(GG_E_INVAL, "null rowptr or col");
    if (d->weight && d->n > (1 << 24)) return fail(GG_E_RANGE, "weighted graphs need n <= 2^24");
    gg_graph* g = new (std::nothrow) gg_graph();
    if (!g) return fail(GG_E_NOMEM, "host allocation failed");
    g->n = d->n;
    g->m = d->m;
    g->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&g->device) != hipSuccess) {
      (void)hipGetLastError();
      delete g;
      return fail(GG_E_DEVICE, "no current device");
    }
    const size_t n = (size_t)d->n, m = (size_t)d->m;
    int rc = GG_OK;
    auto bail = [&](int code) {
      free_graph(g);
      return code;
    };
    if (hipHostMalloc(&g->pin, kPinBytes, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
      void* dp = nullptr;
      if (hipHostGetDevicePointer(&dp, g->pin, 0) == hipSuccess) {
        g->pin_dev = (uint32_t*)dp;
        std::memset(g->pin, 0, kPinBytes);
      } else {
        (void)hipGetLastError();
      }
    } else {
      (void)hipGetLastError();
      g->pin = nullptr;
      if (hipHostMalloc(&g->pin, kPinBytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        g->pin = nullptr;
        return bail(fail(GG_E_NOMEM, "pinned readback buffer"));
      }
    }
    if (d->flags & GG_CSR_DEVICE_PTRS) {
      g->owns_csr = false;
      g->rowptr = const_cast<int32_t*>(d->rowptr);
      g->col = const_cast<int32_t*>(d->col);
      g->weight = const_cast<int32_t*>(d->weight);
    } else {
      g->owns_csr = true;
      if ((rc = dalloc(&g->rowptr, n + 1)) != GG_OK) return bail(rc);
      if ((rc = dalloc(&g->col, m)) != GG_OK) return bail(rc);
      hipError_t e = hipMemcpyAsync(g->rowptr, d->rowptr, (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, g->stream);
      if (e == hipSuccess && m) e = hipMemcpyAsync(g->col, d->col, m * sizeof(int32_t), hipMemcpyHostToDevice, g->stream);
      if (e == hipSuccess && d->weight) {
        if ((rc = dalloc(&g->weight, m)) != GG_OK) return bail(rc);
        if (m) e = hipMemcpyAsync(g->weight, d->weight, m * sizeof(int32_t), hipMemcpyHostToDevice, g->stream);
      }
      if (e != hipSuccess) return bail(fail(GG_E_DEVICE, std::string("copy CSR: ") + hipGetErrorString(e)));
    }
    if ((rc = dalloc(&g->i32_scratch, 4)) != GG_OK) return bail(rc);
    if (!(d->flags & GG_CSR_SKIP_VALIDATE)) {
      hipError_t e = launch_validate(g->rowptr, g->col, g->weight, g->n, g->m, g->i32_scratch + 1, g->stream);
      int32_t flags = 0;
      if (e == hipSuccess)
        e = hipMemcpyAsync(&flags, g->i32_scratch + 1, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
      if (e != hipSuccess) return bail(fail(GG_E_DEVICE, std::string("validate: ") + hipGetErrorString(e)));
      if (flags & 1) return bail(fail(GG_E_RANGE, "rowptr[0] != 0 or rowptr[n] != m"));
      if (flags & 2) return bail(fail(GG_E_RANGE, "rowptr is not non-decreasing"));
      if (flags & 4) return bail(fail(GG_E_RANGE, "column index out of [0, n)"));
      if (flags & 8) return bail(fail(GG_E_RANGE, "weight outside [0, 255]"));
      // the source-segmented kernels need every row's sources in ascending order
      e = launch_rows_sorted(g->rowptr, g->col, g->n, g->i32_scratch + 1, g->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(&flags, g->i32_scratch + 1, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
      if (e != hipSuccess) return bail(fail(GG_E_DEVICE, std::string("validate: ") + hipGetErrorString(e)));
      if (flags & 16) {
        g->rows_sorted = false;
        g->tune.seg_enable = 0;
      }
    }
    const int nblk = (d->n + kBlock - 1) / kBlock;
    const size_t scratch_bytes = (size_t)(3 * nblk + 2) * sizeof(int32_t) + (size_t)(nblk + 1) * sizeof(int64_t);
    if ((rc = dalloc(&g->blk_scratch, (scratch_bytes + 7) / 8)) != GG_OK) return bail(rc);
    if ((rc = dalloc(&g->outdeg, n)) != GG_OK) return bail(rc);
    if ((rc = dalloc(&g->dang, n)) != GG_OK) return bail(rc);
    hipError_t e = launch_outdeg(g->col, g->m, g->outdeg, g->n, g->stream);
    if (e == hipSuccess) e = launch_dangling_list(g->outdeg, g->n, g->dang, g->i32_scratch, (int32_t*)g->blk_scratch,
                                                   g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&g->n_dang, g->i32_scratch, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess && d->weight) {
      if ((rc = dalloc(&g->wedges, m)) != GG_OK) return bail(rc);
      e = launch_pack_weights(g->col, g->weight, g->m, g->wedges, g->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return bail(fail(GG_E_DEVICE, std::string("load: ") + hipGetErrorString(e)));
    if ((rc = alloc_bins(g->full, g->n)) != GG_OK) return bail(rc);
    if ((rc = rebin_full(g)) != GG_OK) return bail(rc);
    g->full_valid = true;
    *out = g;
    return GG_OK;
  });
}

int gg_graph_set_stream(gg_graph* g, void* hip_stream) {
  return guard([&]() -> int {
    if (!g) return fail(GG_E_INVAL, "null graph");
    if (g->stream) GG_HIP(hipStreamSynchronize(g->stream));
    g->stream = (hipStream_t)hip_stream;
    return GG_OK;
  });
}

void gg_graph_free(gg_graph* g) {
  try {
    if (!g) return;
    if (g->active_run) end_run(g->active_run);
    free_graph(g);
  } catch (...) {
  }
}

int gg_graph_set_parts(gg_graph* g, int32_t n_parts, const int32_t* part_start_host,
                       const int32_t* part_sources_host) {
  return guard([&]() -> int {
    if (!g) return fail(GG_E_INVAL, "null graph");
    if (g->active_run) return fail(GG_E_STATE, "a run is active on this graph");
    g->gen++;
    dfree(g->part_start);
    dfree(g->part_of);
    dfree(g->part_e0);
    dfree(g->part_dstart);
    dfree(g->part_src);
    dfree(g->part_dang);
    g->n_parts = 0;
    if (n_parts == 0) return GG_OK;
    if (n_parts < 0 || !part_start_host) return fail(GG_E_INVAL, "bad part description");
    if (part_start_host[0] != 0 || part_start_host[n_parts] != g->n) return fail(GG_E_RANGE, "parts must cover [0, n)");
    for (int32_t p = 0; p < n_parts; ++p) {
      if (part_start_host[p + 1] < part_start_host[p]) return fail(GG_E_RANGE, "part starts must not decrease");
      if (part_sources_host &&
          (part_sources_host[p] < part_start_host[p] || part_sources_host[p] >= part_start_host[p + 1]))
        return fail(GG_E_RANGE, "part source outside its part");
    }
    const size_t np = (size_t)n_parts;
    GG_TRY(dalloc(&g->part_start, np + 1));
    GG_TRY(dalloc(&g->part_of, (size_t)g->n));
    GG_TRY(dalloc(&g->part_e0, np + 1));
    GG_TRY(dalloc(&g->part_dstart, np + 1));
    GG_TRY(dalloc(&g->part_dang, np * (1 + (size_t)kPartDangBlocks)));
    GG_HIP(hipMemcpyAsync(g->part_start, part_start_host, sizeof(int32_t) * (np + 1), hipMemcpyHostToDevice,
                          g->stream));
    if (part_sources_host) {
      GG_TRY(dalloc(&g->part_src, np));
      GG_HIP(hipMemcpyAsync(g->part_src, part_sources_host, sizeof(int32_t) * np, hipMemcpyHostToDevice, g->stream));
    }
    GG_HIP(launch_gather_i32(g->rowptr, g->part_start, n_parts + 1, g->part_e0, g->stream));
    GG_HIP(launch_parts_setup(g->rowptr, g->col, g->n, g->m, n_parts, g->part_start, g->part_of, g->i32_scratch + 2,
                              g->stream));
    GG_HIP(launch_parts_dangling_ranges(g->dang, g->n_dang, n_parts, g->part_start, g->part_dstart, g->stream));
    int32_t bad = 0;
    GG_HIP(hipMemcpyAsync(&bad, g->i32_scratch + 2, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
    GG_HIP(hipStreamSynchronize(g->stream));
    if (bad) {
      dfree(g->part_start);
      dfree(g->part_of);
      dfree(g->part_e0);
      dfree(g->part_dstart);
      dfree(g->part_src);
      dfree(g->part_dang);
      return fail(GG_E_RANGE, "an edge crosses parts");
    }
    g->n_parts = n_parts;
    return GG_OK;
  });
}

int gg_graph_get_tuning(const gg_graph* g, gg_tuning* out) {
  return guard([&]() -> int {
    if (!g || !out) return fail(GG_E_INVAL, "null argument");
    *out = g->tune;
    return GG_OK;
  });
}

int gg_graph_set_tuning(gg_graph* g, const gg_tuning* t) {
  return guard([&]() -> int {
    if (!g || !t) return fail(GG_E_INVAL, "null argument");
    if (!valid_tuning(*t)) return fail(GG_E_INVAL, "invalid tuning");
    if (g->active_run) return fail(GG_E_STATE, "a run is active on this graph");
    g->tune = *t;
    if (!g->rows_sorted) g->tune.seg_enable = 0;
    GG_TRY(rebin_full(g));
    if (g->ws) GG_TRY(ensure_parts(g));
    return GG_OK;
  });
}

int gg_graph_set_capture(gg_graph* g, int enable) {
  return guard([&]() -> int {
    if (!g) return fail(GG_E_INVAL, "null graph");
    if (g->active_run) return fail(GG_E_STATE, "a run is active on this graph");
    g->capture = enable != 0;
    return GG_OK;
  });
}

int gg_graph_set_wait_limit(gg_graph* g, int32_t polls) {
  return guard([&]() -> int {
    if (!g) return fail(GG_E_INVAL, "null graph");
    if (g->active_run) return fail(GG_E_STATE, "a run is active on this graph");
    g->hub_spin = polls;
    return GG_OK;
  });
}

int gg_graph_set_profiling(gg_graph* g, int enable) {
  return guard([&]() -> int {
    if (!g) return fail(GG_E_INVAL, "null graph");
    if (g->stream) GG_HIP(hipStreamSynchronize(g->stream));
    g->prof = enable != 0;
    g->recs.clear();
    g->pool_used = 0;
    return GG_OK;
  });
}

int gg_graph_get_profile(gg_graph* g, int kind, int app, gg_kernel_profile* out) {
  return guard([&]() -> int {
    if (!g || !out) return fail(GG_E_INVAL, "null argument");
    if (kind < 0 || kind > 4 || app < GG_APP_PR || app > GG_APP_BP) return fail(GG_E_INVAL, "bad kind or app");
    GG_HIP(hipStreamSynchronize(g->stream));
    gg_kernel_profile p{0, 0.0, 0.0, 0};
    for (const auto& r : g->recs) {
      if (r.kind != kind || r.app != app) continue;
      float ms = 0.f;
      GG_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
      p.launches++;
      p.total_ms += ms;
      p.alg_bytes += r.bytes;
      p.edges += r.edges;
    }
    *out = p;
    return GG_OK;
  });
}

int gg_batch_run(gg_graph* g, const gg_app_params* params, int32_t n_queries, const int32_t* sources_host,
                 double sample_ratio, const gg_correction_policy* policy, void* out_values, uint32_t out_flags,
                 gg_run_stats* stats) {
  return guard([&]() -> int {
    return batch_run(g, params, n_queries, sources_host, sample_ratio, policy, out_values, out_flags, stats);
  });
}

// Autotuner: coordinate descent over the tuning knobs that the workload
// reads, timing the workload itself (median of reps runs after one warm-up,
// device time from the library's own events). A candidate replaces the best
// one only when it is at least 1% faster, so timing noise does not walk the
// search away from the default.
int gg_graph_autotune(gg_graph* g, const gg_app_params* params, double sample_ratio,
                      const gg_correction_policy* policy, int32_t n_queries, const int32_t* sources_host,
                      int32_t reps, gg_tuning* out_best, double* out_ms) {
  return guard([&]() -> int {
    if (!g || !params || !out_best) return fail(GG_E_INVAL, "null argument");
    if (g->active_run) return fail(GG_E_STATE, "a run is active on this graph");
    if (n_queries < 0 || (n_queries > 0 && !sources_host)) return fail(GG_E_INVAL, "bad queries");
    if (reps < 1 || reps > 64) return fail(GG_E_INVAL, "reps outside [1, 64]");
    gg_correction_policy exact;
    std::memset(&exact, 0, sizeof(exact));
    exact.kind = GG_POLICY_EXACT;
    const gg_correction_policy* pol = policy ? policy : &exact;
    const bool batch = n_queries > 0;
    const size_t elems = (size_t)(g->n > 0 ? g->n : 1) * (size_t)(batch ? n_queries : 1);
    uint32_t* out = nullptr;
    GG_TRY(dalloc(&out, elems));
    const gg_tuning start = g->tune;
    auto measure = [&](const gg_tuning& t, double* ms) -> int {
      GG_TRY(gg_graph_set_tuning(g, &t));
      std::vector<double> v;
      for (int32_t r = 0; r <= reps; ++r) {
        gg_run_stats st;
        std::memset(&st, 0, sizeof(st));
        int rc;
        if (batch)
          rc = gg_batch_run(g, params, n_queries, sources_host, sample_ratio, pol, out, 0u, &st);
        else
          rc = whole_run(g, params, pol->kind == GG_POLICY_EXACT ? 1.0 : sample_ratio, pol, out, 0u, &st);
        if (rc != GG_OK) return rc;
        if (r > 0) v.push_back(st.device_ms);
      }
      std::sort(v.begin(), v.end());
      *ms = v[v.size() / 2];
      return GG_OK;
    };
    // knob value lists; a workload only varies the knobs it reads
    const bool single = !batch;
    const bool minapp = params->app == GG_APP_SSSP || params->app == GG_APP_CC;
    struct Knob {
      int32_t gg_tuning::*field;
      std::vector<int32_t> values;
      bool used;
    };
    const Knob knobs[] = {
        {&gg_tuning::small_max, {8, 16, 32, 64}, true},
        {&gg_tuning::small_team, {4, 8, 16, 32}, single},
        {&gg_tuning::wave_max, {128, 256, 512, 1024, 2048}, true},
        {&gg_tuning::hub_chunk, {512, 1024, 2048, 4096}, true},
        {&gg_tuning::seg_vertices, {0, 1 << 17, 1 << 18, 1 << 20}, single && start.seg_enable != 0},
        {&gg_tuning::frontier_div, {4, 16, 64}, single && minapp && start.frontier_enable != 0},
    };
    gg_tuning best = start;
    double best_ms = 0.0;
    int rc = measure(best, &best_ms);
    for (int pass = 0; rc == GG_OK && pass < 2; ++pass) {
      bool moved = false;
      for (const Knob& k : knobs) {
        if (!k.used) continue;
        for (int32_t v : k.values) {
          gg_tuning t = best;
          t.*(k.field) = v;
          if (t.*(k.field) == best.*(k.field) || !valid_tuning(t)) continue;
          double ms = 0.0;
          rc = measure(t, &ms);
          if (rc != GG_OK) break;
          if (ms < 0.99 * best_ms) {
            best = t;
            best_ms = ms;
            moved = true;
          }
        }
        if (rc != GG_OK) break;
      }
      if (!moved) break;
    }
    dfree(out);
    if (rc != GG_OK) {
      const std::string msg = gg_last_error();
      (void)gg_graph_set_tuning(g, &start);
      return fail(rc, "autotune: " + msg);
    }
    GG_TRY(gg_graph_set_tuning(g, &best));
    *out_best = g->tune;
    if (out_ms) *out_ms = best_ms;
    return GG_OK;
  });
}

int gg_exact_run(gg_graph* g, const gg_app_params* params, void* out_values, uint32_t out_flags, gg_run_stats* st) {
  return guard([&]() -> int {
    gg_correction_policy pol;
    std::memset(&pol, 0, sizeof(pol));
    pol.kind = GG_POLICY_EXACT;
    return whole_run(g, params, 1.0, &pol, out_values, out_flags, st);
  });
}

int gg_exact_run_noalloc(gg_graph* g, const gg_app_params* params, void* out_values_dev, gg_run_stats* st) {
  return guard([&]() -> int { return exact_noalloc(g, params, out_values_dev, st); });
}

int gg_approx_run(gg_graph* g, const gg_app_params* params, double sample_ratio, const gg_correction_policy* policy,
                  void* out_values, uint32_t out_flags, gg_run_stats* st) {
  return guard([&]() -> int {
    return whole_run(g, params, sample_ratio, policy, out_values, out_flags, st);
  });
}

int gg_run_begin(gg_graph* g, const gg_app_params* params, double sample_ratio, const gg_correction_policy* policy,
                 gg_run** out) {
  return guard([&]() -> int {
    if (!g || !out) return fail(GG_E_INVAL, "null argument");
    *out = nullptr;
    gg_run* r = nullptr;
    GG_TRY(run_begin(g, params, sample_ratio, policy, &r));
    r->write_x_each_step = true;
    *out = r;
    return GG_OK;
  });
}

int gg_run_step(gg_run* run, gg_step_info* info) {
  return guard([&]() -> int {
    if (!run) return fail(GG_E_INVAL, "null run");
    return run_step(run, info, true);
  });
}

int gg_run_values(gg_run* run, void* out_values, uint32_t out_flags) {
  return guard([&]() -> int {
    if (!run) return fail(GG_E_INVAL, "null run");
    return run_values(run, out_values, out_flags);
  });
}

int gg_run_mask(gg_run* run, uint32_t* out_bits_host) {
  return guard([&]() -> int {
    if (!run || !out_bits_host) return fail(GG_E_INVAL, "null argument");
    gg_graph* g = run->g;
    const size_t nw = (size_t)((g->m + 31) / 32);
    if (run->pol.kind == GG_POLICY_EXACT) {
      for (size_t w = 0; w < nw; ++w) {
        const int64_t rem = g->m - (int64_t)w * 32;
        out_bits_host[w] = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
      }
      return GG_OK;
    }
    if (nw == 0) return GG_OK;
    GG_TRY(check_hub_sync(g));
    return copy_out(g, g->bits[run->bcur], out_bits_host, nw * sizeof(uint32_t), GG_OUT_HOST);
  });
}

int gg_run_vstatus(gg_run* run, uint8_t* out_host) {
  return guard([&]() -> int {
    if (!run || !out_host) return fail(GG_E_INVAL, "null argument");
    if (run->pol.vstatus == GG_VSTATUS_NONE) return fail(GG_E_STATE, "the run has no vertex status");
    gg_graph* g = run->g;
    if (g->n == 0) return GG_OK;
    return copy_out(g, g->vact, out_host, (size_t)g->n, GG_OUT_HOST);
  });
}

int gg_run_stats_get(gg_run* run, gg_run_stats* st) {
  return guard([&]() -> int {
    if (!run || !st) return fail(GG_E_INVAL, "null argument");
    st->iterations = run->iter;
    st->supersteps = run->supersteps;
    st->edges_gathered = run->edges_total;
    st->active_edges = run->pol.kind == GG_POLICY_EXACT ? run->g->m : run->g->act.h.edges;
    st->device_ms = 0.0;
    st->edges_processed = run->edges_processed;
    st->sparse_iterations = run->sparse_iters;
    return learned_stats(run, st);
  });
}

int gg_run_features(gg_run* run, uint16_t* feat_host) {
  return guard([&]() -> int {
    if (!run || !feat_host) return fail(GG_E_INVAL, "null argument");
    if (!run->have_feat) return fail(GG_E_STATE, "no features computed yet");
    gg_graph* g = run->g;
    GG_HIP(hipMemcpyAsync(feat_host, g->feat, (size_t)g->n * 16, hipMemcpyDeviceToHost, g->stream));
    GG_HIP(hipStreamSynchronize(g->stream));
    return GG_OK;
  });
}

int gg_run_selection(gg_run* run, uint8_t* sel_host, float* logits_host) {
  return guard([&]() -> int {
    if (!run) return fail(GG_E_INVAL, "null run");
    if (!run->have_sel) return fail(GG_E_STATE, "the last step made no selection");
    gg_graph* g = run->g;
    if (sel_host) GG_HIP(hipMemcpyAsync(sel_host, g->sel, (size_t)g->n, hipMemcpyDeviceToHost, g->stream));
    if (logits_host)
      GG_HIP(hipMemcpyAsync(logits_host, g->logits, (size_t)g->n * 4, hipMemcpyDeviceToHost, g->stream));
    GG_HIP(hipStreamSynchronize(g->stream));
    return GG_OK;
  });
}

int gg_run_labels(gg_run* run, uint8_t* labels_host) {
  return guard([&]() -> int {
    if (!run || !labels_host) return fail(GG_E_INVAL, "null argument");
    if (!run->have_labels) return fail(GG_E_STATE, "the last step computed no labels");
    gg_graph* g = run->g;
    GG_HIP(hipMemcpyAsync(labels_host, g->labels, (size_t)g->n, hipMemcpyDeviceToHost, g->stream));
    GG_HIP(hipStreamSynchronize(g->stream));
    return GG_OK;
  });
}

int gg_run_state_size(gg_run* run, int64_t* bytes) {
  return guard([&]() -> int {
    if (!run || !bytes) return fail(GG_E_INVAL, "null argument");
    return run_state_size(run, bytes);
  });
}

int gg_run_export_state(gg_run* run, void* state_host, int64_t bytes) {
  return guard([&]() -> int {
    if (!run || !state_host) return fail(GG_E_INVAL, "null argument");
    return run_export_state(run, state_host, bytes);
  });
}

int gg_run_import_state(gg_run* run, const void* state_host, int64_t bytes) {
  return guard([&]() -> int {
    if (!run || !state_host) return fail(GG_E_INVAL, "null argument");
    return run_import_state(run, state_host, bytes);
  });
}

void gg_run_end(gg_run* run) {
  try {
    end_run(run);
  } catch (...) {
  }
}

int gg_graph_update(gg_graph* g, const gg_update_batch* batch) {
  return guard([&]() -> int {
    if (!g) return fail(GG_E_INVAL, "null graph");
    if (g->active_run) return fail(GG_E_STATE, "a run is active on this graph: use gg_run_update");
    return update_graph(g, batch, nullptr, 0, nullptr);
  });
}

int gg_run_update(gg_run* run, const gg_update_batch* batch, int32_t more_iters, uint8_t* reset_host) {
  return guard([&]() -> int {
    if (!run) return fail(GG_E_INVAL, "null run");
    return update_graph(run->g, batch, run, more_iters, reset_host);
  });
}

int64_t gg_graph_num_arcs(const gg_graph* g) { return g ? g->m : -1; }

int gg_graph_get_csr(gg_graph* g, int32_t* rowptr_host, int32_t* col_host, int32_t* weight_host) {
  return guard([&]() -> int {
    if (!g || !rowptr_host) return fail(GG_E_INVAL, "null argument");
    if (weight_host && !g->weight) return fail(GG_E_INVAL, "the graph has no weights");
    GG_HIP(hipMemcpyAsync(rowptr_host, g->rowptr, sizeof(int32_t) * ((size_t)g->n + 1), hipMemcpyDeviceToHost,
                          g->stream));
    if (g->m > 0) {
      if (col_host)
        GG_HIP(hipMemcpyAsync(col_host, g->col, sizeof(int32_t) * (size_t)g->m, hipMemcpyDeviceToHost, g->stream));
      if (weight_host)
        GG_HIP(hipMemcpyAsync(weight_host, g->weight, sizeof(int32_t) * (size_t)g->m, hipMemcpyDeviceToHost,
                              g->stream));
    }
    GG_HIP(hipStreamSynchronize(g->stream));
    return GG_OK;
  });
}

// ---- learned correction network and traces ---------------------------------

namespace {

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double unit(uint64_t& x) { return (double)(splitmix64(x) >> 11) * (1.0 / 9007199254740992.0); }

int mlp_upload(gg_mlp* n, const float* host) {
  GG_HIP(hipMemcpyAsync(n->d.master, host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, n->stream));
  GG_HIP(launch_fill_u32((uint32_t*)n->d.m, kMlpParams, 0u, n->stream));
  GG_HIP(launch_fill_u32((uint32_t*)n->d.v, kMlpParams, 0u, n->stream));
  GG_HIP(launch_mlp_sync_bf16(n->d, n->stream));
  GG_HIP(hipStreamSynchronize(n->stream));
  n->t = 0;
  return GG_OK;
}

void mlp_release(gg_mlp* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  dfree(n->d.master);
  dfree(n->d.m);
  dfree(n->d.v);
  dfree(n->d.w1b);
  dfree(n->d.w2b);
  dfree(n->d.w3b);
  dfree(n->grad);
  dfree(n->scratch);
  dfree(n->loss);
  delete n;
}

int mlp_scratch(gg_mlp* n, int64_t samples) {
  const int64_t need = mlp_grad_scratch(samples);
  if (n->scratch_cap >= need) return GG_OK;
  dfree(n->scratch);
  n->scratch_cap = 0;
  GG_TRY(dalloc(&n->scratch, (size_t)need));
  n->scratch_cap = need;
  return GG_OK;
}

int mlp_adam(gg_mlp* n, const float* grad, float lr) {
  n->t++;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)n->t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)n->t));
  GG_HIP(launch_mlp_adam(n->d, grad, lr, c1, c2, n->stream));
  return GG_OK;
}

}  // namespace

int gg_mlp_create(void* hip_stream, uint64_t seed, gg_mlp** out) {
  return guard([&]() -> int {
    if (!out) return fail(GG_E_INVAL, "null output");
    *out = nullptr;
    std::unique_ptr<gg_mlp, void (*)(gg_mlp*)> n(new (std::nothrow) gg_mlp(), mlp_release);
    if (!n) return fail(GG_E_NOMEM, "host allocation failed");
    n->stream = (hipStream_t)hip_stream;
    GG_TRY(dalloc(&n->d.master, kMlpParams));
    GG_TRY(dalloc(&n->d.m, kMlpParams));
    GG_TRY(dalloc(&n->d.v, kMlpParams));
    GG_TRY(dalloc(&n->d.w1b, kMlpIn * kMlpHidden));
    GG_TRY(dalloc(&n->d.w2b, kMlpHidden * kMlpHidden));
    GG_TRY(dalloc(&n->d.w3b, kMlpHidden));
    GG_TRY(dalloc(&n->grad, kMlpParams + 1));
    // He-uniform weights (bound sqrt(6 / fan_in)), zero biases
    std::vector<float> h(kMlpParams, 0.0f);
    uint64_t x = seed;
    const double a1 = std::sqrt(6.0 / kMlpIn), a2 = std::sqrt(6.0 / kMlpHidden);
    for (int i = 0; i < kMlpIn * kMlpHidden; ++i) h[kMlpW1 + i] = (float)((2.0 * unit(x) - 1.0) * a1);
    for (int i = 0; i < kMlpHidden * kMlpHidden; ++i) h[kMlpW2 + i] = (float)((2.0 * unit(x) - 1.0) * a2);
    for (int i = 0; i < kMlpHidden; ++i) h[kMlpW3 + i] = (float)((2.0 * unit(x) - 1.0) * a2);
    GG_TRY(mlp_upload(n.get(), h.data()));
    *out = n.release();
    return GG_OK;
  });
}

void gg_mlp_free(gg_mlp* mlp) {
  try {
    mlp_release(mlp);
  } catch (...) {
  }
}

int gg_mlp_set_weights(gg_mlp* mlp, const float* params_host) {
  return guard([&]() -> int {
    if (!mlp || !params_host) return fail(GG_E_INVAL, "null argument");
    for (int i = 0; i < kMlpParams; ++i)
      if (!std::isfinite(params_host[i])) return fail(GG_E_INVAL, "non-finite parameter");
    return mlp_upload(mlp, params_host);
  });
}

int gg_mlp_get_weights(gg_mlp* mlp, float* params_host) {
  return guard([&]() -> int {
    if (!mlp || !params_host) return fail(GG_E_INVAL, "null argument");
    GG_HIP(hipMemcpyAsync(params_host, mlp->d.master, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, mlp->stream));
    GG_HIP(hipStreamSynchronize(mlp->stream));
    return GG_OK;
  });
}

int gg_mlp_forward(gg_mlp* mlp, const uint16_t* feat_dev, int64_t n, float* logits_dev) {
  return guard([&]() -> int {
    if (!mlp || (n > 0 && (!feat_dev || !logits_dev))) return fail(GG_E_INVAL, "null argument");
    if (n < 0) return fail(GG_E_INVAL, "n < 0");
    if (((uintptr_t)feat_dev & 7) != 0) return fail(GG_E_INVAL, "feat_dev is not 8-byte aligned");
    GG_HIP(launch_mlp_forward(mlp->d, feat_dev, n, logits_dev, nullptr, 0.0f, nullptr, nullptr, nullptr, mlp->stream));
    GG_HIP(hipStreamSynchronize(mlp->stream));
    return GG_OK;
  });
}

int gg_mlp_loss_grad(gg_mlp* mlp, const uint16_t* feat_dev, const float* label_dev, int64_t n, float pos_weight,
                     float* grad_dev) {
  return guard([&]() -> int {
    if (!mlp || !grad_dev || (n > 0 && (!feat_dev || !label_dev))) return fail(GG_E_INVAL, "null argument");
    if (n <= 0) return fail(GG_E_INVAL, "n <= 0");
    if (!(pos_weight > 0.0f)) return fail(GG_E_INVAL, "pos_weight <= 0");
    GG_TRY(mlp_scratch(mlp, n));
    GG_HIP(launch_mlp_grad(mlp->d, feat_dev, label_dev, n, pos_weight, mlp->scratch, grad_dev, mlp->stream));
    GG_HIP(hipStreamSynchronize(mlp->stream));
    return GG_OK;
  });
}

int gg_mlp_adam_step(gg_mlp* mlp, const float* grad_dev, float lr) {
  return guard([&]() -> int {
    if (!mlp || !grad_dev) return fail(GG_E_INVAL, "null argument");
    if (!(lr > 0.0f)) return fail(GG_E_INVAL, "lr <= 0");
    GG_TRY(mlp_adam(mlp, grad_dev, lr));
    GG_HIP(hipStreamSynchronize(mlp->stream));
    return GG_OK;
  });
}

int gg_mlp_train(gg_mlp* mlp, const gg_trace* trace, int32_t epochs, int32_t batch, float lr, float pos_weight,
                 uint64_t seed, float* epoch_loss_host) {
  return guard([&]() -> int {
    if (!mlp || !trace) return fail(GG_E_INVAL, "null argument");
    if (epochs < 1 || batch < 16) return fail(GG_E_INVAL, "epochs < 1 or batch < 16");
    if (!(lr > 0.0f) || !(pos_weight > 0.0f)) return fail(GG_E_INVAL, "lr and pos_weight must be > 0");
    const int64_t size = trace->size;
    if (size <= 0) return fail(GG_E_STATE, "empty trace");
    // the trace was filled on a graph's stream
    GG_HIP(hipDeviceSynchronize());
    GG_TRY(mlp_scratch(mlp, batch));
    if (mlp->loss_cap < epochs) {
      dfree(mlp->loss);
      mlp->loss_cap = 0;
      GG_TRY(dalloc(&mlp->loss, (size_t)epochs));
      mlp->loss_cap = epochs;
    }
    GG_HIP(launch_fill_u32((uint32_t*)mlp->loss, epochs, 0u, mlp->stream));
    const int64_t nb = (size + batch - 1) / batch;
    std::vector<int64_t> order((size_t)nb);
    uint64_t x = seed;
    for (int32_t e = 0; e < epochs; ++e) {
      for (int64_t b = 0; b < nb; ++b) order[(size_t)b] = b;
      for (int64_t b = nb - 1; b > 0; --b) {
        const int64_t j = (int64_t)(splitmix64(x) % (uint64_t)(b + 1));
        std::swap(order[(size_t)b], order[(size_t)j]);
      }
      for (int64_t k = 0; k < nb; ++k) {
        const int64_t b0 = order[(size_t)k] * batch;
        const int64_t bn = size - b0 < batch ? size - b0 : batch;
        GG_HIP(launch_mlp_grad(mlp->d, trace->feat + b0 * 8, trace->label + b0, bn, pos_weight, mlp->scratch, mlp->grad,
                               mlp->stream));
        GG_TRY(mlp_adam(mlp, mlp->grad, lr));
        GG_HIP(launch_add_f32(mlp->grad + kMlpParams, mlp->loss + e, mlp->stream));
      }
    }
    std::vector<float> h((size_t)epochs);
    GG_HIP(hipMemcpyAsync(h.data(), mlp->loss, sizeof(float) * epochs, hipMemcpyDeviceToHost, mlp->stream));
    GG_HIP(hipStreamSynchronize(mlp->stream));
    if (epoch_loss_host)
      for (int32_t e = 0; e < epochs; ++e) epoch_loss_host[e] = h[(size_t)e] / (float)size;
    return GG_OK;
  });
}

int gg_trace_create(int64_t capacity, gg_trace** out) {
  return guard([&]() -> int {
    if (!out) return fail(GG_E_INVAL, "null output");
    *out = nullptr;
    if (capacity < 1 || capacity > ((int64_t)1 << 34)) return fail(GG_E_INVAL, "capacity outside [1, 2^34]");
    gg_trace* t = new (std::nothrow) gg_trace();
    if (!t) return fail(GG_E_NOMEM, "host allocation failed");
    t->cap = capacity;
    int rc = dalloc(&t->feat, (size_t)capacity * 8);
    if (rc == GG_OK) rc = dalloc(&t->label, (size_t)capacity);
    if (rc == GG_OK) rc = dalloc(&t->pos, 1);
    if (rc == GG_OK && hipMemset(t->pos, 0, sizeof(unsigned long long)) != hipSuccess)
      rc = fail(GG_E_DEVICE, "trace counter reset failed");
    if (rc != GG_OK) {
      gg_trace_free(t);
      return rc;
    }
    *out = t;
    return GG_OK;
  });
}

void gg_trace_free(gg_trace* t) {
  try {
    if (!t) return;
    (void)hipDeviceSynchronize();
    dfree(t->feat);
    dfree(t->label);
    dfree(t->pos);
    delete t;
  } catch (...) {
  }
}

int gg_trace_clear(gg_trace* t) {
  return guard([&]() -> int {
    if (!t) return fail(GG_E_INVAL, "null trace");
    GG_HIP(hipDeviceSynchronize());
    GG_HIP(hipMemset(t->pos, 0, sizeof(unsigned long long)));
    t->size = t->dropped = 0;
    return GG_OK;
  });
}

int gg_trace_info(gg_trace* t, int64_t* size, int64_t* positives, int64_t* dropped) {
  return guard([&]() -> int {
    if (!t) return fail(GG_E_INVAL, "null trace");
    GG_HIP(hipDeviceSynchronize());
    unsigned long long p = 0;
    GG_HIP(hipMemcpy(&p, t->pos, sizeof(p), hipMemcpyDeviceToHost));
    if (size) *size = t->size;
    if (positives) *positives = (int64_t)p;
    if (dropped) *dropped = t->dropped;
    return GG_OK;
  });
}

int gg_trace_export(gg_trace* t, int64_t first, int64_t count, uint16_t* feat_host, float* label_host) {
  return guard([&]() -> int {
    if (!t) return fail(GG_E_INVAL, "null trace");
    if (first < 0 || count < 0 || first + count > t->size) return fail(GG_E_RANGE, "samples outside the trace");
    GG_HIP(hipDeviceSynchronize());
    if (count == 0) return GG_OK;
    if (feat_host) GG_HIP(hipMemcpy(feat_host, t->feat + first * 8, (size_t)count * 16, hipMemcpyDeviceToHost));
    if (label_host) GG_HIP(hipMemcpy(label_host, t->label + first, (size_t)count * 4, hipMemcpyDeviceToHost));
    return GG_OK;
  });
}

}  // extern "C"

// Internal interface between the host runtime (gg_runtime.hip) and the
// device kernels (gg_kernels.hip) of the GraphGuess sweep library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ggk {

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr int kBlock = 256;  // threads per workgroup of every sweep kernel
constexpr int kHubPre = 8;   // 256-edge steps of a hub chunk whose loads are issued together
constexpr int kFlatWin = 1024;  // edges staged per round of a flattened batch of short rows
constexpr int kSegWin = 2048;  // edges gathered per window of a segmented gather's flattened batch
constexpr int kPartDangBlocks = 32;  // blocks per part of the per-part dangling sums
constexpr int kHubSpinLimit = 1 << 20;  // default polls before a single-pass hub chunk gives up waiting

enum App : int { kPR = 0, kSSSP = 1, kCC = 2, kPPR = 3, kBP = 4 };

// Counts of one degree binning, on the device (filled by the rebin kernels)
// and mirrored on the host after a rebin.
struct BinCounts {
  int32_t small;   // rows processed by sub-wave teams (includes empty rows)
  int32_t wave;    // rows processed by one wavefront each
  int32_t hub;     // rows processed by workgroups, chunked
  int32_t chunks;  // total hub chunks
  int64_t edges;   // total row length (edges in the binned edge set)
  uint32_t hub_err;  // copy of a superstep's hub error word (0 unless asked for)
  uint32_t pad;
};

// A degree binning of the rows: one list, partitioned [small | wave | hub].
struct Bins {
  int32_t* list = nullptr;         // n
  int32_t* hub_start = nullptr;    // n+1: first chunk of each hub row
  BinCounts* dcounts = nullptr;    // device counts
  BinCounts h{};                   // host mirror
};

// Arguments of a sweep launch (gather-apply, superstep or pack).
struct Sweep {
  int32_t n;
  int32_t small_max, wave_max, hub_chunk;
  // binned row set
  const int32_t* list;
  const int32_t* hub_start;
  int32_t n_small, n_wave, n_hub, n_chunks;
  // edge set: row u spans edges[rowptr[u] .. rowptr[u] + len(u)), where len is
  // cnt[u] when cnt is non-null (active edges) and the in-degree otherwise
  const int32_t* rowptr;
  const int32_t* cnt;
  const uint32_t* edges;
  // PR / PPR
  const float* c_in;
  float* c_out;
  float* x_out;  // nullable: PR value (written when non-null)
  const int32_t* outdeg;
  const double* dangling;  // device scalar: dangling mass of the previous iteration
  // independent parts (block-diagonal union), nullable: PR uses each part's
  // vertex count and dangling mass part_dang[p]
  const int32_t* part_of;
  const int32_t* part_start;
  const double* part_dang;
  double damping;
  double base;  // (1 - d) / n for PR
  int32_t source;
  // SSSP / CC
  const uint32_t* x_in;
  uint32_t* x_next;
  int32_t* changed;  // device counter of changed rows (nullable: not counted)
  uint8_t* chg;      // nullable: per-vertex changed flag written by dense iterations
  // hub partial results (one per chunk)
  double* part_f;
  uint32_t* part_u;
  int32_t* part_cnt;
  // superstep
  const uint32_t* old_bits;
  uint32_t* new_bits;
  uint32_t* act_edges;   // active edge array written by supersteps / packing
  int32_t* act_cnt;      // active edge counts written by supersteps / packing
  double theta;
  uint64_t theta_q;
  int32_t mask_union;
  // source-segmented gather of the long rows (list positions
  // [n_small, n_small + n_wave + n_hub)): seg_off[s * nl + i] is the first edge
  // of long row i whose source is >= s * seg_z, for s in [0, seg_s]
  int32_t seg_s;
  int32_t seg_z;
  int32_t seg_qw;  // blocks per segment for the wavefront-bin long rows
  const int32_t* seg_off;
  double* seg_part_f;
  uint32_t* seg_part_u;
  int32_t flat_list;  // flat superstep: short rows from list[0, n_small) instead of every vertex
  const int32_t* chunk_order;  // superstep hub chunks in source-segment order (null: natural order)
  // single-pass hub chunks of the flat superstep (null: two-pass), 3 *
  // n_chunks + 2 words: [0] error word (a wait hit its spin limit), [1]
  // ticket counter, [2, 2 + 2 n_chunks) chunk totals (64-bit), then the
  // chunk counts (count + 1)
  uint32_t* hub_sync;
  int32_t hub_spin;  // polls before a hub chunk's wait gives up (<= 0: at once)
  // PR/PPR TOTAL influence: row sums of the superstep's contributions (null:
  // PREFIX, the running sum); sum_out (nullable) receives each applied row's sum
  const double* row_total;
  double* sum_out;
  // PR/PPR GG-VStatus (nullable): the apply compares each row's new value
  // with x_prev (the previous one, binary32, updated in place) and sets
  // vact[u] = |x - x_prev| > (vs_rel ? vs_eps * |x_prev| : vs_eps)
  uint8_t* vact;
  float* x_prev;
  double vs_eps;
  int32_t vs_rel;
  // BP: prior log-odds per vertex and the coupling kappa of the potential;
  // c_in / c_out hold the message log-ratios, x_out the belief log-odds
  const float* bp_prior;
  double bp_kappa;
  // SSSP/CC influence in push order: a superstep row's running minimum
  // starts at the row's own value x_in[u] instead of the identity
  int32_t push_infl;
  // gathers (nullable): rows u with skip[u] != 0 are neither gathered nor
  // applied; another launch of the same iteration computes them
  const uint8_t* skip;
};

// Segmented gather constants.
constexpr int kSegRowsPerBlock = 64;  // wavefront-bin rows per (segment, batch) block

// Arguments of a multi-query batch launch (gg_batch.hip). Values are
// vertex-major with padded query stride qp: value(u, q) = X[u * qp + q].
struct BatchSweep {
  int32_t n, qp, nslice;  // nslice = qp / 64
  const int32_t* list;
  const int32_t* hub_start;
  int32_t n_small, n_wave, n_hub, n_chunks, hub_chunk;
  const int32_t* rowptr;
  const int32_t* cnt;
  const uint32_t* edges;
  // PPR
  const float* c_in;
  float* c_out;
  float* x_out;  // nullable
  const int32_t* outdeg;
  const double* dang;  // per query dangling mass of the previous iteration
  double damping;
  const int32_t* src;  // qp sources (-1 for padding)
  // SSSP
  const uint32_t* x_in;
  uint32_t* x_next;
  int32_t* changed;
  // hub partials (chunk-major, qp per chunk)
  double* part_f;
  uint32_t* part_u;
  // early exit of captured SSSP loops (nullable)
  const int32_t* done;
};

// ---- launchers (gg_kernels.hip) -------------------------------------------
hipError_t launch_outdeg(const int32_t* col, int64_t m, int32_t* outdeg, int32_t n, hipStream_t st);
hipError_t launch_pack_weights(const int32_t* col, const int32_t* w, int64_t m, uint32_t* packed, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t st);
hipError_t launch_iota(int32_t* p, int32_t n, hipStream_t st);
hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t count, hipStream_t st);
hipError_t launch_validate(const int32_t* rowptr, const int32_t* col, const int32_t* w, int32_t n, int64_t m,
                           int32_t* flags, hipStream_t st);
// flags |= 16 when some row lists its sources out of ascending order (rowptr
// must be valid).
hipError_t launch_rows_sorted(const int32_t* rowptr, const int32_t* col, int32_t n, int32_t* flags, hipStream_t st);

// Dangling list of the graph (vertices without out-edges), in vertex order.
hipError_t launch_dangling_list(const int32_t* outdeg, int32_t n, int32_t* list, int32_t* count,
                                int32_t* blk_scratch, hipStream_t st);
// D = sum of c over the dangling list (fixed order): two stages.
hipError_t launch_dangling_sum(const float* c, const int32_t* list, const int32_t* count_dev, int32_t count,
                               double* partial, double* out, hipStream_t st);

// Degree binning. blk_scratch holds 3 * ceil(n / kBlock) int32 + ceil(n / kBlock) int64.
hipError_t launch_rebin(const int32_t* rowptr, const int32_t* cnt, int32_t n, int32_t small_max,
                        int32_t wave_max, int32_t hub_chunk, Bins& bins, void* blk_scratch, hipStream_t st, const uint8_t* rowsel = nullptr,
                        int selwant = 0, const uint32_t* hub_err = nullptr);

// BP initial messages c[u] = message of the prior log-odds prior[u].
hipError_t launch_bp_init(const float* prior, int32_t n, double kappa, float* c, hipStream_t st);
// PR/PPR initial contributions.
// part_of / part_start nullable (PR: 1/N per part when set).
hipError_t launch_pr_init(int app, const int32_t* outdeg, int32_t n, int32_t source, const int32_t* part_of,
                          const int32_t* part_start, float* c, hipStream_t st);
hipError_t launch_min_init(int app, int32_t n, int32_t source, uint32_t* x, hipStream_t st);

// Initial sampling of the edge flags: bit (e mod 32) of word e/32 is set iff
// the Philox draw of edge e is below keep (keep in [0, 2^32]).
hipError_t launch_sample_bits(int64_t m, uint64_t seed, uint64_t epoch, uint64_t keep, uint32_t* bits,
                              hipStream_t st);

// One gather-apply iteration over the binned rows (plain, no influence).
// ev0/ev1 (nullable) are recorded around the main kernel only.
hipError_t launch_gather(int app, int team, const Sweep& s, hipStream_t st, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// Superstep: accurate gather-apply plus influence, flags and repacking.
hipError_t launch_superstep(int app, int team, const Sweep& s, hipStream_t st, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);
// Superstep with flattened batches for rows of degree <= wave_max (owner
// threads walk each row in CSR order) and the chunked path for longer rows.
// Source segment (width z, nseg segments) of the first edge of each hub
// chunk of s's bins: seg_of[0, n_chunks).
hipError_t launch_chunk_seg(const Sweep& s, const int32_t* col, int32_t z, int32_t nseg, int32_t* seg_of,
                            hipStream_t st);
hipError_t launch_superstep_flat(int app, const Sweep& s, hipStream_t st, hipEvent_t ev0 = nullptr,
                                 hipEvent_t ev1 = nullptr);
// Pack the active edges selected by s.old_bits (used after the initial sampling).
hipError_t launch_pack(const Sweep& s, hipStream_t st);
// Segment offsets of the long rows of the binned edge set in s (source mask:
// 0xFFFFFF for packed SSSP edge words, else all ones).
hipError_t launch_seg_offsets(const Sweep& s, uint32_t src_mask, int32_t* seg_off, hipStream_t st);
// ---- frontier (SSSP / CC) ---------------------------------------------------
// Counters of a frontier list: [0] count, [1] spare, [2..3] int64 sum of
// out-degrees.
struct FrontCounters {
  int32_t count;
  int32_t touched;
  int64_t outdeg_sum;
};
// Exclusive scan of n int32 values (multi-block); scratch: ceil(n/1024)+1 int32.
hipError_t launch_scan(const int32_t* in, int32_t* out, int32_t n, int32_t* total, int32_t* scratch,
                       hipStream_t st);
// Out-CSR structure of an in-CSR: orow[n+1] (from outdeg), oedge[m] = in-edge
// id, odst[m] = destination row, osrc[m] = source. cursor: n int32 of scratch.
hipError_t launch_build_out(const int32_t* rowptr, const int32_t* col, int32_t n, int64_t m, const int32_t* orow,
                            int32_t* cursor, int32_t* oedge, int32_t* odst, int32_t* osrc, hipStream_t st);
// List of vertices whose chg flag is set (vertex order) with out-degree sum.
// psum: int64 scratch of max(ceil(n / kBlock), 1024) entries.
hipError_t launch_compact_changed(const uint8_t* chg, const int32_t* outdeg, int32_t n, int32_t* list,
                                  FrontCounters* fc, int32_t* blk_scratch, int64_t* psum, hipStream_t st);
// Sparse push iteration from the frontier list `front` (count on the host):
// x_next[v] = min(x_next[v], x_in[v]) for frontier v, then x_next[u] =
// min(x_next[u], x_in[v] (+ w)) over the (active, when bits is non-null)
// out-edges; touched destinations are appended to `touched` (stamp dedup),
// then the changed ones (x_next < x_in) to `next`.
// Edge-balanced: fdeg (n) and fscan (n + 1) hold the frontier out-degrees and
// their scan; front_outdeg (host) sizes the grid.
hipError_t launch_push(int app, const Sweep& s, const int32_t* front, int32_t nfront, int64_t front_outdeg,
                       const int32_t* orow, const int32_t* oedge, const int32_t* odst, const uint32_t* bits,
                       uint32_t* stamp, uint32_t epoch, int32_t* touched, int32_t* next, FrontCounters* fc,
                       int32_t* fdeg, int32_t* fscan, int32_t* scan_scratch, int64_t* psum, hipStream_t st);

// GG-VStatus active-vertex list [Alg. 2; Sec. 2.1]: dirty[u] = 1 for every
// row u that an active in-edge (bit set in bits) from a vertex of front
// reaches, edge-balanced over the list's out-edges (front_outdeg of them;
// fdeg: nfront int32, fscan: nfront + 1 int32, scan_scratch as for
// launch_scan). dirty is not cleared here.
hipError_t launch_vs_mark(const int32_t* front, int32_t nfront, int64_t front_outdeg, const int32_t* orow,
                          const int32_t* oedge, const int32_t* odst, const uint32_t* bits, int32_t* fdeg,
                          int32_t* fscan, int32_t* scan_scratch, uint8_t* dirty, hipStream_t st);

// ACTIVE out-degree of PageRank: odeg[v] = flags set among v's out-edges
// (edge e's source is col[e]; PR/PPR edge words are the sources).
hipError_t launch_active_degree(const int32_t* col, int64_t m, const uint32_t* bits, int32_t n, int32_t* odeg,
                                hipStream_t st);
// c[v] = x[v] / deg[v] (x[v] when deg[v] = 0), from binary32 values.
hipError_t launch_recontrib(const float* x, const int32_t* deg, int32_t n, float* c, hipStream_t st);

// ---- independent parts (block-diagonal union) ------------------------------
// part_of[u] for every vertex; bad |= 1 if an edge crosses parts.
hipError_t launch_parts_setup(const int32_t* rowptr, const int32_t* col, int32_t n, int64_t m, int32_t np,
                              const int32_t* part_start, int32_t* part_of, int32_t* bad, hipStream_t st);
// Range of each part in the (vertex-sorted) dangling list: dstart[np+1].
hipError_t launch_parts_dangling_ranges(const int32_t* dlist, int32_t ndang, int32_t np, const int32_t* part_start,
                                        int32_t* dstart, hipStream_t st);
// part_dang[p] = sum of c over part p's dangling vertices (fixed order);
// partial: np * kPartDangBlocks doubles of scratch.
hipError_t launch_parts_dangling_sum(const float* c, const int32_t* dlist, int32_t np, const int32_t* dstart,
                                     double* part_dang, double* partial, hipStream_t st);
// Sampling with part-local edge ids: edge e of part p draws with seed + p at
// local index e - part_e0[p].
hipError_t launch_sample_bits_parts(int64_t m, uint64_t seed, uint64_t epoch, uint64_t keep, int32_t np,
                                    const int32_t* part_e0, uint32_t* bits, hipStream_t st);
// out[i] = src[idx[i]]
hipError_t launch_gather_i32(const int32_t* src, const int32_t* idx, int32_t count, int32_t* out, hipStream_t st);
// x[src[p]] = 0 for every part source.
hipError_t launch_set_sources(const int32_t* src, int32_t count, uint32_t* x, hipStream_t st);

// ---- multi-query batch (gg_batch.hip) -----------------------------------------
// Chunks of the dangling list in a batched PPR iteration (partials of
// kBDangChunks x query slots, added in a fixed order).
constexpr int kBDangChunks = 1024;
hipError_t launch_batch_init(int app, int32_t n, int32_t qp, const int32_t* src, const int32_t* outdeg, float* c,
                             uint32_t* x0, uint32_t* x1, hipStream_t st);
hipError_t launch_batch_dangling(const BatchSweep& s, const int32_t* dlist, int32_t ndang, double* partial,
                                 double* out, hipStream_t st);
hipError_t launch_batch_gather(int app, const BatchSweep& s, hipStream_t st, hipEvent_t ev0 = nullptr,
                               hipEvent_t ev1 = nullptr);
hipError_t launch_batch_done(int32_t* changed, int32_t* done, int32_t* iters, hipStream_t st);

// Plain gather with the long rows split by source segment.
hipError_t launch_gather_seg(int app, int team, const Sweep& s, hipStream_t st, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);


// ---- learned correction: features, MLP, labels ----------------------------
constexpr int kMlpIn = 8;
constexpr int kMlpHidden = 64;
constexpr int kMlpW1 = 0;
constexpr int kMlpB1 = kMlpW1 + kMlpIn * kMlpHidden;
constexpr int kMlpW2 = kMlpB1 + kMlpHidden;
constexpr int kMlpB2 = kMlpW2 + kMlpHidden * kMlpHidden;
constexpr int kMlpW3 = kMlpB2 + kMlpHidden;
constexpr int kMlpB3 = kMlpW3 + kMlpHidden;
constexpr int kMlpParams = kMlpB3 + 1;

// Device state of the network: binary32 master parameters with their Adam
// moments, and the bfloat16 copies of the weight matrices the kernels use.
struct MlpDev {
  float* master;  // kMlpParams
  float* m;
  float* v;
  uint16_t* w1b;  // [8][64]
  uint16_t* w2b;  // [64][64]
  uint16_t* w3b;  // [64]
};

// With sel: sel[v] = logit > tau, *sel_count += |S| and, with rowptr,
// *sel_edges += the in-edges of the rows in S.
hipError_t launch_mlp_forward(const MlpDev& w, const uint16_t* feat, int64_t n, float* logits, uint8_t* sel,
                              float tau, int32_t* sel_count, const int32_t* rowptr, unsigned long long* sel_edges,
                              hipStream_t st);
// Partial-sum slots (floats) the gradient launch needs for n samples.
int64_t mlp_grad_scratch(int64_t n);
hipError_t launch_mlp_grad(const MlpDev& w, const uint16_t* feat, const float* label, int64_t n, float pos_weight,
                           float* scratch, float* grad, hipStream_t st);
hipError_t launch_mlp_adam(const MlpDev& w, const float* grad, float lr, float c1, float c2, hipStream_t st);
hipError_t launch_mlp_sync_bf16(const MlpDev& w, hipStream_t st);
hipError_t launch_feat_base(int32_t n, const int32_t* rowptr, const int32_t* outdeg, const int32_t* act_cnt,
                            uint16_t* feat, hipStream_t st);
hipError_t launch_feat_shift(int app, int32_t n, const uint32_t* now, const uint32_t* before, uint16_t* feat,
                             hipStream_t st);
hipError_t launch_labels(int app, int32_t n, const uint32_t* acc, const uint32_t* apx, float eps, const uint8_t* sel,
                         uint8_t* label_u8, float* label_f, int32_t nf, unsigned long long* audit,
                         unsigned long long* trace_pos, hipStream_t st);
hipError_t launch_add_f32(const float* src, float* dst, hipStream_t st);
hipError_t launch_sel_active(const int32_t* list, int32_t count, const int32_t* act_cnt, unsigned long long* act_sum,
                             hipStream_t st);
hipError_t launch_clear_rows(const int32_t* list, int32_t n_short, int32_t count, const int32_t* rowptr,
                             uint32_t* bits, hipStream_t st);

// ---- dynamic graphs (gg_update.hip) -----------------------------------------
// flags |= 1 for a vertex id outside [0, n), |= 2 for a weight outside [0, 255].
hipError_t launch_batch_check(const int32_t* src, const int32_t* dst, const int32_t* w, int64_t k, int32_t n,
                              int32_t* flags, hipStream_t st);
// keys[j] = (dst[j] << 32) | src[j]; idx[j] = j when idx is non-null.
hipError_t launch_arc_keys(const int32_t* src, const int32_t* dst, int64_t k, uint64_t* keys, int32_t* idx,
                           hipStream_t st);
// Temporary storage of the stable 64-bit radix sorts below.
hipError_t sort_keys_bytes(int64_t k, size_t* bytes);
hipError_t sort_pairs_bytes(int64_t k, size_t* bytes);
hipError_t launch_sort_keys(const uint64_t* in, uint64_t* out, int64_t k, void* temp, size_t bytes, hipStream_t st);
hipError_t launch_sort_pairs(const uint64_t* kin, uint64_t* kout, const int32_t* vin, int32_t* vout, int64_t k,
                             void* temp, size_t bytes, hipStream_t st);
// Row of every edge: dst[e] = u for e in [rowptr[u], rowptr[u+1]).
hipError_t launch_row_ids(const int32_t* rowptr, int32_t n, int32_t* dst, hipStream_t st);
// For every distinct sorted deletion key: keep[e] = 0 for the matching edges
// (rows sorted by source), od_new[s] decreased by their count, rowflag[d] = 1
// for a row that lost edges (rowflag: n bytes, zeroed). With x non-null,
// destinations of deleted edges that support their value are appended to
// list (count) once each (taint[v] set).
hipError_t launch_mark_deleted(const int32_t* rowptr, const int32_t* col, const int32_t* weight,
                               const uint64_t* dkeys, int64_t nd, int32_t* keep, int32_t* od_new, uint8_t* rowflag,
                               int app, const uint32_t* x, int32_t source, int32_t* taint, int32_t* list,
                               int32_t* count, hipStream_t st);
// od_new[s] and ins_cnt[s] (nullable) increased for every inserted arc s -> d.
hipError_t launch_ins_outdeg(const uint64_t* ikeys, int64_t ni, int32_t* od_new, int32_t* ins_cnt, hipStream_t st);
// ins_rp[u] (u in [0, n]) = first sorted insertion with destination >= u.
hipError_t launch_ins_rows(const uint64_t* ikeys, int64_t ni, int32_t n, int32_t* ins_rp, hipStream_t st);
// New row lengths: survivors (keep_ex: exclusive scan of keep, m+1 entries)
// plus insertions; rowflag[u] gains 2 for a row with insertions.
hipError_t launch_new_len(const int32_t* rowptr, const int32_t* keep_ex, const int32_t* ins_rp, int32_t n,
                          int32_t* len, uint8_t* rowflag, hipStream_t st);
// Merge of survivors and insertions into the new CSR (rows sorted by source,
// old edges first on equal sources); old_of_new[e'] = old edge or -1,
// new_of_old[e] = new position or -1. With noedge non-null, scatter_ins also
// places each inserted arc in the new out-CSR (after its source's surviving
// entries: orow_new[s+1] - ins_cnt[s] + its turn from icur[s], zeroed).
hipError_t launch_scatter_old(const int32_t* rowptr, const int32_t* row_of_edge, const int32_t* col,
                              const int32_t* weight, int64_t m, const int32_t* keep, const int32_t* keep_ex,
                              const uint64_t* ikeys, const int32_t* ins_rp, const int32_t* new_rp, int32_t* ncol,
                              int32_t* nweight, int32_t* old_of_new, int32_t* new_of_old, hipStream_t st);
hipError_t launch_scatter_ins(const int32_t* rowptr, const int32_t* col, const int32_t* keep_ex,
                              const uint64_t* ikeys, const int32_t* iidx, int64_t ni, const int32_t* ins_rp,
                              const int32_t* ins_w, const int32_t* new_rp, int32_t* ncol, int32_t* nweight,
                              int32_t* old_of_new, const int32_t* orow_new, const int32_t* ins_cnt, int32_t* icur,
                              int32_t* noedge, int32_t* nodst, int32_t* nosrc, hipStream_t st);
// Out-CSR carried over an update. move[u]: how row u's old edges move (the
// row shift when rowflag[u] is 0, else a marker to look edges up in
// new_of_old). Then per out-entry its new in-edge id ne[k] (-1: deleted) and
// kout[k] = 1 for a survivor; the offset of every source's survivors
// (obase[v] = orow_new[v] - kout_ex[orow_old[v]]); and their compaction into
// the new out-CSR (kout_ex: exclusive scan of kout, m+1 entries).
hipError_t launch_row_move(const int32_t* rp_old, const int32_t* rp_new, const uint8_t* rowflag, int32_t n,
                           int32_t* move, hipStream_t st);
hipError_t launch_out_keep(const int32_t* oedge, const int32_t* odst, int64_t m, const int32_t* move,
                           const int32_t* new_of_old, int32_t* ne, int32_t* kout, hipStream_t st);
hipError_t launch_out_base(const int32_t* orow_old, const int32_t* orow_new, const int32_t* kout_ex, int32_t n,
                           int32_t* obase, hipStream_t st);
hipError_t launch_out_compact(const int32_t* ne, const int32_t* odst, const int32_t* osrc, int64_t m,
                              const int32_t* kout, const int32_t* kout_ex, const int32_t* obase, int32_t* noedge,
                              int32_t* nodst, int32_t* nosrc, hipStream_t st);
// New flag bitmap: continued edges keep their flag, inserted ones are set.
hipError_t launch_remap_bits(const uint32_t* old_bits, const int32_t* old_of_new, int64_t m, uint32_t* new_bits,
                             hipStream_t st);
// PR contributions c = x / outdeg recomputed where the out-degree changed.
hipError_t launch_rescale_contrib(float* c, const int32_t* od_old, const int32_t* od_new, int32_t n, hipStream_t st);
// Taint closure over a work list of row chunks (wv[i], wc[i]): vertex and
// chunk of kTaintChunk edges of its row. row_chunks appends the chunks of the
// rows (in offsets: orow or rowptr) of list[0, count) at wcount. One round
// of the closure: the out-edges of the work entries [lo, hi) that support
// their destination taint it (appended to tlist at counts[0], its out-row
// chunks to the work list at counts[1]). Work lists hold at most
// n + m / kTaintChunk entries.
constexpr int32_t kTaintChunk = 2048;
hipError_t launch_row_chunks(const int32_t* list, int32_t count, const int32_t* offsets, int32_t* wv, int32_t* wc,
                             int32_t* wcount, hipStream_t st);
hipError_t launch_taint_push(int32_t* wv, int32_t* wc, int32_t lo, int32_t hi, const int32_t* orow,
                             const int32_t* oedge, const int32_t* odst, const int32_t* weight, int app,
                             const uint32_t* x, int32_t source, int32_t* taint, int32_t* tlist, int32_t* counts,
                             hipStream_t st);
// Initial values (SSSP: INF, 0 at the source; CC: own id) for the listed vertices, in both buffers.
hipError_t launch_taint_reset(const int32_t* list, int32_t count, int app, int32_t source, uint32_t* x0,
                              uint32_t* x1, hipStream_t st);
// chg[s] = 1 for every in-edge s -> v of the work entries (v, chunk) [0, count).
hipError_t launch_mark_in_neighbors(const int32_t* wv, const int32_t* wc, int32_t count, const int32_t* rowptr,
                                    const int32_t* col, uint8_t* chg, hipStream_t st);
// chg[s] = 1 for the source of every (sorted) inserted arc.
hipError_t launch_mark_sources(const uint64_t* ikeys, int64_t ni, uint8_t* chg, hipStream_t st);

// Small readback through mapped coherent host memory: copies `words` 32-bit
// words of src to host[1..] and then publishes seq in host[0] (system-scope
// release), after all earlier work on the stream. words <= 63.
hipError_t launch_post(const uint32_t* src, int32_t words, uint32_t* host, uint32_t seq, hipStream_t st);

}  // namespace ggk

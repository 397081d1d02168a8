// Internal interface between the host runtime (gg_runtime.hip) and the
// device kernels (gg_kernels.hip) of the GraphGuess sweep library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ggk {

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr int kBlock = 256;  // threads per workgroup of every sweep kernel

enum App : int { kPR = 0, kSSSP = 1, kCC = 2, kPPR = 3 };

// Counts of one degree binning, on the device (filled by the rebin kernels)
// and mirrored on the host after a rebin.
struct BinCounts {
  int32_t small;   // rows processed by sub-wave teams (includes empty rows)
  int32_t wave;    // rows processed by one wavefront each
  int32_t hub;     // rows processed by workgroups, chunked
  int32_t chunks;  // total hub chunks
  int64_t edges;   // total row length (edges in the binned edge set)
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
  double damping;
  double base;  // (1 - d) / n for PR
  int32_t source;
  // SSSP / CC
  const uint32_t* x_in;
  uint32_t* x_next;
  int32_t* changed;  // device counter
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
};

// Segmented gather constants.
constexpr int kSegRowsPerBlock = 64;  // wavefront-bin rows per (segment, batch) block

// ---- launchers (gg_kernels.hip) -------------------------------------------
hipError_t launch_outdeg(const int32_t* col, int64_t m, int32_t* outdeg, int32_t n, hipStream_t st);
hipError_t launch_pack_weights(const int32_t* col, const int32_t* w, int64_t m, uint32_t* packed, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t st);
hipError_t launch_iota(int32_t* p, int32_t n, hipStream_t st);
hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t count, hipStream_t st);
hipError_t launch_validate(const int32_t* rowptr, const int32_t* col, const int32_t* w, int32_t n, int64_t m,
                           int32_t* flags, hipStream_t st);

// Dangling list of the graph (vertices without out-edges), in vertex order.
hipError_t launch_dangling_list(const int32_t* outdeg, int32_t n, int32_t* list, int32_t* count,
                                int32_t* blk_scratch, hipStream_t st);
// D = sum of c over the dangling list (fixed order): two stages.
hipError_t launch_dangling_sum(const float* c, const int32_t* list, const int32_t* count_dev, int32_t count,
                               double* partial, double* out, hipStream_t st);

// Degree binning. blk_scratch holds 3 * ceil(n / kBlock) int32 + ceil(n / kBlock) int64.
hipError_t launch_rebin(const int32_t* rowptr, const int32_t* cnt, int32_t n, int32_t small_max,
                        int32_t wave_max, int32_t hub_chunk, Bins& bins, void* blk_scratch, hipStream_t st);

// PR/PPR initial contributions.
hipError_t launch_pr_init(int app, const int32_t* outdeg, int32_t n, int32_t source, float* c, hipStream_t st);
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
// Pack the active edges selected by s.old_bits (used after the initial sampling).
hipError_t launch_pack(int team, const Sweep& s, hipStream_t st);
// Segment offsets of the long rows of the binned edge set in s (source mask:
// 0xFFFFFF for packed SSSP edge words, else all ones).
hipError_t launch_seg_offsets(const Sweep& s, uint32_t src_mask, int32_t* seg_off, hipStream_t st);
// Plain gather with the long rows split by source segment.
hipError_t launch_gather_seg(int app, int team, const Sweep& s, hipStream_t st, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);

}  // namespace ggk

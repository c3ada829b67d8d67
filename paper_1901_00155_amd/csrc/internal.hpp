// internal.hpp -- shared declarations of libdiscord's kernels and host runtime.
// Not part of the public ABI (include/discord.h is).
#pragma once

#include <hip/hip_runtime.h>
#include "../../include/discord.h"
#include "spiral.hpp"

#include <cstddef>
#include <cstdint>

namespace dd {

// The device copy of the series is padded with zeros on both sides so that the
// scan kernels can read whole aligned vectors past either end without bounds
// checks; pad values never reach a valid pair (masked by the non-self rule and
// the row/column limits).
constexpr int64_t kFrontPad = 64;    // floats before t_0 (keeps t_0 256-byte aligned)
constexpr int64_t kBackPad = 2048;   // floats after t_{m-1}

constexpr int kRowGroup = 8;         // rows sharing one FP32 scan micro-tile
constexpr int kColBlock = 8;         // columns per lane in the FP32 scan micro-tile
constexpr int kColBlockSearch = 4;   // ... in a near-first early-abandon search (256-column steps)
constexpr int kWave = 64;

constexpr int kMaxWords = 256;       // |A|^w limit (eq. 9 hash fits a byte)
constexpr int kStatBlocks = 1024;    // fixed grid of the FP64 reductions (deterministic)
constexpr int kFp64Cols = 256;       // columns per block of the FP64 row rescan (one per thread)
constexpr int kFp64BatchRows = 64;   // rows per launch of the FP64 row rescan

// Packed (distance, index) keys.  Non-negative IEEE floats order like their bit
// patterns, so one 64-bit integer min/max compares distance first and index
// second.
__host__ __device__ inline uint64_t pack_min(float d, uint32_t j) {
  return (static_cast<uint64_t>(__builtin_bit_cast(uint32_t, d)) << 32) | j;
}
// For a max over rows where the lowest row must win ties, store ~i.
__host__ __device__ inline uint64_t pack_max(float d, uint32_t i) {
  return (static_cast<uint64_t>(__builtin_bit_cast(uint32_t, d)) << 32) | (0xFFFFFFFFu - i);
}
__host__ __device__ inline float key_dist(uint64_t k) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(k >> 32));
}
constexpr uint64_t kEmptyMin = ~0ull;

// Row states written by the scans.
enum RowState : int32_t { kRowUnscanned = 0, kRowFull = 1, kRowAbandoned = 2 };

// Exact result of the FP64 stage.
struct Exact {
  double d2;
  int64_t i;    // discord row
  int64_t j;    // its nearest non-self match
};

// ---- prep.hip -----------------------------------------------------------------
void launch_stats(const float* Tp, int64_t m, double* partials, double* stats, int* bad,
                  hipStream_t s);
// row_sigma: nullptr, or receives each row's standard deviation (per-window
// normalisation)
void launch_row_stats(const float* Tp, int64_t N, int n, double* row_mean, double* row_cnorm,
                      double* row_sigma, hipStream_t s);
// zmu/zsg: nullptr (the series normalised once by eq. (2)), or the row means and
// standard deviations of per-window normalisation
void launch_sax(const float* Tp, int64_t N, int n, int w, int alpha, const double* stats,
                const double* zmu, const double* zsg, int32_t* words, int32_t* hist,
                hipStream_t s);
void launch_cand(const int32_t* words, const int32_t* hist, int64_t N, int dict,
                 int32_t* flags_scratch, int32_t* wave_counts, int32_t* cand, int32_t* cand_count,
                 hipStream_t s);
void launch_csr(const int32_t* words, const int32_t* hist, int64_t N, int dict,
                int32_t* wave_counts, int32_t* offsets, int32_t* members, hipStream_t s);
int64_t csr_waves(int64_t N);
int64_t compact_waves(int64_t N);
void launch_compact_flags(const int32_t* flags, int64_t count, int32_t* seg_counts, int32_t* out,
                          int32_t* out_count, hipStream_t s);
void launch_cand_group_flags(const int32_t* cand, const int32_t* cand_count, int64_t max_cand,
                             int shift, int32_t* flags, hipStream_t s);
void launch_bucket_groups(const int32_t* offsets, const int32_t* members, int dict, int shift,
                          int32_t* counts, int32_t* goff, int32_t* groups, hipStream_t s);
// largest bucket (entries of bgrp per word) into *out
void launch_max_bucket(const int32_t* goff, int dict, int32_t* out, hipStream_t s);

// ---- scan_fp32.hip ------------------------------------------------------------
// One launch of the pair scan.  Every row group (an item of 8 rows for the FP32
// scan, of kWaves * RB blocks of 32 rows for the MFMA scan) has a column
// sequence: its word's bucket (when `words` is given; Index_Word, eq. (10)),
// then all column blocks in matrix order or in the near-first order of
// spiral.hpp.  A launch covers entries [seq_begin, seq_begin + chunks *
// seq_chunk) of every listed item's sequence, split into `chunks` consecutive
// chunks that run in parallel; when that reaches the end of an item's sequence
// the launch is final for it and its rows still live are complete, else they
// are appended to `survivors` for a later launch that resumes at the next entry.
// The work of one scan launch when the search decides it on the device: the
// control kernels (control.hip) write it from the counts the previous launches
// left, and the scan reads it instead of ScanJob's own n_groups, chunks,
// seq_begin and seq_chunk; its item list starts at groups + list_off.
struct WinDesc {
  int64_t n_groups;
  int64_t chunks;
  int64_t seq_begin;
  int64_t seq_chunk;
  int64_t list_off;
};

struct ScanJob {
  const float* Tp;            // padded series (t_0 at Tp[0])
  int32_t n;
  int64_t N;
  const int32_t* groups;      // item list (FP32: row groups; MFMA: sets of row blocks) or
                              // nullptr: items 0 .. n_groups - 1
  int64_t n_groups;           // items in the launch
  int64_t chunks;
  int64_t seq_begin;          // first sequence entry of this launch
  int64_t seq_chunk;          // entries per chunk
  // visiting order
  const int32_t* words;       // word id per row, or nullptr: no bucket in the sequence
  const int32_t* bgrp_off;    // per word: offsets into bgrp
  const int32_t* bgrp;        // bucket column blocks, ascending per word
  const int32_t* skip;        // per item: 1 = already searched, or nullptr
  int32_t near_first;         // 1: near-first order after the bucket, 0: matrix order
  int32_t precheck;           // 1: rows whose published minimum is below the best-so-far
                              //    leave before any work (later launches of a search)
  // early abandon against the best-so-far
  int32_t abandon;
  uint32_t* bsf;              // float bits of the best-so-far squared distance
  float raise_scale;          // completed rows raise bsf to
  float raise_sub;            //   max(0, (their minimum) * raise_scale - raise_sub)
  // per-window normalisation (FP32 scan): row centres c_i and scales r_i =
  // fp32(1 / sigma_i) (0: flat window), padded with zeros to N + 64; nullptr:
  // distances between raw windows
  const float* zc;
  const float* zr;
  uint32_t* alive;            // per row group: bit r set while row r is searched
  uint32_t* done;             // per item: chunks finished (reset by the last one)
  int32_t* survivors;         // items left with live rows by a non-final launch
  uint32_t* n_survivors;
  uint64_t* best;             // per row: packed (approximate distance, column) minimum
  uint64_t* pairs;            // pair distances evaluated (non-self, in range), counted in
                              // kPairSlots slots kPairStride words apart (see pair_slot)
  // nullptr: the fields above describe the launch's work and the grid covers
  // it; else the work is read from here and the launch's grid (sized for the
  // most work the descriptor can hold) strides over it
  const WinDesc* win;
  int64_t max_work;           // work items (item x chunk) the grid is sized for
};

// Reads the device-side work descriptor into J (kernels call it first).
__device__ __forceinline__ void apply_win(ScanJob& J) {
  if (J.win) {
    const WinDesc w = *J.win;
    J.n_groups = w.n_groups;
    J.chunks = w.chunks;
    J.seq_begin = w.seq_begin;
    J.seq_chunk = w.seq_chunk;
    if (J.groups) J.groups += w.list_off;
  }
}
void launch_scan_fp32(const ScanJob& J, hipStream_t s);

// The pair counter is spread over slots on cache lines of their own, chosen by
// workgroup number: device-scope atomics on one address are serialised in the
// memory system, and one counter added to by every wavefront of a launch cost
// a few per cent of the scan.  launch_sum_pairs folds the slots into one total.
constexpr int kPairSlots = 64;
constexpr int kPairStride = 16;   // 128 bytes
__device__ __forceinline__ unsigned long long* pair_slot(uint64_t* pairs) {
  return reinterpret_cast<unsigned long long*>(pairs + (blockIdx.x % kPairSlots) * kPairStride);
}
void launch_sum_pairs(const uint64_t* slots, uint64_t* total, hipStream_t s);

// ---- scan_mfma.hip ------------------------------------------------------------
// Row statistics of the split-BF16 scan (FP32, padded with zeros to N + 64):
// mu = fp32 row mean (the centre), smu = sqrt(n) (mean - series mean),
// cnorm = squared norm about the centre, r = per-window normalisation scales
// (nullptr: distances between raw windows).  The operands are built from the
// padded series (ScanJob::Tp).
struct MixedRows {
  const float* mu;
  const float* smu;
  const float* cnorm;
  const float* r;
};
constexpr int kMixedBlock = 32;      // rows per MFMA row block (one alive mask)
constexpr int kMixedItemBlocks = 4;  // row blocks per work item (one per wavefront)
constexpr int kMixedCols = 128;      // columns per step = per sequence entry
constexpr int kMixedMaxN = DISCORD_MIXED_MAX_N;  // longest window of the split-BF16 scan (128 K-steps)
// false for windows beyond kMixedMaxN
bool launch_scan_mfma(const ScanJob& J, const MixedRows& R, hipStream_t s);
// row_sigma/r32: nullptr, or per-window normalisation (see prep.hip)
void launch_row_stats32(const float* Tp, int64_t N, int n, int64_t padded, const double* row_mean,
                        const double* row_sigma, const double* stats, float* c32, float* smu32,
                        float* cn32, float* r32, hipStream_t s);

// ---- control.hip ----------------------------------------------------------------
// The loop of an early-abandon search, decided on the device.  The host
// enqueues a fixed sequence of launches (it depends only on the plan's sizes
// and options); one-thread control kernels between them turn the counts the
// scans leave behind into the next launch's work (WinDesc).  count == 0 means
// the loop is over: every later launch then finds no work.
struct SearchCtl {
  int64_t count;    // items listed for the next window (0: done)
  int64_t covered;  // sequence entries every listed item has already seen
  int64_t width;    // entries of the next window
  int64_t in_off;   // first entry of the next window's item list
  int64_t end;      // end of the current window
  int64_t k;        // items of the round's completion launch (ranked rounds)
};
struct CtlParams {
  int64_t seq_max;      // longest column sequence (entries)
  int64_t gran;         // entries per 512 columns (the chunk granule)
  int64_t target;       // work items a window launch aims at
  int64_t seed_target;  // work items the launch completing the bound-ranked items aims at
  int64_t growth;       // window growth per round
  int64_t seeds;        // ranked rounds: best-ranked items completed after each window
  int32_t near_first;   // 1: windows grow by `growth`; 0: the second window ends the sequences
  // shortest chunk (entries) of the launches that complete whole sequences
  // (Cand, bound-ranked items; 0: one granule)
  int64_t min_chunk_full;
};
// ctl := (count, 0, width, 0); cand_win (if given): the Cand launch covers the
// whole sequence of *cand_count items; bound_win (if given): the launch that
// completes bound_items items.  A series that eq. (2) rejects (bad[0] set, or
// stats[1] = sigma not > 0) ends the loop before it starts: count = 0 and both
// launches empty.
void launch_ctl_start(SearchCtl* ctl, int64_t count, int64_t width, const int32_t* cand_count,
                      WinDesc* cand_win, int64_t bound_items, WinDesc* bound_win,
                      const double* stats, const int32_t* bad, const CtlParams& P, hipStream_t s);
// the next window: entries [covered, covered + width) of the listed items;
// clears the survivor count
void launch_ctl_window(SearchCtl* ctl, WinDesc* win, uint32_t* n_surv, const CtlParams& P,
                       hipStream_t s);
// after a window: the loop ends when the sequences are done or no item has a
// live row; else the survivors are the next list and the window grows
void launch_ctl_after(SearchCtl* ctl, const uint32_t* n_surv, const CtlParams& P, hipStream_t s);
// launch_ctl_after, then launch_ctl_window, as one launch
void launch_ctl_next(SearchCtl* ctl, WinDesc* win, uint32_t* n_surv, const CtlParams& P,
                     hipStream_t s);
// ranked rounds: after the survivors were ranked, the best-ranked
// min(count, seeds) items are completed over the rest of their sequences ...
void launch_ctl_seeds(SearchCtl* ctl, WinDesc* win, const CtlParams& P, hipStream_t s);
// ... and the rest continue from the ranked list in the next window
void launch_ctl_post(SearchCtl* ctl, hipStream_t s);

// ---- bound.hip ----------------------------------------------------------------
// lb[i] <= NN(i): n times the squared gap from row i's mean to the nearest mean
// of a non-self row, at the resolution of bound_bins() bins over the range of
// the row means (range: 2 x u64, bmin/bmax: bound_bins() each, scratch)
size_t bound_bins();
void launch_row_bound(const double* row_mean, int64_t N, int n, uint64_t* range, int32_t* bmin,
                      int32_t* bmax, float* lb, hipStream_t s);
// score[t] = bits of the largest lb over item t's rows (item_rows rows each)
void launch_item_bound(const float* lb, int64_t N, int64_t item_rows, int64_t n_items,
                       uint32_t* score, hipStream_t s);
// flags[list[t]] = 1 (and flags2[list[t]] = 1, if given) for t < min(count,
// win->n_groups): the items a launch described by `win` covered (the list may
// hold fewer valid entries than count when the device decided on less work)
void launch_flag_items(const int32_t* list, int64_t count, const WinDesc* win, int32_t* flags,
                       int32_t* flags2, hipStream_t s);

// ---- rank.hip -----------------------------------------------------------------
// A descending counting sort of the *count entries of `list` (nullptr: 0, 1,
// ...) by score[k] (the bits of a non-negative float; hist is scratch of
// rank_hist_bins() entries, cleared first when clear_hist).  The count is read
// on the device; the grids are sized for max_count.
size_t rank_hist_bins();
// The *count items of `list` (item_rows consecutive rows each; alive masks per
// gsz rows) by the largest published minimum of a live row (score is scratch
// of max_count entries).
void launch_rank_groups(const int32_t* list, const int64_t* count, int64_t max_count,
                        int64_t item_rows, int gsz, const uint32_t* alive, const uint64_t* best,
                        int64_t N, uint32_t* score, uint32_t* hist, int32_t* out, hipStream_t s);
void launch_rank_scores(const int32_t* list, const int64_t* count, int64_t max_count,
                        const uint32_t* score, uint32_t* hist, int32_t* out, hipStream_t s,
                        bool clear_hist = true);

// ---- certify.hip --------------------------------------------------------------
// Fills of several buffers (32- or 64-bit elements) in one launch.
struct FillOp {
  void* p;
  int64_t count;
  uint64_t value;
  int32_t wide;   // 1: 64-bit elements, 0: 32-bit
};
constexpr int kMaxFills = 8;
struct FillList {
  int32_t n;
  FillOp op[kMaxFills];
};
void launch_fill_many(const FillOp* ops, int count, hipStream_t s);
void launch_init_u64(uint64_t* p, int64_t count, uint64_t v, hipStream_t s);
void launch_init_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);
void launch_unpack_best(const uint64_t* best, int64_t N, const uint32_t* alive, int gsz,
                        float* nn_approx, int32_t* nn_witness, int32_t* row_state,
                        uint32_t* n_abandoned, hipStream_t s);
void launch_init_alive(uint32_t* alive, int64_t G, int64_t N, int gsz, hipStream_t s);
void launch_seed_argmax(const uint64_t* best, const int32_t* row_state, int64_t N,
                        uint64_t* seed_key, hipStream_t s);
void launch_seed_row(const uint64_t* seed_key, int64_t* rows_out, hipStream_t s);
// FP64 distances of the certification.  zmu/zsg: nullptr (raw windows), or the
// row means and standard deviations of per-window normalisation.
struct ZStats {
  const double* mu;
  const double* sg;
};
// dev_count (optional): only the first min(count, *dev_count) rows are rescanned
// (a batch sized on the host, filled to a count known only on the device)
void launch_rows_nn_fp64(const float* Tp, int n, int64_t N, const int64_t* rows, int64_t count,
                         ZStats z, double* part_d, int64_t* part_j, double* out_d, int64_t* out_j,
                         hipStream_t s, const uint32_t* dev_count = nullptr);
void launch_exact_from_rows(const int64_t* rows, const double* d, const int64_t* j,
                            int64_t count, Exact* ex, hipStream_t s);
void launch_verify(const float* Tp, int n, int64_t N, ZStats z, const int32_t* nn_witness,
                   const float* nn_approx, const Exact* ex, int64_t* uncertain,
                   uint32_t* uncertain_count, uint32_t* max_rel_err_bits, hipStream_t s);
void launch_merge_exact(const int64_t* rows, const double* d, const int64_t* j, int64_t count,
                        Exact* ex, int32_t* nn_witness, hipStream_t s,
                        const uint32_t* dev_count = nullptr);

}  // namespace dd

namespace dd {
// ---- api.hip: one series prepared and searched in caller-provided device
// memory, with a plan on the stack; all work on `stream`, which it
// synchronises before returning (once: preparation and search are enqueued as
// one sequence, except for the PhiDD order, whose sequences need the bucket
// sizes on the host).  Creates no stream, event, heap object or device
// allocation; with `timed`, it takes the calling thread's pooled HIP events
// (ms_search brackets the whole sequence, ms_scan sums the scan launches).
// ERANGE if the plan does not fit in arena_bytes.
int search_series_in_arena(const float* T, int64_t m, int32_t n, const discord_opts* opts,
                           void* arena, size_t arena_bytes, hipStream_t stream,
                           discord_result* out, char* err, size_t err_len, bool timed = false);
// Sets the calling thread's error text (discord_plan_error(NULL)).
void set_thread_error(const char* fmt, ...);

// The same request run as one HIP graph: preparation and search (every
// decision of the search is taken on the device) captured from `stream` into
// a graph that `*cache` keeps, together with the plan and a pinned readback
// block.  A later call with the same series pointer, (m, n), options,
// workspace and stream replays the graph (one launch, one synchronisation);
// any other call drops the cached graph and either captures a new one
// (capture = true) or runs the request with ordinary launches.  The PhiDD
// order (its sequences need host-side sizes) always runs with ordinary
// launches.  out->graph tells which happened (0 ordinary, 1 captured now,
// 2 replayed).  The caller owns *cache and frees it with request_graph_free.
struct RequestGraph;
int search_series_graph(RequestGraph** cache, bool capture, const float* T, int64_t m, int32_t n,
                        const discord_opts* opts, void* arena, size_t arena_bytes,
                        hipStream_t stream, discord_result* out, char* err, size_t err_len);
void request_graph_free(RequestGraph* g);
}  // namespace dd

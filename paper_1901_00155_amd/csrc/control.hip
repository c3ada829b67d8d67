// control.hip -- the early-abandon search loop decided on the device.
//
// Algorithms 3 and 4 visit rows, and each row's columns, in some order and
// stop a row at its first distance below the best-so-far.  On the GPU every
// item (a fixed set of consecutive rows) walks its column sequence in windows:
// the first window for every item, then the items that still have a live row
// continue in a longer window.  Which items a launch covers and how they are
// split into chunks depends on how many survived the previous launch, a count
// that exists only on the device.  These one-thread kernels turn those counts
// into the next launch's WinDesc, so the host enqueues the whole loop at once
// and synchronises once per search; launches past the loop's end find
// count == 0 and do nothing.
#include "internal.hpp"

namespace dd {
namespace {

__device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// the split of entries [begin, end) of `items` items into chunks (a multiple of
// the granule each) so that the launch holds about `target` work items, with
// no chunk shorter than `min_chunk` entries (0: one granule) unless the whole
// window is
__device__ inline void set_window(WinDesc* w, int64_t items, int64_t begin, int64_t end,
                                  int64_t target, int64_t gran, int64_t list_off,
                                  int64_t min_chunk = 0) {
  const int64_t it = items > 1 ? items : 1;
  const int64_t width = end - begin > 1 ? end - begin : 1;
  int64_t maxc = ceil_div(width, gran);
  if (min_chunk > gran) {
    const int64_t m = width / min_chunk;
    maxc = m < 1 ? 1 : (m < maxc ? m : maxc);
  }
  int64_t c = ceil_div(target, it);
  c = c < 1 ? 1 : c;
  c = c < maxc ? c : maxc;
  w->n_groups = items;
  w->seq_begin = begin;
  w->seq_chunk = ceil_div(ceil_div(width, c), gran) * gran;
  w->chunks = ceil_div(width, w->seq_chunk);
  w->list_off = list_off;
}

__global__ void k_ctl_start(SearchCtl* ctl, int64_t count, int64_t width,
                            const int32_t* cand_count, WinDesc* cand_win, int64_t bound_items,
                            WinDesc* bound_win, const double* stats, const int32_t* bad,
                            CtlParams P) {
  // eq. (2) undefined (sigma = 0) or the series not finite: nothing to search
  const bool go = !bad[0] && stats[1] > 0.0;
  ctl->count = go ? count : 0;
  ctl->covered = 0;
  ctl->width = width;
  ctl->in_off = 0;
  ctl->end = 0;
  ctl->k = 0;
  if (cand_win)
    set_window(cand_win, go ? *cand_count : 0, 0, P.seq_max, P.target, P.gran, 0, P.min_chunk_full);
  if (bound_win)
    set_window(bound_win, go ? bound_items : 0, 0, P.seq_max, P.seed_target, P.gran, 0,
               P.min_chunk_full);
}

__device__ void ctl_window(SearchCtl* ctl, WinDesc* win, uint32_t* n_surv, const CtlParams& P) {
  const int64_t c = ctl->count;
  const int64_t end = ctl->covered + ctl->width < P.seq_max ? ctl->covered + ctl->width : P.seq_max;
  set_window(win, c, ctl->covered, end, P.target, P.gran, ctl->in_off);
  ctl->end = end;
  *n_surv = 0;
}

__device__ void ctl_after(SearchCtl* ctl, const uint32_t* n_surv, const CtlParams& P) {
  if (ctl->count == 0) return;
  const int64_t hs = *n_surv;
  if (ctl->end >= P.seq_max || hs == 0) {   // every sequence done, or no live row left
    ctl->count = 0;
    return;
  }
  ctl->covered = ctl->end;
  ctl->count = hs;
  ctl->in_off = 0;
  // near-first: the next window `growth` times longer; else the survivors
  // finish in one more window
  ctl->width = P.near_first ? ctl->width * P.growth : P.seq_max;
}

__global__ void k_ctl_window(SearchCtl* ctl, WinDesc* win, uint32_t* n_surv, CtlParams P) {
  ctl_window(ctl, win, n_surv, P);
}

__global__ void k_ctl_after(SearchCtl* ctl, const uint32_t* n_surv, CtlParams P) {
  ctl_after(ctl, n_surv, P);
}

// the two decisions between consecutive windows in one launch
__global__ void k_ctl_next(SearchCtl* ctl, WinDesc* win, uint32_t* n_surv, CtlParams P) {
  ctl_after(ctl, n_surv, P);
  ctl_window(ctl, win, n_surv, P);
}

__global__ void k_ctl_seeds(SearchCtl* ctl, WinDesc* win, CtlParams P) {
  const int64_t c = ctl->count;
  const int64_t k = c < P.seeds ? c : P.seeds;
  set_window(win, k, ctl->covered, P.seq_max, P.seed_target, P.gran, 0);
  ctl->k = k;
}

__global__ void k_ctl_post(SearchCtl* ctl) {
  const int64_t c = ctl->count;
  if (c == 0) return;
  if (ctl->k >= c) {   // the ranked list was completed whole
    ctl->count = 0;
    return;
  }
  ctl->in_off = ctl->k;
  ctl->count = c - ctl->k;
}

}  // namespace

void launch_ctl_start(SearchCtl* ctl, int64_t count, int64_t width, const int32_t* cand_count,
                      WinDesc* cand_win, int64_t bound_items, WinDesc* bound_win,
                      const double* stats, const int32_t* bad, const CtlParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_start, dim3(1), dim3(1), 0, s, ctl, count, width, cand_count, cand_win,
                     bound_items, bound_win, stats, bad, P);
}

void launch_ctl_window(SearchCtl* ctl, WinDesc* win, uint32_t* n_surv, const CtlParams& P,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_window, dim3(1), dim3(1), 0, s, ctl, win, n_surv, P);
}

void launch_ctl_after(SearchCtl* ctl, const uint32_t* n_surv, const CtlParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_after, dim3(1), dim3(1), 0, s, ctl, n_surv, P);
}

void launch_ctl_next(SearchCtl* ctl, WinDesc* win, uint32_t* n_surv, const CtlParams& P,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_next, dim3(1), dim3(1), 0, s, ctl, win, n_surv, P);
}

void launch_ctl_seeds(SearchCtl* ctl, WinDesc* win, const CtlParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_seeds, dim3(1), dim3(1), 0, s, ctl, win, P);
}

void launch_ctl_post(SearchCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_post, dim3(1), dim3(1), 0, s, ctl);
}

}  // namespace dd

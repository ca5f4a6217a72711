// runtime.h -- host-side objects behind the C ABI (fits, batches, schedules).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cwb.h"
#include "cwb_internal.h"
#include "setup.h"

namespace cwb {

constexpr int kGraphIters = 8;  // iterations per captured batch graph

// Sizes of a fit, known before the (expensive) setup.
struct FitShape {
  int64_t n = 0, n_pad = 0, n_train = 0;
  int p = 0, M = 0, variant = 0, nsig_max = 1;
  int nb_max = 0, d_max = 0, sum_d = 0;
  int nb_stride = 0;  // nb_max rounded up to a multiple of 4
  int64_t sum_nb = 0, sum_d2 = 0;
  int n_row_blocks = 0, n_val_blocks = 0;
  bool unbinned = false;  // learners are unbinned cubic P-splines
  bool copies = false;    // some binned learner gets LDS histogram copies (copy_mask)
  bool x12 = false;       // the workspace holds a packed copy of X, 10 or 12 bits
                          // per index (every bin below 4,096)
  // HCWB with every bin below 1,024: a second, 10-bit copy for the
  // one-signal passes after the switch (the ACWB phase reads 12 bits)
  bool x10_after_switch() const {
    return x12 && !external_x && variant == CWB_HCWB && nb_max <= 1024;
  }
  // Folds of a cross-validation share one index matrix and one histogram
  // pass: the first fold's shape has share = the number of folds (the
  // others follow it in the fit list, with share = 0); other fits have 1.
  int share = 1;
  int64_t n_scan = 0;     // rows the histogram pass reads (before an HCWB switch)
  bool external_x = false;  // the index matrix lives outside the fit's workspace
  // fold group head: first row of each fold's block (share + 1 entries, the
  // last n); segments are split at these rows so that most hold one fold
  std::vector<int64_t> fold_start;
  // per learner, known after setup (empty before, and for unbinned fits and
  // folds): 1 if its histogram sums fit 32-bit fixed point (every bin holds
  // fewer than 2^acc32_bits rows and the learner takes no LDS copies)
  std::vector<uint8_t> acc32;
  // per learner with LDS copies: its number of copies (else 0).  Its sums
  // fit 32 bits in a segment whose rows give each copy fewer than
  // 2^acc32_bits rows (group_acc32), whatever its bin counts.
  std::vector<uint8_t> acc32_copies;
  int acc32_bits = 0;
};

// First schedule unit whose rows (as the histogram pass maps units onto the
// n_scan rows it reads) start at or after `row`.
int64_t unit_at_row(const FitShape& sh, int64_t row);
// Rows [r0, r1) the histogram pass reads for units [u0, u1).
void unit_rows(const FitShape& sh, int64_t u0, int64_t u1, int64_t* r0, int64_t* r1);
// The fold that holds out every row of [r0, min(r1, n)), or -1.
int segment_fold(const FitShape& sh, int64_t r0, int64_t r1);

// A fold of a cross-validation: the shared index matrix and fold ids (device)
// and the fold it holds out.
struct FoldSpec {
  const uint16_t* X = nullptr;
  const uint8_t* fold = nullptr;
  int k = 0;
};

int shape_from_problem(const cwb_problem* pr, FitShape* sh, std::string* err);

// Histogram tile shape: threads per block, learners per group (F) and the
// compiled group capacity (fmax), blocks per CU, row slices (XCD affinity).
struct Tune {
  int nt = 512;
  int F = 0;
  int fmax = 0;
  int blocks_per_cu = 1;
  int slices = 1;
  int blocks = 0;  // total histogram blocks; 0 = cus * blocks_per_cu
  int cus = 256;
  int lds_kb = 64;
};

Tune make_tune(int nb_stride, int nsig_max, int p_max, bool unbinned);

struct Schedule {
  std::vector<Seg> segs;         // traversal order
  std::vector<int64_t> blk;      // 2 per physical block: segment range
  std::vector<int64_t> grp_ptr;  // per (fit, group): range in grp_seg (+1 sentinel)
  std::vector<int64_t> grp_seg;  // segment indices, grouped
  std::vector<int64_t> grp_base; // per fit: first group index
  std::vector<int64_t> sel_off;  // per learner and signal: word offsets of its histograms
  std::vector<int64_t> sel_begin;// per (fit, learner): start in sel_off (fit-major)
  std::vector<int32_t> sel_n;    // per (fit, learner): segments of its group
  int64_t partial_words = 0;
  int blocks = 0;
  int nsig_max = 1;  // most signals of any fit in the schedule
  bool unbinned = false;  // the fits' learners are unbinned (one kind per schedule)
  bool folds = false;     // some segment serves a fold group (nfit > 1)
  bool copies = false;    // some fit's learners get LDS histogram copies
  size_t lds = 0;
};

Schedule build_schedule(const std::vector<const FitShape*>& fits, const Tune& t);

// Offsets (bytes) of everything inside a fit's workspace.
struct Layout {
  size_t ctl, fg, h, c, q, theta, table, trk, trth, trkc, trthc, trrisk, trval, trgap, coef_f,
      coef_h;
  size_t state_begin, state_end;  // mutable state region (checkpoint)
  size_t X, y, r, feat, bstart, bval, jr, ainv[2], gram[2], riskpart, amaxpart, valpart, fitdev;
  size_t X12, X10h;
  size_t segs, blk, sel_off, partials, st_items, sel_items, val_items;
  size_t total;
};

// Largest schedule arrays over the tile shapes a fit or batch may use: the
// workspace is sized for all of them, so the autotuner can try each.
struct SchedCap {
  size_t segs = 0, blk = 0, sel_off = 0;
  int64_t partial_words = 0;
  void add(const Schedule& S);
};

std::vector<Tune> tune_candidates(int nb_stride, int nsig_max, int p_max, bool unbinned, bool all,
                                  int64_t work);

Layout make_layout(const FitShape& sh, const SchedCap& s);

struct KernelTimer {
  std::vector<hipEvent_t> ev;  // start/stop pairs
  size_t used = 0;
  double total_ms = 0.0;
  int64_t launches = 0;
};

}  // namespace cwb

struct cwb_fit {
  int device = 0;
  hipStream_t stream = nullptr;
  cwb::FitShape shape;
  cwb::Tune tune;
  cwb::Schedule sched;
  cwb::Layout lay;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double f0 = 0.0;
  std::vector<int64_t> perm;
  std::vector<int32_t> d;      // basis size per learner
  std::vector<cwb::FeatDev> feat;  // host copy of the learner table
  cwb::FitDev dev;             // host copy (device pointers)
  cwb::FitDev* d_fit = nullptr;
  int iters = 0;
  int n_st = 0, n_sel = 0, n_val = 0;
  int timing = 0;  // bit set: 1 hist, 2 state, 4 select
  int timing_period = 1;  // time every period-th iteration
  int64_t timing_counter = 0;
  cwb::KernelTimer t_hist, t_state, t_select;
  int n_cands = 1;        // tile shapes considered
  double tuned_us = 0.0;  // histogram pass time of the chosen shape (0: not tuned)
  int batch_share = 1;    // fold group size in a batch (first fold: K, others 0)
  cwb::FitShape bshape;   // shape as seen by batch schedules (share = batch_share)
  long long* partials = nullptr;  // histogram partials of solo runs: in the workspace,
                                  // or in the library's static scratch array
};

struct cwb_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<cwb_fit*> fits;
  cwb::Tune tune;
  cwb::Schedule sched;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int nb_max = 0;
  int d_max = 0;
  bool any_hcwb = false;
  cwb::FitDev* d_fits = nullptr;
  cwb::Seg* d_segs = nullptr;
  int64_t* d_blk = nullptr;
  int64_t* d_sel_off = nullptr;
  long long* d_partials = nullptr;
  cwb::RowItem* d_st = nullptr;
  cwb::SelItem* d_sel = nullptr;
  cwb::StateItem* d_val = nullptr;
  int n_st = 0, n_sel = 0, n_val = 0;
  int n_cands = 1;
  double tuned_us = 0.0;
  hipGraphExec_t graph_exec = nullptr;  // kGraphIters captured iterations
  int64_t eager_iters = 0, graph_launches = 0;
};

namespace cwb {
int set_error(int code, const std::string& msg);
// Enqueue one finalize (apply pending updates, record the current risk).
int finalize_fit(cwb_fit* f);
RowItem make_row_item(int fit, int blk, const FitDev& D, int chunks = 1);
// Row chunks per row-pass block for a launch over `total` chunks: one,
// unless the launch holds far more chunks than the chip holds blocks (a
// large batch), so that each block's selection and table staging serve
// several chunks.
int row_chunks(int64_t total, int cus);
// Learners of a schedule whose groups take 32-bit LDS words.
int learners32(const Schedule& S);
// The row-pass work list of one fit: blocks of `chunks` chunks each.
void append_row_items(std::vector<RowItem>* out, int fit, const FitDev& D, int n_row_blocks,
                      int chunks);
SelItem make_sel_item(int fit, int k, const FeatDev& fd, const FitDev& D, const Schedule& S,
                      const int64_t* d_sel_off, size_t idx);
// Every candidate tile shape for these fits (only the default unless `all`),
// its schedules validated; `cap` receives the largest schedule arrays and
// `first` (if not null) the default schedule.
int plan_candidates(const std::vector<const FitShape*>& shapes, bool all, std::vector<Tune>* cands,
                    SchedCap* cap, Schedule* first);
// Time the histogram pass of each candidate on the fits' current data and
// return the index of the fastest.  The pass only reads the model state and
// writes the histogram partials (exact integer sums), so trying candidates
// changes no result.  With `row` (a fit that has made no selection yet,
// whose row pass then recomputes the same residuals however often it runs),
// every timed pass follows a row pass, as inside an iteration, and the row
// pass's own time is taken off.
struct TuneRowPass {
  const RowItem* items = nullptr;
  int n = 0, nb_max = 0;
  bool unbinned = false;
};
int autotune_hist(hipStream_t st, const FitDev* d_fits, const std::vector<const FitShape*>& shapes,
                  const std::vector<Tune>& cands, const SchedCap& cap, Seg* d_segs, int64_t* d_blk,
                  long long* d_part, int* best, double* best_us, const TuneRowPass* row = nullptr);
// Device bytes of a fit of this shape (its workspace layout, sized for every
// candidate tile shape when `all`).
int fit_footprint(const FitShape& sh, size_t* bytes, bool all);
// Upload a fit whose host setup is done into `dev_ws` on `stream`, autotune
// its histogram tiles if asked, and wait; the new fit enqueues its
// iterations on the same stream.  With `bin_on_device` (the problem), the
// host setup ran its first phase only and the binning pass runs on the
// device first.
// With `scratch` (device memory of `scratch_bytes` that the fit does not
// own), the histogram partials of solo runs live there instead of in the
// workspace, whose layout then leaves them out.
int fit_upload(const FitShape& sh, HostFit& hf, void* dev_ws, size_t ws_bytes, hipStream_t stream,
               bool autotune, cwb_fit** out, const cwb_problem* bin_on_device = nullptr,
               const FoldSpec* fold = nullptr, long long* scratch = nullptr,
               size_t scratch_bytes = 0);
// cwb_fit_create with the histogram partials in `scratch`: host setup, the
// default tile shape, and no device allocation of any kind.
int fit_create_with_scratch(const cwb_problem* pr, void* dev_ws, size_t ws_bytes, void* stream,
                            cwb_fit** out, long long* scratch, size_t scratch_bytes);
// Device bytes of the batch workspace (combined schedule, partials, work
// lists) for fits of these shapes; 0 for none.
int batch_footprint(const std::vector<const FitShape*>& shapes, size_t* bytes, bool all);
int batch_create(cwb_fit* const* fits, int32_t count, void* dev_ws, size_t ws_bytes, hipStream_t stream,
                 bool autotune, cwb_batch** out);
}  // namespace cwb

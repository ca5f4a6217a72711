// cwb_internal.h -- device data layout shared by the host runtime and the
// gfx950 kernels of the binned componentwise-boosting library.
//
// HBM layout of one fit (all inside the caller's workspace):
//   X      p x n_pad uint16, feature-major: the index vectors of Section 3.1.1,
//          one contiguous row of n_pad entries per learner (16-byte aligned);
//          for unbinned learners p x n_pad uint32 knot-interval codes
//   y, fg, h, c, r   n_pad floats each (model state, Algorithm 2 notation:
//          fg holds f, or g while an ACWB update is pending)
//   per-bin tables: first nonzero basis index and the (degree+1) nonzero
//          reduced-design values of every design point (banded Z^b)
//   per-learner d x d FP64: inverse penalised Gram (G + lambda D)^-1 and G,
//          one set for the training rows and one for all rows (HCWB)
//   q, theta, candidate update tables for every learner (per iteration)
//   traces, aggregated coefficients, risk partials, control block.
// Rows are permuted so that training rows come first: [0, n_train) train,
// [n_train, n) validation, [n, n_pad) zero padding.
#pragma once
#include <cstdint>

namespace cwb {

constexpr int kRowsPerThread = 8;                       // one 16-byte X load
constexpr int kStateThreads = 256;
constexpr int kStateRows = kStateThreads * kRowsPerThread;  // rows per row-pass block
constexpr int kSelectThreads = 256;
constexpr int kMaxBand = 4;      // nonzero basis values per design point (cubic)
constexpr int kMaxD = 64;        // largest basis size
constexpr int kMaxBins = 8192;   // largest n* (one learner's histogram must fit LDS)
constexpr int kNumSig = 2;       // signals: pseudo-residuals r, corrected residuals c
constexpr int kStageBins = 2048; // learners up to this many bins are solved from LDS
constexpr int kMaxSlots = 512;   // segment slots staged per learner group and pass
constexpr int kInlineOffs = 8;   // segment offsets carried in a select item (signal 0)
constexpr int kHistMaxLds = 152 * 1024;  // dynamic LDS of one histogram block
constexpr int kMaxFolds = 8;     // folds of a cross-validation sharing one histogram pass

// Unbinned cubic P-spline learners.  Knots are equally spaced, so the four
// nonzero basis functions at x are those of its knot interval j, and their
// values are fixed cubic polynomials of the position t in [0, 1] inside the
// interval.  Each (learner, row) is stored as one 32-bit code
// (j << 24) | round(t * kUnbFracMax).  Their per-iteration sums go into
// kUnbCopies interleaved LDS copies of each learner's basis sums (one per
// lane mod kUnbCopies), which spreads the lanes of a wave over more
// addresses.
constexpr uint32_t kUnbFracMax = 0xffffffu;
constexpr int kUnbCopies = 4;

// One base learner.
struct FeatDev {
  int32_t nb;        // design points (P-spline) or levels (ridge)
  int32_t band;      // nonzeros per reduced-design row: degree+1, or 1 for ridge
  int32_t d;         // basis size
  int32_t coef_off;  // offset in the concatenated coefficient vectors
  int64_t bin_off;   // offset into the per-bin arrays
  int64_t mat_off;   // offset (doubles) into the d x d matrix arrays
  double xmin, xmax; // P-spline: training range (knots equally spaced on it)
  int32_t kind;      // CWB_PSPLINE or CWB_RIDGE_CAT
  int32_t degree;    // P-spline degree
  int32_t n_int;     // P-spline interior knots
  int32_t pad;
};

// Mutable per-fit control block, written only by kernels after create.
// Each field has one writing kernel, and no block of that kernel reads it,
// so no kernel races with itself:
//   sel_done, sel_acwb      written by k_select (learner 0's block)
//   pick_done               written by k_state (block 0) and k_finalize
//   fin_done                written by k_finalize
//   switched, switch_iter, counter, rval_prev   written by k_valdecide
struct Ctl {
  int32_t sel_done;     // selections made (iterations whose criteria are in q)
  int32_t pick_done;    // selections recorded in the traces and applied
  int32_t fin_done;     // sel_done at the last finalize (which applied it)
  int32_t sel_acwb;     // selection sel_done was an ACWB step (two signals)
  int32_t switched;     // HCWB: CWB phase reached
  int32_t switch_iter;  // HCWB: first CWB iteration (-1 until switched)
  int32_t counter;      // HCWB: consecutive validation-risk rises
  int32_t error;        // bit 0: non-finite model state seen; bit 1: a
                        // histogram segment larger than its launch's LDS
  double rval_prev;     // HCWB: validation risk of the previous model
};

struct FitDev {
  int64_t n, n_pad, n_train;
  int64_t n_scan;        // rows the histogram pass reads before an HCWB switch:
                         // n_train (training rows first), or n for a fold fit
  const uint8_t* fold;   // fold fit: fold id of every row (rows of fold_k are
                         // held out and carry zero residuals), else null
  int32_t fold_k;
  int32_t xbits;         // bits per index of the packed copy X12: 12 (8 rows in
                         // 3 words), 10 (8 rows in 80 bits: learner k's rows
                         // as one 10-bit stream of 5 n_pad / 16 words), or 0
  int32_t p, nb_max, d_max, sum_d;
  int32_t loss, variant, M, patience;
  double nu, gamma;
  int32_t n_row_blocks;  // row-pass blocks: ceil(n_pad / kStateRows)
  int32_t n_val_blocks;  // validation blocks over [n_train, n)
  int32_t nsig_max;      // 2 for ACWB / HCWB, else 1
  int32_t nb_stride;     // histogram words per learner and signal (a multiple of 4)
  int32_t unbinned;      // learners are unbinned cubic P-splines (X holds 32-bit codes)
  int32_t acc32_bits;    // > 0: the histogram values are rounded at the 32-bit
                         // scale (scale_exponent32 with these bits) for every
                         // learner; groups whose learners' bins all hold fewer
                         // than 2^acc32_bits rows then take 32-bit LDS words.
                         // 0: truncated at the int64 scale (scale_exponent).
  const uint16_t* X;
  const uint32_t* X12;   // packed copy of X read by 32-bit histogram groups, at
                         // xbits per index (learner k at word 3 k n_pad / 8 for
                         // 12 bits, 5 k n_pad / 16 for 10), or null
  const uint32_t* X10h;  // HCWB: a 10-bit copy read by the one-signal passes
                         // after the switch (the ACWB phase reads X12), or null
  const float* y;
  float* fg;
  float* h;
  float* c;
  float* r;
  const FeatDev* feat;
  const int32_t* bstart;   // per design point: first nonzero basis index
  const double* bval;      // per design point: kMaxBand values
  const int32_t* jr;       // per basis index: [first, last] design point in its support
  const double* ainv[2];   // [0] training rows, [1] all rows
  const double* gram[2];
  double* q;               // [kNumSig][p]
  double* theta;           // [kNumSig][p][d_max]
  float* table;            // [kNumSig][p][nb_max] candidate update tables Z^b theta
  int32_t* tr_k;
  double* tr_theta;        // [M][d_max]
  int32_t* tr_kcor;
  double* tr_thetacor;
  double* tr_risk;         // [M+1]
  double* tr_val;          // [M+1]
  double* tr_gap;          // [M]
  double* coef_f;          // [sum_d]
  double* coef_h;          // [sum_d]
  double* risk_part;       // [n_row_blocks][2]
  float* amax_part;        // [n_row_blocks][2] largest |r|, |c| per row-pass block
  double* val_part;        // [n_val_blocks]
  Ctl* ctl;
};

// Histogram schedule.  A segment is one (fit, feature group, row range)
// whose histogram is accumulated in LDS and flushed once, as int64, to its
// own partial slot.  Row ranges are in 8-row units of the fit's n_pad and
// are rescaled at run time to the rows the current phase fits.  The folds
// of a cross-validation share one index matrix: their segment covers nfit
// consecutive fits, one histogram per fit and signal, from one read of X.
// Their rows are grouped by fold, so most segments lie in one fold's rows:
// that fold (skip) holds them out and is left out of the segment's work.
struct Seg {
  int32_t fit;
  int32_t k0;      // first learner of the group
  int32_t nf;      // learners in the group
  int16_t nfit;    // fits sharing the segment (1, or the number of folds)
  int16_t skip;    // the fold all of the segment's rows belong to, or -1
  int32_t acc32;   // 1: every learner of the group keeps its sums in int32 (its
                   // fit's acc32_bits bound its bins' counts), so the LDS
                   // histograms take 32-bit words (two signals: one packed
                   // 64-bit word); else 64-bit words per signal
  int32_t pad;
  int64_t u0, u1;  // unit range within [0, n_pad / 8)
  int64_t slot;    // offset (int64 words) of the partial slot
};

struct StateItem {   // one row-pass block
  int32_t fit;
  int32_t blk;       // block index within the fit
};

// A row-pass block with every pointer and size it needs.
struct RowItem {
  Ctl* ctl;
  const double* q;      // the fit's criteria [kNumSig][p] of the last selection
  const uint16_t* X;
  const float* y;
  float* fg;
  float* h;
  float* c;
  float* r;
  const float* table;   // candidate tables [kNumSig][p][nb_max]
  double* risk_part;    // &risk_part[2 * blk]
  float* amax_part;     // &amax_part[2 * blk]
  int64_t n, n_pad, n_train, base;  // base: first row of the block
  double nu, gamma;
  int32_t p, nb_max, loss, variant;
  int32_t M, two, blk, fit;          // two: the fit keeps h and c
  int32_t unbinned;                  // X holds 32-bit unbinned codes
  int32_t fold_k;                    // fold fit: its held-out fold
  const uint8_t* fold;               // fold fit: fold id per row, else null
  int32_t chunks;                    // consecutive kStateRows chunks from base;
  int32_t pad_;                      // risk_part and amax_part hold 2 per chunk
};

// One learner's solve, with every pointer and size it needs, so that a block
// issues all of its independent loads in one round.
struct SelItem {
  Ctl* ctl;
  const float* amax_part;     // the fit's per-block signal maxima
  const double* ainv[2];      // this learner's (G + lambda D)^-1, both row sets
  const double* gram[2];      // this learner's G, both row sets
  const double* bval;         // this learner's banded reduced design
  const int32_t* bstart;
  const int32_t* jr;
  const int64_t* offs;        // its histogram offsets: offs[sig * n_off + i]
  int64_t off0[kInlineOffs];  // the first offsets of signal 0, inline
  int64_t off1[kInlineOffs];  // and of signal 1 (two-signal fits)
  double* q;                  // &q[k] (signal 1 at + p)
  double* theta;              // &theta[k * d_max] (signal 1 at + p * d_max)
  float* table;               // &table[k * nb_max] (signal 1 at + p * nb_max)
  double* tr_risk;            // the fit's risk traces (written by learner 0's block)
  double* tr_val;
  const double* risk_part;    // the fit's row-pass risk partials
  int64_t n, n_train, n_scan;
  int32_t k, nb, band, d;
  int32_t n_off, d_max, nb_max, p;
  int32_t M, variant, n_row_blocks, fit;
  int32_t kind;               // learner kind (CWB_BINARY_CAT: best class only)
  int32_t acc32_bits;         // its fit's: > 0, sums at the 32-bit scale
                              // (scale_exponent32 with these bits), else int64
};

// One learner solve of the device setup pass (alg::learner_solve): the Gram
// matrix from the bin counts of one row set, lambda for the learner's df,
// and the inverse of G + lambda D, written into the fit's tables.
struct SolveJob {
  const int32_t* bstart;   // the learner's band starts (nb)
  const double* bval;      // its banded reduced design (nb x kMaxBand)
  const uint32_t* cnt;     // its bin counts over the row set (nb)
  double* gram;            // out: d x d
  double* ainv;            // out: d x d
  double df, lambda;       // df target (> 0), else the fixed lambda
  int32_t kind, d, nb, band;
  int32_t pen_order, pad;
};

// Fixed-point exponent for the int64 histogram of a signal whose largest
// magnitude is `amax`, summed over at most n_fit rows: |r| * 2^e < 2^(62 - N)
// with n_fit < 2^N, so no sum of n_fit terms can overflow.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline int scale_exponent(float amax, int64_t n_fit) {
  if (!(amax > 0.0f)) return 0;
  uint32_t bits;
  __builtin_memcpy(&bits, &amax, 4);
  const uint32_t ex = (bits >> 23) & 0xffu;     // biased exponent of max |r|
  const int E = (ex == 0u) ? -125 : (int)ex - 126;  // max |r| < 2^E
  int N = 0;
  for (int64_t v = n_fit; v > 0; v >>= 1) ++N;  // n_fit < 2^N
  return 62 - N - E;
}

// 32-bit accumulation.  When every bin of a learner holds fewer than 2^B
// rows (B = acc32_bits), its residuals are rounded to integers below
// 2^(31 - B) in magnitude: |r| * 2^e < 2^(31 - B), so no bin's sum, over any
// subset of the rows, leaves the int32 range.  The LDS then takes 4-byte
// atomics (one signal), or one 8-byte atomic carrying both ACWB signals
// (r in the high word, c in the low word; see pack_signals).
constexpr int kAcc32MaxBits = 14;  // at least 17 bits of resolution below max |r|
#if defined(__HIPCC__)
__host__ __device__
#endif
inline int scale_exponent32(float amax, int bits) {
  if (!(amax > 0.0f)) return 0;
  uint32_t b;
  __builtin_memcpy(&b, &amax, 4);
  const uint32_t ex = (b >> 23) & 0xffu;
  const int E = (ex == 0u) ? -125 : (int)ex - 126;  // max |r| < 2^E
  return 31 - bits - E;
}

// Learners with few bins (categorical levels, coarse binnings) get several
// interleaved copies of their histogram inside their LDS region of `region`
// words: lane l of a wave adds into copy l mod C, so the lanes seldom add
// into the same word, which the LDS would serialise.  Copies start
// s = nb | 1 words apart (an odd stride puts the copies of one bin on
// different banks) and C * s <= region.  Returns C - 1 (a lane mask) and s.
constexpr int kMaxCopies = 32;
#if defined(__HIPCC__)
__host__ __device__
#endif
inline int copy_mask(int nbk, int region, int* stride) {
  const int s = nbk | 1;
  int c = 1;
  while (c < kMaxCopies && 2 * c * s <= region) c *= 2;
  *stride = s;
  return c - 1;
}

}  // namespace cwb

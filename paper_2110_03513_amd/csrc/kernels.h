// kernels.h -- host launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include "cwb_internal.h"

namespace cwb {

// unbinned: the fits' learners are unbinned (every fit of the launch alike).
hipError_t launch_state(hipStream_t st, const FitDev* fits, const RowItem* items, int nitems,
                        int nb_max, int final_mode, bool unbinned);
// folds: the schedule has fold-group segments (nfit > 1); only the variant
// compiled for them handles such segments.
hipError_t launch_hist(hipStream_t st, int nt, int fmax, int nsmax, bool unbinned, bool folds,
                       bool copies, int blocks, size_t lds, const FitDev* fits, const Seg* segs,
                       const int64_t* blk, long long* partials);
hipError_t launch_select(hipStream_t st, const SelItem* items, int nitems, int nsig, int nb_max, int d_max,
                         const long long* partials);
hipError_t launch_valrisk(hipStream_t st, const FitDev* fits, const StateItem* items, int nitems,
                          int nb_max);
hipError_t launch_valdecide(hipStream_t st, const FitDev* fits, int nfits);
hipError_t launch_finalize(hipStream_t st, const FitDev* fits, int nfits);
// The fit's primary model (learners [k0, k1) plus f0) at n new rows of the
// column-major device array x (column j: learner k0 + j).
hipError_t launch_predict(hipStream_t st, const FitDev* fit, const double* x, int64_t n, int64_t ldx,
                          double f0, int k0, int k1, double* out);
// Aggregated coefficients of one fit (sum_d of them) from its traces.
hipError_t launch_coef(hipStream_t st, const FitDev* fit, int sum_d);
// Device binning pass of fit setup (binning.hip).  mm: the column's range as
// order-preserving integers (minimum, maximum), to be initialised to
// (all ones, 0); flag |= 1 when a value is not finite.
hipError_t launch_range(hipStream_t st, const double* x, int64_t n, unsigned long long* mm, int* flag);
// Bin indices of rows [0, n_pad) in the fit's order (perm: fit row -> x row,
// or NULL for the identity; rows from n on get 0), and the bin counts of
// the training rows (counts[0, nb)) and of all rows (counts[half, half+nb)),
// added to the counters.  flag |= 2 when a categorical code is invalid.
hipError_t launch_bin(hipStream_t st, const double* x, const int32_t* perm, int64_t n, int64_t n_pad,
                      int64_t n_train, int categorical, int nb, const unsigned long long* mm,
                      uint16_t* out, uint32_t* counts, int64_t half, int* flag);

// The learners' solves of the device setup pass (binning.hip): njobs blocks,
// LDS for basis sizes up to d_max (at most kDeviceSolveMaxD).
hipError_t launch_solve(hipStream_t st, const SolveJob* jobs, int njobs, int d_max, int* status,
                        double* lam);
// The 12-bit copy of the index matrix (binning.hip): groups = p n_pad / 8,
// every index below 4,096.
hipError_t launch_pack12(hipStream_t st, const uint16_t* X, int64_t groups, uint32_t* X12);
// The 10-bit copy (binning.hip): pairs = p n_pad / 16, every index below 1,024.
hipError_t launch_pack10(hipStream_t st, const uint16_t* X, int64_t pairs, uint32_t* X10);

}  // namespace cwb

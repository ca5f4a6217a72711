// binning.hip -- the device binning pass of fit setup (Sec. 3.1.1 and the
// counts of binMatMat, Algorithm 1), one feature column at a time:
//   k_range  largest and smallest value of a numeric column (and whether any
//            value is not finite);
//   k_bin    every row's design-point index, nearest of the nb equally
//            spaced points on [min, max] with ties to the lower point, by the
//            same FP64 operations in the same order as the host rule (this
//            file is built without floating-point contraction), or the
//            level code of a categorical column; the rows are taken in the
//            fit's order (training rows first), and the bin counts over the
//            training rows and over all rows are accumulated in LDS and added
//            to the column's counters.
#include <hip/hip_runtime.h>

#include "cwb_internal.h"
#include "algebra.h"
#include "kernels.h"

namespace cwb {
namespace {

constexpr int kSetupThreads = 256;

// Doubles as unsigned integers whose order is the order of the values, so
// that 64-bit integer atomics give the exact minimum and maximum.
__device__ __forceinline__ unsigned long long ordered(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double from_ordered(unsigned long long o) {
  const unsigned long long b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
  const double v = __longlong_as_double((long long)b);
  return v == 0.0 ? 0.0 : v;  // one zero for both signs
}

__device__ __forceinline__ double grid_point(double xmin, double xmax, double h, int l, int nb) {
  return (l == nb - 1) ? xmax : xmin + (double)l * h;
}

// Closest design point, ties to the lower one: an arithmetic estimate of the
// enclosing interval, corrected by exact comparisons with the design points,
// then the two distances decide.
__device__ __forceinline__ int bin_of(double x, double xmin, double xmax, double h, int nb) {
  if (x <= xmin) return 0;
  if (x >= xmax) return nb - 1;
  int l = (int)((x - xmin) / h);
  if (l < 0) l = 0;
  if (l > nb - 2) l = nb - 2;
  while (l > 0 && grid_point(xmin, xmax, h, l, nb) > x) --l;
  while (l < nb - 2 && grid_point(xmin, xmax, h, l + 1, nb) <= x) ++l;
  const double dlo = x - grid_point(xmin, xmax, h, l, nb);
  const double dhi = grid_point(xmin, xmax, h, l + 1, nb) - x;
  return (dhi < dlo) ? l + 1 : l;
}

__global__ void __launch_bounds__(kSetupThreads)
k_range(const double* __restrict__ x, int64_t n, unsigned long long* __restrict__ mm,
        int* __restrict__ flag) {
  __shared__ unsigned long long s_lo[kSetupThreads / 64], s_hi[kSetupThreads / 64];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  unsigned long long lo = ~0ull, hi = 0ull;
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * kSetupThreads;
  for (int64_t i = (int64_t)blockIdx.x * kSetupThreads + threadIdx.x; i < n; i += stride) {
    const double v = x[i];
    if (!isfinite(v)) {
      bad = true;
      continue;
    }
    const unsigned long long o = ordered(v);
    lo = o < lo ? o : lo;
    hi = o > hi ? o : hi;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long a = __shfl_down(lo, off, 64), b = __shfl_down(hi, off, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if (bad) s_bad = 1;
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    s_lo[w] = lo;
    s_hi[w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kSetupThreads / 64; ++k) {
      lo = s_lo[k] < lo ? s_lo[k] : lo;
      hi = s_hi[k] > hi ? s_hi[k] : hi;
    }
    if (lo != ~0ull) atomicMin(mm, lo);
    if (hi != 0ull) atomicMax(mm + 1, hi);
    if (s_bad) atomicOr(flag, 1);
  }
}

// rows_per_block consecutive rows of the fit's order per block.  counts:
// training-row counts at [0, nb), all-row counts at [half, half + nb).
__global__ void __launch_bounds__(kSetupThreads)
k_bin(const double* __restrict__ x, const int32_t* __restrict__ perm, int64_t n, int64_t n_pad,
      int64_t n_train, int categorical, int nb, const unsigned long long* __restrict__ mm,
      int64_t rows_per_block, uint16_t* __restrict__ out, uint32_t* __restrict__ counts,
      int64_t half, int* __restrict__ flag) {
  extern __shared__ uint32_t s_cnt[];  // [2][nb]
  for (int l = threadIdx.x; l < 2 * nb; l += kSetupThreads) s_cnt[l] = 0u;
  __syncthreads();
  double xmin = 0.0, xmax = 0.0, h = 0.0;
  bool ok = true;
  if (!categorical) {
    xmin = from_ordered(mm[0]);
    xmax = from_ordered(mm[1]);
    ok = xmax > xmin;  // a constant column is reported by the host
    h = (xmax - xmin) / (double)(nb - 1);
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = (r0 + rows_per_block < n_pad) ? r0 + rows_per_block : n_pad;
  bool bad = false;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += kSetupThreads) {
    int l = 0;
    if (i < n && ok) {
      const double v = x[perm ? (int64_t)perm[i] : i];
      if (categorical) {
        if (!(v >= 0.0) || v >= (double)nb || v != floor(v)) bad = true;
        else l = (int)v;
      } else {
        l = bin_of(v, xmin, xmax, h, nb);
      }
      atomicAdd(&s_cnt[nb + l], 1u);
      if (i < n_train) atomicAdd(&s_cnt[l], 1u);
    }
    out[i] = (uint16_t)l;
  }
  if (bad) atomicOr(flag, 2);
  __syncthreads();
  for (int l = threadIdx.x; l < nb; l += kSetupThreads) {
    if (s_cnt[l]) atomicAdd(counts + l, s_cnt[l]);
    if (s_cnt[nb + l]) atomicAdd(counts + half + l, s_cnt[nb + l]);
  }
}

}  // namespace

hipError_t launch_range(hipStream_t st, const double* x, int64_t n, unsigned long long* mm, int* flag) {
  int64_t blocks = (n + kSetupThreads * 16 - 1) / (kSetupThreads * 16);
  if (blocks < 1) blocks = 1;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_range, dim3((unsigned)blocks), dim3(kSetupThreads), 0, st, x, n, mm, flag);
  return hipGetLastError();
}

hipError_t launch_bin(hipStream_t st, const double* x, const int32_t* perm, int64_t n, int64_t n_pad,
                      int64_t n_train, int categorical, int nb, const unsigned long long* mm,
                      uint16_t* out, uint32_t* counts, int64_t half, int* flag) {
  if (nb < 1 || nb > kMaxBins || (!categorical && nb < 2) || n_pad < n || n_pad % 64 != 0)
    return hipErrorInvalidValue;
  int64_t rows = 4 * (int64_t)nb;
  if (rows < 4096) rows = 4096;
  rows = (rows + kSetupThreads - 1) / kSetupThreads * kSetupThreads;
  const int64_t blocks = (n_pad + rows - 1) / rows;
  const size_t lds = (size_t)2 * nb * sizeof(uint32_t);
  hipLaunchKernelGGL(k_bin, dim3((unsigned)blocks), dim3(kSetupThreads), lds, st, x, perm, n, n_pad,
                     n_train, categorical, nb, mm, rows, out, counts, half, flag);
  return hipGetLastError();
}

// 12-bit copy of the bin-index matrix for the histogram pass: every 8
// consecutive uint16 indices (16 bytes, all below 4,096) become 3 words,
// index j in bits [12 j, 12 j + 12) of the 96.  `groups` = p n_pad / 8;
// group t is X[8t, 8t + 8) -> X12[3t, 3t + 3), so every learner's row of
// n_pad indices maps to n_pad / 8 * 3 contiguous words.
__global__ void __launch_bounds__(kSetupThreads)
k_pack12(const uint16_t* __restrict__ X, int64_t groups, uint32_t* __restrict__ X12) {
  for (int64_t t = (int64_t)blockIdx.x * kSetupThreads + threadIdx.x; t < groups;
       t += (int64_t)gridDim.x * kSetupThreads) {
    const uint4 v = *reinterpret_cast<const uint4*>(X + 8 * t);
    const uint32_t a[8] = {v.x & 0xfffu, (v.x >> 16) & 0xfffu, v.y & 0xfffu, (v.y >> 16) & 0xfffu,
                           v.z & 0xfffu, (v.z >> 16) & 0xfffu, v.w & 0xfffu, (v.w >> 16) & 0xfffu};
    X12[3 * t] = a[0] | (a[1] << 12) | (a[2] << 24);
    X12[3 * t + 1] = (a[2] >> 8) | (a[3] << 4) | (a[4] << 16) | (a[5] << 28);
    X12[3 * t + 2] = (a[5] >> 4) | (a[6] << 8) | (a[7] << 20);
  }
}

// 10-bit copy (every index below 1,024): each learner's n_pad indices as one
// stream of 10-bit fields, row i at bits [10 i, 10 i + 10); 16 rows fill 5
// words.  `pairs` = p n_pad / 16; pair t is X[16t, 16t + 16) -> X10[5t, 5t + 5)
// (n_pad is a multiple of 16, so no pair spans two learners).
__global__ void __launch_bounds__(kSetupThreads)
k_pack10(const uint16_t* __restrict__ X, int64_t pairs, uint32_t* __restrict__ X10) {
  for (int64_t t = (int64_t)blockIdx.x * kSetupThreads + threadIdx.x; t < pairs;
       t += (int64_t)gridDim.x * kSetupThreads) {
    const uint4 v0 = *reinterpret_cast<const uint4*>(X + 16 * t);
    const uint4 v1 = *reinterpret_cast<const uint4*>(X + 16 * t + 8);
    const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
    uint32_t out[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t a = (w[i >> 1] >> (16 * (i & 1))) & 0x3ffu;
      const int bit = 10 * i, m = bit >> 5, sh = bit & 31;
      out[m] |= a << sh;
      if (sh > 22) out[m + 1] |= a >> (32 - sh);  // the field runs into the next word
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) X10[5 * t + m] = out[m];
  }
}

hipError_t launch_pack10(hipStream_t st, const uint16_t* X, int64_t pairs, uint32_t* X10) {
  if (pairs <= 0) return hipSuccess;
  const int64_t want = (pairs + kSetupThreads - 1) / kSetupThreads;
  const int blocks = (int)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(k_pack10, dim3(blocks), dim3(kSetupThreads), 0, st, X, pairs, X10);
  return hipGetLastError();
}

hipError_t launch_pack12(hipStream_t st, const uint16_t* X, int64_t groups, uint32_t* X12) {
  if (groups <= 0) return hipSuccess;
  const int64_t want = (groups + kSetupThreads - 1) / kSetupThreads;
  const int blocks = (int)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(k_pack12, dim3(blocks), dim3(kSetupThreads), 0, st, X, groups, X12);
  return hipGetLastError();
}

// The learners' solves of the device setup pass, one block of one wavefront
// per (learner, row set): alg::learner_solve in LDS -- the routine the host
// setup runs, each value by the same operations, built without contraction
// -- with its element loops spread over the 64 lanes; then the block copies
// the Gram matrix and the inverse out.  status[job]: 0, -1 (df out of
// reach) or -5 (singular); lam[job]: lambda.
__global__ void __launch_bounds__(64)
k_solve(const SolveJob* __restrict__ jobs, int* __restrict__ status, double* __restrict__ lam) {
  extern __shared__ double s_m[];
  const SolveJob jb = jobs[blockIdx.x];
  const int d = jb.d;
  double* G = s_m;
  double* inv = s_m + d * d;
  double* scr = s_m + 2 * d * d;
  const alg::Lanes ex{(int)threadIdx.x, (int)blockDim.x};
  double l = 0.0;
  const int rc = alg::learner_solve(ex, jb.kind, d, jb.nb, jb.band, jb.bstart, jb.bval, kMaxBand,
                                    jb.cnt, jb.pen_order, jb.df, jb.lambda, G, inv, &l, scr);
  if (threadIdx.x == 0) {
    status[blockIdx.x] = rc;
    lam[blockIdx.x] = l;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < d * d; i += blockDim.x) {
    jb.gram[i] = G[i];
    jb.ainv[i] = inv[i];
  }
}

hipError_t launch_solve(hipStream_t st, const SolveJob* jobs, int njobs, int d_max, int* status,
                        double* lam) {
  if (njobs <= 0) return hipSuccess;
  if (d_max < 1 || d_max > 64) return hipErrorInvalidValue;
  const size_t lds = ((size_t)2 * d_max * d_max + alg::solve_scratch(d_max)) * sizeof(double);
  if (lds > 152 * 1024) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
  hipLaunchKernelGGL(k_solve, dim3(njobs), dim3(64), lds, st, jobs, status, lam);
  return hipGetLastError();
}

}  // namespace cwb

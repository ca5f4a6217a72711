// hist.hip -- the histogram pass over the bin-index matrix (binMatVec,
// Algorithm 1, first stage): for every learner k and design point l,
// s_kl = sum of r_i over the rows with ind_ki = l, and the same for the
// ACWB corrected residuals c.  Each block accumulates int64 fixed-point
// sums in LDS and flushes them once per segment; int64 addition is exact,
// so the result does not depend on the order of the atomics or on the
// schedule.
#include "device_common.h"
#include "kernels.h"

namespace cwb {

// The lane index, opaque to the optimiser: the copy bases derived from it
// are recomputed at each use (a few VALU operations next to many LDS
// atomics) rather than held in a register per learner across the row loop.
__device__ __forceinline__ int opaque_lane() {
  int l = (int)threadIdx.x & 63;
  asm volatile("" : "+v"(l));
  return l;
}

// The 8 rows of one index load of one learner into its histogram h (this
// lane's copy).
template <int NSIG>
__device__ __forceinline__ void hist_add(unsigned long long* __restrict__ h, const u32x4& x,
                                         const long long* q) {
  const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    __hip_atomic_fetch_add(h + (w[j] & 0xffffu), (unsigned long long)q[2 * j], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(h + (w[j] >> 16), (unsigned long long)q[2 * j + 1], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// 32-bit words: one signal's values, 4-byte LDS atomics.
__device__ __forceinline__ void hist_add32(uint32_t* __restrict__ h, const u32x4& x, const int* q) {
  const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    __hip_atomic_fetch_add(h + (w[j] & 0xffffu), (uint32_t)q[2 * j], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(h + (w[j] >> 16), (uint32_t)q[2 * j + 1], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Packed words: both ACWB signals of a row in one 8-byte LDS atomic.
__device__ __forceinline__ void hist_add_packed(unsigned long long* __restrict__ h, const u32x4& x,
                                                const unsigned long long* q) {
  const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    __hip_atomic_fetch_add(h + (w[j] & 0xffffu), q[2 * j], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(h + (w[j] >> 16), q[2 * j + 1], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

__device__ __forceinline__ u32x4 load_idx(const uint16_t* p) {
  return __builtin_nontemporal_load((const GLOBAL u32x4*)p);
}


template <int FMAX, int NSIG>
__device__ __forceinline__ void hist_step_load(const FitDev& F, const uint16_t* __restrict__ Xg,
                                               size_t ld, int nf, int64_t base, float* rv, float* cv,
                                               u32x4* xw) {
  load8f(F.r + base, rv);
  if (NSIG == 2) load8f(F.c + base, cv);
#pragma unroll
  for (int f = 0; f < FMAX; ++f)
    if (f < nf) xw[f] = load_idx(Xg + f * ld + base);
}

// Rows [r0, r1) of one segment with 64-bit LDS words.  Every thread takes
// 8 consecutive rows per step: one 32-byte load of residuals per signal and
// one 16-byte load of bin indices per learner of the group, then 8 LDS
// atomics per learner and signal.  The next step's loads are issued before
// this step's atomics.  The values are at the fit's scale: rounded at the
// 32-bit one when the fit has acc32_bits, else truncated at the int64 one,
// the same for every learner and group.  With `need_e`, the fit's scale
// exponents are computed (by all threads) while the first step's loads are
// in flight.
template <int NT, int FMAX, int NSIG, bool COPIES>
__device__ __forceinline__ void hist_rows(const FitDev& F, const Seg& sg,
                                          unsigned long long* __restrict__ hist, int nb,
                                          int64_t r0, int64_t r1, Exps& ex, bool need_e,
                                          int64_t n_fit, float* red, const int (*cp)[16]) {
  const uint16_t* __restrict__ Xg = F.X + (size_t)sg.k0 * F.n_pad;
  const int nf = sg.nf;
  const size_t ld = (size_t)F.n_pad;
  int cm[FMAX], cs[FMAX];  // copy masks and strides, wave-uniform
#pragma unroll
  for (int f = 0; f < FMAX; ++f) {
    cm[f] = COPIES ? __builtin_amdgcn_readfirstlane(cp[0][f]) : 0;
    cs[f] = COPIES ? __builtin_amdgcn_readfirstlane(cp[1][f]) : 0;
  }
  const bool r32 = F.acc32_bits > 0;
  int64_t base = r0 + (int64_t)threadIdx.x * 8;
  const bool any = base < r1;
  float rv[8], cv[8];
  u32x4 xw[FMAX];
  if (any) hist_step_load<FMAX, NSIG>(F, Xg, ld, nf, base, rv, cv, xw);
  if (need_e) fit_exponents<NT>(F, n_fit, &ex, red);
  if (!any) return;
  const int e0 = r32 ? ex.e32[0] : ex.e[0], e1 = r32 ? ex.e32[1] : ex.e[1];
  for (;;) {
    const int64_t nxt = base + (int64_t)NT * 8;
    const bool more = nxt < r1;
    long long q0[8], q1[8];
    if (r32) {
#pragma unroll
      for (int j = 0; j < 8; ++j) q0[j] = (long long)fixed32(rv[j], e0);
      if (NSIG == 2) {
#pragma unroll
        for (int j = 0; j < 8; ++j) q1[j] = (long long)fixed32(cv[j], e1);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) q0[j] = fixed_point(rv[j], e0);
      if (NSIG == 2) {
#pragma unroll
        for (int j = 0; j < 8; ++j) q1[j] = fixed_point(cv[j], e1);
      }
    }
    u32x4 xc[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; ++f) xc[f] = xw[f];
    if (more) hist_step_load<FMAX, NSIG>(F, Xg, ld, nf, nxt, rv, cv, xw);
    const int lane = COPIES ? opaque_lane() : 0;
#pragma unroll
    for (int f = 0; f < FMAX; ++f) {
      if (f < nf) {
        const int cb = COPIES ? (lane & cm[f]) * cs[f] : 0;  // this lane's copy
        hist_add<NSIG>(hist + (size_t)f * nb + cb, xc[f], q0);
        if (NSIG == 2) hist_add<NSIG>(hist + (size_t)(nf + f) * nb + cb, xc[f], q1);
      }
    }
    if (!more) break;
    base = nxt;
  }
}

typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));

// The 8 bin indices of one 12-byte word triple of the 10-bit copy of X, in
// the 16-bit layout of a uint16 load: the 80 bits start at bit 0 of w.x, or
// at bit 16 for an odd 8-row block (`odd`).
__device__ __forceinline__ u32x4 unpack10(const u32x3& w, bool odd) {
  const uint32_t a = odd ? __builtin_amdgcn_alignbit(w.y, w.x, 16) : w.x;
  const uint32_t b = odd ? __builtin_amdgcn_alignbit(w.z, w.y, 16) : w.y;
  const uint32_t c = odd ? (w.z >> 16) : w.z;
  u32x4 o;
  o.x = (a & 0x3ffu) | (((a >> 10) & 0x3ffu) << 16);
  o.y = ((a >> 20) & 0x3ffu) | ((__builtin_amdgcn_alignbit(b, a, 30) & 0x3ffu) << 16);
  o.z = ((b >> 8) & 0x3ffu) | (((b >> 18) & 0x3ffu) << 16);
  o.w = (__builtin_amdgcn_alignbit(c, b, 28) & 0x3ffu) | (((c >> 6) & 0x3ffu) << 16);
  return o;
}

// The 8 bin indices of one 12-byte word triple of the 12-bit copy of X, in
// the 16-bit layout of a uint16 load (two indices per word), so the same
// adders serve both.
__device__ __forceinline__ u32x4 unpack12(const u32x3& w) {
  u32x4 o;
  o.x = (w.x & 0xfffu) | (((w.x >> 12) & 0xfffu) << 16);
  o.y = __builtin_amdgcn_alignbit(w.y, w.x, 24) & 0xfffu;
  o.y |= ((w.y >> 4) & 0xfffu) << 16;
  o.z = ((w.y >> 16) & 0xfffu) | ((__builtin_amdgcn_alignbit(w.z, w.y, 28) & 0xfffu) << 16);
  o.w = ((w.z >> 8) & 0xfffu) | ((w.z >> 20) << 16);
  return o;
}

// Rows [r0, r1) of a segment whose learners all take 32-bit accumulation
// (Seg.acc32).  One signal: 4-byte words, learner f at word f * nb.  Two
// signals: both values of a row packed into one 8-byte word (pack_signals),
// learner f at word f * nb, so an ACWB row costs one LDS atomic per
// learner, as a CWB row does.  XB is the index width read: 16 (the uint16
// matrix), 12 or 10 (the packed copy `xpk`: F.X12 at F.xbits, or an HCWB
// fit's 10-bit F.X10h after its switch; 12 or 10 bytes per 8 rows and
// learner instead of 16), a template parameter so that each
// instantiation unpacks one way only.  With COPIES a learner of few bins
// spreads over copies of its histogram by lane, as in hist_rows (the
// schedule takes 32-bit words for it only while each copy receives fewer
// than 2^acc32_bits rows of the segment).
template <int NT, int FMAX, int NSIG, int XB, bool COPIES>
__device__ __forceinline__ void hist_rows32(const FitDev& F, const uint32_t* xpk, const Seg& sg,
                                            void* __restrict__ hist, int nb, int64_t r0, int64_t r1,
                                            Exps& ex, bool need_e, int64_t n_fit, float* red,
                                            const int (*cp)[16]) {
  int cm[FMAX], cs[FMAX];  // copy masks and strides, wave-uniform
#pragma unroll
  for (int f = 0; f < FMAX; ++f) {
    cm[f] = COPIES ? __builtin_amdgcn_readfirstlane(cp[0][f]) : 0;
    cs[f] = COPIES ? __builtin_amdgcn_readfirstlane(cp[1][f]) : 0;
  }
  const uint16_t* __restrict__ Xg = F.X + (size_t)sg.k0 * F.n_pad;
  // the packed copy: 12 bits (3 words per 8-row block) or 10 bits (8 rows in
  // 80 bits; block b starts at bit 80 b, and its 12-byte load at word
  // floor(5 b / 2), so consecutive blocks' loads overlap by half a word)
  constexpr bool X12 = XB != 16;
  constexpr bool x10 = XB == 10;
  const size_t ldp = x10 ? (size_t)F.n_pad / 16 * 5 : (size_t)F.n_pad / 8 * 3;  // words per learner
  const uint32_t* __restrict__ Xp = X12 ? xpk + (size_t)sg.k0 * ldp : nullptr;
  const int nf = sg.nf;
  const size_t ld = (size_t)F.n_pad;
  int64_t base = r0 + (int64_t)threadIdx.x * 8;
  const bool any = base < r1;
  // a thread's 8-row blocks keep their parity: each step moves 8 NT rows
  const bool odd = ((base >> 3) & 1) != 0;
  float rv[8], cv[8];
  u32x4 xw[FMAX];
  u32x3 xp[FMAX];
  auto load = [&](int64_t b) {
    if (!X12) {
      hist_step_load<FMAX, NSIG>(F, Xg, ld, nf, b, rv, cv, xw);
      return;
    }
    load8f(F.r + b, rv);
    if (NSIG == 2) load8f(F.c + b, cv);
    const size_t w0 = x10 ? (size_t)((b >> 3) * 5 >> 1) : (size_t)(b >> 3) * 3;
#pragma unroll
    for (int f = 0; f < FMAX; ++f)
      if (f < nf)
        xp[f] = __builtin_nontemporal_load((const GLOBAL u32x3*)(Xp + f * ldp + w0));
  };
  if (any) load(base);
  if (need_e) fit_exponents<NT>(F, n_fit, &ex, red);
  if (!any) return;
  const int g0 = ex.e32[0], g1 = ex.e32[1];
  uint32_t* __restrict__ h32 = static_cast<uint32_t*>(hist);
  unsigned long long* __restrict__ h64 = static_cast<unsigned long long*>(hist);
  for (;;) {
    const int64_t nxt = base + (int64_t)NT * 8;
    const bool more = nxt < r1;
    int p0[8];
    unsigned long long pk[8];
    if (NSIG == 1) {
#pragma unroll
      for (int j = 0; j < 8; ++j) p0[j] = fixed32(rv[j], g0);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) pk[j] = pack_signals(fixed32(rv[j], g0), fixed32(cv[j], g1));
    }
    u32x4 xc[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; ++f) xc[f] = X12 ? (x10 ? unpack10(xp[f], odd) : unpack12(xp[f])) : xw[f];
    if (more) load(nxt);
    const int lane = COPIES ? opaque_lane() : 0;
#pragma unroll
    for (int f = 0; f < FMAX; ++f) {
      if (f < nf) {
        const int cb = COPIES ? (lane & cm[f]) * cs[f] : 0;  // this lane's copy
        if (NSIG == 1) hist_add32(h32 + (size_t)f * nb + cb, xc[f], p0);
        else hist_add_packed(h64 + (size_t)f * nb + cb, xc[f], pk);
      }
    }
    if (!more) break;
    base = nxt;
  }
}

// Rows [r0, r1) of a segment shared by the nfit folds of a cross-validation:
// one read of the group's bin indices feeds every fold's signals.  Held-out
// rows carry zero residuals; the fold that holds out all of the segment's
// rows (skip) is left out.  Exponents in e[2q], e[2q+1]: the folds' 32-bit
// scale (rounded values) when `r32`, else the int64 one (truncated).  W32
// (a group of 32-bit learners, Seg.acc32): fold q, learner f at word
// (q nf + f) nb of 4-byte words (one signal) or of packed 8-byte words
// (two signals); else 8-byte words, fold q, signal s, learner f at
// ((q NSIG + s) nf + f) nb.
template <int NT, int FMAX, int NSIG, bool COPIES, bool W32>
__device__ __forceinline__ void hist_rows_folds(const FitDev* __restrict__ fits, const Seg& sg,
                                                unsigned long long* __restrict__ hist, int nb,
                                                int64_t r0, int64_t r1, const int* e, bool r32,
                                                const int (*cp)[16]) {
  int cm[FMAX], cs[FMAX];
#pragma unroll
  for (int f = 0; f < FMAX; ++f) {
    cm[f] = COPIES ? __builtin_amdgcn_readfirstlane(cp[0][f]) : 0;
    cs[f] = COPIES ? __builtin_amdgcn_readfirstlane(cp[1][f]) : 0;
  }
  const FitDev& F0 = fits[sg.fit];
  const uint16_t* __restrict__ Xg = F0.X + (size_t)sg.k0 * F0.n_pad;
  const int nf = sg.nf;
  const size_t ld = (size_t)F0.n_pad;
  const int nfit = sg.nfit, skip = sg.skip;
  const int first = (skip == 0) ? 1 : 0;  // first fold with work (nfit >= 2)
  auto next_fold = [&](int q) {
    ++q;
    if (q == skip) ++q;
    return q < nfit ? q : -1;
  };
  int64_t base = r0 + (int64_t)threadIdx.x * 8;
  if (base >= r1) return;
  uint32_t* __restrict__ h32 = reinterpret_cast<uint32_t*>(hist);
  // Each row step loads the learners' indices once and the residuals of up
  // to QB folds at a time, all issued before the first of their atomics, so
  // that a step waits on one round of loads per QB folds rather than one per
  // fold; the next step's indices are loaded before this step's atomics.
  // Two signals hold r and c per fold, so they take two folds a round.
  constexpr int QB = NSIG == 2 ? 2 : 4;
  u32x4 xw[FMAX];
#pragma unroll
  for (int f = 0; f < FMAX; ++f)
    if (f < nf) xw[f] = load_idx(Xg + f * ld + base);
  for (;;) {
    const int64_t nxt = base + (int64_t)NT * 8;
    const bool more = nxt < r1;
    u32x4 xc[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; ++f) xc[f] = xw[f];
    if (more) {
#pragma unroll
      for (int f = 0; f < FMAX; ++f)
        if (f < nf) xw[f] = load_idx(Xg + f * ld + nxt);
    }
    const int lane = COPIES ? opaque_lane() : 0;
    for (int q = first; q >= 0;) {
      int qs[QB];
      float rv[QB][8], cv[QB][8];
#pragma unroll
      for (int i = 0; i < QB; ++i) {
        qs[i] = q;
        if (q >= 0) {
          load8f(fits[sg.fit + q].r + base, rv[i]);
          if (NSIG == 2) load8f(fits[sg.fit + q].c + base, cv[i]);
          q = next_fold(q);
        }
      }
#pragma unroll
      for (int i = 0; i < QB; ++i) {
        const int qf = qs[i];
        if (qf < 0) continue;
        long long q0[8], q1[8];
        int p0[8];
        unsigned long long pk[8];
        if (W32 && NSIG == 1) {
#pragma unroll
          for (int j = 0; j < 8; ++j) p0[j] = fixed32(rv[i][j], e[2 * qf]);
        } else if (W32) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            pk[j] = pack_signals(fixed32(rv[i][j], e[2 * qf]), fixed32(cv[i][j], e[2 * qf + 1]));
        } else if (r32) {
#pragma unroll
          for (int j = 0; j < 8; ++j) q0[j] = (long long)fixed32(rv[i][j], e[2 * qf]);
          if (NSIG == 2) {
#pragma unroll
            for (int j = 0; j < 8; ++j) q1[j] = (long long)fixed32(cv[i][j], e[2 * qf + 1]);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) q0[j] = fixed_point(rv[i][j], e[2 * qf]);
          if (NSIG == 2) {
#pragma unroll
            for (int j = 0; j < 8; ++j) q1[j] = fixed_point(cv[i][j], e[2 * qf + 1]);
          }
        }
#pragma unroll
        for (int f = 0; f < FMAX; ++f) {
          if (f < nf) {
            const int cb = COPIES ? (lane & cm[f]) * cs[f] : 0;
            if (W32) {
              const size_t w = (size_t)(qf * nf + f) * nb + cb;
              if (NSIG == 1) hist_add32(h32 + w, xc[f], p0);
              else hist_add_packed(hist + w, xc[f], pk);
            } else {
              unsigned long long* hq = hist + (size_t)qf * NSIG * nf * nb;
              hist_add<NSIG>(hq + (size_t)f * nb + cb, xc[f], q0);
              if (NSIG == 2) hist_add<NSIG>(hq + (size_t)(nf + f) * nb + cb, xc[f], q1);
            }
          }
        }
      }
    }
    if (!more) break;
    base = nxt;
  }
}

// Rows [r0, r1) of one segment of unbinned learners: per row and learner,
// the four basis values at the row's code times r (and c), as int64 fixed
// point, into the learner's basis sums (copy lane mod kUnbCopies, stride
// d_max words).  |B r| <= |r|, and each basis sum gets at most one term per
// row, so the exponent of the binned pass is safe here too.
template <int NT, int FMAX, int NSIG>
__device__ __forceinline__ void uhist_rows(const FitDev& F, const Seg& sg,
                                           unsigned long long* __restrict__ hist, int nb,
                                           int64_t r0, int64_t r1, int e0, int e1) {
  const uint32_t* __restrict__ Xg =
      reinterpret_cast<const uint32_t*>(F.X) + (size_t)sg.k0 * F.n_pad;
  const int nf = sg.nf;
  const size_t ld = (size_t)F.n_pad;
  const int copy = ((int)threadIdx.x & (kUnbCopies - 1)) * F.d_max;
  for (int64_t base = r0 + (int64_t)threadIdx.x * 8; base < r1; base += (int64_t)NT * 8) {
    float rv[8], cv[8];
    load8f(F.r + base, rv);
    if (NSIG == 2) load8f(F.c + base, cv);
    uint32_t code[FMAX][8];
#pragma unroll
    for (int f = 0; f < FMAX; ++f)
      if (f < nf) load8c(Xg + f * ld + base, code[f]);
#pragma unroll
    for (int f = 0; f < FMAX; ++f) {
      if (f >= nf) continue;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float b[4];
        cubic4(code[f][j], b);
        const int iv = (int)(code[f][j] >> 24);
        unsigned long long* h0 = hist + (size_t)f * nb + copy + iv;
#pragma unroll
        for (int a = 0; a < 4; ++a)
          __hip_atomic_fetch_add(h0 + a, (unsigned long long)fixed_point(b[a] * rv[j], e0),
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (NSIG == 2) {
          unsigned long long* h1 = hist + (size_t)(nf + f) * nb + copy + iv;
#pragma unroll
          for (int a = 0; a < 4; ++a)
            __hip_atomic_fetch_add(h1 + a, (unsigned long long)fixed_point(b[a] * cv[j], e1),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
  }
}

// NSMAX: most signals any fit of the launch can have (1 when every fit is
// plain CWB, so the two-signal path is not compiled in).  KIND: kBinned
// (one fit per segment), kUnbinned (every fit has unbinned learners) or
// kFolds (binned, with fold groups of a cross-validation).  The fold path
// is compiled into its own variant so that it does not raise the register
// use of the others.  COPIES (binned kinds): some learner of the launch has
// few enough bins for LDS copies (copy_mask); without it the row loops keep
// no copy bases.
constexpr int kBinned = 0, kUnbinned = 1, kFolds = 2;

template <int NT, int FMAX, int NSMAX, int KIND, bool COPIES>
__global__ void __launch_bounds__(NT)
k_hist(const FitDev* __restrict__ fits, const Seg* __restrict__ segs,
       const int64_t* __restrict__ blk, long long* __restrict__ partials, int lds_bytes) {
  constexpr bool UNB = KIND == kUnbinned;
  constexpr bool FOLDS = KIND == kFolds;
  static_assert(FMAX <= 16, "copy table holds 16 learners");
  extern __shared__ unsigned long long s_hist[];
  __shared__ float s_red[NT + 16];
  __shared__ int s_e[2 * kMaxFolds];
  __shared__ int s_cp[2][16];  // binned learners of the segment: copy mask, copy stride
  const int64_t s0 = blk[2 * blockIdx.x], s1 = blk[2 * blockIdx.x + 1];
  int cached_fit = -1;
  Exps ex{};
  for (int64_t s = s0; s < s1; ++s) {
    const Seg sg = segs[s];
    const FitDev& F = fits[sg.fit];
    Ctl* ctl = F.ctl;
    if (ctl->pick_done >= F.M) continue;
    const int switched = ctl->switched;
    const int nsig = is_acwb_step(F, switched) ? 2 : 1;
    const int64_t n_fit = rows_fitted(F, switched);
    const int nb = F.nb_stride;
    const bool w32 = !UNB && sg.acc32 != 0;         // 32-bit (or packed) LDS words
    const int words = sg.nfit * nsig * sg.nf * nb;  // 64-bit LDS words, and partial words
    const int nw32 = sg.nfit * sg.nf * nb;          // 32-bit or packed words
    const int lds_words = w32 ? (nsig == 1 ? (nw32 + 1) / 2 : nw32) : words;
    if ((int64_t)lds_words * 8 > lds_bytes) {  // a schedule the launch's LDS cannot hold
      if (threadIdx.x == 0) atomicOr(&ctl->error, 2);
      continue;
    }
    for (int i = threadIdx.x; i < lds_words; i += NT) s_hist[i] = 0ull;
    if (COPIES && (int)threadIdx.x < sg.nf) {
      int st = 0;
      s_cp[0][threadIdx.x] = copy_mask(F.feat[sg.k0 + threadIdx.x].nb, nb, &st);
      s_cp[1][threadIdx.x] = st;
    }
    __syncthreads();
    const int64_t n8 = (n_fit + 7) >> 3;
    const int64_t U = F.n_pad >> 3;
    const int64_t r0 = 8 * (sg.u0 * n8 / U);
    const int64_t r1 = 8 * (sg.u1 * n8 / U);
    const bool need_e = sg.fit != cached_fit;
    cached_fit = sg.fit;
    if (FOLDS && sg.nfit > 1) {  // the folds of a cross-validation
      const bool r32 = F.acc32_bits > 0;  // the same for every fold of the group
      if (need_e) {
        for (int q = 0; q < sg.nfit; ++q) {
          Exps xq{};
          fit_exponents<NT>(fits[sg.fit + q], n_fit, &xq, s_red);
          if (threadIdx.x == 0) {
            s_e[2 * q] = r32 ? xq.e32[0] : xq.e[0];
            s_e[2 * q + 1] = r32 ? xq.e32[1] : xq.e[1];
          }
        }
        __syncthreads();
      }
      if (w32) {
        if (NSMAX == 1 || nsig == 1)
          hist_rows_folds<NT, FMAX, 1, COPIES, true>(fits, sg, s_hist, nb, r0, r1, s_e, r32, s_cp);
        else
          hist_rows_folds<NT, FMAX, NSMAX, COPIES, true>(fits, sg, s_hist, nb, r0, r1, s_e, r32, s_cp);
      } else {
        if (NSMAX == 1 || nsig == 1)
          hist_rows_folds<NT, FMAX, 1, COPIES, false>(fits, sg, s_hist, nb, r0, r1, s_e, r32, s_cp);
        else
          hist_rows_folds<NT, FMAX, NSMAX, COPIES, false>(fits, sg, s_hist, nb, r0, r1, s_e, r32, s_cp);
      }
    } else if (UNB) {
      if (need_e) fit_exponents<NT>(F, n_fit, &ex, s_red);
      if (NSMAX == 1 || nsig == 1)
        uhist_rows<NT, FMAX, 1>(F, sg, s_hist, nb, r0, r1, ex.e[0], 0);
      else
        uhist_rows<NT, FMAX, NSMAX>(F, sg, s_hist, nb, r0, r1, ex.e[0], ex.e[1]);
    } else if (w32) {
      // 10-bit copies serve one-signal passes only: a one-signal fit's X12,
      // or an HCWB fit's X10h after its switch
      if (F.X12 && F.xbits == 10) {
        hist_rows32<NT, FMAX, 1, 10, COPIES>(F, F.X12, sg, s_hist, nb, r0, r1, ex, need_e, n_fit, s_red, s_cp);
      } else if (nsig == 1 && F.X10h) {
        hist_rows32<NT, FMAX, 1, 10, COPIES>(F, F.X10h, sg, s_hist, nb, r0, r1, ex, need_e, n_fit, s_red, s_cp);
      } else if (F.X12) {
        if (NSMAX == 1 || nsig == 1)
          hist_rows32<NT, FMAX, 1, 12, COPIES>(F, F.X12, sg, s_hist, nb, r0, r1, ex, need_e, n_fit, s_red, s_cp);
        else
          hist_rows32<NT, FMAX, NSMAX, 12, COPIES>(F, F.X12, sg, s_hist, nb, r0, r1, ex, need_e, n_fit, s_red, s_cp);
      } else {
        if (NSMAX == 1 || nsig == 1)
          hist_rows32<NT, FMAX, 1, 16, COPIES>(F, nullptr, sg, s_hist, nb, r0, r1, ex, need_e, n_fit, s_red, s_cp);
        else
          hist_rows32<NT, FMAX, NSMAX, 16, COPIES>(F, nullptr, sg, s_hist, nb, r0, r1, ex, need_e, n_fit, s_red, s_cp);
      }
    } else {
      if (NSMAX == 1 || nsig == 1)
        hist_rows<NT, FMAX, 1, COPIES>(F, sg, s_hist, nb, r0, r1, ex, need_e, n_fit, s_red, s_cp);
      else
        hist_rows<NT, FMAX, NSMAX, COPIES>(F, sg, s_hist, nb, r0, r1, ex, need_e, n_fit, s_red, s_cp);
    }
    __syncthreads();
    GLOBAL long long* out = gp(partials + sg.slot);
    if (w32) {  // 32-bit sums to int64 partials, in the 64-bit layout
      const int nw = sg.nf * nb;
      const uint32_t* h32 = reinterpret_cast<const uint32_t*>(s_hist);
      for (int i = threadIdx.x; i < nw32; i += NT) {
        const int qf = (sg.nfit > 1) ? i / nw : 0;  // fold
        const int j = i - qf * nw;                  // learner j / nb, bin j % nb
        int cm = 0, cs = 0;
        int b = j;
        if (COPIES) {  // the sum of the learner's copies
          const int f = j / nb;
          b = j - f * nb;
          cm = s_cp[0][f];
          cs = s_cp[1][f];
        }
        long long R = 0, Cs = 0;
        if (cm == 0 || b < cs) {
          for (int c = 0, w = i; c <= cm; ++c, w += cs) {
            if (nsig == 1) {
              R += (long long)(int32_t)h32[w];
            } else {
              long long a, e;
              unpack_signals(s_hist[w], &a, &e);
              R += a;
              Cs += e;
            }
          }
        }
        GLOBAL long long* o = out + (size_t)qf * nsig * nw;  // fold qf's slot
        o[j] = R;                    // signal 0 of learner j / nb, bin j % nb
        if (nsig == 2) o[nw + j] = Cs;  // signal 1 at (nf + f) * nb + b
      }
    } else if (UNB) {  // sum the copies: basis sums at the start of each learner's slot
      const int d = F.d_max;
      for (int i = threadIdx.x; i < nsig * sg.nf * d; i += NT) {
        const int lf = i / d, b = i - lf * d;
        long long acc = 0;
#pragma unroll
        for (int c = 0; c < kUnbCopies; ++c) acc += (long long)s_hist[(size_t)lf * nb + c * d + b];
        out[(size_t)lf * nb + b] = acc;
      }
    } else if (!COPIES) {
      for (int i = threadIdx.x; i < words; i += NT) out[i] = (long long)s_hist[i];
    } else {  // sum each learner's copies; words past its copies' stride are zero
      const int nlf = sg.nfit * nsig * sg.nf;
      for (int lf = 0, f = 0; lf < nlf; ++lf, f = (f + 1 == sg.nf) ? 0 : f + 1) {
        const unsigned long long* h = s_hist + (size_t)lf * nb;
        GLOBAL long long* o = out + (size_t)lf * nb;
        const int cm = s_cp[0][f], cs = s_cp[1][f];
        if (cm == 0) {
          for (int b = threadIdx.x; b < nb; b += NT) o[b] = (long long)h[b];
        } else {
          for (int b = threadIdx.x; b < nb; b += NT) {
            long long acc = 0;
            if (b < cs)
              for (int c = 0; c <= cm; ++c) acc += (long long)h[b + c * cs];
            o[b] = acc;
          }
        }
      }
    }
    __syncthreads();
  }
}


namespace {

template <int NT, int FMAX, int NSMAX, int KIND, bool COPIES>
hipError_t launch_hist_t(hipStream_t st, int blocks, size_t lds, const FitDev* fits, const Seg* segs,
                         const int64_t* blk, long long* partials) {
  // 160 KiB per workgroup minus the kernel's static LDS (at most ~4 KiB);
  // set once (thread-safe static initialisation), before any graph capture
  static const bool attr = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hist<NT, FMAX, NSMAX, KIND, COPIES>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kHistMaxLds);
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_hist<NT, FMAX, NSMAX, KIND, COPIES>), dim3(blocks), dim3(NT), lds, st, fits, segs,
                     blk, partials, (int)lds);
  return hipGetLastError();
}

template <int NT, int NSMAX, int KIND, bool COPIES>
hipError_t launch_hist_nt(hipStream_t st, int fmax, int blocks, size_t lds, const FitDev* fits,
                          const Seg* segs, const int64_t* blk, long long* partials) {
  switch (fmax) {
    case 1: return launch_hist_t<NT, 1, NSMAX, KIND, COPIES>(st, blocks, lds, fits, segs, blk, partials);
    case 2: return launch_hist_t<NT, 2, NSMAX, KIND, COPIES>(st, blocks, lds, fits, segs, blk, partials);
    case 4: return launch_hist_t<NT, 4, NSMAX, KIND, COPIES>(st, blocks, lds, fits, segs, blk, partials);
    case 8: return launch_hist_t<NT, 8, NSMAX, KIND, COPIES>(st, blocks, lds, fits, segs, blk, partials);
    case 16:  // binned kinds only (the unbinned variant holds 32-bit codes)
      if (KIND == kBinned) return launch_hist_t<NT, 16, NSMAX, kBinned, COPIES>(st, blocks, lds, fits, segs, blk, partials);
      if (KIND == kFolds) return launch_hist_t<NT, 16, NSMAX, kFolds, COPIES>(st, blocks, lds, fits, segs, blk, partials);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int NSMAX, int KIND, bool COPIES>
hipError_t launch_hist_ns(hipStream_t st, int nt, int fmax, int blocks, size_t lds,
                          const FitDev* fits, const Seg* segs, const int64_t* blk,
                          long long* partials) {
  switch (nt) {
    case 256: return launch_hist_nt<256, NSMAX, KIND, COPIES>(st, fmax, blocks, lds, fits, segs, blk, partials);
    case 512: return launch_hist_nt<512, NSMAX, KIND, COPIES>(st, fmax, blocks, lds, fits, segs, blk, partials);
    case 1024: return launch_hist_nt<1024, NSMAX, KIND, COPIES>(st, fmax, blocks, lds, fits, segs, blk, partials);
    default: return hipErrorInvalidValue;
  }
}

template <int KIND, bool COPIES>
hipError_t launch_hist_k(hipStream_t st, int nt, int fmax, int nsmax, int blocks, size_t lds,
                         const FitDev* fits, const Seg* segs, const int64_t* blk, long long* partials) {
  if (nsmax == 1) return launch_hist_ns<1, KIND, COPIES>(st, nt, fmax, blocks, lds, fits, segs, blk, partials);
  return launch_hist_ns<2, KIND, COPIES>(st, nt, fmax, blocks, lds, fits, segs, blk, partials);
}

}  // namespace

hipError_t launch_hist(hipStream_t st, int nt, int fmax, int nsmax, bool unbinned, bool folds,
                       bool copies, int blocks, size_t lds, const FitDev* fits, const Seg* segs,
                       const int64_t* blk, long long* partials) {
  if (blocks <= 0) return hipSuccess;
  if (unbinned && folds) return hipErrorInvalidValue;
  if (unbinned) return launch_hist_k<kUnbinned, false>(st, nt, fmax, nsmax, blocks, lds, fits, segs, blk, partials);
  if (folds) {
    if (copies) return launch_hist_k<kFolds, true>(st, nt, fmax, nsmax, blocks, lds, fits, segs, blk, partials);
    return launch_hist_k<kFolds, false>(st, nt, fmax, nsmax, blocks, lds, fits, segs, blk, partials);
  }
  if (copies) return launch_hist_k<kBinned, true>(st, nt, fmax, nsmax, blocks, lds, fits, segs, blk, partials);
  return launch_hist_k<kBinned, false>(st, nt, fmax, nsmax, blocks, lds, fits, segs, blk, partials);
}

}  // namespace cwb

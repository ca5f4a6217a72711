// kernels.hip -- gfx950 kernels of one boosting iteration.
//
// Per iteration m (Algorithm A1 for CWB, Algorithm 2 for ACWB, Algorithm 3
// for HCWB) the host enqueues, for every fit of a batch at once:
//   k_state   row pass: apply the update tables selected in iteration m-1
//             (f += nu b_k, h += eta b_kcor), form g = (1-theta_m) f +
//             theta_m h (ACWB), the pseudo-residuals r = -dL/df and the
//             error-corrected residuals c (ACWB), FP64 partial risks, and the
//             per-block largest |r|, |c| (fixed-point scale of the histograms).
//   k_hist    histogram pass over the uint16 bin-index matrix: for every
//             learner k and design point l, s_kl = sum of r_i over the rows
//             with ind_ki = l (binMatVec, Algorithm 1, first stage), and the
//             same for c.  Each block accumulates int64 fixed-point sums in
//             LDS and flushes them once per segment; int64 addition is exact,
//             so the result does not depend on the order of the atomics or on
//             the schedule.
//   k_select  one block per learner: merge the segment partials, v = Z^bT s
//             (second stage of binMatVec), theta = (G + lambda D)^-1 v with
//             the cached inverse (Section 2.4), criterion
//             q = theta^T G theta - 2 theta^T v, so SSE_k = r^T r + q_k
//             (Algorithm A1's SSE), and the candidate update table Z^b theta.
//   k_pick    one block per fit: argmin_k q (ties to the lowest k), traces,
//             aggregated coefficients (Section 2.3 / 3.2.1), and the update
//             armed for the next row pass.
//   k_valrisk (HCWB, ACWB phase) validation-risk partials of the new primary
//   k_valdecide  model, then the patience counter that decides the switch.
// Cross-block results pass through kernel boundaries only: on this chip a
// device-scope fence writes back the issuing XCD's L2, which is far more
// expensive than one more launch.
#include <hip/hip_runtime.h>

#include "../../include/cwb.h"
#include "cwb_internal.h"
#include "kernels.h"

namespace cwb {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Pointers read out of the fit descriptors are generic; casting them to the
// global address space makes the compiler emit global_load/global_store
// instead of flat accesses (flat accesses also count against the LDS
// wait counter, which would serialise HBM loads behind LDS atomics).
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* gp(T* p) {
  return (GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const GLOBAL T* gp(const T* p) {
  return (const GLOBAL T*)p;
}

__device__ __forceinline__ bool is_acwb_step(const FitDev& F, int switched) {
  return F.variant == CWB_ACWB || (F.variant == CWB_HCWB && !switched);
}
__device__ __forceinline__ int64_t rows_fitted(const FitDev& F, int switched) {
  return (F.variant == CWB_HCWB && switched) ? F.n : F.n_train;
}
__device__ __forceinline__ int gram_set(const FitDev& F, int switched) {
  return (F.variant == CWB_HCWB && switched) ? 1 : 0;
}

// Pseudo-residual -dL/df (L2: (y-f)^2/2; binomial: log(1+e^f) - y f).
__device__ __forceinline__ float neg_gradient(int loss, float y, float f) {
  if (loss == CWB_L2) return y - f;
  return y - 1.0f / (1.0f + expf(-f));
}

__device__ __forceinline__ double loss_value(int loss, float y, float f) {
  const double fd = (double)f, yd = (double)y;
  if (loss == CWB_L2) {
    const double e = yd - fd;
    return 0.5 * e * e;
  }
  const double sp = fd > 0.0 ? fd + log1p(exp(-fd)) : log1p(exp(fd));
  return sp - yd * fd;
}

// Deterministic block sum (thread 0 gets the result): every thread stores its
// value, 16 threads add 16 consecutive chunks in order, thread 0 adds those.
// red must hold NT + 16 doubles.
template <int NT>
__device__ double block_sum(double v, double* red) {
  constexpr int kParts = 16, kPer = NT / kParts;
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < kParts) {
    double a = 0.0;
    for (int i = 0; i < kPer; ++i) a += red[threadIdx.x * kPer + i];
    red[NT + threadIdx.x] = a;
  }
  __syncthreads();
  double sum = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kParts; ++i) sum += red[NT + i];
  __syncthreads();
  return sum;
}

// Block maximum of non-negative floats (every thread gets the result);
// red must hold NT + 16 floats.
template <int NT>
__device__ float block_max(float v, float* red) {
  constexpr int kParts = 16, kPer = NT / kParts;
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < kParts) {
    float a = 0.0f;
    for (int i = 0; i < kPer; ++i) a = fmaxf(a, red[threadIdx.x * kPer + i]);
    red[NT + threadIdx.x] = a;
  }
  __syncthreads();
  float m = 0.0f;
  for (int i = 0; i < kParts; ++i) m = fmaxf(m, red[NT + i]);
  __syncthreads();
  return m;
}

// Scale exponent of signal `sig` of a fit: maximum over the row-pass blocks
// maxima (order-free, so every block computes the same value).  red must
// hold NT + 16 floats.
template <int NT>
__device__ int fit_scale_exponent(const FitDev& F, int sig, int64_t n_fit, float* red) {
  float a = 0.0f;
  const GLOBAL float* am = gp(F.amax_part);
  for (int b0 = 0; b0 < F.n_row_blocks; b0 += 4 * NT) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * NT + (int)threadIdx.x;
      v[u] = (b < F.n_row_blocks) ? am[2 * b + sig] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) a = fmaxf(a, v[u]);
  }
  return scale_exponent(block_max<NT>(a, red), n_fit);
}

// Copy `count` elements from global memory to LDS with all of a thread's
// loads (up to U per pass) issued before its stores, so a block pays one
// memory round trip per pass instead of one per element it copies.
template <int NT, int U, typename T>
__device__ __forceinline__ void stage(T* dst, const T* src, int count) {
  const GLOBAL T* g = gp(src);
  for (int i0 = 0; i0 < count; i0 += NT * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT + (int)threadIdx.x;
      if (i < count) v[u] = g[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT + (int)threadIdx.x;
      if (i < count) dst[i] = v[u];
    }
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef long long i64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void load8f(const float* p, float* v) {
  const GLOBAL f32x4* q = (const GLOBAL f32x4*)p;
  const f32x4 a = q[0], b = q[1];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ __forceinline__ void store8f(float* p, const float* v) {
  GLOBAL f32x4* q = (GLOBAL f32x4*)p;
  f32x4 a, b;
  a.x = v[0]; a.y = v[1]; a.z = v[2]; a.w = v[3];
  b.x = v[4]; b.y = v[5]; b.z = v[6]; b.w = v[7];
  q[0] = a;
  q[1] = b;
}

__device__ __forceinline__ void load8u(const uint16_t* p, uint32_t* idx) {
  const u32x4 w = *(const GLOBAL u32x4*)p;
  idx[0] = w.x & 0xffffu; idx[1] = w.x >> 16;
  idx[2] = w.y & 0xffffu; idx[3] = w.y >> 16;
  idx[4] = w.z & 0xffffu; idx[5] = w.z >> 16;
  idx[6] = w.w & 0xffffu; idx[7] = w.w >> 16;
}

// 8 unbinned codes (32-bit) of consecutive rows.
__device__ __forceinline__ void load8c(const uint32_t* p, uint32_t* c) {
  const u32x4 a = *(const GLOBAL u32x4*)p;
  const u32x4 b = *(const GLOBAL u32x4*)(p + 4);
  c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w;
  c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
}

// The four nonzero cubic B-spline values at position t of a knot interval
// (equally spaced knots: the uniform cubic segments).
__device__ __forceinline__ void cubic4(uint32_t code, float* b) {
  const float t = (float)(code & kUnbFracMax) * (1.0f / (float)kUnbFracMax);
  const float s = 1.0f - t, t2 = t * t, t3 = t2 * t;
  b[0] = s * s * s * (1.0f / 6.0f);
  b[1] = (3.0f * t3 - 6.0f * t2 + 4.0f) * (1.0f / 6.0f);
  b[2] = (-3.0f * t3 + 3.0f * t2 + 3.0f * t + 1.0f) * (1.0f / 6.0f);
  b[3] = t3 * (1.0f / 6.0f);
}

// (Z theta)_i of an unbinned learner: its basis at the row's code against
// the coefficient table.
__device__ __forceinline__ float unb_eval(uint32_t code, const float* tab) {
  float b[4];
  cubic4(code, b);
  const int iv = (int)(code >> 24);
  return b[0] * tab[iv] + b[1] * tab[iv + 1] + b[2] * tab[iv + 2] + b[3] * tab[iv + 3];
}

// Update-table lookup of one row: the bin's entry, or the basis expansion.
__device__ __forceinline__ float table_at(bool unb, uint32_t idx, const float* tab) {
  return unb ? unb_eval(idx, tab) : tab[idx];
}

}  // namespace

// ---------------------------------------------------------------------------
// Row pass.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kStateThreads)
k_state(const RowItem* __restrict__ items, int final_mode) {
  extern __shared__ float s_tab[];  // [2][nb_max]
  __shared__ double s_red[kStateThreads + 16];
  __shared__ float s_fred[kStateThreads + 16];
  __shared__ int s_bad;
  const RowItem it = items[blockIdx.x];
  // one round: the control block and this thread's rows of the model state
  const Ctl* ctl = it.ctl;
  const int m_done = ctl->m_done;
  const int pending = ctl->pending;
  const int pend_acwb = ctl->pend_acwb;
  const int kk = ctl->k;
  const int kc = ctl->kcor;
  const int switched = ctl->switched;
  const float eta = (float)ctl->eta;
  const int64_t base = it.base + (int64_t)threadIdx.x * kRowsPerThread;
  const bool rows = base < it.n_pad;
  const bool two = it.two != 0;
  float f[8], yv[8], hv[8], cv[8], rr[8], cc[8];
  if (rows) {
    load8f(it.fg + base, f);
    load8f(it.y + base, yv);
    if (two) {
      load8f(it.h + base, hv);
      load8f(it.c + base, cv);
    }
  }
  if (!final_mode && m_done >= it.M) return;
  const float nu = (float)it.nu;
  const int m = m_done + 1;
  const bool acwb =
      !final_mode && (it.variant == CWB_ACWB || (it.variant == CWB_HCWB && !switched));
  const int64_t n_fit = (it.variant == CWB_HCWB && switched) ? it.n : it.n_train;
  const int nb = it.nb_max;
  float* tf = s_tab;
  float* tc = s_tab + nb;
  const bool use_t = pending != 0;
  const bool use_h = pending && pend_acwb && kc >= 0;
  const bool use_cc = acwb && m > 1 && kc >= 0;
  uint32_t ik[8], ic[8];
  const bool unb = it.unbinned != 0;
  if (unb) {
    const uint32_t* XU = reinterpret_cast<const uint32_t*>(it.X);
    if (rows && use_t) load8c(XU + (size_t)kk * it.n_pad + base, ik);
    if (rows && (use_h || use_cc)) load8c(XU + (size_t)kc * it.n_pad + base, ic);
  } else {
    if (rows && use_t) load8u(it.X + (size_t)kk * it.n_pad + base, ik);
    if (rows && (use_h || use_cc)) load8u(it.X + (size_t)kc * it.n_pad + base, ic);
  }
  if (use_t) stage<kStateThreads, 4>(tf, it.table + (size_t)kk * nb, nb);
  if (use_h || use_cc) stage<kStateThreads, 4>(tc, it.table + ((size_t)it.p + kc) * nb, nb);
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();

  double risk_t = 0.0, risk_v = 0.0;
  float amax_r = 0.0f, amax_c = 0.0f;
  bool bad = false;
  if (rows) {
    const float vt = 2.0f / (float)(m + 1);
    const float cw = (float)m / (float)(m + 1);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t i = base + j;
      const bool live = i < it.n;
      float fj = f[j];
      float hj = two ? hv[j] : 0.0f;
      if (live && use_t) fj = fj + nu * table_at(unb, ik[j], tf);
      if (live && use_h) hj = hj + eta * table_at(unb, ic[j], tc);
      if (live) {
        const double L = loss_value(it.loss, yv[j], fj);
        if (i < it.n_train) risk_t += L; else risk_v += L;
        if (!isfinite(fj) || !isfinite(hj)) bad = true;
      }
      f[j] = fj;
      hv[j] = hj;
      rr[j] = 0.0f;
      cc[j] = 0.0f;
      if (final_mode || !live) continue;
      const bool fitrow = i < n_fit;
      if (acwb) {
        const float g = (1.0f - vt) * fj + vt * hj;
        const float r = neg_gradient(it.loss, yv[j], g);
        float c = r;
        if (use_cc) c = r + cw * (cv[j] - table_at(unb, ic[j], tc));
        f[j] = g;  // the primary model update f = g + nu b_k is pending
        if (fitrow) {
          rr[j] = r;
          cc[j] = c;
        }
      } else {
        const float r = neg_gradient(it.loss, yv[j], fj);
        if (fitrow) rr[j] = r;
      }
      amax_r = fmaxf(amax_r, fabsf(rr[j]));
      amax_c = fmaxf(amax_c, fabsf(cc[j]));
    }
    store8f(it.fg + base, f);
    if (two) store8f(it.h + base, hv);
    if (!final_mode) {
      store8f(it.r + base, rr);
      if (acwb) store8f(it.c + base, cc);
    }
  }
  if (bad) s_bad = 1;
  const double st = block_sum<kStateThreads>(risk_t, s_red);
  const double sv = block_sum<kStateThreads>(risk_v, s_red);
  const float a = block_max<kStateThreads>(amax_r, s_fred);
  const float b = block_max<kStateThreads>(amax_c, s_fred);
  if (threadIdx.x == 0) {
    it.risk_part[0] = st;
    it.risk_part[1] = sv;
    if (!final_mode) {
      if (!isfinite(a) || !isfinite(b)) s_bad = 1;
      it.amax_part[0] = a;
      it.amax_part[1] = b;
    }
    if (s_bad) atomicOr(&it.ctl->error, 1);
  }
}

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

__device__ __forceinline__ u32x4 load_idx(const uint16_t* p) {
  return __builtin_nontemporal_load((const GLOBAL u32x4*)p);
}

// trunc(r * 2^e) as int64, from the bits of the float: r = +-m 2^(x-150)
// with a 24-bit integer m, so the product is m shifted by x - 150 + e.
// Equal to casting the exact double product r * 2^e to int64.
__device__ __forceinline__ long long fixed_point(float r, int e) {
  const uint32_t u = __float_as_uint(r);
  const uint32_t ex = (u >> 23) & 0xffu;
  const uint32_t m = (u & 0x7fffffu) | (ex ? 0x800000u : 0u);
  const int sh = (ex ? (int)ex : 1) - 150 + e;
  unsigned long long mag;
  if (sh >= 0) mag = (unsigned long long)m << sh;  // sh <= 62 - 24 by the choice of e
  else mag = (sh > -32) ? (unsigned long long)(m >> (-sh)) : 0ull;
  return (u >> 31) ? -(long long)mag : (long long)mag;
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

// Rows [r0, r1) of one segment.  Every thread takes 8 consecutive rows per
// step: one 32-byte load of residuals per signal and one 16-byte load of bin
// indices per learner of the group, then 8 LDS atomics per learner and
// signal.  The next step's loads are issued before this step's atomics.
template <int NT, int FMAX, int NSIG>
__device__ __forceinline__ void hist_rows(const FitDev& F, const Seg& sg,
                                          unsigned long long* __restrict__ hist, int nb,
                                          int64_t r0, int64_t r1, int e0, int e1) {
  const uint16_t* __restrict__ Xg = F.X + (size_t)sg.k0 * F.n_pad;
  const int nf = sg.nf;
  const size_t ld = (size_t)F.n_pad;
  int64_t base = r0 + (int64_t)threadIdx.x * 8;
  if (base >= r1) return;
  float rv[8], cv[8];
  u32x4 xw[FMAX];
  hist_step_load<FMAX, NSIG>(F, Xg, ld, nf, base, rv, cv, xw);
  for (;;) {
    const int64_t nxt = base + (int64_t)NT * 8;
    const bool more = nxt < r1;
    long long q0[8], q1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) q0[j] = fixed_point(rv[j], e0);
    if (NSIG == 2) {
#pragma unroll
      for (int j = 0; j < 8; ++j) q1[j] = fixed_point(cv[j], e1);
    }
    u32x4 xc[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; ++f) xc[f] = xw[f];
    if (more) hist_step_load<FMAX, NSIG>(F, Xg, ld, nf, nxt, rv, cv, xw);
#pragma unroll
    for (int f = 0; f < FMAX; ++f) {
      if (f < nf) {
        hist_add<NSIG>(hist + (size_t)f * nb, xc[f], q0);
        if (NSIG == 2) hist_add<NSIG>(hist + (size_t)(nf + f) * nb, xc[f], q1);
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
// plain CWB, so the two-signal path is not compiled in).  UNB: every fit of
// the launch has unbinned learners.
template <int NT, int FMAX, int NSMAX, bool UNB>
__global__ void __launch_bounds__(NT)
k_hist(const FitDev* __restrict__ fits, const Seg* __restrict__ segs,
       const int64_t* __restrict__ blk, long long* __restrict__ partials) {
  extern __shared__ unsigned long long s_hist[];
  __shared__ float s_red[NT + 16];
  const int64_t s0 = blk[2 * blockIdx.x], s1 = blk[2 * blockIdx.x + 1];
  int cached_fit = -1;
  int e0 = 0, e1 = 0;
  for (int64_t s = s0; s < s1; ++s) {
    const Seg sg = segs[s];
    const FitDev& F = fits[sg.fit];
    const Ctl* ctl = F.ctl;
    if (ctl->m_done >= F.M) continue;
    const int switched = ctl->switched;
    const int nsig = is_acwb_step(F, switched) ? 2 : 1;
    const int64_t n_fit = rows_fitted(F, switched);
    const int nb = F.nb_stride;
    const int words = nsig * sg.nf * nb;
    for (int i = threadIdx.x; i < words; i += NT) s_hist[i] = 0ull;
    __syncthreads();
    const int64_t n8 = (n_fit + 7) >> 3;
    const int64_t U = F.n_pad >> 3;
    const int64_t r0 = 8 * (sg.u0 * n8 / U);
    const int64_t r1 = 8 * (sg.u1 * n8 / U);
    if (sg.fit != cached_fit) {
      e0 = fit_scale_exponent<NT>(F, 0, n_fit, s_red);
      e1 = (nsig == 2) ? fit_scale_exponent<NT>(F, 1, n_fit, s_red) : 0;
      cached_fit = sg.fit;
    }
    if (UNB) {
      if (NSMAX == 1 || nsig == 1)
        uhist_rows<NT, FMAX, 1>(F, sg, s_hist, nb, r0, r1, e0, 0);
      else
        uhist_rows<NT, FMAX, NSMAX>(F, sg, s_hist, nb, r0, r1, e0, e1);
    } else {
      if (NSMAX == 1 || nsig == 1)
        hist_rows<NT, FMAX, 1>(F, sg, s_hist, nb, r0, r1, e0, 0);
      else
        hist_rows<NT, FMAX, NSMAX>(F, sg, s_hist, nb, r0, r1, e0, e1);
    }
    __syncthreads();
    GLOBAL long long* out = gp(partials + sg.slot);
    if (UNB) {  // sum the copies: basis sums at the start of each learner's slot
      const int d = F.d_max;
      for (int i = threadIdx.x; i < nsig * sg.nf * d; i += NT) {
        const int lf = i / d, b = i - lf * d;
        long long acc = 0;
#pragma unroll
        for (int c = 0; c < kUnbCopies; ++c) acc += (long long)s_hist[(size_t)lf * nb + c * d + b];
        out[(size_t)lf * nb + b] = acc;
      }
    } else {
      for (int i = threadIdx.x; i < words; i += NT) out[i] = (long long)s_hist[i];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-learner solve and selection.
// ---------------------------------------------------------------------------
namespace {

struct Best {
  double q;
  int k;
};

__device__ __forceinline__ bool better(double qa, int ka, double qb, int kb) {
  return qa < qb || (qa == qb && ka < kb);
}

// Running argmin (ties: lowest k) with the runner-up value.
struct Arg2 {
  double b1, b2;
  int k1;
  __device__ __forceinline__ void add(double v, int k) {
    if (better(v, k, b1, k1)) {
      b2 = b1;
      b1 = v;
      k1 = k;
    } else if (v < b2) {
      b2 = v;
    }
  }
  __device__ __forceinline__ void merge(double c1, double c2, int kc) {
    if (better(c1, kc, b1, k1)) {
      b2 = fmin(b1, c2);
      b1 = c1;
      k1 = kc;
    } else {
      b2 = fmin(b2, c1);
    }
  }
};

// Deterministic sum of risk partials of the row-pass blocks.
__device__ double sum_partials(const double* part, int count, int stride, int offset,
                               double* red) {
  const GLOBAL double* g = gp(part);
  double s = 0.0;
  for (int b0 = 0; b0 < count; b0 += 4 * kSelectThreads) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * kSelectThreads + (int)threadIdx.x;
      v[u] = (b < count) ? g[(size_t)b * stride + offset] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += v[u];
  }
  return block_sum<kSelectThreads>(s, red);
}

// Selection of iteration m (Algorithm A1's argmin; with `nsig` = 2 also the
// ACWB correction fit of Algorithm 2): argmin of the criteria, the traces,
// and the update armed for the next row pass.  Two rounds of global loads:
// the criteria of both signals with the risk partials, then the winners'
// coefficients.  The aggregated coefficients are formed from the traces
// when the model is read (k_coef).
__device__ void pick(const FitDev& F, Ctl* ctl, int m, bool acwb, int nsig) {
  __shared__ double s_b1[2][kSelectThreads], s_b2[2][kSelectThreads];
  __shared__ int s_k[2][kSelectThreads];
  __shared__ double s_red[kSelectThreads + 16];
  const int p = F.p;
  const GLOBAL double* q = gp(F.q);
  const GLOBAL double* rp = gp(F.risk_part);
  Arg2 a0{INFINITY, INFINITY, p}, a1{INFINITY, INFINITY, p};
  double rt = 0.0, rv = 0.0;
  const int n = p > F.n_row_blocks ? p : F.n_row_blocks;
  for (int t = threadIdx.x; t < n; t += kSelectThreads) {
    double v0 = INFINITY, v1 = INFINITY, r0 = 0.0, r1 = 0.0;
    if (t < p) {
      v0 = q[t];
      if (nsig == 2) v1 = q[p + t];
    }
    if (t < F.n_row_blocks) {
      r0 = rp[2 * (size_t)t];
      r1 = rp[2 * (size_t)t + 1];
    }
    if (t < p) {
      a0.add(v0, t);
      if (nsig == 2) a1.add(v1, t);
    }
    rt += r0;
    rv += r1;
  }
  s_b1[0][threadIdx.x] = a0.b1;
  s_b2[0][threadIdx.x] = a0.b2;
  s_k[0][threadIdx.x] = a0.k1;
  s_b1[1][threadIdx.x] = a1.b1;
  s_b2[1][threadIdx.x] = a1.b2;
  s_k[1][threadIdx.x] = a1.k1;
  __syncthreads();
  for (int stride = kSelectThreads / 2; stride > 0; stride >>= 1) {
    if (threadIdx.x < stride) {
      const int o = threadIdx.x + stride;
#pragma unroll
      for (int sig = 0; sig < 2; ++sig) {
        Arg2 a{s_b1[sig][threadIdx.x], s_b2[sig][threadIdx.x], s_k[sig][threadIdx.x]};
        a.merge(s_b1[sig][o], s_b2[sig][o], s_k[sig][o]);
        s_b1[sig][threadIdx.x] = a.b1;
        s_b2[sig][threadIdx.x] = a.b2;
        s_k[sig][threadIdx.x] = a.k1;
      }
    }
    __syncthreads();
  }
  const double sum_t = block_sum<kSelectThreads>(rt, s_red);
  const double sum_v = block_sum<kSelectThreads>(rv, s_red);
  int k0 = s_k[0][0];
  int k1 = (nsig == 2) ? s_k[1][0] : -1;
  // criteria that are all non-finite select nothing: flag the fit
  const bool bad = k0 >= p || (nsig == 2 && k1 >= p);
  if (bad) {
    k0 = 0;
    k1 = (nsig == 2) ? 0 : -1;
  }
  const int mi = m - 1;
  const int dmax = F.d_max;
  const double vt = 2.0 / ((double)m + 1.0);
  const double eta = acwb ? F.gamma * F.nu / vt : 0.0;
  const GLOBAL double* th = gp(F.theta);
  for (int j = threadIdx.x; j < dmax; j += kSelectThreads) {
    const double t0 = th[(size_t)k0 * dmax + j];
    const double t1 = (k1 >= 0) ? th[((size_t)p + k1) * dmax + j] : 0.0;
    F.tr_theta[(size_t)mi * dmax + j] = t0;
    F.tr_thetacor[(size_t)mi * dmax + j] = t1;
  }
  if (threadIdx.x == 0) {
    F.tr_k[mi] = k0;
    F.tr_kcor[mi] = k1;
    F.tr_gap[mi] = s_b2[0][0] - s_b1[0][0];
    F.tr_risk[mi] = sum_t / (double)F.n_train;  // risk of f^[m-1]
    F.tr_val[mi] = (F.n > F.n_train) ? sum_v / (double)(F.n - F.n_train) : 0.0;
    if (bad) ctl->error = 1;
    ctl->pending = 1;
    ctl->pend_acwb = acwb ? 1 : 0;
    ctl->k = k0;
    ctl->kcor = k1;
    ctl->eta = eta;
    ctl->m_done = m;
  }
}

}  // namespace

constexpr int kChunks = 8;  // partial sums per output of a small contraction

// out = M x for a d x d matrix in LDS, as fixed-order two-level sums.
__device__ __forceinline__ void mat_vec(const double* M, const double* x, double* out, int d,
                                        double* part) {
  const int per = (d + kChunks - 1) / kChunks;
  for (int t = threadIdx.x; t < d * kChunks; t += kSelectThreads) {
    const int j = t / kChunks, c = t % kChunks;
    const int i0 = c * per, i1 = (i0 + per < d) ? i0 + per : d;
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) acc += M[j * d + i] * x[i];
    part[t] = acc;
  }
  __syncthreads();
  if (threadIdx.x < d) {
    double acc = 0.0;
    for (int c = 0; c < kChunks; ++c) acc += part[threadIdx.x * kChunks + c];
    out[threadIdx.x] = acc;
  }
  __syncthreads();
}

// Loads for one learner's solve: from LDS when the learner's reduced design
// was staged there, else from global memory.
struct Basis {
  const double* bval;    // [nb][kMaxBand]
  const int32_t* bstart; // [nb]
};

template <bool STAGED>
__global__ void __launch_bounds__(kSelectThreads)
k_select(const SelItem* __restrict__ items, const long long* __restrict__ partials, int nb_cap,
         int d_cap) {
  // dynamic LDS: s[nb_cap] | Ainv[d_cap^2] | G[d_cap^2] | (STAGED) bval[nb_cap*4] | bstart[nb_cap]
  extern __shared__ double s_dyn[];
  __shared__ double s_v[kMaxD], s_th[kMaxD], s_gt[kMaxD];
  __shared__ double s_part[kMaxD * kChunks];
  __shared__ long long s_off[kNumSig][kMaxSlots];
  __shared__ int s_jr[2 * kMaxD];
  __shared__ float s_red[kSelectThreads + 16];
  double* s_bins = s_dyn;
  double* s_ai = s_dyn + nb_cap;
  double* s_g = s_ai + (size_t)d_cap * d_cap;
  double* s_bv = s_g + (size_t)d_cap * d_cap;
  int* s_bs = reinterpret_cast<int*>(s_bv + (size_t)nb_cap * kMaxBand);
  const SelItem it = items[blockIdx.x];
  const int d = it.d, nb = it.nb, band = it.band, n_off = it.n_off;
  // one round of independent loads: control block, signal maxima, offsets,
  // the learner's tables for the training-row Gram set
  const int m_done = it.ctl->m_done;
  const int switched = it.ctl->switched;
  float am0 = 0.0f, am1 = 0.0f;
  {
    const GLOBAL f32x2* am = (const GLOBAL f32x2*)it.amax_part;
    for (int b0 = 0; b0 < it.n_row_blocks; b0 += 4 * kSelectThreads) {
      f32x2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + u * kSelectThreads + (int)threadIdx.x;
        if (b < it.n_row_blocks) v[u] = am[b];
        else v[u].x = v[u].y = 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        am0 = fmaxf(am0, v[u].x);
        am1 = fmaxf(am1, v[u].y);
      }
    }
  }
  const int n_stage = n_off < kMaxSlots ? n_off : kMaxSlots;
  {
    stage<kSelectThreads, 2>(s_off[0], (const long long*)it.offs, n_stage);
    if (it.variant != CWB_CWB) stage<kSelectThreads, 2>(s_off[1], (const long long*)it.offs + n_off, n_stage);
    stage<kSelectThreads, 4>(s_ai, it.ainv[0], d * d);
    stage<kSelectThreads, 4>(s_g, it.gram[0], d * d);
    stage<kSelectThreads, 1>(s_jr, it.jr, 2 * d);
    if (STAGED) {
      stage<kSelectThreads, 16>(s_bv, it.bval, nb * kMaxBand);
      stage<kSelectThreads, 4>(s_bs, it.bstart, nb);
    }
  }
  if (m_done >= it.M) return;
  const bool hcwb_all = it.variant == CWB_HCWB && switched;
  const bool acwb = it.variant == CWB_ACWB || (it.variant == CWB_HCWB && !switched);
  const int nsig = acwb ? 2 : 1;
  const int64_t n_fit = hcwb_all ? it.n : it.n_train;
  if (hcwb_all) {  // HCWB after the switch: Grams over all rows
    __syncthreads();
    stage<kSelectThreads, 4>(s_ai, it.ainv[1], d * d);
    stage<kSelectThreads, 4>(s_g, it.gram[1], d * d);
  }
  const Basis B = STAGED ? Basis{s_bv, s_bs} : Basis{it.bval, it.bstart};
  const float amax[2] = {block_max<kSelectThreads>(am0, s_red), block_max<kSelectThreads>(am1, s_red)};
  for (int sig = 0; sig < nsig; ++sig) {
    const double isc = ldexp(1.0, -scale_exponent(amax[sig], n_fit));
    // bin sums s_l: exact int64 merge of the group's segment partials
    for (int l0 = 0; l0 < nb; l0 += 4 * kSelectThreads) {
      long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      const int l = l0 + 4 * threadIdx.x;
      for (int c0 = 0; c0 < n_off; c0 += kMaxSlots) {
        const int cnt = (n_off - c0) < kMaxSlots ? (n_off - c0) : kMaxSlots;
        const long long* so = s_off[sig];
        if (n_off > kMaxSlots) {  // more segments than the staged list holds
          __syncthreads();
          stage<kSelectThreads, 2>(s_off[sig], (const long long*)(it.offs + (int64_t)sig * n_off + c0), cnt);
          __syncthreads();
        }
        if (l < nb) {
#pragma unroll 16
          for (int i = 0; i < cnt; ++i) {
            const GLOBAL i64x2* src = (const GLOBAL i64x2*)(partials + so[i] + l);
            const i64x2 u = src[0], w = src[1];
            a0 += u.x;
            a1 += u.y;
            a2 += w.x;
            a3 += w.y;
          }
        }
      }
      if (l < nb) s_bins[l] = (double)a0 * isc;
      if (l + 1 < nb) s_bins[l + 1] = (double)a1 * isc;
      if (l + 2 < nb) s_bins[l + 2] = (double)a2 * isc;
      if (l + 3 < nb) s_bins[l + 3] = (double)a3 * isc;
    }
    __syncthreads();
    // Small FP64 contractions, each as fixed-order two-level sums: thread
    // (j, c) adds a chunk of terms into s_part[j][c], then thread j adds its
    // kChunks partials in order.
    // v_j = sum_l Z^b[l, j] s_l over the design points supporting basis j
    for (int t = threadIdx.x; t < d * kChunks; t += kSelectThreads) {
      const int j = t / kChunks, c = t % kChunks;
      const int lo = s_jr[2 * j], hi = s_jr[2 * j + 1];
      double acc = 0.0;
      for (int l = lo + c; l <= hi; l += kChunks)
        acc += B.bval[(size_t)l * kMaxBand + (j - B.bstart[l])] * s_bins[l];
      s_part[t] = acc;
    }
    __syncthreads();
    if (threadIdx.x < d) {
      double acc = 0.0;
      for (int c = 0; c < kChunks; ++c) acc += s_part[threadIdx.x * kChunks + c];
      s_v[threadIdx.x] = acc;
    }
    __syncthreads();
    // theta = (G + lambda D)^-1 v
    mat_vec(s_ai, s_v, s_th, d, s_part);
    // G theta
    mat_vec(s_g, s_th, s_gt, d, s_part);
    // q = theta^T G theta - 2 theta^T v
    if (threadIdx.x == 0) {
      double w = 0.0;
      for (int j = 0; j < d; ++j) w += s_th[j] * (s_gt[j] - 2.0 * s_v[j]);
      it.q[(size_t)sig * it.p] = w;
    }
    GLOBAL double* th = gp(it.theta + (size_t)sig * it.p * it.d_max);
    for (int j = threadIdx.x; j < it.d_max; j += kSelectThreads) th[j] = (j < d) ? s_th[j] : 0.0;
    // candidate update table Z^b theta
    GLOBAL float* tab = gp(it.table + (size_t)sig * it.p * it.nb_max);
    for (int l = threadIdx.x; l < nb; l += kSelectThreads) {
      const int b0 = B.bstart[l];
      double t = 0.0;
      for (int b = 0; b < band; ++b) t += B.bval[(size_t)l * kMaxBand + b] * s_th[b0 + b];
      tab[l] = (float)t;
    }
    __syncthreads();
  }
}

// Selection for every fit of the batch (one block per fit).
__global__ void __launch_bounds__(kSelectThreads) k_pick(const FitDev* __restrict__ fits) {
  const FitDev& F = fits[blockIdx.x];
  Ctl* ctl = F.ctl;
  const int m_done = ctl->m_done;
  if (m_done >= F.M) return;
  const bool acwb = is_acwb_step(F, ctl->switched);
  pick(F, ctl, m_done + 1, acwb, acwb ? 2 : 1);
}

// ---------------------------------------------------------------------------
// HCWB validation risk and patience (Algorithm 3).
// ---------------------------------------------------------------------------
namespace {
// The validation check runs after an ACWB step of an HCWB fit that has not
// switched yet, and once before the first iteration (m_done = 0).
__device__ __forceinline__ bool valcheck_due(const FitDev& F, const Ctl* ctl) {
  if (F.variant != CWB_HCWB || ctl->switched) return false;
  return ctl->m_done == 0 || (ctl->pending && ctl->pend_acwb);
}
}  // namespace

__global__ void __launch_bounds__(kStateThreads)
k_valrisk(const FitDev* __restrict__ fits, const StateItem* __restrict__ items) {
  extern __shared__ float s_tf[];
  __shared__ double s_red[kStateThreads + 16];
  const StateItem it = items[blockIdx.x];
  const FitDev& F = fits[it.fit];
  const Ctl* ctl = F.ctl;
  if (!valcheck_due(F, ctl)) return;
  const bool init = ctl->m_done == 0;
  const int kk = ctl->k;
  const int nb = F.nb_max;
  const float nu = (float)F.nu;
  if (!init)
    for (int l = threadIdx.x; l < nb; l += kStateThreads) s_tf[l] = F.table[(size_t)kk * nb + l];
  __syncthreads();
  double acc = 0.0;
  const int64_t start = F.n_train + (int64_t)it.blk * kStateRows;
  for (int j = 0; j < kRowsPerThread; ++j) {
    const int64_t i = start + (int64_t)j * kStateThreads + threadIdx.x;
    if (i < F.n) {
      float f = F.fg[i];
      if (!init) {
        const uint32_t idx = F.unbinned
            ? reinterpret_cast<const uint32_t*>(F.X)[(size_t)kk * F.n_pad + i]
            : (uint32_t)F.X[(size_t)kk * F.n_pad + i];
        f = f + nu * table_at(F.unbinned != 0, idx, s_tf);
      }
      acc += loss_value(F.loss, F.y[i], f);
    }
  }
  const double s = block_sum<kStateThreads>(acc, s_red);
  if (threadIdx.x == 0) F.val_part[it.blk] = s;
}

// Patience counter of Algorithm 3: count consecutive rises of the validation
// risk; switch to CWB on all rows once it reaches pat_0.
__global__ void __launch_bounds__(kSelectThreads) k_valdecide(const FitDev* __restrict__ fits) {
  __shared__ double s_red[kSelectThreads + 16];
  const FitDev& F = fits[blockIdx.x];
  Ctl* ctl = F.ctl;
  if (!valcheck_due(F, ctl)) return;
  const bool init = ctl->m_done == 0;
  double t = 0.0;
  for (int b = threadIdx.x; b < F.n_val_blocks; b += kSelectThreads) t += F.val_part[b];
  const double tot = block_sum<kSelectThreads>(t, s_red);
  if (threadIdx.x == 0) {
    const double R = tot / (double)(F.n - F.n_train);
    if (!init) {
      if (R > ctl->rval_prev) ctl->counter += 1; else ctl->counter = 0;
      if (ctl->counter >= F.patience) {
        ctl->switched = 1;
        ctl->switch_iter = ctl->m_done + 1;
      }
    }
    ctl->rval_prev = R;
  }
}

// ---------------------------------------------------------------------------
// Finalize: after a final-mode row pass, record the risk of f^[m_done].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSelectThreads) k_finalize(const FitDev* __restrict__ fits) {
  __shared__ double s_red[kSelectThreads + 16];
  const FitDev& F = fits[blockIdx.x];
  Ctl* ctl = F.ctl;
  const int m = ctl->m_done;
  const double rt = sum_partials(F.risk_part, F.n_row_blocks, 2, 0, s_red);
  const double rv = sum_partials(F.risk_part, F.n_row_blocks, 2, 1, s_red);
  if (threadIdx.x == 0) {
    F.tr_risk[m] = rt / (double)F.n_train;
    F.tr_val[m] = (F.n > F.n_train) ? rv / (double)(F.n - F.n_train) : 0.0;
    ctl->pending = 0;
  }
}

// Aggregated coefficients of the primary and momentum models from the
// traces (Section 2.3; the ACWB parameter recurrences of Section 3.2.1):
// thread a owns coefficient a of both models and replays the iterations in
// order.  An iteration with a correction learner (k_cor >= 0) is an ACWB
// step: theta_f = (1 - t_m) theta_f + t_m theta_h + nu e_k theta and
// theta_h += eta_m e_kcor theta_cor with t_m = 2/(m+1), eta_m = gamma nu / t_m;
// otherwise theta_f += nu e_k theta.
constexpr int kCoefChunk = 256;
__global__ void __launch_bounds__(kSelectThreads) k_coef(const FitDev* __restrict__ fits) {
  __shared__ int s_off[kCoefChunk], s_d[kCoefChunk], s_offc[kCoefChunk], s_dc[kCoefChunk];
  const FitDev& F = fits[blockIdx.y];
  const int a = blockIdx.x * kSelectThreads + threadIdx.x;
  const int m_done = F.ctl->m_done;
  const int dmax = F.d_max;
  double cf = 0.0, ch = 0.0;
  for (int m0 = 0; m0 < m_done; m0 += kCoefChunk) {
    const int cnt = (m_done - m0 < kCoefChunk) ? m_done - m0 : kCoefChunk;
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += kSelectThreads) {
      const int k = F.tr_k[m0 + t], kc = F.tr_kcor[m0 + t];
      s_off[t] = F.feat[k].coef_off;
      s_d[t] = F.feat[k].d;
      s_offc[t] = kc >= 0 ? F.feat[kc].coef_off : -1;
      s_dc[t] = kc >= 0 ? F.feat[kc].d : 0;
    }
    __syncthreads();
    if (a < F.sum_d) {
      for (int t = 0; t < cnt; ++t) {
        const int mi = m0 + t;
        if (s_offc[t] >= 0) {
          const double vt = 2.0 / ((double)(mi + 1) + 1.0);
          const double eta = F.gamma * F.nu / vt;
          cf = (1.0 - vt) * cf + vt * ch;
          if (a >= s_offc[t] && a < s_offc[t] + s_dc[t])
            ch += eta * F.tr_thetacor[(size_t)mi * dmax + (a - s_offc[t])];
        }
        if (a >= s_off[t] && a < s_off[t] + s_d[t])
          cf += F.nu * F.tr_theta[(size_t)mi * dmax + (a - s_off[t])];
      }
    }
  }
  if (a < F.sum_d) {
    F.coef_f[a] = cf;
    F.coef_h[a] = ch;
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
namespace {

template <int NT, int FMAX, int NSMAX, bool UNB>
hipError_t launch_hist_t(hipStream_t st, int blocks, size_t lds, const FitDev* fits, const Seg* segs,
                         const int64_t* blk, long long* partials) {
  // 160 KiB per workgroup minus the kernel's static LDS (at most ~4 KiB);
  // set once (thread-safe static initialisation), before any graph capture
  static const bool attr = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hist<NT, FMAX, NSMAX, UNB>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kHistMaxLds);
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_hist<NT, FMAX, NSMAX, UNB>), dim3(blocks), dim3(NT), lds, st, fits, segs, blk,
                     partials);
  return hipGetLastError();
}

template <int NT, int NSMAX, bool UNB>
hipError_t launch_hist_nt(hipStream_t st, int fmax, int blocks, size_t lds, const FitDev* fits,
                          const Seg* segs, const int64_t* blk, long long* partials) {
  switch (fmax) {
    case 1: return launch_hist_t<NT, 1, NSMAX, UNB>(st, blocks, lds, fits, segs, blk, partials);
    case 2: return launch_hist_t<NT, 2, NSMAX, UNB>(st, blocks, lds, fits, segs, blk, partials);
    case 4: return launch_hist_t<NT, 4, NSMAX, UNB>(st, blocks, lds, fits, segs, blk, partials);
    case 8: return launch_hist_t<NT, 8, NSMAX, UNB>(st, blocks, lds, fits, segs, blk, partials);
    case 16:
      if (!UNB) return launch_hist_t<NT, 16, NSMAX, false>(st, blocks, lds, fits, segs, blk, partials);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int NSMAX, bool UNB>
hipError_t launch_hist_ns(hipStream_t st, int nt, int fmax, int blocks, size_t lds,
                          const FitDev* fits, const Seg* segs, const int64_t* blk,
                          long long* partials) {
  switch (nt) {
    case 256: return launch_hist_nt<256, NSMAX, UNB>(st, fmax, blocks, lds, fits, segs, blk, partials);
    case 512: return launch_hist_nt<512, NSMAX, UNB>(st, fmax, blocks, lds, fits, segs, blk, partials);
    case 1024: return launch_hist_nt<1024, NSMAX, UNB>(st, fmax, blocks, lds, fits, segs, blk, partials);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_state(hipStream_t st, const RowItem* items, int nitems, int nb_max,
                        int final_mode) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * nb_max * sizeof(float);
  hipLaunchKernelGGL(k_state, dim3(nitems), dim3(kStateThreads), lds, st, items, final_mode);
  return hipGetLastError();
}

hipError_t launch_hist(hipStream_t st, int nt, int fmax, int nsmax, bool unbinned, int blocks,
                       size_t lds, const FitDev* fits, const Seg* segs, const int64_t* blk,
                       long long* partials) {
  if (blocks <= 0) return hipSuccess;
  if (unbinned) {
    if (nsmax == 1) return launch_hist_ns<1, true>(st, nt, fmax, blocks, lds, fits, segs, blk, partials);
    return launch_hist_ns<2, true>(st, nt, fmax, blocks, lds, fits, segs, blk, partials);
  }
  if (nsmax == 1) return launch_hist_ns<1, false>(st, nt, fmax, blocks, lds, fits, segs, blk, partials);
  return launch_hist_ns<2, false>(st, nt, fmax, blocks, lds, fits, segs, blk, partials);
}

hipError_t launch_select(hipStream_t st, const SelItem* items, int nitems, int nb_max, int d_max,
                         const long long* partials) {
  if (nitems <= 0) return hipSuccess;
  // static LDS of the kernel (incl. the selection step) stays below 16 KiB
  size_t lds = ((size_t)nb_max + 2 * (size_t)d_max * d_max) * sizeof(double);
  const size_t extra = (size_t)nb_max * kMaxBand * sizeof(double) + (size_t)nb_max * sizeof(int);
  const bool staged = nb_max <= kStageBins && lds + extra <= 144 * 1024;
  if (staged) lds += extra;
  // 160 KiB per workgroup minus the kernel's own static LDS (< 16 KiB)
  static const bool attr = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_select<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 144 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_select<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 144 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  if (staged)
    hipLaunchKernelGGL(k_select<true>, dim3(nitems), dim3(kSelectThreads), lds, st, items,
                       partials, nb_max, d_max);
  else
    hipLaunchKernelGGL(k_select<false>, dim3(nitems), dim3(kSelectThreads), lds, st, items,
                       partials, nb_max, d_max);
  return hipGetLastError();
}

hipError_t launch_valrisk(hipStream_t st, const FitDev* fits, const StateItem* items, int nitems,
                          int nb_max) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)nb_max * sizeof(float);
  hipLaunchKernelGGL(k_valrisk, dim3(nitems), dim3(kStateThreads), lds, st, fits, items);
  return hipGetLastError();
}

hipError_t launch_pick(hipStream_t st, const FitDev* fits, int nfits) {
  if (nfits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pick, dim3(nfits), dim3(kSelectThreads), 0, st, fits);
  return hipGetLastError();
}

hipError_t launch_valdecide(hipStream_t st, const FitDev* fits, int nfits) {
  if (nfits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_valdecide, dim3(nfits), dim3(kSelectThreads), 0, st, fits);
  return hipGetLastError();
}

hipError_t launch_coef(hipStream_t st, const FitDev* fits, int sum_d) {
  if (sum_d <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coef, dim3((sum_d + kSelectThreads - 1) / kSelectThreads, 1), dim3(kSelectThreads),
                     0, st, fits);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t st, const FitDev* fits, int nfits) {
  if (nfits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(nfits), dim3(kSelectThreads), 0, st, fits);
  return hipGetLastError();
}

}  // namespace cwb

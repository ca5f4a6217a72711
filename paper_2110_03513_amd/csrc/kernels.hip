// kernels.hip -- gfx950 kernels of one boosting iteration.
//
// Per iteration m (Algorithm A1 for CWB, Algorithm 2 for ACWB, Algorithm 3
// for HCWB) the host enqueues, for every fit of a batch at once:
//   k_state   row pass: take over the selection of iteration m-1 (every block
//             computes the chosen learners from the criteria; the fit's first
//             block records them in the traces), apply its update
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
//             (Algorithm A1's SSE), and the candidate update table Z^b theta;
//             learner 0's block also records the risk of f^[m-1].
//   k_valrisk (HCWB, ACWB phase) validation-risk partials of the new primary
//   k_valdecide  model, then the patience counter that decides the switch.
// The argmin over q needs every learner's criterion, so it cannot run in
// k_select; instead each block of the next kernel that needs the chosen
// learners computes it from q (p values).
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

// Two FP64 sums and two float maxima of a block in one pass: butterfly
// shuffles within each wavefront (every lane gets the same, fixed-order
// result), then thread 0 combines the wavefronts in order.  `red` holds
// 4 * (NT / 64) doubles.  Results are valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_sum2_max2(double& s0, double& s1, float& m0, float& m1,
                                                double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
    m0 = fmaxf(m0, __shfl_xor(m0, off, 64));
    m1 = fmaxf(m1, __shfl_xor(m1, off, 64));
  }
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    red[4 * w] = s0;
    red[4 * w + 1] = s1;
    red[4 * w + 2] = (double)m0;
    red[4 * w + 3] = (double)m1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s0 = red[0];
    s1 = red[1];
    m0 = (float)red[2];
    m1 = (float)red[3];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) {
      s0 += red[4 * i];
      s1 += red[4 * i + 1];
      m0 = fmaxf(m0, (float)red[4 * i + 2]);
      m1 = fmaxf(m1, (float)red[4 * i + 3]);
    }
  }
}

// Block maxima of two non-negative floats (every thread gets both).  `red`
// holds 2 * (NT / 64) floats.
template <int NT>
__device__ __forceinline__ void block_max2(float& m0, float& m1, float* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m0 = fmaxf(m0, __shfl_xor(m0, off, 64));
    m1 = fmaxf(m1, __shfl_xor(m1, off, 64));
  }
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = m0;
    red[2 * w + 1] = m1;
  }
  __syncthreads();
  m0 = red[0];
  m1 = red[1];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) {
    m0 = fmaxf(m0, red[2 * i]);
    m1 = fmaxf(m1, red[2 * i + 1]);
  }
  __syncthreads();
}

// Scale exponents of both signals of a fit: maxima over the row-pass
// blocks' maxima (order-free, so every block computes the same values).
template <int NT>
__device__ void fit_scale_exponents(const FitDev& F, int64_t n_fit, int* e0, int* e1, float* red) {
  float a = 0.0f, b = 0.0f;
  const GLOBAL float* am = gp(F.amax_part);
  for (int b0 = 0; b0 < F.n_row_blocks; b0 += 4 * NT) {
    float v[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = b0 + u * NT + (int)threadIdx.x;
      v[u] = (k < F.n_row_blocks) ? am[2 * k] : 0.0f;
      w[u] = (k < F.n_row_blocks) ? am[2 * k + 1] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a = fmaxf(a, v[u]);
      b = fmaxf(b, w[u]);
    }
  }
  block_max2<NT>(a, b, red);
  *e0 = scale_exponent(a, n_fit);
  *e1 = scale_exponent(b, n_fit);
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

// The learners chosen by the last selection (Algorithm A1's argmin over the
// criteria q, ties to the lowest k; with nsig = 2 also the ACWB correction
// fit of Algorithm 2), computed by every block that needs them from q
// itself, so that no kernel publishes them to the blocks of the next one.
// `gap` is the runner-up minus the best criterion of signal 0; `bad` flags
// criteria that are all non-finite (the learners are then 0).
struct Picked {
  int k0, k1;
  double gap;
  bool bad;
};

// Argmin of one signal within a wavefront (64 lanes) by butterfly shuffles;
// every lane ends with the wavefront's result.
__device__ __forceinline__ void wave_arg2(Arg2& a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double c1 = __shfl_xor(a.b1, off, 64);
    const double c2 = __shfl_xor(a.b2, off, 64);
    const int kc = __shfl_xor(a.k1, off, 64);
    a.merge(c1, c2, kc);
  }
}

// `v0`, `v1`: this thread's criteria q[t], q[p + t] for t = threadIdx.x,
// loaded early by the caller (INFINITY past p); the rest is loaded here.
template <int NT>
__device__ Picked block_pick(const double* q_, int p, int nsig, double v0, double v1,
                             Arg2 (*s_w)[NT / 64]) {
  const GLOBAL double* q = gp(q_);
  Arg2 a0{INFINITY, INFINITY, p}, a1{INFINITY, INFINITY, p};
  if ((int)threadIdx.x < p) {
    a0.add(v0, threadIdx.x);
    if (nsig == 2) a1.add(v1, threadIdx.x);
  }
  for (int t = threadIdx.x + NT; t < p; t += NT) {
    a0.add(q[t], t);
    if (nsig == 2) a1.add(q[p + t], t);
  }
  wave_arg2(a0);
  if (nsig == 2) wave_arg2(a1);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    s_w[0][w] = a0;
    s_w[1][w] = a1;
  }
  __syncthreads();
  Arg2 r0 = s_w[0][0], r1 = s_w[1][0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) {  // fixed order: the same result in every block
    r0.merge(s_w[0][i].b1, s_w[0][i].b2, s_w[0][i].k1);
    r1.merge(s_w[1][i].b1, s_w[1][i].b2, s_w[1][i].k1);
  }
  __syncthreads();
  Picked r;
  r.k0 = r0.k1;
  r.k1 = (nsig == 2) ? r1.k1 : -1;
  r.gap = r0.b2 - r0.b1;
  r.bad = r.k0 >= p || (nsig == 2 && r.k1 >= p);
  if (r.bad) {
    r.k0 = 0;
    r.k1 = (nsig == 2) ? 0 : -1;
  }
  return r;
}

}  // namespace

// ---------------------------------------------------------------------------
// Row pass.
// ---------------------------------------------------------------------------
// Row pass of iteration m = sel_done + 1 (in final mode: no new
// iteration).  It first takes over the selection made by the last k_select,
// unless a finalize already did: every block computes the chosen learners
// from q, block 0 records them in the traces, and every block applies the
// update to its rows (f = g + nu b_k; ACWB: h += eta b_kcor with
// eta = gamma nu (S + 1) / 2 for selection S).
__global__ void __launch_bounds__(kStateThreads)
k_state(const FitDev* __restrict__ fits, const RowItem* __restrict__ items, int final_mode) {
  extern __shared__ float s_tab[];  // [2][nb_max]
  __shared__ double s_red[kStateThreads + 16];
  __shared__ Arg2 s_w[2][kStateThreads / 64];
  __shared__ int s_bad;
  const RowItem it = items[blockIdx.x];
  // one round: the control block, the criteria of the last selection and
  // this thread's rows of the model state
  double qv0 = INFINITY, qv1 = INFINITY;
  if ((int)threadIdx.x < it.p) {
    qv0 = gp(it.q)[threadIdx.x];
    qv1 = gp(it.q)[it.p + threadIdx.x];  // used only after an ACWB selection
  }
  Ctl* ctl = it.ctl;
  const int S = ctl->sel_done;
  const int fin = ctl->fin_done;
  const int sel_acwb = ctl->sel_acwb;
  const int switched = ctl->switched;
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
  if (!final_mode && S >= it.M) {
    // all M selections made (a batch runs on for other fits): mark the fit
    // done for the histogram and select passes; finalize records the last
    // selection
    if (it.blk == 0 && threadIdx.x == 0) ctl->pick_done = it.M;
    return;
  }
  const float nu = (float)it.nu;
  const int m = S + 1;
  const bool acwb =
      !final_mode && (it.variant == CWB_ACWB || (it.variant == CWB_HCWB && !switched));
  const int64_t n_fit = (it.variant == CWB_HCWB && switched) ? it.n : it.n_train;
  const int nb = it.nb_max;
  float* tf = s_tab;
  float* tc = s_tab + nb;
  // the last selection: its learners, and whether its update is still to apply
  const bool have_sel = S >= 1;
  const bool do_pick = have_sel && fin != S;
  Picked pk{0, -1, 0.0, false};
  if (have_sel) pk = block_pick<kStateThreads>(it.q, it.p, sel_acwb ? 2 : 1, qv0, qv1, s_w);
  const int kk = pk.k0;
  const int kc = pk.k1;
  const float eta = (float)(it.gamma * it.nu / (2.0 / ((double)S + 1.0)));
  if (do_pick && it.blk == 0) {  // the fit's first row block records the selection
    const FitDev& F = fits[it.fit];
    const int mi = S - 1;
    const int dmax = F.d_max;
    const GLOBAL double* th = gp(F.theta);
    for (int j = threadIdx.x; j < dmax; j += kStateThreads) {
      F.tr_theta[(size_t)mi * dmax + j] = th[(size_t)kk * dmax + j];
      F.tr_thetacor[(size_t)mi * dmax + j] = (kc >= 0) ? th[((size_t)F.p + kc) * dmax + j] : 0.0;
    }
    if (threadIdx.x == 0) {
      F.tr_k[mi] = kk;
      F.tr_kcor[mi] = kc;
      F.tr_gap[mi] = pk.gap;
      ctl->pick_done = S;
    }
  }
  if (pk.bad && threadIdx.x == 0) atomicOr(&ctl->error, 1);
  const bool use_t = do_pick;
  const bool use_h = do_pick && sel_acwb && kc >= 0;
  const bool use_cc = acwb && have_sel && sel_acwb && kc >= 0;
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
  double st = risk_t, sv = risk_v;
  float a = amax_r, b = amax_c;
  block_sum2_max2<kStateThreads>(st, sv, a, b, s_red);
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
// With `need_e`, the fit's scale exponents are computed (by all threads)
// while the first step's loads are in flight.
template <int NT, int FMAX, int NSIG>
__device__ __forceinline__ void hist_rows(const FitDev& F, const Seg& sg,
                                          unsigned long long* __restrict__ hist, int nb,
                                          int64_t r0, int64_t r1, int& e0, int& e1, bool need_e,
                                          int64_t n_fit, float* red) {
  const uint16_t* __restrict__ Xg = F.X + (size_t)sg.k0 * F.n_pad;
  const int nf = sg.nf;
  const size_t ld = (size_t)F.n_pad;
  int64_t base = r0 + (int64_t)threadIdx.x * 8;
  const bool any = base < r1;
  float rv[8], cv[8];
  u32x4 xw[FMAX];
  if (any) hist_step_load<FMAX, NSIG>(F, Xg, ld, nf, base, rv, cv, xw);
  if (need_e) fit_scale_exponents<NT>(F, n_fit, &e0, &e1, red);
  if (!any) return;
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
    if (ctl->pick_done >= F.M) continue;
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
    const bool need_e = sg.fit != cached_fit;
    cached_fit = sg.fit;
    if (UNB) {
      if (need_e) fit_scale_exponents<NT>(F, n_fit, &e0, &e1, s_red);
      if (NSMAX == 1 || nsig == 1)
        uhist_rows<NT, FMAX, 1>(F, sg, s_hist, nb, r0, r1, e0, 0);
      else
        uhist_rows<NT, FMAX, NSMAX>(F, sg, s_hist, nb, r0, r1, e0, e1);
    } else {
      if (NSMAX == 1 || nsig == 1)
        hist_rows<NT, FMAX, 1>(F, sg, s_hist, nb, r0, r1, e0, e1, need_e, n_fit, s_red);
      else
        hist_rows<NT, FMAX, NSMAX>(F, sg, s_hist, nb, r0, r1, e0, e1, need_e, n_fit, s_red);
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
  // the first chunk of signal 0's partials, loaded in the first round when
  // its offsets are inline (bins 4t .. 4t+3 of every segment)
  const bool pre = n_off <= kInlineOffs && nb <= 4 * kSelectThreads;
  i64x2 pv[kInlineOffs][2];
  if (pre && 4 * (int)threadIdx.x < nb) {
#pragma unroll
    for (int i = 0; i < kInlineOffs; ++i) {
      if (i < n_off) {
        const GLOBAL i64x2* src = (const GLOBAL i64x2*)(partials + it.off0[i] + 4 * threadIdx.x);
        pv[i][0] = src[0];
        pv[i][1] = src[1];
      }
    }
  }
  // one round of independent loads: control block, signal maxima, offsets,
  // the learner's tables for the training-row Gram set
  const int P = it.ctl->pick_done;  // = iterations before this selection
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
  if (P >= it.M) return;
  const bool hcwb_all = it.variant == CWB_HCWB && switched;
  const bool acwb = it.variant == CWB_ACWB || (it.variant == CWB_HCWB && !switched);
  const int nsig = acwb ? 2 : 1;
  const int64_t n_fit = hcwb_all ? it.n : it.n_train;
  if (it.k == 0) {
    // learner 0's block: the risk of f^[P] from this iteration's row pass,
    // and the count and kind of this selection for the next row pass
    const double rt = sum_partials(it.risk_part, it.n_row_blocks, 2, 0, s_part);
    const double rv = sum_partials(it.risk_part, it.n_row_blocks, 2, 1, s_part);
    if (threadIdx.x == 0) {
      it.tr_risk[P] = rt / (double)it.n_train;
      it.tr_val[P] = (it.n > it.n_train) ? rv / (double)(it.n - it.n_train) : 0.0;
      it.ctl->sel_done = P + 1;
      it.ctl->sel_acwb = acwb ? 1 : 0;
    }
  }
  if (hcwb_all) {  // HCWB after the switch: Grams over all rows
    __syncthreads();
    stage<kSelectThreads, 4>(s_ai, it.ainv[1], d * d);
    stage<kSelectThreads, 4>(s_g, it.gram[1], d * d);
  }
  const Basis B = STAGED ? Basis{s_bv, s_bs} : Basis{it.bval, it.bstart};
  block_max2<kSelectThreads>(am0, am1, s_red);
  const float amax[2] = {am0, am1};
  for (int sig = 0; sig < nsig; ++sig) {
    const double isc = ldexp(1.0, -scale_exponent(amax[sig], n_fit));
    // bin sums s_l: exact int64 merge of the group's segment partials
    for (int l0 = 0; l0 < nb; l0 += 4 * kSelectThreads) {
      long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      const int l = l0 + 4 * threadIdx.x;
      if (pre && sig == 0) {  // l0 == 0: the preloaded chunk
        if (l < nb) {
#pragma unroll
          for (int i = 0; i < kInlineOffs; ++i) {
            if (i < n_off) {
              a0 += pv[i][0].x;
              a1 += pv[i][0].y;
              a2 += pv[i][1].x;
              a3 += pv[i][1].y;
            }
          }
        }
      } else
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

// ---------------------------------------------------------------------------
// HCWB validation risk and patience (Algorithm 3).
// ---------------------------------------------------------------------------
namespace {
// The validation check runs after an ACWB selection of an HCWB fit that has
// not switched yet, and once before the first iteration (no selection yet).
__device__ __forceinline__ bool valcheck_due(const FitDev& F, const Ctl* ctl) {
  if (F.variant != CWB_HCWB || ctl->switched) return false;
  const int S = ctl->sel_done;
  return S == 0 || (ctl->sel_acwb && S == ctl->pick_done + 1);  // a new ACWB selection
}
}  // namespace

// Validation risk of the new primary model f^[m] = g + nu b_k (the
// selection's update applied to the validation rows), or of f^[0].
__global__ void __launch_bounds__(kStateThreads)
k_valrisk(const FitDev* __restrict__ fits, const StateItem* __restrict__ items) {
  extern __shared__ float s_tf[];
  __shared__ double s_red[kStateThreads + 16];
  __shared__ Arg2 s_w[2][kStateThreads / 64];
  const StateItem it = items[blockIdx.x];
  const FitDev& F = fits[it.fit];
  const Ctl* ctl = F.ctl;
  if (!valcheck_due(F, ctl)) return;
  const bool init = ctl->sel_done == 0;
  int kk = 0;
  if (!init) {
    const double v0 = ((int)threadIdx.x < F.p) ? gp(F.q)[threadIdx.x] : INFINITY;
    kk = block_pick<kStateThreads>(F.q, F.p, 1, v0, INFINITY, s_w).k0;
  }
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
  const bool init = ctl->sel_done == 0;
  double t = 0.0;
  for (int b = threadIdx.x; b < F.n_val_blocks; b += kSelectThreads) t += F.val_part[b];
  const double tot = block_sum<kSelectThreads>(t, s_red);
  if (threadIdx.x == 0) {
    const double R = tot / (double)(F.n - F.n_train);
    if (!init) {
      if (R > ctl->rval_prev) ctl->counter += 1; else ctl->counter = 0;
      if (ctl->counter >= F.patience) {
        ctl->switched = 1;
        ctl->switch_iter = ctl->sel_done + 1;
      }
    }
    ctl->rval_prev = R;
  }
}

// ---------------------------------------------------------------------------
// Finalize: after a final-mode row pass (which applied the last selection),
// record the risk of f^[S] for the S selections made, and mark S applied.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSelectThreads) k_finalize(const FitDev* __restrict__ fits) {
  __shared__ double s_red[kSelectThreads + 16];
  const FitDev& F = fits[blockIdx.x];
  Ctl* ctl = F.ctl;
  const int S = ctl->sel_done;
  const double rt = sum_partials(F.risk_part, F.n_row_blocks, 2, 0, s_red);
  const double rv = sum_partials(F.risk_part, F.n_row_blocks, 2, 1, s_red);
  if (threadIdx.x == 0) {
    F.tr_risk[S] = rt / (double)F.n_train;
    F.tr_val[S] = (F.n > F.n_train) ? rv / (double)(F.n - F.n_train) : 0.0;
    ctl->pick_done = S;
    ctl->fin_done = S;
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
  const int m_done = F.ctl->pick_done;
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

hipError_t launch_state(hipStream_t st, const FitDev* fits, const RowItem* items, int nitems,
                        int nb_max, int final_mode) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * nb_max * sizeof(float);
  hipLaunchKernelGGL(k_state, dim3(nitems), dim3(kStateThreads), lds, st, fits, items, final_mode);
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

// kernels.hip -- gfx950 kernels of one boosting iteration.
//
// Per iteration m (Algorithm A1 for CWB, Algorithm 2 for ACWB, Algorithm 3
// for HCWB) the host enqueues, for every fit of a batch at once:
//   k_state   row pass: apply the update tables selected in iteration m-1
//             (f += nu b_k, h += eta b_kcor), form g = (1-theta_m) f +
//             theta_m h (ACWB), the pseudo-residuals r = -dL/df and the
//             error-corrected residuals c (ACWB), FP64 partial risks, and the
//             largest |r|, |c| (fixed-point scale of the histograms).
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
//             The last block of a fit takes argmin_k q (ties to the lowest k),
//             records the traces, aggregates the coefficients (Section 2.3 /
//             3.2.1) and arms the update for the next row pass.
//   k_valrisk (HCWB, ACWB phase) validation risk of the new primary model and
//             the patience counter that decides the switch to CWB.
#include <hip/hip_runtime.h>

#include "../../include/cwb.h"
#include "cwb_internal.h"
#include "kernels.h"

namespace cwb {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// Deterministic block sum: fixed butterfly per wave, then waves in order.
template <int NT>
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  __syncthreads();
  return s;  // valid in thread 0
}

__device__ __forceinline__ void load8f(const float* p, float* v) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ __forceinline__ void store8f(float* p, const float* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  *reinterpret_cast<float4*>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
}

__device__ __forceinline__ void load8u(const uint16_t* p, uint32_t* idx) {
  const uint4 w = *reinterpret_cast<const uint4*>(p);
  idx[0] = w.x & 0xffffu; idx[1] = w.x >> 16;
  idx[2] = w.y & 0xffffu; idx[3] = w.y >> 16;
  idx[4] = w.z & 0xffffu; idx[5] = w.z >> 16;
  idx[6] = w.w & 0xffffu; idx[7] = w.w >> 16;
}

}  // namespace

// ---------------------------------------------------------------------------
// Row pass.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kStateThreads)
k_state(const FitDev* __restrict__ fits, const StateItem* __restrict__ items, int final_mode) {
  extern __shared__ float s_tab[];  // [2][nb_max]
  __shared__ double s_red[kStateThreads / 64];
  __shared__ float s_fmax[2][kStateThreads / 64];
  __shared__ int s_bad;
  const StateItem it = items[blockIdx.x];
  const FitDev& F = fits[it.fit];
  Ctl* ctl = F.ctl;
  const int m_done = ctl->m_done;
  if (!final_mode && m_done >= F.M) return;
  const int pending = ctl->pending;
  const int pend_acwb = ctl->pend_acwb;
  const int kk = ctl->k;
  const int kc = ctl->kcor;
  const int switched = ctl->switched;
  const float eta = (float)ctl->eta;
  const float nu = (float)F.nu;
  const int m = m_done + 1;
  const bool acwb = !final_mode && is_acwb_step(F, switched);
  const int64_t n_fit = rows_fitted(F, switched);
  const int nb = F.nb_max;
  float* tf = s_tab;
  float* tc = s_tab + nb;
  const bool use_t = pending != 0;
  const bool use_h = pending && pend_acwb && kc >= 0;
  const bool use_cc = acwb && m > 1 && kc >= 0;
  if (use_t)
    for (int l = threadIdx.x; l < nb; l += kStateThreads) tf[l] = F.table[((size_t)kk) * nb + l];
  if (use_h || use_cc)
    for (int l = threadIdx.x; l < nb; l += kStateThreads)
      tc[l] = F.table[((size_t)F.p + kc) * nb + l];
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();

  double risk_t = 0.0, risk_v = 0.0;
  float amax_r = 0.0f, amax_c = 0.0f;
  bool bad = false;
  const int64_t base = (int64_t)it.blk * kStateRows + (int64_t)threadIdx.x * kRowsPerThread;
  if (base < F.n_pad) {
    const bool two = F.nsig_max == 2;
    float f[8], yv[8], hv[8], cv[8], rr[8], cc[8];
    uint32_t ik[8], ic[8];
    load8f(F.fg + base, f);
    load8f(F.y + base, yv);
    if (two) load8f(F.h + base, hv);
    if (use_cc) load8f(F.c + base, cv);
    if (use_t) load8u(F.X + (size_t)kk * F.n_pad + base, ik);
    if (use_h || use_cc) load8u(F.X + (size_t)kc * F.n_pad + base, ic);
    const float vt = 2.0f / (float)(m + 1);
    const float cw = (float)m / (float)(m + 1);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t i = base + j;
      const bool live = i < F.n;
      float fj = f[j];
      float hj = two ? hv[j] : 0.0f;
      if (live && use_t) fj = fj + nu * tf[ik[j]];
      if (live && use_h) hj = hj + eta * tc[ic[j]];
      if (live) {
        const double L = loss_value(F.loss, yv[j], fj);
        if (i < F.n_train) risk_t += L; else risk_v += L;
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
        const float r = neg_gradient(F.loss, yv[j], g);
        float c = r;
        if (use_cc) c = r + cw * (cv[j] - tc[ic[j]]);
        f[j] = g;  // the primary model update f = g + nu b_k is pending
        if (fitrow) {
          rr[j] = r;
          cc[j] = c;
        }
      } else {
        const float r = neg_gradient(F.loss, yv[j], fj);
        if (fitrow) rr[j] = r;
      }
      amax_r = fmaxf(amax_r, fabsf(rr[j]));
      amax_c = fmaxf(amax_c, fabsf(cc[j]));
    }
    store8f(F.fg + base, f);
    if (two) store8f(F.h + base, hv);
    if (!final_mode) {
      store8f(F.r + base, rr);
      if (acwb) store8f(F.c + base, cc);
    }
  }
  if (bad) s_bad = 1;
  const double st = block_sum<kStateThreads>(risk_t, s_red);
  const double sv = block_sum<kStateThreads>(risk_v, s_red);
  amax_r = wave_max(amax_r);
  amax_c = wave_max(amax_c);
  if ((threadIdx.x & 63) == 0) {
    s_fmax[0][threadIdx.x >> 6] = amax_r;
    s_fmax[1][threadIdx.x >> 6] = amax_c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.0f, b = 0.0f;
    for (int w = 0; w < kStateThreads / 64; ++w) {
      a = fmaxf(a, s_fmax[0][w]);
      b = fmaxf(b, s_fmax[1][w]);
    }
    F.risk_part[2 * it.blk] = st;
    F.risk_part[2 * it.blk + 1] = sv;
    if (!final_mode) {
      // non-negative floats order like their bit patterns
      if (!isfinite(a) || !isfinite(b)) s_bad = 1;
      if (a > 0.0f) atomicMax(&ctl->absmax[0], __float_as_uint(a));
      if (b > 0.0f) atomicMax(&ctl->absmax[1], __float_as_uint(b));
    }
    if (s_bad) atomicOr(&ctl->error, 1);
  }
}

// ---------------------------------------------------------------------------
// Histogram pass.
// ---------------------------------------------------------------------------
template <int NT, int FMAX, int NSIG>
__device__ __forceinline__ void hist_rows(const FitDev& F, const Seg& sg,
                                          unsigned long long* __restrict__ hist, int nb,
                                          int64_t r0, int64_t r1, double sc0, double sc1) {
  const uint16_t* __restrict__ Xg = F.X + (size_t)sg.k0 * F.n_pad;
  const int nf = sg.nf;
  const size_t ld = (size_t)F.n_pad;
  for (int64_t base = r0 + (int64_t)threadIdx.x * 8; base < r1; base += (int64_t)NT * 8) {
    float rv[8], cv[8];
    load8f(F.r + base, rv);
    long long q0[8], q1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) q0[j] = (long long)((double)rv[j] * sc0);
    if (NSIG == 2) {
      load8f(F.c + base, cv);
#pragma unroll
      for (int j = 0; j < 8; ++j) q1[j] = (long long)((double)cv[j] * sc1);
    }
    u32x4 xw[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; ++f)
      if (f < nf) xw[f] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(Xg + f * ld + base));
#pragma unroll
    for (int f = 0; f < FMAX; ++f) {
      if (f < nf) {
        unsigned long long* h0 = hist + (size_t)f * nb;
        const uint32_t w[4] = {xw[f].x, xw[f].y, xw[f].z, xw[f].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          __hip_atomic_fetch_add(h0 + (w[j] & 0xffffu), (unsigned long long)q0[2 * j],
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          __hip_atomic_fetch_add(h0 + (w[j] >> 16), (unsigned long long)q0[2 * j + 1],
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (NSIG == 2) {
          unsigned long long* h1 = hist + (size_t)(nf + f) * nb;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            __hip_atomic_fetch_add(h1 + (w[j] & 0xffffu), (unsigned long long)q1[2 * j],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(h1 + (w[j] >> 16), (unsigned long long)q1[2 * j + 1],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
    }
  }
}

template <int NT, int FMAX>
__global__ void __launch_bounds__(NT)
k_hist(const FitDev* __restrict__ fits, const Seg* __restrict__ segs,
       const int64_t* __restrict__ blk, long long* __restrict__ partials) {
  extern __shared__ unsigned long long s_hist[];
  const int64_t s0 = blk[2 * blockIdx.x], s1 = blk[2 * blockIdx.x + 1];
  for (int64_t s = s0; s < s1; ++s) {
    const Seg sg = segs[s];
    const FitDev& F = fits[sg.fit];
    const Ctl* ctl = F.ctl;
    if (ctl->m_done >= F.M) continue;
    const int switched = ctl->switched;
    const int nsig = is_acwb_step(F, switched) ? 2 : 1;
    const int64_t n_fit = rows_fitted(F, switched);
    const int nb = F.nb_max;
    const int words = nsig * sg.nf * nb;
    for (int i = threadIdx.x; i < words; i += NT) s_hist[i] = 0ull;
    __syncthreads();
    const int64_t n8 = (n_fit + 7) >> 3;
    const int64_t U = F.n_pad >> 3;
    const int64_t r0 = 8 * (sg.u0 * n8 / U);
    const int64_t r1 = 8 * (sg.u1 * n8 / U);
    const double sc0 = ldexp(1.0, scale_exponent(ctl->absmax[0], n_fit));
    if (nsig == 1) {
      hist_rows<NT, FMAX, 1>(F, sg, s_hist, nb, r0, r1, sc0, 0.0);
    } else {
      const double sc1 = ldexp(1.0, scale_exponent(ctl->absmax[1], n_fit));
      hist_rows<NT, FMAX, 2>(F, sg, s_hist, nb, r0, r1, sc0, sc1);
    }
    __syncthreads();
    long long* out = partials + sg.slot;
    for (int i = threadIdx.x; i < words; i += NT) out[i] = (long long)s_hist[i];
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

// argmin_k q[k] over the fit's learners (ties: lowest k) and the runner-up value.
__device__ void block_argmin(const double* q, int p, int* k_out, double* gap_out,
                             double* sq, int* sk, double* sq2) {
  double b1 = INFINITY, b2 = INFINITY;
  int k1 = p;
  for (int k = threadIdx.x; k < p; k += kSelectThreads) {
    const double v = q[k];
    if (better(v, k, b1, k1)) {
      b2 = b1;
      b1 = v;
      k1 = k;
    } else if (v < b2) {
      b2 = v;
    }
  }
  sq[threadIdx.x] = b1;
  sk[threadIdx.x] = k1;
  sq2[threadIdx.x] = b2;
  __syncthreads();
  for (int stride = kSelectThreads / 2; stride > 0; stride >>= 1) {
    if (threadIdx.x < stride) {
      const int o = threadIdx.x + stride;
      const double a1 = sq[threadIdx.x], a2 = sq2[threadIdx.x], c1 = sq[o], c2 = sq2[o];
      const int ka = sk[threadIdx.x], kb = sk[o];
      if (better(c1, kb, a1, ka)) {
        sq[threadIdx.x] = c1;
        sk[threadIdx.x] = kb;
        sq2[threadIdx.x] = fmin(a1, c2);
      } else {
        sq2[threadIdx.x] = fmin(a2, c1);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *k_out = sk[0];
    *gap_out = sq2[0] - sq[0];
  }
  __syncthreads();
}

// Deterministic sum of risk partials of the row-pass blocks.
__device__ double sum_partials(const double* part, int count, int stride, int offset,
                               double* red) {
  double s = 0.0;
  for (int b = threadIdx.x; b < count; b += kSelectThreads) s += part[(size_t)b * stride + offset];
  return block_sum<kSelectThreads>(s, red);
}

__device__ void pick(const FitDev& F, Ctl* ctl, int m, bool acwb, int nsig) {
  __shared__ double sq[kSelectThreads], sq2[kSelectThreads];
  __shared__ int sk[kSelectThreads];
  __shared__ int s_k[2];
  __shared__ double s_gap[2];
  __shared__ double s_red[kSelectThreads / 64];
  for (int sig = 0; sig < nsig; ++sig)
    block_argmin(F.q + (size_t)sig * F.p, F.p, &s_k[sig], &s_gap[sig], sq, sk, sq2);
  const int k0 = s_k[0];
  const int k1 = (nsig == 2) ? s_k[1] : -1;
  const int mi = m - 1;
  const int dmax = F.d_max;
  for (int j = threadIdx.x; j < dmax; j += kSelectThreads) {
    F.tr_theta[(size_t)mi * dmax + j] = F.theta[(size_t)k0 * dmax + j];
    F.tr_thetacor[(size_t)mi * dmax + j] =
        (k1 >= 0) ? F.theta[((size_t)F.p + k1) * dmax + j] : 0.0;
  }
  // aggregated coefficients (Section 2.3; ACWB bookkeeping of Section 3.2.1)
  const FeatDev f0 = F.feat[k0];
  double eta = 0.0;
  if (!acwb) {
    for (int j = threadIdx.x; j < f0.d; j += kSelectThreads)
      F.coef_f[f0.coef_off + j] += F.nu * F.theta[(size_t)k0 * dmax + j];
  } else {
    const double vt = 2.0 / ((double)m + 1.0);
    eta = F.gamma * F.nu / vt;
    for (int a = threadIdx.x; a < F.sum_d; a += kSelectThreads)
      F.coef_f[a] = (1.0 - vt) * F.coef_f[a] + vt * F.coef_h[a];
    __syncthreads();
    for (int j = threadIdx.x; j < f0.d; j += kSelectThreads)
      F.coef_f[f0.coef_off + j] += F.nu * F.theta[(size_t)k0 * dmax + j];
    const FeatDev f1 = F.feat[k1];
    for (int j = threadIdx.x; j < f1.d; j += kSelectThreads)
      F.coef_h[f1.coef_off + j] += eta * F.theta[((size_t)F.p + k1) * dmax + j];
  }
  // risk of f^[m-1], from the row pass of this iteration
  const double rt = sum_partials(F.risk_part, F.n_row_blocks, 2, 0, s_red);
  const double rv = sum_partials(F.risk_part, F.n_row_blocks, 2, 1, s_red);
  if (threadIdx.x == 0) {
    F.tr_k[mi] = k0;
    F.tr_kcor[mi] = k1;
    F.tr_gap[mi] = s_gap[0];
    F.tr_risk[mi] = rt / (double)F.n_train;
    F.tr_val[mi] = (F.n > F.n_train) ? rv / (double)(F.n - F.n_train) : 0.0;
    ctl->pending = 1;
    ctl->pend_acwb = acwb ? 1 : 0;
    ctl->k = k0;
    ctl->kcor = k1;
    ctl->eta = eta;
    ctl->absmax[0] = 0u;
    ctl->absmax[1] = 0u;
    ctl->sel_done = 0u;
    ctl->m_done = m;
  }
}

}  // namespace

__global__ void __launch_bounds__(kSelectThreads)
k_select(const FitDev* __restrict__ fits, const SelItem* __restrict__ items,
         const int64_t* __restrict__ grp_ptr, const int64_t* __restrict__ grp_seg,
         const Seg* __restrict__ segs, const long long* __restrict__ partials) {
  extern __shared__ double s_bins[];  // nb_max
  __shared__ double s_v[kMaxD], s_th[kMaxD], s_w[kMaxD];
  __shared__ int s_last;
  const SelItem it = items[blockIdx.x];
  const FitDev& F = fits[it.fit];
  Ctl* ctl = F.ctl;
  const int m_done = ctl->m_done;
  if (m_done >= F.M) return;
  const int switched = ctl->switched;
  const bool acwb = is_acwb_step(F, switched);
  const int nsig = acwb ? 2 : 1;
  const int64_t n_fit = rows_fitted(F, switched);
  const int set = gram_set(F, switched);
  const int k = it.k;
  const FeatDev fd = F.feat[k];
  const int d = fd.d;
  const int64_t g0 = grp_ptr[it.grp], g1 = grp_ptr[it.grp + 1];
  const int f_local = k - segs[grp_seg[g0]].k0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t* bstart = F.bstart + fd.bin_off;
  const double* bval = F.bval + fd.bin_off * kMaxBand;
  const int32_t* jr = F.jr + 2 * (size_t)fd.coef_off;
  for (int sig = 0; sig < nsig; ++sig) {
    const double isc = ldexp(1.0, -scale_exponent(ctl->absmax[sig], n_fit));
    // bin sums s_l: exact int64 merge of the segment partials, then scaled
    for (int l = threadIdx.x; l < fd.nb; l += kSelectThreads) {
      long long acc = 0;
      for (int64_t g = g0; g < g1; ++g) {
        const Seg sg = segs[grp_seg[g]];
        acc += partials[sg.slot + (int64_t)(sig * sg.nf + f_local) * F.nb_max + l];
      }
      s_bins[l] = (double)acc * isc;
    }
    __syncthreads();
    // v_j = sum_l Z^b[l, j] s_l over the design points supporting basis j
    for (int j = wave; j < d; j += kSelectThreads / 64) {
      const int lo = jr[2 * j], hi = jr[2 * j + 1];
      double acc = 0.0;
      for (int l = lo + lane; l <= hi; l += 64) acc += bval[(size_t)l * kMaxBand + (j - bstart[l])] * s_bins[l];
      acc = wave_sum(acc);
      if (lane == 0) s_v[j] = acc;
    }
    __syncthreads();
    const double* Ai = F.ainv[set] + fd.mat_off;
    const double* G = F.gram[set] + fd.mat_off;
    if (threadIdx.x < d) {
      double t = 0.0;
      for (int i = 0; i < d; ++i) t += Ai[(size_t)threadIdx.x * d + i] * s_v[i];
      s_th[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x < d) {
      double gt = 0.0;
      for (int i = 0; i < d; ++i) gt += G[(size_t)threadIdx.x * d + i] * s_th[i];
      s_w[threadIdx.x] = s_th[threadIdx.x] * (gt - 2.0 * s_v[threadIdx.x]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double qq = 0.0;
      for (int j = 0; j < d; ++j) qq += s_w[j];
      F.q[(size_t)sig * F.p + k] = qq;
    }
    for (int j = threadIdx.x; j < F.d_max; j += kSelectThreads)
      F.theta[((size_t)sig * F.p + k) * F.d_max + j] = (j < d) ? s_th[j] : 0.0;
    float* tab = F.table + ((size_t)sig * F.p + k) * F.nb_max;
    for (int l = threadIdx.x; l < fd.nb; l += kSelectThreads) {
      const int b0 = bstart[l];
      double t = 0.0;
      for (int b = 0; b < fd.band; ++b) t += bval[(size_t)l * kMaxBand + b] * s_th[b0 + b];
      tab[l] = (float)t;
    }
    __syncthreads();
  }
  // the last learner block of this fit selects: every thread fences its own
  // writes, the barrier orders them before the counter increment
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = atomicAdd(&ctl->sel_done, 1u);
    s_last = (prev == (unsigned)F.p - 1u) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  pick(F, ctl, m_done + 1, acwb, nsig);
}

// ---------------------------------------------------------------------------
// HCWB validation risk and patience (Algorithm 3).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kStateThreads)
k_valrisk(const FitDev* __restrict__ fits, const StateItem* __restrict__ items) {
  extern __shared__ float s_tf[];
  __shared__ double s_red[kStateThreads / 64];
  __shared__ int s_last;
  const StateItem it = items[blockIdx.x];
  const FitDev& F = fits[it.fit];
  Ctl* ctl = F.ctl;
  if (F.variant != CWB_HCWB || ctl->switched) return;
  const int m_done = ctl->m_done;
  const bool init = (m_done == 0);
  if (!init && !(ctl->pending && ctl->pend_acwb)) return;
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
      if (!init) f = f + nu * s_tf[F.X[(size_t)kk * F.n_pad + i]];
      acc += loss_value(F.loss, F.y[i], f);
    }
  }
  const double s = block_sum<kStateThreads>(acc, s_red);
  if (threadIdx.x == 0) F.val_part[it.blk] = s;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = atomicAdd(&ctl->val_done, 1u);
    s_last = (prev == (unsigned)F.n_val_blocks - 1u) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double t = 0.0;
  for (int b = threadIdx.x; b < F.n_val_blocks; b += kStateThreads) t += F.val_part[b];
  const double tot = block_sum<kStateThreads>(t, s_red);
  if (threadIdx.x == 0) {
    const double R = tot / (double)(F.n - F.n_train);
    if (!init) {
      if (R > ctl->rval_prev) ctl->counter += 1; else ctl->counter = 0;
      if (ctl->counter >= F.patience) {
        ctl->switched = 1;
        ctl->switch_iter = m_done + 1;
      }
    }
    ctl->rval_prev = R;
    ctl->val_done = 0u;
  }
}

// ---------------------------------------------------------------------------
// Finalize: after a final-mode row pass, record the risk of f^[m_done].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSelectThreads) k_finalize(const FitDev* __restrict__ fits) {
  __shared__ double s_red[kSelectThreads / 64];
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

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
namespace {

template <int NT, int FMAX>
hipError_t launch_hist_t(hipStream_t st, int blocks, size_t lds, const FitDev* fits, const Seg* segs,
                         const int64_t* blk, long long* partials) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hist<NT, FMAX>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((k_hist<NT, FMAX>), dim3(blocks), dim3(NT), lds, st, fits, segs, blk, partials);
  return hipGetLastError();
}

template <int NT>
hipError_t launch_hist_nt(hipStream_t st, int fmax, int blocks, size_t lds, const FitDev* fits,
                          const Seg* segs, const int64_t* blk, long long* partials) {
  switch (fmax) {
    case 1: return launch_hist_t<NT, 1>(st, blocks, lds, fits, segs, blk, partials);
    case 2: return launch_hist_t<NT, 2>(st, blocks, lds, fits, segs, blk, partials);
    case 4: return launch_hist_t<NT, 4>(st, blocks, lds, fits, segs, blk, partials);
    case 8: return launch_hist_t<NT, 8>(st, blocks, lds, fits, segs, blk, partials);
    case 16: return launch_hist_t<NT, 16>(st, blocks, lds, fits, segs, blk, partials);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_state(hipStream_t st, const FitDev* fits, const StateItem* items, int nitems,
                        int nb_max, int final_mode) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * nb_max * sizeof(float);
  hipLaunchKernelGGL(k_state, dim3(nitems), dim3(kStateThreads), lds, st, fits, items, final_mode);
  return hipGetLastError();
}

hipError_t launch_hist(hipStream_t st, int nt, int fmax, int blocks, size_t lds, const FitDev* fits,
                       const Seg* segs, const int64_t* blk, long long* partials) {
  if (blocks <= 0) return hipSuccess;
  switch (nt) {
    case 256: return launch_hist_nt<256>(st, fmax, blocks, lds, fits, segs, blk, partials);
    case 512: return launch_hist_nt<512>(st, fmax, blocks, lds, fits, segs, blk, partials);
    case 1024: return launch_hist_nt<1024>(st, fmax, blocks, lds, fits, segs, blk, partials);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_select(hipStream_t st, const FitDev* fits, const SelItem* items, int nitems,
                         int nb_max, const int64_t* grp_ptr, const int64_t* grp_seg,
                         const Seg* segs, const long long* partials) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)nb_max * sizeof(double);
  hipLaunchKernelGGL(k_select, dim3(nitems), dim3(kSelectThreads), lds, st, fits, items, grp_ptr,
                     grp_seg, segs, partials);
  return hipGetLastError();
}

hipError_t launch_valrisk(hipStream_t st, const FitDev* fits, const StateItem* items, int nitems,
                          int nb_max) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)nb_max * sizeof(float);
  hipLaunchKernelGGL(k_valrisk, dim3(nitems), dim3(kStateThreads), lds, st, fits, items);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t st, const FitDev* fits, int nfits) {
  if (nfits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(nfits), dim3(kSelectThreads), 0, st, fits);
  return hipGetLastError();
}

}  // namespace cwb

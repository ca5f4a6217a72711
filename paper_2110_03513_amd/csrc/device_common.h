// device_common.h -- device helpers shared by the gfx950 kernels of the
// boosting iteration (kernels.hip) and the histogram pass (hist.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/cwb.h"
#include "cwb_internal.h"

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
  return (F.variant == CWB_HCWB && switched) ? F.n : F.n_scan;
}
__device__ __forceinline__ int gram_set(const FitDev& F, int switched) {
  return (F.variant == CWB_HCWB && switched) ? 1 : 0;
}

// Pseudo-residual -dL/df (L2: (y-f)^2/2; binomial: log(1+e^f) - y f).
__device__ __forceinline__ float neg_gradient(int loss, float y, float f) {
  if (loss == CWB_L2) return y - f;
  return y - 1.0f / (1.0f + expf(-f));
}

// Row loss for the row pass's risk partials: the binomial softplus term
// log(1 + e^-|f|) in FP32 (relative error about 1e-7, and the term is
// below log 2), its linear part max(f, 0) - y f exact in FP64.
__device__ __forceinline__ double row_loss(int loss, float y, float f) {
  const double fd = (double)f, yd = (double)y;
  if (loss == CWB_L2) {
    const double e = yd - fd;
    return 0.5 * e * e;
  }
  const float t = log1pf(expf(-fabsf(f)));
  return (double)t + ((fd > 0.0 ? fd : 0.0) - yd * fd);
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

// Fixed-point exponents of a fit's two signals: at the int64 scale
// (scale_exponent) and at the 32-bit scale (scale_exponent32).
struct Exps {
  int e[2];
  int e32[2];
};

// Scale exponents of both signals of a fit: maxima over the row-pass
// blocks' maxima (order-free, so every block computes the same values).
template <int NT>
__device__ void fit_exponents(const FitDev& F, int64_t n_fit, Exps* x, float* red) {
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
  x->e[0] = scale_exponent(a, n_fit);
  x->e[1] = scale_exponent(b, n_fit);
  x->e32[0] = scale_exponent32(a, F.acc32_bits);
  x->e32[1] = scale_exponent32(b, F.acc32_bits);
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

// The first pass of a stage(), split in two so that a block can issue the
// loads of several arrays before storing any of them: each array then costs
// one memory round trip in total, not one after the other.  Elements past
// the first pass (NT * U) are left to stage_rest().
template <int NT, int U, typename T>
struct StagePass {
  T v[U];
  __device__ __forceinline__ void load(const T* src, int count) {
    const GLOBAL T* g = gp(src);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = u * NT + (int)threadIdx.x;
      if (i < count) v[u] = g[i];
    }
  }
  // the same, with zeros past `count` (for reductions over the values)
  __device__ __forceinline__ void load_or_zero(const T* src, int count) {
    const GLOBAL T* g = gp(src);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = u * NT + (int)threadIdx.x;
      if (i < count) v[u] = g[i];
      else v[u] = T();
    }
  }
  __device__ __forceinline__ void store(T* dst, int count) const {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = u * NT + (int)threadIdx.x;
      if (i < count) dst[i] = v[u];
    }
  }
};

// stage() of the elements from `first` on.
template <int NT, int U, typename T>
__device__ __forceinline__ void stage_rest(T* dst, const T* src, int count, int first) {
  if (count > first) stage<NT, U>(dst + first, src + first, count - first);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef long long i64x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

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


// r * 2^e rounded to the nearest integer (ties to even), as int32: the
// 32-bit scale keeps |r| * 2^e below 2^30, and the scaling by a power of two
// is exact, so this is the exact rounding of the product.
__device__ __forceinline__ int fixed32(float r, int e) {
  return (int)rintf(ldexpf(r, e));
}

// Both ACWB signals of a row in one 64-bit word: r's value times 2^32 plus
// c's (two's complement).  A sum of such words is R 2^32 + C for the sums R
// of the r values and C of the c values, so while |C| < 2^31 the low word
// read as int32 is C, and R = (W - C) / 2^32 (unpack_signals).
__device__ __forceinline__ unsigned long long pack_signals(int qr, int qc) {
  return ((unsigned long long)(uint32_t)qr << 32) + (unsigned long long)(long long)qc;
}

__device__ __forceinline__ void unpack_signals(unsigned long long w, long long* R, long long* Cs) {
  const long long c = (long long)(int32_t)(uint32_t)w;
  *Cs = c;
  *R = (long long)(w - (unsigned long long)c) >> 32;
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

}  // namespace
}  // namespace cwb

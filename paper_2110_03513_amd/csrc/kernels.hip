// kernels.hip -- gfx950 kernels of one boosting iteration (the histogram
// pass is in hist.hip) and of model evaluation.
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
//   k_hist    histogram pass over the uint16 bin-index matrix (hist.hip):
//             for every learner k and design point l, s_kl = sum of r_i over
//             the rows with ind_ki = l (binMatVec, Algorithm 1, first stage),
//             and the same for c, as exact int64 fixed-point sums.
//   k_select  one block per learner and signal: merge the segment partials, v = Z^bT s
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
#include "device_common.h"
#include "kernels.h"

namespace cwb {


// ---------------------------------------------------------------------------
// Row pass.
// ---------------------------------------------------------------------------
// Row pass of iteration m = sel_done + 1 (in final mode: no new
// iteration).  It first takes over the selection made by the last k_select,
// unless a finalize already did: every block computes the chosen learners
// from q, block 0 records them in the traces, and every block applies the
// update to its rows (f = g + nu b_k; ACWB: h += eta b_kcor with
// eta = gamma nu (S + 1) / 2 for selection S).  A block covers it.chunks
// consecutive chunks of kStateRows rows (several when a launch has many
// more chunks than the chip has room for blocks, as a large batch does):
// the selection and the winners' tables are taken once, and each chunk
// writes its own risk and maximum partials.
// UNB: the launch's fits have unbinned learners (32-bit codes per row);
// else the winners' columns stay as packed uint16 pairs until used.
template <bool UNB>
__global__ void __launch_bounds__(kStateThreads)
k_state(const FitDev* __restrict__ fits, const RowItem* __restrict__ items, int final_mode) {
  extern __shared__ float s_tab[];  // [2][nb_max]
  __shared__ double s_red[kStateThreads + 16];
  __shared__ Arg2 s_w[2][kStateThreads / 64];
  __shared__ int s_bad;
  const RowItem it = items[blockIdx.x];
  int64_t base = it.base + (int64_t)threadIdx.x * kRowsPerThread;
  bool rows = base < it.n_pad;
  const bool two = it.two != 0;
  // One round of loads, none of the model state's behind a branch (a branch
  // join makes the compiler wait for loads issued inside it): threads past
  // the end read the last 8 rows and store nothing, and a one-signal fit,
  // which keeps no h and c, reads f again there (cache hits).  The control
  // block comes in through scalar loads, so testing it does not wait for
  // the model state.
  float f[8], yv[8], hv[8], cv[8];
  int64_t lb = rows ? base : it.n_pad - kRowsPerThread;
  load8f((two ? it.h : it.fg) + lb, hv);
  load8f((two ? it.c : it.fg) + lb, cv);
  double qv0 = INFINITY, qv1 = INFINITY;
  if ((int)threadIdx.x < it.p) {
    qv0 = gp(it.q)[threadIdx.x];
    qv1 = gp(it.q)[it.p + threadIdx.x];  // used only after an ACWB selection
  }
  Ctl* ctl = it.ctl;
  const GLOBAL Ctl* gctl = gp(it.ctl);
  const int S = gctl->sel_done;
  const int fin = gctl->fin_done;
  const int sel_acwb = gctl->sel_acwb;
  const int switched = gctl->switched;
  load8f(it.fg + lb, f);
  load8f(it.y + lb, yv);
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
  // fitted rows: all rows after an HCWB switch; else the training rows (a
  // prefix, or for a fold fit every row outside its held-out fold)
  const bool all_rows = it.variant == CWB_HCWB && switched;
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
  constexpr bool unb = UNB;
  constexpr int NW = UNB ? 8 : 4;  // index registers per winner column
  uint32_t ik[NW], ic[NW];
  // row j's index in a winner column
  auto idx = [](const uint32_t* a, int j) -> uint32_t {
    return UNB ? a[j] : ((a[j >> 1] >> (16 * (j & 1))) & 0xffffu);
  };
  uint32_t fold_lo = 0u, fold_hi = 0u;  // fold fit: the 8 rows' fold ids, one byte each
  // this thread's winner-column and fold loads for the chunk at `base`
  auto load_cols = [&]() {
    if (rows && it.fold) {
      const unsigned long long fv =
          *reinterpret_cast<const GLOBAL unsigned long long*>(gp(it.fold) + base);
      fold_lo = (uint32_t)fv;
      fold_hi = (uint32_t)(fv >> 32);
    }
    if (UNB) {
      const uint32_t* XU = reinterpret_cast<const uint32_t*>(it.X);
      if (rows && use_t) load8c(XU + (size_t)kk * it.n_pad + base, ik);
      if (rows && (use_h || use_cc)) load8c(XU + (size_t)kc * it.n_pad + base, ic);
    } else {
      auto load4 = [&](int k, uint32_t* a) {
        const u32x4 w = *(const GLOBAL u32x4*)(it.X + (size_t)k * it.n_pad + base);
        a[0] = w.x;
        a[1] = w.y;
        a[2] = w.z;
        a[3] = w.w;
      };
      if (rows && use_t) load4(kk, ik);
      if (rows && (use_h || use_cc)) load4(kc, ic);
    }
  };
  load_cols();
  if (use_t) stage<kStateThreads, 4>(tf, it.table + (size_t)kk * nb, nb);
  if (use_h || use_cc) stage<kStateThreads, 4>(tc, it.table + ((size_t)it.p + kc) * nb, nb);
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();

  const float vt = 2.0f / (float)(m + 1);
  const float cw = (float)m / (float)(m + 1);
  for (int ch = 0;;) {
    double risk_t = 0.0, risk_v = 0.0;
    float amax_r = 0.0f, amax_c = 0.0f;
    bool bad = false;
    if (rows) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t i = base + j;
        const bool live = i < it.n;
        float fj = f[j];
        float hj = two ? hv[j] : 0.0f;
        if (live && use_t) fj = fj + nu * table_at(unb, idx(ik, j), tf);
        if (live && use_h) hj = hj + eta * table_at(unb, idx(ic, j), tc);
        const bool train =
            it.fold ? (int)(((j < 4 ? fold_lo : fold_hi) >> (8 * (j & 3))) & 0xffu) != it.fold_k
                    : i < it.n_train;
        if (live) {
          const double L = row_loss(it.loss, yv[j], fj);
          if (train) risk_t += L; else risk_v += L;
          if (!isfinite(fj) || !isfinite(hj)) bad = true;
        }
        f[j] = fj;
        hv[j] = hj;
        float rj = 0.0f, cj = 0.0f;
        if (!final_mode && live) {
          const bool fitrow = all_rows || train;
          if (acwb) {
            const float g = (1.0f - vt) * fj + vt * hj;
            const float r = neg_gradient(it.loss, yv[j], g);
            float c = r;
            if (use_cc) c = r + cw * (cv[j] - table_at(unb, idx(ic, j), tc));
            f[j] = g;  // the primary model update f = g + nu b_k is pending
            if (fitrow) {
              rj = r;
              cj = c;
            }
          } else {
            const float r = neg_gradient(it.loss, yv[j], fj);
            if (fitrow) rj = r;
          }
        }
        // r and c take the registers of y and the previous c, which this
        // row no longer needs
        yv[j] = rj;
        cv[j] = cj;
        amax_r = fmaxf(amax_r, fabsf(rj));
        amax_c = fmaxf(amax_c, fabsf(cj));
      }
      store8f(it.fg + base, f);
      if (two) store8f(it.h + base, hv);
      if (!final_mode) {
        store8f(it.r + base, yv);
        if (acwb) store8f(it.c + base, cv);
      }
    }
    if (bad) s_bad = 1;
    const bool last = ch + 1 >= it.chunks;
    if (!last) {
      // the next chunk's rows and winner columns, loaded into the registers
      // this chunk has finished with, so that they arrive while this
      // chunk's partials are reduced
      base += kStateRows;
      rows = base < it.n_pad;
      lb = rows ? base : it.n_pad - kRowsPerThread;
      load8f((two ? it.h : it.fg) + lb, hv);
      load8f((two ? it.c : it.fg) + lb, cv);
      load8f(it.fg + lb, f);
      load8f(it.y + lb, yv);
      load_cols();
    }
    double st = risk_t, sv = risk_v;
    float a = amax_r, b = amax_c;
    block_sum2_max2<kStateThreads>(st, sv, a, b, s_red);
    if (threadIdx.x == 0) {
      it.risk_part[2 * ch] = st;
      it.risk_part[2 * ch + 1] = sv;
      if (!final_mode) {
        if (!isfinite(a) || !isfinite(b)) s_bad = 1;
        it.amax_part[2 * ch] = a;
        it.amax_part[2 * ch + 1] = b;
      }
    }
    if (last) break;
    ++ch;
    __syncthreads();  // thread 0's partial writes and s_red reads precede the next reduction
  }
  if (threadIdx.x == 0 && s_bad) atomicOr(&it.ctl->error, 1);
}

// ---------------------------------------------------------------------------
// Per-learner solve and selection.
// ---------------------------------------------------------------------------
namespace {

// This thread's share of the deterministic sums of the row-pass risk
// partials (training rows, validation rows), continued from the partials
// before `first` (a multiple of 4 * kSelectThreads) already in *st, *sv;
// block_sum completes them.
__device__ void risk_shares(const double* part, int count, double* st, double* sv, int first = 0) {
  const GLOBAL f64x2* g = (const GLOBAL f64x2*)gp(part);
  double a = *st, b = *sv;
  for (int b0 = first; b0 < count; b0 += 4 * kSelectThreads) {
    f64x2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = b0 + u * kSelectThreads + (int)threadIdx.x;
      if (i < count) v[u] = g[i];
      else v[u].x = v[u].y = 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a += v[u].x;
      b += v[u].y;
    }
  }
  *st = a;
  *sv = b;
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
  // dynamic LDS: s[nb_cap] | Ainv[d_cap^2] | G[d_cap^2] | bstart[nb_cap, padded to even]
  // | (STAGED) bval[nb_cap*4]
  extern __shared__ double s_dyn[];
  __shared__ double s_v[kMaxD], s_th[kMaxD], s_gt[kMaxD];
  __shared__ double s_part[kMaxD * kChunks];
  __shared__ long long s_off[kMaxSlots];  // this signal's segment offsets
  __shared__ int s_jr[2 * kMaxD];
  __shared__ float s_red[kSelectThreads + 16];
  double* s_bins = s_dyn;
  double* s_ai = s_dyn + nb_cap;
  double* s_g = s_ai + (size_t)d_cap * d_cap;
  int* s_bs = reinterpret_cast<int*>(s_g + (size_t)d_cap * d_cap);
  double* s_bv = reinterpret_cast<double*>(s_bs + ((nb_cap + 1) & ~1));
  const SelItem it = items[blockIdx.x];
  // blockIdx.y is the signal this block solves (ACWB: 0 for r, 1 for c)
  const int sig = (int)blockIdx.y;
  if (sig > 0 && it.variant == CWB_CWB) return;
  const int d = it.d, nb = it.nb, band = it.band, n_off = it.n_off;
  // the first chunk of the signal's partials, loaded in the first round when
  // its offsets are inline (bins 4t .. 4t+3 of every segment).  The variant
  // for large launches (a batch, STAGED false) preloads at most half as many
  // segments: 32 fewer registers per lane, more blocks resident per CU; its
  // learner groups rarely span more segments.
  constexpr int NPRE = STAGED ? kInlineOffs : kInlineOffs / 2;
  const bool pre = n_off <= NPRE && nb <= 4 * kSelectThreads;
  i64x2 pv[NPRE][2];
  if (pre && 4 * (int)threadIdx.x < nb) {
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
      if (i < n_off) {
        const int64_t o = sig ? it.off1[i] : it.off0[i];
        const GLOBAL i64x2* src = (const GLOBAL i64x2*)(partials + o + 4 * threadIdx.x);
        pv[i][0] = src[0];
        pv[i][1] = src[1];
      }
    }
  }
  // one round of independent loads: control block, signal maxima, (learner
  // 0) risk partials, offsets and the learner's tables for the training-row
  // Gram set.  Every load of the round is issued before the first use of
  // any: the memory counter drains in order, so consuming a load waits for
  // every load issued before it.
  constexpr int NT = kSelectThreads;
  const GLOBAL Ctl* ctl = gp(it.ctl);
  const int P = ctl->pick_done;  // = iterations before this selection
  const int switched = ctl->switched;
  StagePass<NT, 4, f32x2> pm;  // per row-pass block: largest |r|, |c|
  StagePass<NT, 4, f64x2> pr;  // per row-pass block: training, validation risk
  pm.load_or_zero((const f32x2*)it.amax_part, it.n_row_blocks);
  const bool book = it.k == 0 && sig == 0;  // the fit's risk bookkeeping
  if (book) pr.load_or_zero((const f64x2*)it.risk_part, it.n_row_blocks);
  const int n_stage = n_off < kMaxSlots ? n_off : kMaxSlots;
  const long long* offs = (const long long*)it.offs + (int64_t)sig * n_off;  // this signal's
  {
    // the band starts always (the loops below index the design through
    // them); the design values only when they fit.  First passes here (one
    // round trip for the usual sizes: d <= 32, n* <= 1,024, up to 1,024
    // row-pass blocks); longer arrays finish below.
    StagePass<NT, 2, long long> po0;
    StagePass<NT, 4, double> pa, pg;
    StagePass<NT, 1, int> pj;
    StagePass<NT, 4, int> pb;
    StagePass<NT, 16, double> pv;
    po0.load(offs, n_stage);
    pa.load(it.ainv[0], d * d);
    pg.load(it.gram[0], d * d);
    pj.load(it.jr, 2 * d);
    pb.load(it.bstart, nb);
    if (STAGED) pv.load(it.bval, nb * kMaxBand);
    po0.store(s_off, n_stage);
    pa.store(s_ai, d * d);
    pg.store(s_g, d * d);
    pj.store(s_jr, 2 * d);
    pb.store(s_bs, nb);
    if (STAGED) pv.store(s_bv, nb * kMaxBand);
  }
  stage_rest<NT, 2>(s_off, offs, n_stage, 2 * NT);
  stage_rest<NT, 4>(s_ai, it.ainv[0], d * d, 4 * NT);
  stage_rest<NT, 4>(s_g, it.gram[0], d * d, 4 * NT);
  stage_rest<NT, 1>(s_jr, it.jr, 2 * d, NT);
  stage_rest<NT, 4>(s_bs, it.bstart, nb, 4 * NT);
  if (STAGED) stage_rest<NT, 16>(s_bv, it.bval, nb * kMaxBand, 16 * NT);
  float am0 = 0.0f, am1 = 0.0f;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    am0 = fmaxf(am0, pm.v[u].x);
    am1 = fmaxf(am1, pm.v[u].y);
  }
  {
    const GLOBAL f32x2* am = (const GLOBAL f32x2*)it.amax_part;
    for (int b0 = 4 * NT; b0 < it.n_row_blocks; b0 += 4 * NT) {
      f32x2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + u * NT + (int)threadIdx.x;
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
  // learner 0's signal-0 block: its shares of the risk sums (first pass in
  // order, then the rest)
  double risk_t = 0.0, risk_v = 0.0;
  if (book) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      risk_t += pr.v[u].x;
      risk_v += pr.v[u].y;
    }
    risk_shares(it.risk_part, it.n_row_blocks, &risk_t, &risk_v, 4 * NT);
  }
  if (P >= it.M) return;
  const bool hcwb_all = it.variant == CWB_HCWB && switched;
  const bool acwb = it.variant == CWB_ACWB || (it.variant == CWB_HCWB && !switched);
  const int nsig = acwb ? 2 : 1;
  if (sig >= nsig) return;  // the fit fits one signal this iteration
  const int64_t n_fit = hcwb_all ? it.n : it.n_scan;
  if (book) {
    // learner 0's block: the risk of f^[P] from this iteration's row pass,
    // and the count and kind of this selection for the next row pass
    const double rt = block_sum<kSelectThreads>(risk_t, s_part);
    const double rv = block_sum<kSelectThreads>(risk_v, s_part);
    if (threadIdx.x == 0) {
      it.tr_risk[P] = rt / (double)it.n_train;
      it.tr_val[P] = (it.n > it.n_train) ? rv / (double)(it.n - it.n_train) : 0.0;
      gp(it.ctl)->sel_done = P + 1;
      gp(it.ctl)->sel_acwb = acwb ? 1 : 0;
    }
  }
  if (hcwb_all) {  // HCWB after the switch: Grams over all rows
    __syncthreads();
    stage<kSelectThreads, 4>(s_ai, it.ainv[1], d * d);
    stage<kSelectThreads, 4>(s_g, it.gram[1], d * d);
  }
  const Basis B = STAGED ? Basis{s_bv, s_bs} : Basis{it.bval, s_bs};
  block_max2<kSelectThreads>(am0, am1, s_red);
  const float amax[2] = {am0, am1};
  {  // this block's signal
    // the histogram pass's scale for this learner: 32-bit (rounded) or int64
    const int e = it.acc32_bits > 0 ? scale_exponent32(amax[sig], it.acc32_bits)
                                    : scale_exponent(amax[sig], n_fit);
    const double isc = ldexp(1.0, -e);
    // bin sums s_l: exact int64 merge of the group's segment partials.  Many
    // segments and few bins (a small fit spread over many histogram blocks):
    // the threads split the segments as well as the bins, and their int64
    // sums meet in LDS through atomic adds (exact, so in any order).
    const int nch = (nb + 3) / 4;  // 4-bin chunks
    const int slices =
        (!pre && 2 * nch <= kSelectThreads) ? min(kSelectThreads / nch, n_off) : 1;
    if (slices > 1) {
      unsigned long long* s_acc = reinterpret_cast<unsigned long long*>(s_part);  // 4 nch <= 512
      for (int i = threadIdx.x; i < 4 * nch; i += kSelectThreads) s_acc[i] = 0ull;
      __syncthreads();
      const int ch = (int)threadIdx.x % nch, sl = (int)threadIdx.x / nch;
      const int l = 4 * ch;
      long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      for (int c0 = 0; c0 < n_off; c0 += kMaxSlots) {
        const int cnt = (n_off - c0) < kMaxSlots ? (n_off - c0) : kMaxSlots;
        if (n_off > kMaxSlots) {  // more segments than the staged list holds
          __syncthreads();
          stage<kSelectThreads, 2>(s_off, offs + c0, cnt);
          __syncthreads();
        }
        if (sl < slices) {
#pragma unroll 8
          for (int i = sl; i < cnt; i += slices) {
            const GLOBAL i64x2* src = (const GLOBAL i64x2*)(partials + s_off[i] + l);
            const i64x2 u = src[0], w = src[1];
            a0 += u.x;
            a1 += u.y;
            a2 += w.x;
            a3 += w.y;
          }
        }
      }
      if (sl < slices) {
        __hip_atomic_fetch_add(s_acc + l, (unsigned long long)a0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(s_acc + l + 1, (unsigned long long)a1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(s_acc + l + 2, (unsigned long long)a2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(s_acc + l + 3, (unsigned long long)a3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      __syncthreads();
      for (int i = threadIdx.x; i < nb; i += kSelectThreads) s_bins[i] = (double)(long long)s_acc[i] * isc;
    } else
    for (int l0 = 0; l0 < nb; l0 += 4 * kSelectThreads) {
      long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      const int l = l0 + 4 * threadIdx.x;
      if (pre) {  // l0 == 0: the preloaded chunk
        if (l < nb) {
#pragma unroll
          for (int i = 0; i < NPRE; ++i) {
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
        const long long* so = s_off;
        if (n_off > kMaxSlots) {  // more segments than the staged list holds
          __syncthreads();
          stage<kSelectThreads, 2>(s_off, offs + c0, cnt);
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
#pragma unroll 4
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
    if (it.kind == CWB_BINARY_CAT) {
      // one learner per class (indicator column, no penalty): theta_l =
      // s_l / n_l and q_l = theta_l (n_l theta_l - 2 s_l); the best class
      // (ties to the lower one) stands for the feature.  Empty classes
      // (n_l = 0) have no estimate and are skipped.
      if (threadIdx.x == 0) {
        int bl = -1;
        double bq = INFINITY, bt = 0.0;
        for (int j = 0; j < d; ++j) {
          const double nl = s_g[(size_t)j * d + j];
          if (!(nl > 0.0)) continue;
          const double t = s_v[j] / nl;
          const double qj = t * (nl * t - 2.0 * s_v[j]);
          if (qj < bq) {
            bq = qj;
            bt = t;
            bl = j;
          }
        }
        for (int j = 0; j < d; ++j) s_th[j] = (j == bl) ? bt : 0.0;
        it.q[(size_t)sig * it.p] = bq;
      }
      __syncthreads();
    } else {
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
    }
    GLOBAL double* th = gp(it.theta + (size_t)sig * it.p * it.d_max);
    for (int j = threadIdx.x; j < it.d_max; j += kSelectThreads) th[j] = (j < d) ? s_th[j] : 0.0;
    // candidate update table Z^b theta
    GLOBAL float* tab = gp(it.table + (size_t)sig * it.p * it.nb_max);
    for (int l = threadIdx.x; l < nb; l += kSelectThreads) {
      const int b0 = B.bstart[l];
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < kMaxBand; ++b)
        if (b < band) t += B.bval[(size_t)l * kMaxBand + b] * s_th[b0 + b];
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
  double st = 0.0, sv = 0.0;
  risk_shares(F.risk_part, F.n_row_blocks, &st, &sv);
  const double rt = block_sum<kSelectThreads>(st, s_red);
  const double rv = block_sum<kSelectThreads>(sv, s_red);
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

// The fitted primary model at new feature values (Section 2.3: the
// intercept plus every learner's fitted function).  Thread i takes row i of
// the column-major x (column stride ldx) and adds, per learner, the B-spline
// basis of degree 1..3 at x (clamped to the training range; equally spaced
// knots, so the degree+1 nonzero values are the uniform segment polynomials
// of the position t inside the knot interval) against the learner's
// aggregated coefficients, or the coefficient of a categorical level (an
// invalid level gives NaN).  FP64 throughout.
__device__ __forceinline__ void uniform_basis(int degree, double t, double* b) {
  const double s = 1.0 - t;
  if (degree == 1) {
    b[0] = s;
    b[1] = t;
  } else if (degree == 2) {
    b[0] = 0.5 * s * s;
    b[1] = 0.5 * (-2.0 * t * t + 2.0 * t + 1.0);
    b[2] = 0.5 * t * t;
  } else {
    const double t2 = t * t, t3 = t2 * t;
    b[0] = s * s * s / 6.0;
    b[1] = (3.0 * t3 - 6.0 * t2 + 4.0) / 6.0;
    b[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) / 6.0;
    b[3] = t3 / 6.0;
  }
}

// Learners [k0, k1) only: column k - k0 of x holds learner k's values (a
// partial effect is one learner with f0 = 0).
__global__ void __launch_bounds__(kStateThreads)
k_predict(const FitDev* __restrict__ fits, const double* __restrict__ x, int64_t n, int64_t ldx,
          double f0, int k0, int k1, double* __restrict__ out) {
  const FitDev& F = fits[0];
  const int64_t i = (int64_t)blockIdx.x * kStateThreads + threadIdx.x;
  if (i >= n) return;
  const GLOBAL double* xg = gp(x);
  const GLOBAL double* cf = gp(F.coef_f);
  double acc = f0;
  for (int k = k0; k < k1; ++k) {
    const FeatDev fd = F.feat[k];
    const double v = xg[(size_t)(k - k0) * ldx + i];
    if (fd.kind != CWB_PSPLINE) {  // categorical: the level's coefficient
      const int lev = (int)v;
      acc += (v >= 0.0 && lev < fd.d && (double)lev == v) ? cf[fd.coef_off + lev] : NAN;
      continue;
    }
    const double xv = fmin(fmax(v, fd.xmin), fd.xmax);
    const double hk = (fd.xmax - fd.xmin) / (double)(fd.n_int + 1);
    const double u = (xv - fd.xmin) / hk;
    int j = (int)floor(u);
    j = j < 0 ? 0 : (j > fd.n_int ? fd.n_int : j);
    const double t = fmin(fmax(u - (double)j, 0.0), 1.0);
    double b[4];
    uniform_basis(fd.degree, t, b);
    for (int a = 0; a <= fd.degree; ++a) acc += b[a] * cf[fd.coef_off + j + a];
  }
  out[i] = acc;
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------

hipError_t launch_state(hipStream_t st, const FitDev* fits, const RowItem* items, int nitems,
                        int nb_max, int final_mode, bool unbinned) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * nb_max * sizeof(float);
  if (unbinned)
    hipLaunchKernelGGL(k_state<true>, dim3(nitems), dim3(kStateThreads), lds, st, fits, items, final_mode);
  else
    hipLaunchKernelGGL(k_state<false>, dim3(nitems), dim3(kStateThreads), lds, st, fits, items, final_mode);
  return hipGetLastError();
}


hipError_t launch_select(hipStream_t st, const SelItem* items, int nitems, int nsig, int nb_max,
                         int d_max, const long long* partials) {
  if (nitems <= 0) return hipSuccess;
  if (nsig < 1 || nsig > kNumSig) return hipErrorInvalidValue;
  // static LDS of the kernel (incl. the selection step) stays below 16 KiB
  size_t lds = ((size_t)nb_max + 2 * (size_t)d_max * d_max) * sizeof(double) +
               (size_t)((nb_max + 1) & ~1) * sizeof(int);
  const size_t extra = (size_t)nb_max * kMaxBand * sizeof(double);
  bool staged = nb_max <= kStageBins && lds + extra <= 144 * 1024;
  if (staged) {
    // Staging the reduced design in LDS shortens each block, but a large
    // footprint can leave fewer blocks per CU: with many learners (a batch)
    // keep the variant that needs fewer rounds of blocks over the chip.
    struct Occ {
      int cus = 0;
      size_t stat = 16 * 1024;
    };
    static Occ occ[64];
    int dev = 0;
    (void)hipGetDevice(&dev);
    Occ& o = occ[dev & 63];
    if (o.cus == 0) {
      int cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 1;
      hipFuncAttributes fa;
      if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_select<true>)) == hipSuccess)
        o.stat = fa.sharedSizeBytes;
      (void)hipGetLastError();
      o.cus = cus;
    }
    const size_t cu_lds = 160 * 1024;
    auto rounds = [&](size_t per_block) {
      int bpc = (int)(cu_lds / (per_block + o.stat));
      bpc = bpc < 1 ? 1 : (bpc > 8 ? 8 : bpc);  // 8 blocks of 4 waves fill a CU
      const int64_t slots = (int64_t)o.cus * bpc;
      return ((int64_t)nitems * nsig + slots - 1) / slots;
    };
    staged = rounds(lds + extra) <= rounds(lds);
  }
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
    hipLaunchKernelGGL(k_select<true>, dim3(nitems, nsig), dim3(kSelectThreads), lds, st, items,
                       partials, nb_max, d_max);
  else
    hipLaunchKernelGGL(k_select<false>, dim3(nitems, nsig), dim3(kSelectThreads), lds, st, items,
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

hipError_t launch_predict(hipStream_t st, const FitDev* fit, const double* x, int64_t n, int64_t ldx,
                          double f0, int k0, int k1, double* out) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + kStateThreads - 1) / kStateThreads;
  hipLaunchKernelGGL(k_predict, dim3((unsigned)blocks), dim3(kStateThreads), 0, st, fit, x, n, ldx,
                     f0, k0, k1, out);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t st, const FitDev* fits, int nfits) {
  if (nfits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(nfits), dim3(kSelectThreads), 0, st, fits);
  return hipGetLastError();
}

}  // namespace cwb

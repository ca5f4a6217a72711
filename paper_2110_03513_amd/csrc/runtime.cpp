// runtime.cpp -- C ABI of the library: fit and batch objects, the histogram
// schedule, the workspace layout and the per-iteration launch sequence.
#include "runtime.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>

#include "kernels.h"

namespace cwb {

namespace {
thread_local std::string g_err;

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return set_error(CWB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int device_cus(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
  return prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
}

}  // namespace

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int shape_from_problem(const cwb_problem* pr, FitShape* sh, std::string* err) {
  if (!pr) { *err = "null problem"; return CWB_E_INVALID_ARG; }
  if (pr->n < 2 || pr->p < 1 || !pr->specs) { *err = "need n >= 2, p >= 1 and specs"; return CWB_E_INVALID_ARG; }
  if (pr->M < 1) { *err = "M must be >= 1"; return CWB_E_INVALID_ARG; }
  if (pr->n > (int64_t)INT32_MAX) { *err = "n above 2^31 - 1 rows is not supported"; return CWB_E_UNSUPPORTED; }
  sh->n = pr->n;
  sh->n_pad = (pr->n + 63) / 64 * 64;
  int64_t nt = pr->n;
  if (pr->val_mask) {
    nt = 0;
    for (int64_t i = 0; i < pr->n; ++i) nt += pr->val_mask[i] ? 0 : 1;
  }
  sh->n_train = nt;
  sh->n_scan = nt;
  sh->p = pr->p;
  sh->M = pr->M;
  sh->variant = pr->variant;
  sh->nsig_max = (pr->variant == CWB_CWB) ? 1 : 2;
  sh->nb_max = sh->d_max = sh->sum_d = 0;
  sh->sum_nb = sh->sum_d2 = 0;
  sh->unbinned = false;
  int nb_min = kMaxBins;
  for (int j = 0; j < pr->p; ++j) {
    const cwb_learner_spec& s = pr->specs[j];
    int nb, d;
    if (s.kind == CWB_RIDGE_CAT || s.kind == CWB_BINARY_CAT) {
      nb = s.n_levels;
      d = s.n_levels;
    } else if (s.n_bins == 0) {  // unbinned: the basis functions take the place of bins
      d = s.n_interior_knots + s.degree + 1;
      nb = d;
      sh->unbinned = true;
    } else {
      nb = bins_for(s.n_bins, pr->n);
      d = s.n_interior_knots + s.degree + 1;
    }
    if (nb < 1 || nb > kMaxBins || d < 1 || d > kMaxD) {
      *err = "learner " + std::to_string(j) + ": bins must be 2..8192 and basis size 1..64";
      return (nb > kMaxBins && nb <= 65535) ? CWB_E_UNSUPPORTED : CWB_E_INVALID_ARG;
    }
    sh->nb_max = std::max(sh->nb_max, nb);
    nb_min = std::min(nb_min, nb);
    sh->d_max = std::max(sh->d_max, d);
    sh->sum_d += d;
    sh->sum_nb += nb;
    sh->sum_d2 += (int64_t)d * d;
  }
  sh->nb_stride = (sh->nb_max + 3) / 4 * 4;
  if (sh->unbinned) sh->nb_stride = (kUnbCopies * sh->d_max + 3) / 4 * 4;
  int st = 0;
  sh->copies = !sh->unbinned && copy_mask(nb_min, sh->nb_stride, &st) != 0;
  sh->x12 = !sh->unbinned && sh->nb_max <= 4096;
  sh->n_row_blocks = (int)((sh->n_pad + kStateRows - 1) / kStateRows);
  const int64_t nv = sh->n - sh->n_train;
  sh->n_val_blocks = (sh->variant == CWB_HCWB && nv > 0) ? (int)((nv + kStateRows - 1) / kStateRows) : 0;
  return CWB_OK;
}

namespace {

bool hist_env_set() {
  for (const char* v : {"CWB_HIST_NT", "CWB_HIST_LDS_KB", "CWB_HIST_BPC", "CWB_HIST_SLICES",
                        "CWB_HIST_BLOCKS", "CWB_HIST_F"}) {
    const char* e = std::getenv(v);
    if (e && *e) return true;
  }
  return false;
}

Tune tune_with(int nt, int lds_kb, int bpc, int slices, int blocks, int fset, int nb_stride,
               int nsig_max, int p_max, bool unbinned, int cus) {
  Tune t;
  t.cus = cus;
  t.nt = (nt == 256 || nt == 512 || nt == 1024) ? nt : 512;
  t.lds_kb = std::max(8, std::min(152, lds_kb));
  t.blocks_per_cu = std::max(1, std::min(8, bpc));
  t.slices = std::max(1, std::min(64, slices));
  t.blocks = std::max(0, std::min(65536, blocks));
  const size_t per_learner = (size_t)nsig_max * nb_stride * sizeof(long long);
  int F = (int)((size_t)t.lds_kb * 1024 / per_learner);
  if (fset > 0) F = fset;
  F = std::max(1, std::min(16, F));
  F = std::min(F, std::max(1, p_max));
  while (F > 1 && (size_t)F * per_learner > (size_t)kHistMaxLds) --F;
  // register budget at 1024 threads: groups of at most 8 learners (one
  // signal) or 4 learners (two signals); wider groups would spill
  if (t.nt == 1024) F = std::min(F, nsig_max == 1 ? 8 : 4);
  // unbinned groups hold 32 bytes of codes per learner and thread
  if (unbinned) F = std::min(F, t.nt == 1024 ? (nsig_max == 1 ? 4 : 2) : 8);
  t.F = F;
  t.fmax = 1;
  while (t.fmax < F) t.fmax *= 2;
  return t;
}

}  // namespace

// Default tile shape (measured on the headline and momentum workloads): 512
// threads; one signal with a 32 KiB histogram budget (four learners per
// group at 1,000 bins), two signals with 128 KiB (eight).  Timed back to back
// the 512- and 1,024-thread one-signal tiles tie, but inside the iteration
// (after the row pass) the 512-thread tile ran 1-4 us faster in every A/B
// run, with either index copy, so it is the one the autotuner keeps unless
// another is clearly faster.
Tune make_tune(int nb_stride, int nsig_max, int p_max, bool unbinned) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const bool two = nsig_max == 2;
  return tune_with(env_int("CWB_HIST_NT", 512), env_int("CWB_HIST_LDS_KB", two ? 128 : 32),
                   env_int("CWB_HIST_BPC", 1), env_int("CWB_HIST_SLICES", 1),
                   env_int("CWB_HIST_BLOCKS", 0), env_int("CWB_HIST_F", 0), nb_stride, nsig_max,
                   p_max, unbinned, device_cus(dev));
}

// Tile shapes the autotuner tries: the default first, then threads x LDS
// budget x blocks per CU, and for small work (`work`, 8-row units times
// learners, at most 512 per block at one block per CU) grids of 16 to 64
// blocks, whose fewer segments per learner group also shorten the select
// pass's merge.  Explicit CWB_HIST_* settings, or CWB_AUTOTUNE=0, leave the
// default alone.
std::vector<Tune> tune_candidates(int nb_stride, int nsig_max, int p_max, bool unbinned, bool all,
                                  int64_t work) {
  std::vector<Tune> out{make_tune(nb_stride, nsig_max, p_max, unbinned)};
  const int cus = out[0].cus;
  const bool small = work <= (int64_t)512 * 256;
  // small work: by default about 512 units (4,096 rows) per learner group
  // and block, so that each group's segments stay few for the select merge
  if (small && !hist_env_set())
    out[0].blocks = (int)std::max<int64_t>(16, std::min<int64_t>(cus, work / 512));
  if (!all || hist_env_set() || env_int("CWB_AUTOTUNE", 1) == 0) return out;
  auto add = [&](const Tune& t) {
    bool dup = false;
    for (const Tune& u : out)
      dup = dup || (u.nt == t.nt && u.F == t.F && u.blocks_per_cu == t.blocks_per_cu &&
                    u.slices == t.slices && u.blocks == t.blocks);
    if (!dup) out.push_back(t);
  };
  for (int nt : {1024, 512, 256})
    for (int kb : {32, 64, 128})
      for (int bpc : {1, 2}) add(tune_with(nt, kb, bpc, 1, 0, 0, nb_stride, nsig_max, p_max, unbinned, cus));
  // two learners per group: where a learner's histograms are large (the
  // folds of a cross-validation share a group's LDS, 5 folds x 1,000 bins)
  // the budgets above step from one learner to three, and two ran fastest
  // there (5 folds, n = 1e6, p = 50: 9,379 iterations/s at 1,024 threads
  // against 9,197 with one learner and 6,345 with three)
  for (int nt : {1024, 512}) add(tune_with(nt, 152, 1, 1, 0, 2, nb_stride, nsig_max, p_max, unbinned, cus));
  if (small)
    for (int nt : {512, 256})
      for (int blocks : {16, 32, 64})
        add(tune_with(nt, 32, 1, 1, blocks, 0, nb_stride, nsig_max, p_max, unbinned, cus));
  return out;
}

void SchedCap::add(const Schedule& S) {
  segs = std::max(segs, S.segs.size());
  blk = std::max(blk, S.blk.size());
  sel_off = std::max(sel_off, S.sel_off.size());
  partial_words = std::max(partial_words, S.partial_words);
}

int64_t unit_at_row(const FitShape& sh, int64_t row) {
  const int64_t U = sh.n_pad / 8, n8 = (sh.n_scan + 7) / 8;
  const int64_t r8 = (row + 7) / 8;  // first whole 8-row unit at or after row
  if (n8 <= 0) return 0;
  return std::min(U, (r8 * U + n8 - 1) / n8);
}

void unit_rows(const FitShape& sh, int64_t u0, int64_t u1, int64_t* r0, int64_t* r1) {
  const int64_t U = sh.n_pad / 8, n8 = (sh.n_scan + 7) / 8;
  *r0 = 8 * (u0 * n8 / U);
  *r1 = 8 * (u1 * n8 / U);
}

int segment_fold(const FitShape& sh, int64_t r0, int64_t r1) {
  const int K = (int)sh.fold_start.size() - 1;
  r1 = std::min(r1, sh.n);
  if (K < 1 || r1 <= r0) return -1;
  for (int j = 0; j < K; ++j)
    if (r0 >= sh.fold_start[j] && r1 <= sh.fold_start[j + 1]) return j;
  return -1;
}

// 1 if every learner of [k0, k0 + nf) takes 32-bit accumulation.
// 1 if every learner of the group keeps its sums over the segment's units
// [u0, u1) in int32 at the fit's 32-bit scale, with nt threads per block: a
// learner whose bins all hold fewer than 2^acc32_bits rows, or one with c
// LDS copies, each of which takes the rows of nt / c threads -- at most
// 8 rows per thread per step of 8 nt rows -- as long as those stay below
// 2^acc32_bits.  The segment's rows are bounded by 8 (u1 - u0 + 1) for
// either row count the pass maps its units onto (before and after an HCWB
// switch).
int group_acc32(const FitShape& sh, int k0, int nf, int64_t u0, int64_t u1, int nt) {
  if ((int)sh.acc32.size() != sh.p || sh.acc32_bits < 1 || sh.acc32_bits > kAcc32MaxBits) return 0;
  const int64_t rows = 8 * (u1 - u0 + 1), step = 8 * (int64_t)nt;
  const int64_t limit = ((int64_t)1 << sh.acc32_bits) - 1;
  for (int k = k0; k < k0 + nf; ++k) {
    if (sh.acc32[k]) continue;
    const int c = (int)sh.acc32_copies.size() == sh.p ? sh.acc32_copies[k] : 0;
    if (c < 2 || nt % c != 0) return 0;
    const int64_t per_copy = (rows + step - 1) / step * 8 * (nt / c);
    if (per_copy > limit) return 0;
  }
  return 1;
}

// LDS bytes the histogram pass takes for a segment (at the fit's most
// signals): 32-bit groups hold 4-byte words (one signal) or one packed
// 8-byte word per bin (two signals), the others 8-byte words per signal
// and fold.
size_t seg_lds_bytes(const Seg& sg, const FitShape& sh) {
  const int64_t nw = (int64_t)sg.nfit * sg.nf * sh.nb_stride;  // every fold's learners
  const int64_t words = sg.acc32 ? (sh.nsig_max == 1 ? (nw + 1) / 2 : nw) : sh.nsig_max * nw;
  return (size_t)words * sizeof(long long);
}

// Relative histogram work of one (row, learner) pair of a fit: a
// two-signal fit reads c beside r and adds 8-byte words, about 1.5 times a
// one-signal fit's cost, so the schedule balances blocks on 2 and 3 (on the
// 64-fit mixed batch, 3:2 ran its histogram pass in 294 us against 321 us
// unweighted, 305 us at 7:4 and 321 us at 2:1).
int sig_weight(const FitShape& sh) { return sh.nsig_max == 2 ? 3 : 2; }

Schedule build_schedule(const std::vector<const FitShape*>& fits, const Tune& t) {
  Schedule S;
  struct Item {
    int fit, k0, nf, nfit;
    int64_t u0, u1;
  };
  std::vector<Item> items;
  int64_t W = 0;
  for (int fi = 0; fi < (int)fits.size(); ++fi) {
    const FitShape& sh = *fits[fi];
    if (sh.share == 0) continue;  // a later fold: its group head's segments cover it
    const int nfit = sh.share;
    const int64_t U = sh.n_pad / 8;
    const int groups = (sh.p + t.F - 1) / t.F;
    const int slices = (int)std::max<int64_t>(1, std::min<int64_t>(t.slices, U));
    // a fold group's rows split at the fold blocks
    std::vector<int64_t> cuts;
    if (nfit > 1)
      for (size_t j = 1; j + 1 < sh.fold_start.size(); ++j) cuts.push_back(unit_at_row(sh, sh.fold_start[j]));
    for (int s = 0; s < slices; ++s) {
      const int64_t a = U * s / slices, b = U * (s + 1) / slices;
      std::vector<int64_t> pts{a};
      for (int64_t c : cuts)
        if (c > a && c < b) pts.push_back(c);
      pts.push_back(b);
      for (size_t i = 0; i + 1 < pts.size(); ++i) {
        const int64_t u0 = pts[i], u1 = pts[i + 1];
        if (u1 <= u0) continue;
        for (int g = 0; g < groups; ++g) {
          const int k0 = g * t.F;
          const int nf = std::min(t.F, sh.p - k0);
          items.push_back({fi, k0, nf, nfit, u0, u1});
          W += (int64_t)nf * nfit * sig_weight(sh) * (u1 - u0);
        }
      }
    }
  }
  const int B = t.blocks > 0 ? t.blocks : std::max(1, t.cus * t.blocks_per_cu);
  S.blocks = B;
  // Blocks get equal shares of the work, counting for every segment a block
  // starts a fixed cost of kSegUnits 8-row units of its group (at most a
  // quarter of a block's share): zeroing and flushing its LDS histograms
  // and refilling the row pipeline.  Timed per block at n = 1e6, p = 200
  // (512- and 1,024-thread tiles), a block with two segments took 4 us more
  // than one with a single segment of the same rows, about 1,700 units; with
  // 1,600 units charged they still ran 1 us (about 400 units) over the
  // others, so a segment counts 2,000.
  // Block v's share ends at (v + 1) Wt / B on the running cost; a segment
  // that would hold less than its own fixed cost starts in the next block
  // instead, and Wt (the work plus the fixed costs plus the room so left)
  // is refined until the last block gets its share.
  constexpr int64_t kSegUnits = 2000;
  const int64_t cs_cap = std::max<int64_t>(1, W / B / 4);
  auto seg_cost = [&](int64_t w) { return std::min(kSegUnits * w, cs_cap); };
  struct Cut {
    size_t item;
    int64_t u0, u1, vb;
  };
  std::vector<Cut> cuts_out;
  auto split = [&](int64_t Wt, std::vector<Cut>* out) -> int64_t {
    out->clear();
    int64_t vb = 0, pos = 0, used = -1;  // current block, running cost, last block given work
    for (size_t ii = 0; ii < items.size(); ++ii) {
      const Item& it = items[ii];
      const int64_t w = (int64_t)it.nf * it.nfit * sig_weight(*fits[it.fit]);  // work per 8-row unit
      const int64_t cs = seg_cost(w);
      int64_t u = it.u0;
      while (u < it.u1) {
        while (vb < B - 1) {
          const int64_t room = ((vb + 1) * Wt) / B - pos;
          if (room > 0 && (vb != used || room >= cs + w)) break;
          pos = std::max(pos, ((vb + 1) * Wt) / B);  // the block's unused room
          ++vb;
        }
        pos += cs;
        int64_t take = it.u1 - u;
        if (vb < B - 1) take = (((vb + 1) * Wt) / B - pos + w - 1) / w;
        const int64_t ue = std::min(it.u1, u + std::max<int64_t>(1, take));
        pos += (ue - u) * w;
        out->push_back({ii, u, ue, vb});
        used = vb;
        u = ue;
      }
    }
    return pos;
  };
  {
    // split() returns the running cost at the end: the last block's load
    // is that minus (B - 1) Wt / B, and it falls as Wt grows (a step
    // function, as segments move between blocks).  Bisect for the Wt that
    // leaves the last block closest to its share.
    int64_t cs_max = 0;
    for (const Item& it : items)
      cs_max = std::max(cs_max, seg_cost((int64_t)it.nf * it.nfit * sig_weight(*fits[it.fit])));
    int64_t lo = W, hi = W + (int64_t)(items.size() + 2 * (size_t)B) * (cs_max + 1);
    int64_t best = hi, best_err = INT64_MAX;
    for (int step = 0; step < 48 && lo <= hi; ++step) {
      const int64_t mid = lo + (hi - lo) / 2;
      const int64_t excess = split(mid, &cuts_out) - mid;  // the last block's load above its share
      if (std::llabs(excess) < best_err) {
        best_err = std::llabs(excess);
        best = mid;
      }
      if (excess == 0) break;
      if (excess > 0) lo = mid + 1;
      else hi = mid - 1;
    }
    split(best, &cuts_out);
  }
  std::vector<int64_t> seg_vb;
  for (const Cut& cu : cuts_out) {
    const Item& it = items[cu.item];
    const int64_t u = cu.u0, ue = cu.u1, vb = cu.vb;
    Seg sg;
    sg.fit = it.fit;
    sg.k0 = it.k0;
    sg.nf = it.nf;
    sg.nfit = (int16_t)it.nfit;
    sg.skip = -1;
    sg.acc32 = 1;  // every fold of the group must keep 32-bit sums
    for (int q = 0; q < it.nfit; ++q)
      sg.acc32 &= group_acc32(*fits[it.fit + q], it.k0, it.nf, u, ue, t.nt);
    sg.pad = 0;
    if (it.nfit > 1) {
      int64_t r0, r1;
      unit_rows(*fits[it.fit], u, ue, &r0, &r1);
      sg.skip = (int16_t)segment_fold(*fits[it.fit], r0, r1);
    }
    sg.u0 = u;
    sg.u1 = ue;
    sg.slot = 0;
    S.segs.push_back(sg);
    seg_vb.push_back(vb);
  }
  // partial slots
  int64_t off = 0;
  for (Seg& sg : S.segs) {
    sg.slot = off;
    const FitShape& sh = *fits[sg.fit];
    off += (int64_t)sg.nfit * sh.nsig_max * sg.nf * sh.nb_stride;
  }
  S.partial_words = off;
  // virtual block ranges, then XCD-aware physical mapping: consecutive
  // virtual blocks go to the same XCD (workgroups are dealt round-robin
  // over the 8 XCDs), so a row slice stays in one XCD's L2.
  std::vector<int64_t> vbeg(B, 0), vend(B, 0);
  {
    size_t s = 0;
    for (int v = 0; v < B; ++v) {
      vbeg[v] = (int64_t)s;
      while (s < S.segs.size() && seg_vb[s] == v) ++s;
      vend[v] = (int64_t)s;
    }
  }
  S.blk.assign(2 * (size_t)B, 0);
  const int X = 8;
  for (int b = 0; b < B; ++b) {
    const int v = (B % X == 0) ? (b % X) * (B / X) + b / X : b;
    S.blk[2 * b] = vbeg[v];
    S.blk[2 * b + 1] = vend[v];
  }
  // group tables
  S.grp_base.resize(fits.size() + 1);
  int64_t ng = 0;
  for (size_t fi = 0; fi < fits.size(); ++fi) {
    S.grp_base[fi] = ng;
    ng += (fits[fi]->p + t.F - 1) / t.F;
  }
  S.grp_base[fits.size()] = ng;
  std::vector<std::vector<int64_t>> lists(ng);
  for (size_t s = 0; s < S.segs.size(); ++s) {  // a fold segment serves every fold
    const Seg& sg = S.segs[s];
    for (int q = 0; q < sg.nfit; ++q)
      lists[S.grp_base[sg.fit + q] + sg.k0 / t.F].push_back((int64_t)s);
  }
  S.grp_ptr.assign(ng + 1, 0);
  for (int64_t g = 0; g < ng; ++g) {
    S.grp_ptr[g + 1] = S.grp_ptr[g] + (int64_t)lists[g].size();
    for (int64_t v : lists[g]) S.grp_seg.push_back(v);
  }
  // per learner: word offsets of its histogram in every segment slot of its
  // group, for each signal the fit can have
  for (size_t fi = 0; fi < fits.size(); ++fi) {
    const FitShape& sh = *fits[fi];
    for (int k = 0; k < sh.p; ++k) {
      const int64_t g = S.grp_base[fi] + k / t.F;
      const int64_t n = S.grp_ptr[g + 1] - S.grp_ptr[g];
      S.sel_begin.push_back((int64_t)S.sel_off.size());
      S.sel_n.push_back((int32_t)n);
      for (int sig = 0; sig < sh.nsig_max; ++sig)
        for (int64_t q = S.grp_ptr[g]; q < S.grp_ptr[g + 1]; ++q) {
          const Seg& sg = S.segs[S.grp_seg[q]];
          const int member = (int)fi - sg.fit;  // 0 unless a later fold
          S.sel_off.push_back(sg.slot + (int64_t)((member * sh.nsig_max + sig) * sg.nf + (k - sg.k0)) *
                                            sh.nb_stride);
        }
    }
  }
  int ns_max = 1;
  for (const FitShape* f : fits) ns_max = std::max(ns_max, f->nsig_max);
  S.lds = 4 * sizeof(long long);  // the largest segment's histograms
  for (const Seg& sg : S.segs) S.lds = std::max(S.lds, seg_lds_bytes(sg, *fits[sg.fit]));
  S.nsig_max = ns_max;
  S.unbinned = !fits.empty() && fits[0]->unbinned;
  for (const Seg& sg : S.segs) S.folds = S.folds || sg.nfit > 1;
  for (const FitShape* f : fits) S.copies = S.copies || (f->copies && !S.unbinned);
  return S;
}

// Every (fit, group) must be covered by its segments exactly once over
// [0, n_pad/8), slots must be disjoint and inside the partial buffer, and
// every block range must index existing segments.  Checked on the host
// before a schedule is uploaded.
bool schedule_is_valid(const Schedule& S, const std::vector<const FitShape*>& fits, const Tune& t,
                       std::string* why) {
  const int64_t nseg = (int64_t)S.segs.size();
  if ((int64_t)S.blk.size() != 2 * (int64_t)S.blocks) { *why = "block table size"; return false; }
  std::vector<int> seen(nseg, 0);
  for (int b = 0; b < S.blocks; ++b) {
    const int64_t a = S.blk[2 * b], e = S.blk[2 * b + 1];
    if (a < 0 || e < a || e > nseg) { *why = "block range"; return false; }
    for (int64_t s = a; s < e; ++s) seen[s] += 1;
  }
  for (int64_t s = 0; s < nseg; ++s)
    if (seen[s] != 1) { *why = "segment not owned by exactly one block"; return false; }
  // fold groups: a head with share = K followed by K - 1 folds of its shape
  std::vector<int> head(fits.size(), -1);
  for (size_t fi = 0; fi < fits.size(); ++fi) {
    const FitShape& sh = *fits[fi];
    if (sh.share < 0 || sh.share > kMaxFolds) { *why = "fold group size"; return false; }
    if (sh.share >= 1) {
      if (fi + sh.share > fits.size()) { *why = "fold group past the fit list"; return false; }
      for (int q = 0; q < sh.share; ++q) {
        const FitShape& m = *fits[fi + q];
        if ((q > 0 && m.share != 0) || m.n_pad != sh.n_pad || m.p != sh.p ||
            m.nb_stride != sh.nb_stride || m.nsig_max != sh.nsig_max || m.unbinned != sh.unbinned) {
          *why = "fold group members differ";
          return false;
        }
        head[fi + q] = (int)fi;
      }
    }
    if (head[fi] < 0) { *why = "fold without a group head"; return false; }
  }
  int64_t slot_end = 0;
  for (const Seg& sg : S.segs) {
    if (sg.fit < 0 || sg.fit >= (int)fits.size()) { *why = "segment fit"; return false; }
    const FitShape& sh = *fits[sg.fit];
    if (sh.share < 1 || sg.nfit != sh.share) { *why = "segment fold count"; return false; }
    if (sg.skip < -1 || sg.skip >= sg.nfit) { *why = "segment fold"; return false; }
    if (sg.skip >= 0) {  // every row it leaves out must belong to that fold
      int64_t r0, r1;
      unit_rows(sh, sg.u0, sg.u1, &r0, &r1);
      if (segment_fold(sh, r0, r1) != sg.skip) { *why = "segment rows outside its fold"; return false; }
    }
    if (sg.nf < 1 || sg.nf > t.F || sg.nf > t.fmax || sg.k0 < 0 || sg.k0 + sg.nf > sh.p ||
        sg.k0 % t.F != 0) { *why = "segment learners"; return false; }
    if (sg.u0 < 0 || sg.u1 <= sg.u0 || sg.u1 > sh.n_pad / 8) { *why = "segment rows"; return false; }
    if (sg.acc32 != 0) {
      bool ok = sg.acc32 == 1 && !sh.unbinned;
      for (int q = 0; ok && q < sg.nfit; ++q)
        ok = group_acc32(*fits[sg.fit + q], sg.k0, sg.nf, sg.u0, sg.u1, t.nt) == 1;
      if (!ok) {
        *why = "32-bit group";
        return false;
      }
    }
    if (sg.slot != slot_end) { *why = "slot order"; return false; }
    const int64_t words = (int64_t)sg.nfit * sh.nsig_max * sg.nf * sh.nb_stride;
    slot_end += words;
    if (seg_lds_bytes(sg, sh) > S.lds) { *why = "LDS size"; return false; }
  }
  if (slot_end != S.partial_words) { *why = "partial size"; return false; }
  for (int64_t o : S.sel_off)
    if (o < 0 || o % 4 != 0 || o + 4 > S.partial_words) { *why = "learner offset"; return false; }
  if (S.lds > (size_t)kHistMaxLds) { *why = "histogram LDS above its limit"; return false; }
  const int64_t ng = (int64_t)S.grp_ptr.size() - 1;
  for (size_t fi = 0; fi < fits.size(); ++fi) {
    const int groups = (fits[fi]->p + t.F - 1) / t.F;
    for (int g = 0; g < groups; ++g) {
      const int64_t gi = S.grp_base[fi] + g;
      if (gi >= ng) { *why = "group table"; return false; }
      std::vector<std::pair<int64_t, int64_t>> iv;
      for (int64_t q = S.grp_ptr[gi]; q < S.grp_ptr[gi + 1]; ++q) {
        const Seg& sg = S.segs[S.grp_seg[q]];
        if (sg.fit != head[fi] || sg.k0 != g * t.F) { *why = "group membership"; return false; }
        iv.push_back({sg.u0, sg.u1});
      }
      std::sort(iv.begin(), iv.end());
      int64_t pos = 0;
      for (auto& v : iv) {
        if (v.first != pos) { *why = "group rows not covered exactly once"; return false; }
        pos = v.second;
      }
      if (pos != fits[fi]->n_pad / 8) { *why = "group rows incomplete"; return false; }
    }
  }
  return true;
}

Layout make_layout(const FitShape& sh, const SchedCap& s) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    const size_t o = off;
    off += bytes;
    return o;
  };
  const size_t np = (size_t)sh.n_pad;
  const bool two = sh.nsig_max == 2;
  // mutable state first (contiguous, for checkpoints)
  L.state_begin = take(0);
  L.ctl = take(sizeof(Ctl));
  L.fg = take(np * 4);
  L.h = take(two ? np * 4 : 0);
  L.c = take(two ? np * 4 : 0);
  L.q = take((size_t)kNumSig * sh.p * 8);
  L.theta = take((size_t)kNumSig * sh.p * sh.d_max * 8);
  L.table = take((size_t)kNumSig * sh.p * sh.nb_max * 4);
  L.trk = take((size_t)sh.M * 4);
  L.trth = take((size_t)sh.M * sh.d_max * 8);
  L.trkc = take((size_t)sh.M * 4);
  L.trthc = take((size_t)sh.M * sh.d_max * 8);
  L.trrisk = take((size_t)(sh.M + 1) * 8);
  L.trval = take((size_t)(sh.M + 1) * 8);
  L.trgap = take((size_t)sh.M * 8);
  L.coef_f = take((size_t)sh.sum_d * 8);
  L.coef_h = take((size_t)sh.sum_d * 8);
  L.state_end = align_up(off, 256);
  // inputs and tables
  L.X = take(sh.external_x ? 0 : (size_t)sh.p * np * (sh.unbinned ? 4 : 2));
  L.X12 = take(sh.x12 && !sh.external_x ? (size_t)sh.p * np / 8 * 12 : 0);
  L.X10h = take(sh.x10_after_switch() ? (size_t)sh.p * np / 16 * 20 : 0);
  L.y = take(np * 4);
  L.r = take(np * 4);
  L.feat = take((size_t)sh.p * sizeof(FeatDev));
  L.bstart = take((size_t)sh.sum_nb * 4);
  L.bval = take((size_t)sh.sum_nb * kMaxBand * 8);
  L.jr = take((size_t)sh.sum_d * 2 * 4);
  for (int set = 0; set < 2; ++set) {
    L.ainv[set] = take((size_t)sh.sum_d2 * 8);
    L.gram[set] = take((size_t)sh.sum_d2 * 8);
  }
  L.riskpart = take((size_t)sh.n_row_blocks * 2 * 8);
  L.amaxpart = take((size_t)sh.n_row_blocks * 2 * 4);
  L.valpart = take((size_t)std::max(1, sh.n_val_blocks) * 8);
  L.fitdev = take(sizeof(FitDev));
  // solo schedule
  L.segs = take(s.segs * sizeof(Seg));
  L.blk = take(s.blk * 8);
  L.sel_off = take(s.sel_off * 8);
  L.partials = take((size_t)s.partial_words * 8);
  L.st_items = take((size_t)sh.n_row_blocks * sizeof(RowItem));
  L.sel_items = take((size_t)sh.p * sizeof(SelItem));
  L.val_items = take((size_t)std::max(1, sh.n_val_blocks) * sizeof(StateItem));
  L.total = align_up(off, 256);
  return L;
}

namespace {

void timer_reset(KernelTimer& t) {
  t.used = 0;
  t.total_ms = 0.0;
  t.launches = 0;
}

// Record a start or stop event when timing is on.
hipError_t timer_mark(KernelTimer& t, hipStream_t st) {
  if (t.used == t.ev.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    t.ev.push_back(e);
  }
  return hipEventRecord(t.ev[t.used++], st);
}

hipError_t timer_collect(KernelTimer& t) {
  for (size_t i = 0; i + 1 < t.used; i += 2) {
    hipError_t r = hipEventSynchronize(t.ev[i + 1]);
    if (r != hipSuccess) return r;
    float ms = 0.0f;
    r = hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]);
    if (r != hipSuccess) return r;
    t.total_ms += ms;
    t.launches += 1;
  }
  t.used = 0;
  return hipSuccess;
}

void timer_free(KernelTimer& t) {
  for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  t.ev.clear();
  t.used = 0;
}

// One iteration for a set of fits sharing a schedule.
int enqueue_iteration(hipStream_t st, const FitDev* d_fits, int nfits, const Schedule& S, const Tune& t,
                      const RowItem* d_st, int n_st, const SelItem* d_sel, int n_sel,
                      const StateItem* d_val, int n_val, int nb_max, int d_max, const Seg* d_segs,
                      const int64_t* d_blk, const int64_t* d_off, long long* d_part,
                      cwb_fit* timed) {
  // timed launches: every timing_period-th iteration of a timed fit
  int tm = timed ? timed->timing : 0;
  if (tm && (timed->timing_counter++ % timed->timing_period) != 0) tm = 0;
  if (tm & 2) HIP_TRY(timer_mark(timed->t_state, st));
  HIP_TRY(launch_state(st, d_fits, d_st, n_st, nb_max, 0, S.unbinned));
  if (tm & 2) HIP_TRY(timer_mark(timed->t_state, st));
  if (tm & 1) HIP_TRY(timer_mark(timed->t_hist, st));
  HIP_TRY(launch_hist(st, t.nt, t.fmax, S.nsig_max, S.unbinned, S.folds, S.copies, S.blocks, S.lds, d_fits, d_segs, d_blk, d_part));
  if (tm & 1) HIP_TRY(timer_mark(timed->t_hist, st));
  if (tm & 4) HIP_TRY(timer_mark(timed->t_select, st));
  HIP_TRY(launch_select(st, d_sel, n_sel, S.nsig_max, nb_max, d_max, d_part));
  if (tm & 4) HIP_TRY(timer_mark(timed->t_select, st));
  if (n_val > 0) {
    HIP_TRY(launch_valrisk(st, d_fits, d_val, n_val, nb_max));
    HIP_TRY(launch_valdecide(st, d_fits, nfits));
  }
  return CWB_OK;
}

template <typename T>
T* dptr(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

}  // namespace

int learners32(const Schedule& S) {
  int n = 0;
  for (size_t g = 0; g + 1 < S.grp_ptr.size(); ++g) {
    if (S.grp_ptr[g] == S.grp_ptr[g + 1]) continue;
    const Seg& sg = S.segs[(size_t)S.grp_seg[(size_t)S.grp_ptr[g]]];
    if (sg.acc32) n += sg.nf;
  }
  return n;
}

int row_chunks(int64_t total, int cus) {
  const int forced = env_int("CWB_ROW_CHUNKS", 0);  // testing: force a chunk count
  if (forced > 0) return std::min(forced, 16);
  const int64_t room = 8 * (int64_t)std::max(cus, 1);  // about 8 row blocks per CU at a time
  return (int)std::max<int64_t>(1, std::min<int64_t>(16, (total + room - 1) / room));
}

void append_row_items(std::vector<RowItem>* out, int fit, const FitDev& D, int n_row_blocks,
                      int chunks) {
  for (int b = 0; b < n_row_blocks; b += chunks)
    out->push_back(make_row_item(fit, b, D, std::min(chunks, n_row_blocks - b)));
}

RowItem make_row_item(int fit, int blk, const FitDev& D, int chunks) {
  RowItem it;
  std::memset(&it, 0, sizeof(it));
  it.chunks = chunks;
  it.ctl = D.ctl;
  it.q = D.q;
  it.X = D.X;
  it.y = D.y;
  it.fg = D.fg;
  it.h = D.h;
  it.c = D.c;
  it.r = D.r;
  it.table = D.table;
  it.risk_part = D.risk_part + 2 * (int64_t)blk;
  it.amax_part = D.amax_part + 2 * (int64_t)blk;
  it.n = D.n;
  it.n_pad = D.n_pad;
  it.n_train = D.n_train;
  it.fold = D.fold;
  it.fold_k = D.fold_k;
  it.base = (int64_t)blk * kStateRows;
  it.nu = D.nu;
  it.gamma = D.gamma;
  it.p = D.p;
  it.nb_max = D.nb_max;
  it.loss = D.loss;
  it.variant = D.variant;
  it.M = D.M;
  it.two = D.nsig_max == 2 ? 1 : 0;
  it.blk = blk;
  it.fit = fit;
  it.unbinned = D.unbinned;
  return it;
}

SelItem make_sel_item(int fit, int k, const FeatDev& fd, const FitDev& D, const Schedule& S,
                      const int64_t* d_sel_off, size_t idx) {
  SelItem it;
  std::memset(&it, 0, sizeof(it));
  it.ctl = D.ctl;
  it.amax_part = D.amax_part;
  for (int set = 0; set < 2; ++set) {
    it.ainv[set] = D.ainv[set] + fd.mat_off;
    it.gram[set] = D.gram[set] + fd.mat_off;
  }
  it.bval = D.bval + fd.bin_off * kMaxBand;
  it.bstart = D.bstart + fd.bin_off;
  it.jr = D.jr + 2 * (int64_t)fd.coef_off;
  it.offs = d_sel_off + S.sel_begin[idx];
  for (int i = 0; i < kInlineOffs && i < S.sel_n[idx]; ++i) {
    it.off0[i] = S.sel_off[S.sel_begin[idx] + i];
    if (D.nsig_max == 2) it.off1[i] = S.sel_off[S.sel_begin[idx] + S.sel_n[idx] + i];
  }
  it.q = D.q + k;
  it.theta = D.theta + (int64_t)k * D.d_max;
  it.table = D.table + (int64_t)k * D.nb_max;
  it.tr_risk = D.tr_risk;
  it.tr_val = D.tr_val;
  it.risk_part = D.risk_part;
  it.n = D.n;
  it.n_train = D.n_train;
  it.n_scan = D.n_scan;
  it.k = k;
  it.nb = fd.nb;
  it.band = fd.band;
  it.d = fd.d;
  it.n_off = S.sel_n[idx];
  it.d_max = D.d_max;
  it.nb_max = D.nb_max;
  it.p = D.p;
  it.M = D.M;
  it.variant = D.variant;
  it.n_row_blocks = D.n_row_blocks;
  it.fit = fit;
  it.kind = fd.kind;
  it.acc32_bits = D.acc32_bits;
  return it;
}

int finalize_fit(cwb_fit* f) {
  HIP_TRY(hipSetDevice(f->device));
  RowItem* d_st = dptr<RowItem>(f->ws, f->lay.st_items);
  HIP_TRY(launch_state(f->stream, f->d_fit, d_st, f->n_st, f->shape.nb_max, 1, f->shape.unbinned));
  HIP_TRY(launch_finalize(f->stream, f->d_fit, 1));
  return CWB_OK;
}

int plan_candidates(const std::vector<const FitShape*>& shapes, bool all, std::vector<Tune>* cands,
                    SchedCap* cap, Schedule* first) {
  int nb = 1, ns = 1, pmax = 1;
  int64_t work = 0;  // 8-row units times learners over the fits
  for (const FitShape* sh : shapes) {
    nb = std::max(nb, sh->nb_stride * std::max(1, sh->share));  // a fold group's histograms
    ns = std::max(ns, sh->nsig_max);
    pmax = std::max(pmax, sh->p);
    work += sh->n_pad / 8 * sh->p;
    if (sh->unbinned != shapes[0]->unbinned)
      return set_error(CWB_E_UNSUPPORTED, "binned and unbinned fits cannot share a batch");
  }
  *cands = tune_candidates(nb, ns, pmax, shapes[0]->unbinned, all, work);
  *cap = SchedCap();
  for (size_t i = 0; i < cands->size(); ++i) {
    Schedule S = build_schedule(shapes, (*cands)[i]);
    std::string why;
    if (!schedule_is_valid(S, shapes, (*cands)[i], &why))
      return set_error(CWB_E_INVALID_ARG, "internal schedule error: " + why);
    cap->add(S);
    if (i == 0 && first) *first = std::move(S);
  }
  return CWB_OK;
}

namespace {

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

int autotune_hist(hipStream_t st, const FitDev* d_fits, const std::vector<const FitShape*>& shapes,
                  const std::vector<Tune>& cands, const SchedCap& cap, Seg* d_segs, int64_t* d_blk,
                  long long* d_part, int* best, double* best_us, const TuneRowPass* row) {
  *best = 0;
  *best_us = 0.0;
  if (cands.size() < 2) return CWB_OK;
  constexpr int kWarm = 2, kTimed = 5;
  EventPair ev;
  HIP_TRY(hipEventCreate(&ev.a));
  HIP_TRY(hipEventCreate(&ev.b));
  // the row pass before each histogram pass (a fit's first iteration: it
  // rewrites the same residuals), and its own time to take off
  auto row_pass = [&]() -> hipError_t {
    return row ? launch_state(st, d_fits, row->items, row->n, row->nb_max, 0, row->unbinned)
               : hipSuccess;
  };
  double row_us = 0.0;
  if (row) {
    for (int w = 0; w < kWarm; ++w) HIP_TRY(row_pass());
    HIP_TRY(hipEventRecord(ev.a, st));
    for (int r = 0; r < kTimed; ++r) HIP_TRY(row_pass());
    HIP_TRY(hipEventRecord(ev.b, st));
    HIP_TRY(hipEventSynchronize(ev.b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
    row_us = (double)ms * 1e3 / kTimed;
  }
  double best_t = 0.0, default_t = 0.0;
  for (size_t i = 0; i < cands.size(); ++i) {
    const Tune& t = cands[i];
    Schedule S = build_schedule(shapes, t);
    if (S.segs.size() > cap.segs || S.blk.size() > cap.blk || S.partial_words > cap.partial_words)
      continue;
    HIP_TRY(hipMemcpyAsync(d_segs, S.segs.data(), S.segs.size() * sizeof(Seg), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_blk, S.blk.data(), S.blk.size() * 8, hipMemcpyHostToDevice, st));
    for (int w = 0; w < kWarm; ++w) {
      HIP_TRY(row_pass());
      HIP_TRY(launch_hist(st, t.nt, t.fmax, S.nsig_max, S.unbinned, S.folds, S.copies, S.blocks, S.lds, d_fits, d_segs, d_blk, d_part));
    }
    HIP_TRY(hipEventRecord(ev.a, st));
    for (int r = 0; r < kTimed; ++r) {
      HIP_TRY(row_pass());
      HIP_TRY(launch_hist(st, t.nt, t.fmax, S.nsig_max, S.unbinned, S.folds, S.copies, S.blocks, S.lds, d_fits, d_segs, d_blk, d_part));
    }
    HIP_TRY(hipEventRecord(ev.b, st));
    HIP_TRY(hipEventSynchronize(ev.b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
    const double us = std::max(0.0, (double)ms * 1e3 / kTimed - row_us);
    if (i == 0) default_t = us;
    if (*best_us == 0.0 || us < best_t) {
      best_t = us;
      *best = (int)i;
      *best_us = us;
    }
  }
  // keep the default shape unless another is clearly faster: shapes within
  // timing noise would otherwise change from run to run
  if (*best != 0 && default_t > 0.0 && best_t > 0.98 * default_t) {
    *best = 0;
    *best_us = default_t;
  }
  return CWB_OK;
}

int fit_footprint(const FitShape& sh, size_t* bytes, bool all) {
  std::vector<Tune> cands;
  SchedCap cap;
  int rc = plan_candidates({&sh}, all, &cands, &cap, nullptr);
  if (rc) return rc;
  *bytes = make_layout(sh, cap).total;
  return CWB_OK;
}

// Upload a schedule and the select work list that indexes its partials.
static int fit_install(cwb_fit* f, const Tune& t, Schedule&& S) {
  const Layout& L = f->lay;
  char* ws = f->ws;
  hipStream_t st = f->stream;
  std::vector<SelItem> sel_items(f->shape.p);
  for (int k = 0; k < f->shape.p; ++k)
    sel_items[k] = make_sel_item(0, k, f->feat[k], f->dev, S, dptr<int64_t>(ws, L.sel_off), k);
  HIP_TRY(hipMemcpyAsync(ws + L.segs, S.segs.data(), S.segs.size() * sizeof(Seg), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.blk, S.blk.data(), S.blk.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.sel_off, S.sel_off.data(), S.sel_off.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.sel_items, sel_items.data(), sel_items.size() * sizeof(SelItem),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  f->tune = t;
  f->sched = std::move(S);
  return CWB_OK;
}

namespace {

// Host view of the order-preserving integers of the device range pass.
double from_ordered(unsigned long long o) {
  const unsigned long long b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
  double v;
  std::memcpy(&v, &b, 8);
  return v == 0.0 ? 0.0 : v;
}

}  // namespace

// Binning pass on the device (binning.hip) for a fit whose host setup ran
// its first phase only: each column of x is copied into the workspace (the
// label and residual vectors, not yet written, hold one FP64 column), its
// range found, and its rows binned straight into X with the bin counts.
// The ranges, counts and error flags come back to the host, which builds
// the learner tables (finish_host_fit).  Other scratch used here, all
// written later by the upload: the state vector f (row order), theta (the
// ranges), q (the flags), the partials (the counts).
int device_binning(const cwb_problem* pr, const FitShape& sh, HostFit& hf, const Layout& L,
                   char* ws, hipStream_t st) {
  const int64_t n = sh.n, np = sh.n_pad;
  const int p = sh.p;
  if (sh.unbinned || n >= (int64_t)INT32_MAX)
    return set_error(CWB_E_UNSUPPORTED, "device setup covers binned fits with n < 2^31");
  const int64_t cstride = 2 * (int64_t)sh.nb_stride;  // per feature: training | all rows
  if (L.r != L.y + (size_t)np * 4 || L.st_items - L.partials < (size_t)p * cstride * 4 ||
      L.theta - L.q < (size_t)p * 4 || L.table - L.theta < (size_t)p * 16)
    return set_error(CWB_E_INVALID_ARG, "internal: scratch regions of the device setup");
  double* stage = dptr<double>(ws, L.y);
  const bool permuted = hf.n_train < n;
  int32_t* d_perm = permuted ? dptr<int32_t>(ws, L.fg) : nullptr;
  unsigned long long* d_mm = dptr<unsigned long long>(ws, L.theta);
  int* d_flag = dptr<int>(ws, L.q);
  uint32_t* d_cnt = dptr<uint32_t>(ws, L.partials);
  uint16_t* d_X = dptr<uint16_t>(ws, L.X);
  std::vector<unsigned long long> mm((size_t)2 * p);
  for (int j = 0; j < p; ++j) {
    mm[2 * j] = ~0ull;
    mm[2 * j + 1] = 0ull;
  }
  std::vector<int32_t> perm32;
  HIP_TRY(hipMemcpyAsync(d_mm, mm.data(), mm.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(d_flag, 0, (size_t)p * 4, st));
  HIP_TRY(hipMemsetAsync(d_cnt, 0, (size_t)p * cstride * 4, st));
  if (permuted) {
    perm32.assign(hf.perm.begin(), hf.perm.end());
    HIP_TRY(hipMemcpyAsync(d_perm, perm32.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
  }
  const int64_t ldx = pr->ldx ? pr->ldx : n;
  for (int j = 0; j < p; ++j) {
    const bool cat = pr->specs[j].kind != CWB_PSPLINE;
    HIP_TRY(hipMemcpyAsync(stage, pr->x + (size_t)j * ldx, (size_t)n * 8, hipMemcpyHostToDevice, st));
    if (!cat) HIP_TRY(launch_range(st, stage, n, d_mm + 2 * j, d_flag + j));
    HIP_TRY(launch_bin(st, stage, d_perm, n, np, hf.n_train, cat ? 1 : 0, hf.L[j].nb, d_mm + 2 * j,
                       d_X + (size_t)j * np, d_cnt + (size_t)j * cstride, cstride / 2, d_flag + j));
  }
  std::vector<int> flag(p);
  std::vector<uint32_t> cnt((size_t)p * cstride);
  HIP_TRY(hipMemcpyAsync(mm.data(), d_mm, mm.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(flag.data(), d_flag, flag.size() * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(cnt.data(), d_cnt, cnt.size() * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<double> xr((size_t)2 * p, 0.0);
  for (int j = 0; j < p; ++j) {
    if (flag[j] & 1) return set_error(CWB_E_INVALID_ARG, "non-finite x");
    if (flag[j] & 2) return set_error(CWB_E_INVALID_ARG, "level code out of range in feature " + std::to_string(j));
    if (pr->specs[j].kind != CWB_PSPLINE) continue;
    xr[2 * j] = from_ordered(mm[2 * j]);
    xr[2 * j + 1] = from_ordered(mm[2 * j + 1]);
    if (!(xr[2 * j + 1] > xr[2 * j])) return set_error(CWB_E_INVALID_ARG, "constant feature " + std::to_string(j));
  }
  std::string err;
  const int rc = finish_host_fit(pr, &hf, xr.data(), cnt.data(), cstride, &err,
                                 env_int("CWB_DEVICE_SOLVES", 1) != 0);
  if (rc) return set_error(rc, err);
  return CWB_OK;
}

// The device setup pass's learner solves (after device_binning): Gram
// matrices from the bin counts still in the partials region, lambda and the
// inverses, for every learner left to the device (solve_on_device), written
// into the fit's tables.  The job list borrows the select work-list region
// and the status and lambda outputs the criterion and theta regions, which
// are cleared again.
int device_solves(const cwb_problem* pr, const FitShape& sh, const HostFit& hf,
                  const std::vector<FeatDev>& feat, const FitDev& D, const Layout& L, char* ws,
                  hipStream_t st) {
  const int64_t cstride = 2 * (int64_t)sh.nb_stride;
  const uint32_t* d_cnt = dptr<uint32_t>(ws, L.partials);
  std::vector<SolveJob> jobs;
  std::vector<int> job_feat;
  int dmax = 0;
  for (int j = 0; j < sh.p; ++j) {
    const HostLearner& hl = hf.L[j];
    if (!hl.solve_on_device) continue;
    const cwb_learner_spec& s = pr->specs[j];
    const FeatDev& fd = feat[j];
    for (int set = 0; set < 2; ++set) {
      SolveJob jb;
      std::memset(&jb, 0, sizeof(jb));
      jb.bstart = D.bstart + fd.bin_off;
      jb.bval = D.bval + fd.bin_off * kMaxBand;
      jb.cnt = d_cnt + (size_t)j * cstride + (set ? cstride / 2 : 0);
      jb.gram = const_cast<double*>(D.gram[set]) + fd.mat_off;
      jb.ainv = const_cast<double*>(D.ainv[set]) + fd.mat_off;
      jb.df = s.df;
      jb.lambda = s.lambda;
      jb.kind = s.kind;
      jb.d = hl.d;
      jb.nb = hl.nb;
      jb.band = hl.band;
      jb.pen_order = s.penalty_order;
      jobs.push_back(jb);
      job_feat.push_back(j);
      dmax = std::max(dmax, hl.d);
    }
  }
  if (jobs.empty()) return CWB_OK;
  static_assert(2 * sizeof(SolveJob) <= sizeof(SelItem), "solve jobs fit the select work list");
  if (jobs.size() * sizeof(SolveJob) > (size_t)sh.p * sizeof(SelItem) ||
      jobs.size() * sizeof(int) > (size_t)kNumSig * sh.p * 8 ||
      jobs.size() * sizeof(double) > (size_t)kNumSig * sh.p * sh.d_max * 8)
    return set_error(CWB_E_INVALID_ARG, "internal: device solve scratch");
  SolveJob* d_jobs = dptr<SolveJob>(ws, L.sel_items);
  int* d_status = dptr<int>(ws, L.q);
  double* d_lam = dptr<double>(ws, L.theta);
  HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(SolveJob), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_solve(st, d_jobs, (int)jobs.size(), dmax, d_status, d_lam));
  std::vector<int> status(jobs.size());
  HIP_TRY(hipMemcpyAsync(status.data(), d_status, status.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemsetAsync(d_status, 0, jobs.size() * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(d_lam, 0, jobs.size() * sizeof(double), st));
  for (size_t i = 0; i < jobs.size(); ++i) {
    if (status[i] == 0) continue;
    const std::string what = status[i] == -1 ? "df target not reachable for this basis and penalty"
                                             : "penalised Gram matrix is singular or degenerate";
    return set_error(status[i] == -1 ? CWB_E_INVALID_ARG : CWB_E_NUMERIC,
                     what + " (feature " + std::to_string(job_feat[i]) + ")");
  }
  return CWB_OK;
}

int fit_upload(const FitShape& sh, HostFit& hf, void* dev_ws, size_t ws_bytes, hipStream_t stream,
               bool autotune, cwb_fit** out, const cwb_problem* bin_on_device, const FoldSpec* fold,
               long long* scratch, size_t scratch_bytes) {
  if (fold && (!sh.external_x || sh.n_scan != sh.n || bin_on_device))
    return set_error(CWB_E_INVALID_ARG, "internal: fold fit shape");
  if (scratch && (autotune || bin_on_device || fold))
    return set_error(CWB_E_INVALID_ARG, "internal: scratch partials with tuning, device setup or folds");
  *out = nullptr;
  std::unique_ptr<cwb_fit> f(new cwb_fit());
  f->stream = stream;
  f->shape = sh;
  std::vector<Tune> cands;
  SchedCap cap;
  {
    int rc = plan_candidates({&f->shape}, autotune, &cands, &cap, &f->sched);
    if (rc) return rc;
  }
  f->tune = cands[0];
  f->n_cands = (int)cands.size();
  if (scratch) {
    const size_t need = (size_t)cap.partial_words * sizeof(long long);
    if (need > scratch_bytes)
      return set_error(CWB_E_NO_MEMORY, "histogram partials need " + std::to_string(need) +
                                            " bytes, above the static scratch of " +
                                            std::to_string(scratch_bytes) + " bytes");
    SchedCap in_ws = cap;
    in_ws.partial_words = 0;  // the partials live in the scratch array
    f->lay = make_layout(sh, in_ws);
  } else {
    f->lay = make_layout(sh, cap);
  }
  if (ws_bytes < f->lay.total)
    return set_error(CWB_E_NO_MEMORY, "workspace too small: need " + std::to_string(f->lay.total) +
                                          " bytes, got " + std::to_string(ws_bytes));
  HIP_TRY(hipGetDevice(&f->device));
  f->ws = reinterpret_cast<char*>(dev_ws);
  f->ws_bytes = ws_bytes;
  f->partials = scratch ? scratch : dptr<long long>(f->ws, f->lay.partials);
  if (bin_on_device) {
    const int rc = device_binning(bin_on_device, sh, hf, f->lay, f->ws, f->stream);
    if (rc) return rc;
  }
  f->f0 = hf.f0;
  f->perm = std::move(hf.perm);
  // 32-bit histogram accumulation, now that the bins are counted: a binned
  // learner without LDS copies whose fullest bin holds fewer than
  // 2^kAcc32MaxBits rows (CWB_ACC32=0 keeps int64 sums throughout)
  if (!sh.unbinned && env_int("CWB_ACC32", 1) != 0) {
    std::vector<uint8_t> acc(sh.p, 0), copies(sh.p, 0);
    int bits = 0;
    for (int j = 0; j < sh.p; ++j) {
      const HostLearner& hl = hf.L[j];
      int N = 0;
      for (int64_t v = hl.cnt_max; v > 0; v >>= 1) ++N;  // cnt_max < 2^N
      int stride = 0;
      const int cm = hl.nb > 0 ? copy_mask(hl.nb, sh.nb_stride, &stride) : 0;
      if (hl.nb > 0 && cm > 0) {
        copies[j] = (uint8_t)(cm + 1);  // 32-bit words where its segments allow
      } else if (hl.nb > 0 && hl.cnt_max > 0 && N <= kAcc32MaxBits) {
        acc[j] = 1;
        bits = std::max(bits, N);
      }
    }
    if (bits > 0) {
      f->shape.acc32 = std::move(acc);
      f->shape.acc32_copies = std::move(copies);
      f->shape.acc32_bits = bits;
      f->sched = build_schedule({&f->shape}, f->tune);
      std::string why;
      if (!schedule_is_valid(f->sched, {&f->shape}, f->tune, &why))
        return set_error(CWB_E_INVALID_ARG, "internal schedule error: " + why);
    }
  }
  const Layout& L = f->lay;
  char* ws = f->ws;
  hipStream_t st = f->stream;

  // per-learner tables, concatenated
  std::vector<FeatDev> feat(sh.p);
  std::vector<int32_t> bstart;
  std::vector<double> bval;
  std::vector<int32_t> jr;
  std::vector<double> ainv[2], gram[2];
  bstart.reserve(sh.sum_nb);
  bval.reserve(sh.sum_nb * kMaxBand);
  int64_t bin_off = 0, mat_off = 0;
  int coef_off = 0;
  f->d.resize(sh.p);
  for (int j = 0; j < sh.p; ++j) {
    const HostLearner& hl = hf.L[j];
    FeatDev& fd = feat[j];
    fd.nb = hl.nb;
    fd.band = hl.band;
    fd.d = hl.d;
    fd.coef_off = coef_off;
    fd.bin_off = bin_off;
    fd.mat_off = mat_off;
    fd.xmin = hl.xmin;
    fd.xmax = hl.xmax;
    fd.kind = hl.kind;
    fd.degree = hl.degree;
    fd.n_int = hl.n_int;
    fd.pad = 0;
    f->d[j] = hl.d;
    bstart.insert(bstart.end(), hl.bstart.begin(), hl.bstart.end());
    bval.insert(bval.end(), hl.bval.begin(), hl.bval.end());
    jr.insert(jr.end(), hl.jr.begin(), hl.jr.end());
    for (int set = 0; set < 2; ++set) {
      ainv[set].insert(ainv[set].end(), hl.ainv[set].begin(), hl.ainv[set].end());
      gram[set].insert(gram[set].end(), hl.gram[set].begin(), hl.gram[set].end());
    }
    bin_off += hl.nb;
    mat_off += (int64_t)hl.d * hl.d;
    coef_off += hl.d;
  }
  if (bin_off != sh.sum_nb || coef_off != sh.sum_d)
    return set_error(CWB_E_INVALID_ARG, "learner sizes disagree with the specification");

  FitDev& D = f->dev;
  std::memset(&D, 0, sizeof(D));
  D.n = sh.n;
  D.n_pad = sh.n_pad;
  D.n_train = sh.n_train;
  D.n_scan = sh.n_scan;
  D.fold = nullptr;
  D.fold_k = -1;
  D.p = sh.p;
  D.nb_max = sh.nb_max;
  D.d_max = sh.d_max;
  D.sum_d = sh.sum_d;
  D.loss = hf.loss;
  D.variant = hf.variant;
  D.M = hf.M;
  D.patience = hf.patience;
  D.nu = hf.nu;
  D.gamma = hf.gamma;
  D.n_row_blocks = sh.n_row_blocks;
  D.n_val_blocks = sh.n_val_blocks;
  D.nsig_max = sh.nsig_max;
  D.nb_stride = sh.nb_stride;
  D.unbinned = sh.unbinned ? 1 : 0;
  D.acc32_bits = f->shape.acc32_bits;
  if (sh.unbinned != hf.unbinned)
    return set_error(CWB_E_INVALID_ARG, "learner kinds disagree with the specification");
  D.X = fold ? fold->X : dptr<uint16_t>(ws, L.X);
  // the packed copy serves the 32-bit histogram groups only
  const bool pack12 = sh.x12 && !fold && !sh.external_x && f->shape.acc32_bits > 0 &&
                      env_int("CWB_X12", 1) != 0;
  D.X12 = pack12 ? dptr<uint32_t>(ws, L.X12) : nullptr;
  // 10 bits per index for a one-signal fit whose indices are all below
  // 1,024 (CWB_X10=0 keeps 12): at the headline shape 84.6 us per iteration
  // against 86.2 with the 12-bit copy.  With two signals the 10-bit
  // unpacking's extra work outweighed the saved bytes in most tiles.
  D.xbits = !pack12 ? 0
            : (sh.nb_max <= 1024 && sh.nsig_max == 1 && env_int("CWB_X10", 1) != 0) ? 10 : 12;
  // HCWB: its passes after the switch have one signal and read a 10-bit copy
  // of their own (at n = 2e6, p = 160 the CWB phase's pass is HBM-bound)
  D.X10h = (pack12 && D.xbits == 12 && sh.x10_after_switch() && env_int("CWB_X10", 1) != 0)
               ? dptr<uint32_t>(ws, L.X10h)
               : nullptr;
  if (fold) {
    D.fold = fold->fold;
    D.fold_k = fold->k;
  }
  D.y = dptr<float>(ws, L.y);
  D.fg = dptr<float>(ws, L.fg);
  D.h = sh.nsig_max == 2 ? dptr<float>(ws, L.h) : nullptr;
  D.c = sh.nsig_max == 2 ? dptr<float>(ws, L.c) : nullptr;
  D.r = dptr<float>(ws, L.r);
  D.feat = dptr<FeatDev>(ws, L.feat);
  D.bstart = dptr<int32_t>(ws, L.bstart);
  D.bval = dptr<double>(ws, L.bval);
  D.jr = dptr<int32_t>(ws, L.jr);
  for (int set = 0; set < 2; ++set) {
    D.ainv[set] = dptr<double>(ws, L.ainv[set]);
    D.gram[set] = dptr<double>(ws, L.gram[set]);
  }
  D.q = dptr<double>(ws, L.q);
  D.theta = dptr<double>(ws, L.theta);
  D.table = dptr<float>(ws, L.table);
  D.tr_k = dptr<int32_t>(ws, L.trk);
  D.tr_theta = dptr<double>(ws, L.trth);
  D.tr_kcor = dptr<int32_t>(ws, L.trkc);
  D.tr_thetacor = dptr<double>(ws, L.trthc);
  D.tr_risk = dptr<double>(ws, L.trrisk);
  D.tr_val = dptr<double>(ws, L.trval);
  D.tr_gap = dptr<double>(ws, L.trgap);
  D.coef_f = dptr<double>(ws, L.coef_f);
  D.coef_h = dptr<double>(ws, L.coef_h);
  D.risk_part = dptr<double>(ws, L.riskpart);
  D.amax_part = dptr<float>(ws, L.amaxpart);
  D.val_part = dptr<double>(ws, L.valpart);
  D.ctl = dptr<Ctl>(ws, L.ctl);
  f->d_fit = dptr<FitDev>(ws, L.fitdev);

  Ctl ctl;
  std::memset(&ctl, 0, sizeof(ctl));
  ctl.switch_iter = -1;
  if (hf.variant == CWB_HCWB && hf.patience == 0) {
    ctl.switched = 1;
    ctl.switch_iter = 1;
  }

  // state and inputs
  HIP_TRY(hipSetDevice(f->device));
  HIP_TRY(hipMemsetAsync(ws + L.state_begin, 0, L.state_end - L.state_begin, st));
  HIP_TRY(hipMemcpyAsync(ws + L.ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, st));
  std::vector<float> init((size_t)sh.n_pad, 0.0f);
  std::fill(init.begin(), init.begin() + sh.n, (float)hf.f0);
  HIP_TRY(hipMemcpyAsync(ws + L.fg, init.data(), init.size() * 4, hipMemcpyHostToDevice, st));
  if (sh.nsig_max == 2)
    HIP_TRY(hipMemcpyAsync(ws + L.h, init.data(), init.size() * 4, hipMemcpyHostToDevice, st));
  if (sh.unbinned)
    HIP_TRY(hipMemcpyAsync(ws + L.X, hf.XU.data(), hf.XU.size() * 4, hipMemcpyHostToDevice, st));
  else if (!bin_on_device && !fold)  // else X is in place already (device pass, shared folds)
    HIP_TRY(hipMemcpyAsync(ws + L.X, hf.X.data(), hf.X.size() * 2, hipMemcpyHostToDevice, st));
  if (D.xbits == 10)
    HIP_TRY(launch_pack10(st, dptr<uint16_t>(ws, L.X), (int64_t)sh.p * sh.n_pad / 16,
                          dptr<uint32_t>(ws, L.X12)));
  else if (D.xbits == 12)
    HIP_TRY(launch_pack12(st, dptr<uint16_t>(ws, L.X), (int64_t)sh.p * sh.n_pad / 8,
                          dptr<uint32_t>(ws, L.X12)));
  if (D.X10h)
    HIP_TRY(launch_pack10(st, dptr<uint16_t>(ws, L.X), (int64_t)sh.p * sh.n_pad / 16,
                          dptr<uint32_t>(ws, L.X10h)));
  HIP_TRY(hipMemcpyAsync(ws + L.y, hf.y.data(), hf.y.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(ws + L.r, 0, (size_t)sh.n_pad * 4, st));
  HIP_TRY(hipMemcpyAsync(ws + L.feat, feat.data(), feat.size() * sizeof(FeatDev), hipMemcpyHostToDevice, st));
  f->feat = feat;
  HIP_TRY(hipMemcpyAsync(ws + L.bstart, bstart.data(), bstart.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.bval, bval.data(), bval.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.jr, jr.data(), jr.size() * 4, hipMemcpyHostToDevice, st));
  for (int set = 0; set < 2; ++set) {
    HIP_TRY(hipMemcpyAsync(ws + L.ainv[set], ainv[set].data(), ainv[set].size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ws + L.gram[set], gram[set].data(), gram[set].size() * 8, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(ws + L.fitdev, &D, sizeof(D), hipMemcpyHostToDevice, st));
  if (bin_on_device) {  // the learners' solves left to the device
    const int rc = device_solves(bin_on_device, sh, hf, feat, D, L, ws, st);
    if (rc) return rc;
  }

  // solo schedule and work lists
  const Schedule& S = f->sched;
  HIP_TRY(hipMemcpyAsync(ws + L.segs, S.segs.data(), S.segs.size() * sizeof(Seg), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.blk, S.blk.data(), S.blk.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.sel_off, S.sel_off.data(), S.sel_off.size() * 8, hipMemcpyHostToDevice, st));
  std::vector<RowItem> st_items;
  {
    int dev = 0;
    (void)hipGetDevice(&dev);
    append_row_items(&st_items, 0, D, sh.n_row_blocks, row_chunks(sh.n_row_blocks, device_cus(dev)));
  }
  std::vector<SelItem> sel_items(sh.p);
  for (int k = 0; k < sh.p; ++k)
    sel_items[k] = make_sel_item(0, k, feat[k], D, S, dptr<int64_t>(ws, L.sel_off), k);
  std::vector<StateItem> val_items(std::max(1, sh.n_val_blocks));
  for (int b = 0; b < sh.n_val_blocks; ++b) val_items[b] = {0, b};
  f->n_st = (int)st_items.size();
  f->n_sel = sh.p;
  f->n_val = sh.n_val_blocks;
  HIP_TRY(hipMemcpyAsync(ws + L.st_items, st_items.data(), st_items.size() * sizeof(RowItem), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.sel_items, sel_items.data(), sel_items.size() * sizeof(SelItem), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L.val_items, val_items.data(), val_items.size() * sizeof(StateItem), hipMemcpyHostToDevice, st));
  // HCWB: validation risk of f^[0]
  if (f->n_val > 0 && !ctl.switched) {
    HIP_TRY(launch_valrisk(st, f->d_fit, dptr<StateItem>(ws, L.val_items), f->n_val, sh.nb_max));
    HIP_TRY(launch_valdecide(st, f->d_fit, 1));
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (cands.size() > 1) {
    int best = 0;
    // no selection is made yet, so the row pass only recomputes r^[0]
    TuneRowPass row;
    row.items = dptr<RowItem>(ws, L.st_items);
    row.n = f->n_st;
    row.nb_max = sh.nb_max;
    row.unbinned = sh.unbinned;
    int rc = autotune_hist(st, f->d_fit, {&f->shape}, cands, cap, dptr<Seg>(ws, L.segs),
                           dptr<int64_t>(ws, L.blk), f->partials, &best, &f->tuned_us, &row);
    if (rc) return rc;
    Schedule S = build_schedule({&f->shape}, cands[best]);
    rc = fit_install(f.get(), cands[best], std::move(S));
    if (rc) return rc;
  }
  *out = f.release();
  return CWB_OK;
}

int fit_create_with_scratch(const cwb_problem* pr, void* dev_ws, size_t ws_bytes, void* stream,
                            cwb_fit** out, long long* scratch, size_t scratch_bytes) {
  try {
    if (!out) return set_error(CWB_E_INVALID_ARG, "null output handle");
    *out = nullptr;
    if (!dev_ws) return set_error(CWB_E_INVALID_ARG, "null workspace");
    if (reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0)
      return set_error(CWB_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if (!scratch) return set_error(CWB_E_INVALID_ARG, "internal: no scratch array");
    std::string err;
    FitShape sh;
    int rc = shape_from_problem(pr, &sh, &err);
    if (rc) return set_error(rc, err);
    if (pr->setup < CWB_SETUP_AUTO || pr->setup > CWB_SETUP_DEVICE)
      return set_error(CWB_E_INVALID_ARG, "unknown setup mode");
    if (pr->setup == CWB_SETUP_DEVICE)
      return set_error(CWB_E_UNSUPPORTED, "the no-allocation fit runs its setup on the host");
    HostFit hf;
    rc = build_host_fit(pr, &hf, &err);
    if (rc) return set_error(rc, err);
    return fit_upload(sh, hf, dev_ws, ws_bytes, reinterpret_cast<hipStream_t>(stream), false, out,
                      nullptr, nullptr, scratch, scratch_bytes);
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(CWB_E_INVALID_ARG, e.what());
  } catch (...) {
    return set_error(CWB_E_INVALID_ARG, "unexpected error");
  }
}

}  // namespace cwb

using namespace cwb;

extern "C" {

int cwb_version(int* major, int* minor) {
  if (major) *major = CWB_VERSION_MAJOR;
  if (minor) *minor = CWB_VERSION_MINOR;
  return CWB_OK;
}

const char* cwb_last_error(void) { return g_err.c_str(); }

int cwb_bin_feature(const double* x, int64_t n, int32_t n_bins, uint16_t* ind_out, double* z_out) {
  try {
    std::string err;
    const int rc = bin_one_feature(x, n, n_bins, ind_out, z_out, &err);
    return rc ? set_error(rc, err) : CWB_OK;
  } catch (...) {
    return set_error(CWB_E_INVALID_ARG, "unexpected error");
  }
}

int cwb_lambda_for_df(int32_t d, const double* G, const double* D, double df, double* lambda) {
  try {
    if (!G || !D || !lambda) return set_error(CWB_E_INVALID_ARG, "null pointer");
    if (d < 1 || d > kMaxD) return set_error(CWB_E_INVALID_ARG, "matrix size must be 1..64");
    if (!(df > 0.0) || !(df < (double)d)) return set_error(CWB_E_INVALID_ARG, "df must lie in (0, d)");
    std::vector<double> g(G, G + (size_t)d * d), p(D, D + (size_t)d * d);
    std::string err;
    const int rc = lambda_for_df(d, g, p, df, lambda, &err);
    return rc ? set_error(rc == -5 ? CWB_E_NUMERIC : CWB_E_INVALID_ARG, err) : CWB_OK;
  } catch (...) {
    return set_error(CWB_E_INVALID_ARG, "unexpected error");
  }
}

int cwb_workspace_bytes(const cwb_problem* pr, size_t* bytes) {
  try {
    if (!bytes) return set_error(CWB_E_INVALID_ARG, "null bytes pointer");
    std::string err;
    FitShape sh;
    int rc = shape_from_problem(pr, &sh, &err);
    if (rc) return set_error(rc, err);
    return fit_footprint(sh, bytes, true);
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return set_error(CWB_E_INVALID_ARG, "unexpected error");
  }
}

static int fit_create_impl(const cwb_problem* pr, void* dev_ws, size_t ws_bytes, void* stream,
                           cwb_fit** out) {
  if (!out) return set_error(CWB_E_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!dev_ws) return set_error(CWB_E_INVALID_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0)
    return set_error(CWB_E_INVALID_ARG, "workspace must be 256-byte aligned");
  std::string err;
  FitShape sh;
  int rc = shape_from_problem(pr, &sh, &err);
  if (rc) return set_error(rc, err);
  if (pr->setup < CWB_SETUP_AUTO || pr->setup > CWB_SETUP_DEVICE)
    return set_error(CWB_E_INVALID_ARG, "unknown setup mode");
  const bool device_ok = !sh.unbinned && sh.n < (int64_t)INT32_MAX;
  if (pr->setup == CWB_SETUP_DEVICE && !device_ok)
    return set_error(CWB_E_UNSUPPORTED, "device setup covers binned fits with n < 2^31");
  const bool on_device = pr->setup == CWB_SETUP_DEVICE || (pr->setup == CWB_SETUP_AUTO && device_ok);
  HostFit hf;
  rc = on_device ? prepare_host_fit(pr, &hf, &err) : build_host_fit(pr, &hf, &err);
  if (rc) return set_error(rc, err);
  return fit_upload(sh, hf, dev_ws, ws_bytes, reinterpret_cast<hipStream_t>(stream), true, out,
                    on_device ? pr : nullptr);
}

int cwb_fit_create(const cwb_problem* pr, void* dev_ws, size_t ws_bytes, void* stream, cwb_fit** out) {
  try {
    return fit_create_impl(pr, dev_ws, ws_bytes, stream, out);
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(CWB_E_INVALID_ARG, e.what());
  } catch (...) {
    return set_error(CWB_E_INVALID_ARG, "unexpected error");
  }
}

int cwb_fit_run(cwb_fit* f, int32_t iters) {
  if (!f) return set_error(CWB_E_INVALID_ARG, "null fit");
  if (iters < 0) return set_error(CWB_E_INVALID_ARG, "negative iteration count");
  if ((int64_t)f->iters + iters > f->shape.M)
    return set_error(CWB_E_STATE, "run would exceed M iterations");
  HIP_TRY(hipSetDevice(f->device));
  const Layout& L = f->lay;
  char* ws = f->ws;
  for (int i = 0; i < iters; ++i) {
    int rc = enqueue_iteration(f->stream, f->d_fit, 1, f->sched, f->tune, dptr<RowItem>(ws, L.st_items),
                               f->n_st, dptr<SelItem>(ws, L.sel_items), f->n_sel,
                               dptr<StateItem>(ws, L.val_items), f->n_val, f->shape.nb_max,
                               f->shape.d_max,
                               dptr<Seg>(ws, L.segs), dptr<int64_t>(ws, L.blk),
                               dptr<int64_t>(ws, L.sel_off), f->partials, f);
    if (rc) return rc;
  }
  f->iters += iters;
  return CWB_OK;
}

static int check_device_error(cwb_fit* f) {
  int32_t e = 0;
  HIP_TRY(hipMemcpy(&e, f->ws + f->lay.ctl + offsetof(Ctl, error), sizeof(e), hipMemcpyDeviceToHost));
  if (e & 2) return set_error(CWB_E_DEVICE, "internal: a histogram segment larger than its launch's LDS");
  if (e) return set_error(CWB_E_NUMERIC, "non-finite model state (diverged)");
  return CWB_OK;
}

int cwb_fit_sync(cwb_fit* f) {
  if (!f) return set_error(CWB_E_INVALID_ARG, "null fit");
  HIP_TRY(hipSetDevice(f->device));
  HIP_TRY(hipStreamSynchronize(f->stream));
  return check_device_error(f);
}

int cwb_fit_info(const cwb_fit* f, cwb_info* info) {
  if (!f || !info) return set_error(CWB_E_INVALID_ARG, "null argument");
  info->n = f->shape.n;
  info->p = f->shape.p;
  info->M = f->shape.M;
  info->d_max = f->shape.d_max;
  info->sum_d = f->shape.sum_d;
  info->nb_max = f->shape.nb_max;
  info->iters_done = f->iters;
  info->n_train = f->shape.n_train;
  info->f0 = f->f0;
  return CWB_OK;
}

static int finalize_and_sync(cwb_fit* f) {
  int rc = finalize_fit(f);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(f->stream));
  return check_device_error(f);
}

int cwb_fit_get_trace(cwb_fit* f, int32_t* k, double* theta, int32_t* k_cor, double* theta_cor,
                      double* train_risk, double* val_risk, double* crit_gap, int32_t* switch_iter) {
  if (!f) return set_error(CWB_E_INVALID_ARG, "null fit");
  int rc = finalize_and_sync(f);
  if (rc) return rc;
  const Layout& L = f->lay;
  const size_t m = (size_t)f->iters;
  const size_t dm = (size_t)f->shape.d_max;
  if (k) HIP_TRY(hipMemcpy(k, f->ws + L.trk, m * 4, hipMemcpyDeviceToHost));
  if (theta) HIP_TRY(hipMemcpy(theta, f->ws + L.trth, m * dm * 8, hipMemcpyDeviceToHost));
  if (k_cor) HIP_TRY(hipMemcpy(k_cor, f->ws + L.trkc, m * 4, hipMemcpyDeviceToHost));
  if (theta_cor) HIP_TRY(hipMemcpy(theta_cor, f->ws + L.trthc, m * dm * 8, hipMemcpyDeviceToHost));
  if (train_risk) HIP_TRY(hipMemcpy(train_risk, f->ws + L.trrisk, (m + 1) * 8, hipMemcpyDeviceToHost));
  if (val_risk) HIP_TRY(hipMemcpy(val_risk, f->ws + L.trval, (m + 1) * 8, hipMemcpyDeviceToHost));
  if (crit_gap) HIP_TRY(hipMemcpy(crit_gap, f->ws + L.trgap, m * 8, hipMemcpyDeviceToHost));
  if (switch_iter) {
    Ctl c;
    HIP_TRY(hipMemcpy(&c, f->ws + L.ctl, sizeof(c), hipMemcpyDeviceToHost));
    *switch_iter = c.switched ? c.switch_iter : -1;
  }
  return CWB_OK;
}

int cwb_fit_get_model(cwb_fit* f, double* intercept, double* coef_f, double* coef_h) {
  if (!f) return set_error(CWB_E_INVALID_ARG, "null fit");
  HIP_TRY(hipSetDevice(f->device));
  int rc0 = finalize_fit(f);  // records the last selection
  if (rc0) return rc0;
  HIP_TRY(launch_coef(f->stream, f->d_fit, f->shape.sum_d));
  HIP_TRY(hipStreamSynchronize(f->stream));
  int rc = check_device_error(f);
  if (rc) return rc;
  if (intercept) *intercept = f->f0;
  const size_t sd = (size_t)f->shape.sum_d;
  if (coef_f) HIP_TRY(hipMemcpy(coef_f, f->ws + f->lay.coef_f, sd * 8, hipMemcpyDeviceToHost));
  if (coef_h) {
    if (f->shape.nsig_max == 2)
      HIP_TRY(hipMemcpy(coef_h, f->ws + f->lay.coef_h, sd * 8, hipMemcpyDeviceToHost));
    else
      std::memset(coef_h, 0, sd * 8);
  }
  return CWB_OK;
}

int cwb_fit_predict(cwb_fit* f, const double* x, int64_t n, int64_t ldx, double* out) {
  if (!f) return set_error(CWB_E_INVALID_ARG, "null fit");
  if (n < 0 || (n > 0 && (!x || !out))) return set_error(CWB_E_INVALID_ARG, "null x or out");
  if (ldx < n) return set_error(CWB_E_INVALID_ARG, "ldx must be at least n");
  HIP_TRY(hipSetDevice(f->device));
  int rc = finalize_fit(f);
  if (rc) return rc;
  HIP_TRY(launch_coef(f->stream, f->d_fit, f->shape.sum_d));
  HIP_TRY(launch_predict(f->stream, f->d_fit, x, n, ldx, f->f0, 0, f->shape.p, out));
  return CWB_OK;
}

int cwb_fit_partial_effect(cwb_fit* f, int32_t k, const double* x, int64_t n, double* out) {
  if (!f) return set_error(CWB_E_INVALID_ARG, "null fit");
  if (k < 0 || k >= f->shape.p) return set_error(CWB_E_INVALID_ARG, "learner index out of range");
  if (n < 0 || (n > 0 && (!x || !out))) return set_error(CWB_E_INVALID_ARG, "null x or out");
  HIP_TRY(hipSetDevice(f->device));
  int rc = finalize_fit(f);
  if (rc) return rc;
  HIP_TRY(launch_coef(f->stream, f->d_fit, f->shape.sum_d));
  HIP_TRY(launch_predict(f->stream, f->d_fit, x, n, n, 0.0, k, k + 1, out));
  return CWB_OK;
}

int cwb_fit_get_pred(cwb_fit* f, float* f_out) {
  if (!f || !f_out) return set_error(CWB_E_INVALID_ARG, "null argument");
  int rc = finalize_and_sync(f);
  if (rc) return rc;
  std::vector<float> buf((size_t)f->shape.n);
  HIP_TRY(hipMemcpy(buf.data(), f->ws + f->lay.fg, buf.size() * 4, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < f->shape.n; ++i) f_out[f->perm[i]] = buf[i];
  return CWB_OK;
}

int cwb_fit_state_bytes(const cwb_fit* f, size_t* bytes) {
  if (!f || !bytes) return set_error(CWB_E_INVALID_ARG, "null argument");
  *bytes = sizeof(int64_t) + (f->lay.state_end - f->lay.state_begin);
  return CWB_OK;
}

int cwb_fit_save_state(cwb_fit* f, void* host_buf, size_t bytes) {
  size_t need = 0;
  int rc = cwb_fit_state_bytes(f, &need);
  if (rc) return rc;
  if (!host_buf || bytes < need) return set_error(CWB_E_INVALID_ARG, "state buffer too small");
  HIP_TRY(hipSetDevice(f->device));
  HIP_TRY(hipStreamSynchronize(f->stream));
  int64_t it = f->iters;
  std::memcpy(host_buf, &it, sizeof(it));
  HIP_TRY(hipMemcpy(static_cast<char*>(host_buf) + sizeof(it), f->ws + f->lay.state_begin,
                    need - sizeof(it), hipMemcpyDeviceToHost));
  return CWB_OK;
}

int cwb_fit_load_state(cwb_fit* f, const void* host_buf, size_t bytes) {
  size_t need = 0;
  int rc = cwb_fit_state_bytes(f, &need);
  if (rc) return rc;
  if (!host_buf || bytes != need) return set_error(CWB_E_INVALID_ARG, "state buffer has the wrong size");
  int64_t it = 0;
  std::memcpy(&it, host_buf, sizeof(it));
  if (it < 0 || it > f->shape.M) return set_error(CWB_E_INVALID_ARG, "corrupt state buffer");
  HIP_TRY(hipSetDevice(f->device));
  HIP_TRY(hipStreamSynchronize(f->stream));
  HIP_TRY(hipMemcpy(f->ws + f->lay.state_begin, static_cast<const char*>(host_buf) + sizeof(it),
                    need - sizeof(it), hipMemcpyHostToDevice));
  f->iters = (int)it;
  return CWB_OK;
}

int cwb_fit_set_timing(cwb_fit* f, int32_t mask) {
  return cwb_fit_set_timing_period(f, mask, 1);
}

int cwb_fit_set_timing_period(cwb_fit* f, int32_t mask, int32_t period) {
  if (!f) return set_error(CWB_E_INVALID_ARG, "null fit");
  if (mask < 0 || mask > 7) return set_error(CWB_E_INVALID_ARG, "timing mask must be 0..7");
  if (period < 1) return set_error(CWB_E_INVALID_ARG, "timing period must be >= 1");
  f->timing = mask;
  f->timing_period = period;
  f->timing_counter = 0;
  timer_reset(f->t_hist);
  timer_reset(f->t_state);
  timer_reset(f->t_select);
  return CWB_OK;
}

int cwb_fit_kernel_time(cwb_fit* f, const char* kernel, double* total_ms, int64_t* launches) {
  if (!f || !kernel) return set_error(CWB_E_INVALID_ARG, "null argument");
  KernelTimer* t = nullptr;
  if (!std::strcmp(kernel, "hist")) t = &f->t_hist;
  else if (!std::strcmp(kernel, "state")) t = &f->t_state;
  else if (!std::strcmp(kernel, "select")) t = &f->t_select;
  if (!t) return set_error(CWB_E_INVALID_ARG, "unknown kernel name");
  HIP_TRY(hipSetDevice(f->device));
  HIP_TRY(timer_collect(*t));
  if (total_ms) *total_ms = t->total_ms;
  if (launches) *launches = t->launches;
  return CWB_OK;
}

namespace {
// Bits per bin index the fit's histogram pass reads (its packed copy, or
// the uint16 matrix).
int fit_index_bits(const cwb_fit* f) { return f->dev.X12 ? f->dev.xbits : 16; }
}  // namespace

int cwb_fit_tile(const cwb_fit* f, cwb_tile* out) {
  if (!f || !out) return set_error(CWB_E_INVALID_ARG, "null argument");
  out->threads = f->tune.nt;
  out->learners = f->tune.F;
  out->blocks = f->sched.blocks;
  out->candidates = f->n_cands;
  out->learners32 = learners32(f->sched);
  out->acc32_bits = f->shape.acc32_bits;
  out->index_bits = fit_index_bits(f);
  out->tuned_us = f->tuned_us;
  return CWB_OK;
}

void cwb_fit_destroy(cwb_fit* f) {
  if (!f) return;
  (void)hipSetDevice(f->device);  // destroy reports nothing: a failure here leaves no state behind
  (void)hipStreamSynchronize(f->stream);
  timer_free(f->t_hist);
  timer_free(f->t_state);
  timer_free(f->t_select);
  delete f;
}

}  // extern "C"

// ---- batches ----------------------------------------------------------------

namespace cwb {
namespace {

struct BatchLayout {
  size_t fits, segs, blk, sel_off, partials, st, sel, val, total;
};

BatchLayout batch_layout(const SchedCap& S, int count, int n_st, int n_sel, int n_val) {
  BatchLayout L;
  size_t off = 0;
  auto take = [&](size_t b) {
    off = align_up(off, 256);
    const size_t o = off;
    off += b;
    return o;
  };
  L.fits = take((size_t)count * sizeof(FitDev));
  L.segs = take(S.segs * sizeof(Seg));
  L.blk = take(S.blk * 8);
  L.sel_off = take(S.sel_off * 8);
  L.partials = take((size_t)S.partial_words * 8);
  L.st = take((size_t)std::max(1, n_st) * sizeof(RowItem));
  L.sel = take((size_t)std::max(1, n_sel) * sizeof(SelItem));
  L.val = take((size_t)std::max(1, n_val) * sizeof(StateItem));
  L.total = align_up(off, 256);
  return L;
}

void work_counts(const std::vector<const FitShape*>& shapes, int* n_st, int* n_sel, int* n_val) {
  *n_st = *n_sel = *n_val = 0;
  for (const FitShape* sh : shapes) {
    *n_st += sh->n_row_blocks;
    *n_sel += sh->p;
    *n_val += sh->n_val_blocks;
  }
}

int batch_shapes(cwb_fit* const* fits, int32_t count, std::vector<const FitShape*>* shapes) {
  if (!fits || count < 1) return set_error(CWB_E_INVALID_ARG, "need at least one fit");
  for (int i = 0; i < count; ++i) {
    if (!fits[i]) return set_error(CWB_E_INVALID_ARG, "null fit in batch");
    for (int j = 0; j < i; ++j)
      if (fits[j] == fits[i]) return set_error(CWB_E_INVALID_ARG, "fit listed twice in batch");
    fits[i]->bshape = fits[i]->shape;
    fits[i]->bshape.share = fits[i]->batch_share;
    shapes->push_back(&fits[i]->bshape);
  }
  return CWB_OK;
}

// Upload a schedule and the select work list that indexes its partials.
int batch_install(cwb_batch* b, const Tune& t, Schedule&& S) {
  std::vector<SelItem> sel;
  for (size_t i = 0; i < b->fits.size(); ++i) {
    cwb_fit* f = b->fits[i];
    for (int k = 0; k < f->shape.p; ++k)
      sel.push_back(make_sel_item((int)i, k, f->feat[k], f->dev, S, b->d_sel_off, sel.size()));
  }
  hipStream_t s = b->stream;
  HIP_TRY(hipMemcpyAsync(b->d_segs, S.segs.data(), S.segs.size() * sizeof(Seg), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b->d_blk, S.blk.data(), S.blk.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b->d_sel_off, S.sel_off.data(), S.sel_off.size() * 8, hipMemcpyHostToDevice, s));
  if (!sel.empty())
    HIP_TRY(hipMemcpyAsync(b->d_sel, sel.data(), sel.size() * sizeof(SelItem), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  b->tune = t;
  b->sched = std::move(S);
  return CWB_OK;
}

}  // namespace

int batch_footprint(const std::vector<const FitShape*>& shapes, size_t* bytes, bool all) {
  if (shapes.empty()) {
    *bytes = 0;
    return CWB_OK;
  }
  std::vector<Tune> cands;
  SchedCap cap;
  int rc = plan_candidates(shapes, all, &cands, &cap, nullptr);
  if (rc) return rc;
  int n_st, n_sel, n_val;
  work_counts(shapes, &n_st, &n_sel, &n_val);
  *bytes = batch_layout(cap, (int)shapes.size(), n_st, n_sel, n_val).total;
  return CWB_OK;
}

int batch_create(cwb_fit* const* fits, int32_t count, void* dev_ws, size_t ws_bytes, hipStream_t stream,
                 bool autotune, cwb_batch** out) {
  if (!out) return set_error(CWB_E_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!dev_ws || reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0)
    return set_error(CWB_E_INVALID_ARG, "workspace must be non-null and 256-byte aligned");
  std::vector<const FitShape*> shapes;
  int rc = batch_shapes(fits, count, &shapes);
  if (rc) return rc;
  std::unique_ptr<cwb_batch> b(new cwb_batch());
  std::vector<Tune> cands;
  SchedCap cap;
  Schedule first;
  rc = plan_candidates(shapes, autotune, &cands, &cap, &first);
  if (rc) return rc;
  work_counts(shapes, &b->n_st, &b->n_sel, &b->n_val);
  const BatchLayout L = batch_layout(cap, count, b->n_st, b->n_sel, b->n_val);
  if (ws_bytes < L.total)
    return set_error(CWB_E_NO_MEMORY, "batch workspace too small: need " + std::to_string(L.total));
  HIP_TRY(hipGetDevice(&b->device));
  for (int i = 0; i < count; ++i)
    if (fits[i]->device != b->device) return set_error(CWB_E_INVALID_ARG, "fits on different devices");
  b->stream = stream;
  b->ws = reinterpret_cast<char*>(dev_ws);
  b->ws_bytes = ws_bytes;
  b->fits.assign(fits, fits + count);
  b->n_cands = (int)cands.size();
  std::vector<FitDev> fd(count);
  std::vector<RowItem> st;
  std::vector<StateItem> val;
  int64_t chunks_total = 0;
  for (int i = 0; i < count; ++i) chunks_total += fits[i]->shape.n_row_blocks;
  const int chunks = row_chunks(chunks_total, cands[0].cus);
  for (int i = 0; i < count; ++i) {
    fd[i] = fits[i]->dev;
    b->nb_max = std::max(b->nb_max, fits[i]->shape.nb_max);
    b->d_max = std::max(b->d_max, fits[i]->shape.d_max);
    if (fits[i]->shape.variant == CWB_HCWB) b->any_hcwb = true;
    append_row_items(&st, i, fits[i]->dev, fits[i]->shape.n_row_blocks, chunks);
    for (int r = 0; r < fits[i]->shape.n_val_blocks; ++r) val.push_back({i, r});
  }
  b->n_st = (int)st.size();
  char* ws = b->ws;
  hipStream_t s = b->stream;
  b->d_fits = dptr<FitDev>(ws, L.fits);
  b->d_segs = dptr<Seg>(ws, L.segs);
  b->d_blk = dptr<int64_t>(ws, L.blk);
  b->d_sel_off = dptr<int64_t>(ws, L.sel_off);
  b->d_partials = dptr<long long>(ws, L.partials);
  b->d_st = dptr<RowItem>(ws, L.st);
  b->d_sel = dptr<SelItem>(ws, L.sel);
  b->d_val = dptr<StateItem>(ws, L.val);
  HIP_TRY(hipMemcpyAsync(b->d_fits, fd.data(), fd.size() * sizeof(FitDev), hipMemcpyHostToDevice, s));
  if (!st.empty()) HIP_TRY(hipMemcpyAsync(b->d_st, st.data(), st.size() * sizeof(RowItem), hipMemcpyHostToDevice, s));
  if (!val.empty()) HIP_TRY(hipMemcpyAsync(b->d_val, val.data(), val.size() * sizeof(StateItem), hipMemcpyHostToDevice, s));
  rc = batch_install(b.get(), cands[0], std::move(first));
  if (rc) return rc;
  if (cands.size() > 1) {
    int best = 0;
    rc = autotune_hist(s, b->d_fits, shapes, cands, cap, b->d_segs, b->d_blk, b->d_partials, &best,
                       &b->tuned_us);
    if (rc) return rc;
    rc = batch_install(b.get(), cands[best], build_schedule(shapes, cands[best]));
    if (rc) return rc;
  }
  *out = b.release();
  return CWB_OK;
}

}  // namespace cwb

extern "C" {

int cwb_batch_workspace_bytes(cwb_fit* const* fits, int32_t count, size_t* bytes) {
  try {
    if (!bytes) return set_error(CWB_E_INVALID_ARG, "null bytes pointer");
    std::vector<const FitShape*> shapes;
    int rc = batch_shapes(fits, count, &shapes);
    if (rc) return rc;
    return batch_footprint(shapes, bytes, true);
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  }
}

int cwb_batch_create(cwb_fit* const* fits, int32_t count, void* dev_ws, size_t ws_bytes, void* stream,
                     cwb_batch** out) {
  try {
    return batch_create(fits, count, dev_ws, ws_bytes, reinterpret_cast<hipStream_t>(stream), true, out);
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  }
}

int cwb_batch_run(cwb_batch* b, int32_t iters) {
  if (!b) return set_error(CWB_E_INVALID_ARG, "null batch");
  if (iters < 0) return set_error(CWB_E_INVALID_ARG, "negative iteration count");
  HIP_TRY(hipSetDevice(b->device));
  int most = 0;
  for (cwb_fit* f : b->fits) most = std::max(most, std::min(iters, f->shape.M - f->iters));
  // Eager launches are timed with the first fit's timer when its timing is
  // on (the batch's kernels, not that fit's share); captured ones never are.
  auto eager = [&](bool capturing = false) {
    cwb_fit* timed = (!capturing && b->fits[0]->timing) ? b->fits[0] : nullptr;
    return enqueue_iteration(b->stream, b->d_fits, (int)b->fits.size(), b->sched, b->tune, b->d_st,
                             b->n_st, b->d_sel, b->n_sel, b->d_val, b->any_hcwb ? b->n_val : 0,
                             b->nb_max, b->d_max, b->d_segs, b->d_blk, b->d_sel_off,
                             b->d_partials, timed);
  };
  int i = 0;
  // The first iteration runs eagerly; after it, chunks of kGraphIters
  // iterations replay one captured graph.  Every kernel reads its iteration
  // from the fits' control blocks, so one graph serves every chunk.
  const bool graphs = b->stream != nullptr && env_int("CWB_GRAPH", 1) != 0;
  if (graphs && !b->graph_exec && most > kGraphIters && b->eager_iters == 0) {
    int rc = eager();
    if (rc) return rc;
    ++i;
    ++b->eager_iters;
  }
  while (graphs && most - i >= kGraphIters && b->eager_iters > 0) {
    if (!b->graph_exec) {
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
      int rc = CWB_OK;
      for (int c = 0; c < kGraphIters && !rc; ++c) rc = eager(true);
      const hipError_t e = hipStreamEndCapture(b->stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return set_error(CWB_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
      const hipError_t e2 = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e2 != hipSuccess) {
        b->graph_exec = nullptr;
        return set_error(CWB_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e2));
      }
    }
    HIP_TRY(hipGraphLaunch(b->graph_exec, b->stream));
    i += kGraphIters;
    b->graph_launches += 1;
  }
  for (; i < most; ++i) {
    int rc = eager();
    if (rc) return rc;
    ++b->eager_iters;
  }
  for (cwb_fit* f : b->fits) f->iters += std::min(most, f->shape.M - f->iters);
  return CWB_OK;
}

int cwb_batch_tile(const cwb_batch* b, cwb_tile* out) {
  if (!b || !out) return set_error(CWB_E_INVALID_ARG, "null argument");
  out->threads = b->tune.nt;
  out->learners = b->tune.F;
  out->blocks = b->sched.blocks;
  out->candidates = b->n_cands;
  out->learners32 = learners32(b->sched);
  out->acc32_bits = 0;
  out->index_bits = 0;
  for (const cwb_fit* f : b->fits) {
    out->acc32_bits = std::max(out->acc32_bits, f->shape.acc32_bits);
    out->index_bits = std::max(out->index_bits, fit_index_bits(f));
  }
  out->tuned_us = b->tuned_us;
  return CWB_OK;
}

int cwb_batch_sync(cwb_batch* b) {
  if (!b) return set_error(CWB_E_INVALID_ARG, "null batch");
  HIP_TRY(hipSetDevice(b->device));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (cwb_fit* f : b->fits) {
    int rc = check_device_error(f);
    if (rc) return rc;
  }
  return CWB_OK;
}

void cwb_batch_destroy(cwb_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Cross-validation: K folds sharing one index matrix and one histogram pass.
// ---------------------------------------------------------------------------

struct cwb_cv {
  int K = 0;
  int64_t n = 0;
  std::vector<int64_t> rows;       // rows held out by each fold
  std::vector<cwb_fit*> fits;      // fold k's fit (owned)
  cwb_batch* batch = nullptr;      // all folds (owned)
};

namespace cwb {
namespace {

struct CvPlan {
  FitShape sh;                     // a fold's shape (external index matrix, every row read)
  std::vector<int64_t> rows;       // rows of each fold
  size_t x_bytes = 0, fold_bytes = 0, fit_bytes = 0, batch_bytes = 0, total = 0;
};

int cv_plan(const cwb_problem* pr, int32_t K, const int32_t* fold, CvPlan* pl) {
  if (!pr) return set_error(CWB_E_INVALID_ARG, "null problem");
  if (K < 2 || K > kMaxFolds)
    return set_error(CWB_E_INVALID_ARG, "fold count must be 2.." + std::to_string(kMaxFolds));
  if (!fold) return set_error(CWB_E_INVALID_ARG, "null fold ids");
  if (pr->n < 2) return set_error(CWB_E_INVALID_ARG, "n must be >= 2");
  pl->rows.assign(K, 0);
  for (int64_t i = 0; i < pr->n; ++i) {
    if (fold[i] < 0 || fold[i] >= K) return set_error(CWB_E_INVALID_ARG, "fold id out of range");
    pl->rows[fold[i]] += 1;
  }
  for (int k = 0; k < K; ++k)
    if (pl->rows[k] < 1 || pr->n - pl->rows[k] < 2)
      return set_error(CWB_E_INVALID_ARG, "every fold needs a row, and two training rows");
  if (pr->val_mask) return set_error(CWB_E_INVALID_ARG, "a cross-validation takes no validation mask");
  if (pr->variant != CWB_CWB && pr->variant != CWB_ACWB)
    return set_error(CWB_E_UNSUPPORTED, "cross-validation runs CWB or ACWB folds");
  std::string err;
  int rc = shape_from_problem(pr, &pl->sh, &err);
  if (rc) return set_error(rc, err);
  if (pl->sh.unbinned) return set_error(CWB_E_UNSUPPORTED, "cross-validation covers binned learners");
  if ((size_t)K * pl->sh.nsig_max * pl->sh.nb_stride * sizeof(long long) > (size_t)kHistMaxLds)
    return set_error(CWB_E_UNSUPPORTED, "the folds' histograms of one learner exceed the LDS");
  pl->sh.n_scan = pl->sh.n;
  pl->sh.external_x = true;
  pl->sh.x12 = false;
  rc = fit_footprint(pl->sh, &pl->fit_bytes, false);
  if (rc) return rc;
  pl->sh.fold_start.assign(K + 1, 0);  // rows grouped by fold
  for (int k = 0; k < K; ++k) pl->sh.fold_start[k + 1] = pl->sh.fold_start[k] + pl->rows[k];
  std::vector<FitShape> shapes(K, pl->sh);
  std::vector<const FitShape*> sp;
  for (int k = 0; k < K; ++k) {
    shapes[k].share = (k == 0) ? K : 0;
    sp.push_back(&shapes[k]);
  }
  rc = batch_footprint(sp, &pl->batch_bytes, true);
  if (rc) return rc;
  pl->x_bytes = align_up((size_t)pl->sh.p * pl->sh.n_pad * 2, 256);
  pl->fold_bytes = align_up((size_t)pl->sh.n_pad, 256);
  pl->fit_bytes = align_up(pl->fit_bytes, 256);
  pl->total = pl->x_bytes + pl->fold_bytes + (size_t)K * pl->fit_bytes + pl->batch_bytes;
  return CWB_OK;
}

int cv_create_impl(const cwb_problem* pr, int32_t K, const int32_t* fold, void* dev_ws,
                   size_t ws_bytes, hipStream_t stream, cwb_cv** out) {
  if (!out) return set_error(CWB_E_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!fold) return set_error(CWB_E_INVALID_ARG, "null fold ids");
  if (!dev_ws || reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0)
    return set_error(CWB_E_INVALID_ARG, "workspace must be non-null and 256-byte aligned");
  CvPlan pl;
  int rc = cv_plan(pr, K, fold, &pl);
  if (rc) return rc;
  if (ws_bytes < pl.total)
    return set_error(CWB_E_NO_MEMORY, "workspace too small: need " + std::to_string(pl.total) +
                                          " bytes, got " + std::to_string(ws_bytes));
  const int64_t n = pr->n;
  std::unique_ptr<cwb_cv> cv(new cwb_cv());
  cv->K = K;
  cv->n = n;
  cv->rows = pl.rows;
  HostFit full;
  std::vector<HostFit> folds;
  std::string err;
  rc = cv_host_fits(pr, K, fold, &full, &folds, &err);
  if (rc) return set_error(rc, err);
  char* ws = reinterpret_cast<char*>(dev_ws);
  uint16_t* d_X = reinterpret_cast<uint16_t*>(ws);
  uint8_t* d_fold = reinterpret_cast<uint8_t*>(ws + pl.x_bytes);
  std::vector<uint8_t> f8((size_t)pl.sh.n_pad, (uint8_t)K);  // padding rows: no fold
  for (int64_t i = 0; i < n; ++i) f8[i] = (uint8_t)fold[full.perm[i]];  // fold-grouped order
  HIP_TRY(hipMemcpyAsync(d_X, full.X.data(), full.X.size() * 2, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(d_fold, f8.data(), f8.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  full.X.clear();
  char* fit_ws = ws + pl.x_bytes + pl.fold_bytes;
  struct Cleanup {
    cwb_cv* cv;
    ~Cleanup() {
      if (!cv) return;
      cwb_batch_destroy(cv->batch);
      for (cwb_fit* f : cv->fits) cwb_fit_destroy(f);
    }
  } guard{cv.get()};
  for (int k = 0; k < K; ++k) {
    FitShape sh = pl.sh;
    sh.n_train = n - cv->rows[k];
    FoldSpec fs;
    fs.X = d_X;
    fs.fold = d_fold;
    fs.k = k;
    cwb_fit* f = nullptr;
    rc = fit_upload(sh, folds[k], fit_ws + (size_t)k * pl.fit_bytes, pl.fit_bytes, stream, false, &f,
                    nullptr, &fs);
    if (rc) return rc;
    f->batch_share = (k == 0) ? K : 0;
    cv->fits.push_back(f);
  }
  rc = batch_create(cv->fits.data(), K, fit_ws + (size_t)K * pl.fit_bytes, pl.batch_bytes, stream,
                    true, &cv->batch);
  if (rc) return rc;
  guard.cv = nullptr;
  *out = cv.release();
  return CWB_OK;
}

}  // namespace
}  // namespace cwb

extern "C" {

int cwb_cv_workspace_bytes(const cwb_problem* pr, int32_t n_folds, const int32_t* fold,
                           size_t* bytes) {
  try {
    if (!bytes) return set_error(CWB_E_INVALID_ARG, "null bytes pointer");
    CvPlan pl;
    const int rc = cv_plan(pr, n_folds, fold, &pl);
    if (rc) return rc;
    *bytes = pl.total;
    return CWB_OK;
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  }
}

int cwb_cv_create(const cwb_problem* pr, int32_t n_folds, const int32_t* fold, void* dev_ws,
                  size_t ws_bytes, void* stream, cwb_cv** out) {
  try {
    return cv_create_impl(pr, n_folds, fold, dev_ws, ws_bytes, reinterpret_cast<hipStream_t>(stream),
                          out);
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(CWB_E_INVALID_ARG, e.what());
  }
}

int cwb_cv_run(cwb_cv* cv, int32_t iters) {
  if (!cv) return set_error(CWB_E_INVALID_ARG, "null cross-validation");
  return cwb_batch_run(cv->batch, iters);
}

int cwb_cv_sync(cwb_cv* cv) {
  if (!cv) return set_error(CWB_E_INVALID_ARG, "null cross-validation");
  return cwb_batch_sync(cv->batch);
}

int cwb_cv_fold(cwb_cv* cv, int32_t k, cwb_fit** out) {
  if (!cv || !out) return set_error(CWB_E_INVALID_ARG, "null argument");
  if (k < 0 || k >= cv->K) return set_error(CWB_E_INVALID_ARG, "fold index out of range");
  *out = cv->fits[k];
  return CWB_OK;
}

int cwb_cv_risk(cwb_cv* cv, double* risk) {
  if (!cv || !risk) return set_error(CWB_E_INVALID_ARG, "null argument");
  try {
    const int M = cv->fits[0]->shape.M;
    const int m = cv->fits[0]->iters;
    std::vector<double> rv((size_t)M + 1);
    for (int i = 0; i <= m; ++i) risk[i] = 0.0;
    for (int k = 0; k < cv->K; ++k) {
      const int rc = cwb_fit_get_trace(cv->fits[k], nullptr, nullptr, nullptr, nullptr, nullptr,
                                       rv.data(), nullptr, nullptr);
      if (rc) return rc;
      for (int i = 0; i <= m; ++i) risk[i] += rv[i] * (double)cv->rows[k] / (double)cv->n;
    }
    return CWB_OK;
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  }
}

int cwb_cv_tile(const cwb_cv* cv, cwb_tile* out) {
  if (!cv) return set_error(CWB_E_INVALID_ARG, "null cross-validation");
  return cwb_batch_tile(cv->batch, out);
}

void cwb_cv_destroy(cwb_cv* cv) {
  if (!cv) return;
  cwb_batch_destroy(cv->batch);
  for (cwb_fit* f : cv->fits) cwb_fit_destroy(f);
  delete cv;
}

}  // extern "C"

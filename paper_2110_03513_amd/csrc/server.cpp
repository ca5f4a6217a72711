// server.cpp -- continuous-batching fit server.
//
// Requests flow through four stages:
//   submit    the request is queued for setup (the caller's arrays are read
//             in place, so they stay valid until its result is polled);
//   setup     host threads check the request and compute its device
//             footprint; a request set up on the host also has its FP64
//             setup run here (binning, bases, Grams, smoothing parameters);
//   admission the device thread admits set-up requests in arrival order while
//             the arena holds their workspace and the batch workspace of the
//             grown set, and a slot is free;
//   run       all admitted fits advance together, `quantum` iterations per
//             round (one launch per kernel per iteration covers every fit);
//             finished fits retire at the end of a round: their results are
//             copied to the host and their arena space is released.
// Uploads of newly admitted fits run on their own host thread and a second
// stream, so neither the rounds nor the GPU wait for them; an uploaded fit
// joins the batch at the next round boundary.  A request set up on the GPU
// (cwb_problem.setup AUTO or DEVICE, binned, n < 2^31) is binned, counted
// and solved during its upload, in its own arena space, on that stream.
// A fit's result does not depend on which other fits share its rounds: the
// histograms are exact integer sums and every selection is per fit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>

#include "admission.h"
#include "runtime.h"

namespace cwb {
namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum class Stage { kQueued, kSetup, kReady, kAdmitted, kRunning, kDone };

struct Request {
  uint64_t ticket = 0;
  Stage stage = Stage::kQueued;
  double t_submit = 0, t_admit = 0, t_done = 0;
  // the problem (caller-owned arrays, copied specifications)
  cwb_problem pr;
  std::vector<cwb_learner_spec> specs;
  double setup_s = 0;  // host setup, plus the upload (and device setup pass)
  bool dev_setup = false;  // binning, counts and solves during the upload
  // setup result, dropped after upload
  FitShape shape;
  HostFit hf;
  size_t footprint = 0;
  // device residency
  cwb_fit* fit = nullptr;
  size_t off = 0;
  // result
  int status = CWB_OK;
  std::string err;
  int M = 0;
  double intercept = 0;
  std::vector<float> pred;
  std::vector<int32_t> k;
};

}  // namespace
}  // namespace cwb

using namespace cwb;

struct cwb_server {
  cwb_server_cfg cfg;
  int device = 0;
  hipStream_t stream = nullptr;   // rounds
  hipStream_t upload = nullptr;   // uploads of admitted fits
  char* base = nullptr;

  std::mutex mu;
  std::condition_variable cv_setup, cv_dev, cv_up;
  bool stop = false;
  bool stop_up = false;  // the upload thread ends (after the device thread)
  uint64_t next_ticket = 1;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;  // every request not yet polled
  std::deque<Request*> setup_q;
  std::deque<Request*> ready_q;
  std::deque<Request*> upload_q;   // admitted, for the upload thread
  std::vector<Request*> uploaded;  // uploaded (or failed), to join at a round boundary
  Arena arena;
  int64_t submitted = 0, completed = 0, rejected = 0;
  int32_t in_flight = 0;
  double t_first = -1.0, t_last_done = 0.0;
  double sum_setup_s = 0.0, sum_queue_s = 0.0;
  double round_s = 0.0, t_first_round = -1.0, t_last_round = 0.0;
  int64_t rounds = 0;
  std::vector<double> latencies;

  // device thread only
  std::vector<Request*> active;
  std::vector<Request*> pending;   // admitted and not yet joined
  cwb_batch* batch = nullptr;
  size_t batch_off = 0, batch_bytes = 0;
  // batch workspace set aside at admission for the grown set (active and
  // pending fits), so that the pending fits can always join
  bool have_res = false;
  size_t res_off = 0, res_bytes = 0;

  std::vector<std::thread> workers;
  std::thread dev, up;
};

namespace {

// Mark a request finished (lock held).
void finish_locked(cwb_server* s, Request* r, int status, const std::string& err) {
  r->status = status;
  r->err = err;
  r->stage = Stage::kDone;
  r->t_done = now_s();
  r->hf = HostFit();
  if (status == CWB_OK) {
    s->completed += 1;
    s->latencies.push_back(r->t_done - r->t_submit);
    s->t_last_done = r->t_done;
    s->sum_setup_s += r->setup_s;
    s->sum_queue_s += r->t_admit > 0 ? r->t_admit - r->t_submit : 0.0;
  } else {
    s->rejected += 1;
  }
}

void setup_worker(cwb_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_setup.wait(lk, [&] { return s->stop || !s->setup_q.empty(); });
      if (s->setup_q.empty()) return;  // stopping
      r = s->setup_q.front();
      s->setup_q.pop_front();
      r->stage = Stage::kSetup;
    }
    std::string err;
    int rc = CWB_OK;
    size_t fp = 0;
    const double t0 = now_s();
    try {
      rc = shape_from_problem(&r->pr, &r->shape, &err);
      if (!rc) {
        const bool device_ok = !r->shape.unbinned && r->shape.n < (int64_t)INT32_MAX;
        if (r->pr.setup < CWB_SETUP_AUTO || r->pr.setup > CWB_SETUP_DEVICE) {
          rc = CWB_E_INVALID_ARG;
          err = "unknown setup mode";
        } else if (r->pr.setup == CWB_SETUP_DEVICE && !device_ok) {
          rc = CWB_E_UNSUPPORTED;
          err = "device setup covers binned fits with n < 2^31";
        } else {
          r->dev_setup = r->pr.setup == CWB_SETUP_DEVICE ||
                         (r->pr.setup == CWB_SETUP_AUTO && device_ok);
        }
      }
      if (!rc) rc = r->dev_setup ? prepare_host_fit(&r->pr, &r->hf, &err)
                                 : build_host_fit(&r->pr, &r->hf, &err);
      if (!rc) {
        rc = fit_footprint(r->shape, &fp, false);
        if (rc) err = cwb_last_error();
      }
    } catch (const std::bad_alloc&) {
      rc = CWB_E_NO_MEMORY;
      err = "host allocation failed during setup";
    } catch (...) {
      rc = CWB_E_INVALID_ARG;
      err = "unexpected error during setup";
    }
    r->setup_s = now_s() - t0;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!rc) {
      size_t bb = 0;
      std::vector<const FitShape*> one{&r->shape};
      if (batch_footprint(one, &bb, false) || fp + bb + 512 > s->arena.size()) {
        rc = CWB_E_NO_MEMORY;
        err = "request needs " + std::to_string(fp + bb) + " device bytes, arena holds " +
              std::to_string(s->arena.size());
      }
    }
    if (rc) {
      finish_locked(s, r, rc, err);
      continue;
    }
    r->footprint = fp;
    r->stage = Stage::kReady;
    s->ready_q.push_back(r);
    s->cv_dev.notify_one();
  }
}

// Retire a fit whose iterations are done (device thread; the round's stream
// is idle).  Returns the request's status.
int retire(cwb_server* s, Request* r) {
  cwb_fit* f = r->fit;
  std::string err;
  int rc = cwb_fit_sync(f);
  if (!rc) {
    r->M = f->shape.M;
    r->k.resize((size_t)r->M);
    rc = cwb_fit_get_trace(f, r->k.data(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr);
  }
  if (!rc) {
    r->pred.resize((size_t)f->shape.n);
    rc = cwb_fit_get_pred(f, r->pred.data());
  }
  if (rc) err = cwb_last_error();
  r->intercept = f->f0;
  cwb_fit_destroy(f);
  r->fit = nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  s->arena.release(r->off, r->footprint);
  s->in_flight -= 1;
  finish_locked(s, r, rc, err);
  return rc;
}

// Drop a fit from the device after an error (device thread).
void fail_fit(cwb_server* s, Request* r, int status, const std::string& err) {
  if (r->fit) cwb_fit_destroy(r->fit);
  r->fit = nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  s->arena.release(r->off, r->footprint);
  s->in_flight -= 1;
  finish_locked(s, r, status, err);
}

// Replace the batch by one over the active fits.  The old batch is never run
// again once a fit it covers has retired, so it is destroyed first.  The new
// batch workspace is a fresh allocation, else the admission reservation; the
// reservation is spent or released once no admitted fit is pending.  If
// neither holds the new set, the fits that have just joined (`joined`) wait
// for a later round and the batch covers the others; only when nothing else
// runs are they failed.
void rebuild_batch(cwb_server* s, std::vector<Request*> joined) {
  if (s->batch) {
    cwb_batch_destroy(s->batch);
    s->batch = nullptr;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->batch_bytes) s->arena.release(s->batch_off, s->batch_bytes);
    s->batch_bytes = 0;
  }
  std::vector<const FitShape*> shapes;
  std::vector<cwb_fit*> fits;
  for (Request* r : s->active) {
    shapes.push_back(&r->fit->shape);
    fits.push_back(r->fit);
  }
  size_t need = 0;
  int rc = fits.empty() ? CWB_OK : batch_footprint(shapes, &need, false);
  size_t off = 0;
  bool ok = false;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!rc && !fits.empty()) {
      if (s->have_res && s->pending.empty() && need <= s->res_bytes) {
        off = s->res_off;
        need = s->res_bytes;
        s->have_res = false;
        ok = true;
      } else {
        ok = s->arena.alloc(need, &off);
        if (!ok && s->have_res && need <= s->res_bytes) {
          off = s->res_off;
          need = s->res_bytes;
          s->have_res = false;
          ok = true;
        }
      }
      if (ok) {
        s->batch_off = off;
        s->batch_bytes = need;
      }
    }
    if (s->have_res && s->pending.empty()) {
      s->arena.release(s->res_off, s->res_bytes);
      s->have_res = false;
    }
  }
  if (fits.empty()) return;
  if (!rc && !ok && !joined.empty() && joined.size() < s->active.size()) {
    // no room with the newcomers: they wait (still admitted) for a later round
    std::vector<Request*> keep;
    for (Request* r : s->active)
      if (std::find(joined.begin(), joined.end(), r) == joined.end()) keep.push_back(r);
    s->active.swap(keep);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (Request* r : joined) r->stage = Stage::kAdmitted;
      s->uploaded.insert(s->uploaded.end(), joined.begin(), joined.end());
    }
    for (Request* r : joined) s->pending.push_back(r);
    rebuild_batch(s, {});
    return;
  }
  std::string err;
  if (rc) {
    err = cwb_last_error();
  } else if (!ok) {
    rc = CWB_E_NO_MEMORY;
    err = "no arena space for the batch workspace";
  } else {
    rc = batch_create(fits.data(), (int32_t)fits.size(), s->base + off, need, s->stream, false, &s->batch);
    if (rc) err = cwb_last_error();
  }
  if (rc) {  // the active fits cannot run: report the failure on each
    for (Request* r : s->active) fail_fit(s, r, rc, err);
    s->active.clear();
  }
}

// Upload thread: copies admitted fits into their arena space on the upload
// stream while the rounds go on.
void upload_worker(cwb_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_up.wait(lk, [&] { return s->stop_up || !s->upload_q.empty(); });
      if (s->upload_q.empty()) return;  // stopping
      r = s->upload_q.front();
      s->upload_q.pop_front();
    }
    cwb_fit* f = nullptr;
    int rc = CWB_OK;
    std::string err;
    const double t0 = now_s();
    try {
      rc = fit_upload(r->shape, r->hf, s->base + r->off, r->footprint, s->upload, false, &f,
                      r->dev_setup ? &r->pr : nullptr);
      if (rc) err = cwb_last_error();
    } catch (const std::bad_alloc&) {
      rc = set_error(CWB_E_NO_MEMORY, "host allocation failed during upload");
      err = cwb_last_error();
    } catch (...) {
      rc = set_error(CWB_E_DEVICE, "unexpected error during upload");
      err = cwb_last_error();
    }
    r->hf = HostFit();
    if (!rc) f->stream = s->stream;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      r->setup_s += now_s() - t0;
      r->fit = rc ? nullptr : f;
      if (rc) {
        r->status = rc;
        r->err = err;
      }
      s->uploaded.push_back(r);
    }
    s->cv_dev.notify_one();
  }
}

void device_loop(cwb_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    // 1. admission, in arrival order, while slots and arena space last: each
    //    admitted fit's workspace, and the batch workspace of the grown set
    //    (active and pending fits) as the new reservation
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_dev.wait(lk, [&] {
        if (!s->active.empty() || !s->uploaded.empty()) return true;
        return s->pending.empty() && (s->stop || !s->ready_q.empty());
      });
      if (s->stop && s->active.empty() && s->pending.empty() && s->uploaded.empty()) break;
      std::vector<const FitShape*> shapes;
      for (Request* r : s->active) shapes.push_back(&r->fit->shape);
      for (Request* r : s->pending) shapes.push_back(&r->shape);
      const int free_slots =
          s->stop ? 0 : s->cfg.max_slots - (int)(s->active.size() + s->pending.size());
      // the batch workspace of the set grown by r, or kNoFit
      auto batch_need = [&](Request* r) -> size_t {
        shapes.push_back(&r->shape);
        size_t bb = 0;
        const int rc = batch_footprint(shapes, &bb, false);
        shapes.pop_back();
        return rc ? kNoFit : bb;
      };
      auto admit = [&](Request* r, size_t off) {
        shapes.push_back(&r->shape);
        r->off = off;
        r->stage = Stage::kAdmitted;
        r->t_admit = now_s();
        s->in_flight += 1;
        s->pending.push_back(r);
        s->upload_q.push_back(r);
      };
      Reservation res{s->have_res, s->res_off, s->res_bytes};
      const int any = admit_in_order(s->ready_q, free_slots, s->arena, res, batch_need, admit);
      s->have_res = res.have;
      s->res_off = res.off;
      s->res_bytes = res.bytes;
      if (any) s->cv_up.notify_one();
    }
    // 2. one round of the current batch
    int32_t q = 0;
    const double t_round = now_s();
    if (s->batch && !s->active.empty()) {
      q = s->cfg.quantum;
      for (Request* r : s->active) q = std::min(q, r->fit->shape.M - r->fit->iters);
      q = std::max(q, 1);
      if (cwb_batch_run(s->batch, q)) {
        const std::string e = cwb_last_error();
        for (Request* r : s->active) r->status = CWB_E_DEVICE, r->err = e;
      }
    }
    // 3. end of the round: retire finished or failed fits
    if (q > 0) {
      (void)hipStreamSynchronize(s->stream);
      const double t_end = now_s();
      std::lock_guard<std::mutex> lk(s->mu);
      s->round_s += t_end - t_round;
      if (s->t_first_round < 0) s->t_first_round = t_round;
      s->t_last_round = t_end;
      s->rounds += 1;
    }
    bool changed = false;
    std::vector<Request*> keep;
    for (Request* r : s->active) {
      if (r->status != CWB_OK) {
        fail_fit(s, r, r->status, r->err);
        changed = true;
      } else if (r->fit->iters >= r->fit->shape.M) {
        retire(s, r);
        changed = true;
      } else {
        keep.push_back(r);
      }
    }
    s->active.swap(keep);
    // 4. uploaded fits join (their uploads are complete: fit_upload waits)
    std::vector<Request*> got, joined;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      got.swap(s->uploaded);
    }
    for (Request* r : got) {
      const auto pos = std::find(s->pending.begin(), s->pending.end(), r);
      if (pos != s->pending.end()) s->pending.erase(pos);
      changed = true;
      if (r->status != CWB_OK) {
        fail_fit(s, r, r->status, r->err);
        continue;
      }
      {
        std::lock_guard<std::mutex> lk(s->mu);
        r->stage = Stage::kRunning;
      }
      s->active.push_back(r);
      joined.push_back(r);
    }
    // 5. a new batch whenever the membership changed
    if (changed) rebuild_batch(s, joined);
  }
  if (s->batch) {
    cwb_batch_destroy(s->batch);
    s->batch = nullptr;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->batch_bytes) s->arena.release(s->batch_off, s->batch_bytes);
  s->batch_bytes = 0;
  if (s->have_res) s->arena.release(s->res_off, s->res_bytes);
  s->have_res = false;
}

}  // namespace

extern "C" {

int cwb_server_create(const cwb_server_cfg* cfg, cwb_server** out) {
  if (!out) return set_error(CWB_E_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!cfg) return set_error(CWB_E_INVALID_ARG, "null configuration");
  if (!cfg->arena || reinterpret_cast<uintptr_t>(cfg->arena) % 256 != 0)
    return set_error(CWB_E_INVALID_ARG, "arena must be non-null and 256-byte aligned");
  if (cfg->arena_bytes < (1u << 20)) return set_error(CWB_E_INVALID_ARG, "arena below 1 MiB");
  if (cfg->max_slots < 1 || cfg->max_slots > 4096)
    return set_error(CWB_E_INVALID_ARG, "max_slots must be 1..4096");
  if (cfg->quantum < 1) return set_error(CWB_E_INVALID_ARG, "quantum must be >= 1");
  if (cfg->setup_threads < 0 || cfg->setup_threads > 64)
    return set_error(CWB_E_INVALID_ARG, "setup_threads must be 0..64");
  try {
    std::unique_ptr<cwb_server> s(new cwb_server());
    s->cfg = *cfg;
    s->base = static_cast<char*>(cfg->arena);
    s->stream = static_cast<hipStream_t>(cfg->stream);
    s->arena.reset(cfg->arena_bytes);
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking);
    if (e != hipSuccess) return set_error(CWB_E_DEVICE, std::string("server streams: ") + hipGetErrorString(e));
    const int nw = cfg->setup_threads > 0 ? cfg->setup_threads : 4;
    cwb_server* sp = s.get();
    for (int i = 0; i < nw; ++i) s->workers.emplace_back(setup_worker, sp);
    s->up = std::thread(upload_worker, sp);
    s->dev = std::thread(device_loop, sp);
    *out = s.release();
    return CWB_OK;
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed");
  } catch (const std::exception& ex) {
    return set_error(CWB_E_INVALID_ARG, ex.what());
  }
}

int cwb_server_submit(cwb_server* s, const cwb_problem* pr, uint64_t* ticket) {
  if (!s || !pr || !ticket) return set_error(CWB_E_INVALID_ARG, "null argument");
  if (!pr->x || !pr->y || !pr->specs) return set_error(CWB_E_INVALID_ARG, "null problem array");
  FitShape sh;
  std::string err;
  int rc = shape_from_problem(pr, &sh, &err);
  if (!rc && sh.unbinned) {
    rc = CWB_E_UNSUPPORTED;
    err = "the server batches binned fits only";
  }
  if (rc) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->rejected += 1;
    return set_error(rc, err);
  }
  try {
    std::unique_ptr<Request> r(new Request());
    r->specs.assign(pr->specs, pr->specs + pr->p);
    r->pr = *pr;  // x, y and val_mask stay the caller's until the result is polled
    r->pr.specs = r->specs.data();
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_error(CWB_E_STATE, "server is stopping");
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    if (s->t_first < 0) s->t_first = r->t_submit;
    s->submitted += 1;
    s->setup_q.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
    s->cv_setup.notify_one();
    return CWB_OK;
  } catch (const std::bad_alloc&) {
    return set_error(CWB_E_NO_MEMORY, "host allocation failed copying the request");
  }
}

int cwb_server_poll(cwb_server* s, uint64_t ticket, cwb_result* res, float* pred_out, int32_t* k_out) {
  if (!s || !res) return set_error(CWB_E_INVALID_ARG, "null argument");
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(CWB_E_INVALID_ARG, "unknown ticket (or already collected)");
    if (it->second->stage != Stage::kDone) return CWB_E_AGAIN;
    r = std::move(it->second);
    s->reqs.erase(it);
  }
  std::memset(res, 0, sizeof(*res));
  res->status = r->status;
  res->M = r->M;
  res->latency_s = r->t_done - r->t_submit;
  res->queue_s = r->t_admit > 0 ? r->t_admit - r->t_submit : 0.0;
  res->intercept = r->intercept;
  if (r->status == CWB_OK) {
    if (pred_out && !r->pred.empty()) std::memcpy(pred_out, r->pred.data(), r->pred.size() * 4);
    if (k_out && !r->k.empty()) std::memcpy(k_out, r->k.data(), r->k.size() * 4);
    return CWB_OK;
  }
  set_error(r->status, r->err);
  return CWB_OK;
}

int cwb_server_stats(cwb_server* s, cwb_stats* st) {
  if (!s || !st) return set_error(CWB_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(st, 0, sizeof(*st));
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->rejected = s->rejected;
  st->in_flight = s->in_flight;
  st->queued = (int32_t)(s->setup_q.size() + s->ready_q.size());
  const double span = s->t_last_done - s->t_first;
  st->fits_per_s = (s->completed > 0 && span > 0) ? (double)s->completed / span : 0.0;
  if (!s->latencies.empty()) {
    std::vector<double> v = s->latencies;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * v.size()) - 1);
      return v[i];
    };
    st->p50_latency_s = pct(0.50);
    st->p99_latency_s = pct(0.99);
  }
  st->arena_in_use = s->arena.in_use;
  st->arena_peak = s->arena.peak;
  if (s->completed > 0) {
    st->mean_setup_s = s->sum_setup_s / (double)s->completed;
    st->mean_queue_s = s->sum_queue_s / (double)s->completed;
  }
  st->round_s = s->round_s;
  st->busy_s = s->t_first_round >= 0 ? s->t_last_round - s->t_first_round : 0.0;
  st->rounds = s->rounds;
  return CWB_OK;
}

void cwb_server_destroy(cwb_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // requests not yet admitted are cancelled
    for (Request* r : s->setup_q) finish_locked(s, r, CWB_E_STATE, "server stopped");
    s->setup_q.clear();
    for (Request* r : s->ready_q) finish_locked(s, r, CWB_E_STATE, "server stopped");
    s->ready_q.clear();
  }
  s->cv_setup.notify_all();
  s->cv_dev.notify_all();
  for (auto& t : s->workers) t.join();
  // a worker may have queued a request after the cancellation above
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Request* r : s->ready_q) finish_locked(s, r, CWB_E_STATE, "server stopped");
    s->ready_q.clear();
  }
  s->cv_dev.notify_all();
  if (s->dev.joinable()) s->dev.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop_up = true;
  }
  s->cv_up.notify_all();
  if (s->up.joinable()) s->up.join();
  if (s->upload) (void)hipStreamDestroy(s->upload);
  delete s;
}

}  // extern "C"

// Stub executor for the fit server's admission policy (admission.h): a byte
// budget (the arena), a mock clock and requests that each run for a given
// number of ticks.  No device is involved.  Input lines, one case each:
//   S arena_bytes slots batch_per_fit n  footprint_1 ticks_1 ... footprint_n ticks_n
//     a stream: every request is ready at tick 0, in this order; a set of k
//     fits needs a batch workspace of k * batch_per_fit bytes.  Prints, for
//     every request, its admit tick and finish tick (-1: never admitted),
//     then "|", the arena's peak use, 1 if it ended empty, 1 if the stream
//     stalled (nothing running and the head of the queue never fits).
//   A arena_bytes n  op_1 ... op_n
//     arena operations: a positive op allocates that many bytes, a negative
//     op -k releases the k-th allocation (1-based).  Prints the offset of
//     every allocation (-1 when it failed) and the bytes in use at the end.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <vector>

#include "../paper_2110_03513_amd/csrc/admission.h"

struct Req {
  size_t footprint = 0;
  int ticks = 0;
  size_t off = 0;
  long admit_t = -1, done_t = -1;
};

static bool read_size(size_t* v) { return std::scanf("%zu", v) == 1; }
static bool read_int(long* v) { return std::scanf("%ld", v) == 1; }

static int stream_case() {
  size_t arena_bytes, per_fit, slots_u, n_u;
  if (!read_size(&arena_bytes) || !read_size(&slots_u) || !read_size(&per_fit) || !read_size(&n_u))
    return 1;
  const int slots = (int)slots_u;
  std::vector<Req> reqs(n_u);
  for (Req& r : reqs) {
    size_t f, k;
    if (!read_size(&f) || !read_size(&k)) return 1;
    r.footprint = f;
    r.ticks = (int)k;
  }
  cwb::Arena arena;
  arena.reset(arena_bytes);
  cwb::Reservation res;
  std::deque<Req*> ready;
  for (Req& r : reqs) ready.push_back(&r);
  std::vector<Req*> active;
  long t = 0;
  bool stalled = false;
  while ((!ready.empty() || !active.empty()) && t < 100000) {
    size_t set = active.size();
    auto need = [&](Req*) { return (set + 1) * per_fit; };
    auto admit = [&](Req* r, size_t off) {
      r->off = off;
      r->admit_t = t;
      active.push_back(r);
      ++set;
    };
    cwb::admit_in_order(ready, slots - (int)active.size(), arena, res, need, admit);
    if (active.empty()) {
      stalled = true;
      break;
    }
    ++t;  // one tick of work; finished requests retire and free their space
    std::vector<Req*> keep;
    for (Req* r : active) {
      if (t - r->admit_t >= r->ticks) {
        r->done_t = t;
        arena.release(r->off, r->footprint);
      } else {
        keep.push_back(r);
      }
    }
    active.swap(keep);
    if (active.empty() && res.have) {  // the reservation ends with the set
      arena.release(res.off, res.bytes);
      res.have = false;
    }
  }
  for (const Req& r : reqs) std::printf("%ld %ld ", r.admit_t, r.done_t);
  std::printf("| %zu %d %d\n", arena.peak, arena.in_use == 0 ? 1 : 0, stalled ? 1 : 0);
  return 0;
}

static int arena_case() {
  size_t bytes, n;
  if (!read_size(&bytes) || !read_size(&n)) return 1;
  cwb::Arena arena;
  arena.reset(bytes);
  std::vector<size_t> off, size;
  std::vector<int> live;
  for (size_t i = 0; i < n; ++i) {
    long op;
    if (!read_int(&op)) return 1;
    if (op > 0) {
      size_t o = 0;
      const bool ok = arena.alloc((size_t)op, &o);
      off.push_back(ok ? o : ~size_t(0));
      size.push_back((size_t)op);
      live.push_back(ok ? 1 : 0);
      std::printf("%ld ", ok ? (long)o : -1L);
    } else {
      const size_t k = (size_t)(-op) - 1;
      if (k < off.size() && live[k]) {
        arena.release(off[k], size[k]);
        live[k] = 0;
      }
    }
  }
  std::printf("| %zu\n", arena.in_use);
  return 0;
}

int main() {
  char kind[4];
  while (std::scanf("%3s", kind) == 1) {
    const int rc = (kind[0] == 'S') ? stream_case() : (kind[0] == 'A') ? arena_case() : 1;
    if (rc) return rc;
    std::fflush(stdout);
  }
  return 0;
}

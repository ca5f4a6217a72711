// admission.h -- host-side admission policy of the fit server (server.cpp),
// free of any device call so that it can be exercised against a stub
// executor on the CPU.
//
// The server's device memory is one caller-owned arena.  Each admitted fit
// holds its workspace in it, and the server reserves the batch workspace of
// the set it would run (the active and admitted fits) so that the next
// batch rebuild finds room.  Requests are admitted strictly in arrival
// order: the first request that does not fit stops admission, so a large
// request is never overtaken by smaller ones (no starvation).
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>

namespace cwb {

// First-fit allocator over [0, size) in 256-byte units; neighbouring free
// ranges are merged on release.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    size_ = bytes / 256 * 256;
    if (size_) free_[0] = size_;
    in_use = peak = 0;
  }
  size_t size() const { return size_; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = std::max<size_t>(256, (bytes + 255) / 256 * 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      in_use += bytes;
      peak = std::max(peak, in_use);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = std::max<size_t>(256, (bytes + 255) / 256 * 256);
    in_use -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t in_use = 0, peak = 0;

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0;
};

// A reserved range of the arena (the batch workspace of the admitted set).
struct Reservation {
  bool have = false;
  size_t off = 0, bytes = 0;
};

constexpr size_t kNoFit = ~size_t(0);  // a set that no batch workspace can hold

// Admit requests from the front of `ready`, in order, while fewer than
// `free_slots` have been admitted and the arena holds both the request's
// workspace (r->footprint bytes) and the batch workspace of the set grown by
// it (batch_need(r), or kNoFit).  The batch workspace becomes the new
// reservation (the previous one is released); admit(r, off) receives each
// admitted request with the offset of its workspace.  Returns the number
// admitted.
template <class R, class Need, class Admit>
int admit_in_order(std::deque<R*>& ready, int free_slots, Arena& arena, Reservation& res,
                   Need batch_need, Admit admit) {
  int n = 0;
  while (n < free_slots && !ready.empty()) {
    R* r = ready.front();
    const size_t bb = batch_need(r);
    size_t off = 0, boff = 0;
    bool ok = bb != kNoFit && arena.alloc(r->footprint, &off);
    if (ok && !arena.alloc(bb, &boff)) {
      arena.release(off, r->footprint);
      ok = false;
    }
    if (!ok) break;  // first come, first served: later requests wait too
    if (res.have) arena.release(res.off, res.bytes);
    res.have = true;
    res.off = boff;
    res.bytes = bb;
    ready.pop_front();
    admit(r, off);
    ++n;
  }
  return n;
}

}  // namespace cwb

// Device memory arena of a context: the bookkeeping of live, pending and
// kept blocks, with the device operations supplied by a policy class, so
// that the library instantiates it with HIP's allocator (runtime.h) and the
// CPU tests with a fake one (tests/cpu/arena_fake_test.cpp).  No HIP here.
//
// Blocks that jobs release are kept, by size, and handed out again to
// requests of that size (or up to 1/8 smaller): repeated registrations of
// similar jobs then make no device allocation, whose cost grows with the
// size of the request (seconds for the tens of GB of a large batch).  A
// released block may still be in use by work in flight (a device free would
// have waited for it), so released blocks wait in a pending list until the
// next request that would reuse one, which first synchronises the device.
// Kept blocks count against the budget: they are returned to the device
// before a new allocation would exceed it, when an allocation fails (every
// arena's kept blocks, then one retry), by trim() and on destruction.
//
// Dev provides:
//   static bool alloc(size_t bytes, void** p);  // false when the device is full
//   static void free(void* p);                  // waits for work in flight
//   static void sync(int device);               // waits for the device's work
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <mutex>
#include <set>
#include <utility>
#include <vector>

namespace muster {

template <class Dev>
class BasicArena {
 public:
  BasicArena(uint64_t budget, int device) : budget_(budget), device_(device) {
    std::lock_guard<std::mutex> lk(registry_mu());
    registry().insert(this);
  }
  ~BasicArena() {
    {
      std::lock_guard<std::mutex> lk(registry_mu());
      registry().erase(this);
    }
    trim();
  }
  BasicArena(const BasicArena&) = delete;
  BasicArena& operator=(const BasicArena&) = delete;

  // Returns nullptr (no throw) when the budget or the device is full.
  void* try_alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    for (int attempt = 0; attempt < 2; ++attempt) {
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (budget_ && used_ + bytes > budget_) return nullptr;
        if (void* p = take_kept(bytes)) return p;
        if (budget_ && used_ + kept_ + bytes > budget_) free_kept(budget_ - used_ - bytes);
        void* p = nullptr;
        if (Dev::alloc(bytes, &p) && p) {
          live_[p] = bytes;
          used_ += bytes;
          peak_ = std::max(peak_, used_);
          return p;
        }
        if (attempt == 1) return nullptr;
        free_kept(0);
      }
      trim_others();
    }
    return nullptr;
  }

  void release(void* p) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    used_ -= it->second;
    pending_.emplace_back(it->second, p);
    kept_ += it->second;
    live_.erase(it);
  }

  // Returns the kept blocks to the device; the bytes returned.
  uint64_t trim() {
    std::lock_guard<std::mutex> lk(mu_);
    return free_kept(0);
  }

  uint64_t used() const { return used_; }
  uint64_t kept() const { return kept_; }
  uint64_t budget() const { return budget_; }
  // Largest used() since the arena was made or the mark was last reset.
  uint64_t peak() const { return peak_; }
  void reset_peak() {
    std::lock_guard<std::mutex> lk(mu_);
    peak_ = used_;
  }
  bool fits(uint64_t bytes) const { return budget_ == 0 || used_ + bytes <= budget_; }

 private:
  // every arena of the process (of this policy), so that an allocation that
  // fails can first take back what the others keep
  static std::mutex& registry_mu() {
    static std::mutex m;
    return m;
  }
  static std::set<BasicArena*>& registry() {
    static std::set<BasicArena*> s;
    return s;
  }
  void trim_others() {
    std::vector<BasicArena*> all;
    {
      std::lock_guard<std::mutex> lk(registry_mu());
      all.assign(registry().begin(), registry().end());
    }
    // one arena lock at a time (never two), after the registry lock is dropped
    for (BasicArena* a : all)
      if (a != this) a->trim();
  }

  // under mu_: a kept block for a request of `bytes`, or nullptr
  void* take_kept(size_t bytes) {
    auto it = free_.lower_bound(bytes);
    const bool fit = it != free_.end() && it->first <= bytes + bytes / 8;
    if (!fit && !pending_.empty()) {
      // released blocks become reusable once the device has finished the
      // work that may still read or write them
      Dev::sync(device_);
      for (const auto& e : pending_) free_.emplace(e.first, e.second);
      pending_.clear();
      it = free_.lower_bound(bytes);
    }
    if (it == free_.end() || it->first > bytes + bytes / 8) return nullptr;
    if (budget_ && used_ + it->first > budget_) return nullptr;
    void* p = it->second;
    const size_t sz = it->first;
    free_.erase(it);
    kept_ -= sz;
    live_[p] = sz;
    used_ += sz;
    peak_ = std::max(peak_, used_);
    return p;
  }

  // under mu_: frees kept blocks (pending first: a device free waits for the
  // work in flight; then the largest) until kept_ <= target
  uint64_t free_kept(uint64_t target) {
    uint64_t freed = 0;
    while (kept_ > target && !pending_.empty()) {
      Dev::free(pending_.back().second);
      kept_ -= pending_.back().first;
      freed += pending_.back().first;
      pending_.pop_back();
    }
    while (kept_ > target && !free_.empty()) {
      auto it = std::prev(free_.end());
      Dev::free(it->second);
      kept_ -= it->first;
      freed += it->first;
      free_.erase(it);
    }
    return freed;
  }

  std::mutex mu_;
  uint64_t budget_;
  int device_;
  uint64_t used_ = 0;
  uint64_t kept_ = 0;  // pending_ and free_
  uint64_t peak_ = 0;
  std::map<void*, size_t> live_;
  std::vector<std::pair<size_t, void*>> pending_;  // released since the last device sync
  std::multimap<size_t, void*> free_;              // safe to hand out
};

}  // namespace muster

// Per-kernel timing with HIP events recorded on the library's stream.
#pragma once

#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"

namespace ic {

class KernelTimer {
 public:
  struct Scope {
    KernelTimer* t = nullptr;
    size_t idx = 0;
    Scope() = default;
    Scope(KernelTimer* tt, size_t i) : t(tt), idx(i) {}
    Scope(const Scope&) = delete;
    Scope(Scope&& o) noexcept : t(o.t), idx(o.idx) { o.t = nullptr; }
    ~Scope() {
      if (t) (void)hipEventRecord(t->recs_[idx].stop, t->stream_);
    }
  };

  void set_stream(hipStream_t s) { stream_ = s; }
  bool enabled() const { return on_; }
  // True while every kernel is recorded (no single-kernel filter).
  bool all() const { return on_ && only_.empty(); }

  // Starts (resetting the records) or stops recording.  A non-empty only
  // restricts recording to the kernels of that name, so the timed code runs
  // with two events per such launch and nothing else added.
  void enable(bool on, const std::string& only = std::string()) {
    on_ = on;
    only_ = on ? only : std::string();
    if (on) used_ = 0, recs_used_ = 0;
  }

  Scope scope(const char* name, double bytes) {
    if (!on_ || (!only_.empty() && only_ != name)) return Scope();
    if (recs_used_ == recs_.size()) {
      Rec r;
      IC_HIP(hipEventCreate(&r.start));
      IC_HIP(hipEventCreate(&r.stop));
      recs_.push_back(r);
    }
    Rec& r = recs_[recs_used_];
    r.name = name;
    r.bytes = bytes;
    IC_HIP(hipEventRecord(r.start, stream_));
    return Scope(this, recs_used_++);
  }

  // "name count total_ms bytes_per_launch" per kernel, in first-seen order.
  std::string report() {
    IC_HIP(hipStreamSynchronize(stream_));
    struct Agg {
      long count = 0;
      double ms = 0, bytes = 0;
      size_t first = 0;
    };
    std::map<std::string, Agg> agg;
    for (size_t i = 0; i < recs_used_; ++i) {
      float ms = 0;
      IC_HIP(hipEventElapsedTime(&ms, recs_[i].start, recs_[i].stop));
      auto it = agg.find(recs_[i].name);
      if (it == agg.end()) it = agg.emplace(recs_[i].name, Agg{0, 0, 0, i}).first;
      it->second.count += 1;
      it->second.ms += ms;
      it->second.bytes = recs_[i].bytes;
    }
    std::vector<std::pair<std::string, Agg>> v(agg.begin(), agg.end());
    std::sort(v.begin(), v.end(),
              [](const auto& a, const auto& b) { return a.second.first < b.second.first; });
    std::ostringstream os;
    os.precision(9);
    for (auto& kv : v)
      os << kv.first << " " << kv.second.count << " " << kv.second.ms << " " << kv.second.bytes
         << "\n";
    return os.str();
  }

  ~KernelTimer() {
    for (auto& r : recs_) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.stop);
    }
  }

 private:
  struct Rec {
    std::string name;
    double bytes = 0;
    hipEvent_t start = nullptr, stop = nullptr;
  };
  bool on_ = false;
  std::string only_;
  hipStream_t stream_ = nullptr;
  std::vector<Rec> recs_;
  size_t recs_used_ = 0, used_ = 0;
};

}  // namespace ic

// agg_policy.hpp -- when to launch aggregated batches of sub-grid tasks.
//
// This is the explicit work aggregation of the paper (Section V-D, strategy
// 3), written as a small policy with no GPU dependency: tasks that arrive
// while the device is busy are held back and launched together as one batch
// (one kernel per shape class) when
//   * the batch reaches the maximum width W (the paper's "max aggregated
//     kernels" parameter; W = 1 disables aggregation), or
//   * a stream (the paper's executor) becomes idle -- aggregation only
//     happens while the device is busy -- if flush_when_idle is set, or
//   * the oldest held task has waited `timeout_us`, or
//   * the caller flushes, or a task with a different (dt, dx) arrives.
// Admission is bounded by a byte budget: the output bytes of held and
// in-flight tasks may not exceed it (HYDRO_EAGAIN otherwise; the caller
// retries after progress).
//
// The policy drives an Executor and reads a Clock, both template parameters,
// so the same code runs on HIP streams in the library and on a fake executor
// with a virtual clock in the CPU tests.  Not thread-safe: the C ABI wraps it
// in a mutex.
//
// Executor interface:
//   int  streams() const;
//   bool idle(int stream);                     // nothing of ours in flight
//   int  launch(int stream, const Task* t, int n, double dt, double dx,
//               uint64_t batch);               // async; 0 or error code
//   bool done(uint64_t batch);                 // non-blocking
//   int  wait(uint64_t batch);                 // blocking; 0 or error code
//   void results(uint64_t batch, double* amax);// after done: n values
//   void release(uint64_t batch);
// Clock: double now_us();
#pragma once

#include <stdint.h>

#include <deque>
#include <unordered_map>
#include <vector>

namespace hydro {

struct Task {
  const double* u_in;
  double* u_out;
  int32_t n, nfields, level;
  uint64_t ticket;
  uint64_t bytes;
  double t_submit;
  int32_t out_layout = 0;  // HYDRO_OUT_STORED or HYDRO_OUT_INTERIOR
};

struct AggStats {
  uint64_t submitted = 0, launched_batches = 0, launched_tasks = 0;
  uint64_t flush_width = 0, flush_idle = 0, flush_timeout = 0, flush_manual = 0,
           flush_param = 0;
  uint64_t refused = 0;
  uint64_t width_hist[11] = {0};  // batches of width 1, 2-3, 4-7, ..., >= 1024
};

enum FlushWhy { kWidth, kIdle, kTimeout, kManual, kParam };

template <class Exec, class Clock>
class AggPolicy {
 public:
  AggPolicy(Exec& ex, Clock& clk, int max_width, double timeout_us, uint64_t budget,
            bool flush_when_idle)
      : ex_(ex), clk_(clk), W_(max_width), timeout_(timeout_us), budget_(budget),
        idle_flush_(flush_when_idle) {}

  // Queue one task; may launch.  Returns 0, HYDRO-style negative codes.  A
  // task submitted with `forget` keeps no completion record: its ticket is
  // unknown once its batch has been collected (fire-and-forget tasks whose
  // completion the caller learns from drain()).
  int submit(const Task& t_in, double dt, double dx, uint64_t* ticket, bool forget = false) {
    if (!pending_.empty() && (dt != dt_ || dx != dx_)) {
      int rc = launch_pending(kParam);
      if (rc) return rc;
    }
    if (budget_ && held_bytes_ + t_in.bytes > budget_) {
      stats_.refused++;
      return -4;  // HYDRO_EAGAIN
    }
    Task t = t_in;
    t.ticket = next_ticket_++;
    t.t_submit = clk_.now_us();
    if (pending_.empty()) {
      dt_ = dt;
      dx_ = dx;
    }
    pending_.push_back(t);
    held_bytes_ += t.bytes;
    state_[t.ticket] = Where{kPendingBatch, 0, 0.0, forget};
    stats_.submitted++;
    *ticket = t.ticket;
    if ((int)pending_.size() >= W_) return launch_pending(kWidth);
    if (idle_flush_ && pick_idle() >= 0) return launch_pending(kIdle);
    return 0;
  }

  // Launch whatever is held now.
  int flush() { return pending_.empty() ? 0 : launch_pending(kManual); }

  // Collect finished batches; launch on timeout or idle stream.
  int progress() {
    collect();
    if (pending_.empty()) return 0;
    if (timeout_ >= 0 && clk_.now_us() - pending_.front().t_submit >= timeout_)
      return launch_pending(kTimeout);
    if (idle_flush_ && pick_idle() >= 0) return launch_pending(kIdle);
    return 0;
  }

  // done = 1 and amax once the task's batch has completed.
  int poll(uint64_t ticket, int* done, double* amax) {
    int rc = progress();
    if (rc) return rc;
    auto it = state_.find(ticket);
    if (it == state_.end()) return -1;  // unknown or already retrieved
    if (it->second.kind != kDone) {
      *done = 0;
      return 0;
    }
    *done = 1;
    if (amax) *amax = it->second.amax;
    state_.erase(it);
    return 0;
  }

  int wait(uint64_t ticket, double* amax) {
    auto it = state_.find(ticket);
    if (it == state_.end()) return -1;
    if (it->second.kind == kPendingBatch) {
      int rc = launch_pending(kManual);
      if (rc) return rc;
      it = state_.find(ticket);
    }
    if (it->second.kind == kInFlight) {
      int rc = ex_.wait(it->second.batch);
      if (rc) return rc;
      collect();
      it = state_.find(ticket);
    }
    if (it == state_.end() || it->second.kind != kDone) return -2;
    if (amax) *amax = it->second.amax;
    state_.erase(it);
    return 0;
  }

  // Launch held tasks and wait for everything in flight.
  int drain() {
    int rc = flush();
    if (rc) return rc;
    while (!inflight_.empty()) {
      rc = ex_.wait(inflight_.front().batch);
      if (rc) return rc;
      collect();
    }
    return 0;
  }

  // Completed (ticket, amax) pairs are also queued here when enabled; the
  // owner takes them with take_completed() and must then not poll/wait them.
  void record_completions(bool on) { record_ = on; }
  void take_completed(std::vector<std::pair<uint64_t, double>>& out) {
    out.clear();
    out.swap(completed_);
    for (auto& c : out) state_.erase(c.first);
  }

  bool quiescent() const { return pending_.empty() && inflight_.empty(); }
  size_t held() const { return pending_.size(); }
  size_t in_flight_batches() const { return inflight_.size(); }
  uint64_t held_bytes() const { return held_bytes_; }
  const AggStats& stats() const { return stats_; }

 private:
  enum Kind { kPendingBatch, kInFlight, kDone };
  struct Where {
    Kind kind;
    uint64_t batch;
    double amax = 0.0;
    bool forget = false;
  };
  struct Batch {
    uint64_t batch;
    int stream;
    std::vector<uint64_t> tickets;
    uint64_t bytes;
  };

  int pick_idle() {
    const int ns = ex_.streams();
    for (int k = 0; k < ns; ++k) {
      const int s = (rr_ + k) % ns;
      if (ex_.idle(s)) return s;
    }
    return -1;
  }

  int launch_pending(FlushWhy why) {
    if (pending_.empty()) return 0;
    int s = pick_idle();
    if (s < 0) {
      s = rr_;  // all busy: queue behind the next stream in turn
    }
    rr_ = (s + 1) % ex_.streams();
    const uint64_t b = next_batch_++;
    int rc = ex_.launch(s, pending_.data(), (int)pending_.size(), dt_, dx_, b);
    if (rc) return rc;
    Batch rec{b, s, {}, 0};
    for (const Task& t : pending_) {
      rec.tickets.push_back(t.ticket);
      rec.bytes += t.bytes;
      Where& w = state_[t.ticket];
      w.kind = kInFlight;
      w.batch = b;
    }
    const int w = (int)pending_.size();
    int bin = 0;
    while (bin < 10 && (2 << bin) <= w) ++bin;
    stats_.width_hist[bin]++;
    stats_.launched_batches++;
    stats_.launched_tasks += w;
    switch (why) {
      case kWidth: stats_.flush_width++; break;
      case kIdle: stats_.flush_idle++; break;
      case kTimeout: stats_.flush_timeout++; break;
      case kManual: stats_.flush_manual++; break;
      case kParam: stats_.flush_param++; break;
    }
    inflight_.push_back(std::move(rec));
    pending_.clear();
    return 0;
  }

  void collect() {
    // Batches on one stream finish in order, across streams in any order:
    // once a batch is found unfinished, later batches of its stream are not
    // polled.
    uint64_t blocked[2] = {0, 0};   // streams 0..127
    for (auto it = inflight_.begin(); it != inflight_.end();) {
      const int sb = it->stream & 127;
      const uint64_t bit = 1ull << (sb & 63);
      if ((blocked[sb >> 6] & bit) || !ex_.done(it->batch)) {
        blocked[sb >> 6] |= bit;
        ++it;
        continue;
      }
      amax_buf_.resize(it->tickets.size());
      ex_.results(it->batch, amax_buf_.data());
      for (size_t i = 0; i < it->tickets.size(); ++i) {
        auto st = state_.find(it->tickets[i]);
        if (st != state_.end() && st->second.forget) {
          state_.erase(st);
          continue;
        }
        if (st != state_.end()) st->second = Where{kDone, it->batch, amax_buf_[i]};
        if (record_) completed_.emplace_back(it->tickets[i], amax_buf_[i]);
      }
      held_bytes_ -= it->bytes;
      ex_.release(it->batch);
      it = inflight_.erase(it);
    }
  }

  Exec& ex_;
  Clock& clk_;
  int W_;
  double timeout_;
  uint64_t budget_;
  bool idle_flush_;
  std::vector<Task> pending_;
  double dt_ = 0.0, dx_ = 1.0;
  std::deque<Batch> inflight_;
  std::unordered_map<uint64_t, Where> state_;
  std::vector<double> amax_buf_;
  uint64_t held_bytes_ = 0;
  uint64_t next_ticket_ = 1, next_batch_ = 1;
  int rr_ = 0;
  bool record_ = false;
  std::vector<std::pair<uint64_t, double>> completed_;
  AggStats stats_;
};

}  // namespace hydro

// region_core.hpp -- the aggregation region of the paper's explicit work
// aggregation executor (Section V-D), independent of the hydro kernels.
//
// A region is a piece of task code -- staging buffers, filling them, a kernel
// launch, copies back -- that several tasks may run together as one team.
// A task that reaches the region enters it (enter()):
//   * at once, as a team of its own plus whoever is waiting, when one of the
//     region's executors (streams) is idle (no team inside the region on it);
//   * otherwise it waits until an executor becomes idle, or until max_team
//     tasks are waiting, which then enter as one team whether an executor is
//     idle or not: the team queues its work behind the team already on an
//     executor (there are two team slots per executor, each with its own
//     arena, so one team can fill its buffers while the other's kernels run).
// Inside the region every member makes the same sequence of calls ("single
// GPU workload, multiple tasks"):
//   * alloc(bytes): the k-th allocation of every member is one buffer of the
//     team: the first member to arrive reserves size x stride bytes of the
//     executor's arena (device memory with a host mirror), the member with
//     index j gets the chunk at j x stride (stride = bytes rounded up to 8,
//     so a buffer of 8-byte-aligned records is a plain array of them);
//   * upload(buffer) / launch(kernel, ...) / download(buffer): counted; the
//     operation runs once, on the team's executor, when the last member has
//     called it (so every member has filled its chunk before the upload);
//     a launch's grid is size x blocks_per_task work-groups and its
//     arguments are those of the last caller (they name team buffers, which
//     are the same for every member);
//   * wait(): the last member records the team's completion on the
//     executor; every member returns when the team's device work is done.
//     Its downloaded chunks are then valid until it leaves; only leave()
//     may follow;
//   * leave(): as wait() if the team has not recorded its completion yet;
//     when the last member has left, the team's slot (and its arena) may be
//     reused by the next team.
// A member whose k-th call differs from the team's k-th operation (another
// kind or size) is an error (kMismatch), as is an arena overflow (kNoSpace):
// either fails the whole team -- every member's later calls return that
// error and nothing more is launched for it -- and wakes the members waiting
// in wait() or leave().  Every member must still call leave() once, which frees the
// team's slot when the last one has.
//
// Exec (the HIP streams in region_api.hip, a fake in the CPU test); team
// slot k runs on executor k % streams() and owns arena k:
//   int  streams() const;
//   char* arena_host(int k); char* arena_dev(int k); uint64_t arena_bytes() const;
//   int  upload(int k, uint64_t off, uint64_t bytes);     // host mirror -> device
//   int  download(int k, uint64_t off, uint64_t bytes);   // device -> host mirror
//   int  launch(int k, const void* kernel, unsigned blocks, unsigned threads,
//               unsigned shmem, void** args);
//   int  record(int k, uint64_t team);   // completion marker of the team
//   int  wait(int k, uint64_t team);     // until that marker has passed
#pragma once

#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <vector>

namespace hydro {

enum RegionRc { kRegionOk = 0, kMismatch = -1, kNoSpace = -3 };

struct RegionTask {
  int32_t team;    // team slot (its arena; executor team % streams)
  int32_t index;   // position in the team, 0..size-1
  int32_t size;    // members of the team
  int32_t stream;  // the team's executor
  uint64_t id;     // team serial number
};

struct RegionStats {
  uint64_t tasks = 0, teams = 0, full_teams = 0, uploads = 0, launches = 0, downloads = 0;
  uint64_t size_hist[11] = {0};   // teams of size 1, 2-3, 4-7, ..., >= 1024
};

template <class Exec>
class RegionCore {
 public:
  enum Kind { kAlloc, kUpload, kLaunch, kDownload, kWait, kLeave };

  static constexpr int kSlotsPerStream = 2;

  RegionCore(Exec& ex, int max_team) : ex_(ex), max_team_(max_team) {
    slots_.resize((size_t)ex_.streams() * kSlotsPerStream);
  }

  int enter(RegionTask* out) {
    std::unique_lock<std::mutex> lk(mu_);
    const uint64_t me = next_waiter_++;
    waiting_.push_back(me);
    for (;;) {
      auto it = seat_.find_seat(me);
      if (it >= 0) {
        *out = seat_.take(it);
        return kRegionOk;
      }
      try_form();
      if (seat_.find_seat(me) >= 0) continue;
      // wait for an executor to become idle or the team to fill up; idle
      // is polled (device completion does not signal this condition)
      cv_.wait_for(lk, std::chrono::microseconds(20));
    }
  }

  int alloc(const RegionTask& t, uint64_t bytes, int32_t* buffer, char** host, char** dev) {
    std::lock_guard<std::mutex> lk(mu_);
    if (!valid(t)) return kMismatch;
    Team& tm = slots_[t.team];
    Op* op = next_op(tm, t, kAlloc, bytes);
    if (!op) return tm.err;
    if (op->arrived == 1) {
      const uint64_t stride = (bytes + 7) / 8 * 8;
      const uint64_t base = (tm.used + 255) / 256 * 256;
      if (base + stride * tm.size > ex_.arena_bytes()) {
        fail_team(tm, kNoSpace);
        return kNoSpace;
      }
      op->off = base;
      op->stride = stride;
      tm.used = base + stride * tm.size;
      op->buffer = tm.nbuf++;
      tm.buf_off.push_back(base);
      tm.buf_bytes.push_back(stride * tm.size);
    }
    *buffer = op->buffer;
    *host = ex_.arena_host(t.team) + op->off + t.index * op->stride;
    *dev = ex_.arena_dev(t.team) + op->off + t.index * op->stride;
    return kRegionOk;
  }

  // Device base and stride of a team buffer (for kernel arguments).
  int buffer(const RegionTask& t, int32_t b, char** dev_base, uint64_t* stride) {
    std::lock_guard<std::mutex> lk(mu_);
    if (!valid(t)) return kMismatch;
    Team& tm = slots_[t.team];
    if (tm.err) return tm.err;
    if (b < 0 || b >= tm.nbuf) return kMismatch;
    *dev_base = ex_.arena_dev(t.team) + tm.buf_off[b];
    *stride = tm.buf_bytes[b] / tm.size;
    return kRegionOk;
  }

  int upload(const RegionTask& t, int32_t b) { return transfer(t, b, kUpload); }
  int download(const RegionTask& t, int32_t b) { return transfer(t, b, kDownload); }

  int launch(const RegionTask& t, const void* kernel, unsigned blocks_per_task, unsigned threads,
             unsigned shmem, void** args) {
    std::lock_guard<std::mutex> lk(mu_);
    if (!valid(t)) return kMismatch;
    Team& tm = slots_[t.team];
    Op* op = next_op(tm, t, kLaunch, ((uint64_t)blocks_per_task << 32) | threads);
    if (!op) return tm.err;
    if (op->arrived < tm.size) return kRegionOk;
    stats_.launches++;
    return ex_.launch(t.team, kernel, blocks_per_task * (unsigned)tm.size, threads, shmem, args);
  }

  int wait(const RegionTask& t) {
    std::unique_lock<std::mutex> lk(mu_);
    if (!valid(t)) return kMismatch;
    return complete(lk, slots_[t.team], t, kWait);
  }

  int leave(const RegionTask& t) {
    std::unique_lock<std::mutex> lk(mu_);
    if (!valid(t)) return kMismatch;
    Team& tm = slots_[t.team];
    const int rc = complete(lk, tm, t, kLeave);
    if (++tm.left == tm.size) {
      tm.active = false;   // slot reusable: its device work is done
      cv_.notify_all();
    }
    return rc;
  }

  RegionStats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    return stats_;
  }

 private:
  struct Op {
    Kind kind;
    uint64_t arg;
    int arrived = 0;
    int32_t buffer = -1;
    uint64_t off = 0, stride = 0;
  };
  struct Team {
    bool active = false;
    uint64_t id = 0;
    int size = 0, stream = 0, nbuf = 0, left = 0;
    int err = kRegionOk;   // the team's failure, if any
    bool recorded = false;
    bool waiting = false, done = false;   // one member waits on the executor
    int wait_rc = kRegionOk;
    uint64_t used = 0;
    std::vector<Op> ops;
    std::vector<int> next;   // next op index of each member
    std::vector<uint64_t> buf_off, buf_bytes;
  };
  // Seats handed to waiting tasks when their team forms.
  struct Seats {
    std::vector<std::pair<uint64_t, RegionTask>> v;
    long find_seat(uint64_t w) const {
      for (size_t i = 0; i < v.size(); ++i)
        if (v[i].first == w) return (long)i;
      return -1;
    }
    RegionTask take(long i) {
      RegionTask t = v[i].second;
      v.erase(v.begin() + i);
      return t;
    }
  };

  // A handle names a seated member of the team now in its slot.
  bool valid(const RegionTask& t) const {
    if (t.team < 0 || t.team >= (int)slots_.size()) return false;
    const Team& tm = slots_[t.team];
    return tm.active && t.id == tm.id && t.index >= 0 && t.index < tm.size;
  }

  void fail_team(Team& tm, int err) {
    if (!tm.err) tm.err = err;
    tm.recorded = true;   // nothing more will be recorded; wake leave()
    cv_.notify_all();
  }

  // The member's next operation must be the team's operation of that
  // position (created by the first member to get there); otherwise the team
  // fails.  nullptr when the team has failed.
  Op* next_op(Team& tm, const RegionTask& t, Kind k, uint64_t arg) {
    const int pos = tm.next[t.index]++;
    if (tm.err) return nullptr;
    if (tm.recorded && k != kLeave) {   // only leave() follows the completion
      fail_team(tm, kMismatch);
      return nullptr;
    }
    if (pos == (int)tm.ops.size()) tm.ops.push_back(Op{k, arg});
    Op& op = tm.ops[pos];
    if (op.kind != k || op.arg != arg) {
      fail_team(tm, kMismatch);
      return nullptr;
    }
    op.arrived++;
    return &op;
  }

  // wait() and leave(): the last member to arrive records the team's
  // completion (unless a wait() already has).  One member then waits for it
  // on the executor; the others wait for that member (one runtime wait per
  // team, not one per member).  Under mu_ (released while waiting).
  int complete(std::unique_lock<std::mutex>& lk, Team& tm, const RegionTask& t, Kind k) {
    Op* op = next_op(tm, t, k, 0);
    int rc = op ? kRegionOk : tm.err;
    if (op && op->arrived == tm.size && !tm.recorded) {
      rc = ex_.record(t.team, tm.id);
      tm.recorded = true;
      cv_.notify_all();
    }
    while (!tm.recorded) cv_.wait(lk);
    if (!tm.err && !tm.done) {
      if (!tm.waiting) {
        tm.waiting = true;
        const uint64_t id = tm.id;
        lk.unlock();
        const int w = ex_.wait(t.team, id);
        lk.lock();
        tm.wait_rc = w;
        tm.done = true;
        cv_.notify_all();
      } else {
        while (!tm.done) cv_.wait(lk);
      }
    }
    if (!rc) rc = tm.err ? tm.err : tm.wait_rc;
    return rc;
  }

  int transfer(const RegionTask& t, int32_t b, Kind k) {
    std::lock_guard<std::mutex> lk(mu_);
    if (!valid(t)) return kMismatch;
    Team& tm = slots_[t.team];
    Op* op = next_op(tm, t, k, (uint64_t)b);
    if (!op) return tm.err;
    if (b < 0 || b >= tm.nbuf) {
      fail_team(tm, kMismatch);
      return kMismatch;
    }
    if (op->arrived < tm.size) return kRegionOk;
    if (k == kUpload) {
      stats_.uploads++;
      return ex_.upload(t.team, tm.buf_off[b], tm.buf_bytes[b]);
    }
    stats_.downloads++;
    return ex_.download(t.team, tm.buf_off[b], tm.buf_bytes[b]);
  }

  // Form a team of the waiting tasks if an executor is idle (no team inside
  // the region on it), or, when max_team tasks wait, in any free team slot
  // (behind the team of its executor); under mu_.
  void try_form() {
    if (waiting_.empty()) return;
    const int ns = ex_.streams();
    int k = -1;
    for (int s = 0; s < ns && k < 0; ++s) {
      bool busy = false;
      int free_slot = -1;
      for (int j = s; j < (int)slots_.size(); j += ns) {
        if (slots_[j].active) busy = true;
        else if (free_slot < 0) free_slot = j;
      }
      if (!busy) k = free_slot;
    }
    if (k < 0 && (int)waiting_.size() >= max_team_) {
      for (int j = 0; j < (int)slots_.size() && k < 0; ++j)
        if (!slots_[j].active) k = j;
    }
    if (k < 0) return;
    Team& tm = slots_[k];
    const int m = (int)waiting_.size() < max_team_ ? (int)waiting_.size() : max_team_;
    tm = Team();
    tm.active = true;
    tm.id = ++team_serial_;
    tm.size = m;
    tm.stream = k % ns;
    tm.next.assign(m, 0);
    for (int j = 0; j < m; ++j) {
      seat_.v.emplace_back(waiting_.front(), RegionTask{k, j, m, tm.stream, tm.id});
      waiting_.pop_front();
    }
    stats_.tasks += m;
    stats_.teams++;
    if (m == max_team_) stats_.full_teams++;
    int bin = 0;
    while (bin < 10 && (2 << bin) <= m) ++bin;
    stats_.size_hist[bin]++;
    cv_.notify_all();
  }

  Exec& ex_;
  int max_team_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<uint64_t> waiting_;
  Seats seat_;
  std::vector<Team> slots_;
  uint64_t next_waiter_ = 0, team_serial_ = 0;
  RegionStats stats_;
};

}  // namespace hydro

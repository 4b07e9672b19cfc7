// CPU test of the aggregation region (paper Section V-D: tasks entering a
// region together share buffers chunk by chunk; the first member allocates,
// the last member's call launches) with a fake executor and real threads.
// Built with g++ by test_region_core_cpu.py.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <future>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "../paper_2210_06438_amd/csrc/region_core.hpp"

using hydro::RegionCore;
using hydro::RegionTask;

static std::atomic<int> g_fail{0};
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);         \
      g_fail++;                                                   \
    }                                                             \
  } while (0)

struct Call {
  char what;   // 'u' upload, 'd' download, 'l' launch, 'r' record
  int slot;
  uint64_t a, b;
};

struct FakeExec {
  int ns = 1;
  uint64_t bytes = 1 << 16;
  std::vector<std::vector<char>> host, dev;
  std::mutex mu;
  std::vector<Call> calls;
  explicit FakeExec(int nstreams, uint64_t arena = 1 << 16) : ns(nstreams), bytes(arena) {
    host.assign(ns * RegionCore<FakeExec>::kSlotsPerStream, std::vector<char>(arena));
    dev.assign(ns * RegionCore<FakeExec>::kSlotsPerStream, std::vector<char>(arena));
  }
  int streams() const { return ns; }
  char* arena_host(int k) { return host[k].data(); }
  char* arena_dev(int k) { return dev[k].data(); }
  uint64_t arena_bytes() const { return bytes; }
  void log(char w, int k, uint64_t a, uint64_t b) {
    std::lock_guard<std::mutex> lk(mu);
    calls.push_back({w, k, a, b});
  }
  // the "device": copies between the mirrors, a launch adds 1 to every
  // 8-byte word of the buffer at offset 0 per block (blocks = team x per task)
  int upload(int k, uint64_t off, uint64_t n) {
    memcpy(dev[k].data() + off, host[k].data() + off, n);
    log('u', k, off, n);
    return 0;
  }
  int download(int k, uint64_t off, uint64_t n) {
    memcpy(host[k].data() + off, dev[k].data() + off, n);
    log('d', k, off, n);
    return 0;
  }
  int launch(int k, const void*, unsigned blocks, unsigned threads, unsigned, void** args) {
    const uint64_t words = *(uint64_t*)args[0];
    uint64_t* p = (uint64_t*)dev[k].data();
    for (uint64_t i = 0; i < words; ++i) p[i] += 1000;
    log('l', k, blocks, threads);
    return 0;
  }
  int record(int k, uint64_t team) {
    log('r', k, team, 0);
    return 0;
  }
  int wait(int, uint64_t) { return 0; }
};

using R = RegionCore<FakeExec>;

// One task through the whole region: its chunk holds (its value, 0); after
// the team's launch, download and wait it must read (value + 1000, 1000).
static int run_task(R& r, uint64_t value, RegionTask* seat, std::promise<void>* hold = nullptr,
                    std::shared_future<void>* gate = nullptr) {
  RegionTask t;
  if (r.enter(&t)) return -100;
  if (seat) *seat = t;
  if (hold) hold->set_value();
  if (gate) gate->wait();
  int32_t b;
  char *h, *d;
  int rc = r.alloc(t, 16, &b, &h, &d);
  if (rc) return rc;
  ((uint64_t*)h)[0] = value;
  ((uint64_t*)h)[1] = 0;
  if ((rc = r.upload(t, b))) return rc;
  char* base;
  uint64_t stride;
  if ((rc = r.buffer(t, b, &base, &stride))) return rc;
  uint64_t words = (uint64_t)t.size * stride / 8;
  void* args[1] = {&words};
  if ((rc = r.launch(t, nullptr, 3, 64, 0, args))) return rc;
  if ((rc = r.download(t, b))) return rc;
  if ((rc = r.wait(t))) return rc;
  CHECK(((uint64_t*)h)[0] == value + 1000 && ((uint64_t*)h)[1] == 1000);
  if ((rc = r.leave(t))) return rc;
  CHECK(stride == 16);
  CHECK(d == base + t.index * 16);
  return 0;
}

static void single_task() {
  FakeExec ex(1);
  R r(ex, 8);
  RegionTask t;
  CHECK(run_task(r, 7, &t) == 0);
  CHECK(t.size == 1 && t.index == 0);
  // upload, launch (3 blocks of 64), download, record (at wait): once each
  CHECK(ex.calls.size() == 4);
  CHECK(ex.calls[0].what == 'u' && ex.calls[0].a == 0 && ex.calls[0].b == 16);
  CHECK(ex.calls[1].what == 'l' && ex.calls[1].a == 3 && ex.calls[1].b == 64);
  CHECK(ex.calls[2].what == 'd' && ex.calls[3].what == 'r');
  hydro::RegionStats s = r.stats();
  CHECK(s.tasks == 1 && s.teams == 1 && s.launches == 1 && s.uploads == 1);
}

// The first task finds the executor idle and enters alone; it holds its
// seat while 8 more arrive: the first 4 of them fill a team (max_team 4)
// that enters behind it in the executor's second slot; the last 4 wait for
// a free slot and form the third team.  Every operation runs once per team
// with the team's size.
static void teams_from_threads() {
  FakeExec ex(1);
  R r(ex, 4);
  std::promise<void> seated, release;
  std::shared_future<void> gate = release.get_future().share();
  RegionTask first;
  std::thread t0([&] { CHECK(run_task(r, 100, &first, &seated, &gate) == 0); });
  seated.get_future().wait();
  std::vector<std::thread> ts;
  std::vector<RegionTask> seats(8);
  for (int i = 0; i < 8; ++i) {
    ts.emplace_back([&, i] { CHECK(run_task(r, 200 + i, &seats[i]) == 0); });
  }
  // wait until the full team of four has been seated (tasks = 1 + 4)
  for (int spin = 0; spin < 20000 && r.stats().tasks < 5; ++spin)
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  CHECK(r.stats().tasks >= 5);
  release.set_value();
  t0.join();
  for (auto& t : ts) t.join();
  hydro::RegionStats s = r.stats();
  CHECK(first.size == 1);
  CHECK(s.tasks == 9);
  CHECK(s.launches == s.teams && s.uploads == s.teams && s.downloads == s.teams);
  CHECK(s.full_teams >= 1);
  std::set<std::pair<uint64_t, int>> distinct;
  int total = first.size;
  std::set<uint64_t> ids;
  for (auto& q : seats) {
    distinct.insert({q.id, q.index});
    ids.insert(q.id);
    CHECK(q.size >= 1 && q.size <= 4 && q.index < q.size);
  }
  CHECK(distinct.size() == 8);
  for (uint64_t id : ids) {
    for (auto& q : seats)
      if (q.id == id) {
        total += q.size;
        break;
      }
  }
  CHECK(total == 9);
  // every launch covers 3 blocks per member of its team
  for (auto& c : ex.calls)
    if (c.what == 'l') CHECK(c.a % 3 == 0 && c.a / 3 <= 4);
}

// Two members that allocate different sizes fail their team; both get the
// error, both leave, and the region keeps serving new tasks.
static void mismatch_fails_the_team() {
  FakeExec ex(1);
  R r(ex, 2);
  std::promise<void> s0;
  std::shared_future<void> go;
  std::atomic<int> rc0{1}, rc1{1}, l0{1}, l1{1};
  RegionTask a, b;
  // both arrive before the executor frees: hold the executor with a task
  std::promise<void> holder_seated, holder_release;
  std::shared_future<void> hgate = holder_release.get_future().share();
  std::thread h([&] { CHECK(run_task(r, 1, nullptr, &holder_seated, &hgate) == 0); });
  holder_seated.get_future().wait();
  std::thread t0([&] {
    CHECK(r.enter(&a) == 0);
    int32_t bb;
    char *x, *y;
    rc0 = r.alloc(a, 32, &bb, &x, &y);
    l0 = r.leave(a);
  });
  std::thread t1([&] {
    CHECK(r.enter(&b) == 0);
    int32_t bb;
    char *x, *y;
    rc1 = r.alloc(b, 64, &bb, &x, &y);
    l1 = r.leave(b);
  });
  for (int spin = 0; spin < 20000 && r.stats().tasks < 3; ++spin)
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  holder_release.set_value();
  h.join();
  t0.join();
  t1.join();
  CHECK(a.id == b.id && a.size == 2);
  // one of the two allocations came second and differs: the team failed
  CHECK((rc0 == 0) != (rc1 == 0));
  CHECK(rc0 == hydro::kMismatch || rc1 == hydro::kMismatch);
  CHECK(l0 == hydro::kMismatch && l1 == hydro::kMismatch);
  RegionTask t;
  CHECK(run_task(r, 5, &t) == 0);   // slot freed
}

// Chunks of 8-byte records are a plain array of them (stride 8); other
// sizes round up to a multiple of 8.
static void chunk_strides() {
  FakeExec ex(1);
  R r(ex, 4);
  RegionTask t;
  CHECK(r.enter(&t) == 0);
  int32_t b;
  char *h, *d, *base;
  uint64_t stride;
  CHECK(r.alloc(t, 8, &b, &h, &d) == 0 && r.buffer(t, b, &base, &stride) == 0 && stride == 8);
  CHECK(r.alloc(t, 12, &b, &h, &d) == 0 && r.buffer(t, b, &base, &stride) == 0 && stride == 16);
  CHECK(((uintptr_t)(base - ex.arena_dev(t.team))) % 256 == 0);
  CHECK(r.leave(t) == 0);
}

// wait() records the completion once; leave() after it records nothing
// more; any other call after wait() fails the team.
static void wait_then_leave() {
  FakeExec ex(1);
  R r(ex, 4);
  RegionTask t;
  CHECK(r.enter(&t) == 0);
  int32_t b;
  char *h, *d;
  CHECK(r.alloc(t, 8, &b, &h, &d) == 0);
  CHECK(r.wait(t) == 0);
  CHECK(r.leave(t) == 0);
  int records = 0;
  for (auto& c : ex.calls) records += c.what == 'r';
  CHECK(records == 1);
  RegionTask u;
  CHECK(r.enter(&u) == 0);
  CHECK(r.alloc(u, 8, &b, &h, &d) == 0);
  CHECK(r.wait(u) == 0);
  CHECK(r.download(u, b) == hydro::kMismatch);   // after the completion marker
  CHECK(r.leave(u) == hydro::kMismatch);
  CHECK(run_task(r, 3, &t) == 0);                 // slot freed
}

static void arena_overflow() {
  FakeExec ex(1, 1024);
  R r(ex, 4);
  RegionTask t;
  CHECK(r.enter(&t) == 0);
  int32_t b;
  char *h, *d;
  CHECK(r.alloc(t, 2048, &b, &h, &d) == hydro::kNoSpace);
  CHECK(r.upload(t, 0) == hydro::kNoSpace);
  CHECK(r.leave(t) == hydro::kNoSpace);
  CHECK(run_task(r, 9, &t) == 0);
  RegionTask stale = t;
  CHECK(r.leave(stale) == hydro::kMismatch);   // a handle of a team that has left
}

int main() {
  single_task();
  teams_from_threads();
  mismatch_fails_the_team();
  chunk_strides();
  wait_then_leave();
  arena_overflow();
  if (g_fail) {
    printf("%d checks failed\n", (int)g_fail);
    return 1;
  }
  printf("all region checks passed\n");
  return 0;
}

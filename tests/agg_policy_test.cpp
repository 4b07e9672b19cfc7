// CPU test of the aggregation policy (paper Section V-D semantics) with a
// fake executor and a virtual clock.  Built with g++ by test_agg_policy_cpu.py.
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <vector>

#include "../paper_2210_06438_amd/csrc/agg_policy.hpp"

using hydro::AggPolicy;
using hydro::Task;

static int g_fail = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);         \
      g_fail++;                                                   \
    }                                                             \
  } while (0)

struct VClock {
  double t = 0.0;
  double now_us() { return t; }
};

// Batches stay in flight until the test completes them.
struct FakeExec {
  int ns = 1;
  struct B {
    int stream;
    std::vector<Task> tasks;
    double dt, dx;
    bool done = false;
  };
  std::map<uint64_t, B> b;
  std::vector<uint64_t> order;
  int fail_next = 0;
  int streams() const { return ns; }
  bool idle(int s) {
    for (auto& kv : b)
      if (kv.second.stream == s && !kv.second.done) return false;
    return true;
  }
  int launch(int s, const Task* t, int n, double dt, double dx, uint64_t id) {
    if (fail_next) return fail_next;
    B x;
    x.stream = s;
    x.tasks.assign(t, t + n);
    x.dt = dt;
    x.dx = dx;
    b[id] = x;
    order.push_back(id);
    return 0;
  }
  bool done(uint64_t id) { return b.at(id).done; }
  // A stream runs its batches in order: waiting for one also completes every
  // earlier batch of its stream.
  int wait(uint64_t id) {
    const int s = b.at(id).stream;
    for (auto& kv : b)
      if (kv.first <= id && kv.second.stream == s) kv.second.done = true;
    return 0;
  }
  void results(uint64_t id, double* amax) {
    B& x = b.at(id);
    for (size_t i = 0; i < x.tasks.size(); ++i) amax[i] = x.tasks[i].level + 0.5;
  }
  void release(uint64_t id) { b.erase(id); }
  void complete_all() {
    for (auto& kv : b) kv.second.done = true;
  }
  int width(uint64_t id) { return (int)b.at(id).tasks.size(); }
};

static Task task(int id, uint64_t bytes = 100) {
  Task t;
  t.u_in = nullptr;
  t.u_out = nullptr;
  t.n = 8;
  t.nfields = 11;
  t.level = id;
  t.ticket = 0;
  t.bytes = bytes;
  t.t_submit = 0;
  return t;
}

using P = AggPolicy<FakeExec, VClock>;

static void width_rule() {
  FakeExec ex;
  VClock clk;
  P p(ex, clk, 4, -1.0, 0, false);
  uint64_t tk[10];
  for (int i = 0; i < 10; ++i) CHECK(p.submit(task(i), 0.1, 1.0, &tk[i]) == 0);
  CHECK(ex.order.size() == 2);
  CHECK(ex.width(ex.order[0]) == 4 && ex.width(ex.order[1]) == 4);
  CHECK(p.held() == 2);
  CHECK(p.flush() == 0);
  CHECK(ex.order.size() == 3 && ex.width(ex.order[2]) == 2);
  CHECK(p.stats().flush_width == 2 && p.stats().flush_manual == 1);
  // tickets map to their own results, in order
  ex.complete_all();
  for (int i = 0; i < 10; ++i) {
    int done = 0;
    double am = -1;
    CHECK(p.poll(tk[i], &done, &am) == 0);
    CHECK(done == 1 && am == i + 0.5);
    CHECK(p.poll(tk[i], &done, &am) == -1);  // retrieved once
  }
  CHECK(p.quiescent());
}

static void idle_rule() {
  // the paper's rule: aggregate only while the executor is busy
  FakeExec ex;
  VClock clk;
  P p(ex, clk, 64, -1.0, 0, true);
  uint64_t t0, t;
  CHECK(p.submit(task(0), 0.1, 1.0, &t0) == 0);
  CHECK(ex.order.size() == 1 && ex.width(ex.order[0]) == 1);  // idle: goes at once
  for (int i = 1; i <= 5; ++i) CHECK(p.submit(task(i), 0.1, 1.0, &t) == 0);
  CHECK(ex.order.size() == 1 && p.held() == 5);                 // busy: held
  CHECK(p.progress() == 0 && ex.order.size() == 1);
  ex.complete_all();
  CHECK(p.progress() == 0);                                     // stream idle again
  CHECK(ex.order.size() == 2 && ex.width(ex.order[1]) == 5);
  CHECK(p.stats().flush_idle == 2);
}

static void timeout_rule() {
  FakeExec ex;
  VClock clk;
  P p(ex, clk, 8, 50.0, 0, false);
  uint64_t t;
  clk.t = 10.0;
  CHECK(p.submit(task(0), 0.1, 1.0, &t) == 0);
  clk.t = 30.0;
  CHECK(p.submit(task(1), 0.1, 1.0, &t) == 0);
  clk.t = 59.0;
  CHECK(p.progress() == 0 && ex.order.empty());
  clk.t = 60.0;  // the oldest has waited 50 us
  CHECK(p.progress() == 0 && ex.order.size() == 1 && ex.width(ex.order[0]) == 2);
  CHECK(p.stats().flush_timeout == 1);
}

static void budget_rule() {
  FakeExec ex;
  VClock clk;
  P p(ex, clk, 2, -1.0, 300, false);
  uint64_t t;
  CHECK(p.submit(task(0, 100), 0.1, 1.0, &t) == 0);
  CHECK(p.submit(task(1, 100), 0.1, 1.0, &t) == 0);  // batch of 2 launched
  CHECK(p.submit(task(2, 100), 0.1, 1.0, &t) == 0);
  CHECK(p.submit(task(3, 100), 0.1, 1.0, &t) == -4);  // 400 > 300: refused
  CHECK(p.stats().refused == 1 && p.held() == 1);
  ex.complete_all();
  CHECK(p.progress() == 0);                            // frees 200 bytes
  CHECK(p.submit(task(3, 100), 0.1, 1.0, &t) == 0);
  CHECK(p.held_bytes() == 200);
}

static void param_rule() {
  FakeExec ex;
  VClock clk;
  P p(ex, clk, 8, -1.0, 0, false);
  uint64_t t;
  CHECK(p.submit(task(0), 0.1, 1.0, &t) == 0);
  CHECK(p.submit(task(1), 0.1, 1.0, &t) == 0);
  CHECK(p.submit(task(2), 0.2, 1.0, &t) == 0);  // new dt: held batch goes first
  CHECK(ex.order.size() == 1 && ex.width(ex.order[0]) == 2);
  CHECK(ex.b.at(ex.order[0]).dt == 0.1);
  CHECK(p.flush() == 0 && ex.b.at(ex.order[1]).dt == 0.2);
}

static void streams_and_wait() {
  FakeExec ex;
  ex.ns = 2;
  VClock clk;
  P p(ex, clk, 3, -1.0, 0, true);
  uint64_t a, b, c;
  CHECK(p.submit(task(0), 0.1, 1.0, &a) == 0);  // stream 0 idle
  CHECK(p.submit(task(1), 0.1, 1.0, &b) == 0);  // stream 1 idle
  CHECK(ex.order.size() == 2);
  CHECK(ex.b.at(ex.order[0]).stream != ex.b.at(ex.order[1]).stream);
  CHECK(p.submit(task(2), 0.1, 1.0, &c) == 0);  // both busy: held
  CHECK(p.held() == 1);
  double am = 0;
  CHECK(p.wait(c, &am) == 0 && am == 2.5);      // wait flushes and completes
  CHECK(p.wait(c, &am) == -1);
  int done = 0;
  // c was queued behind a on stream 0, so a is done too; b (stream 1) is not
  CHECK(p.poll(a, &done, &am) == 0 && done == 1 && am == 0.5);
  CHECK(p.poll(b, &done, &am) == 0 && done == 0);
  CHECK(p.drain() == 0);
  CHECK(p.poll(b, &done, &am) == 0 && done == 1 && am == 1.5);
}

static void launch_error_keeps_tasks() {
  FakeExec ex;
  VClock clk;
  P p(ex, clk, 2, -1.0, 0, false);
  uint64_t t;
  CHECK(p.submit(task(0), 0.1, 1.0, &t) == 0);
  ex.fail_next = -2;
  CHECK(p.submit(task(1), 0.1, 1.0, &t) == -2);  // launch failed: error surfaces
  CHECK(p.held() == 2);                          // nothing lost
  ex.fail_next = 0;
  CHECK(p.flush() == 0 && ex.order.size() == 1 && ex.width(ex.order[0]) == 2);
}

static void completion_queue() {
  FakeExec ex;
  VClock clk;
  P p(ex, clk, 4, -1.0, 0, false);
  p.record_completions(true);
  uint64_t t[4];
  for (int i = 0; i < 4; ++i) CHECK(p.submit(task(10 + i), 0.1, 1.0, &t[i]) == 0);
  std::vector<std::pair<uint64_t, double>> done;
  CHECK(p.progress() == 0);
  p.take_completed(done);
  CHECK(done.empty());
  ex.complete_all();
  CHECK(p.progress() == 0);
  p.take_completed(done);
  CHECK(done.size() == 4);
  for (int i = 0; i < 4; ++i) CHECK(done[i].first == t[i] && done[i].second == 10 + i + 0.5);
}

// Fire-and-forget tasks keep no completion record once their batch is
// collected; tasks with tickets beside them are unaffected.  Streams beyond
// 32 (up to 128) are tracked separately when collecting.
static void forget_and_many_streams() {
  FakeExec ex;
  ex.ns = 40;
  VClock clk;
  P p(ex, clk, 2, -1.0, 0, false);
  uint64_t f[4], k;
  for (int i = 0; i < 4; ++i) CHECK(p.submit(task(i), 0.1, 1.0, &f[i], true) == 0);
  CHECK(p.submit(task(7), 0.1, 1.0, &k) == 0);
  CHECK(p.flush() == 0);
  CHECK(ex.order.size() == 3);   // widths 2, 2, 1 on streams 0, 1, 2
  int done = 0;
  double am = 0;
  CHECK(p.poll(f[0], &done, &am) == 0 && done == 0);   // still in flight: known
  CHECK(p.drain() == 0);
  for (int i = 0; i < 4; ++i) CHECK(p.poll(f[i], &done, &am) == -1);   // dropped
  CHECK(p.poll(k, &done, &am) == 0 && done == 1 && am == 7.5);
  CHECK(p.quiescent());
  // batches on streams 0 and 32 (same bit in a 32-bit mask): completing the
  // one on stream 32 must be collected while stream 0's is still running
  FakeExec ex2;
  ex2.ns = 40;
  VClock clk2;
  P q(ex2, clk2, 1, -1.0, 0, false);
  uint64_t t[40];
  for (int i = 0; i < 33; ++i) CHECK(q.submit(task(i), 0.1, 1.0, &t[i]) == 0);   // width 1
  CHECK(ex2.order.size() == 33 && ex2.b.at(ex2.order[32]).stream == 32);
  ex2.b.at(ex2.order[32]).done = true;
  CHECK(q.poll(t[32], &done, &am) == 0 && done == 1 && am == 32.5);
  CHECK(q.poll(t[0], &done, &am) == 0 && done == 0);
}

int main() {
  forget_and_many_streams();
  width_rule();
  idle_rule();
  timeout_rule();
  budget_rule();
  param_rule();
  streams_and_wait();
  launch_error_keeps_tasks();
  completion_queue();
  if (g_fail) {
    printf("%d checks failed\n", g_fail);
    return 1;
  }
  printf("all policy checks passed\n");
  return 0;
}

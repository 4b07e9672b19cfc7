// agg_api.hip -- the submit/flush aggregator on HIP streams, and a
// continuous-batching serving loop built on it.
//
// The aggregator (paper Section V-D, strategy 3) holds sub-grid tasks while
// its streams are busy and launches them as one batch (one multi-class
// kernel per field count) by the rules of agg_policy.hpp.  Every resource a
// batch needs -- a pinned descriptor table, a device descriptor table, a
// pinned array of amax partials, a pinned completion word -- comes from
// slots allocated at create time, as are the streams: nothing is allocated
// or created on the submit path (Section V-C).
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "agg_policy.hpp"
#include "internal.hpp"

using hydro::DevDesc;
using hydro::Task;
using hydro::api::fail;

namespace {

#define HIP_OK(expr)                                                         \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(HYDRO_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct SteadyClock {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};

// The most streams of one aggregator (the paper's largest executor count).
constexpr int kAggMaxStreams = 128;

// Executor on HIP streams.
class HipExec {
 public:
  int init(int nstreams, int width, int slots_per_stream) {
    ns_ = nstreams;
    cap_ = width;
    for (int s = 0; s < ns_; ++s) {
      HIP_OK(hipStreamCreateWithFlags(&streams_[s], hipStreamNonBlocking));
      created_ = s + 1;
    }
    slots_.resize((size_t)ns_ * slots_per_stream);
    HIP_OK(hipHostMalloc((void**)&flags_, sizeof(uint64_t) * slots_.size(), hipHostMallocDefault));
    for (size_t k = 0; k < slots_.size(); ++k) flags_[k] = 0;
    for (Slot& sl : slots_) {
      HIP_OK(hipHostMalloc((void**)&sl.htab, sizeof(DevDesc) * cap_, hipHostMallocDefault));
      HIP_OK(hipMalloc((void**)&sl.dtab, sizeof(DevDesc) * cap_));
      HIP_OK(hipHostMalloc((void**)&sl.hamax, sizeof(double) * cap_ * hydro::kAmaxParts,
                           hipHostMallocDefault));
      sl.parts.assign((size_t)cap_, 0);
      HIP_OK(hipHostGetDevicePointer((void**)&sl.hamax_dev, sl.hamax, 0));
    }
    return HYDRO_OK;
  }

  void teardown() {
    for (int s = 0; s < created_; ++s) (void)hipStreamSynchronize(streams_[s]);
    for (Slot& sl : slots_) {
      if (sl.htab) (void)hipHostFree(sl.htab);
      if (sl.hamax) (void)hipHostFree(sl.hamax);
      if (sl.dtab) (void)hipFree(sl.dtab);
    }
    slots_.clear();
    if (flags_) (void)hipHostFree(flags_);
    flags_ = nullptr;
    for (int s = 0; s < created_; ++s) (void)hipStreamDestroy(streams_[s]);
    created_ = 0;
  }

  int streams() const { return ns_; }
  hipStream_t stream(int s) const { return streams_[s]; }

  // A stream runs its batches in order, so it is idle once its newest batch
  // has finished (or was already collected).
  bool idle(int s) {
    const uint64_t b = last_[s];
    if (b == 0 || retired_.count(b)) return true;
    auto it = live_.find(b);
    return it == live_.end() || finished(it->second);
  }

  // Host time spent in launch() (descriptor packing and the runtime calls).
  double launch_us() const { return launch_us_; }

  int launch(int s, const Task* t, int n, double dt, double dx, uint64_t batch) {
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = launch_batch(s, t, n, dt, dx, batch);
    launch_us_ +=
        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    return rc;
  }

 private:
  int launch_batch(int s, const Task* t, int n, double dt, double dx, uint64_t batch) {
    if (n > cap_) return fail(HYDRO_ENOMEM, "batch of %d exceeds the width %d", n, cap_);
    int k = free_slot();
    if (k < 0) {
      int rc = retire_oldest();
      if (rc) return rc;
      k = free_slot();
      if (k < 0) return fail(HYDRO_ENOMEM, "no batch slot");
    }
    Slot& sl = slots_[k];
    int num[hydro::api::kNumClasses] = {0}, off[hydro::api::kNumClasses], fill[hydro::api::kNumClasses];
    for (int i = 0; i < n; ++i) num[hydro::api::class_of_task(t[i].n, t[i].nfields)]++;
    int pos = 0;
    for (int c = 0; c < hydro::api::kNumClasses; ++c) {
      off[c] = fill[c] = pos;
      pos += num[c];
    }
    for (int i = 0; i < n; ++i) {
      DevDesc& d = sl.htab[fill[hydro::api::class_of_task(t[i].n, t[i].nfields)]++];
      d.u_in = t[i].u_in;
      d.u_out = t[i].u_out;
      d.level = (int16_t)t[i].level;
      d.compact = (int16_t)(t[i].out_layout == HYDRO_OUT_INTERIOR);
      d.index = i;
    }
    hipStream_t st = streams_[s];
    // One launch per field count present (hydro_mixed.hpp: its classes side
    // by side), descriptors in the kernel arguments when every class has at
    // most kArgDescs, else in the slot's device table.  Every work-group
    // stores its amax partial straight into the slot's pinned host array
    // (device-accessible) with a plain store: no zeroing, no atomics, no
    // copy back; the completion word below is written after the kernels, so
    // the host reads the partials only after they finished.
    bool small = true;
    for (int c = 0; c < hydro::api::kNumClasses; ++c) small = small && num[c] <= hydro::kArgDescs;
    if (!small)
      HIP_OK(hipMemcpyAsync(sl.dtab, sl.htab, sizeof(DevDesc) * n, hipMemcpyHostToDevice, st));
    int groups[hydro::api::kNumClasses] = {0};
    for (int f = 0; f < 2; ++f) {
      int numf[hydro::api::kNumClasses] = {0}, nf = 0;
      for (int c = f; c < hydro::api::kNumClasses; c += 2) {
        numf[c] = num[c];
        nf += num[c];
      }
      if (!nf) continue;
      int rc = hydro::api::launch_mixed(numf, off, sl.htab, sl.dtab, nf, dt, dx, sl.hamax_dev, st,
                                        true, groups);
      if (rc) return rc;
    }
    for (int i = 0; i < n; ++i)
      sl.parts[i] = (uint8_t)groups[hydro::api::class_of_task(t[i].n, t[i].nfields)];
    // Completion word: the stream stores the batch id into pinned host memory
    // after the kernels, so polling completion is a memory read, not a
    // runtime call, and blocking waits spin on it (no event per batch: each
    // runtime call is ~2 us of the serving thread's time).
    HIP_OK(hipStreamWriteValue64(st, &flags_[k], batch, 0));
    sl.busy = true;
    sl.finished = false;
    sl.stream = s;
    sl.n = n;
    sl.batch = batch;
    live_[batch] = k;
    order_.push_back(batch);
    last_[s] = batch;
    return HYDRO_OK;
  }

 public:
  bool done(uint64_t batch) {
    auto r = retired_.find(batch);
    if (r != retired_.end()) return true;
    return finished(live_.at(batch));
  }

  int wait(uint64_t batch) {
    if (retired_.count(batch)) return HYDRO_OK;
    return spin(live_.at(batch));
  }

  void results(uint64_t batch, double* amax) {
    auto r = retired_.find(batch);
    if (r != retired_.end()) {
      std::copy(r->second.begin(), r->second.end(), amax);
      return;
    }
    reduce(slots_[live_.at(batch)], amax);
  }

  void release(uint64_t batch) {
    auto r = retired_.find(batch);
    if (r != retired_.end()) {
      retired_.erase(r);
      return;
    }
    auto it = live_.find(batch);
    if (it == live_.end()) return;
    slots_[it->second].busy = false;
    live_.erase(it);
    order_.erase(std::find(order_.begin(), order_.end(), batch));
  }

 private:
  struct Slot {
    DevDesc* htab = nullptr;
    DevDesc* dtab = nullptr;
    double* hamax = nullptr;      // kAmaxParts amax partials per task (pinned)
    double* hamax_dev = nullptr;  // the device's address of hamax
    std::vector<uint8_t> parts;   // partials written for each task
    bool busy = false, finished = false;
    int stream = 0, n = 0;
    uint64_t batch = 0;
  };

  // Task i's amax: the largest of its work-groups' partials.
  static void reduce(const Slot& sl, double* amax) {
    for (int i = 0; i < sl.n; ++i) {
      const double* p = sl.hamax + (size_t)i * hydro::kAmaxParts;
      double m = p[0];
      for (int b = 1; b < sl.parts[i]; ++b) m = std::max(m, p[b]);
      amax[i] = m;
    }
  }

  bool finished(int k) {
    Slot& sl = slots_[k];
    if (!sl.finished && __atomic_load_n(&flags_[k], __ATOMIC_ACQUIRE) == sl.batch)
      sl.finished = true;
    return sl.finished;
  }

  int free_slot() const {
    for (size_t k = 0; k < slots_.size(); ++k)
      if (!slots_[k].busy) return (int)k;
    return -1;
  }

  // Wait for slot k's completion word.  Every 4096 polls the slot's stream
  // is queried, so that a failed launch (which never writes the word) ends
  // the wait with its error instead of spinning forever; a stream that
  // stays idle for 256 queries without the word having arrived is an error
  // too.
  int spin(int k) {
    Slot& sl = slots_[k];
    int idle = 0;
    for (unsigned i = 1; !finished(k); ++i) {
      if (i % 4096) continue;
      const hipError_t e = hipStreamQuery(streams_[sl.stream]);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return fail(HYDRO_EHIP, "batch stream failed: %s", hipGetErrorString(e));
      if (++idle > 256)
        return fail(HYDRO_EHIP, "stream idle but batch %llu not complete",
                    (unsigned long long)sl.batch);
    }
    return HYDRO_OK;
  }

  // All slots in use: wait for the oldest batch, keep its results on the host.
  int retire_oldest() {
    const uint64_t b = order_.front();
    Slot& sl = slots_[live_.at(b)];
    {
      const int rc = spin(live_.at(b));
      if (rc) return rc;
    }
    std::vector<double> a((size_t)sl.n);
    reduce(sl, a.data());
    retired_[b] = std::move(a);
    sl.busy = false;
    live_.erase(b);
    order_.pop_front();
    return HYDRO_OK;
  }

  int ns_ = 0, created_ = 0, cap_ = 0;
  double launch_us_ = 0.0;
  hipStream_t streams_[kAggMaxStreams] = {};
  std::vector<Slot> slots_;
  uint64_t* flags_ = nullptr;   // pinned; flags_[k] = id of the last finished batch of slot k
  uint64_t last_[kAggMaxStreams] = {};  // newest batch launched on each stream
  std::unordered_map<uint64_t, int> live_;
  std::deque<uint64_t> order_;
  std::unordered_map<uint64_t, std::vector<double>> retired_;
};

using Policy = hydro::AggPolicy<HipExec, SteadyClock>;

// Output bytes of a task (what the byte budget of the aggregator counts).
uint64_t out_bytes(int n, int nfields, int out_layout) {
  const uint64_t e = out_layout == HYDRO_OUT_INTERIOR ? (uint64_t)n : (uint64_t)n + 2 * HYDRO_GHOST;
  return (uint64_t)nfields * e * e * e * sizeof(double);
}

uint64_t task_bytes(const hydro_subgrid_t& s) { return out_bytes(s.n, s.nfields, s.out_layout); }

}  // namespace

struct hydro_agg {
  std::mutex mu;
  HipExec ex;
  SteadyClock clk;
  Policy* pol = nullptr;
  int width = 1;
};

extern "C" {

int hydro_agg_create(hydro_agg_t** out, int32_t max_width, double timeout_us,
                     int32_t n_streams, uint64_t hbm_budget_bytes, int32_t flush_when_idle) {
  hydro::api::clear_error();
  if (!out) return fail(HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_width < 1 || max_width > 65536) return fail(HYDRO_EINVAL, "max_width %d", max_width);
  if (n_streams < 1 || n_streams > kAggMaxStreams)
    return fail(HYDRO_EINVAL, "n_streams %d", n_streams);
  if (timeout_us != timeout_us) return fail(HYDRO_EINVAL, "timeout is NaN");
  hydro_agg* a = new hydro_agg();
  a->width = max_width;
  // batch slots (in-flight batches): 32 per stream up to 8 streams, then
  // 256 in all, at least 4 per stream
  const int per_stream = n_streams <= 8 ? 32 : std::max(4, 256 / n_streams);
  int rc = a->ex.init(n_streams, max_width, per_stream);
  if (rc) {
    a->ex.teardown();
    delete a;
    return rc;
  }
  a->pol = new Policy(a->ex, a->clk, max_width, timeout_us, hbm_budget_bytes, flush_when_idle != 0);
  *out = a;
  return HYDRO_OK;
}

int hydro_submit(hydro_agg_t* a, const hydro_subgrid_t* sg, double dt, double dx,
                 uint64_t* ticket) {
  hydro::api::clear_error();
  if (!a || !ticket) return fail(HYDRO_EINVAL, "NULL aggregator or ticket");
  int rc = hydro::api::validate_batch(sg, 1, dt, dx);
  if (rc) return rc;
  Task t;
  t.u_in = sg->u_in;
  t.u_out = sg->u_out;
  t.n = sg->n;
  t.nfields = sg->nfields;
  t.level = sg->level;
  t.out_layout = sg->out_layout;
  t.bytes = task_bytes(*sg);
  std::lock_guard<std::mutex> lk(a->mu);
  rc = a->pol->submit(t, dt, dx, ticket);
  if (rc == HYDRO_EAGAIN) return fail(HYDRO_EAGAIN, "admission refused: byte budget in use");
  return rc;
}

int hydro_submit_many(hydro_agg_t* a, const hydro_subgrid_t* sg, int32_t count, double dt,
                      double dx, uint64_t* tickets, int32_t* submitted) {
  hydro::api::clear_error();
  if (!a || !submitted) return fail(HYDRO_EINVAL, "NULL aggregator or count out-pointer");
  *submitted = 0;
  int rc = hydro::api::validate_batch(sg, count, dt, dx);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(a->mu);
  for (int32_t i = 0; i < count; ++i) {
    Task t;
    t.u_in = sg[i].u_in;
    t.u_out = sg[i].u_out;
    t.n = sg[i].n;
    t.nfields = sg[i].nfields;
    t.level = sg[i].level;
    t.out_layout = sg[i].out_layout;
    t.bytes = task_bytes(sg[i]);
    uint64_t ticket = 0;
    rc = a->pol->submit(t, dt, dx, &ticket, tickets == nullptr);
    if (rc == HYDRO_EAGAIN) return fail(HYDRO_EAGAIN, "admission refused after %d tasks", i);
    if (rc) return rc;
    if (tickets) tickets[i] = ticket;
    *submitted = i + 1;
  }
  return HYDRO_OK;
}

int hydro_agg_drain(hydro_agg_t* a) {
  hydro::api::clear_error();
  if (!a) return fail(HYDRO_EINVAL, "NULL aggregator");
  std::lock_guard<std::mutex> lk(a->mu);
  return a->pol->drain();
}

int hydro_flush(hydro_agg_t* a) {
  hydro::api::clear_error();
  if (!a) return fail(HYDRO_EINVAL, "NULL aggregator");
  std::lock_guard<std::mutex> lk(a->mu);
  return a->pol->flush();
}

int hydro_progress(hydro_agg_t* a) {
  hydro::api::clear_error();
  if (!a) return fail(HYDRO_EINVAL, "NULL aggregator");
  std::lock_guard<std::mutex> lk(a->mu);
  return a->pol->progress();
}

int hydro_poll(hydro_agg_t* a, uint64_t ticket, int32_t* done, double* amax) {
  hydro::api::clear_error();
  if (!a || !done) return fail(HYDRO_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(a->mu);
  int d = 0;
  int rc = a->pol->poll(ticket, &d, amax);
  if (rc == -1) return fail(HYDRO_EINVAL, "unknown or already retrieved ticket %llu",
                            (unsigned long long)ticket);
  *done = d;
  return rc;
}

int hydro_wait(hydro_agg_t* a, uint64_t ticket, double* amax) {
  hydro::api::clear_error();
  if (!a) return fail(HYDRO_EINVAL, "NULL aggregator");
  std::lock_guard<std::mutex> lk(a->mu);
  int rc = a->pol->wait(ticket, amax);
  if (rc == -1) return fail(HYDRO_EINVAL, "unknown or already retrieved ticket %llu",
                            (unsigned long long)ticket);
  return rc;
}

int hydro_agg_stats(hydro_agg_t* a, hydro_agg_stats_t* out) {
  hydro::api::clear_error();
  if (!a || !out) return fail(HYDRO_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(a->mu);
  const hydro::AggStats& s = a->pol->stats();
  memset(out, 0, sizeof *out);
  out->submitted = s.submitted;
  out->batches = s.launched_batches;
  out->launched = s.launched_tasks;
  out->flush_width = s.flush_width;
  out->flush_idle = s.flush_idle;
  out->flush_timeout = s.flush_timeout;
  out->flush_manual = s.flush_manual + s.flush_param;
  out->refused = s.refused;
  for (int i = 0; i < 11; ++i) out->width_hist[i] = s.width_hist[i];
  out->held = a->pol->held();
  out->held_bytes = a->pol->held_bytes();
  return HYDRO_OK;
}

int hydro_agg_destroy(hydro_agg_t* a) {
  hydro::api::clear_error();
  if (!a) return HYDRO_OK;
  int rc;
  {
    std::lock_guard<std::mutex> lk(a->mu);
    rc = a->pol->drain();
  }
  delete a->pol;
  a->ex.teardown();
  delete a;
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving loop
// ---------------------------------------------------------------------------
namespace {

// Free output slabs of one edge class, carved from caller-provided device
// memory (the HBM budget of the loop).
struct SlabPool {
  std::vector<double*> free_list;
  uint64_t words = 0;  // doubles per slab
};

}  // namespace

extern "C" int hydro_serve_run(const hydro_serve_config_t* cfg, const hydro_subgrid_t* pool,
                               int32_t pool_count, const int32_t* task_subgrid,
                               const double* arrival_us, int32_t ntasks,
                               double* latency_us, double* amax_out, double** out_slab,
                               hydro_serve_stats_t* stats) {
  hydro::api::clear_error();
  if (!cfg || !pool || pool_count <= 0 || !task_subgrid || !arrival_us || ntasks < 0 ||
      !latency_us || !stats)
    return fail(HYDRO_EINVAL, "NULL or empty argument");
  if (cfg->max_width < 1 || cfg->n_streams < 1) return fail(HYDRO_EINVAL, "bad aggregator config");
  if (cfg->out_layout != HYDRO_OUT_STORED && cfg->out_layout != HYDRO_OUT_INTERIOR)
    return fail(HYDRO_EINVAL, "out_layout %d", cfg->out_layout);
  int rc = HYDRO_OK;
  for (int i = 1; i < ntasks; ++i)
    if (!(arrival_us[i] >= arrival_us[i - 1]))
      return fail(HYDRO_EINVAL, "arrival times must be non-decreasing");
  // slab pools per edge class
  SlabPool pools[3];
  for (int e = 0; e < 3; ++e) {
    const int n = 8 + 4 * e;
    if (cfg->slabs[e] < 0) return fail(HYDRO_EINVAL, "negative slab count");
    if (cfg->slabs[e] > 0 && !cfg->slab_base[e]) return fail(HYDRO_EINVAL, "NULL slab arena");
    const uint64_t words = out_bytes(n, cfg->nfields, cfg->out_layout) / sizeof(double);
    pools[e].words = words;
    for (int k = cfg->slabs[e] - 1; k >= 0; --k)
      pools[e].free_list.push_back(cfg->slab_base[e] + (uint64_t)k * words);
  }
  // every resident sub-grid must be a valid task with an output slab of its class
  for (int s = 0; s < pool_count; ++s) {
    if (hydro::api::class_of_task(pool[s].n, pool[s].nfields) < 0 || pool[s].nfields != cfg->nfields)
      return fail(HYDRO_EINVAL, "sub-grid %d: n=%d nfields=%d", s, pool[s].n, pool[s].nfields);
    const int e = (pool[s].n - 8) / 4;
    if (cfg->slabs[e] == 0) return fail(HYDRO_EINVAL, "sub-grid %d: no slabs for n=%d", s, pool[s].n);
    hydro_subgrid_t probe = pool[s];
    probe.u_out = cfg->slab_base[e];
    probe.out_layout = cfg->out_layout;
    rc = hydro::api::validate_batch(&probe, 1, cfg->dt, cfg->dx);
    if (rc) return rc;
    // no slab of any class may overlap a resident input
    const uint64_t in_bytes = out_bytes(pool[s].n, pool[s].nfields, HYDRO_OUT_STORED);
    const uintptr_t a0 = (uintptr_t)pool[s].u_in, a1 = a0 + in_bytes;
    for (int f = 0; f < 3; ++f) {
      if (cfg->slabs[f] == 0) continue;
      const uintptr_t b0 = (uintptr_t)cfg->slab_base[f];
      const uintptr_t b1 = b0 + (uint64_t)cfg->slabs[f] * pools[f].words * sizeof(double);
      if (a0 < b1 && b0 < a1)
        return fail(HYDRO_EINVAL, "sub-grid %d: the slab arena of class %d overlaps it", s, f);
    }
  }
  for (int i = 0; i < ntasks; ++i)
    if (task_subgrid[i] < 0 || task_subgrid[i] >= pool_count)
      return fail(HYDRO_EINVAL, "task %d: sub-grid %d", i, task_subgrid[i]);

  hydro_agg_t* agg = nullptr;
  rc = hydro_agg_create(&agg, cfg->max_width, cfg->timeout_us, cfg->n_streams, 0,
                        cfg->flush_when_idle);
  if (rc) return rc;
  agg->pol->record_completions(true);

  struct Live {
    int task;
    int cls;
    double* slab;
  };
  std::deque<int> waiting[3];  // arrived, waiting for an output slab
  std::unordered_map<uint64_t, Live> live;
  std::vector<std::pair<uint64_t, double>> done;
  SteadyClock clk;
  int next = 0, finished = 0;
  uint64_t max_live = 0, slab_waits = 0;
  double t_first = -1.0, t_last = 0.0;
  const double t0 = clk.now_us();
  while (finished < ntasks && rc == HYDRO_OK) {
    const double now = clk.now_us() - t0;
    // 1. arrivals
    while (next < ntasks && arrival_us[next] <= now) {
      waiting[(pool[task_subgrid[next]].n - 8) / 4].push_back(next);
      ++next;
    }
    // 2. admission: a task enters as soon as an output slab of its class is
    //    free, and joins whatever batch the aggregator is forming
    for (int e = 0; e < 3 && rc == HYDRO_OK; ++e) {
      while (!waiting[e].empty() && !pools[e].free_list.empty()) {
        const int i = waiting[e].front();
        waiting[e].pop_front();
        double* slab = pools[e].free_list.back();
        pools[e].free_list.pop_back();
        Task t;
        const hydro_subgrid_t& src = pool[task_subgrid[i]];
        t.u_in = src.u_in;
        t.u_out = slab;
        t.n = src.n;
        t.nfields = src.nfields;
        t.level = src.level;
        t.out_layout = cfg->out_layout;
        t.bytes = out_bytes(src.n, src.nfields, cfg->out_layout);
        uint64_t ticket = 0;
        rc = agg->pol->submit(t, cfg->dt, cfg->dx, &ticket);
        if (rc) break;
        live[ticket] = Live{i, e, slab};
        if (t_first < 0) t_first = now;
      }
      if (!waiting[e].empty()) slab_waits++;
    }
    if (rc) break;
    max_live = std::max<uint64_t>(max_live, live.size());
    // 3. flush rules (timeout, idle stream) and completions
    rc = agg->pol->progress();
    if (rc) break;
    agg->pol->take_completed(done);
    if (!done.empty()) {
      const double t_done = clk.now_us() - t0;
      for (auto& c : done) {
        auto it = live.find(c.first);
        const Live lv = it->second;
        live.erase(it);
        latency_us[lv.task] = t_done - arrival_us[lv.task];
        if (amax_out) amax_out[lv.task] = c.second;
        if (out_slab) out_slab[lv.task] = lv.slab;
        if (!cfg->keep_slabs) pools[lv.cls].free_list.push_back(lv.slab);
        ++finished;
      }
      t_last = t_done;
    }
  }
  if (rc == HYDRO_OK) {
    hydro_agg_stats_t as;
    hydro_agg_stats(agg, &as);
    memset(stats, 0, sizeof *stats);
    stats->agg = as;
    stats->makespan_us = t_last;
    stats->first_admit_us = t_first;
    stats->max_live = max_live;
    stats->slab_waits = slab_waits;
    stats->launch_host_us = agg->ex.launch_us();
  }
  {
    const int rc2 = hydro_agg_destroy(agg);
    if (!rc) rc = rc2;
  }
  return rc;
}

// region_api.hip -- the generic aggregation region (region_core.hpp) on HIP
// streams, its C ABI, and library kernels that run inside a region.
//
// The executor owns n_streams streams and two team slots per stream, each
// slot with an arena of arena_bytes of device memory and a pinned host
// mirror of the same size, all created by hydro_region_create: entering,
// allocating, copying and launching never allocate (Section V-C).  A team's
// uploads, launches and downloads go to its slot's stream in the order the
// members make them; its completion is an event of the slot.
#include <hip/hip_runtime.h>

#include <string.h>

#include <string>
#include <system_error>

#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "hydro_lds8.hpp"
#include "internal.hpp"
#include "region_core.hpp"

using hydro::api::fail;

namespace {

#define HIP_OK(expr)                                                         \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(HYDRO_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kRegionMaxStreams = 32;

class HipRegionExec {
 public:
  int init(int ns, uint64_t bytes) {
    ns_ = ns;
    bytes_ = bytes;
    const int slots = ns * hydro::RegionCore<HipRegionExec>::kSlotsPerStream;
    for (int s = 0; s < ns; ++s) {
      HIP_OK(hipStreamCreateWithFlags(&streams_[s], hipStreamNonBlocking));
      made_streams_ = s + 1;
    }
    host_.assign(slots, nullptr);
    dev_.assign(slots, nullptr);
    ev_.assign(slots, nullptr);
    for (int k = 0; k < slots; ++k) {
      HIP_OK(hipHostMalloc((void**)&host_[k], bytes, hipHostMallocDefault));
      HIP_OK(hipMalloc((void**)&dev_[k], bytes));
      HIP_OK(hipEventCreateWithFlags(&ev_[k], hipEventDisableTiming));
    }
    return HYDRO_OK;
  }

  void teardown() {
    for (int s = 0; s < made_streams_; ++s) (void)hipStreamSynchronize(streams_[s]);
    for (size_t k = 0; k < host_.size(); ++k) {
      if (host_[k]) (void)hipHostFree(host_[k]);
      if (dev_[k]) (void)hipFree(dev_[k]);
      if (ev_[k]) (void)hipEventDestroy(ev_[k]);
    }
    host_.clear();
    dev_.clear();
    ev_.clear();
    for (int s = 0; s < made_streams_; ++s) (void)hipStreamDestroy(streams_[s]);
    made_streams_ = 0;
  }

  int streams() const { return ns_; }
  char* arena_host(int k) { return host_[k]; }
  char* arena_dev(int k) { return dev_[k]; }
  uint64_t arena_bytes() const { return bytes_; }

  int upload(int k, uint64_t off, uint64_t n) {
    HIP_OK(hipMemcpyAsync(dev_[k] + off, host_[k] + off, n, hipMemcpyHostToDevice, stream(k)));
    return HYDRO_OK;
  }
  int download(int k, uint64_t off, uint64_t n) {
    HIP_OK(hipMemcpyAsync(host_[k] + off, dev_[k] + off, n, hipMemcpyDeviceToHost, stream(k)));
    return HYDRO_OK;
  }
  int launch(int k, const void* kernel, unsigned blocks, unsigned threads, unsigned shmem,
             void** args) {
    HIP_OK(hipLaunchKernel(kernel, dim3(blocks), dim3(threads), args, shmem, stream(k)));
    return HYDRO_OK;
  }
  int record(int k, uint64_t) {
    HIP_OK(hipEventRecord(ev_[k], stream(k)));
    return HYDRO_OK;
  }
  int wait(int k, uint64_t) {
    HIP_OK(hipEventSynchronize(ev_[k]));
    return HYDRO_OK;
  }

 private:
  hipStream_t stream(int k) const { return streams_[k % ns_]; }
  int ns_ = 0, made_streams_ = 0;
  uint64_t bytes_ = 0;
  hipStream_t streams_[kRegionMaxStreams] = {};
  std::vector<char*> host_, dev_;
  std::vector<hipEvent_t> ev_;
};

// A core return code as the library's: mismatched calls are argument errors.
int core_rc(int rc) {
  if (rc == hydro::kMismatch)
    return fail(HYDRO_EINVAL, "region call does not match the team's sequence, or stale task");
  if (rc == hydro::kNoSpace) return fail(HYDRO_ENOMEM, "team buffers exceed the region arena");
  return rc;   // HYDRO_OK or a HIP error already recorded
}

}  // namespace

struct hydro_region {
  HipRegionExec ex;
  hydro::RegionCore<HipRegionExec>* core = nullptr;
};

namespace hydro {

// The 8^3 hydro step of a team's table of public descriptors (one per
// member, in member order): work-group s steps table[s] exactly as
// hydro_lds8_kernel steps it, amax of member s to amax[s].
template <int F>
__global__ void __launch_bounds__(Lds8::kThreads, 2)
    region_step8_kernel(const hydro_subgrid_t* __restrict__ table, int count, double dt,
                        double dx, double* __restrict__ amax) {
  const int s = blockIdx.x;
  if (s >= count) return;
  const hydro_subgrid_t g = table[s];
  DevDesc d;
  d.u_in = g.u_in;
  d.u_out = g.u_out;
  d.level = (int16_t)g.level;
  d.compact = (int16_t)(g.out_layout == HYDRO_OUT_INTERIOR);
  d.index = s;
  lds8_step<F, 14, false>(d, 0, 0, 0, 0, 0, 0, 0, dt, dx, amax);
}

// out = a x + b y over n doubles for each member's entry; blocks_per_task
// work-groups of 256 lanes per member.
__global__ void __launch_bounds__(256)
    region_axpby_kernel(const hydro_region_axpby_t* __restrict__ table, int count,
                        int blocks_per_task) {
  const int task = blockIdx.x / blocks_per_task;
  if (task >= count) return;
  const hydro_region_axpby_t e = table[task];
  const int64_t stride = (int64_t)blocks_per_task * blockDim.x;
  for (int64_t i = (int64_t)(blockIdx.x % blocks_per_task) * blockDim.x + threadIdx.x; i < e.n;
       i += stride)
    e.out[i] = e.a * e.x[i] + e.b * e.y[i];
}

}  // namespace hydro

extern "C" {

int hydro_region_create(hydro_region_t** out, int32_t max_team, int32_t n_streams,
                        uint64_t arena_bytes) {
  hydro::api::clear_error();
  if (!out) return fail(HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_team < 1 || max_team > 65536) return fail(HYDRO_EINVAL, "max_team %d", max_team);
  if (n_streams < 1 || n_streams > kRegionMaxStreams)
    return fail(HYDRO_EINVAL, "n_streams %d outside 1..%d", n_streams, kRegionMaxStreams);
  if (arena_bytes < 256 || arena_bytes > (1ull << 34))
    return fail(HYDRO_EINVAL, "arena_bytes %llu", (unsigned long long)arena_bytes);
  hydro_region* r = new hydro_region();
  int rc = r->ex.init(n_streams, arena_bytes);
  if (rc) {
    r->ex.teardown();
    delete r;
    return rc;
  }
  r->core = new hydro::RegionCore<HipRegionExec>(r->ex, max_team);
  *out = r;
  return HYDRO_OK;
}

int hydro_region_enter(hydro_region_t* r, hydro_region_task_t* task) {
  hydro::api::clear_error();
  if (!r || !task) return fail(HYDRO_EINVAL, "NULL region or task");
  hydro::RegionTask t;
  int rc = r->core->enter(&t);
  if (rc) return core_rc(rc);
  task->team = t.team;
  task->index = t.index;
  task->size = t.size;
  task->stream = t.stream;
  task->id = t.id;
  return HYDRO_OK;
}

static hydro::RegionTask to_core(const hydro_region_task_t* t) {
  return hydro::RegionTask{t->team, t->index, t->size, t->stream, t->id};
}

int hydro_region_alloc(hydro_region_t* r, const hydro_region_task_t* task, uint64_t bytes,
                       int32_t* buffer, void** host_chunk, void** dev_chunk) {
  hydro::api::clear_error();
  if (!r || !task || !buffer || !host_chunk || !dev_chunk) return fail(HYDRO_EINVAL, "NULL argument");
  if (bytes == 0) return fail(HYDRO_EINVAL, "zero-byte allocation");
  char *h = nullptr, *d = nullptr;
  int rc = r->core->alloc(to_core(task), bytes, buffer, &h, &d);
  if (rc) return core_rc(rc);
  *host_chunk = h;
  *dev_chunk = d;
  return HYDRO_OK;
}

int hydro_region_buffer(hydro_region_t* r, const hydro_region_task_t* task, int32_t buffer,
                        void** dev_base, uint64_t* stride) {
  hydro::api::clear_error();
  if (!r || !task || !dev_base || !stride) return fail(HYDRO_EINVAL, "NULL argument");
  char* b = nullptr;
  int rc = r->core->buffer(to_core(task), buffer, &b, stride);
  if (rc) return core_rc(rc);
  *dev_base = b;
  return HYDRO_OK;
}

int hydro_region_upload(hydro_region_t* r, const hydro_region_task_t* task, int32_t buffer) {
  hydro::api::clear_error();
  if (!r || !task) return fail(HYDRO_EINVAL, "NULL argument");
  return core_rc(r->core->upload(to_core(task), buffer));
}

int hydro_region_download(hydro_region_t* r, const hydro_region_task_t* task, int32_t buffer) {
  hydro::api::clear_error();
  if (!r || !task) return fail(HYDRO_EINVAL, "NULL argument");
  return core_rc(r->core->download(to_core(task), buffer));
}

int hydro_region_launch(hydro_region_t* r, const hydro_region_task_t* task, const void* kernel,
                        uint32_t blocks_per_task, uint32_t threads, uint32_t shmem, void** args) {
  hydro::api::clear_error();
  if (!r || !task || !kernel) return fail(HYDRO_EINVAL, "NULL argument");
  if (blocks_per_task < 1 || threads < 1 || threads > 1024)
    return fail(HYDRO_EINVAL, "launch shape %u x %u", blocks_per_task, threads);
  return core_rc(r->core->launch(to_core(task), kernel, blocks_per_task, threads, shmem, args));
}

int hydro_region_wait(hydro_region_t* r, const hydro_region_task_t* task) {
  hydro::api::clear_error();
  if (!r || !task) return fail(HYDRO_EINVAL, "NULL argument");
  return core_rc(r->core->wait(to_core(task)));
}

int hydro_region_leave(hydro_region_t* r, const hydro_region_task_t* task) {
  hydro::api::clear_error();
  if (!r || !task) return fail(HYDRO_EINVAL, "NULL argument");
  return core_rc(r->core->leave(to_core(task)));
}

int hydro_region_stats(hydro_region_t* r, hydro_region_stats_t* out) {
  hydro::api::clear_error();
  if (!r || !out) return fail(HYDRO_EINVAL, "NULL argument");
  const hydro::RegionStats s = r->core->stats();
  memset(out, 0, sizeof *out);
  out->tasks = s.tasks;
  out->teams = s.teams;
  out->full_teams = s.full_teams;
  out->uploads = s.uploads;
  out->launches = s.launches;
  out->downloads = s.downloads;
  for (int i = 0; i < 11; ++i) out->size_hist[i] = s.size_hist[i];
  return HYDRO_OK;
}

int hydro_region_destroy(hydro_region_t* r) {
  hydro::api::clear_error();
  if (!r) return HYDRO_OK;
  delete r->core;
  r->ex.teardown();
  delete r;
  return HYDRO_OK;
}

// One task through the region: its descriptor in a team table, the team's
// 8^3 step, its amax back (read between wait and leave).
static int drive_region_task(hydro_region_t* r, const void* kernel, const hydro_subgrid_t& sg,
                             double dt, double dx, double* amax) {
  hydro_region_task_t t;
  int rc = hydro_region_enter(r, &t);
  if (rc) return rc;
  int32_t bd = -1, ba = -1;
  void *hd = nullptr, *dd = nullptr, *ha = nullptr, *da = nullptr;
  void* base_d = nullptr;
  void* base_a = nullptr;
  uint64_t stride = 0;
  int32_t size = t.size;
  void* args[5] = {&base_d, &size, &dt, &dx, &base_a};
  if (!(rc = hydro_region_alloc(r, &t, sizeof(hydro_subgrid_t), &bd, &hd, &dd)) &&
      !(rc = hydro_region_alloc(r, &t, sizeof(double), &ba, &ha, &da))) {
    memcpy(hd, &sg, sizeof sg);
    if (!(rc = hydro_region_upload(r, &t, bd)) &&
        !(rc = hydro_region_buffer(r, &t, bd, &base_d, &stride)) &&
        !(rc = hydro_region_buffer(r, &t, ba, &base_a, &stride)) &&
        !(rc = hydro_region_launch(r, &t, kernel, 1, hydro::Lds8::kThreads, 0, args)) &&
        !(rc = hydro_region_download(r, &t, ba)) && !(rc = hydro_region_wait(r, &t)) && amax)
      *amax = *(const double*)ha;
  }
  const int rl = hydro_region_leave(r, &t);   // every member leaves once
  return rc ? rc : rl;
}

int hydro_region_drive(hydro_region_t* r, const hydro_subgrid_t* sg, int32_t count,
                       int32_t n_threads, double dt, double dx, int32_t mode,
                       double* amax_host, double* seconds) {
  hydro::api::clear_error();
  if (!sg || !seconds) return fail(HYDRO_EINVAL, "NULL argument");
  if (mode != HYDRO_DRIVE_REGION && mode != HYDRO_DRIVE_EACH)
    return fail(HYDRO_EINVAL, "mode %d", mode);
  if (mode == HYDRO_DRIVE_REGION && !r) return fail(HYDRO_EINVAL, "region is NULL");
  if (count < 1 || count > (1 << 20)) return fail(HYDRO_EINVAL, "count %d", count);
  if (n_threads < 1 || n_threads > 256) return fail(HYDRO_EINVAL, "n_threads %d", n_threads);
  if (!(dt >= 0.0) || !(dx > 0.0)) return fail(HYDRO_EINVAL, "dt >= 0 and dx > 0 required");
  const int nf = sg[0].nfields;
  for (int32_t i = 0; i < count; ++i)
    if (sg[i].n != 8 || sg[i].nfields != nf || (nf != 6 && nf != 11))
      return fail(HYDRO_EINVAL, "task %d: n=%d nfields=%d (n = 8, one field count of 6 or 11)",
                  i, sg[i].n, sg[i].nfields);
  const void* kernel = hydro_region_kernel(nf == 11 ? HYDRO_REGION_STEP8_F11 : HYDRO_REGION_STEP8_F6);
  std::atomic<int32_t> next{0};
  std::atomic<int> first_rc{HYDRO_OK};
  // the clock starts once every worker has made its per-thread set-up
  std::atomic<int> ready{0};
  std::atomic<bool> go{false};
  std::vector<std::string> errs((size_t)n_threads);
  auto worker = [&](int w) {
    hipStream_t st = nullptr;
    double* dev_amax = nullptr;
    double* pinned = nullptr;
    if (mode == HYDRO_DRIVE_EACH) {
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
          hipMalloc((void**)&dev_amax, sizeof(double)) != hipSuccess ||
          hipHostMalloc((void**)&pinned, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        int z = HYDRO_OK;
        first_rc.compare_exchange_strong(z, HYDRO_EHIP);
        errs[w] = "per-thread stream or buffers";
      }
    }
    ready.fetch_add(1);
    while (!go.load()) std::this_thread::yield();
    while (first_rc.load() == HYDRO_OK) {
      const int32_t i = next.fetch_add(1);
      if (i >= count) break;
      double a = 0.0;
      int rc;
      if (mode == HYDRO_DRIVE_REGION) {
        rc = drive_region_task(r, kernel, sg[i], dt, dx, &a);
      } else {
        rc = hydro_step(&sg[i], 1, dt, dx, dev_amax, st);
        if (!rc && (hipMemcpyAsync(pinned, dev_amax, sizeof(double), hipMemcpyDeviceToHost, st) !=
                        hipSuccess || hipStreamSynchronize(st) != hipSuccess))
          rc = HYDRO_EHIP;
        a = rc ? 0.0 : *pinned;
      }
      if (rc) {
        int z = HYDRO_OK;
        if (first_rc.compare_exchange_strong(z, rc)) errs[w] = hydro_last_error();
        break;
      }
      if (amax_host) amax_host[i] = a;
    }
    if (pinned) (void)hipHostFree(pinned);
    if (dev_amax) (void)hipFree(dev_amax);
    if (st) (void)hipStreamDestroy(st);
  };
  std::vector<std::thread> ts;
  std::string start_err;
  try {
    for (int w = 0; w < n_threads; ++w) ts.emplace_back(worker, w);
  } catch (const std::system_error&) {
    // fewer threads than asked for: the ones started end without tasks
    int z = HYDRO_OK;
    first_rc.compare_exchange_strong(z, HYDRO_EINVAL);
    start_err = "could not start the worker threads";
  }
  while (ready.load() < (int)ts.size()) std::this_thread::yield();
  const auto t0 = std::chrono::steady_clock::now();
  go.store(true);
  for (auto& th : ts) th.join();
  *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  const int rc = first_rc.load();
  if (rc) {
    if (!start_err.empty()) return fail(rc, "%s", start_err.c_str());
    for (auto& e : errs)
      if (!e.empty()) return fail(rc, "%s", e.c_str());
    return fail(rc, "a task failed");
  }
  return HYDRO_OK;
}

const void* hydro_region_kernel(int32_t which) {
  switch (which) {
    case HYDRO_REGION_STEP8_F6: return (const void*)&hydro::region_step8_kernel<6>;
    case HYDRO_REGION_STEP8_F11: return (const void*)&hydro::region_step8_kernel<11>;
    case HYDRO_REGION_AXPBY: return (const void*)&hydro::region_axpby_kernel;
  }
  return nullptr;
}

}  // extern "C"

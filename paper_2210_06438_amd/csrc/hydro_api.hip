// hydro_api.hip -- host side of libhydroagg.so: argument checks, descriptor
// tables, and the aggregated / per-sub-grid launches of the hydro step.
//
// Aggregation (paper Section V-D, strategy 3): a batch of sub-grid tasks is
// sorted into shape classes (n, nfields) and each class runs as ONE launch in
// which work-group s steps sub-grid s of the class.  The descriptors go to
// the device through a library-owned table: a ring of slots, each a pinned
// host buffer plus a device buffer plus an event, all created once per device
// at first use (no device allocation or stream creation on the step path,
// Section V-C).  Small classes carry their descriptors in kernel arguments.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/hydroagg.h"
#include "hydro_kernel.hpp"
#include "hydro_lds8.hpp"
#include "hydro_q4.hpp"
#include "hydro_mixed.hpp"
#include "hydro_pattern.hpp"
#include "hydro_step26.hpp"
#include "internal.hpp"

using hydro::ArgDescs;
using hydro::DevDesc;

namespace hydro {
namespace api {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = '\0'; }

}  // namespace api
}  // namespace hydro

using hydro::api::fail;
using hydro::api::g_err;

namespace {

#define HIP_TRY(expr)                                                       \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(HYDRO_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Shape classes: (n, nfields) -> index.
constexpr int kEdges[3] = {8, 12, 16};
constexpr int kFields[2] = {6, 11};
constexpr int kClasses = 6;

int class_of(int n, int nf) {
  int e = n == 8 ? 0 : n == 12 ? 1 : n == 16 ? 2 : -1;
  int f = nf == 6 ? 0 : nf == 11 ? 1 : -1;
  return (e < 0 || f < 0) ? -1 : e * 2 + f;
}

// ---- descriptor ring ------------------------------------------------------
constexpr int kSlots = 8;
constexpr int kSlotCap = 1 << 16;

// A slot is taken round-robin under the device mutex and then held, by its
// own mutex, from the wait for its previous use through the fill of its
// pinned buffer, the copy, the launches and the record of `done`: two host
// threads that land on the same slot (more than kSlots calls in flight)
// take turns, and the second waits for the first one's work to finish
// before it overwrites the pinned buffer.
struct Slot {
  std::mutex mu;
  DevDesc* host = nullptr;  // pinned
  DevDesc* dev = nullptr;
  hipEvent_t done = nullptr;
  bool used = false;
};

struct DeviceState {
  std::mutex mu;
  bool ready = false;
  Slot slots[kSlots];
  int next = 0;
};

constexpr int kMaxDevices = 16;
DeviceState g_dev[kMaxDevices];

Slot* take_slot(DeviceState* st) {
  std::lock_guard<std::mutex> lk(st->mu);
  Slot* slot = &st->slots[st->next];
  st->next = (st->next + 1) % kSlots;
  return slot;
}

int device_state(DeviceState** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HYDRO_EINVAL, "device %d out of range", dev);
  DeviceState& st = g_dev[dev];
  std::lock_guard<std::mutex> lk(st.mu);
  if (!st.ready) {
    for (int i = 0; i < kSlots; ++i) {
      Slot& s = st.slots[i];
      HIP_TRY(hipHostMalloc((void**)&s.host, sizeof(DevDesc) * kSlotCap, hipHostMallocDefault));
      HIP_TRY(hipMalloc((void**)&s.dev, sizeof(DevDesc) * kSlotCap));
      HIP_TRY(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
    }
    st.ready = true;
  }
  *out = &st;
  return HYDRO_OK;
}

int validate(const hydro_subgrid_t* sg, int32_t count, double dt, double dx) {
  if (count < 0) return fail(HYDRO_EINVAL, "count %d < 0", count);
  if (count > 0 && !sg) return fail(HYDRO_EINVAL, "sg is NULL");
  if (!(dt >= 0.0) || !isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be finite and >= 0");
  if (!(dx > 0.0) || !isfinite(dx)) return fail(HYDRO_EINVAL, "dx must be finite and > 0");
  for (int32_t i = 0; i < count; ++i) {
    const hydro_subgrid_t& s = sg[i];
    if (class_of(s.n, s.nfields) < 0)
      return fail(HYDRO_EINVAL, "sub-grid %d: unsupported n=%d nfields=%d", i, s.n, s.nfields);
    if (!s.u_in || !s.u_out) return fail(HYDRO_EINVAL, "sub-grid %d: NULL buffer", i);
    if (s.out_layout != HYDRO_OUT_STORED && s.out_layout != HYDRO_OUT_INTERIOR)
      return fail(HYDRO_EINVAL, "sub-grid %d: out_layout %d", i, s.out_layout);
    {
      const uint64_t M = (uint64_t)s.n + 2 * HYDRO_GHOST;
      const uint64_t e = s.out_layout == HYDRO_OUT_INTERIOR ? (uint64_t)s.n : M;
      const uintptr_t a0 = (uintptr_t)s.u_in, a1 = a0 + s.nfields * M * M * M * sizeof(double);
      const uintptr_t b0 = (uintptr_t)s.u_out, b1 = b0 + s.nfields * e * e * e * sizeof(double);
      if (a0 < b1 && b0 < a1) return fail(HYDRO_EINVAL, "sub-grid %d: u_out overlaps u_in", i);
    }
    if (((uintptr_t)s.u_in | (uintptr_t)s.u_out) & 15)
      return fail(HYDRO_EINVAL, "sub-grid %d: buffers must be 16-byte aligned", i);
    if (s.level < 0 || s.level > 30) return fail(HYDRO_EINVAL, "sub-grid %d: level %d", i, s.level);
  }
  return HYDRO_OK;
}

// Tile of each shape class: the edge of the blocks a sub-grid is stepped as
// (8: hydro_lds8.hpp, 4: hydro_q4.hpp).  Set by hydro_set_tile (from the
// autotuner); read at every launch.  g_tile_epoch lets captured plans notice
// a change.
std::atomic<int> g_tile[kClasses] = {{8}, {8}, {4}, {4}, {8}, {8}};
std::atomic<uint64_t> g_tile_epoch{0};


template <int N, int F>
int launch_table(const DevDesc* table, int n, double dt, double dx, double* amax,
                 hipStream_t stream) {
  if (n <= 0) return HYDRO_OK;
  const int tile = g_tile[class_of(N, F)].load(std::memory_order_relaxed);
  const int B = hydro::groups_per_subgrid<N + 6>(tile);
  if (B > 1 && amax) {
    hipLaunchKernelGGL(hydro::amax_zero_table, dim3((n + 255) / 256), dim3(256), 0, stream,
                       table, n, amax);
    HIP_TRY(hipGetLastError());
  }
  if (tile == 4)
    hipLaunchKernelGGL((hydro::hydro_q4_kernel<F, N + 6>), dim3(hydro::grid_for(n, B)),
                       dim3(hydro::Q4::kThreads), 0, stream, table, n, dt, dx, amax);
  else
    hipLaunchKernelGGL((hydro::hydro_lds8_kernel<F, N + 6>), dim3(hydro::grid_for(n, B)),
                       dim3(hydro::Lds8::kThreads), 0, stream, table, n, dt, dx, amax);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

template <int N, int F>
int launch_args(const ArgDescs& a, int n, double dt, double dx, double* amax,
                hipStream_t stream) {
  if (n <= 0) return HYDRO_OK;
  const int tile = g_tile[class_of(N, F)].load(std::memory_order_relaxed);
  const int B = hydro::groups_per_subgrid<N + 6>(tile);
  if (B > 1 && amax) {
    hipLaunchKernelGGL(hydro::amax_zero_args, dim3(1), dim3(64), 0, stream, a, n, amax);
    HIP_TRY(hipGetLastError());
  }
  if (tile == 4)
    hipLaunchKernelGGL((hydro::hydro_q4_arg_kernel<F, N + 6>), dim3(n * B),
                       dim3(hydro::Q4::kThreads), 0, stream, a, dt, dx, amax);
  else
    hipLaunchKernelGGL((hydro::hydro_lds8_arg_kernel<F, N + 6>), dim3(n * B),
                       dim3(hydro::Lds8::kThreads), 0, stream, a, dt, dx, amax);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int dispatch_table(int cls, const DevDesc* table, int n, double dt, double dx,
                   double* amax, hipStream_t s) {
  switch (cls) {
    case 0: return launch_table<8, 6>(table, n, dt, dx, amax, s);
    case 1: return launch_table<8, 11>(table, n, dt, dx, amax, s);
    case 2: return launch_table<12, 6>(table, n, dt, dx, amax, s);
    case 3: return launch_table<12, 11>(table, n, dt, dx, amax, s);
    case 4: return launch_table<16, 6>(table, n, dt, dx, amax, s);
    case 5: return launch_table<16, 11>(table, n, dt, dx, amax, s);
  }
  return fail(HYDRO_EINVAL, "bad class");
}

int dispatch_args(int cls, const ArgDescs& a, int n, double dt, double dx,
                  double* amax, hipStream_t s) {
  switch (cls) {
    case 0: return launch_args<8, 6>(a, n, dt, dx, amax, s);
    case 1: return launch_args<8, 11>(a, n, dt, dx, amax, s);
    case 2: return launch_args<12, 6>(a, n, dt, dx, amax, s);
    case 3: return launch_args<12, 11>(a, n, dt, dx, amax, s);
    case 4: return launch_args<16, 6>(a, n, dt, dx, amax, s);
    case 5: return launch_args<16, 11>(a, n, dt, dx, amax, s);
  }
  return fail(HYDRO_EINVAL, "bad class");
}


DevDesc to_dev(const hydro_subgrid_t& s, int index) {
  DevDesc d;
  d.u_in = s.u_in;
  d.u_out = s.u_out;
  d.level = (int16_t)s.level;
  d.compact = (int16_t)(s.out_layout == HYDRO_OUT_INTERIOR);
  d.index = index;
  return d;
}

// Work-groups of one table launch of class c over n sub-grids (current tile).
int class_groups(int c, int n) {
  const int tile = g_tile[c].load(std::memory_order_relaxed);
  const int B = c < 2 ? hydro::groups_per_subgrid<14>(tile)
              : c < 4 ? hydro::groups_per_subgrid<18>(tile)
                      : hydro::groups_per_subgrid<22>(tile);
  return hydro::grid_for(n, B);
}

// In a graph of a plan with two field counts, a class becomes a branch of
// its own only when its grid is at least two full rounds of resident
// work-groups (2 per CU on 256 CUs): a branch's fork and join cost the step
// ~25 us, which only the overlap of large launches (their partly filled
// last waves) pays back; small classes run in sequence on the capture
// stream (several of one field count as one multi-class launch).
constexpr int kBranchGroups = 1024;

// Where a chunk's device descriptor table comes from: a slot of the ring
// (held under its mutex from the wait for its previous use to the record of
// its event), or, when `fixed` is given, fixed arrays (host staging and
// device table) that the caller owns and serialises.
struct TableLease {
  Slot* slot = nullptr;
  std::unique_lock<std::mutex> held;
  DevDesc* host = nullptr;
  DevDesc* dev = nullptr;
};

struct FixedTable {
  DevDesc* host;
  DevDesc* dev;
};

int lease_table(DeviceState* st, const FixedTable* fixed, TableLease& t) {
  if (fixed) {
    t.host = fixed->host;
    t.dev = fixed->dev;
    return HYDRO_OK;
  }
  t.slot = take_slot(st);
  t.held = std::unique_lock<std::mutex>(t.slot->mu);
  if (t.slot->used) HIP_TRY(hipEventSynchronize(t.slot->done));
  t.host = t.slot->host;
  t.dev = t.slot->dev;
  return HYDRO_OK;
}

int release_table(TableLease& t, hipStream_t stream) {
  if (!t.slot) return HYDRO_OK;
  HIP_TRY(hipEventRecord(t.slot->done, stream));
  t.slot->used = true;
  return HYDRO_OK;
}

// One chunk of at most kSlotCap sub-grids starting at batch offset `base`.
int step_chunk(DeviceState* st, const FixedTable* fixed, const hydro_subgrid_t* sg, int count,
               int base, double dt, double dx, double* amax, hipStream_t stream) {
  int per_class[kClasses] = {0};
  for (int i = 0; i < count; ++i) per_class[class_of(sg[i].n, sg[i].nfields)]++;
  int need_table = 0;
  for (int c = 0; c < kClasses; ++c)
    if (per_class[c] > hydro::kArgDescs) need_table += per_class[c];

  // A small batch of several classes of one field count: one launch with
  // every descriptor in the kernel arguments.
  if (need_table == 0 && hydro::api::mixed_eligible(per_class)) {
    DevDesc host[kClasses * hydro::kArgDescs];
    int off[kClasses], fill[kClasses], pos = 0;
    for (int c = 0; c < kClasses; ++c) {
      off[c] = fill[c] = pos;
      pos += per_class[c];
    }
    for (int i = 0; i < count; ++i) {
      const int c = class_of(sg[i].n, sg[i].nfields);
      host[fill[c]++] = to_dev(sg[i], base + i);
    }
    return hydro::api::launch_mixed(per_class, off, host, nullptr, count, dt, dx, amax, stream);
  }
  // A larger one: one launch from a device table (classes side by side; for
  // large classes this overlaps the partly filled last waves of their
  // grids, which one launch per class would run one after another).
  if (hydro::api::mixed_eligible(per_class)) {
    TableLease t;
    int rc = lease_table(st, fixed, t);
    if (rc) return rc;
    int off[kClasses], fill[kClasses], pos = 0;
    for (int c = 0; c < kClasses; ++c) {
      off[c] = fill[c] = pos;
      pos += per_class[c];
    }
    for (int i = 0; i < count; ++i) {
      const int c = class_of(sg[i].n, sg[i].nfields);
      t.host[fill[c]++] = to_dev(sg[i], base + i);
    }
    HIP_TRY(hipMemcpyAsync(t.dev, t.host, sizeof(DevDesc) * count, hipMemcpyHostToDevice,
                           stream));
    rc = hydro::api::launch_mixed(per_class, off, nullptr, t.dev, count, dt, dx, amax, stream);
    if (rc) return rc;
    return release_table(t, stream);
  }

  // Small classes: descriptors travel in the kernel arguments.
  for (int c = 0; c < kClasses; ++c) {
    if (per_class[c] == 0 || per_class[c] > hydro::kArgDescs) continue;
    ArgDescs a;
    memset(&a, 0, sizeof a);
    int k = 0;
    for (int i = 0; i < count; ++i)
      if (class_of(sg[i].n, sg[i].nfields) == c) a.d[k++] = to_dev(sg[i], base + i);
    int rc = dispatch_args(c, a, k, dt, dx, amax, stream);
    if (rc) return rc;
  }
  if (need_table == 0) return HYDRO_OK;

  TableLease t;
  int rc = lease_table(st, fixed, t);
  if (rc) return rc;
  int off[kClasses];
  int pos = 0;
  for (int c = 0; c < kClasses; ++c) {
    off[c] = pos;
    if (per_class[c] > hydro::kArgDescs) pos += per_class[c];
  }
  int fill[kClasses];
  memcpy(fill, off, sizeof fill);
  for (int i = 0; i < count; ++i) {
    int c = class_of(sg[i].n, sg[i].nfields);
    if (per_class[c] > hydro::kArgDescs) t.host[fill[c]++] = to_dev(sg[i], base + i);
  }
  HIP_TRY(hipMemcpyAsync(t.dev, t.host, sizeof(DevDesc) * pos, hipMemcpyHostToDevice, stream));
  for (int c = 0; c < kClasses; ++c) {
    if (per_class[c] <= hydro::kArgDescs) continue;
    rc = dispatch_table(c, t.dev + off[c], per_class[c], dt, dx, amax, stream);
    if (rc) return rc;
  }
  return release_table(t, stream);
}

// ---- strategy 2: one launch per sub-grid over a pool of streams -----------
// The pool's streams (the paper's GPU executors, Section V-C) are created at
// first use, up to the largest count asked for, and kept until the process
// ends: creating a stream is set-up, not step work.
constexpr int kPoolMax = 128;

struct StreamPool {
  std::mutex mu;
  int created = 0;
  hipStream_t s[kPoolMax] = {};
  hipEvent_t done[kPoolMax] = {};
  hipEvent_t fork = nullptr;
};
StreamPool g_pool[kMaxDevices];

int pool_reserve(StreamPool& p, int k) {
  if (!p.fork) HIP_TRY(hipEventCreateWithFlags(&p.fork, hipEventDisableTiming));
  while (p.created < k) {
    HIP_TRY(hipStreamCreateWithFlags(&p.s[p.created], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&p.done[p.created], hipEventDisableTiming));
    ++p.created;
  }
  return HYDRO_OK;
}

// ---- allocation-free step (hydro_step_static) ----------------------------
// The descriptor table of hydro_step_static lives in `scratch`, a static
// device array (each GPU holds its own copy at its own address), and its host
// staging in a static host array per device.  In host code `scratch` names a
// host-side stand-in, never the device memory: its device address is taken
// once per device, with that device current, by hipGetSymbolAddress and used
// everywhere instead (copy destination, kernel arguments).
constexpr int kStaticMax = HYDRO_STATIC_MAX;
static __device__ __align__(256) DevDesc scratch[kStaticMax];

struct StaticState {
  std::mutex mu;
  DevDesc* dev = nullptr;  // device address of this device's `scratch`
  DevDesc host[kStaticMax];
};
StaticState g_static[kMaxDevices];

}  // namespace

namespace hydro {
namespace api {
int class_of_task(int n, int nf) { return class_of(n, nf); }

int launch_class_table(int cls, const DevDesc* table, int n, double dt, double dx, double* amax,
                       hipStream_t s) {
  return dispatch_table(cls, table, n, dt, dx, amax, s);
}

DevDesc device_desc(const hydro_subgrid_t& sg, int index) { return to_dev(sg, index); }

bool mixed_eligible(const int* num) {
  int present = 0, f = -1;
  for (int c = 0; c < kClasses; ++c) {
    if (!num[c]) continue;
    ++present;
    if (f < 0)
      f = c & 1;
    else if ((c & 1) != f)
      return false;
  }
  return present >= 2;
}

int launch_mixed(const int* num, const int* off, const DevDesc* host, const DevDesc* table,
                 int n, double dt, double dx, double* amax, hipStream_t s, bool parts,
                 int* groups) {
  int f = -1, present = 0;
  bool args = host != nullptr;
  for (int c = 0; c < kClasses; ++c)
    if (num[c]) {
      if (f >= 0 && (c & 1) != f) return fail(HYDRO_EINVAL, "multi-class launch of two field counts");
      f = c & 1;
      ++present;
      args = args && num[c] <= kArgDescs;
    }
  if (present < (parts ? 1 : 2)) return fail(HYDRO_EINVAL, "multi-class launch of %d classes", present);
  if (!args && !table) return fail(HYDRO_EINVAL, "%d descriptors need a device table", n);
  const bool f11 = f == 1;
  // segments in edge order; a class's path from its current tile
  int path[kMixedSegs], cls[kMixedSegs], nseg = 0;
  for (int e = 0; e < kMixedSegs; ++e) {
    const int c = 2 * e + f;
    if (!num[c]) continue;
    cls[nseg] = c;
    path[nseg++] = 2 * e + (g_tile[c].load(std::memory_order_relaxed) == 4 ? 1 : 0);
    if (groups) groups[c] = path_groups(path[nseg - 1]);
  }
  if (args) {
    MixedArgs m;
    memset(&m, 0, sizeof m);
    int start = 0, first = 0;
    for (int j = 0; j < nseg; ++j) {
      const int c = cls[j];
      m.seg[m.nseg++] = MixedSeg{start, num[c], path[j], first};
      for (int i = 0; i < num[c]; ++i) m.d[first + i] = host[off[c] + i];
      start += num[c] * path_groups(path[j]);
      first += num[c];
    }
    if (amax && !parts) {
      hipLaunchKernelGGL(amax_zero_mixed, dim3(1), dim3(64), 0, s, m, first, amax);
      HIP_TRY(hipGetLastError());
    }
    if (f11 && parts)
      hipLaunchKernelGGL((hydro_mixed_arg_kernel<11, true>), dim3(start), dim3(Lds8::kThreads), 0, s,
                         m, dt, dx, amax);
    else if (f11)
      hipLaunchKernelGGL((hydro_mixed_arg_kernel<11, false>), dim3(start), dim3(Lds8::kThreads), 0,
                         s, m, dt, dx, amax);
    else if (parts)
      hipLaunchKernelGGL((hydro_mixed_arg_kernel<6, true>), dim3(start), dim3(Lds8::kThreads), 0, s,
                         m, dt, dx, amax);
    else
      hipLaunchKernelGGL((hydro_mixed_arg_kernel<6, false>), dim3(start), dim3(Lds8::kThreads), 0, s,
                         m, dt, dx, amax);
    HIP_TRY(hipGetLastError());
    return HYDRO_OK;
  }
  MixedTable m;
  memset(&m, 0, sizeof m);
  int start = 0, most = 0;
  for (int j = 0; j < nseg; ++j) {
    const int c = cls[j];
    m.seg[m.nseg++] = MixedSeg{start, num[c], path[j], off[c]};
    most = num[c] > most ? num[c] : most;
    // segments start at multiples of 8: a sub-grid's work-groups stay on one XCD
    start += grid_for(num[c], path_groups(path[j]));
    start = (start + 7) / 8 * 8;
  }
  if (amax && !parts) {
    hipLaunchKernelGGL(amax_zero_mixed_table, dim3((most + 255) / 256), dim3(256), 0, s, table, m,
                       amax);
    HIP_TRY(hipGetLastError());
  }
  if (f11 && parts)
    hipLaunchKernelGGL((hydro_mixed_kernel<11, true>), dim3(start), dim3(Lds8::kThreads), 0, s,
                       table, m, dt, dx, amax);
  else if (f11)
    hipLaunchKernelGGL((hydro_mixed_kernel<11, false>), dim3(start), dim3(Lds8::kThreads), 0, s,
                       table, m, dt, dx, amax);
  else if (parts)
    hipLaunchKernelGGL((hydro_mixed_kernel<6, true>), dim3(start), dim3(Lds8::kThreads), 0, s,
                       table, m, dt, dx, amax);
  else
    hipLaunchKernelGGL((hydro_mixed_kernel<6, false>), dim3(start), dim3(Lds8::kThreads), 0, s,
                       table, m, dt, dx, amax);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int validate_batch(const hydro_subgrid_t* sg, int32_t count, double dt, double dx) {
  return validate(sg, count, dt, dx);
}
}  // namespace api
}  // namespace hydro

// ---- plans ---------------------------------------------------------------
struct hydro_plan {
  int device = 0;
  DevDesc* table = nullptr;  // device, classes contiguous
  int count = 0;
  int off[kClasses] = {0};
  int num[kClasses] = {0};
  // graph of one step, captured on a private stream for given (dt, dx, amax)
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double g_dt = -1.0, g_dx = -1.0;
  double* g_amax = nullptr;
  uint64_t g_tiles = ~0ull;  // tile epoch of the captured graph
  // Branches of the captured graph: every class after the first is captured
  // on a side stream forked from the capture stream (fork event) and joined
  // back (its own event), so the classes are independent graph nodes that
  // run concurrently and the partly filled last wave of one class's
  // work-groups overlaps the work of the others.
  hipStream_t side[kClasses] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kClasses] = {};
};

namespace {

int plan_launches(hydro_plan* p, double dt, double dx, double* amax, hipStream_t s) {
  // several classes of one field count: one multi-class launch (as
  // hydro_step does)
  if (hydro::api::mixed_eligible(p->num))
    return hydro::api::launch_mixed(p->num, p->off, nullptr, p->table, p->count, dt, dx, amax, s);
  for (int c = 0; c < kClasses; ++c) {
    if (!p->num[c]) continue;
    int rc = dispatch_table(c, p->table + p->off[c], p->num[c], dt, dx, amax, s);
    if (rc) return rc;
  }
  return HYDRO_OK;
}

// Record one step into the graph being captured on p->capture.  Never
// returns early: a failed call still leaves every side stream joined, so
// the caller can always end the capture.
int plan_capture_branches(hydro_plan* p, double dt, double dx, double* amax) {
  int rc = HYDRO_OK;
  auto hip = [&rc](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == HYDRO_OK)
      rc = fail(HYDRO_EHIP, "%s failed: %s", what, hipGetErrorString(e));
    return e == hipSuccess;
  };
  // several classes of one field count: one multi-class launch, whatever
  // their sizes (as fast as branches for large classes, without the fork
  // and join)
  if (hydro::api::mixed_eligible(p->num))
    return hydro::api::launch_mixed(p->num, p->off, nullptr, p->table, p->count, dt, dx, amax,
                                    p->capture);
  bool big[kClasses] = {};
  int nbig = 0;
  for (int c = 0; c < kClasses; ++c)
    if (p->num[c] && class_groups(c, p->num[c]) >= kBranchGroups) {
      big[c] = true;
      ++nbig;
    }
  bool done[kClasses] = {};
  if (nbig >= 2 && hip(hipEventRecord(p->fork, p->capture), "hipEventRecord(fork)")) {
    // the first large class on the capture stream, every other large class
    // on a branch of its own (captured in class order: the graph starts its
    // nodes in that order)
    bool first = true;
    for (int c = 0; c < kClasses; ++c) {
      if (!big[c]) continue;
      if (first) {
        first = false;
        done[c] = true;
        if (rc == HYDRO_OK) rc = dispatch_table(c, p->table + p->off[c], p->num[c], dt, dx, amax, p->capture);
        continue;
      }
      if (!hip(hipStreamWaitEvent(p->side[c], p->fork, 0), "hipStreamWaitEvent(fork)")) continue;
      done[c] = true;
      if (rc == HYDRO_OK) {
        int r = dispatch_table(c, p->table + p->off[c], p->num[c], dt, dx, amax, p->side[c]);
        if (r) rc = r;
      }
      if (hip(hipEventRecord(p->join[c], p->side[c]), "hipEventRecord(join)"))
        hip(hipStreamWaitEvent(p->capture, p->join[c], 0), "hipStreamWaitEvent(join)");
    }
  }
  // the rest on the capture stream: the small classes (below kBranchGroups)
  // as one multi-class launch when they are several of one field count, the
  // others one launch each
  for (int f = 0; f < 2; ++f) {
    int small[kClasses] = {0}, n = 0;
    for (int c = f; c < kClasses; c += 2)
      if (!done[c] && p->num[c] && !big[c]) {
        small[c] = p->num[c];
        n += small[c];
      }
    if (!hydro::api::mixed_eligible(small)) continue;
    for (int c = f; c < kClasses; c += 2)
      if (small[c]) done[c] = true;
    if (rc == HYDRO_OK)
      rc = hydro::api::launch_mixed(small, p->off, nullptr, p->table, n, dt, dx, amax, p->capture);
  }
  for (int c = 0; c < kClasses; ++c) {
    if (!p->num[c] || done[c]) continue;
    if (rc == HYDRO_OK) rc = dispatch_table(c, p->table + p->off[c], p->num[c], dt, dx, amax, p->capture);
  }
  return rc;
}

void plan_free(hydro_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->table) (void)hipFree(p->table);
  for (int c = 0; c < kClasses; ++c) {
    if (p->join[c]) (void)hipEventDestroy(p->join[c]);
    if (p->side[c]) (void)hipStreamDestroy(p->side[c]);
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->capture) (void)hipStreamDestroy(p->capture);
  delete p;
}

}  // namespace

namespace hydro {
namespace api {
int plan_enqueue(hydro_plan* p, double dt, double dx, double* amax, hipStream_t s) {
  return plan_launches(p, dt, dx, amax, s);
}
}  // namespace api
}  // namespace hydro

extern "C" {

int hydro_step(const hydro_subgrid_t* sg, int32_t count, double dt, double dx,
               double* amax_dev, void* stream) {
  g_err[0] = '\0';
  int rc = validate(sg, count, dt, dx);
  if (rc) return rc;
  if (count == 0) return HYDRO_OK;
  DeviceState* st;
  rc = device_state(&st);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int base = 0; base < count; base += kSlotCap) {
    int n = count - base < kSlotCap ? count - base : kSlotCap;
    rc = step_chunk(st, nullptr, sg + base, n, base, dt, dx, amax_dev, s);
    if (rc) return rc;
  }
  return HYDRO_OK;
}

int hydro_step_static(const hydro_subgrid_t* sg, int32_t count, double dt, double dx,
                      double* amax_dev, void* stream) {
  g_err[0] = '\0';
  int rc = validate(sg, count, dt, dx);
  if (rc) return rc;
  if (count > kStaticMax)
    return fail(HYDRO_EINVAL, "count %d exceeds HYDRO_STATIC_MAX (%d) of hydro_step_static", count,
                kStaticMax);
  if (count == 0) return HYDRO_OK;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HYDRO_EINVAL, "device %d out of range", dev);
  StaticState& st = g_static[dev];
  std::lock_guard<std::mutex> lk(st.mu);
  if (!st.dev) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HYDRO_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
    st.dev = static_cast<DevDesc*>(p);
  }
  const FixedTable fixed{st.host, st.dev};
  return step_chunk(nullptr, &fixed, sg, count, 0, dt, dx, amax_dev, (hipStream_t)stream);
}

int hydro_step_streams(const hydro_subgrid_t* sg, int32_t count, double dt, double dx,
                       double* amax_dev, int32_t n_streams, void* stream) {
  g_err[0] = '\0';
  int rc = validate(sg, count, dt, dx);
  if (rc) return rc;
  if (n_streams < 1 || n_streams > kPoolMax)
    return fail(HYDRO_EINVAL, "n_streams %d outside 1..%d", n_streams, kPoolMax);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HYDRO_EINVAL, "device %d out of range", dev);
  StreamPool& p = g_pool[dev];
  std::lock_guard<std::mutex> lk(p.mu);
  rc = pool_reserve(p, n_streams);
  if (rc || count == 0) return rc;
  hipStream_t caller = (hipStream_t)stream;
  const int k = n_streams < count ? n_streams : count;
  // the pool's streams start after the work already queued on `stream` ...
  HIP_TRY(hipEventRecord(p.fork, caller));
  for (int j = 0; j < k; ++j) HIP_TRY(hipStreamWaitEvent(p.s[j], p.fork, 0));
  for (int i = 0; i < count; ++i) {
    ArgDescs a;
    memset(&a, 0, sizeof a);
    a.d[0] = to_dev(sg[i], i);
    rc = dispatch_args(class_of(sg[i].n, sg[i].nfields), a, 1, dt, dx, amax_dev, p.s[i % k]);
    if (rc) return rc;
  }
  // ... and `stream` continues after all of them
  for (int j = 0; j < k; ++j) {
    HIP_TRY(hipEventRecord(p.done[j], p.s[j]));
    HIP_TRY(hipStreamWaitEvent(caller, p.done[j], 0));
  }
  return HYDRO_OK;
}

int hydro_step26(const hydro_subgrid_t* sg, int32_t count, double dt, double dx,
                 double* amax_dev, void* stream) {
  g_err[0] = '\0';
  int rc = validate(sg, count, dt, dx);
  if (rc) return rc;
  if (count == 0) return HYDRO_OK;
  const int nf = sg[0].nfields;
  for (int i = 0; i < count; ++i)
    if (sg[i].n != 8 || sg[i].nfields != nf)
      return fail(HYDRO_EINVAL, "sub-grid %d: the 26-point step takes n = 8 and one field count", i);
  DeviceState* st;
  rc = device_state(&st);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int base = 0; base < count; base += kSlotCap) {
    const int n = count - base < kSlotCap ? count - base : kSlotCap;
    TableLease t;
    rc = lease_table(st, nullptr, t);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) t.host[i] = to_dev(sg[base + i], base + i);
    HIP_TRY(hipMemcpyAsync(t.dev, t.host, sizeof(DevDesc) * n, hipMemcpyHostToDevice, s));
    if (nf == 11)
      hipLaunchKernelGGL(hydro::hydro_step26_kernel<11>, dim3(n), dim3(hydro::S26::kThreads), 0, s,
                         t.dev, n, dt, dx, amax_dev);
    else
      hipLaunchKernelGGL(hydro::hydro_step26_kernel<6>, dim3(n), dim3(hydro::S26::kThreads), 0, s,
                         t.dev, n, dt, dx, amax_dev);
    HIP_TRY(hipGetLastError());
    rc = release_table(t, s);
    if (rc) return rc;
  }
  return HYDRO_OK;
}

int hydro_step_each(const hydro_subgrid_t* sg, int32_t count, double dt,
                    double dx, double* amax_dev, void* stream) {
  g_err[0] = '\0';
  int rc = validate(sg, count, dt, dx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < count; ++i) {
    ArgDescs a;
    memset(&a, 0, sizeof a);
    a.d[0] = to_dev(sg[i], i);
    rc = dispatch_args(class_of(sg[i].n, sg[i].nfields), a, 1, dt, dx, amax_dev, s);
    if (rc) return rc;
  }
  return HYDRO_OK;
}


int hydro_plan_create(hydro_plan_t** out, const hydro_subgrid_t* sg, int32_t count) {
  g_err[0] = '\0';
  if (!out) return fail(HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(sg, count, 0.0, 1.0);
  if (rc) return rc;
  hydro_plan* p = new hydro_plan();
  HIP_TRY(hipGetDevice(&p->device));
  p->count = count;
  std::vector<DevDesc> host((size_t)(count > 0 ? count : 1));
  for (int i = 0; i < count; ++i) p->num[class_of(sg[i].n, sg[i].nfields)]++;
  int pos = 0;
  for (int c = 0; c < kClasses; ++c) {
    p->off[c] = pos;
    pos += p->num[c];
  }
  int fill[kClasses];
  memcpy(fill, p->off, sizeof fill);
  for (int i = 0; i < count; ++i) host[fill[class_of(sg[i].n, sg[i].nfields)]++] = to_dev(sg[i], i);
  {
    // capture stream, and a side stream + join event for every class present
    // after the first (see plan_capture_branches)
    hipError_t e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    bool first = true;
    for (int c = 0; c < kClasses && e == hipSuccess; ++c) {
      if (!p->num[c]) continue;
      if (first) {
        first = false;
        continue;
      }
      e = hipStreamCreateWithFlags(&p->side[c], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[c], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      plan_free(p);
      return fail(HYDRO_EHIP, "plan streams/events: %s", hipGetErrorString(e));
    }
  }
  if (count > 0) {
    hipError_t e = hipMalloc((void**)&p->table, sizeof(DevDesc) * count);
    if (e != hipSuccess) {
      plan_free(p);
      return fail(HYDRO_EHIP, "hipMalloc(plan table): %s", hipGetErrorString(e));
    }
    e = hipMemcpy(p->table, host.data(), sizeof(DevDesc) * count, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      plan_free(p);
      return fail(HYDRO_EHIP, "hipMemcpy(plan table): %s", hipGetErrorString(e));
    }
  }
  *out = p;
  return HYDRO_OK;
}

int hydro_plan_step(hydro_plan_t* p, double dt, double dx, double* amax_dev, void* stream) {
  g_err[0] = '\0';
  if (!p) return fail(HYDRO_EINVAL, "plan is NULL");
  int rc = validate(nullptr, 0, dt, dx);
  if (rc) return rc;
  return plan_launches(p, dt, dx, amax_dev, (hipStream_t)stream);
}

int hydro_plan_launch_graph(hydro_plan_t* p, double dt, double dx, double* amax_dev, void* stream) {
  g_err[0] = '\0';
  if (!p) return fail(HYDRO_EINVAL, "plan is NULL");
  int rc = validate(nullptr, 0, dt, dx);
  if (rc) return rc;
  if (p->count == 0) return HYDRO_OK;
  const uint64_t tiles = g_tile_epoch.load(std::memory_order_acquire);
  if (!p->exec || p->g_dt != dt || p->g_dx != dx || p->g_amax != amax_dev || p->g_tiles != tiles) {
    // (re)capture one step on the plan's private stream
    if (p->exec) {
      (void)hipGraphExecDestroy(p->exec);
      p->exec = nullptr;
    }
    if (p->graph) {
      (void)hipGraphDestroy(p->graph);
      p->graph = nullptr;
    }
    HIP_TRY(hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal));
    rc = plan_capture_branches(p, dt, dx, amax_dev);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->capture, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(HYDRO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    p->graph = g;
    HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->g_dt = dt;
    p->g_dx = dx;
    p->g_amax = amax_dev;
    p->g_tiles = tiles;
  }
  HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream));
  return HYDRO_OK;
}

int hydro_plan_pattern_floor(hydro_plan_t* p, int32_t same_lds, void* stream) {
  g_err[0] = '\0';
  if (!p) return fail(HYDRO_EINVAL, "plan is NULL");
  if (p->count == 0) return HYDRO_OK;
  int cls = -1;
  for (int c = 0; c < kClasses; ++c)
    if (p->num[c]) {
      if (cls >= 0 || (c != class_of(8, 6) && c != class_of(8, 11)))
        return fail(HYDRO_EINVAL, "the pattern kernel takes plans of n = 8 and one field count");
      cls = c;
    }
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid(p->count), block(hydro::Lds8::kThreads);
  const DevDesc* table = p->table + p->off[cls];
  const bool f11 = cls == class_of(8, 11);
  if (f11 && same_lds)
    hipLaunchKernelGGL((hydro::hydro_pattern_kernel<11, true>), grid, block, 0, s, table, p->count);
  else if (f11)
    hipLaunchKernelGGL((hydro::hydro_pattern_kernel<11, false>), grid, block, 0, s, table, p->count);
  else if (same_lds)
    hipLaunchKernelGGL((hydro::hydro_pattern_kernel<6, true>), grid, block, 0, s, table, p->count);
  else
    hipLaunchKernelGGL((hydro::hydro_pattern_kernel<6, false>), grid, block, 0, s, table, p->count);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int hydro_plan_destroy(hydro_plan_t* p) {
  g_err[0] = '\0';
  if (!p) return HYDRO_OK;
  int rc = HYDRO_OK;
  if (hipDeviceSynchronize() != hipSuccess) rc = fail(HYDRO_EHIP, "hipDeviceSynchronize failed");
  plan_free(p);
  return rc;
}

const char* hydro_last_error(void) { return g_err; }

#ifndef HYDRO_SRC_HASH
#define HYDRO_SRC_HASH "unknown"
#endif
#ifndef HYDRO_KERNEL_HASH
#define HYDRO_KERNEL_HASH "unknown"
#endif
int hydro_set_tile(int32_t n, int32_t nfields, int32_t tile) {
  hydro::api::clear_error();
  const int c = class_of(n, nfields);
  if (c < 0) return fail(HYDRO_EINVAL, "unsupported n=%d nfields=%d", n, nfields);
  if (tile != 4 && tile != 8) return fail(HYDRO_EINVAL, "tile %d (4 or 8)", tile);
  g_tile[c].store(tile, std::memory_order_relaxed);
  g_tile_epoch.fetch_add(1, std::memory_order_acq_rel);
  return HYDRO_OK;
}

int hydro_get_tile(int32_t n, int32_t nfields, int32_t* tile) {
  hydro::api::clear_error();
  const int c = class_of(n, nfields);
  if (c < 0) return fail(HYDRO_EINVAL, "unsupported n=%d nfields=%d", n, nfields);
  if (!tile) return fail(HYDRO_EINVAL, "tile is NULL");
  *tile = g_tile[c].load(std::memory_order_relaxed);
  return HYDRO_OK;
}

}  // extern "C"

namespace hydro {
// The kernels' reciprocal and reciprocal square root on caller-given
// arguments (diagnostic entry point hydro_math_check).
__global__ void math_check_kernel(const double* __restrict__ x, int n,
                                  double* __restrict__ r, double* __restrict__ q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    r[i] = recip(x[i]);
    q[i] = rsq_pos(x[i]);
  }
}
}  // namespace hydro

extern "C" {

int hydro_math_check(const double* x, int32_t n, double* recip_out, double* rsqrt_out,
                     void* stream) {
  g_err[0] = '\0';
  if (n < 0) return fail(HYDRO_EINVAL, "n %d < 0", n);
  if (n == 0) return HYDRO_OK;
  if (!x || !recip_out || !rsqrt_out) return fail(HYDRO_EINVAL, "NULL pointer");
  hipLaunchKernelGGL(hydro::math_check_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, x, n, recip_out, rsqrt_out);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

const char* hydro_version(void) {
  return "hydroagg gfx950 src " HYDRO_SRC_HASH " kernels " HYDRO_KERNEL_HASH;
}

}  // extern "C"

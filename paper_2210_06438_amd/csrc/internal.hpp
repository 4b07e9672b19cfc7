// internal.hpp -- helpers shared by the translation units of libhydroagg.so
// (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/hydroagg.h"
#include "hydro_kernel.hpp"

namespace hydro {
namespace api {

// Record the calling thread's error text; returns `code`.
int fail(int code, const char* fmt, ...);
void clear_error();

// Shape class (0..5) of an (n, nfields) pair, or -1.
int class_of_task(int n, int nf);
constexpr int kNumClasses = 6;

// One table launch of shape class `cls` (current tile) over n sub-grids
// whose descriptors are table[0..n).
int launch_class_table(int cls, const DevDesc* table, int n, double dt, double dx, double* amax,
                       hipStream_t s);

// Device descriptor of task `sg` at batch position `index`.
DevDesc device_desc(const hydro_subgrid_t& sg, int index);

// Argument checks of hydro_step (0 or HYDRO_EINVAL).
int validate_batch(const hydro_subgrid_t* sg, int32_t count, double dt, double dx);

// True when a batch with per-class counts num[] can be one launch_mixed:
// at least two classes present, all of one field count.
bool mixed_eligible(const int* num);

// One launch for every class of such a batch (hydro_mixed.hpp): class c has
// num[c] sub-grids whose descriptors start at index off[c], n in all.  When
// `host` is given and every class has at most kArgDescs they are read from
// `host` into the kernel arguments; otherwise from the device table `table`
// (table + off[c] for class c).  amax: without `parts`, one slot per
// sub-grid, zeroed first on the same stream; with `parts` (one class or
// more), kAmaxParts partials per sub-grid written with plain stores and
// nothing zeroed, and groups[c] receives the work-groups per sub-grid of
// class c (the partials to read).
int launch_mixed(const int* num, const int* off, const DevDesc* host, const DevDesc* table,
                 int n, double dt, double dx, double* amax, hipStream_t s, bool parts = false,
                 int* groups = nullptr);

// The launches of one step of a plan (hydro_plan_step without its argument
// checks) on stream s; usable inside a stream capture.
int plan_enqueue(hydro_plan* p, double dt, double dx, double* amax, hipStream_t s);

}  // namespace api
}  // namespace hydro

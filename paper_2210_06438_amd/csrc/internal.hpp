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

// Argument checks of hydro_step (0 or HYDRO_EINVAL).
int validate_batch(const hydro_subgrid_t* sg, int32_t count, double dt, double dx);

// One aggregated launch of `n` sub-grids of class `cls` whose descriptors are
// at `table` (device memory), on stream `s`.
int launch_class(int cls, const DevDesc* table, int n, double dt, double dx, double* amax,
                 hipStream_t s);
// True when class `cls` steps each sub-grid with one work-group, which then
// writes its amax slot with a plain store (no zeroing, no atomics).
bool class_single_block(int cls);

// The same with at most kArgDescs descriptors read from host memory and
// passed in the kernel arguments (no descriptor copy on the stream).
int launch_class_args(int cls, const DevDesc* host, int n, double dt, double dx, double* amax,
                      hipStream_t s);

// True when a batch with per-class counts num[] can be one launch_mixed:
// at least two classes present, all of one field count.
bool mixed_eligible(const int* num);

// One launch for every class of such a batch (hydro_mixed.hpp): class c has
// num[c] sub-grids whose descriptors start at index off[c], n in all.  When
// `host` is given and every class has at most kArgDescs they are read from
// `host` into the kernel arguments; otherwise from the device table `table`
// (table + off[c] for class c).  amax slots (if amax is not NULL) are
// zeroed first, on the same stream.
int launch_mixed(const int* num, const int* off, const DevDesc* host, const DevDesc* table,
                 int n, double dt, double dx, double* amax, hipStream_t s);

}  // namespace api
}  // namespace hydro

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

}  // namespace api
}  // namespace hydro

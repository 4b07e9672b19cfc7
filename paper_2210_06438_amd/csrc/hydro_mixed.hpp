// hydro_mixed.hpp -- one launch for a batch whose sub-grids fall in several
// shape classes of one field count (edges 8, 12, 16).
//
// The class kernels of hydro_lds8.hpp and hydro_q4.hpp step one class per
// launch, so a batch of three classes is three launches in sequence: the
// second class starts only once the last work-group of the first has
// finished, and a lightly loaded batch (a few work-groups per class) takes
// the sum of three work-group lifetimes.  Here the grid is the
// concatenation of the classes' grids, in segments; a work-group finds its
// segment from its index and runs that class's tile path (the same step
// functions, so every sub-grid gets the same arithmetic as in its class
// kernel).  The classes then run side by side and the batch takes about
// the longest of them.  All paths share the LDS arrays of hydro_lds8.hpp,
// so the kernel needs the LDS of one work-group of the largest path.
#pragma once

#include "hydro_q4.hpp"

namespace hydro {

// Tile path of a segment: edge n and tile.
enum MixedPath : int { kP8T8 = 0, kP8T4, kP12T8, kP12T4, kP16T8, kP16T4, kPaths };

constexpr int kMixedSegs = 3;   // classes of one field count: n = 8, 12, 16

// Work-groups per sub-grid of a path.
__host__ __device__ constexpr int path_groups(int path) {
  return path == kP8T8 ? Blocks<14>::kPerSubgrid
       : path == kP8T4 ? Q4Grid<14>::kGroups
       : path == kP12T8 ? Blocks<18>::kPerSubgrid
       : path == kP12T4 ? Q4Grid<18>::kGroups
       : path == kP16T8 ? Blocks<22>::kPerSubgrid
                        : Q4Grid<22>::kGroups;
}

struct MixedSeg {
  int start;   // first work-group of the segment in the grid
  int count;   // sub-grids
  int path;    // MixedPath
  int first;   // first descriptor of the segment
};

// Segments of a batch whose descriptors are in device memory: one table,
// passed to the kernel as a separate restrict-qualified argument (the
// compiler then treats its loads as invariant and keeps the descriptor out
// of the registers that the step needs -- with the table pointers inside
// this struct instead, the kernel spilled 52-60 bytes per lane).
struct MixedTable {
  MixedSeg seg[kMixedSegs];
  int nseg;
};

// Descriptors in the kernel arguments: at most kArgDescs per segment (576
// bytes of arguments; a larger block -- 64 descriptors, 1.5 KB -- made each
// launch measurably slower).
struct MixedArgs {
  DevDesc d[kMixedSegs * kArgDescs];
  MixedSeg seg[kMixedSegs];
  int nseg;
};

template <int F, int MP, bool PARTS>
__device__ __forceinline__ void lds8_block(const DevDesc& d, int b, double dt, double dx,
                                           double* __restrict__ amax_out) {
  constexpr int B = Blocks<MP>::kPerSubgrid;
  int org, ox, oy, oz, lox, loy, loz;
  Blocks<MP>::geo(b, org, ox, oy, oz, lox, loy, loz);
  lds8_step<F, MP, (B > 1), PARTS>(d, org, ox, oy, oz, lox, loy, loz, dt, dx, amax_out, b);
}

// Work-group `b` of sub-grid `d` on tile path PATH.  PARTS: amax as
// per-work-group partials (kAmaxParts per sub-grid, plain stores), else
// combined in the sub-grid's slot as the class kernels do.
template <int F, int PATH, bool PARTS>
__device__ __forceinline__ void run_path(const DevDesc& d, int b, double dt, double dx,
                                         double* __restrict__ amax_out) {
  if constexpr (PATH == kP8T8) lds8_block<F, 14, PARTS>(d, b, dt, dx, amax_out);
  if constexpr (PATH == kP8T4) q4_step<F, 14, PARTS>(d, b, dt, dx, amax_out);
  if constexpr (PATH == kP12T8) lds8_block<F, 18, PARTS>(d, b, dt, dx, amax_out);
  if constexpr (PATH == kP12T4) q4_step<F, 18, PARTS>(d, b, dt, dx, amax_out);
  if constexpr (PATH == kP16T8) lds8_block<F, 22, PARTS>(d, b, dt, dx, amax_out);
  if constexpr (PATH == kP16T4) q4_step<F, 22, PARTS>(d, b, dt, dx, amax_out);
}

// Work-group lw of a table segment: the mapping of the class kernels, with
// the path's work-groups per sub-grid a compile-time constant (the
// descriptor index then stays scalar and the descriptor in scalar
// registers).
template <int F, int PATH, bool PARTS>
__device__ __forceinline__ void table_path(const DevDesc* __restrict__ table, int first, int count,
                                           int lw, double dt, double dx,
                                           double* __restrict__ amax_out) {
  constexpr int B = path_groups(PATH);
  const int s = B == 1 ? lw : (lw / (8 * B)) * 8 + (lw & 7);
  const int b = B == 1 ? 0 : (lw >> 3) % B;
  if (s >= count) return;
  const DevDesc d = table[first + s];
  run_path<F, PATH, PARTS>(d, b, dt, dx, amax_out);
}

template <int F, int PATH, bool PARTS>
__device__ __forceinline__ void arg_path(const MixedArgs& m, int first, int lw, double dt,
                                         double dx, double* __restrict__ amax_out) {
  constexpr int B = path_groups(PATH);
  const DevDesc d = m.d[first + lw / B];
  run_path<F, PATH, PARTS>(d, lw % B, dt, dx, amax_out);
}

// Segment of work-group w: the last segment that starts at or before it.
__device__ __forceinline__ int mixed_segment(const MixedSeg (&seg)[kMixedSegs], int nseg, int w) {
  int j = 0;
  if (nseg > 1 && w >= seg[1].start) j = 1;
  if (nseg > 2 && w >= seg[2].start) j = 2;
  return j;
}

// Table form (a segment of more than kArgDescs sub-grids).  Within a segment
// the work-groups of a sub-grid have indices equal modulo 8 (segments start
// at multiples of 8), as in the class kernels.
template <int F, bool PARTS>
__global__ void __launch_bounds__(Lds8::kThreads, 2)
    hydro_mixed_kernel(const DevDesc* __restrict__ table, MixedTable m, double dt, double dx,
                       double* __restrict__ amax_out) {
  const int w = blockIdx.x;
  const int j = mixed_segment(m.seg, m.nseg, w);
  const MixedSeg sg = m.seg[j];
  const int lw = w - sg.start;
  switch (sg.path) {
    case kP8T8: table_path<F, kP8T8, PARTS>(table, sg.first, sg.count, lw, dt, dx, amax_out); break;
    case kP8T4: table_path<F, kP8T4, PARTS>(table, sg.first, sg.count, lw, dt, dx, amax_out); break;
    case kP12T8: table_path<F, kP12T8, PARTS>(table, sg.first, sg.count, lw, dt, dx, amax_out); break;
    case kP12T4: table_path<F, kP12T4, PARTS>(table, sg.first, sg.count, lw, dt, dx, amax_out); break;
    case kP16T8: table_path<F, kP16T8, PARTS>(table, sg.first, sg.count, lw, dt, dx, amax_out); break;
    default: table_path<F, kP16T4, PARTS>(table, sg.first, sg.count, lw, dt, dx, amax_out); break;
  }
}

// Argument form: segment j holds seg[j].count * path_groups work-groups,
// sub-grid-major.
template <int F, bool PARTS>
__global__ void __launch_bounds__(Lds8::kThreads, 2)
    hydro_mixed_arg_kernel(MixedArgs m, double dt, double dx, double* __restrict__ amax_out) {
  const int w = blockIdx.x;
  const int j = mixed_segment(m.seg, m.nseg, w);
  const MixedSeg sg = m.seg[j];
  const int lw = w - sg.start;
  switch (sg.path) {
    case kP8T8: arg_path<F, kP8T8, PARTS>(m, sg.first, lw, dt, dx, amax_out); break;
    case kP8T4: arg_path<F, kP8T4, PARTS>(m, sg.first, lw, dt, dx, amax_out); break;
    case kP12T8: arg_path<F, kP12T8, PARTS>(m, sg.first, lw, dt, dx, amax_out); break;
    case kP12T4: arg_path<F, kP12T4, PARTS>(m, sg.first, lw, dt, dx, amax_out); break;
    case kP16T8: arg_path<F, kP16T8, PARTS>(m, sg.first, lw, dt, dx, amax_out); break;
    default: arg_path<F, kP16T4, PARTS>(m, sg.first, lw, dt, dx, amax_out); break;
  }
}

// amax slots of a table-form batch set to zero before the launch: lane i of
// the grid clears slot i of every segment that has one.
__global__ void amax_zero_mixed_table(const DevDesc* __restrict__ table, MixedTable m,
                                      double* __restrict__ amax_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int j = 0; j < m.nseg; ++j)
    if (i < m.seg[j].count) amax_out[table[m.seg[j].first + i].index] = 0.0;
}

// amax slots of an argument-form batch set to zero before the launch (one
// work-group of 64 lanes).
__global__ void amax_zero_mixed(MixedArgs m, int count, double* __restrict__ amax_out) {
  const int i = threadIdx.x;
  if (i < count) amax_out[m.d[i].index] = 0.0;
}

}  // namespace hydro

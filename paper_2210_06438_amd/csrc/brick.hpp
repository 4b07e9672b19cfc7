// brick.hpp -- device kernels of the multi-stage time-step on a brick of
// sub-grids: ghost-layer fill from neighbouring interiors (with periodic or
// outflow domain boundaries) and the stage combination of the three-stage
// SSP Runge-Kutta method.  Both are plain HBM-bound copies / blends: no
// MFMA, no LDS; lanes walk the stored cells of one (sub-grid, field) in
// memory order so that loads and stores of a work-group are coalesced rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hydro {

struct BrickGeo {
  int nf;          // fields
  int nb[3];       // sub-grids along x, y, z
  int bc[3];       // 0 periodic, 1 outflow
  long sg_stride;  // doubles per sub-grid: nf * M^3
};

// Domain coordinate that cell coordinate g (possibly outside [0, L))
// stands for under boundary condition bc.
__device__ __forceinline__ int brick_map(int g, int L, int bc) {
  if (bc == 0) {
    g %= L;
    return g < 0 ? g + L : g;
  }
  return g < 0 ? 0 : (g >= L ? L - 1 : g);
}

// One work-group per (sub-grid, field).  Every ghost cell of the stored
// (N+6)^3 block takes the value of the domain cell it stands for, which is
// always an interior cell of some sub-grid (possibly this one): sources are
// interiors, destinations ghosts, so filling in place is race-free.
template <int N>
__global__ void __launch_bounds__(256) ghost_fill_kernel(double* u, BrickGeo g) {
  constexpr int M = N + 6;
  constexpr int M3 = M * M * M;
  const int s = blockIdx.x / g.nf;
  const int f = blockIdx.x - s * g.nf;
  const int bx = s % g.nb[0];
  const int by = (s / g.nb[0]) % g.nb[1];
  const int bz = s / (g.nb[0] * g.nb[1]);
  double* dst = u + s * g.sg_stride + (long)f * M3;
  const double* fld = u + (long)f * M3;   // field f of sub-grid 0
  for (int e = threadIdx.x; e < M3; e += blockDim.x) {
    const int x = e % M, y = (e / M) % M, z = e / (M * M);
    const bool inx = x >= 3 && x < N + 3, iny = y >= 3 && y < N + 3, inz = z >= 3 && z < N + 3;
    if (inx && iny && inz) continue;
    const int gx = brick_map(bx * N + x - 3, N * g.nb[0], g.bc[0]);
    const int gy = brick_map(by * N + y - 3, N * g.nb[1], g.bc[1]);
    const int gz = brick_map(bz * N + z - 3, N * g.nb[2], g.bc[2]);
    const int sx = gx / N, sy = gy / N, sz = gz / N;
    const long src = ((long)(sz * g.nb[1] + sy) * g.nb[0] + sx) * g.sg_stride +
                     ((gz - sz * N + 3) * M + (gy - sy * N + 3)) * M + (gx - sx * N + 3);
    dst[e] = fld[src];
  }
}

// Face ghosts only: the 6 slabs of 3 x N x N ghost cells whose other two
// coordinates are interior -- the only ghosts the face-centre step reads (it
// marches the lines whose transverse coordinates are interior).  Edge and
// corner ghosts are left as they are.  Grid (sub-grids, kFaceParts<N>) of
// 256-lane work-groups, one lane per slab cell; the lane maps its cell once
// and moves its F fields, all loads before the stores, so F loads are in
// flight together (sources are interiors and destinations ghosts, so the
// two views of the buffer never touch the same element: restrict).  Slab
// cells are enumerated with x fastest where x is interior (rows of N).
template <int N>
constexpr int kFaceParts = (6 * 3 * N * N + 255) / 256;

template <int N, int F>
__global__ void __launch_bounds__(256) ghost_fill_faces_kernel(double* __restrict__ dst_all,
                                                               const double* __restrict__ src_all,
                                                               BrickGeo g) {
  constexpr int M = N + 6;
  constexpr long M3 = (long)M * M * M;
  constexpr int SL = 3 * N * N;                   // cells of one slab
  const int s = blockIdx.x;                       // sub-grid
  const int e = blockIdx.y * 256 + threadIdx.x;   // slab cell
  if (e >= 6 * SL) return;
  const int k = e / SL, q = e - k * SL;   // slab k: z low/high, y low/high, x low/high
  const int hi = k & 1;
  int x, y, z;
  if (k < 2) {          // z slab: q = (layer * N + y) * N + x
    x = q % N + 3;
    y = (q / N) % N + 3;
    const int l = q / (N * N);
    z = hi ? N + 3 + l : l;
  } else if (k < 4) {   // y slab: q = (z * 3 + layer) * N + x
    x = q % N + 3;
    const int l = (q / N) % 3;
    y = hi ? N + 3 + l : l;
    z = q / (3 * N) + 3;
  } else {              // x slab: q = (z * N + y) * 3 + layer
    const int l = q % 3;
    x = hi ? N + 3 + l : l;
    y = (q / 3) % N + 3;
    z = q / (3 * N) + 3;
  }
  const int bx = s % g.nb[0];
  const int by = (s / g.nb[0]) % g.nb[1];
  const int bz = s / (g.nb[0] * g.nb[1]);
  const int gx = brick_map(bx * N + x - 3, N * g.nb[0], g.bc[0]);
  const int gy = brick_map(by * N + y - 3, N * g.nb[1], g.bc[1]);
  const int gz = brick_map(bz * N + z - 3, N * g.nb[2], g.bc[2]);
  const int sx = gx / N, sy = gy / N, sz = gz / N;
  const double* __restrict__ src =
      src_all + ((long)(sz * g.nb[1] + sy) * g.nb[0] + sx) * g.sg_stride +
      ((gz - sz * N + 3) * M + (gy - sy * N + 3)) * M + (gx - sx * N + 3);
  double* __restrict__ dst = dst_all + s * g.sg_stride + (z * M + y) * M + x;
  double v[F];
#pragma unroll
  for (int f = 0; f < F; ++f) v[f] = src[f * M3];
#pragma unroll
  for (int f = 0; f < F; ++f) dst[f * M3] = v[f];
}

// out = a x + b y on the interior cells of every sub-grid, each product and
// the sum rounded once (no contraction).  One work-group per (sub-grid,
// field).  out may be x or y itself: each element is read and written by
// the same lane.
template <int N>
__global__ void __launch_bounds__(256) rk_combine_kernel(double* out, const double* x,
                                                         const double* y, double a, double b,
                                                         long sg_stride, int nf) {
  constexpr int M = N + 6;
  constexpr long M3 = (long)M * M * M;
  const int s = blockIdx.x / nf;
  const int f = blockIdx.x - s * nf;
  const long base = s * sg_stride + f * M3;
  for (int e = threadIdx.x; e < N * N * N; e += blockDim.x) {
    const int i = e % N, j = (e / N) % N, k = e / (N * N);
    const long c = base + ((long)(k + 3) * M + (j + 3)) * M + (i + 3);
    out[c] = __dadd_rn(__dmul_rn(a, x[c]), __dmul_rn(b, y[c]));
  }
}

}  // namespace hydro

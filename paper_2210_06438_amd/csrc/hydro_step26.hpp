// hydro_step26.hpp -- the 26-point form of the 8^3 sub-grid step (paper
// Section IV-B: values of the evolved variables at the 26 points of each
// cell's surface -- face centres, edge midpoints, vertices -- from the
// piecewise-parabolic method, central-upwind fluxes at those points, and
// Newton-Cotes quadrature of the fluxes over each face).
//
// The value of cell c toward a surface point c + e/2, e in {-1,0,1}^3 \ 0,
// is the right edge of c's limited parabola on the line of cells c + k e,
// k = -2..2 (monotonised-central slopes, Colella-Woodward interface value
// and monotonicity constraint, in the offset form of hydro_kernel.hpp).  A
// face normal to axis d between cells c and c + n has 9 points (transverse
// offsets s1, s2 in {-1,0,1}); W- is c's value toward n + s1 t1 + s2 t2, W+
// is (c + n)'s value toward -n + s1 t1 + s2 t2.  The face flux is Simpson's
// rule in both transverse directions, (16 F_centre + 4 sum F_edge + sum
// F_vertex) / 36, summed in the fixed order s2 (outer), s1 (inner).
//
// One work-group of 512 lanes per sub-grid (one lane per interior cell; 256
// registers per lane, no spills).  The lanes compute the 3 x 576 faces (9
// points each, lines read from u_in through the caches, primitives recovered
// per cell read) into an LDS face buffer; after a barrier each lane updates
// its cell from its six faces (x, then y, then z differences, as the oracle
// sums them) and writes U - lambda * sum.
// Deterministic: no atomics, fixed summation orders.  The edge and corner
// ghosts of u_in are read.
#pragma once

#include "hydro_lds8.hpp"

namespace hydro {

struct S26 {
  static constexpr int N = 8, M = 14, kThreads = 512, kFaces = 9 * 64;   // faces per direction
  static constexpr long FS = (long)M * M * M;
};

// Right edge (toward +e) of the limited parabola of the middle of five
// values along a line (offset form: half slopes h, right offset dR = qR - q,
// left offset dL = q - qL).
__device__ __forceinline__ double ppm_right5(double qm2, double qm1, double q0, double qp1,
                                             double qp2) {
  const double dm1 = qm1 - qm2, d0 = q0 - qm1, d1 = qp1 - q0, d2 = qp2 - qp1;
  const double hm1 = half_slope(dm1, d0);
  const double h0 = half_slope(d0, d1);
  const double h1 = half_slope(d1, d2);
  const double dR = 0.5 * d1 - (h1 - h0) * (1.0 / 3.0);
  const double dL = d0 - (0.5 * d0 - (h0 - hm1) * (1.0 / 3.0));
  double oL, oR;
  limit_edges(dL, dR, oL, oR);
  return q0 + oR;
}

// Offsets (stored, one field) of the five cells c + k e, k = -2..2.
__device__ __forceinline__ void line5(int x, int y, int z, int e0, int e1, int e2, int (&off)[5]) {
  constexpr int M = S26::M;
#pragma unroll
  for (int k = 0; k < 5; ++k)
    off[k] = ((z + (k - 2) * e2) * M + (y + (k - 2) * e1)) * M + (x + (k - 2) * e0);
}

// Hydro-core primitive state (rho, vx, vy, vz, p) of the cell at off[2]
// toward the direction of its line.
__device__ __forceinline__ void point_core(gcptr u, const int (&off)[5], double (&W)[5]) {
  constexpr long FS = S26::FS;
  double q[5][5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double U[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) U[f] = u[f * FS + off[k]];
    to_prim(U, q[k]);
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) W[f] = ppm_right5(q[0][f], q[1][f], q[2][f], q[3][f], q[4][f]);
}

// Passive field f (stored as is) of the cell at off[2] toward its line.
__device__ __forceinline__ double point_passive(gcptr u, const int (&off)[5], int f) {
  const gcptr p = u + f * S26::FS;
  return ppm_right5(p[off[0]], p[off[1]], p[off[2]], p[off[3]], p[off[4]]);
}



// Face `face` of direction DIR (normal position i, transverse a, b): its
// Simpson-integrated flux into fh[face * F ..]; returns the largest signal
// speed of its 9 points.
template <int DIR, int F>
__device__ __forceinline__ double face26(gcptr u, int face, double* __restrict__ fh) {
  constexpr int T1 = DIR == 0 ? 1 : 0, T2 = DIR == 2 ? 1 : 2;
  constexpr double ex = DIR == 0 ? 1.0 : 0.0, ey = DIR == 1 ? 1.0 : 0.0, ez = DIR == 2 ? 1.0 : 0.0;
  const int i = face >> 6, a = face & 7, b = (face >> 3) & 7;
  int lo[3];
  lo[DIR] = i + 2;
  lo[T1] = a + kGhost;
  lo[T2] = b + kGhost;
  double sum[F];
#pragma unroll
  for (int f = 0; f < F; ++f) sum[f] = 0.0;
  double smax = 0.0;
  // the 9 points one after another (unrolled, their loads would all be
  // hoisted and spill)
#pragma unroll 1
  for (int s2 = -1; s2 <= 1; ++s2) {
#pragma unroll 1
    for (int s1 = -1; s1 <= 1; ++s1) {
      int em[3], ep[3];
      em[DIR] = 1;
      ep[DIR] = -1;
      em[T1] = ep[T1] = s1;
      em[T2] = ep[T2] = s2;
      int om[5], op[5];
      line5(lo[0], lo[1], lo[2], em[0], em[1], em[2], om);
      line5(lo[0] + (DIR == 0), lo[1] + (DIR == 1), lo[2] + (DIR == 2), ep[0], ep[1], ep[2], op);
      double Wm[5], Wp[5], Fh[5], wm, wp;
      point_core(u, om, Wm);
      __builtin_amdgcn_sched_barrier(0);
      point_core(u, op, Wp);
      smax = fmax(smax, core_flux(Wm, Wp, ex, ey, ez, Fh, wm, wp));
      const double w = (s1 == 0 && s2 == 0) ? 16.0 : (s1 == 0 || s2 == 0) ? 4.0 : 1.0;
#pragma unroll
      for (int f = 0; f < 5; ++f) sum[f] = sum[f] + w * Fh[f];
      // passive fields one at a time: flux w- q- + w+ q+ with the core's weights
#pragma unroll
      for (int f = 5; f < F; ++f) {
        __builtin_amdgcn_sched_barrier(0);
        sum[f] = sum[f] + w * (wm * point_passive(u, om, f) + wp * point_passive(u, op, f));
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int f = 0; f < F; ++f) fh[face * F + f] = sum[f] * (1.0 / 36.0);
  return smax;
}

// Face index within its direction of the face above (upper) and below
// (lower) interior cell (cx, cy, cz) along DIR.
template <int DIR>
__device__ __forceinline__ int face_below(int cx, int cy, int cz) {
  const int p = DIR == 0 ? cx : DIR == 1 ? cy : cz;
  const int a = DIR == 0 ? cy : cx;
  const int b = DIR == 2 ? cy : cz;
  return (p * 8 + b) * 8 + a;
}

// The fluxes of all 3 x 576 faces go to LDS (152 KB at 11 fields): lane t
// computes faces t, t + 512, ... (at most 4), then lane t (one per interior
// cell) updates its cell from its six faces, x then y then z.
template <int F>
__global__ void __launch_bounds__(S26::kThreads)
    hydro_step26_kernel(const DevDesc* __restrict__ table, int count, double dt, double dx,
                        double* __restrict__ amax_out) {
  constexpr int NF = 3 * S26::kFaces;
  __shared__ double fh[NF * F];
  __shared__ double red[S26::kThreads / 64];
  constexpr int M = S26::M;
  const int s = blockIdx.x;
  if (s >= count) return;
  const DevDesc d = table[s];
  const gcptr u = as_global(d.u_in);
  const int t = threadIdx.x;
  const double lambda = dt / ldexp(dx, -d.level);

  double smax = 0.0;
  for (int g = t; g < NF; g += S26::kThreads) {
    const int dir = g / S26::kFaces, face = g - dir * S26::kFaces;
    double* const out = fh + dir * S26::kFaces * F;
    if (dir == 0)
      smax = fmax(smax, face26<0, F>(u, face, out));
    else if (dir == 1)
      smax = fmax(smax, face26<1, F>(u, face, out));
    else
      smax = fmax(smax, face26<2, F>(u, face, out));
  }
  __syncthreads();

  // U_out = U - lambda * ((dF_x + dF_y) + dF_z), lane t = interior cell t
  {
    const int cx = t & 7, cy = (t >> 3) & 7, cz = t >> 6;
    const int fx = face_below<0>(cx, cy, cz);
    const int fy = S26::kFaces + face_below<1>(cx, cy, cz);
    const int fz = 2 * S26::kFaces + face_below<2>(cx, cy, cz);
    const bool compact = d.compact != 0;
    const int gin = ((cz + kGhost) * M + (cy + kGhost)) * M + (cx + kGhost);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      double sum = fh[(fx + 64) * F + f] - fh[fx * F + f];
      sum = sum + (fh[(fy + 64) * F + f] - fh[fy * F + f]);
      sum = sum + (fh[(fz + 64) * F + f] - fh[fz * F + f]);
      const double v = u[f * S26::FS + gin] - lambda * sum;
      const long o = compact ? (long)f * 512 + t : f * S26::FS + gin;
      __builtin_nontemporal_store(v, &as_global(d.u_out)[o]);
    }
  }
  if (amax_out) {
    smax = wave_max(smax);
    if ((t & 63) == 0) red[t >> 6] = smax;
    __syncthreads();
    if (t == 0) {
      double m = red[0];
      for (int k = 1; k < S26::kThreads / 64; ++k) m = fmax(m, red[k]);
      amax_out[d.index] = m;
    }
  }
}

}  // namespace hydro

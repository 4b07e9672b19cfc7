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
// One work-group of 576 lanes per sub-grid.  The hydro-core primitives of
// the whole stored block (14^3 cells x 5) are recovered once into LDS.  The
// faces are then taken one direction at a time, one lane per face (576 per
// direction): the lane forms the 9 point states of the hydro core from LDS,
// their central-upwind fluxes and the Simpson sum, keeping the 9 points'
// passive-flux weights in registers; then it takes the passive fields one
// after another, reading each field's 5-cell lines through the caches (the
// work-group's reads at any time cover one field: ~22 KB per sub-grid, which
// the caches hold).  The direction's face fluxes go to an LDS buffer; after a
// barrier, lane t < 512 adds its cell's difference to its running sum (x,
// then y, then z, as the oracle sums them).  Finally U_out = U - lambda sum.
// Deterministic: no atomics, fixed summation orders.  The edge and corner
// ghosts of u_in are read.
#pragma once

#include "hydro_lds8.hpp"

namespace hydro {

struct S26 {
  static constexpr int N = 8, M = 14, kThreads = 576, kFaces = 9 * 64;   // faces per direction
  static constexpr long FS = (long)M * M * M;
  static constexpr int MMM = M * M * M;
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

// Hydro-core state (rho, vx, vy, vz, p) of the cell at off[2] toward the
// direction of its line, from the primitives staged in LDS.
__device__ __forceinline__ void point_core(const double* __restrict__ prim, const int (&off)[5],
                                           double (&W)[5]) {
  constexpr int MMM = S26::MMM;
#pragma unroll
  for (int f = 0; f < 5; ++f)
    W[f] = ppm_right5(prim[f * MMM + off[0]], prim[f * MMM + off[1]], prim[f * MMM + off[2]],
                      prim[f * MMM + off[3]], prim[f * MMM + off[4]]);
}

// Passive field p (stored as is, the pointer at its first cell) of the cell
// at off[2] toward its line.
__device__ __forceinline__ double point_passive(gcptr p, const int (&off)[5]) {
  return ppm_right5(p[off[0]], p[off[1]], p[off[2]], p[off[3]], p[off[4]]);
}

// Line offsets of point (s1, s2) of face `face` of direction DIR: om for
// the cell below the face toward the point, op for the cell above.
template <int DIR>
__device__ __forceinline__ void face_lines(int face, int s1, int s2, int (&om)[5], int (&op)[5]) {
  constexpr int T1 = DIR == 0 ? 1 : 0, T2 = DIR == 2 ? 1 : 2;
  const int i = face >> 6, a = face & 7, b = (face >> 3) & 7;
  int lo[3], em[3], ep[3];
  lo[DIR] = i + 2;
  lo[T1] = a + kGhost;
  lo[T2] = b + kGhost;
  em[DIR] = 1;
  ep[DIR] = -1;
  em[T1] = ep[T1] = s1;
  em[T2] = ep[T2] = s2;
  line5(lo[0], lo[1], lo[2], em[0], em[1], em[2], om);
  line5(lo[0] + (DIR == 0), lo[1] + (DIR == 1), lo[2] + (DIR == 2), ep[0], ep[1], ep[2], op);
}

// The central-upwind flux of core_flux for a face normal to axis DIR known
// at compile time: the normal velocity is that component itself and the
// pressure enters that momentum flux alone, so the products with the zero
// components of the unit normal are not formed (the values are the same up
// to the sign of a zero).
template <int DIR>
__device__ __forceinline__ double core_flux_axis(const double (&Wm)[5], const double (&Wp)[5],
                                                 double (&Fh)[5], double& wm, double& wp) {
  const double vnm = Wm[1 + DIR], vnp = Wp[1 + DIR];
  const double gm = kGamma * Wm[4], gpp = kGamma * Wp[4];
  const double cm = gm * rsq_pos(gm * Wm[0]);
  const double cp = gpp * rsq_pos(gpp * Wp[0]);
  const double ap = fmax(fmax(vnm + cm, vnp + cp), 0.0);
  const double am = fmin(fmin(vnm - cm, vnp - cp), 0.0);
  const double inv = recip(ap - am);
  wm = ap * (vnm - am) * inv;
  wp = am * (ap - vnp) * inv;
  const double Em = Wm[4] * kInvGm1 +
                    0.5 * Wm[0] * (Wm[1] * Wm[1] + Wm[2] * Wm[2] + Wm[3] * Wm[3]);
  const double Ep = Wp[4] * kInvGm1 +
                    0.5 * Wp[0] * (Wp[1] * Wp[1] + Wp[2] * Wp[2] + Wp[3] * Wp[3]);
  const double pt = (ap * Wm[4] - am * Wp[4]) * inv;
  Fh[0] = wm * Wm[0] + wp * Wp[0];
#pragma unroll
  for (int k = 1; k <= 3; ++k) {
    if (k == 1 + DIR)
      Fh[k] = wm * (Wm[0] * Wm[k]) + wp * (Wp[0] * Wp[k]) + pt;
    else
      Fh[k] = wm * (Wm[0] * Wm[k]) + wp * (Wp[0] * Wp[k]);
  }
  Fh[4] = wm * Em + wp * Ep + (ap * (Wm[4] * vnm) - am * (Wp[4] * vnp)) * inv;
  return fmax(ap, -am);
}

// Face `face` of direction DIR (normal position i, transverse a, b): its
// Simpson-integrated flux into fh[face * F ..]; returns the largest signal
// speed of its 9 points.  Points in the order s2 (outer), s1 (inner), weights
// 16 (centre), 4 (edge midpoints), 1 (vertices), over 36.
template <int DIR, int F>
__device__ __forceinline__ double face26(const double* __restrict__ prim, gcptr u, int face,
                                         double* __restrict__ fh) {
  double sum[5], wm[9], wp[9];
#pragma unroll
  for (int f = 0; f < 5; ++f) sum[f] = 0.0;
  double smax = 0.0;
  // hydro core: the 9 points one after another (a scheduling barrier after
  // each keeps the next point's LDS reads from being hoisted)
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const int s1 = p % 3 - 1, s2 = p / 3 - 1;
    int fc = face;   // opaque copy, as in the passive loop below
    asm volatile("" : "+v"(fc));
    int om[5], op[5];
    face_lines<DIR>(fc, s1, s2, om, op);
    double Wm[5], Wp[5], Fh[5];
    point_core(prim, om, Wm);
    __builtin_amdgcn_sched_barrier(0);
    point_core(prim, op, Wp);
    smax = fmax(smax, core_flux_axis<DIR>(Wm, Wp, Fh, wm[p], wp[p]));
    const double w = (s1 == 0 && s2 == 0) ? 16.0 : (s1 == 0 || s2 == 0) ? 4.0 : 1.0;
#pragma unroll
    for (int f = 0; f < 5; ++f) sum[f] = sum[f] + w * Fh[f];
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) fh[face * F + f] = sum[f] * (1.0 / 36.0);
  // passive fields one at a time: flux w- q- + w+ q+ with each point's weights
#pragma unroll 1
  for (int f = 5; f < F; ++f) {
    const gcptr pf = u + f * S26::FS;
    double acc = 0.0;
    if constexpr (F > 6) {
      // the 10 line values of point p + 1 are loaded while point p is
      // computed (compiled for a single passive field this form spilled
      // over 700 bytes per lane, so the plain loop below serves that case)
      double cur[10], nxt[10];
      auto load = [&](int p, double (&v)[10]) {
        int fc = face;   // opaque copy: offsets recomputed, not kept live
        asm volatile("" : "+v"(fc));
        int om[5], op[5];
        face_lines<DIR>(fc, p % 3 - 1, p / 3 - 1, om, op);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          v[k] = pf[om[k]];
          v[5 + k] = pf[op[k]];
        }
      };
      load(0, cur);
#pragma unroll
      for (int p = 0; p < 9; ++p) {
        const int s1 = p % 3 - 1, s2 = p / 3 - 1;
        if (p < 8) load(p + 1, nxt);
        const double w = (s1 == 0 && s2 == 0) ? 16.0 : (s1 == 0 || s2 == 0) ? 4.0 : 1.0;
        const double qm = ppm_right5(cur[0], cur[1], cur[2], cur[3], cur[4]);
        const double qp = ppm_right5(cur[5], cur[6], cur[7], cur[8], cur[9]);
        acc = acc + w * (wm[p] * qm + wp[p] * qp);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 10; ++k) cur[k] = nxt[k];
      }
    } else {
#pragma unroll
      for (int p = 0; p < 9; ++p) {
        const int s1 = p % 3 - 1, s2 = p / 3 - 1;
        // an opaque copy of the face index: the line offsets are recomputed
        // at every point (a few integer ops) instead of being kept live from
        // the hydro points through every field, which would spill them
        int fc = face;
        asm volatile("" : "+v"(fc));
        int om[5], op[5];
        face_lines<DIR>(fc, s1, s2, om, op);
        const double w = (s1 == 0 && s2 == 0) ? 16.0 : (s1 == 0 || s2 == 0) ? 4.0 : 1.0;
        acc = acc + w * (wm[p] * point_passive(pf, om) + wp[p] * point_passive(pf, op));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    fh[face * F + f] = acc * (1.0 / 36.0);
  }
  return smax;
}

// Face index within its direction of the face below interior cell
// (cx, cy, cz) along DIR (the face above is 64 further).
template <int DIR>
__device__ __forceinline__ int face_below(int cx, int cy, int cz) {
  const int p = DIR == 0 ? cx : DIR == 1 ? cy : cz;
  const int a = DIR == 0 ? cy : cx;
  const int b = DIR == 2 ? cy : cz;
  return (p * 8 + b) * 8 + a;
}

// One direction: every lane its face, then lane t < 512 (interior cell t)
// adds the difference of its two faces to its running sum.
template <int DIR, int F>
__device__ __forceinline__ double step26_dir(const double* __restrict__ prim, gcptr u,
                                             double* __restrict__ fh, int t, double (&sum)[F]) {
  const double smax = face26<DIR, F>(prim, u, t, fh);
  __syncthreads();   // the direction's face fluxes complete
  if (t < 512) {
    const int fl = face_below<DIR>(t & 7, (t >> 3) & 7, t >> 6);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const double dF = fh[(fl + 64) * F + f] - fh[fl * F + f];
      sum[f] = DIR == 0 ? dF : sum[f] + dF;
    }
  }
  __syncthreads();   // read before the next direction writes
  return smax;
}

template <int F>
__global__ void __launch_bounds__(S26::kThreads)
    hydro_step26_kernel(const DevDesc* __restrict__ table, int count, double dt, double dx,
                        double* __restrict__ amax_out) {
  constexpr int MMM = S26::MMM;
  __shared__ double prim[5 * MMM];
  __shared__ double fh[S26::kFaces * F];
  __shared__ double red[S26::kThreads / 64];
  constexpr int M = S26::M;
  const int s = blockIdx.x;
  if (s >= count) return;
  const DevDesc d = table[s];
  const gcptr u = as_global(d.u_in);
  const int t = threadIdx.x;
  const double lambda = dt / ldexp(dx, -d.level);

  // hydro-core primitives of every stored cell
  for (int c = t; c < MMM; c += S26::kThreads) {
    double U[5], q[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) U[f] = u[f * S26::FS + c];
    to_prim(U, q);
#pragma unroll
    for (int f = 0; f < 5; ++f) prim[f * MMM + c] = q[f];
  }
  __syncthreads();

  double sum[F];
  double smax = step26_dir<0, F>(prim, u, fh, t, sum);
  smax = fmax(smax, step26_dir<1, F>(prim, u, fh, t, sum));
  smax = fmax(smax, step26_dir<2, F>(prim, u, fh, t, sum));

  // U_out = U - lambda * ((dF_x + dF_y) + dF_z), lane t = interior cell t
  if (t < 512) {
    const int cx = t & 7, cy = (t >> 3) & 7, cz = t >> 6;
    const bool compact = d.compact != 0;
    const int gin = ((cz + kGhost) * M + (cy + kGhost)) * M + (cx + kGhost);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const double v = u[f * S26::FS + gin] - lambda * sum[f];
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

// hydro_kernel.hpp -- gfx950 device code of the aggregated sub-grid hydro step.
//
// One forward-Euler stage of the ideal-gas Euler equations on N^3 sub-grids
// with 3 ghost layers (paper Section IV-B; sub-grid shape Section V-A).
// Every sub-grid of a batch is handled by one work-group of ONE launch (the
// paper's explicit aggregation, Section V-D): the work-group reads its
// descriptor by block index, like the paper's per-task index into the
// aggregated buffers.
//
// Per work-group: three direction passes (x, y, z).  In pass d each lane owns
// one line of n+6 cells along d whose two transverse coordinates are interior
// and marches along it once, keeping a sliding window of the reconstruction
// in registers for all F components:
//   primitives -> limited slopes -> interface offsets -> parabola limiter ->
//   face states -> central-upwind flux -> flux difference of each interior
//   cell.
// The reconstruction is carried in offset form (edge value minus cell value);
// the monotonised-central slope and the Colella-Woodward constraint are
// evaluated through their min/max equivalents, which give the same edge values
// as the case-by-case definitions (they agree exactly at every case boundary).
// The flux is regrouped as w- U(W-) + w+ U(W+) + pressure terms, with
// w- = a+ (v- - a-)/(a+ - a-), w+ = a- (a+ - v+)/(a+ - a-), which is the
// central-upwind flux of Kurganov, Noelle and Petrova expanded.
//
// Pass results are summed in the interior of u_out (x, then y, then z, then
// scaled by dt/dx_s), the order of the flux-divergence sum.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hydro {

constexpr double kGamma = 5.0 / 3.0;
constexpr double kGm1 = kGamma - 1.0;
constexpr double kInvGm1 = 1.0 / kGm1;
constexpr int kGhost = 3;

// 1/x from the hardware estimate refined by two Newton-Raphson steps
// (r <- r + r(1 - x r)); within an ulp or so of the rounded quotient for the
// positive, normal arguments it is used on (densities, wave-speed spans).
// Scaling x by a power of two scales the result exactly.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(y) for positive normal y: hardware 1/sqrt estimate, then the coupled
// Newton iteration for (sqrt(y), 1/(2 sqrt(y))) and a final residual
// correction.
__device__ __forceinline__ double sqrt_pos(double y) {
  const double s = __builtin_amdgcn_rsq(y);
  double g = y * s;
  double h = 0.5 * s;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, y);
  return fma(d, h, g);
}

// Device-side descriptor: one per sub-grid in an aggregated launch.
struct DevDesc {
  const double* u_in;
  double* u_out;
  int32_t level;
  int32_t index;  // position in the caller's batch (amax slot)
};

// Descriptors carried by value in the kernel arguments (small batches and
// the one-launch-per-sub-grid baseline).
constexpr int kArgDescs = 8;
struct ArgDescs {
  DevDesc d[kArgDescs];
};

template <int N>
struct Shape {
  static constexpr int M = N + 2 * kGhost;
  static constexpr int kLines = N * N;
  static constexpr int kThreads = ((kLines + 63) / 64) * 64;
  static constexpr long kFieldStride = (long)M * M * M;
};

// ---- limited slope (half of the monotonised-central slope) -------------
// dl = q_i - q_{i-1}, dr = q_{i+1} - q_i.  Returns
// sgn * min(|dl + dr|/4, |dl|, |dr|) when dl and dr share a sign, else 0.
__device__ __forceinline__ double half_slope(double dl, double dr) {
  const double sg = copysign(1.0, dl);
  const double t = 0.25 * (dl + dr) * sg;
  const double m = fmin(fmin(t, fabs(dl)), dr * sg);
  return sg * fmax(m, 0.0);
}

// ---- parabola constraint on (dL, dR) = (q - qL, qR - q) ------------------
__device__ __forceinline__ void limit_edges(double dL, double dR, double& oL,
                                            double& oR) {
  const double sg = copysign(1.0, dL);
  const double a = fabs(dL);
  const double b = dR * sg;
  oL = sg * fmax(fmin(a, b + b), 0.0);
  oR = sg * fmax(fmin(b, a + a), 0.0);
}

// ---- central-upwind flux between primitive face states ------------------
// Component 1 is the velocity normal to the face, 2 and 3 the transverse
// ones (the caller rotates field offsets so this holds for every pass).
template <int F>
__device__ __forceinline__ double face_flux(const double (&Wm)[F],
                                            const double (&Wp)[F],
                                            double (&Fh)[F]) {
  const double rm = 1.0 / Wm[0];
  const double rp = 1.0 / Wp[0];
  const double cm = sqrt(kGamma * Wm[4] * rm);
  const double cp = sqrt(kGamma * Wp[4] * rp);
  const double ap = fmax(fmax(Wm[1] + cm, Wp[1] + cp), 0.0);
  const double am = fmin(fmin(Wm[1] - cm, Wp[1] - cp), 0.0);
  const double inv = 1.0 / (ap - am);
  const double wm = ap * (Wm[1] - am) * inv;
  const double wp = am * (ap - Wp[1]) * inv;
  const double Em = Wm[4] / kGm1 +
                    0.5 * Wm[0] * (Wm[1] * Wm[1] + Wm[2] * Wm[2] + Wm[3] * Wm[3]);
  const double Ep = Wp[4] / kGm1 +
                    0.5 * Wp[0] * (Wp[1] * Wp[1] + Wp[2] * Wp[2] + Wp[3] * Wp[3]);
  Fh[0] = wm * Wm[0] + wp * Wp[0];
  Fh[1] = wm * (Wm[0] * Wm[1]) + wp * (Wp[0] * Wp[1]) + (ap * Wm[4] - am * Wp[4]) * inv;
  Fh[2] = wm * (Wm[0] * Wm[2]) + wp * (Wp[0] * Wp[2]);
  Fh[3] = wm * (Wm[0] * Wm[3]) + wp * (Wp[0] * Wp[3]);
  Fh[4] = wm * Em + wp * Ep + (ap * (Wm[4] * Wm[1]) - am * (Wp[4] * Wp[1])) * inv;
#pragma unroll
  for (int k = 5; k < F; ++k) Fh[k] = wm * Wm[k] + wp * Wp[k];
  return fmax(ap, -am);
}

// Sliding-window state of one line march.
template <int F>
struct March {
  double q1[F];   // q_{i-1}
  double q2[F];   // q_{i-2}
  double d1[F];   // q_{i-1} - q_{i-2}
  double h2[F];   // half slope at i-2
  double dLp[F];  // q - qL offset of cell i-2 (before limiting)
  double qRp[F];  // limited right edge of cell i-3
  double Fp[F];   // flux through the face (i-4)+1/2
};

// Load the F stored values of position `pos` and convert to primitives.
// fofs[f] is the field offset (in units of the field stride) that plays the
// role of component f in this pass.
template <int F>
__device__ __forceinline__ void load_primitive(const double* __restrict__ base,
                                               long pos, const int (&fofs)[F],
                                               long fstride, double (&q)[F]) {
  double U[F];
#pragma unroll
  for (int f = 0; f < F; ++f) U[f] = base[fofs[f] * fstride + pos];
  const double r = 1.0 / U[0];
  const double v1 = U[1] * r, v2 = U[2] * r, v3 = U[3] * r;
  q[0] = U[0];
  q[1] = v1;
  q[2] = v2;
  q[3] = v3;
  q[4] = kGm1 * (U[4] - 0.5 * (U[1] * v1 + U[2] * v2 + U[3] * v3));
#pragma unroll
  for (int f = 5; f < F; ++f) q[f] = U[f];
}

// One march step at position i.  STAGE is min(i, 6): stages 0..5 warm the
// window up, stage 6 is the steady state that finishes one interior cell.
// Returns true (and fills dF) when a cell's flux difference is complete.
template <int F, int STAGE>
__device__ __forceinline__ void march_step(March<F>& st, const double (&q)[F],
                                           double& smax, double (&dF)[F]) {
  double Wm[F], Wp[F];
#pragma unroll
  for (int k = 0; k < F; ++k) {
    if constexpr (STAGE == 0) {
      st.q1[k] = q[k];
      continue;
    }
    const double dn = q[k] - st.q1[k];
    if constexpr (STAGE == 1) {
      st.d1[k] = dn;
      st.q2[k] = st.q1[k];
      st.q1[k] = q[k];
      continue;
    }
    const double h = half_slope(st.d1[k], dn);
    if constexpr (STAGE == 2) {
      st.h2[k] = h;
      st.d1[k] = dn;
      st.q2[k] = st.q1[k];
      st.q1[k] = q[k];
      continue;
    }
    // right-edge offset of cell i-2: half the difference minus the slope
    // correction (h_{i-1} - h_{i-2}) / 3.
    const double e = 0.5 * st.d1[k] - (h - st.h2[k]) * (1.0 / 3.0);
    if constexpr (STAGE >= 4) {
      double oL, oR;
      limit_edges(st.dLp[k], e, oL, oR);
      const double qL = st.q2[k] - oL;
      const double qR = st.q2[k] + oR;
      if constexpr (STAGE >= 5) {
        Wm[k] = st.qRp[k];
        Wp[k] = qL;
      }
      st.qRp[k] = qR;
    }
    st.dLp[k] = st.d1[k] - e;
    st.h2[k] = h;
    st.d1[k] = dn;
    st.q2[k] = st.q1[k];
    st.q1[k] = q[k];
  }
  if constexpr (STAGE >= 5) {
    double Fh[F];
    const double s = face_flux<F>(Wm, Wp, Fh);
    smax = fmax(smax, s);
#pragma unroll
    for (int k = 0; k < F; ++k) {
      if constexpr (STAGE == 6) dF[k] = Fh[k] - st.Fp[k];
      st.Fp[k] = Fh[k];
    }
  }
}

// Pass modes for the interior accumulation in u_out.
enum PassMode { kStore = 0, kAdd = 1, kFinal = 2 };

// March one line: `in`/`out` point at position 0 of the line in field 0;
// consecutive positions are `ls` elements apart.
template <int N, int F>
__device__ __forceinline__ void march_line(const double* __restrict__ in,
                                           double* __restrict__ out, long ls,
                                           const int (&fofs)[F], int mode,
                                           double lambda, double& smax) {
  constexpr int M = Shape<N>::M;
  constexpr long FS = Shape<N>::kFieldStride;
  March<F> st;
  double q[F], dF[F];
  load_primitive<F>(in, 0 * ls, fofs, FS, q);
  march_step<F, 0>(st, q, smax, dF);
  load_primitive<F>(in, 1 * ls, fofs, FS, q);
  march_step<F, 1>(st, q, smax, dF);
  load_primitive<F>(in, 2 * ls, fofs, FS, q);
  march_step<F, 2>(st, q, smax, dF);
  load_primitive<F>(in, 3 * ls, fofs, FS, q);
  march_step<F, 3>(st, q, smax, dF);
  load_primitive<F>(in, 4 * ls, fofs, FS, q);
  march_step<F, 4>(st, q, smax, dF);
  load_primitive<F>(in, 5 * ls, fofs, FS, q);
  march_step<F, 5>(st, q, smax, dF);
#pragma unroll 2
  for (int i = 6; i < M; ++i) {
    load_primitive<F>(in, i * ls, fofs, FS, q);
    march_step<F, 6>(st, q, smax, dF);
    const long c = (long)(i - 3) * ls;  // the interior cell just finished
#pragma unroll
    for (int k = 0; k < F; ++k) {
      double* o = out + fofs[k] * FS + c;
      if (mode == kStore) {
        *o = dF[k];
      } else if (mode == kAdd) {
        *o = *o + dF[k];
      } else {
        const double u = in[fofs[k] * FS + c];
        *o = u - lambda * (*o + dF[k]);
      }
    }
  }
}

// Wave-level max of non-negative doubles.
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Whole step of one sub-grid by one work-group of Shape<N>::kThreads lanes.
template <int N, int F>
__device__ __forceinline__ void subgrid_step(const DevDesc& d, double dt,
                                             double dx, double* amax_out) {
  constexpr int M = Shape<N>::M;
  constexpr int W = Shape<N>::kThreads / 64;
  __shared__ double red[W];
  const double lambda = dt / ldexp(dx, -d.level);
  const int t = threadIdx.x;
  const int a = t % N, b = t / N;
  double smax = 0.0;
#pragma unroll 1
  for (int dir = 0; dir < 3; ++dir) {
    if (t < N * N) {
      int fofs[F];
      fofs[0] = 0;
      fofs[1] = 1 + dir;
      fofs[2] = 1 + (dir + 1) % 3;
      fofs[3] = 1 + (dir + 2) % 3;
#pragma unroll
      for (int f = 4; f < F; ++f) fofs[f] = f;
      long start, ls;
      if (dir == 0) {          // line along x at (y, z) = (a, b) + ghosts
        start = ((long)(b + kGhost) * M + (a + kGhost)) * M;
        ls = 1;
      } else if (dir == 1) {   // along y at (x, z)
        start = ((long)(b + kGhost) * M) * M + (a + kGhost);
        ls = M;
      } else {                 // along z at (x, y)
        start = ((long)(b + kGhost) * M) + (a + kGhost);
        ls = (long)M * M;
      }
      march_line<N, F>(d.u_in + start, d.u_out + start, ls, fofs,
                       dir == 0 ? kStore : (dir == 1 ? kAdd : kFinal), lambda,
                       smax);
    }
    __syncthreads();
  }
  if (amax_out) {
    smax = wave_max(smax);
    if ((t & 63) == 0) red[t >> 6] = smax;
    __syncthreads();
    if (t == 0) {
      double m = red[0];
#pragma unroll
      for (int w = 1; w < W; ++w) m = fmax(m, red[w]);
      amax_out[d.index] = m;
    }
  }
}

template <int N, int F>
__global__ void __launch_bounds__(Shape<N>::kThreads)
    hydro_table_kernel(const DevDesc* __restrict__ table, double dt, double dx,
                       double* __restrict__ amax_out) {
  const DevDesc d = table[blockIdx.x];
  subgrid_step<N, F>(d, dt, dx, amax_out);
}

template <int N, int F>
__global__ void __launch_bounds__(Shape<N>::kThreads)
    hydro_arg_kernel(ArgDescs descs, double dt, double dx,
                     double* __restrict__ amax_out) {
  const DevDesc d = descs.d[blockIdx.x];
  subgrid_step<N, F>(d, dt, dx, amax_out);
}

}  // namespace hydro

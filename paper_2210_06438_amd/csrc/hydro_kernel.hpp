// hydro_kernel.hpp -- device helpers shared by the gfx950 kernels of the
// sub-grid hydro step (paper Section IV-B): constants, reciprocal and square
// root, the limited PPM slope and parabola constraint in offset form, the
// descriptor types, and a wave-level max.
//
// The reconstruction is carried in offset form (edge value minus cell value).
// The monotonised-central slope and the Colella-Woodward parabola constraint
// are evaluated through min/max equivalents that give the same edge values as
// the case-by-case definitions (the cases agree exactly at their boundaries).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hydro {

constexpr double kGamma = 5.0 / 3.0;
constexpr double kGm1 = kGamma - 1.0;
constexpr double kInvGm1 = 1.0 / kGm1;
constexpr int kGhost = 3;

// 1/x from the hardware estimate refined by two steps of the Newton-Raphson
// iteration for the reciprocal, r <- r + r(1 - x r), each written with
// fused multiply-adds (the form of P. Markstein, "Computation of elementary
// functions on the IBM RISC System/6000 processor", IBM J. Res. Dev. 34(1),
// 1990).  Each step squares the relative error of the estimate, so the
// result is within one ulp of the correctly rounded quotient for positive
// normal arguments (densities, wave-speed spans); the GPU tests bound it
// against IEEE division over 1e-17..1e3.  Scaling x by a power of two scales
// the result exactly.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(y) for positive normal y: the hardware estimate refined by two
// Newton-Raphson steps for the reciprocal square root, r <- r + (r/2)(1 - y r^2),
// with the residual 1 - (y r) r taken by a fused multiply-add (the form of
// Markstein 1990, above).  Each step squares the relative error of the
// estimate; the GPU tests bound the result against the correctly rounded
// 1/sqrt(y) over 1e-17..1e3.  Scaling y by 4^k scales the result by 2^-k
// exactly (the estimate and every step commute with it).
__device__ __forceinline__ double rsq_pos(double y) {
  double r = __builtin_amdgcn_rsq(y);
  double t = y * r;
  double e = fma(-t, r, 1.0);
  r = fma(0.5 * r, e, r);
  t = y * r;
  e = fma(-t, r, 1.0);
  return fma(0.5 * r, e, r);
}

// Device-side descriptor: one per sub-grid in an aggregated launch.
struct DevDesc {
  const double* u_in;
  double* u_out;
  int16_t level;
  int16_t compact;  // 1: u_out holds the interior only, [F][n][n][n]
  int32_t index;    // position in the caller's batch (amax slot)
};

// Descriptors carried by value in the kernel arguments (small batches and
// the one-launch-per-sub-grid baseline).
constexpr int kArgDescs = 8;

// Per-work-group amax partials (the aggregator's launches): work-group b of
// the sub-grid with descriptor index i stores its maximum, with a plain
// store, at amax_out[i * kAmaxParts + b]; the reader takes the maximum of
// the first (work-groups per sub-grid) entries.  16 = the most work-groups
// of one sub-grid (16^3 with 4^3 blocks).
constexpr int kAmaxParts = 16;
struct ArgDescs {
  DevDesc d[kArgDescs];
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

// Wave-level max of non-negative doubles.
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace hydro

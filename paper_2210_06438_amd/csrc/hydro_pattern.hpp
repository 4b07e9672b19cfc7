// hydro_pattern.hpp -- the HBM access pattern of the 8^3 step without its
// arithmetic: a roofline reference for hydro_lds8_kernel.
//
// One work-group of 192 lanes per 8^3 sub-grid, the same lane roles and the
// same loads in the same order as the step (hydro core: interior shares to
// LDS and the six ghost cells of each lane's line to registers; then the
// passive fields in two bursts), the same LDS footprint (so the same number
// of work-groups per CU), and the interior written once in the descriptor's
// output layout with non-temporal stores, by the z lanes.  Each output value
// is the input interior value plus 1e-300 times the sum of the ghost cells
// the lane loaded, so no load can be dropped by the compiler; the values
// have no physical meaning.  The time of this kernel is what the step's data
// movement costs on its own at the step's occupancy.
#pragma once

#include "hydro_lds8.hpp"

namespace hydro {

template <int F0, int NG, int MP>
__device__ __forceinline__ void pattern_group(const double* __restrict__ uin, double* __restrict__ uout,
                                              long ofs, int obase, int ostride, int t, int dir,
                                              int gbase, int gstride, int lbase, int lstride) {
  constexpr long FS = Frame<MP>::FS;
  double* const tin = lds_tin;
  Share<NG> sh;
  load_share<NG, MP>(uin + F0 * FS, t, sh);
  double g[NG][6];
  load_ghosts<NG, MP>(uin + F0 * FS, gbase, gstride, g);
  store_share<NG>(tin, t, sh);
  __syncthreads();
  double gs = 0.0;
#pragma unroll
  for (int k = 0; k < NG; ++k)
#pragma unroll
    for (int j = 0; j < 6; ++j) gs += g[k][j];
  if (dir == 2) {
#pragma unroll
    for (int k = 0; k < NG; ++k)
#pragma unroll
      for (int c = 0; c < Lds8::N; ++c)
        __builtin_nontemporal_store(tin[k * Lds8::P + lbase + c * lstride] + 1e-300 * gs,
                                    &as_global(uout)[(F0 + k) * ofs + obase + c * ostride]);
  } else if (gs != gs) {
    lds_red[dir] = gs;   // never for finite inputs; keeps the x and y lanes' loads
  }
  __syncthreads();
}

template <int F, bool SAME_LDS>
__global__ void __launch_bounds__(Lds8::kThreads, 2)
    hydro_pattern_kernel(const DevDesc* __restrict__ table, int count) {
  constexpr int MP = 14;
  constexpr int NP = F - 5;
  constexpr int NA = (NP + 1) / 2;
  constexpr int NB = NP - NA;
  const int s = blockIdx.x;
  if (s >= count) return;
  const DevDesc d = table[s];
  const int t = threadIdx.x;
  const int dir = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l = t & 63;
  const int a = l & 7, b = l >> 3;
  const int lbase = dir == 0 ? lcell(0, a, b) : dir == 1 ? lcell(a, 0, b) : lcell(a, b, 0);
  const int lstride = dir == 0 ? 1 : dir == 1 ? Lds8::RS : Lds8::PS;
  const int gbase = Frame<MP>::line(dir, a, b, 0);
  const int gstride = Frame<MP>::stride(dir);
  const bool compact = d.compact != 0;
  const long ofs = compact ? 512 : Frame<MP>::FS;
  const int ostride = compact ? 64 : MP * MP;
  const int obase = compact ? b * 8 + a : Frame<MP>::line(2, a, b, kGhost);
  if constexpr (SAME_LDS) {
    // reserve the step's accumulator arrays too (never read)
    if (t == 0) {
      lds_acc[0] = 0.0;
      lds_held[0] = 0.0;
    }
  }
  pattern_group<0, 5, MP>(d.u_in, d.u_out, ofs, obase, ostride, t, dir, gbase, gstride, lbase,
                          lstride);
  pattern_group<5, NA, MP>(d.u_in, d.u_out, ofs, obase, ostride, t, dir, gbase, gstride, lbase,
                           lstride);
  if constexpr (NB > 0)
    pattern_group<5 + NA, NB, MP>(d.u_in, d.u_out, ofs, obase, ostride, t, dir, gbase, gstride,
                                  lbase, lstride);
}

}  // namespace hydro

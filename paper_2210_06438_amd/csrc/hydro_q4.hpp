// hydro_q4.hpp -- sub-grids stepped as disjoint 4^3 blocks, four blocks per
// work-group (the "4^3 tile"; hydro_lds8.hpp is the 8^3 tile).
//
// Every edge n in {8, 12, 16} is a multiple of 4, so the blocks tile the
// interior exactly: nothing is computed twice (8^3 blocks of a 12^3 sub-grid
// overlap and recompute 2.37x the cells).  The step of one block is the step
// of hydro_lds8.hpp on a 4^3 interior with its 3-deep halo (a 10^3 frame
// inside the parent's stored (n+6)^3 array): the same reconstruction, flux and
// update code, marched along lines of 10 stored cells, computing every face
// from the same cells -- results agree with the 8^3 tile to rounding.  A work-group of 192 lanes steps 4 blocks of one sub-grid: wave 0
// marches the x lines of all four (4 x 16 lanes), wave 1 the y lines, wave 2
// the z lines.  A sub-grid's (n/4)^3 blocks (8, 27 or 64; padded to a multiple
// of 4 with idle slots) are 2, 7 or 16 work-groups whose indices are equal
// modulo 8, so they run on one XCD and share its L2 for their common halos.
//
// Direction sums as in hydro_lds8.hpp: for the hydro core exactly two LDS
// atomic adds onto zero per cell (x and y lanes), the z lanes keep
// U - lambda dF_z; the passive fields in groups of three with plain stores
// and a finalization shared by the work-group.  Every block
// owns all of its cells; amax is combined across blocks with an atomic max of
// the bit pattern onto a slot zeroed before the launch.
#pragma once

#include "hydro_lds8.hpp"

namespace hydro {

struct Q4 {
  static constexpr int N = 4;
  static constexpr int M = 10;            // stored cells along a line
  static constexpr int RS = 5;            // LDS row stride (4 cells + 1 pad)
  static constexpr int PS = 21;           // LDS plane stride
  static constexpr int QS = 4 * PS + 1;   // LDS block stride
  static constexpr int P = 4 * QS;        // one field of a cell array: 4 blocks
  static constexpr int kThreads = 192;
};

// Geometry of the 4^3 tiling of a parent with stored edge MP.
template <int MP>
struct Q4Grid {
  static constexpr int NI = MP - 2 * kGhost;       // parent interior edge
  static constexpr int BA = NI / 4;                // blocks per axis
  static constexpr int kBlocks = BA * BA * BA;
  static constexpr int kGroups = (kBlocks + 3) / 4;  // work-groups per sub-grid
  static_assert(NI % 4 == 0, "edge must be a multiple of 4");
};

__device__ __forceinline__ int q4cell(int q, int x, int y, int z) {
  return q * Q4::QS + z * Q4::PS + y * Q4::RS + x;
}

// Stored offset (in the parent) of the frame of block `item`; idle slots
// past the last block repeat it (their results are not stored).
template <int MP>
__device__ __forceinline__ int q4_org(int item, int& bx, int& by, int& bz) {
  constexpr int BA = Q4Grid<MP>::BA;
  item = item < Q4Grid<MP>::kBlocks ? item : Q4Grid<MP>::kBlocks - 1;
  bx = item % BA;
  by = (item / BA) % BA;
  bz = item / (BA * BA);
  return ((4 * bz) * MP + 4 * by) * MP + 4 * bx;
}

// Interior shares of NF consecutive fields of the four blocks: element j of
// a lane is e = t + j*192 of the fields stacked [f][q][z][y][x].
template <int NF>
struct Share4 {
  static constexpr int K = (NF * 256 + Q4::kThreads - 1) / Q4::kThreads;
  double v[K];
};

template <int NF, int MP>
__device__ __forceinline__ void q4_load_share(const double* __restrict__ src, int group, int t,
                                              Share4<NF>& sh) {
  constexpr int K = Share4<NF>::K;
  constexpr int REM = NF * 256 - (K - 1) * Q4::kThreads;
  asm volatile("" : "+v"(t));   // recompute indices here (see load_share)
  const gcptr g = as_global(src);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int e = t + j * Q4::kThreads;
    if (j + 1 < K || REM == Q4::kThreads || e < NF * 256) {
      const int f = e >> 8, q = (e >> 6) & 3, x = e & 3, y = (e >> 2) & 3, z = (e >> 4) & 3;
      int bx, by, bz;
      const int org = q4_org<MP>(4 * group + q, bx, by, bz);
      sh.v[j] = g[f * Frame<MP>::FS + org + Frame<MP>::cell(x, y, z)];
    }
  }
}

template <int NF>
__device__ __forceinline__ void q4_store_share(double* lds, int t, const Share4<NF>& sh) {
  constexpr int K = Share4<NF>::K;
  constexpr int REM = NF * 256 - (K - 1) * Q4::kThreads;
  asm volatile("" : "+v"(t));
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int e = t + j * Q4::kThreads;
    if (j + 1 < K || REM == Q4::kThreads || e < NF * 256) {
      const int f = e >> 8, q = (e >> 6) & 3, x = e & 3, y = (e >> 2) & 3, z = (e >> 4) & 3;
      lds[f * Q4::P + q4cell(q, x, y, z)] = sh.v[j];
    }
  }
}

// The six ghost positions (0, 1, 2, 7, 8, 9) of this lane's line.
template <int NF, int MP>
__device__ __forceinline__ void q4_load_ghosts(const double* __restrict__ src, int gbase,
                                               int gstride, double (&g)[NF][6]) {
  const gcptr p = as_global(src) + gbase;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int i = j < 3 ? j : j + Q4::N;
      g[f][j] = p[f * Frame<MP>::FS + i * gstride];
    }
  }
}

// Finalize `count` (<= 3) passive fields of the four blocks, from field
// `kfirst` on, shared by all lanes (lane t takes elements t, t + 192, ...
// of the fields stacked [r][q][z][y][x]): U_out = Z - lambda * (X + Y), Z
// the z lanes' U - lambda dF_z (zr region r), X and Y the x and y flux
// differences (acc and held region r).  Idle block slots store nothing.
template <int MP>
__device__ __forceinline__ void q4_finalize(const double* __restrict__ zr,
                                            const double* __restrict__ acc,
                                            const double* __restrict__ held, int kfirst,
                                            int count, double lambda, double* __restrict__ uout,
                                            bool compact, long ofs, int group, int t) {
  constexpr int NI = Q4Grid<MP>::NI;
  constexpr int P = Q4::P;
#pragma unroll
  for (int j = 0; j < 4; ++j) {   // 3 fields x 256 cells / 192 lanes
    const int e = t + j * Q4::kThreads;
    const int r = e >> 8, q = (e >> 6) & 3, x = e & 3, y = (e >> 2) & 3, z = (e >> 4) & 3;
    const int item = 4 * group + q;
    if (r < count && item < Q4Grid<MP>::kBlocks) {
      const int lc = r * P + q4cell(q, x, y, z);
      const double v = zr[lc] - lambda * (acc[lc] + held[lc]);
      int bx, by, bz;
      const int org = q4_org<MP>(item, bx, by, bz);
      const long o = compact ? ((long)(4 * bz + z) * NI + 4 * by + y) * NI + 4 * bx + x
                             : (long)org + Frame<MP>::cell(x, y, z);
      __builtin_nontemporal_store(v, &as_global(uout)[(kfirst + r) * ofs + o]);
    }
  }
}

// PARTS: the work-group stores its maximum at partial `group` of the
// sub-grid's slot (kAmaxParts per sub-grid) instead of the atomic max.
template <int F, int MP, bool PARTS = false>
__device__ __forceinline__ void q4_step(const DevDesc& d, int group, double dt, double dx,
                                        double* __restrict__ amax_out) {
  constexpr int M = Q4::M;
  constexpr int N = Q4::N;
  constexpr int NI = Q4Grid<MP>::NI;
  constexpr long FS = Frame<MP>::FS;
  constexpr int P = Q4::P;
  constexpr int NP = F - 5;
  constexpr int NT = NP > 5 ? NP : 5;
  // the file-scope LDS arrays of hydro_lds8.hpp (same roles)
  static_assert(NT * P <= 6 * Lds8::P && 5 * P <= 5 * Lds8::P, "q4 arrays exceed the LDS arrays");
  double* const tin = lds_tin;
  double* const acc = lds_acc;
  double* const held = lds_held;
  double* const red = lds_red;

  const int t = threadIdx.x;
  const int dir = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l = t & 63;
  const int q = l >> 4;                  // block slot of this lane
  const int a = l & 3, b = (l >> 2) & 3; // transverse coordinates of its line
  const int item = 4 * group + q;
  const bool stores = item < Q4Grid<MP>::kBlocks;
  int bx, by, bz;
  const int org = q4_org<MP>(item, bx, by, bz);
  const double ex = dir == 0 ? 1.0 : 0.0;
  const double ey = dir == 1 ? 1.0 : 0.0;
  const double ez = dir == 2 ? 1.0 : 0.0;
  const int lbase = dir == 0 ? q4cell(q, 0, a, b) : dir == 1 ? q4cell(q, a, 0, b) : q4cell(q, a, b, 0);
  const int lstride = dir == 0 ? 1 : dir == 1 ? Q4::RS : Q4::PS;
  const int gbase = org + Frame<MP>::line(dir, a, b, 0);
  const int gstride = Frame<MP>::stride(dir);
  const double lambda = dt / ldexp(dx, -d.level);
  const double* __restrict__ uin = d.u_in;
  // z lanes write column (a, b) of their block, all four cells
  const bool compact = d.compact != 0;
  double* __restrict__ uout = d.u_out;
  const long ofs = compact ? (long)NI * NI * NI : FS;
  const int ostride = compact ? NI * NI : MP * MP;
  const int obase = compact ? ((4 * bz) * NI + 4 * by + b) * NI + 4 * bx + a
                            : org + Frame<MP>::line(2, a, b, kGhost);

  // ---- stage the hydro core ---------------------------------------------
  // loads issued at a raised wave priority, as in the 8^3 tile
  __builtin_amdgcn_s_setprio(2);
  {
    Share4<5> sh;
    q4_load_share<5, MP>(uin, group, t, sh);
    for (int i = t; i < 5 * P; i += Q4::kThreads) acc[i] = 0.0;
    q4_store_share<5>(tin, t, sh);
  }
  double g[5][6];
  q4_load_ghosts<5, MP>(uin, gbase, gstride, g);
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();

  double smax = 0.0;
  double wm[N + 1], wp[N + 1];
  {
    Recon<5> rc;
    double Fprev[5];
    double qv[5], Wm[5], Wp[5];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      double Ui[5];
#pragma unroll
      for (int k = 0; k < 5; ++k)
        Ui[k] = (i >= kGhost && i < kGhost + N) ? tin[k * P + lbase + (i - kGhost) * lstride]
                                                : g[k][i < kGhost ? i : i - N];
      to_prim(Ui, qv);
      switch (i) {
        case 0: rc.step<0>(qv, Wm, Wp); break;
        case 1: rc.step<1>(qv, Wm, Wp); break;
        case 2: rc.step<2>(qv, Wm, Wp); break;
        case 3: rc.step<3>(qv, Wm, Wp); break;
        case 4: rc.step<4>(qv, Wm, Wp); break;
        case 5: rc.step<5>(qv, Wm, Wp); break;
        default: rc.step<6>(qv, Wm, Wp); break;
      }
      if (i >= 5) {
        double Fh[5];
        const int face = i - 5;
        smax = fmax(smax, core_flux(Wm, Wp, ex, ey, ez, Fh, wm[face], wp[face]));
        if (i >= 6) {
          const int cell = lbase + (i - 6) * lstride;
          if (dir == 2) {
#pragma unroll
            for (int k = 0; k < 5; ++k)
              held[k * P + cell] = tin[k * P + cell] - lambda * (Fh[k] - Fprev[k]);
          } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) atomicAdd(&acc[k * P + cell], Fh[k] - Fprev[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) Fprev[k] = Fh[k];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // The largest signal speed is reduced across the wave now and parked in
  // LDS: reduced at the end, the compiler keeps both speeds of every face
  // live through the whole passive phase.  The barriers of that phase order
  // these stores before the final read.
  smax = wave_max(smax);
  if (l == 0) red[dir] = smax;

  // ---- all passive fields in one burst ----------------------------------
  Share4<NP> ps;
  double pg[NP][6];
  q4_load_share<NP, MP>(uin + 5 * FS, group, t, ps);
  q4_load_ghosts<NP, MP>(uin + 5 * FS, gbase, gstride, pg);
  __syncthreads();   // hydro sums complete; tin free
  if (dir == 2) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const int cell = k * P + lbase + c * lstride;
        if (stores)
          __builtin_nontemporal_store(held[cell] - lambda * acc[cell],
                                      &as_global(uout)[k * ofs + obase + c * ostride]);
      }
    }
  }
  q4_store_share<NP>(tin, t, ps);
  __syncthreads();   // tin holds every passive field; the hydro sums are read

  // ---- passive fields from LDS, in groups of at most 3 -------------------
  // As in hydro_lds8.hpp: within a group every lane marches its line for
  // each field in turn, with no barrier between fields, no atomics and no
  // branch on the direction: it stores fma(pa, dF, pz u) -- the x lanes dF
  // to acc region r, the y lanes dF to held region r, the z lanes
  // u - lambda dF to tin region NP + r.  One barrier then lets every lane
  // finalize a share of the group's cells of the four blocks.
  constexpr int G = NP < 3 ? NP : 3;
  static_assert((NP + G) * P <= 6 * Lds8::P && G * P <= 5 * Lds8::P,
                "q4 passive regions exceed the LDS arrays");
  const double pa = dir == 2 ? -lambda : 1.0;
  const double pz = dir == 2 ? 1.0 : 0.0;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int r = p % G;
    double* const dst = dir == 0 ? acc + r * P : dir == 1 ? held + r * P : tin + (NP + r) * P;
    Recon<1> rc;
    double Fprev = 0.0;
    double qv[1], Wm[1], Wp[1];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      qv[0] = (i >= kGhost && i < kGhost + N) ? tin[p * P + lbase + (i - kGhost) * lstride]
                                              : pg[p][i < kGhost ? i : i - N];
      switch (i) {
        case 0: rc.step<0>(qv, Wm, Wp); break;
        case 1: rc.step<1>(qv, Wm, Wp); break;
        case 2: rc.step<2>(qv, Wm, Wp); break;
        case 3: rc.step<3>(qv, Wm, Wp); break;
        case 4: rc.step<4>(qv, Wm, Wp); break;
        case 5: rc.step<5>(qv, Wm, Wp); break;
        default: rc.step<6>(qv, Wm, Wp); break;
      }
      if (i >= 5) {
        const double Fh = wm[i - 5] * Wm[0] + wp[i - 5] * Wp[0];
        if (i >= 6) {
          const int cell = lbase + (i - 6) * lstride;
          dst[cell] = fma(pa, Fh - Fprev, pz * tin[p * P + cell]);
        }
        Fprev = Fh;
      }
    }
    if (r == G - 1 || p == NP - 1) {
      __syncthreads();   // the group's differences are in LDS
      q4_finalize<MP>(tin + NP * P, acc, held, 5 + p - r, r + 1, lambda, uout, compact, ofs,
                      group, t);
      if (p < NP - 1) __syncthreads();   // read before the next group writes
    }
  }

  if (amax_out) {
    if (t == 0) {
      const double m = fmax(fmax(red[0], red[1]), red[2]);
      if constexpr (PARTS)
        amax_out[(long)d.index * kAmaxParts + group] = m;
      else
        atomicMax(reinterpret_cast<unsigned long long*>(&amax_out[d.index]),
                  (unsigned long long)__double_as_longlong(m));
    }
  }
}

// Table form: the B work-groups of sub-grid s have indices equal modulo 8.
// The grid is ceil(count/8)*8*B.
template <int F, int MP>
__global__ void __launch_bounds__(Q4::kThreads, 2)
    hydro_q4_kernel(const DevDesc* __restrict__ table, int count, double dt, double dx,
                    double* __restrict__ amax_out) {
  constexpr int B = Q4Grid<MP>::kGroups;
  const int w = blockIdx.x;
  const int s = (w / (8 * B)) * 8 + (w & 7);
  const int group = (w >> 3) % B;
  if (s >= count) return;
  const DevDesc d = table[s];
  q4_step<F, MP>(d, group, dt, dx, amax_out);
}

template <int F, int MP>
__global__ void __launch_bounds__(Q4::kThreads, 2)
    hydro_q4_arg_kernel(ArgDescs descs, double dt, double dx, double* __restrict__ amax_out) {
  constexpr int B = Q4Grid<MP>::kGroups;
  const DevDesc d = descs.d[blockIdx.x / B];
  q4_step<F, MP>(d, blockIdx.x % B, dt, dx, amax_out);
}

// Launch geometry shared by every table launch.  Work-groups per sub-grid
// of parent edge MP with tile 4 or 8; a table launch over `count` sub-grids
// of B work-groups each rounds the count up to whole multiples of 8 so the
// work-groups of one sub-grid get indices equal modulo 8 (one XCD).
template <int MP>
inline int groups_per_subgrid(int tile) {
  return tile == 4 ? Q4Grid<MP>::kGroups : Blocks<MP>::kPerSubgrid;
}

inline int grid_for(int count, int B) { return B == 1 ? count : ((count + 7) / 8) * 8 * B; }

}  // namespace hydro

// hydro_lds8.hpp -- the gfx950 kernel of the aggregated sub-grid hydro step:
// every needed input byte read from HBM once, direction sums kept on chip.
//
// Unit of work: an 8^3 block.  An 8^3 sub-grid is one block; a 16^3
// sub-grid is 8 blocks, at block origins {0, 8} per axis inside the parent's
// stored array, so a block's ghost cells are simply the parent's neighbouring
// cells and every block computes exactly what the whole sub-grid would.  (The
// geometry also covers n = 12 with origins {0, 4}, where the blocks overlap
// and the second block of an axis writes only its last 4 cells; 12^3
// sub-grids are stepped as 27 disjoint 4^3 blocks by hydro_q4.hpp instead.)
// One launch (per shape class) steps every block of every sub-grid of a batch
// (the paper's explicit aggregation, Section V-D).
//
// One work-group of 192 lanes steps one block: wave 0 owns the 64 lines
// along x, wave 1 the lines along y, wave 2 the lines along z (one lane per
// line of 14 cells whose transverse coordinates are interior).  The interior
// cells (needed by all three directions) are loaded cooperatively with
// coalesced loads into LDS; the six ghost cells of a line (needed by that
// line only) are loaded by its lane straight into registers.  Edge/corner
// ghosts are never read.  Results are written with non-temporal stores: an
// interior row covers only part of its cache lines, and streaming the partial
// lines out avoids filling them from HBM first.
//
// Hydro core (rho, s, E): the lane marches its line (primitive recovery ->
// limited slopes -> interface offsets -> parabola constraint -> central-upwind
// flux, paper Section IV-B with the Kurganov-Noelle-Petrova flux) and keeps,
// for every face, the weights w- = a+(v- - a-)/(a+ - a-) and
// w+ = a-(a+ - v+)/(a+ - a-) of the expanded flux, with which the flux of any
// passively advected density q is w- q(W-) + w+ q(W+).  The passive fields
// (tau, species) are then loaded in two bursts and marched from LDS.
//
// Direction sums: lanes of the x and y waves add their flux differences into
// a zeroed LDS accumulator with atomic adds -- exactly two adds onto zero per
// cell, which is order-independent, so the result is deterministic.  Lanes of
// the z wave store U - lambda*dF_z to LDS; after a barrier every lane of the
// work-group finishes a share of the cells,
// U_out = (U - lambda*dF_z) - lambda*(dF_x + dF_y), so no wave carries the
// finalization alone, and consecutive lanes store consecutive cells.
#pragma once

#include "hydro_kernel.hpp"

namespace hydro {

struct Lds8 {
  static constexpr int N = 8;
  static constexpr int M = 14;
  // LDS cell arrays: row stride 9 and plane stride 72 (= 8 mod 16) make the
  // 64-bit accesses of the x and y lanes bank-conflict free and leave one
  // 2-way conflict per 16 z lanes.
  static constexpr int RS = 9;
  static constexpr int PS = 72;
  static constexpr int P = N * PS; // one field of a cell array: 576 doubles
  static constexpr int kThreads = 192;
  static constexpr long FS = (long)M * M * M;
};

// The LDS arrays of a work-group, at file scope so that every step function
// (both tiles, every edge and field count) uses the same four objects: a
// kernel that holds several of them -- one path per shape class -- allocates
// them once.  Sized for the largest user (the 8^3 tile with 11 fields).
// tin: interiors of the staged fields.  acc: x+y flux differences (two
// atomic adds onto zero per cell).  held: the z lanes' U - lambda*dF_z.
__shared__ double lds_tin[6 * Lds8::P];
__shared__ double lds_acc[5 * Lds8::P];
__shared__ double lds_held[5 * Lds8::P];
__shared__ double lds_red[3];

// LDS index of interior cell (x, y, z), 0 <= x, y, z < 8.
__device__ __forceinline__ int lcell(int x, int y, int z) {
  return z * Lds8::PS + y * Lds8::RS + x;
}

// Sliding-window PPM reconstruction of K components along a line, in offset
// form (see hydro_kernel.hpp).  step<STAGE>() consumes q_i; from stage 5 on it
// returns the face states W-, W+ of the face (i-3)+1/2.
template <int K>
struct Recon {
  double q1[K], q2[K], h2[K], dLp[K], qRp[K];

  template <int STAGE>
  __device__ __forceinline__ void step(const double (&q)[K], double (&Wm)[K],
                                       double (&Wp)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if constexpr (STAGE == 0) {
        q1[k] = q[k];
        continue;
      }
      if constexpr (STAGE == 1) {
        q2[k] = q1[k];
        q1[k] = q[k];
        continue;
      }
      const double d1 = q1[k] - q2[k];  // q_{i-1} - q_{i-2}
      const double dn = q[k] - q1[k];   // q_i - q_{i-1}
      const double h = half_slope(d1, dn);
      if constexpr (STAGE == 2) {
        h2[k] = h;
        q2[k] = q1[k];
        q1[k] = q[k];
        continue;
      }
      const double e = 0.5 * d1 - (h - h2[k]) * (1.0 / 3.0);
      if constexpr (STAGE >= 4) {
        double oL, oR;
        limit_edges(dLp[k], e, oL, oR);
        if constexpr (STAGE >= 5) {
          Wm[k] = qRp[k];
          Wp[k] = q2[k] - oL;
        }
        qRp[k] = q2[k] + oR;
      }
      dLp[k] = d1 - e;
      h2[k] = h;
      q2[k] = q1[k];
      q1[k] = q[k];
    }
  }
};

// Central-upwind flux of the hydro core (fields in x, y, z order) through a
// face normal to the axis selected by the 0/1 masks (ex, ey, ez).  W = (rho,
// vx, vy, vz, p).  Returns max(a+, -a-); writes F[5] and the weights.
__device__ __forceinline__ double core_flux(const double (&Wm)[5],
                                            const double (&Wp)[5], double ex,
                                            double ey, double ez,
                                            double (&Fh)[5], double& wm,
                                            double& wp) {
  const double vnm = ex * Wm[1] + ey * Wm[2] + ez * Wm[3];
  const double vnp = ex * Wp[1] + ey * Wp[2] + ez * Wp[3];
  // sound speeds c = sqrt(gamma p / rho) = (gamma p) / sqrt(gamma p rho)
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
  Fh[1] = wm * (Wm[0] * Wm[1]) + wp * (Wp[0] * Wp[1]) + ex * pt;
  Fh[2] = wm * (Wm[0] * Wm[2]) + wp * (Wp[0] * Wp[2]) + ey * pt;
  Fh[3] = wm * (Wm[0] * Wm[3]) + wp * (Wp[0] * Wp[3]) + ez * pt;
  Fh[4] = wm * Em + wp * Ep + (ap * (Wm[4] * vnm) - am * (Wp[4] * vnp)) * inv;
  return fmax(ap, -am);
}

__device__ __forceinline__ void to_prim(const double (&U)[5], double (&q)[5]) {
  const double r = recip(U[0]);
  const double vx = U[1] * r, vy = U[2] * r, vz = U[3] * r;
  q[0] = U[0];
  q[1] = vx;
  q[2] = vy;
  q[3] = vz;
  q[4] = kGm1 * (U[4] - 0.5 * (U[1] * vx + U[2] * vy + U[3] * vz));
}

// Global-memory views of the caller's buffers (lets the compiler use
// global_* instead of flat_* instructions).
typedef const __attribute__((address_space(1))) double* gcptr;
typedef __attribute__((address_space(1))) double* gptr;
__device__ __forceinline__ gcptr as_global(const double* p) { return (gcptr)p; }
__device__ __forceinline__ gptr as_global(double* p) { return (gptr)p; }

// An 8^3 block inside a parent sub-grid stored with edge MP (14 for n = 8,
// 18 for n = 12, 22 for n = 16).  Block-frame stored coordinates 0..13 map to
// parent stored coordinates by adding the block origin; all offsets below
// are relative to the block frame's origin.
template <int MP>
struct Frame {
  static constexpr long FS = (long)MP * MP * MP;  // one field of the parent
  // stored offset of block-frame line position i for lane (a, b) of `dir`
  __device__ static __forceinline__ int line(int dir, int a, int b, int i) {
    if (dir == 0) return ((b + kGhost) * MP + (a + kGhost)) * MP + i;
    if (dir == 1) return ((b + kGhost) * MP + i) * MP + (a + kGhost);
    return (i * MP + (b + kGhost)) * MP + (a + kGhost);
  }
  __device__ static __forceinline__ int stride(int dir) {
    return dir == 0 ? 1 : dir == 1 ? MP : MP * MP;
  }
  // stored offset of interior cell (x, y, z) of the block
  __device__ static __forceinline__ int cell(int x, int y, int z) {
    return ((z + kGhost) * MP + (y + kGhost)) * MP + (x + kGhost);
  }
};

// This lane's share of the block interior of `NF` consecutive fields
// starting at `src` (block-frame origin): element j is interior cell
// t + j*192 of the fields stacked [f][z][y][x].  (Elements j < K-1 always
// exist because t < 192.)
template <int NF>
struct Share {
  static constexpr int K = (NF * 512 + Lds8::kThreads - 1) / Lds8::kThreads;
  double v[K];
};

template <int NF, int MP>
__device__ __forceinline__ void load_share(const double* __restrict__ src, int t,
                                           Share<NF>& sh) {
  // An opaque copy of the lane index: the cell indices below are then
  // recomputed at every call (a few integer ops) instead of being kept live
  // from the hydro staging to the passive staging, where they would be
  // spilled and their reloads would wait behind every outstanding load and
  // store of the wave (the vector memory counter retires in order).
  asm volatile("" : "+v"(t));
  const gcptr g = as_global(src);
#pragma unroll
  for (int j = 0; j < Share<NF>::K; ++j) {
    const int e = t + j * Lds8::kThreads;
    if (j + 1 < Share<NF>::K || e < NF * 512) {
      const int f = e >> 9, x = e & 7, y = (e >> 3) & 7, z = (e >> 6) & 7;
      sh.v[j] = g[f * Frame<MP>::FS + Frame<MP>::cell(x, y, z)];
    }
  }
}

template <int NF>
__device__ __forceinline__ void store_share(double* lds, int t, const Share<NF>& sh) {
  asm volatile("" : "+v"(t));   // see load_share
#pragma unroll
  for (int j = 0; j < Share<NF>::K; ++j) {
    const int e = t + j * Lds8::kThreads;
    if (j + 1 < Share<NF>::K || e < NF * 512) {
      const int f = e >> 9, x = e & 7, y = (e >> 3) & 7, z = (e >> 6) & 7;
      lds[f * Lds8::P + lcell(x, y, z)] = sh.v[j];
    }
  }
}

// The six ghost positions (0, 1, 2, 11, 12, 13) of this lane's line for NF
// consecutive fields; position i is stored at gbase + i * gstride.
template <int NF, int MP>
__device__ __forceinline__ void load_ghosts(const double* __restrict__ src, int gbase,
                                            int gstride, double (&g)[NF][6]) {
  const gcptr p = as_global(src) + gbase;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int i = j < 3 ? j : j + 8;
      g[f][j] = p[f * Frame<MP>::FS + i * gstride];
    }
  }
}

template <int STAGE, int K>
__device__ __forceinline__ void recon_step(Recon<K>& rc, const double (&q)[K],
                                           double (&Wm)[K], double (&Wp)[K]) {
  rc.template step<STAGE>(q, Wm, Wp);
}

template <int I, int K>
__device__ __forceinline__ void recon_at(Recon<K>& rc, const double (&q)[K],
                                         double (&Wm)[K], double (&Wp)[K]) {
  recon_step<(I < 6 ? I : 6), K>(rc, q, Wm, Wp);
}

// Optional blend of the step's result with another state, for the stages
// of a multi-stage time-step: the stored value becomes a x + b U_out, each
// product and the sum rounded once (no contraction), where x is the element
// `delta` doubles from the output element (another brick buffer of the same
// layout, or the output itself when delta = 0: each element is read and
// written by the same lane).
struct BlendArgs {
  double a, b;
  long delta;
};

// Optional face-ghost writes of the stages of a time-step on a brick of
// sub-grids (the ghost exchange of Section V-A done by the producer): every
// stored interior value within kGhost cells of a face is also a face-ghost
// value of the sub-grid across that face, and is written there too (periodic
// axes wrap around the brick).  Under outflow at the domain's edge the cell
// next to the edge fills this sub-grid's own kGhost layers there (the ghost
// takes the nearest domain cell).  Sub-grid s of the brick sits at
// (s % nb[0], s / nb[0] % nb[1], s / (nb[0] nb[1])), its stored block at
// base + s sg_stride.  Edge and corner ghosts are not written: the
// face-centre step reads none.  Within one launch every destination is a
// ghost cell of the output buffer, which the launch does not read.
struct FacePush {
  double* base;
  long sg_stride;
  int nb[3];
  int bc[3];   // 0 periodic, 1 outflow
};

template <int MP>
__device__ __forceinline__ void push_faces(const FacePush& fp, int sg, int f, int x, int y,
                                           int z, double v) {
  constexpr int N = MP - 2 * kGhost;
  const int c[3] = {x, y, z};
  const int bs[3] = {sg % fp.nb[0], (sg / fp.nb[0]) % fp.nb[1], sg / (fp.nb[0] * fp.nb[1])};
  const long sgs[3] = {1, fp.nb[0], (long)fp.nb[0] * fp.nb[1]};   // sub-grids per step
  const long st[3] = {1, MP, (long)MP * MP};                      // stored cells per step
  double* const own = fp.base + sg * fp.sg_stride + f * Frame<MP>::FS + Frame<MP>::cell(x, y, z);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool lo = bs[a] == 0, hi = bs[a] == fp.nb[a] - 1, outflow = fp.bc[a] != 0;
    if (c[a] < kGhost) {
      if (!(outflow && lo)) {
        // the lower neighbour's ghost at stored coordinate c + N + kGhost
        const long nsg = lo ? (fp.nb[a] - 1) * sgs[a] : -sgs[a];
        as_global(own)[nsg * fp.sg_stride + N * st[a]] = v;
      } else if (c[a] == 0) {
#pragma unroll
        for (int k = 1; k <= kGhost; ++k) as_global(own)[-k * st[a]] = v;
      }
    }
    if (c[a] >= N - kGhost) {
      if (!(outflow && hi)) {
        // the upper neighbour's ghost at stored coordinate c - N + kGhost
        const long nsg = hi ? -(fp.nb[a] - 1) * sgs[a] : sgs[a];
        as_global(own)[nsg * fp.sg_stride - N * st[a]] = v;
      } else if (c[a] == N - 1) {
#pragma unroll
        for (int k = 1; k <= kGhost; ++k) as_global(own)[k * st[a]] = v;
      }
    }
  }
}

// Finalize NFLD fields of a block from LDS, shared by all lanes of the
// work-group (lane t takes the cells t, t + 192, ...): for every interior cell
// the block owns, U_out = Z - lambda * (X + Y), where Z holds the z lanes'
// U - lambda dF_z and X, Y the x and y flux differences.  Field kfirst + r
// takes Z from zreg(r) and X + Y from its sum: the hydro core's atomically
// accumulated acc region r (SPLIT false; X + Y = 0 + dF_x + dF_y), or the
// passive fields' separate x (acc region r) and y (held region r)
// differences (SPLIT true; the same value, dF_x + dF_y).  With interior-only
// outputs of an 8^3 sub-grid the lanes of a wave store 512 contiguous bytes.
template <int NFLD, int MP, bool SPLIT, bool BLEND = false, bool PUSH = false>
__device__ __forceinline__ void finalize_shared(const double* __restrict__ held,
                                                const double* __restrict__ acc, int kfirst,
                                                double lambda, double* __restrict__ uout,
                                                bool compact, long ofs, int ox, int oy, int oz,
                                                int lox, int loy, int loz, int t,
                                                const BlendArgs& bl = BlendArgs{},
                                                const FacePush& fp = FacePush{}, int sg = 0) {
  constexpr int NI = MP - 2 * kGhost;
  constexpr int CELLS = NFLD * 512;
  constexpr int J = (CELLS + Lds8::kThreads - 1) / Lds8::kThreads;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int e = t + j * Lds8::kThreads;
    if (j + 1 < J || e < CELLS) {
      const int r = e >> 9, x = e & 7, y = (e >> 3) & 7, z = (e >> 6) & 7;
      const int lc = lcell(x, y, z);
      double v;
      if constexpr (SPLIT) {
        const double* zb = r < 2 ? acc + (3 + r) * Lds8::P : held + 3 * Lds8::P;
        v = zb[lc] - lambda * (acc[r * Lds8::P + lc] + held[r * Lds8::P + lc]);
      } else {
        v = held[r * Lds8::P + lc] - lambda * acc[r * Lds8::P + lc];
      }
      if (x >= lox && y >= loy && z >= loz) {
        const long o = compact ? (kfirst + r) * ofs + ((long)(oz + z) * NI + oy + y) * NI + ox + x
                               : (kfirst + r) * Frame<MP>::FS + Frame<MP>::cell(x, y, z);
        if constexpr (BLEND)
          v = __dadd_rn(__dmul_rn(bl.a, as_global(uout)[o + bl.delta]), __dmul_rn(bl.b, v));
        __builtin_nontemporal_store(v, &as_global(uout)[o]);
        if constexpr (PUSH) push_faces<MP>(fp, sg, kfirst + r, x, y, z, v);
      }
    }
  }
}

// One sub-grid per work-group.  Loads are issued in two bursts: the hydro
// core (interior shares to LDS, ghosts to registers) at the start, and all
// passive fields together right after the hydro march, so the passive phase
// runs on data that is already on chip.
// One 8^3 block of a sub-grid: `org` is the stored offset of the block
// frame in the parent, (lox, loy, loz) the first block-local coordinate the
// block owns (cells below it belong to another block of the parent and are
// computed but not written).  MULTI: several blocks share the parent's amax
// slot (combined with an atomic max of the bit pattern, which orders like the
// values for non-negative doubles; the slot is zeroed before the launch).
// PARTS: the block stores its own maximum instead, at partial `part` of the
// parent's slot (kAmaxParts per sub-grid), with a plain store.
template <int F, int MP, bool MULTI, bool PARTS = false, bool BLEND = false, bool PUSH = false>
__device__ __forceinline__ void lds8_step(const DevDesc& d, int org, int ox, int oy, int oz,
                                          int lox, int loy, int loz, double dt, double dx,
                                          double* __restrict__ amax_out, int part = 0,
                                          const BlendArgs& bl = BlendArgs{},
                                          const FacePush& fp = FacePush{}) {
  constexpr int M = Lds8::M;
  constexpr int N = Lds8::N;
  constexpr long FS = Frame<MP>::FS;
  constexpr int P = Lds8::P;
  constexpr int NP = F - 5;              // passive fields
  constexpr int NT = NP > 5 ? NP : 5;    // regions of the staged-interior array
  static_assert(NT * P <= 6 * Lds8::P, "staged interiors exceed lds_tin");
  double* const tin = lds_tin;
  double* const acc = lds_acc;
  double* const held = lds_held;
  double* const red = lds_red;

  const int t = threadIdx.x;
  const int dir = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform
  const int l = t & 63;
  const int a = l & 7, b = l >> 3;
  const double ex = dir == 0 ? 1.0 : 0.0;
  const double ey = dir == 1 ? 1.0 : 0.0;
  const double ez = dir == 2 ? 1.0 : 0.0;
  // interior line position c (3..10) -> LDS cell lbase + (c - 3) * lstride
  const int lbase = dir == 0 ? lcell(0, a, b) : dir == 1 ? lcell(a, 0, b) : lcell(a, b, 0);
  const int lstride = dir == 0 ? 1 : dir == 1 ? Lds8::RS : Lds8::PS;
  // stored line position i -> gbase + i * gstride (same for every field)
  const int gbase = Frame<MP>::line(dir, a, b, 0);
  const int gstride = Frame<MP>::stride(dir);
  const double lambda = dt / ldexp(dx, -d.level);
  const double* __restrict__ uin = d.u_in + org;
  // Outputs go to the stored layout of u_in (block frame at `org`) or to the
  // interior-only layout [F][n][n][n] (block origin (ox, oy, oz)); the cells
  // a block owns start at (lox, loy, loz).
  constexpr int NI = MP - 2 * kGhost;
  const bool compact = d.compact != 0;
  double* __restrict__ uout = compact ? d.u_out : d.u_out + org;
  const long ofs = compact ? (long)NI * NI * NI : FS;

  // ---- stage the hydro core ---------------------------------------------
  // The waves issue these loads at a raised priority: a work-group starting
  // beside one in its marches gets its requests out ahead of the other's
  // arithmetic, so their latency overlaps that work (2% on the 8^3 step).
  __builtin_amdgcn_s_setprio(2);
  {
    Share<5> sh;
    load_share<5, MP>(uin, t, sh);
    for (int i = t; i < 5 * P; i += Lds8::kThreads) acc[i] = 0.0;
    store_share<5>(tin, t, sh);
  }
  double g[5][6];
  load_ghosts<5, MP>(uin, gbase, gstride, g);
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();   // tin holds the hydro core; accumulator clear

  double smax = 0.0;
  double wm[N + 1], wp[N + 1];
  {
    Recon<5> rc;
    double Fprev[5];
    double q[5], Wm[5], Wp[5];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      double Ui[5];
#pragma unroll
      for (int k = 0; k < 5; ++k)
        Ui[k] = (i >= kGhost && i < kGhost + N) ? tin[k * P + lbase + (i - kGhost) * lstride]
                                                : g[k][i < kGhost ? i : i - N];
      to_prim(Ui, q);
      switch (i) {
        case 0: rc.step<0>(q, Wm, Wp); break;
        case 1: rc.step<1>(q, Wm, Wp); break;
        case 2: rc.step<2>(q, Wm, Wp); break;
        case 3: rc.step<3>(q, Wm, Wp); break;
        case 4: rc.step<4>(q, Wm, Wp); break;
        case 5: rc.step<5>(q, Wm, Wp); break;
        default: rc.step<6>(q, Wm, Wp); break;
      }
      if (i >= 5) {
        double Fh[5];
        const int face = i - 5;  // face (i-3)+1/2, 0..N
        smax = fmax(smax, core_flux(Wm, Wp, ex, ey, ez, Fh, wm[face], wp[face]));
        if (i >= 6) {
          const int cell = lbase + (i - 6) * lstride;   // interior cell of position i-3
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

  // ---- passive fields: first burst -----------------------------------------
  // The passive inputs arrive in two bursts: fields [0, NA) now, fields
  // [NA, NP) while the first ones are marched, so the registers of the whole
  // burst are never live together with the hydro finalize (with one burst
  // the compiler spilled ~20 registers there; with two, none).
  constexpr int NA = (NP + 1) / 2;
  constexpr int NB = NP - NA;
  constexpr int NBs = NB > 0 ? NB : 1;
  Share<NA> ps;
  double pg[NA][6];
  load_share<NA, MP>(uin + 5 * FS, t, ps);
  load_ghosts<NA, MP>(uin + 5 * FS, gbase, gstride, pg);
  __syncthreads();   // hydro sums complete; tin free
  finalize_shared<5, MP, false, BLEND, PUSH>(held, acc, 0, lambda, uout, compact, ofs, ox, oy,
                                             oz, lox, loy, loz, t, bl, fp, d.index);
  store_share<NA>(tin, t, ps);
  __syncthreads();   // tin holds the first passive fields; the hydro core is written
  // second burst, in flight during the first marches
  Share<NBs> psb;
  double pgb[NBs][6];
  if constexpr (NB > 0) {
    load_share<NB, MP>(uin + (5 + NA) * FS, t, psb);
    load_ghosts<NB, MP>(uin + (5 + NA) * FS, gbase, gstride, pgb);
  }

  // ---- passive fields from LDS, in two groups of at most 3 ----------------
  // Within a group every wave marches its direction for each field in turn,
  // with no barrier between fields and no atomics: the x lanes store their
  // flux differences to acc region r, the y lanes to held region r, the z
  // lanes U - lambda dF_z to zreg(r) (acc regions 3, 4, then held region 3)
  // for the group's r-th field; one barrier then lets every lane finalize the
  // group.  The second burst goes to LDS (tin regions NA..) during the first
  // group, which reads only regions 0..NA-1.
  static_assert(NA <= 3 && NB <= 3, "passive groups of at most 3 fields");
  // Every lane stores fma(pa, dF, pz u) with the cell's staged value u: the
  // x and y lanes their difference dF (pa = 1, pz = 0: dF + 0 is dF), the z
  // lanes u - lambda dF (pa = -lambda, pz = 1), one rounding as before.
  const double pa = dir == 2 ? -lambda : 1.0;
  const double pz = dir == 2 ? 1.0 : 0.0;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int r = p < NA ? p : p - NA;
    double* const zr = r < 2 ? acc + (3 + r) * P : held + 3 * P;
    // the wave's destination region for this field (uniform): no branch in
    // the march, so the scheduler can overlap the positions and fields
    double* const dst = dir == 0 ? acc + r * P : dir == 1 ? held + r * P : zr;
    Recon<1> rc;
    double Fprev = 0.0;
    double q[1], Wm[1], Wp[1];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if (i >= kGhost && i < kGhost + N) {
        q[0] = tin[p * P + lbase + (i - kGhost) * lstride];
      } else {
        const int gi = i < kGhost ? i : i - N;   // ghost slot 0..5
        q[0] = p < NA ? pg[p][gi] : pgb[p - NA][gi];
      }
      switch (i) {
        case 0: rc.step<0>(q, Wm, Wp); break;
        case 1: rc.step<1>(q, Wm, Wp); break;
        case 2: rc.step<2>(q, Wm, Wp); break;
        case 3: rc.step<3>(q, Wm, Wp); break;
        case 4: rc.step<4>(q, Wm, Wp); break;
        case 5: rc.step<5>(q, Wm, Wp); break;
        default: rc.step<6>(q, Wm, Wp); break;
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
    if (p == NA - 1) {
      if constexpr (NB > 0) store_share<NB>(tin + NA * P, t, psb);
      __syncthreads();
      finalize_shared<NA, MP, true, BLEND, PUSH>(held, acc, 5, lambda, uout, compact, ofs, ox,
                                                 oy, oz, lox, loy, loz, t, bl, fp, d.index);
      if constexpr (NB > 0) __syncthreads();   // group 1 read before group 2 writes
    }
    if constexpr (NB > 0) {
      if (p == NP - 1) {
        __syncthreads();
        finalize_shared<NB, MP, true, BLEND, PUSH>(held, acc, 5 + NA, lambda, uout, compact,
                                                   ofs, ox, oy, oz, lox, loy, loz, t, bl, fp,
                                                   d.index);
      }
    }
  }

  if (amax_out) {
    smax = wave_max(smax);
    if (l == 0) red[dir] = smax;
    __syncthreads();
    if (t == 0) {
      const double m = fmax(fmax(red[0], red[1]), red[2]);
      if constexpr (PARTS)
        amax_out[(long)d.index * kAmaxParts + part] = m;
      else if (MULTI)
        atomicMax(reinterpret_cast<unsigned long long*>(&amax_out[d.index]),
                  (unsigned long long)__double_as_longlong(m));
      else
        amax_out[d.index] = m;
    }
  }
}

// Blocks per sub-grid of parent edge MP, and the block geometry of block b.
template <int MP>
struct Blocks {
  static constexpr int N = MP - 2 * kGhost;
  static constexpr int NB = N == 8 ? 1 : 2;        // blocks per axis
  static constexpr int kPerSubgrid = NB * NB * NB;
  static constexpr int kShift = N - 8;             // origin of the second block
  static_assert(N == 8 || N == 12 || N == 16, "edges 8, 12, 16");
  // b -> stored offset of the block frame (org), block origin in interior
  // coordinates (ox, oy, oz), first owned block-local coordinates (lo*).
  __device__ static __forceinline__ void geo(int b, int& org, int& ox, int& oy, int& oz,
                                             int& lox, int& loy, int& loz) {
    const int bx = b % NB, by = (b / NB) % NB, bz = b / (NB * NB);
    ox = bx * kShift;
    oy = by * kShift;
    oz = bz * kShift;
    org = (oz * MP + oy) * MP + ox;
    lox = bx ? 16 - N : 0;   // the second block owns the parent cells 8..N-1
    loy = by ? 16 - N : 0;
    loz = bz ? 16 - N : 0;
  }
};

// Table form.  Blocks of one sub-grid get work-group indices that are equal
// modulo 8, so they run on the same XCD and share its L2 for their
// overlapping halos.  The grid is ceil(count/8)*8*kPerSubgrid.
template <int F, int MP>
__global__ void __launch_bounds__(Lds8::kThreads, 2)
    hydro_lds8_kernel(const DevDesc* __restrict__ table, int count, double dt,
                      double dx, double* __restrict__ amax_out) {
  constexpr int B = Blocks<MP>::kPerSubgrid;
  const int w = blockIdx.x;
  const int s = B == 1 ? w : (w / (8 * B)) * 8 + (w & 7);
  const int b = B == 1 ? 0 : (w >> 3) % B;
  if (s >= count) return;
  int org, ox, oy, oz, lox, loy, loz;
  Blocks<MP>::geo(b, org, ox, oy, oz, lox, loy, loz);
  const DevDesc d = table[s];
  lds8_step<F, MP, (B > 1)>(d, org, ox, oy, oz, lox, loy, loz, dt, dx, amax_out);
}

// Small batches: descriptors in the kernel arguments.
template <int F, int MP>
__global__ void __launch_bounds__(Lds8::kThreads, 2)
    hydro_lds8_arg_kernel(ArgDescs descs, double dt, double dx,
                          double* __restrict__ amax_out) {
  constexpr int B = Blocks<MP>::kPerSubgrid;
  int org, ox, oy, oz, lox, loy, loz;
  Blocks<MP>::geo(blockIdx.x % B, org, ox, oy, oz, lox, loy, loz);
  const DevDesc d = descs.d[blockIdx.x / B];
  lds8_step<F, MP, (B > 1)>(d, org, ox, oy, oz, lox, loy, loz, dt, dx, amax_out);
}

// The stages of the device time-step on a brick of 8^3 sub-grids (stored
// layout, descriptor index = brick index): the step's stores, blended with
// another state when BLEND (BlendArgs), each also written to the face ghosts
// it stands for (FacePush).  amax as the table kernel, when amax_out is set.
// When count is a multiple of 8, XCD k (work-groups w = k mod 8) takes the
// k-th eighth of the brick, a run of consecutive sub-grids in brick order
// (x fastest; a whole z layer of an 8 x 8 x 8 brick): a sub-grid and its x
// neighbours then mostly share one L2, where the 24-byte ghost rows one
// writes and the interior rows the other writes meet in the same lines.
template <int F, bool BLEND>
__global__ void __launch_bounds__(Lds8::kThreads, 2)
    hydro_lds8_stage_kernel(const DevDesc* __restrict__ table, int count, double dt, double dx,
                            BlendArgs bl, FacePush fp, double* __restrict__ amax_out) {
  const int w = blockIdx.x;
  const int s = (count & 7) ? w : (w & 7) * (count >> 3) + (w >> 3);
  if (s >= count) return;
  const DevDesc d = table[s];
  lds8_step<F, 14, false, false, BLEND, true>(d, 0, 0, 0, 0, 0, 0, 0, dt, dx, amax_out, 0, bl,
                                              fp);
}

// amax slots of a batch set to zero before a multi-block launch (a kernel,
// so it can live inside a captured graph).
static __global__ void amax_zero_table(const DevDesc* __restrict__ table, int count,
                                double* __restrict__ amax_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) amax_out[table[i].index] = 0.0;
}

static __global__ void amax_zero_args(ArgDescs descs, int count, double* __restrict__ amax_out) {
  const int i = threadIdx.x;
  if (i < count) amax_out[descs.d[i].index] = 0.0;
}

}  // namespace hydro

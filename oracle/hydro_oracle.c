/*
 * hydro_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of one forward-Euler
 * stage of the sub-grid hydrodynamics step that the paper's work aggregation
 * speeds up (Section IV-B "Hydro Solver"; Section V-A for the sub-grid shape:
 * N^3 interior cells plus 3 ghost layers).  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library; the
 * product path never does.  It shares no code, header or table with the HIP
 * path.
 *
 * Arithmetic is IEEE FP64 (Section VI-A: all floating point work is in double
 * precision), compiled with -ffp-contract=off so every operation rounds once,
 * in the order written below.
 *
 * Method, as read from the paper (Section IV-B) plus the two methods it cites
 * by name (Colella & Woodward 1984 PPM; the Kurganov central-upwind flux):
 *   O1  primitives  rho, v = s/rho, p = (gamma-1)(E - s.v/2); tau and the
 *       species partial densities are carried as stored.
 *   O2  PPM interface values from monotonised-central slopes.
 *   O3  the Colella-Woodward monotonicity constraint on each cell's parabola.
 *   O4  face states: W- = right edge of the left cell, W+ = left edge of the
 *       right cell, at the centre of every face (the 6 face-centre points of
 *       the 26 quadrature points; the full 26-point form, with edge and
 *       vertex points and Newton-Cotes quadrature over each face, is the
 *       separate oracle_step26 below: Q1-Q7).
 *   O5  physical state U(W) and flux F_d(W) of the ideal-gas Euler system.
 *   O6  central-upwind (Kurganov-Noelle-Petrova) numerical flux with
 *       one-sided speeds a+ and a-; amax = max over faces of max(a+, -a-)
 *       (the signal speed behind the Courant limit, Section IV-B).
 *   O7  U_out = U - (dt/dx_s) * sum_d (F_{d,+} - F_{d,-}) on interior cells;
 *       ghost cells of u_out are never written.
 * Readings where the paper is silent are listed in the design notes; the
 * relevant ones are restated next to the code they shape.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Ideal-gas adiabatic index (reading: gamma = 5/3, a monatomic gas). */
static const double GAMMA = 5.0 / 3.0;
static const int GHOST = 3; /* ghost-layer depth (Section V-A) */

/* One sub-grid as the oracle sees it: stored edge M = n + 6, SoA
 * [field][z][y][x] with x fastest.  Same field order as the public ABI:
 * 0 rho, 1 sx, 2 sy, 3 sz, 4 egas, 5 tau, 6.. species partial densities. */
typedef struct {
  const double *u_in;
  double *u_out;
  int32_t n;
  int32_t nfields;
  int32_t level;
  int32_t reserved;
} oracle_subgrid;

/* Branch counters (indices into the optional int64 array of length
 * ORACLE_NCOUNT).  They show which limiter cases the inputs exercise. */
enum {
  CNT_SLOPE_ZERO = 0,     /* O2: neighbouring differences disagree in sign */
  CNT_SLOPE_CENTRAL = 1,  /* O2: central slope kept                        */
  CNT_SLOPE_LIMITED = 2,  /* O2: slope clipped to twice a one-sided diff   */
  CNT_PAR_FLAT = 3,       /* O3: local extremum, parabola flattened        */
  CNT_PAR_LEFT = 4,       /* O3: q_L reset to 3q - 2q_R                    */
  CNT_PAR_RIGHT = 5,      /* O3: q_R reset to 3q - 2q_L                    */
  CNT_PAR_KEEP = 6,       /* O3: parabola already monotone                 */
  CNT_NONPOS_CELL = 7,    /* rho <= 0 or p <= 0 at a cell                  */
  CNT_NONPOS_FACE = 8,    /* rho <= 0 or p <= 0 at a face state            */
  ORACLE_NCOUNT = 9
};

static size_t at(int M, int f, int z, int y, int x) {
  return (((size_t)f * M + z) * M + y) * M + x;
}

/* ---- O1: primitive variables of one cell ------------------------------ */
static void to_primitive(const double *U, int nf, double *q) {
  double rho = U[0];
  double vx = U[1] / rho;
  double vy = U[2] / rho;
  double vz = U[3] / rho;
  double kin = 0.5 * (U[1] * vx + U[2] * vy + U[3] * vz);
  q[0] = rho;
  q[1] = vx;
  q[2] = vy;
  q[3] = vz;
  q[4] = (GAMMA - 1.0) * (U[4] - kin);
  for (int f = 5; f < nf; ++f) q[f] = U[f];
}

/* ---- O2 + O3: PPM along one line ----------------------------------------
 * q[i*nf + f], i = 0..len-1, is the line including 3 ghosts on each side.
 * On return, for every cell i in [2, len-3], qL[i*nf+f] and qR[i*nf+f] hold
 * the limited left and right edge values of its parabola.  Other entries of
 * qL/qR are left untouched.  cnt may be NULL. */
static void ppm_line(const double *q, int len, int nf, double *qL, double *qR,
                     int64_t *cnt) {
  double *dm = (double *)malloc(sizeof(double) * (size_t)len * nf);
  double *face = (double *)malloc(sizeof(double) * (size_t)len * nf);
  for (int f = 0; f < nf; ++f) {
    /* O2a: monotonised-central slope at cells 1..len-2 (CW84 eq. 1.7-1.8) */
    for (int i = 1; i <= len - 2; ++i) {
      double qm = q[(i - 1) * nf + f];
      double q0 = q[i * nf + f];
      double qp = q[(i + 1) * nf + f];
      double dq = 0.5 * (qp - qm);
      double s;
      if ((qp - q0) * (q0 - qm) > 0.0) {
        double lim = fmin(2.0 * fabs(q0 - qm), 2.0 * fabs(qp - q0));
        double mag = fmin(fabs(dq), lim);
        s = (dq > 0.0 ? 1.0 : (dq < 0.0 ? -1.0 : 0.0)) * mag;
        if (cnt) cnt[fabs(dq) <= lim ? CNT_SLOPE_CENTRAL : CNT_SLOPE_LIMITED]++;
      } else {
        s = 0.0;
        if (cnt) cnt[CNT_SLOPE_ZERO]++;
      }
      dm[i * nf + f] = s;
    }
    /* O2b: interface value between cells i and i+1, i = 1..len-3
     * (CW84 eq. 1.6 on a uniform grid). */
    for (int i = 1; i <= len - 3; ++i) {
      double q0 = q[i * nf + f];
      double q1 = q[(i + 1) * nf + f];
      face[i * nf + f] =
          q0 + 0.5 * (q1 - q0) - (dm[(i + 1) * nf + f] - dm[i * nf + f]) / 6.0;
    }
    /* O3: monotonicity constraint for cells i = 2..len-3 (CW84 eq. 1.10) */
    for (int i = 2; i <= len - 3; ++i) {
      double qc = q[i * nf + f];
      double l = face[(i - 1) * nf + f];
      double r = face[i * nf + f];
      if ((r - qc) * (qc - l) <= 0.0) {
        l = qc;
        r = qc;
        if (cnt) cnt[CNT_PAR_FLAT]++;
      } else {
        double d = r - l;
        double c6 = d * (qc - 0.5 * (l + r));
        double d2 = d * d / 6.0;
        if (c6 > d2) {
          l = 3.0 * qc - 2.0 * r;
          if (cnt) cnt[CNT_PAR_LEFT]++;
        } else if (-d2 > c6) {
          r = 3.0 * qc - 2.0 * l;
          if (cnt) cnt[CNT_PAR_RIGHT]++;
        } else {
          if (cnt) cnt[CNT_PAR_KEEP]++;
        }
      }
      qL[i * nf + f] = l;
      qR[i * nf + f] = r;
    }
  }
  free(dm);
  free(face);
}

/* ---- O5: conserved state and physical flux of a primitive state -------- */
static void state_of(const double *W, int nf, double *U) {
  double rho = W[0];
  U[0] = rho;
  U[1] = rho * W[1];
  U[2] = rho * W[2];
  U[3] = rho * W[3];
  U[4] = W[4] / (GAMMA - 1.0) +
         0.5 * rho * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  for (int f = 5; f < nf; ++f) U[f] = W[f];
}

static void flux_of(const double *W, int nf, int d, double *F) {
  double U[16];
  state_of(W, nf, U);
  double vd = W[1 + d];
  double p = W[4];
  F[0] = U[0] * vd;
  F[1] = U[1] * vd;
  F[2] = U[2] * vd;
  F[3] = U[3] * vd;
  F[1 + d] = F[1 + d] + p;
  F[4] = (U[4] + p) * vd;
  for (int f = 5; f < nf; ++f) F[f] = U[f] * vd;
}

/* ---- O6: central-upwind flux at one face -------------------------------
 * Wm = state on the low side, Wp = state on the high side (primitive).
 * Returns max(a+, -a-) and writes Fh[0..nf-1]. */
static double knp_flux(const double *Wm, const double *Wp, int nf, int d,
                       double *Fh) {
  double cm = sqrt(GAMMA * Wm[4] / Wm[0]);
  double cp = sqrt(GAMMA * Wp[4] / Wp[0]);
  double vm = Wm[1 + d];
  double vp = Wp[1 + d];
  double ap = fmax(fmax(vm + cm, vp + cp), 0.0);
  double am = fmin(fmin(vm - cm, vp - cp), 0.0);
  double Um[16], Up[16], Fm[16], Fp[16];
  state_of(Wm, nf, Um);
  state_of(Wp, nf, Up);
  flux_of(Wm, nf, d, Fm);
  flux_of(Wp, nf, d, Fp);
  for (int f = 0; f < nf; ++f)
    Fh[f] = (ap * Fm[f] - am * Fp[f] + ap * am * (Up[f] - Um[f])) / (ap - am);
  return fmax(ap, -am);
}

/* ---- steps shared by both forms ----------------------------------------- */

/* lambda_s = dt / dx_s with dx_s = dx 2^-level */
static double lambda_of(const oracle_subgrid *sg, double dt, double dx) {
  return dt / ldexp(dx, -sg->level);
}

/* F_{+} - F_{-} of direction d for the interior cells of the line through
 * transverse (a, b): Fh[i] is the flux through face i+1/2 (stored i). */
static void line_differences(double *dF, int d, int a, int b, const double *Fh, int N, int nf) {
  const size_t nint = (size_t)N * N * N;
  for (int i = GHOST; i < GHOST + N; ++i) {
    int ix, iy, iz;
    if (d == 0) { ix = i - GHOST; iy = a; iz = b; }
    else if (d == 1) { ix = a; iy = i - GHOST; iz = b; }
    else { ix = a; iy = b; iz = i - GHOST; }
    size_t c = ((size_t)iz * N + iy) * N + ix;
    for (int f = 0; f < nf; ++f)
      dF[((size_t)d * nint + c) * nf + f] = Fh[i * nf + f] - Fh[(i - 1) * nf + f];
  }
}

/* O7 / Q7: x, then y, then z; then scale by dt/dx_s. */
static void apply_update(const oracle_subgrid *sg, const double *dF, double lambda) {
  const int N = sg->n, nf = sg->nfields, M = N + 2 * GHOST;
  const size_t nint = (size_t)N * N * N;
  for (int z = 0; z < N; ++z)
    for (int y = 0; y < N; ++y)
      for (int x = 0; x < N; ++x) {
        size_t c = ((size_t)z * N + y) * N + x;
        for (int f = 0; f < nf; ++f) {
          double s = dF[(0 * nint + c) * nf + f];
          s = s + dF[(1 * nint + c) * nf + f];
          s = s + dF[(2 * nint + c) * nf + f];
          size_t g = at(M, f, z + GHOST, y + GHOST, x + GHOST);
          sg->u_out[g] = sg->u_in[g] - lambda * s;
        }
      }
}

/* ---- O1..O7 for one sub-grid ------------------------------------------- */
static double step_one(const oracle_subgrid *sg, double dt, double dx,
                       int64_t *cnt) {
  const int N = sg->n, nf = sg->nfields, M = N + 2 * GHOST;
  const double lambda = lambda_of(sg, dt, dx);
  const size_t ncell = (size_t)M * M * M;
  double amax = 0.0;

  /* O1 on every stored cell. */
  double *q = (double *)malloc(sizeof(double) * ncell * nf);
  for (int z = 0; z < M; ++z)
    for (int y = 0; y < M; ++y)
      for (int x = 0; x < M; ++x) {
        double U[16];
        size_t c = ((size_t)z * M + y) * M + x;
        for (int f = 0; f < nf; ++f) U[f] = sg->u_in[at(M, f, z, y, x)];
        to_primitive(U, nf, &q[c * nf]);
        /* only cells that some stencil reads are counted */
        int inx = x >= GHOST && x < GHOST + N, iny = y >= GHOST && y < GHOST + N,
            inz = z >= GHOST && z < GHOST + N;
        if (cnt && inx + iny + inz >= 2 && (q[c * nf] <= 0.0 || q[c * nf + 4] <= 0.0))
          cnt[CNT_NONPOS_CELL]++;
      }

  /* Flux differences per direction, interior cells only: dF[d][cell][f]. */
  const size_t nint = (size_t)N * N * N;
  double *dF = (double *)calloc(3 * nint * nf, sizeof(double));
  double *line = (double *)malloc(sizeof(double) * M * nf);
  double *qL = (double *)malloc(sizeof(double) * M * nf);
  double *qR = (double *)malloc(sizeof(double) * M * nf);
  double *Fh = (double *)malloc(sizeof(double) * M * nf);

  for (int d = 0; d < 3; ++d) {
    for (int b = 0; b < N; ++b)
      for (int a = 0; a < N; ++a) {
        /* Line along d whose two transverse coordinates are interior
         * (reading: no reconstruction in transverse ghost layers). */
        for (int i = 0; i < M; ++i) {
          int x, y, z;
          if (d == 0) { x = i; y = GHOST + a; z = GHOST + b; }
          else if (d == 1) { x = GHOST + a; y = i; z = GHOST + b; }
          else { x = GHOST + a; y = GHOST + b; z = i; }
          size_t c = ((size_t)z * M + y) * M + x;
          memcpy(&line[i * nf], &q[c * nf], sizeof(double) * nf);
        }
        ppm_line(line, M, nf, qL, qR, cnt);
        /* O4 + O6: faces i+1/2 for stored i = 2..M-4 (N+1 faces). */
        for (int i = 2; i <= M - 4; ++i) {
          const double *Wm = &qR[i * nf];
          const double *Wp = &qL[(i + 1) * nf];
          if (cnt && (Wm[0] <= 0.0 || Wm[4] <= 0.0 || Wp[0] <= 0.0 || Wp[4] <= 0.0))
            cnt[CNT_NONPOS_FACE]++;
          double s = knp_flux(Wm, Wp, nf, d, &Fh[i * nf]);
          if (s > amax) amax = s;
        }
        /* F_{+} - F_{-} for interior stored cells i = 3..M-4. */
        line_differences(dF, d, a, b, Fh, N, nf);
      }
  }

  /* O7 */
  apply_update(sg, dF, lambda);

  free(q);
  free(dF);
  free(line);
  free(qL);
  free(qR);
  free(Fh);
  return amax;
}

/* ---- the 26-point form (Section IV-B: reconstruction at the 26 points on
 * a cell's surface -- 6 face centres, 12 edge midpoints, 8 vertices --
 * central-upwind fluxes at those points, Newton-Cotes quadrature over each
 * face) ---------------------------------------------------------------------
 *   Q1  primitives of every stored cell (edge and corner ghosts included).
 *   Q2+Q3  the value of cell c at the point c + e/2 of its surface, for each
 *       of the 26 directions e in {-1,0,1}^3 \ {0}: PPM (O2 + O3) along the
 *       line of cells c + k e, k = -2..2, oriented along e; the value is the
 *       right edge (toward +e) of c's limited parabola on that line.
 *   Q4  a face normal to axis d between cells c and c + n (n the unit vector
 *       of d) has 9 points, offsets (s1, s2) in {-1,0,1}^2 along its two
 *       transverse axes t1 < t2: W- = value of c toward n + s1 t1 + s2 t2,
 *       W+ = value of c + n toward -n + s1 t1 + s2 t2.
 *   Q5+Q6  central-upwind flux along d at each point (O5, O6); the face flux
 *       is Simpson's rule in both transverse directions,
 *       (16 F_centre + 4 sum F_edge-midpoints + sum F_vertices) / 36, summed
 *       in the order s2 = -1..1 (outer), s1 = -1..1 (inner); amax covers
 *       every point of every face.
 *   Q7  as O7.
 * The same faces as the face-centre form (N+1 per line, transverse
 * coordinates interior); their stencils reach 2 cells along e from cells
 * 2..M-3 of the normal axis, inside the 3 ghost layers. */

/* value of the stored cell (x, y, z) toward direction e (Q2+Q3) */
static void point_value(const double *q, int M, int nf, int x, int y, int z,
                        const int e[3], double *out, int64_t *cnt) {
  double line[5 * 16], qL[5 * 16], qR[5 * 16];
  for (int k = -2; k <= 2; ++k) {
    size_t c = ((size_t)(z + k * e[2]) * M + (y + k * e[1])) * M + (x + k * e[0]);
    memcpy(&line[(k + 2) * nf], &q[c * nf], sizeof(double) * nf);
  }
  ppm_line(line, 5, nf, qL, qR, cnt);
  memcpy(out, &qR[2 * nf], sizeof(double) * nf);
}

static double step26_one(const oracle_subgrid *sg, double dt, double dx,
                         int64_t *cnt) {
  const int N = sg->n, nf = sg->nfields, M = N + 2 * GHOST;
  const double lambda = lambda_of(sg, dt, dx);
  const size_t ncell = (size_t)M * M * M;
  double amax = 0.0;

  /* Q1 */
  double *q = (double *)malloc(sizeof(double) * ncell * nf);
  for (int z = 0; z < M; ++z)
    for (int y = 0; y < M; ++y)
      for (int x = 0; x < M; ++x) {
        double U[16];
        size_t c = ((size_t)z * M + y) * M + x;
        for (int f = 0; f < nf; ++f) U[f] = sg->u_in[at(M, f, z, y, x)];
        to_primitive(U, nf, &q[c * nf]);
      }

  const size_t nint = (size_t)N * N * N;
  double *dF = (double *)calloc(3 * nint * nf, sizeof(double));
  double *Fh = (double *)malloc(sizeof(double) * M * nf);
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    for (int b = 0; b < N; ++b)
      for (int a = 0; a < N; ++a) {
        /* faces i+1/2 of the line along d through transverse (a, b): the
         * faces of its interior cells GHOST..GHOST+N-1 */
        for (int i = GHOST - 1; i <= GHOST + N - 1; ++i) {
          int lo[3], hi[3];
          lo[d] = i;
          lo[t1] = GHOST + a;
          lo[t2] = GHOST + b;
          memcpy(hi, lo, sizeof lo);
          hi[d] = i + 1;
          double acc[16] = {0};
          for (int s2 = -1; s2 <= 1; ++s2)
            for (int s1 = -1; s1 <= 1; ++s1) {
              int em[3] = {0, 0, 0}, ep[3] = {0, 0, 0};
              em[d] = 1;
              ep[d] = -1;
              em[t1] = ep[t1] = s1;
              em[t2] = ep[t2] = s2;
              double Wm[16], Wp[16], F[16];
              point_value(q, M, nf, lo[0], lo[1], lo[2], em, Wm, cnt);
              point_value(q, M, nf, hi[0], hi[1], hi[2], ep, Wp, cnt);
              if (cnt && (Wm[0] <= 0.0 || Wm[4] <= 0.0 || Wp[0] <= 0.0 || Wp[4] <= 0.0))
                cnt[CNT_NONPOS_FACE]++;
              double sp = knp_flux(Wm, Wp, nf, d, F);
              if (sp > amax) amax = sp;
              const double w = (s1 == 0 && s2 == 0) ? 16.0 : (s1 == 0 || s2 == 0) ? 4.0 : 1.0;
              for (int f = 0; f < nf; ++f) acc[f] = acc[f] + w * F[f];
            }
          for (int f = 0; f < nf; ++f) Fh[i * nf + f] = acc[f] / 36.0;
        }
        line_differences(dF, d, a, b, Fh, N, nf);
      }
  }

  /* Q7 (= O7) */
  apply_update(sg, dF, lambda);
  free(q);
  free(dF);
  free(Fh);
  return amax;
}

/* ---- exported entry points ------------------------------------------- */

int oracle_ncounters(void) { return ORACLE_NCOUNT; }

/* Validate one descriptor the way the step needs it; 0 = fine. */
static int bad_subgrid(const oracle_subgrid *s) {
  if (!s->u_in || !s->u_out || s->u_in == s->u_out) return 1;
  if (s->n < 1 || s->nfields < 5 || s->nfields > 16) return 1;
  return 0;
}

/* One stage over `count` independent sub-grids.  amax (length count) and
 * counters (length ORACLE_NCOUNT, accumulated into) may be NULL.
 * nthreads <= 1 runs sequentially; otherwise an OpenMP loop over sub-grids
 * (used only to time the oracle on all host cores). Returns 0, or -1 on a
 * bad argument. */
int oracle_step(const oracle_subgrid *sg, int count, double dt, double dx,
                double *amax, int64_t *counters, int nthreads) {
  if (count < 0 || (count > 0 && !sg) || !(dx > 0.0) || !(dt >= 0.0)) return -1;
  for (int s = 0; s < count; ++s)
    if (bad_subgrid(&sg[s])) return -1;
  if (nthreads <= 1) {
    for (int s = 0; s < count; ++s) {
      double a = step_one(&sg[s], dt, dx, counters);
      if (amax) amax[s] = a;
    }
    return 0;
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int s = 0; s < count; ++s) {
    double a = step_one(&sg[s], dt, dx, NULL);
    if (amax) amax[s] = a;
  }
  return 0;
#else
  return -1;
#endif
}

/* One stage of the 26-point form over `count` independent sub-grids, with
 * the arguments and results of oracle_step.  Sub-grids need their edge and
 * corner ghosts filled (the face-centre form never reads them). */
int oracle_step26(const oracle_subgrid *sg, int count, double dt, double dx,
                  double *amax, int64_t *counters, int nthreads) {
  if (count < 0 || (count > 0 && !sg) || !(dx > 0.0) || !(dt >= 0.0)) return -1;
  for (int s = 0; s < count; ++s)
    if (bad_subgrid(&sg[s]) || sg[s].n < 1) return -1;
  if (nthreads <= 1) {
    for (int s = 0; s < count; ++s) {
      double a = step26_one(&sg[s], dt, dx, counters);
      if (amax) amax[s] = a;
    }
    return 0;
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int s = 0; s < count; ++s) {
    double a = step26_one(&sg[s], dt, dx, NULL);
    if (amax) amax[s] = a;
  }
  return 0;
#else
  return -1;
#endif
}

/* Q2+Q3 at one cell of a stored block of primitives q[M^3][nf]: the value of
 * cell (x, y, z) toward direction e (for tests of the point geometry). */
int oracle_point_value(const double *q, int M, int nf, int x, int y, int z,
                       const int32_t *e, double *out) {
  int ee[3] = {e[0], e[1], e[2]};
  for (int k = 0; k < 3; ++k) {
    if (ee[k] < -1 || ee[k] > 1) return -1;
    int c = k == 0 ? x : k == 1 ? y : z;
    if (c - 2 * abs(ee[k]) < 0 || c + 2 * abs(ee[k]) >= M) return -1;
  }
  if (!ee[0] && !ee[1] && !ee[2]) return -1;
  point_value(q, M, nf, x, y, z, ee, out, NULL);
  return 0;
}

/* Building blocks exposed so tests can pin them in isolation. */

/* O1 on one cell: U[nf] -> q[nf]. */
void oracle_primitive(const double *U, int nf, double *q) { to_primitive(U, nf, q); }

/* O2+O3 on one line: q[len*nf] -> qL, qR (cells 2..len-3 written). */
int oracle_ppm_line(const double *q, int len, int nf, double *qL, double *qR,
                    int64_t *counters) {
  if (len < 5 || nf < 1) return -1;
  ppm_line(q, len, nf, qL, qR, counters);
  return 0;
}

/* O5 physical state and flux of one primitive state along direction d. */
void oracle_state(const double *W, int nf, double *U) { state_of(W, nf, U); }
void oracle_flux(const double *W, int nf, int d, double *F) { flux_of(W, nf, d, F); }

/* O6 at one face; returns max(a+, -a-). */
double oracle_knp_flux(const double *Wm, const double *Wp, int nf, int d,
                       double *Fh) {
  return knp_flux(Wm, Wp, nf, d, Fh);
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// rk3_api.hip -- host side of the device time-step on a brick of sub-grids:
// ghost-layer fill and the three-stage SSP Runge-Kutta method of Shu and
// Osher composed from the aggregated hydro step (the paper's time-step is
// three solver iterations, Section VI-A; sub-grids with 3-cell ghost layers
// filled from their neighbours, Section V-A).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "../../include/hydroagg.h"
#include "brick.hpp"
#include "hydro_lds8.hpp"
#include "internal.hpp"

using hydro::api::fail;

namespace {

#define HIP_TRY(expr)                                                         \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return fail(HYDRO_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr long kMaxBrickSubgrids = 1l << 20;

long brick_count(const hydro_brick_t& b) { return (long)b.nb[0] * b.nb[1] * b.nb[2]; }

long brick_doubles(const hydro_brick_t& b) {
  const long M = b.n + 2 * HYDRO_GHOST;
  return brick_count(b) * b.nfields * M * M * M;
}

int check_brick(const hydro_brick_t* b) {
  if (!b) return fail(HYDRO_EINVAL, "brick is NULL");
  if (hydro::api::class_of_task(b->n, b->nfields) < 0)
    return fail(HYDRO_EINVAL, "unsupported n=%d nfields=%d", b->n, b->nfields);
  for (int d = 0; d < 3; ++d) {
    if (b->nb[d] < 1) return fail(HYDRO_EINVAL, "nb[%d] = %d < 1", d, b->nb[d]);
    if (b->bc[d] != HYDRO_BC_PERIODIC && b->bc[d] != HYDRO_BC_OUTFLOW)
      return fail(HYDRO_EINVAL, "bc[%d] = %d", d, b->bc[d]);
  }
  if (brick_count(*b) > kMaxBrickSubgrids)
    return fail(HYDRO_EINVAL, "%ld sub-grids (at most %ld)", brick_count(*b), kMaxBrickSubgrids);
  if (b->level < 0 || b->level > 30) return fail(HYDRO_EINVAL, "level %d", b->level);
  return HYDRO_OK;
}

int check_buffer(const double* u, const char* what) {
  if (!u) return fail(HYDRO_EINVAL, "%s is NULL", what);
  if ((uintptr_t)u & 15) return fail(HYDRO_EINVAL, "%s must be 16-byte aligned", what);
  return HYDRO_OK;
}

hydro::BrickGeo geo_of(const hydro_brick_t& b) {
  hydro::BrickGeo g;
  const long M = b.n + 2 * HYDRO_GHOST;
  g.nf = b.nfields;
  for (int d = 0; d < 3; ++d) {
    g.nb[d] = b.nb[d];
    g.bc[d] = b.bc[d];
  }
  g.sg_stride = (long)b.nfields * M * M * M;
  return g;
}

int launch_fill(const hydro_brick_t& b, double* u, hipStream_t s) {
  const hydro::BrickGeo g = geo_of(b);
  const dim3 grid((unsigned)(brick_count(b) * b.nfields)), block(256);
  switch (b.n) {
    case 8: hipLaunchKernelGGL(hydro::ghost_fill_kernel<8>, grid, block, 0, s, u, g); break;
    case 12: hipLaunchKernelGGL(hydro::ghost_fill_kernel<12>, grid, block, 0, s, u, g); break;
    default: hipLaunchKernelGGL(hydro::ghost_fill_kernel<16>, grid, block, 0, s, u, g); break;
  }
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int launch_fill_faces(const hydro_brick_t& b, double* u, hipStream_t s) {
  const hydro::BrickGeo g = geo_of(b);
  const int parts = b.n == 8 ? hydro::kFaceParts<8> : b.n == 12 ? hydro::kFaceParts<12>
                                                                 : hydro::kFaceParts<16>;
  const dim3 grid((unsigned)brick_count(b), (unsigned)parts), block(256);
  const bool f11 = b.nfields == 11;
  switch (b.n) {
    case 8:
      if (f11) hipLaunchKernelGGL((hydro::ghost_fill_faces_kernel<8, 11>), grid, block, 0, s, u, u, g);
      else hipLaunchKernelGGL((hydro::ghost_fill_faces_kernel<8, 6>), grid, block, 0, s, u, u, g);
      break;
    case 12:
      if (f11) hipLaunchKernelGGL((hydro::ghost_fill_faces_kernel<12, 11>), grid, block, 0, s, u, u, g);
      else hipLaunchKernelGGL((hydro::ghost_fill_faces_kernel<12, 6>), grid, block, 0, s, u, u, g);
      break;
    default:
      if (f11) hipLaunchKernelGGL((hydro::ghost_fill_faces_kernel<16, 11>), grid, block, 0, s, u, u, g);
      else hipLaunchKernelGGL((hydro::ghost_fill_faces_kernel<16, 6>), grid, block, 0, s, u, u, g);
      break;
  }
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int launch_combine(const hydro_brick_t& b, double* out, const double* x, const double* y,
                   double a, double c, hipStream_t s) {
  const long M = b.n + 2 * HYDRO_GHOST;
  const long stride = (long)b.nfields * M * M * M;
  const dim3 grid((unsigned)(brick_count(b) * b.nfields)), block(256);
  switch (b.n) {
    case 8:
      hipLaunchKernelGGL(hydro::rk_combine_kernel<8>, grid, block, 0, s, out, x, y, a, c, stride, b.nfields);
      break;
    case 12:
      hipLaunchKernelGGL(hydro::rk_combine_kernel<12>, grid, block, 0, s, out, x, y, a, c, stride, b.nfields);
      break;
    default:
      hipLaunchKernelGGL(hydro::rk_combine_kernel<16>, grid, block, 0, s, out, x, y, a, c, stride, b.nfields);
      break;
  }
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

}  // namespace

struct hydro_rk3 {
  hydro_brick_t b;
  double* u = nullptr;
  double* w = nullptr;
  double* s = nullptr;
  // n = 8: stage kernels with the combinations and the face-ghost writes in
  // their stores (hydro_lds8_stage_kernel):
  hydro::DevDesc* tab_uw = nullptr;  // descriptors of E(u) -> w
  hydro::DevDesc* tab_ws = nullptr;  // descriptors of E(w) -> s
  hydro::DevDesc* tab_su = nullptr;  // descriptors of E(s) -> u
  // other edges: separate steps, combinations and face-ghost fills
  hydro_plan_t* step_uw = nullptr;  // E(u) -> w
  hydro_plan_t* step_ws = nullptr;  // E(w) -> s
  hydro_plan_t* step_sw = nullptr;  // E(s) -> w
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double g_dt = -1.0, g_dx = -1.0;
  double* g_amax = nullptr;
};

namespace {

// Stage k of the Shu-Osher form with E(V) = V + dt L(V) (one hydro step):
//   1: w = E(u)                    (u = U0; w = U1)
//   2: s = 3/4 u + 1/4 E(w)        (s = U2)
//   3: u = 1/3 u + 2/3 E(s)        (u = U3)
// each leaving the face ghosts of the buffer it forms filled (the
// face-centre step reads no edge or corner ghost).  For n = 8 one stage
// kernel does all of it: the combination and the face-ghost writes are part
// of the step's stores.  Otherwise E goes to the free buffer, and a
// combination kernel and the face-ghost fill follow.
template <int F>
int launch_stage(const hydro::DevDesc* table, long count, double dt, double dx, bool blend,
                 const hydro::BlendArgs& bl, const hydro::FacePush& fp, double* amax,
                 hipStream_t st) {
  const dim3 grid((unsigned)count), block(hydro::Lds8::kThreads);
  if (!blend)
    hipLaunchKernelGGL((hydro::hydro_lds8_stage_kernel<F, false>), grid, block, 0, st, table,
                       (int)count, dt, dx, bl, fp, amax);
  else
    hipLaunchKernelGGL((hydro::hydro_lds8_stage_kernel<F, true>), grid, block, 0, st, table,
                       (int)count, dt, dx, bl, fp, amax);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

// bl = nullptr: the plain step (stage 1)
int stage8(hydro_rk3* rk, const hydro::DevDesc* table, double* out, const hydro::BlendArgs* bl,
           double dt, double dx, double* amax, hipStream_t st) {
  const long count = brick_count(rk->b);
  const hydro::BrickGeo g = geo_of(rk->b);
  hydro::FacePush fp;
  fp.base = out;
  fp.sg_stride = g.sg_stride;
  for (int d = 0; d < 3; ++d) {
    fp.nb[d] = g.nb[d];
    fp.bc[d] = g.bc[d];
  }
  const hydro::BlendArgs b = bl ? *bl : hydro::BlendArgs{0.0, 1.0, 0};
  return rk->b.nfields == 11 ? launch_stage<11>(table, count, dt, dx, bl != nullptr, b, fp, amax, st)
                             : launch_stage<6>(table, count, dt, dx, bl != nullptr, b, fp, amax, st);
}

int stage(hydro_rk3* rk, int k, double dt, double dx, double* amax, hipStream_t st) {
  int rc;
  if (rk->tab_uw) {
    if (k == 1) return stage8(rk, rk->tab_uw, rk->w, nullptr, dt, dx, amax, st);
    if (k == 2) {
      // u's element from s's, in doubles (addresses compared as integers:
      // the buffers are separate allocations, both 16-byte aligned)
      const long delta = ((long)(intptr_t)rk->u - (long)(intptr_t)rk->s) / (long)sizeof(double);
      const hydro::BlendArgs bl{0.75, 0.25, delta};
      return stage8(rk, rk->tab_ws, rk->s, &bl, dt, dx, nullptr, st);
    }
    const hydro::BlendArgs bl{1.0 / 3.0, 2.0 / 3.0, 0};
    return stage8(rk, rk->tab_su, rk->u, &bl, dt, dx, nullptr, st);
  }
  if (k == 1) {
    if ((rc = hydro::api::plan_enqueue(rk->step_uw, dt, dx, amax, st))) return rc;
    return launch_fill_faces(rk->b, rk->w, st);
  }
  if (k == 2) {
    if ((rc = hydro::api::plan_enqueue(rk->step_ws, dt, dx, nullptr, st))) return rc;
    if ((rc = launch_combine(rk->b, rk->s, rk->u, rk->s, 0.75, 0.25, st))) return rc;
    return launch_fill_faces(rk->b, rk->s, st);
  }
  if ((rc = hydro::api::plan_enqueue(rk->step_sw, dt, dx, nullptr, st))) return rc;
  if ((rc = launch_combine(rk->b, rk->u, rk->u, rk->w, 1.0 / 3.0, 2.0 / 3.0, st))) return rc;
  return launch_fill_faces(rk->b, rk->u, st);
}

int check_step_args(hydro_rk3* rk, double dt, double dx) {
  if (!rk) return fail(HYDRO_EINVAL, "time-step object is NULL");
  if (!(dt >= 0.0) || !isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be finite and >= 0");
  if (!(dx > 0.0) || !isfinite(dx)) return fail(HYDRO_EINVAL, "dx must be finite and > 0");
  return HYDRO_OK;
}

void rk3_free(hydro_rk3* rk) {
  if (rk->exec) (void)hipGraphExecDestroy(rk->exec);
  if (rk->graph) (void)hipGraphDestroy(rk->graph);
  if (rk->capture) (void)hipStreamDestroy(rk->capture);
  if (rk->step_uw) (void)hydro_plan_destroy(rk->step_uw);
  if (rk->step_ws) (void)hydro_plan_destroy(rk->step_ws);
  if (rk->step_sw) (void)hydro_plan_destroy(rk->step_sw);
  if (rk->tab_uw) (void)hipFree(rk->tab_uw);
  if (rk->tab_ws) (void)hipFree(rk->tab_ws);
  if (rk->tab_su) (void)hipFree(rk->tab_su);
  delete rk;
}

}  // namespace

extern "C" {

int hydro_ghost_fill(const hydro_brick_t* brick, double* u, void* stream) {
  hydro::api::clear_error();
  int rc = check_brick(brick);
  if (rc) return rc;
  if ((rc = check_buffer(u, "u"))) return rc;
  return launch_fill(*brick, u, (hipStream_t)stream);
}

int hydro_ghost_fill_faces(const hydro_brick_t* brick, double* u, void* stream) {
  hydro::api::clear_error();
  int rc = check_brick(brick);
  if (rc) return rc;
  if ((rc = check_buffer(u, "u"))) return rc;
  return launch_fill_faces(*brick, u, (hipStream_t)stream);
}

int hydro_rk3_create(hydro_rk3_t** out, const hydro_brick_t* brick, double* u, double* w,
                     double* s) {
  hydro::api::clear_error();
  if (!out) return fail(HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_brick(brick);
  if (rc) return rc;
  if ((rc = check_buffer(u, "u")) || (rc = check_buffer(w, "w")) || (rc = check_buffer(s, "s")))
    return rc;
  const uintptr_t bytes = (uintptr_t)brick_doubles(*brick) * sizeof(double);
  const uintptr_t p[3] = {(uintptr_t)u, (uintptr_t)w, (uintptr_t)s};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (p[i] < p[j] + bytes && p[j] < p[i] + bytes)
        return fail(HYDRO_EINVAL, "brick buffers overlap");
  const long count = brick_count(*brick);
  const long M = brick->n + 2 * HYDRO_GHOST;
  const long stride = (long)brick->nfields * M * M * M;
  // the steps of the three stages: u -> w, w -> s, s -> (u or w)
  std::vector<hydro_subgrid_t> a((size_t)count), c((size_t)count), e3((size_t)count);
  for (long i = 0; i < count; ++i) {
    a[i].u_in = u + i * stride;
    a[i].u_out = w + i * stride;
    c[i].u_in = w + i * stride;
    c[i].u_out = s + i * stride;
    e3[i].u_in = s + i * stride;
    e3[i].u_out = (brick->n == 8 ? u : w) + i * stride;
    a[i].n = c[i].n = e3[i].n = brick->n;
    a[i].nfields = c[i].nfields = e3[i].nfields = brick->nfields;
    a[i].level = c[i].level = e3[i].level = brick->level;
    a[i].out_layout = c[i].out_layout = e3[i].out_layout = HYDRO_OUT_STORED;
  }
  hydro_rk3* rk = new hydro_rk3();
  rk->b = *brick;
  rk->u = u;
  rk->w = w;
  rk->s = s;
  if (brick->n == 8) {
    // device descriptor tables of the three stage kernels (index = brick index)
    std::vector<hydro::DevDesc> t1((size_t)count), t2((size_t)count), t3((size_t)count);
    for (long i = 0; i < count; ++i) {
      t1[i] = hydro::api::device_desc(a[i], (int)i);
      t2[i] = hydro::api::device_desc(c[i], (int)i);
      t3[i] = hydro::api::device_desc(e3[i], (int)i);
    }
    const size_t tb = sizeof(hydro::DevDesc) * (size_t)count;
    if (hipMalloc((void**)&rk->tab_uw, tb) != hipSuccess ||
        hipMalloc((void**)&rk->tab_ws, tb) != hipSuccess ||
        hipMalloc((void**)&rk->tab_su, tb) != hipSuccess ||
        hipMemcpy(rk->tab_uw, t1.data(), tb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(rk->tab_ws, t2.data(), tb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(rk->tab_su, t3.data(), tb, hipMemcpyHostToDevice) != hipSuccess) {
      rk3_free(rk);
      return fail(HYDRO_EHIP, "time-step descriptor tables");
    }
  } else if ((rc = hydro_plan_create(&rk->step_uw, a.data(), (int32_t)count)) ||
             (rc = hydro_plan_create(&rk->step_ws, c.data(), (int32_t)count)) ||
             (rc = hydro_plan_create(&rk->step_sw, e3.data(), (int32_t)count))) {
    rk3_free(rk);
    return rc;
  }
  hipError_t e = hipStreamCreateWithFlags(&rk->capture, hipStreamNonBlocking);
  if (e != hipSuccess) {
    rk3_free(rk);
    return fail(HYDRO_EHIP, "capture stream: %s", hipGetErrorString(e));
  }
  *out = rk;
  return HYDRO_OK;
}

int hydro_rk3_stage(hydro_rk3_t* rk, int32_t k, double dt, double dx, double* amax_dev,
                    void* stream) {
  hydro::api::clear_error();
  int rc = check_step_args(rk, dt, dx);
  if (rc) return rc;
  if (k < 1 || k > 3) return fail(HYDRO_EINVAL, "stage %d (1, 2 or 3)", k);
  return stage(rk, k, dt, dx, k == 1 ? amax_dev : nullptr, (hipStream_t)stream);
}

int hydro_rk3_step(hydro_rk3_t* rk, double dt, double dx, double* amax_dev, void* stream) {
  hydro::api::clear_error();
  int rc = check_step_args(rk, dt, dx);
  if (rc) return rc;
  for (int k = 1; k <= 3; ++k)
    if ((rc = stage(rk, k, dt, dx, k == 1 ? amax_dev : nullptr, (hipStream_t)stream))) return rc;
  return HYDRO_OK;
}

int hydro_rk3_launch_graph(hydro_rk3_t* rk, double dt, double dx, double* amax_dev,
                           void* stream) {
  hydro::api::clear_error();
  int rc = check_step_args(rk, dt, dx);
  if (rc) return rc;
  if (!rk->exec || rk->g_dt != dt || rk->g_dx != dx || rk->g_amax != amax_dev) {
    if (rk->exec) {
      (void)hipGraphExecDestroy(rk->exec);
      rk->exec = nullptr;
    }
    if (rk->graph) {
      (void)hipGraphDestroy(rk->graph);
      rk->graph = nullptr;
    }
    HIP_TRY(hipStreamBeginCapture(rk->capture, hipStreamCaptureModeThreadLocal));
    for (int k = 1; k <= 3 && rc == HYDRO_OK; ++k)
      rc = stage(rk, k, dt, dx, k == 1 ? amax_dev : nullptr, rk->capture);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(rk->capture, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(HYDRO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    rk->graph = g;
    HIP_TRY(hipGraphInstantiate(&rk->exec, rk->graph, nullptr, nullptr, 0));
    rk->g_dt = dt;
    rk->g_dx = dx;
    rk->g_amax = amax_dev;
  }
  HIP_TRY(hipGraphLaunch(rk->exec, (hipStream_t)stream));
  return HYDRO_OK;
}

int hydro_rk3_destroy(hydro_rk3_t* rk) {
  hydro::api::clear_error();
  if (!rk) return HYDRO_OK;
  int rc = HYDRO_OK;
  if (hipDeviceSynchronize() != hipSuccess) rc = fail(HYDRO_EHIP, "hipDeviceSynchronize failed");
  rk3_free(rk);
  return rc;
}

}  // extern "C"

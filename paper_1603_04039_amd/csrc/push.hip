// Particle push and the time step of the Vlasov-Poisson loop (Sec. 1): the
// particles move in E = grad phi, which the three steps of Sec. 3.2 compute on
// a node cloud re-selected from the current positions every step (Sec. 4).
//
// The paper leaves the time integrator open.  The push is the leapfrog scheme in
// kick-drift form (velocities half a step behind positions), with specular
// reflection at the faces of Omega; it is a pure HBM stream (per particle and
// axis 24 B read, 16 B written).
#include <hip/hip_runtime.h>

#include <cmath>

#include "apc_internal.h"

void apc_free_cloud(apc_cloud *c);

namespace {

// One thread per particle (x) and axis (y).  Contraction is off so that the kick
// and the drift each round the product and the sum separately.  A particle
// outside [lo, lo + L] after the drift is folded back: u = (x - lo) / L, f =
// floor(u) wall crossings, r = u - f; u becomes r (f even) or 1 - r (f odd) and
// the velocity component changes sign for odd f.  Particles inside keep x + dt v.
// On a periodic domain the particle re-enters through the opposite face: u = r,
// velocity unchanged.
__global__ void __launch_bounds__(APC_BLOCK)
    k_push(int64_t N, double *__restrict__ xyz, double *__restrict__ vel,
           const double *__restrict__ grad, double kick, double dt, double lo0, double lo1,
           double lo2, double L, int periodic) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= N) return;
  const int d = blockIdx.y;
  const double lo = d == 0 ? lo0 : (d == 1 ? lo1 : lo2);
  const double hi = lo + L;
  const int64_t e = (int64_t)d * N + i;
  double v = vel[e] + kick * grad[e];
  double x = xyz[e] + dt * v;
  if (x < lo || x > hi) {
    double u = (x - lo) / L;
    const double f = floor(u);
    const double r = u - f;
    const double half = f * 0.5;
    const bool odd = !periodic && floor(half) != half;
    u = odd ? 1.0 - r : r;
    if (odd) v = -v;
    x = lo + u * L;
  }
  xyz[e] = x;
  vel[e] = v;
}

} // namespace

int apc_push_impl(const apc_params *p, int64_t N, double *xyz, double *vel, const double *grad,
                  double kick, double dt, hipStream_t s) {
  if (!p || N < 0 || !(p->L > 0.0) || !std::isfinite(p->L) || !std::isfinite(kick) ||
      !std::isfinite(dt))
    return APC_EINVAL;
  for (int d = 0; d < 3; d++)
    if (!std::isfinite(p->lo[d])) return APC_EINVAL;
  if (N == 0) return APC_OK;
  if (!xyz || !vel || !grad) return APC_EINVAL;
  if (N > (int64_t)0x7fffffff * APC_BLOCK) return APC_EINVAL;
  hipLaunchKernelGGL(k_push, dim3(grid_for(N), 3), dim3(APC_BLOCK), 0, s, N, xyz, vel, grad, kick,
                     dt, p->lo[0], p->lo[1], p->lo[2], p->L, p->periodic ? 1 : 0);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

// One time step: build, assemble, deposit + density solve, Poisson solve (phi = 0
// on the boundary), interpolation to the particles, push.  The node cloud lives
// for the call only.  Device times per phase come from events on the stream.
namespace {
struct StepEvents {
  hipEvent_t e[7] = {};
  int made = 0;
  ~StepEvents() {
    for (int k = 0; k < made; k++) (void)hipEventDestroy(e[k]);
  }
};
struct StepCloud {
  apc_cloud *c = nullptr;
  ~StepCloud() {
    if (c) apc_free_cloud(c);
  }
};
} // namespace

int apc_step_impl(const apc_params *p, double *xyz, double *vel, const double *q, int64_t N,
                  double kick, double dt, double tol_density, double tol, int maxit, int precond,
                  double *phi_p, double *grad_p, apc_step_stats *st, hipStream_t s) {
  if (!p || !xyz || !vel || !phi_p || !grad_p || N < 1 || !(tol > 0.0) ||
      !(tol_density > 0.0) || maxit < 1 || !std::isfinite(kick) || !std::isfinite(dt))
    return APC_EINVAL;
  if (precond != APC_PRECOND_NONE && precond != APC_PRECOND_JACOBI) return APC_EINVAL;
  if (p->mask_level != 0) return APC_EINVAL; // the push knows the box's walls only
  StepEvents ev;
  for (; ev.made < 7; ev.made++) HIPCHK(hipEventCreate(&ev.e[ev.made]));
  HIPCHK(hipEventRecord(ev.e[0], s));
  StepCloud sc;
  APCCHK(apc_build_impl(p, xyz, N, s, &sc.c));
  apc_cloud *c = sc.c;
  HIPCHK(hipEventRecord(ev.e[1], s));
  APCCHK(apc_assemble_impl(c, s));
  HIPCHK(hipEventRecord(ev.e[2], s));
  const int64_t nt = c->n + c->nb;
  double *buf = nullptr;
  HIPCHK(apc_malloc_async((void **)&buf, 3 * (size_t)nt * sizeof(double), s));
  double *rho_M = buf, *rho_t = buf + nt, *phi = buf + 2 * nt;
  apc_stats sd = {}, sp = {};
  int status = APC_OK;
  int rc = apc_deposit_impl(c, q, rho_M, s);
  if (rc >= 0) rc = apc_density_solve_impl(c, rho_M, rho_t, tol_density, maxit, &sd, s);
  if (rc == APC_ENOCONV) status = APC_ENOCONV;
  if (rc >= 0) rc = hipEventRecord(ev.e[3], s) == hipSuccess ? APC_OK : APC_EHIP;
  if (rc >= 0) rc = apc_solve_impl(c, rho_t, nullptr, phi, tol, maxit, precond, &sp, s);
  if (rc == APC_ENOCONV) status = APC_ENOCONV;
  if (rc >= 0) rc = hipEventRecord(ev.e[4], s) == hipSuccess ? APC_OK : APC_EHIP;
  if (rc >= 0) rc = apc_interp_impl(c, phi, phi_p, grad_p, s);
  if (rc >= 0) rc = hipEventRecord(ev.e[5], s) == hipSuccess ? APC_OK : APC_EHIP;
  if (rc >= 0) rc = apc_push_impl(p, N, xyz, vel, grad_p, kick, dt, s);
  if (rc >= 0) rc = hipEventRecord(ev.e[6], s) == hipSuccess ? APC_OK : APC_EHIP;
  HIPCHK(apc_free_async(buf, s));
  APCCHK(rc);
  HIPCHK(hipEventSynchronize(ev.e[6]));
  if (st) {
    st->n = c->n;
    st->nb = c->nb;
    st->nnz = c->nnz;
    st->density_iters = sd.iters;
    st->iters = sp.iters;
    st->status = status;
    st->pad = 0;
    st->rel_resid_true = sp.rel_resid_true;
    for (int k = 0; k < 6; k++) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev.e[k], ev.e[k + 1]));
      st->ms[k] = ms;
    }
  }
  return status;
}

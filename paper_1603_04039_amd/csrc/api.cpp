// C ABI of the gfx950 AP-Cloud library (declared in include/apcloud.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "apc_internal.h"

void apc_free_cloud(apc_cloud *c);

static thread_local char g_err[512] = {0};

void apc_set_hip_error(hipError_t e, const char *what, const char *file, int line) {
  snprintf(g_err, sizeof(g_err), "%s: %s (%s:%d)", hipGetErrorString(e), what, file, line);
}

// Every entry point runs on the device the handle was built on.
namespace {
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};
} // namespace

void apc_set_error_msg(const char *msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }

extern "C" {

void apc_default_params(apc_params *p, int order) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->lo[0] = p->lo[1] = p->lo[2] = 0.0;
  p->L = 1.0;
  p->order = order;
  p->c = 0.35;
  p->max_depth = 6;
  p->ring_min = order == 2 ? 2 : 3;
  p->ring_max = 5;
  p->m_cap = order == 2 ? 40 : 56;
  p->poisson_c = 1.0;
  p->precision = APC_FP64;
}

int apc_build_cloud(const apc_params *p, const double *xyz, int64_t N, hipStream_t stream,
                    apc_cloud **out) {
  if (!out) return APC_EINVAL;
  g_err[0] = 0;
  return apc_build_impl(p, xyz, N, stream, out);
}

int apc_cloud_info(const apc_cloud *c, int64_t *n, int64_t *nb, int64_t *nnz, int64_t *n_opened) {
  if (!c) return APC_EINVAL;
  if (n) *n = c->n;
  if (nb) *nb = c->nb;
  if (nnz) *nnz = c->nnz;
  if (n_opened) *n_opened = c->n_opened;
  return APC_OK;
}

int apc_get_nodes(const apc_cloud *c, int32_t *perm_host, uint64_t *code_host, int32_t *level_host,
                  int32_t *first_host, int32_t *count_host, int32_t *bowner_host,
                  int32_t *bface_host, int32_t *st_off_host, int32_t *st_idx_host,
                  int32_t *ixyz_host) {
  if (!c) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  HIPCHK(hipDeviceSynchronize());
  const int64_t n = c->n, nb = c->nb, ntot = n + nb;
  struct {
    void *dst;
    const void *src;
    size_t bytes;
  } cp[] = {
      {perm_host, c->perm, (size_t)c->N * 4},       {code_host, c->code, (size_t)n * 8},
      {level_host, c->level, (size_t)n * 4},        {first_host, c->first, (size_t)n * 4},
      {count_host, c->count, (size_t)n * 4},        {bowner_host, c->bowner, (size_t)nb * 4},
      {bface_host, c->bface, (size_t)nb * 4},       {st_off_host, c->st_off, (size_t)(n + 1) * 4},
      {st_idx_host, c->st_idx, (size_t)c->nnz * 4}, {ixyz_host, c->crd, (size_t)ntot * 3 * 4},
  };
  for (auto &e : cp)
    if (e.dst && e.bytes) HIPCHK(hipMemcpy(e.dst, e.src, e.bytes, hipMemcpyDeviceToHost));
  return APC_OK;
}

int apc_assemble_gfd(apc_cloud *c, hipStream_t stream) {
  if (!c) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_assemble_impl(c, stream);
}

int apc_get_operator(const apc_cloud *c, double *w_host, double *diag_host) {
  if (!c || !c->assembled) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  HIPCHK(hipDeviceSynchronize());
  const bool mixed = c->P.precision != APC_FP64;
  if (w_host && c->nnz) {
    if (mixed) {
      float *tmp = new float[c->nnz];
      hipError_t e = hipMemcpy(tmp, c->w32, (size_t)c->nnz * 4, hipMemcpyDeviceToHost);
      for (int64_t i = 0; i < c->nnz; i++) w_host[i] = (double)tmp[i];
      delete[] tmp;
      HIPCHK(e);
    } else {
      HIPCHK(hipMemcpy(w_host, c->w64, (size_t)c->nnz * 8, hipMemcpyDeviceToHost));
    }
    // uniform 2-ring rows are not stored: their weights are the shell constants
    // tc_k / h_c^2 over the shells of 6, 12 and 6 entries
    int8_t *rk = new int8_t[c->n];
    int32_t *off = new int32_t[c->n + 1];
    hipError_t e1 = hipMemcpy(rk, c->rkind, (size_t)c->n, hipMemcpyDeviceToHost);
    hipError_t e2 = hipMemcpy(off, c->st_off, (size_t)(c->n + 1) * 4, hipMemcpyDeviceToHost);
    if (e1 == hipSuccess && e2 == hipSuccess) {
      for (int64_t i = 0; i < c->n; i++) {
        if (rk[i] < 0) continue;
        const double hc = c->P.L / (double)(1 << rk[i]);
        for (int j = 0; j < 24; j++) {
          const double w = c->tmpl[j < 6 ? 0 : (j < 18 ? 1 : 2)] * (1.0 / (hc * hc));
          w_host[off[i] + j] = mixed ? (double)(float)w : w;
        }
      }
    }
    delete[] rk;
    delete[] off;
    HIPCHK(e1);
    HIPCHK(e2);
  }
  if (diag_host) HIPCHK(hipMemcpy(diag_host, c->diag, (size_t)c->n * 8, hipMemcpyDeviceToHost));
  return APC_OK;
}

int apc_get_density_operator(const apc_cloud *c, double *bw_host, double *bdiag_host,
                             int8_t *order_host) {
  if (!c || !c->assembled) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  HIPCHK(hipDeviceSynchronize());
  const int64_t n = c->n, nnz = c->nnz;
  const bool mixed = c->P.precision != APC_FP64;
  if (order_host && n > 0) HIPCHK(hipMemcpy(order_host, c->dorder, (size_t)n, hipMemcpyDeviceToHost));
  if (!bw_host && !bdiag_host) return APC_OK;
  std::vector<double> bw((size_t)(nnz > 0 ? nnz : 1)), bd((size_t)(n > 0 ? n : 1));
  if (c->P.order == 4) {
    // B has rows of its own; the diagonal is 1 - sum of the stored row
    if (nnz > 0) {
      if (mixed) {
        std::vector<float> t((size_t)nnz);
        HIPCHK(hipMemcpy(t.data(), c->bw32, (size_t)nnz * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < nnz; i++) bw[i] = (double)t[i];
      } else {
        HIPCHK(hipMemcpy(bw.data(), c->bw64, (size_t)nnz * 8, hipMemcpyDeviceToHost));
      }
    }
  } else {
    // k = 2: b = hs w, diagonal 1 + hs d (hs = h_c^2 mu_2 / 2); hscale 0 is the identity
    // row, hscale < 0 an explicit row (dwx, a kernel reaching past a wall) with
    // diagonal 1 - sum b
    std::vector<double> hs((size_t)(n > 0 ? n : 1)), d((size_t)(n > 0 ? n : 1));
    APCCHK(apc_get_operator(c, bw.data(), d.data()));
    if (n > 0) HIPCHK(hipMemcpy(hs.data(), c->hscale, (size_t)n * 8, hipMemcpyDeviceToHost));
    std::vector<double> dx;
    if (c->dwx && nnz > 0) {
      dx.resize((size_t)nnz);
      HIPCHK(hipMemcpy(dx.data(), c->dwx, (size_t)nnz * 8, hipMemcpyDeviceToHost));
    }
    std::vector<int32_t> off((size_t)n + 1);
    HIPCHK(hipMemcpy(off.data(), c->st_off, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; i++) {
      if (hs[i] < 0.0) {
        double sum = 0.0;
        for (int32_t e = off[i]; e < off[i + 1]; e++) {
          bw[e] = dx[e];
          sum += dx[e];
        }
        bd[i] = 1.0 - sum;
      } else {
        for (int32_t e = off[i]; e < off[i + 1]; e++) bw[e] *= hs[i];
        bd[i] = 1.0 + hs[i] * d[i];
      }
    }
  }
  if (c->P.order == 4) {
    std::vector<int32_t> off((size_t)n + 1);
    HIPCHK(hipMemcpy(off.data(), c->st_off, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; i++) {
      double sum = 0.0;
      for (int32_t e = off[i]; e < off[i + 1]; e++) sum += bw[e];
      bd[i] = 1.0 - sum;
    }
  }
  if (bw_host && nnz > 0) memcpy(bw_host, bw.data(), (size_t)nnz * 8);
  if (bdiag_host && n > 0) memcpy(bdiag_host, bd.data(), (size_t)n * 8);
  return APC_OK;
}

int apc_get_node_orders(const apc_cloud *c, int8_t *order_host) {
  if (!c || !order_host) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  if (c->n > 0) HIPCHK(hipMemcpy(order_host, c->rorder, (size_t)c->n, hipMemcpyDeviceToHost));
  return APC_OK;
}

int apc_operator_boxes(const apc_cloud *c, int64_t *n_boxed) {
  if (!c || !n_boxed) return APC_EINVAL;
  *n_boxed = c->n_boxes;
  return APC_OK;
}

int apc_operator_info(const apc_cloud *c, int64_t *n_uniform, int64_t *nnz_general,
                      int64_t *sell_entries, int64_t *m_entries, int64_t *staged) {
  if (!c || !c->assembled) return APC_EINVAL;
  if (n_uniform) *n_uniform = c->n_template + c->n_uniform4;
  if (nnz_general) *nnz_general = c->nnz - 24 * c->n_template - 56 * c->n_uniform4;
  if (sell_entries) *sell_entries = c->sl_entries;
  if (m_entries) {
    DeviceGuard g(c->device);
    if (!g.ok) return APC_EHIP;
    std::vector<int32_t> off((size_t)c->n + 1);
    HIPCHK(hipMemcpy(off.data(), c->st_off, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int8_t> rk((size_t)(c->n > 0 ? c->n : 1));
    if (c->n > 0)
      HIPCHK(hipMemcpy(rk.data(), c->P.order == 4 ? c->rkind4 : c->rkind, (size_t)c->n,
                       hipMemcpyDeviceToHost));
    int64_t tot = 0;
    for (int64_t i = 0; i < c->n; i++)
      if (rk[i] < 0) tot += std::min<int64_t>(off[i + 1] - off[i], APC_MLP_OUT - 1);
    *m_entries = tot;
  }
  if (staged) {
    staged[0] = staged[1] = staged[2] = 0;
    staged[3] = c->ucap;
    if (c->ucap > 0 && c->nsl > 0) {
      DeviceGuard g(c->device);
      if (!g.ok) return APC_EHIP;
      std::vector<int32_t> un((size_t)c->nsl), len((size_t)c->nsl);
      HIPCHK(hipMemcpy(un.data(), c->sl_un, un.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(len.data(), c->sl_len, len.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
      for (int64_t s = 0; s < c->nsl; s++)
        if (un[s] > 0) {
          staged[0] += 1;
          staged[1] += un[s];
          staged[2] += (int64_t)len[s] * APC_SLICE;
        }
    }
  }
  return APC_OK;
}

int apc_deposit(apc_cloud *c, const double *q, double *rho_M, double *rho_t, double tol, int maxit,
                apc_stats *st, hipStream_t stream) {
  if (!c || !rho_t || !(tol > 0.0) || maxit < 1) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  if (!c->assembled) return APC_EINVAL;
  double *rm = rho_M;
  if (!rm) HIPCHK(apc_malloc_async((void **)&rm, (size_t)(c->n + c->nb) * sizeof(double), stream));
  int rc = apc_deposit_impl(c, q, rm, stream);
  if (rc == APC_OK) rc = apc_density_solve_impl(c, rm, rho_t, tol, maxit, st, stream);
  if (!rho_M) HIPCHK(apc_free_async(rm, stream));
  return rc;
}

int apc_density_solve(apc_cloud *c, const double *rho_M, double *rho_t, double tol, int maxit,
                      apc_stats *st, hipStream_t stream) {
  if (!c || !rho_M || !rho_t || !(tol > 0.0) || maxit < 1) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_density_solve_impl(c, rho_M, rho_t, tol, maxit, st, stream);
}

int apc_solve(apc_cloud *c, const double *rho_t, const double *gvals, double *phi, double tol,
              int maxit, int precond, apc_stats *st, hipStream_t stream) {
  if (!c || !rho_t || !phi || !(tol > 0.0) || maxit < 1) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_solve_impl(c, rho_t, gvals, phi, tol, maxit, precond, st, stream);
}

int apc_interpolate_force(apc_cloud *c, const double *phi, double *phi_p, double *grad_p,
                          hipStream_t stream) {
  if (!c || !phi || !phi_p || !grad_p) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_interp_impl(c, phi, phi_p, grad_p, stream);
}

int apc_interpolate_force_noalloc(apc_cloud *c, const double *phi, double *phi_p,
                                  double *grad_p, hipStream_t stream) {
  if (!c || !phi || !phi_p || !grad_p) return APC_EINVAL;
  g_err[0] = 0;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_interp_noalloc_impl(c, phi, phi_p, grad_p, stream);
}

int apc_node_derivs(apc_cloud *c, const double *f, double *D, hipStream_t stream) {
  if (!c || !f || !D) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_node_derivs_impl(c, f, D, stream);
}

int apc_apply_operator(apc_cloud *c, const double *f, double *out, hipStream_t stream) {
  if (!c || !f || !out) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_apply_impl(c, f, out, stream);
}

int apc_learn_data(apc_cloud *c, const double *Z, int K, float *feat, float *quad,
                   hipStream_t stream) {
  if (!c || !feat || (Z && (K < 1 || !quad))) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_learn_data_impl(c, Z, Z ? K : 0, feat, quad, stream);
}

int apc_mlp_loss_grad(const float *params, const float *feat, const float *quad,
                      const int32_t *rows, int B, float *loss, float *grad, hipStream_t stream) {
  if (!params || !feat || !quad || !rows || B < 1 || !loss || !grad) return APC_EINVAL;
  return apc_mlp_loss_grad_impl(params, feat, quad, rows, B, loss, grad, stream);
}

int apc_mlp_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                 hipStream_t stream) {
  if (!params || !m || !v || !grad || step < 1 || !(lr > 0.0f)) return APC_EINVAL;
  return apc_mlp_adam_impl(params, m, v, grad, step, lr, stream);
}

int apc_mlp_infer(apc_cloud *c, const float *params, const float *feat, int bf16, float *out,
                  hipStream_t stream) {
  if (!c || !params || !feat || !out || (bf16 != 0 && bf16 != 1)) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_mlp_infer_impl(c, params, feat, bf16, out, stream);
}

int apc_set_learned_precond(apc_cloud *c, const float *params, const double *Z, int K,
                            hipStream_t stream) {
  if (!c || !params || (Z && K < 1)) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_set_learned_impl(c, params, Z, Z ? K : 0, stream);
}

int apc_apply_precond(apc_cloud *c, int precond, const double *in, double *out,
                      hipStream_t stream) {
  if (!c || !in || !out) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  return apc_apply_precond_impl(c, precond, in, out, stream);
}

int apc_push(const apc_params *p, int64_t N, double *xyz, double *vel, const double *grad,
             double kick, double dt, hipStream_t stream) {
  g_err[0] = 0;
  return apc_push_impl(p, N, xyz, vel, grad, kick, dt, stream);
}

int apc_step(const apc_params *p, double *xyz, double *vel, const double *q, int64_t N,
             double kick, double dt, double tol_density, double tol, int maxit, int precond,
             double *phi_p, double *grad_p, apc_step_stats *st_host, hipStream_t stream) {
  g_err[0] = 0;
  return apc_step_impl(p, xyz, vel, q, N, kick, dt, tol_density, tol, maxit, precond, phi_p,
                       grad_p, st_host, stream);
}

int apc_build_batch(const apc_params *p, int count, const double *const *xyz, const int64_t *N,
                    hipStream_t stream, apc_batch **out) {
  if (!p || count < 1 || !xyz || !N || !out) return APC_EINVAL;
  *out = nullptr;
  if (p->order != 2) return APC_EINVAL; // the union carries k = 2 operators only
  if (p->periodic) return APC_EINVAL;   // batches hold bounded domains only
  if (p->kernel != APC_KERNEL_NGP) return APC_EINVAL; // and the NGP deposit
  if (p->mask_level != 0) return APC_EINVAL;           // on the whole box
  for (int c = 0; c < count; c++)
    if (!xyz[c] || N[c] < 1) return APC_EINVAL;
  return apc_build_batch_impl(p, count, xyz, N, stream, out);
}

int apc_batch_info(const apc_batch *b, apc_batch_info_t *info, int64_t *cloud_N,
                   int64_t *cloud_n, int64_t *cloud_nb) {
  if (!b) return APC_EINVAL;
  return apc_batch_info_impl(b, info, cloud_N, cloud_n, cloud_nb);
}

int apc_batch_configure(apc_batch *b, int use_graph, int chunk, int spmv_div) {
  if (!b || use_graph > 1 || chunk > 256 ||
      !(spmv_div <= 0 || spmv_div == 1 || spmv_div == 2 || spmv_div == 4 || spmv_div == 8))
    return APC_EINVAL;
  return apc_batch_configure_impl(b, use_graph, chunk, spmv_div);
}

int apc_batch_tune(apc_batch *b, double tol, int *spmv_div, int *chunk, hipStream_t stream) {
  if (!b || !(tol > 0.0)) return APC_EINVAL;
  return apc_batch_tune_impl(b, tol, spmv_div, chunk, stream);
}

int apc_batch_assemble(apc_batch *b, hipStream_t stream) {
  if (!b) return APC_EINVAL;
  return apc_assemble_gfd(apc_batch_union(b), stream);
}

int apc_batch_deposit(apc_batch *b, const double *q, double *rho_M, double *rho_t, double tol,
                      int maxit, apc_stats *st, hipStream_t stream) {
  if (!b || !rho_t || !(tol > 0.0) || maxit < 1) return APC_EINVAL;
  apc_cloud *u = apc_batch_union(b);
  DeviceGuard g(u->device);
  if (!g.ok) return APC_EHIP;
  double *rm = rho_M;
  if (!rm) HIPCHK(apc_malloc_async((void **)&rm, (size_t)(u->n + u->nb) * sizeof(double), stream));
  const int rc = apc_batch_deposit_impl(b, q, rm, rho_t, tol, maxit, st, stream);
  if (!rho_M) HIPCHK(apc_free_async(rm, stream));
  return rc;
}

int apc_batch_solve(apc_batch *b, const double *rho_t, const double *g, double *phi, double tol,
                    int maxit, int precond, apc_stats *st, hipStream_t stream) {
  if (!b || !rho_t || !phi || !(tol > 0.0) || maxit < 1) return APC_EINVAL;
  DeviceGuard gd(apc_batch_union(b)->device);
  if (!gd.ok) return APC_EHIP;
  return apc_batch_solve_impl(b, rho_t, g, phi, tol, maxit, precond, st, stream);
}

int apc_batch_set_learned_precond(apc_batch *b, const float *params, const double *Z, int K,
                                  hipStream_t stream) {
  if (!b || !params || (Z && K < 1)) return APC_EINVAL;
  DeviceGuard gd(apc_batch_union(b)->device);
  if (!gd.ok) return APC_EHIP;
  return apc_batch_set_learned_impl(b, params, Z, Z ? K : 0, stream);
}

int apc_batch_interpolate_force(apc_batch *b, const double *phi, double *phi_p, double *grad_p,
                                hipStream_t stream) {
  if (!b) return APC_EINVAL;
  return apc_interpolate_force(apc_batch_union(b), phi, phi_p, grad_p, stream);
}

int apc_batch_pipeline(apc_batch *b, const double *q, const double *g, double tol_density,
                       double tol, int maxit, int precond, double *rho_t, double *phi,
                       double *phi_p, double *grad_p, apc_stats *st_density, apc_stats *st,
                       int *graph_used, hipStream_t stream) {
  if (!b || !rho_t || !phi || !phi_p || !grad_p || !(tol > 0.0) || !(tol_density > 0.0) ||
      maxit < 1)
    return APC_EINVAL;
  DeviceGuard gd(apc_batch_union(b)->device);
  if (!gd.ok) return APC_EHIP;
  return apc_batch_pipeline_impl(b, q, g, tol_density, tol, maxit, precond, rho_t, phi, phi_p,
                                 grad_p, st_density, st, graph_used, stream);
}

void apc_batch_destroy(apc_batch *b) {
  if (!b) return;
  DeviceGuard g(apc_batch_union(b)->device);
  apc_destroy_batch_impl(b);
}

int apc_set_diagnostics(apc_cloud *c, int flags) {
  if (!c || flags < 0 || flags > (APC_DIAG_KERNEL_TIMES | APC_DIAG_FP64_RESIDUAL)) return APC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return APC_EHIP;
  c->diag_flags = flags;
  // fourth order, mixed modes: the FP64 reference residual needs the FP64 rows,
  // which the next assembly keeps beside the FP32 ones
  if ((flags & APC_DIAG_FP64_RESIDUAL) && c->P.order == 4 && c->P.precision != APC_FP64 &&
      !c->w64ref)
    HIPCHK(apc_dev_alloc((void **)&c->w64ref, (size_t)(c->nnz > 0 ? c->nnz : 1) * sizeof(double)));
  return APC_OK;
}

void apc_destroy(apc_cloud *c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  apc_free_cloud(c);
}

const char *apc_strerror(int code) {
  switch (code) {
  case APC_OK: return "ok";
  case APC_EINVAL: return "invalid argument";
  case APC_ENOMEM: return "out of device memory";
  case APC_EHIP: return "HIP runtime error";
  case APC_EDOMAIN: return "particle outside the domain";
  case APC_ESTENCIL: return "no acceptable stencil up to ring_max";
  case APC_ENOCONV: return "solver did not converge within maxit";
  default: return "unknown error";
  }
}

const char *apc_last_error(void) { return g_err; }

} // extern "C"

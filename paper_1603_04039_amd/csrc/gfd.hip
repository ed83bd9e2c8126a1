// Weighted least-squares GFD on gfx950 (Sec. 3.1) for k = 2.
//
// Per node: delta_j = y_j - y_0 in integer units, h = max |delta|, xi = delta / h,
// v_j = [x, y, z, x^2/2, xy, xz, y^2/2, yz, z^2/2](xi_j) (a row of V0), Gaussian
// weight W_j = (exp(-r_j^2 / r_max^2) - e^-4) / (1 - e^-4).  The WLS solution of
// min || W (V0 a - df) || is reached through the normal equations
// G a = sum_j W_j^2 v_j df_j with G = sum_j W_j^2 v_j v_j^T (9x9, held in 45
// registers per thread), factored by Cholesky; diag(chol) equals |diag R| of the
// QR of W V0, which gives the rank test.  One thread per node: no cross-lane
// reductions, the stencil's neighbour coordinates are Morton-local gathers.
#include <hip/hip_runtime.h>

#include <cmath>

#include "apc_internal.h"

namespace {

constexpr int P9 = 9;
constexpr int G45 = 45;

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; } // j <= i

__device__ __forceinline__ void mono9(double x, double y, double z, double v[P9]) {
  v[0] = x;
  v[1] = y;
  v[2] = z;
  v[3] = (x * x) * 0.5;
  v[4] = x * y;
  v[5] = x * z;
  v[6] = (y * y) * 0.5;
  v[7] = y * z;
  v[8] = (z * z) * 0.5;
}

struct NodeGeom {
  int32_t c0, c1, c2; // own integer coordinates
  int32_t h;          // max |delta| (integer)
  double r2max;       // r_max^2 (integer units)
};

// stencil neighbour list is nb[0..m) with stride 1
__device__ inline NodeGeom node_geom(const int32_t *nb, int m, const int32_t *__restrict__ crd,
                                     int64_t ntot, int32_t y) {
  NodeGeom g;
  g.c0 = crd[y];
  g.c1 = crd[ntot + y];
  g.c2 = crd[2 * ntot + y];
  int32_t h = 0;
  int64_t r2max = 0;
  for (int j = 0; j < m; j++) {
    const int32_t v = nb[j];
    const int32_t d0 = crd[v] - g.c0, d1 = crd[ntot + v] - g.c1, d2 = crd[2 * ntot + v] - g.c2;
    h = max(h, max(abs(d0), max(abs(d1), abs(d2))));
    const int64_t r2 = (int64_t)d0 * d0 + (int64_t)d1 * d1 + (int64_t)d2 * d2;
    r2max = r2 > r2max ? r2 : r2max;
  }
  g.h = h;
  g.r2max = (double)r2max;
  return g;
}

// row v (9) and squared weight of neighbour v of node y
__device__ __forceinline__ double row_w2(const NodeGeom &g, const int32_t *__restrict__ crd,
                                         int64_t ntot, int32_t v, double vv[P9]) {
  const int32_t d0 = crd[v] - g.c0, d1 = crd[ntot + v] - g.c1, d2 = crd[2 * ntot + v] - g.c2;
  const double hd = (double)g.h;
  mono9((double)d0 / hd, (double)d1 / hd, (double)d2 / hd, vv);
  const double r2 = (double)((int64_t)d0 * d0 + (int64_t)d1 * d1 + (int64_t)d2 * d2);
  const double e4 = 0.018315638888734179; // exp(-4)
  const double W = (exp(-r2 / g.r2max) - e4) / (1.0 - e4);
  return W * W;
}

__device__ inline void gram(const int32_t *nb, int m, const NodeGeom &g,
                            const int32_t *__restrict__ crd, int64_t ntot, double G[G45]) {
#pragma unroll
  for (int k = 0; k < G45; k++) G[k] = 0.0;
  for (int j = 0; j < m; j++) {
    double vv[P9];
    const double w2 = row_w2(g, crd, ntot, nb[j], vv);
#pragma unroll
    for (int a = 0; a < P9; a++) {
      const double wa = w2 * vv[a];
#pragma unroll
      for (int b = 0; b <= a; b++) G[tri(a, b)] += wa * vv[b];
    }
  }
}

// in-place Cholesky G = L L^T (packed lower); returns min/max diag(L) (0 if not SPD)
__device__ inline double cholesky9(double G[G45]) {
  double dmin = 1e300, dmax = 0.0;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < P9; i++) {
#pragma unroll
    for (int j = 0; j <= i; j++) {
      double s = G[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; k++) s -= G[tri(i, k)] * G[tri(j, k)];
      if (i == j) {
        ok = ok && (s > 0.0);
        const double d = sqrt(s > 0.0 ? s : 0.0);
        G[tri(i, i)] = d;
        dmin = fmin(dmin, d);
        dmax = fmax(dmax, d);
      } else {
        const double dj = G[tri(j, j)];
        G[tri(i, j)] = dj > 0.0 ? s / dj : 0.0;
      }
    }
  }
  return (ok && dmax > 0.0) ? dmin / dmax : 0.0;
}

// solve L L^T z = c in place
__device__ inline void chol_solve9(const double L[G45], double z[P9]) {
#pragma unroll
  for (int i = 0; i < P9; i++) {
    double s = z[i];
#pragma unroll
    for (int k = 0; k < i; k++) s -= L[tri(i, k)] * z[k];
    z[i] = s / L[tri(i, i)];
  }
#pragma unroll
  for (int i = P9 - 1; i >= 0; i--) {
    double s = z[i];
#pragma unroll
    for (int k = i + 1; k < P9; k++) s -= L[tri(k, i)] * z[k];
    z[i] = s / L[tri(i, i)];
  }
}

// ---------------------------------------------------------------- rank test (build)
__global__ void __launch_bounds__(APC_BLOCK)
    k_rank9(const int32_t *__restrict__ pending, int64_t np, const int32_t *__restrict__ cand,
            int32_t *__restrict__ m, const int32_t *__restrict__ crd, int64_t ntot) {
  int64_t t = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (t >= np) return;
  const int mm = m[t];
  if (mm <= 0) return;
  const int32_t *nb = cand + t * APC_MAXM;
  const NodeGeom g = node_geom(nb, mm, crd, ntot, pending[t]);
  double G[G45];
  gram(nb, mm, g, crd, ntot, G);
  if (!(cholesky9(G) >= APC_TAU_RANK)) m[t] = 0;
}

// ---------------------------------------------------------------- assembly
// Laplacian row of node y: with c = e_xx + e_yy + e_zz and z = G^{-1} c, the
// weight of neighbour j is W_j^2 (v_j . z) / (h unit)^2 (the V0 columns of the
// second derivatives carry 1/2, so their unknowns are h^2 f_dd); diagonal -sum.
//
// A row whose stencil is the full uniform 2-ring of its own level (24 same-level
// nodes at offsets with L1 norm <= 2 cells) has, by symmetry, the same weights as
// every other such row up to 1/h_c^2: c_k / h_c^2 on the shells r^2 = 1, 2, 4
// (cells), which come first, second and third in the (r^2, index) order.  Those
// rows are stored with the canonical constants (the fit of the canonical
// stencil) and flagged by their level in rkind, so the SpMV reads no weights
// for them.
__global__ void k_canon24(const int32_t *__restrict__ crd, double *__restrict__ tc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t ntot = 25;
  int32_t nb[24];
  for (int j = 0; j < 24; j++) nb[j] = j + 1;
  const NodeGeom g = node_geom(nb, 24, crd, ntot, 0);
  double G[G45];
  gram(nb, 24, g, crd, ntot, G);
  cholesky9(G);
  double z[P9] = {0, 0, 0, 1, 0, 0, 1, 0, 1};
  chol_solve9(G, z);
  const double hp = (double)g.h; // spacing 1, unit 1
  const int pick[3] = {0, 6, 18};
  for (int k = 0; k < 3; k++) {
    double vv[P9];
    const double w2 = row_w2(g, crd, ntot, nb[pick[k]], vv);
    double dotv = 0.0;
    for (int q = 0; q < P9; q++) dotv += vv[q] * z[q];
    tc[k] = w2 * dotv / (hp * hp);
  }
}

template <bool MIXED>
__global__ void __launch_bounds__(APC_BLOCK)
    k_assemble(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
               const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
               int D, double unit, double L, const double *__restrict__ tc,
               double *__restrict__ w64, float *__restrict__ w32, double *__restrict__ diag,
               double *__restrict__ inv_diag, double *__restrict__ hscale,
               int8_t *__restrict__ rkind, int *__restrict__ err) {
  int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int32_t a = st_off[y];
  const int m = st_off[y + 1] - a;
  const int32_t *nb = st_idx + a;
  const int l = level[y];
  const double hc = L / (double)(1 << l);
  const NodeGeom g = node_geom(nb, m, crd, ntot, (int32_t)y);
  // uniform 2-ring of the node's own level?
  bool tmpl = (m == 24);
  if (tmpl) {
    const int32_t sp = 1 << (D - l + 1);
    for (int j = 0; j < 24 && tmpl; j++) {
      const int32_t v = nb[j];
      const int32_t d[3] = {abs(crd[v] - g.c0), abs(crd[ntot + v] - g.c1),
                            abs(crd[2 * ntot + v] - g.c2)};
      int32_t l1 = 0;
      for (int k = 0; k < 3; k++) {
        tmpl = tmpl && (d[k] == 0 || d[k] == sp || d[k] == 2 * sp);
        l1 += d[k];
      }
      tmpl = tmpl && l1 <= 2 * sp;
    }
  }
  double sum = 0.0;
  if (tmpl) {
    const double ih2 = 1.0 / (hc * hc);
    for (int j = 0; j < 24; j++) {
      const double w = tc[j < 6 ? 0 : (j < 18 ? 1 : 2)] * ih2;
      if (MIXED) {
        const float wf = (float)w;
        w32[a + j] = wf;
        sum += (double)wf;
      } else {
        w64[a + j] = w;
        sum += w;
      }
    }
    rkind[y] = (int8_t)l;
  } else {
    double G[G45];
    gram(nb, m, g, crd, ntot, G);
    const double ratio = cholesky9(G);
    if (!(ratio >= APC_TAU_RANK)) atomicOr(err, 1);
    double z[P9] = {0, 0, 0, 1, 0, 0, 1, 0, 1};
    chol_solve9(G, z);
    const double hp = (double)g.h * unit;
    const double inv_h2 = 1.0 / (hp * hp);
    for (int j = 0; j < m; j++) {
      double vv[P9];
      const double w2 = row_w2(g, crd, ntot, nb[j], vv);
      double dotv = 0.0;
#pragma unroll
      for (int k = 0; k < P9; k++) dotv += vv[k] * z[k];
      const double w = w2 * dotv * inv_h2;
      if (MIXED) {
        const float wf = (float)w;
        w32[a + j] = wf;
        sum += (double)wf;
      } else {
        w64[a + j] = w;
        sum += w;
      }
    }
    rkind[y] = -1;
  }
  diag[y] = -sum;
  inv_diag[y] = -1.0 / sum;
  hscale[y] = hc * hc / 24.0;
}

// ---------------------------------------------------------------- derivatives
// d = G^{-1} sum_j W_j^2 v_j (f_j - f_0);  d^alpha f = d_alpha / (h unit)^{|alpha|}
__global__ void __launch_bounds__(APC_BLOCK)
    k_node_derivs(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
                  const int32_t *__restrict__ crd, int64_t ntot, double unit,
                  const double *__restrict__ f, double *__restrict__ D) {
  int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int32_t a = st_off[y];
  const int m = st_off[y + 1] - a;
  const int32_t *nb = st_idx + a;
  const NodeGeom g = node_geom(nb, m, crd, ntot, (int32_t)y);
  double G[G45];
  double rhs[P9];
#pragma unroll
  for (int k = 0; k < G45; k++) G[k] = 0.0;
#pragma unroll
  for (int k = 0; k < P9; k++) rhs[k] = 0.0;
  const double f0 = f[y];
  for (int j = 0; j < m; j++) {
    double vv[P9];
    const int32_t v = nb[j];
    const double w2 = row_w2(g, crd, ntot, v, vv);
    const double df = w2 * (f[v] - f0);
#pragma unroll
    for (int p = 0; p < P9; p++) {
      const double wa = w2 * vv[p];
      rhs[p] += vv[p] * df;
#pragma unroll
      for (int q = 0; q <= p; q++) G[tri(p, q)] += wa * vv[q];
    }
  }
  cholesky9(G);
  chol_solve9(G, rhs);
  const double h1 = 1.0 / ((double)g.h * unit);
  const double h2 = h1 * h1;
#pragma unroll
  for (int k = 0; k < P9; k++) D[y * P9 + k] = rhs[k] * (k < 3 ? h1 : h2);
}

// Taylor polynomial of the particle's leaf node (one thread per sorted particle);
// outputs go to the original particle order.
__global__ void __launch_bounds__(APC_BLOCK)
    k_interp(int64_t N, const double *__restrict__ sxyz, const int32_t *__restrict__ perm,
             const int32_t *__restrict__ pnode, const int32_t *__restrict__ crd, int64_t ntot,
             double lo0, double lo1, double lo2, double unit, const double *__restrict__ phi,
             const double *__restrict__ D, double *__restrict__ phi_p, double *__restrict__ grad) {
  int64_t s = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (s >= N) return;
  const int32_t j = pnode[s];
  const double x = sxyz[s] - (lo0 + unit * (double)crd[j]);
  const double y = sxyz[N + s] - (lo1 + unit * (double)crd[ntot + j]);
  const double z = sxyz[2 * N + s] - (lo2 + unit * (double)crd[2 * ntot + j]);
  const double *d = D + (int64_t)j * P9;
  double mv[P9];
  mono9(x, y, z, mv);
  double v = phi[j];
#pragma unroll
  for (int k = 0; k < P9; k++) v += d[k] * mv[k];
  const double gx = d[0] + d[3] * x + d[4] * y + d[5] * z;
  const double gy = d[1] + d[4] * x + d[6] * y + d[7] * z;
  const double gz = d[2] + d[5] * x + d[7] * y + d[8] * z;
  const int64_t i = perm[s];
  phi_p[i] = v;
  grad[i] = gx;
  grad[N + i] = gy;
  grad[2 * N + i] = gz;
}

} // namespace

int apc_rank_check(const apc_cloud *c, const int32_t *pending, int64_t np, const int32_t *cand,
                   int32_t *m, hipStream_t s) {
  hipLaunchKernelGGL(k_rank9, dim3(grid_for(np)), dim3(APC_BLOCK), 0, s, pending, np, cand, m,
                     c->crd, c->n + c->nb);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_assemble_impl(apc_cloud *c, hipStream_t s) {
  const int64_t n = c->n, ntot = c->n + c->nb;
  const bool mixed = c->P.precision != APC_FP64;
  if (!c->diag) {
    HIPCHK(hipMalloc((void **)&c->diag, (size_t)n * sizeof(double)));
    HIPCHK(hipMalloc((void **)&c->inv_diag, (size_t)n * sizeof(double)));
    HIPCHK(hipMalloc((void **)&c->hscale, (size_t)n * sizeof(double)));
    HIPCHK(hipMalloc((void **)&c->rkind, (size_t)n * sizeof(int8_t)));
    if (mixed)
      HIPCHK(hipMalloc((void **)&c->w32, (size_t)(c->nnz > 0 ? c->nnz : 1) * sizeof(float)));
    else
      HIPCHK(hipMalloc((void **)&c->w64, (size_t)(c->nnz > 0 ? c->nnz : 1) * sizeof(double)));
  }
  // canonical uniform 2-ring (spacing 1) around (4,4,4), sorted by r^2
  int32_t hcrd[3 * 25];
  {
    int k = 1;
    hcrd[0] = hcrd[25] = hcrd[50] = 4;
    for (int r2 = 1; r2 <= 4; r2++)
      for (int dx = -2; dx <= 2; dx++)
        for (int dy = -2; dy <= 2; dy++)
          for (int dz = -2; dz <= 2; dz++) {
            if (dx * dx + dy * dy + dz * dz != r2) continue;
            if (abs(dx) + abs(dy) + abs(dz) > 2) continue;
            hcrd[k] = 4 + dx;
            hcrd[25 + k] = 4 + dy;
            hcrd[50 + k] = 4 + dz;
            k++;
          }
  }
  int32_t *dcrd = nullptr;
  double *dtc = nullptr;
  int *err = nullptr;
  HIPCHK(hipMallocAsync((void **)&dcrd, sizeof(hcrd), s));
  HIPCHK(hipMallocAsync((void **)&dtc, 3 * sizeof(double), s));
  HIPCHK(hipMallocAsync((void **)&err, sizeof(int), s));
  HIPCHK(hipMemcpyAsync(dcrd, hcrd, sizeof(hcrd), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_canon24, dim3(1), dim3(64), 0, s, dcrd, dtc);
  if (mixed)
    hipLaunchKernelGGL(k_assemble<true>, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, n, c->st_off,
                       c->st_idx, c->crd, ntot, c->level, c->P.max_depth, c->unit, c->P.L, dtc,
                       c->w64, c->w32, c->diag, c->inv_diag, c->hscale, c->rkind, err);
  else
    hipLaunchKernelGGL(k_assemble<false>, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, n, c->st_off,
                       c->st_idx, c->crd, ntot, c->level, c->P.max_depth, c->unit, c->P.L, dtc,
                       c->w64, c->w32, c->diag, c->inv_diag, c->hscale, c->rkind, err);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->tmpl, dtc, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipFreeAsync(dcrd, s));
  HIPCHK(hipFreeAsync(dtc, s));
  HIPCHK(hipFreeAsync(err, s));
  apc_free_sell(c);
  APCCHK(apc_build_sell(c, s));
  c->assembled = true;
  return APC_OK;
}

int apc_node_derivs_impl(apc_cloud *c, const double *f, double *D, hipStream_t s) {
  hipLaunchKernelGGL(k_node_derivs, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->st_off,
                     c->st_idx, c->crd, c->n + c->nb, c->unit, f, D);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_interp_impl(apc_cloud *c, const double *phi, double *phi_p, double *grad_p,
                    hipStream_t s) {
  double *D = nullptr;
  HIPCHK(hipMallocAsync((void **)&D, (size_t)c->n * P9 * sizeof(double), s));
  APCCHK(apc_node_derivs_impl(c, phi, D, s));
  hipLaunchKernelGGL(k_interp, dim3(grid_for(c->N)), dim3(APC_BLOCK), 0, s, c->N, c->sxyz, c->perm,
                     c->pnode, c->crd, c->n + c->nb, c->P.lo[0], c->P.lo[1], c->P.lo[2], c->unit,
                     phi, D, phi_p, grad_p);
  HIPCHK(hipGetLastError());
  HIPCHK(hipFreeAsync(D, s));
  return APC_OK;
}

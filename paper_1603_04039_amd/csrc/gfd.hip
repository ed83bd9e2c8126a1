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

template <typename T>
__device__ __forceinline__ void mono9(T x, T y, T z, T v[P9]) {
  v[0] = x;
  v[1] = y;
  v[2] = z;
  v[3] = (x * x) * T(0.5);
  v[4] = x * y;
  v[5] = x * z;
  v[6] = (y * y) * T(0.5);
  v[7] = y * z;
  v[8] = (z * z) * T(0.5);
}

struct NodeGeom {
  int32_t c0, c1, c2; // own integer coordinates
  int32_t S;          // periodic side (0: none): offsets are minimum images
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
  g.S = crd[3 * ntot];
  int32_t h = 0;
  int64_t r2max = 0;
  // loops over the stencil are unrolled by 4 so that four neighbours' coordinate
  // gathers are in flight together (the loads of a neighbour depend on its index)
#pragma unroll 4
  for (int j = 0; j < m; j++) {
    const int32_t v = nb[j];
    const int32_t d0 = apc_doff(crd[v], g.c0, g.S), d1 = apc_doff(crd[ntot + v], g.c1, g.S),
                  d2 = apc_doff(crd[2 * ntot + v], g.c2, g.S);
    h = max(h, max(abs(d0), max(abs(d1), abs(d2))));
    const int64_t r2 = (int64_t)d0 * d0 + (int64_t)d1 * d1 + (int64_t)d2 * d2;
    r2max = r2 > r2max ? r2 : r2max;
  }
  g.h = h;
  g.r2max = (double)r2max;
  return g;
}

// row v (9) and squared weight of neighbour v of node y
template <typename T>
__device__ __forceinline__ T row_w2(const NodeGeom &g, const int32_t *__restrict__ crd,
                                    int64_t ntot, int32_t v, T vv[P9]) {
  const int32_t d0 = apc_doff(crd[v], g.c0, g.S), d1 = apc_doff(crd[ntot + v], g.c1, g.S),
                d2 = apc_doff(crd[2 * ntot + v], g.c2, g.S);
  const T hd = (T)g.h;
  mono9<T>((T)d0 / hd, (T)d1 / hd, (T)d2 / hd, vv);
  const T r2 = (T)((int64_t)d0 * d0 + (int64_t)d1 * d1 + (int64_t)d2 * d2);
  const T e4 = T(0.018315638888734179); // exp(-4)
  const T W = (exp(-r2 / (T)g.r2max) - e4) / (T(1) - e4);
  return W * W;
}

template <typename T>
__device__ inline void gram(const int32_t *nb, int m, const NodeGeom &g,
                            const int32_t *__restrict__ crd, int64_t ntot, T G[G45]) {
#pragma unroll
  for (int k = 0; k < G45; k++) G[k] = T(0);
#pragma unroll 4
  for (int j = 0; j < m; j++) {
    T vv[P9];
    const T w2 = row_w2<T>(g, crd, ntot, nb[j], vv);
#pragma unroll
    for (int a = 0; a < P9; a++) {
      const T wa = w2 * vv[a];
#pragma unroll
      for (int b = 0; b <= a; b++) G[tri(a, b)] += wa * vv[b];
    }
  }
}

// in-place Cholesky G = L L^T (packed lower); returns min/max diag(L) (0 if not SPD)
template <typename T>
__device__ inline T cholesky9(T G[G45]) {
  T dmin = T(1e30), dmax = T(0);
  bool ok = true;
#pragma unroll
  for (int i = 0; i < P9; i++) {
#pragma unroll
    for (int j = 0; j <= i; j++) {
      T s = G[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; k++) s -= G[tri(i, k)] * G[tri(j, k)];
      if (i == j) {
        ok = ok && (s > T(0));
        const T d = sqrt(s > T(0) ? s : T(0));
        G[tri(i, i)] = d;
        dmin = fmin(dmin, d);
        dmax = fmax(dmax, d);
      } else {
        const T dj = G[tri(j, j)];
        G[tri(i, j)] = dj > T(0) ? s / dj : T(0);
      }
    }
  }
  return (ok && dmax > T(0)) ? dmin / dmax : T(0);
}

// solve L L^T z = c in place
template <typename T>
__device__ inline void chol_solve9(const T L[G45], T z[P9]) {
#pragma unroll
  for (int i = 0; i < P9; i++) {
    T s = z[i];
#pragma unroll
    for (int k = 0; k < i; k++) s -= L[tri(i, k)] * z[k];
    z[i] = s / L[tri(i, i)];
  }
#pragma unroll
  for (int i = P9 - 1; i >= 0; i--) {
    T s = z[i];
#pragma unroll
    for (int k = i + 1; k < P9; k++) s -= L[tri(k, i)] * z[k];
    z[i] = s / L[tri(i, i)];
  }
}

// Laplacian weights of a general row (fit in precision T): z = G^{-1} (e_xx + e_yy + e_zz),
// w_j = W_j^2 (v_j . z) / (h unit)^2.  Returns the R-diagonal ratio.
template <typename T>
__device__ inline T lap_fit(const int32_t *nb, int m, const NodeGeom &g,
                            const int32_t *__restrict__ crd, int64_t ntot, T z[P9]) {
  T G[G45];
  gram<T>(nb, m, g, crd, ntot, G);
  const T ratio = cholesky9<T>(G);
#pragma unroll
  for (int k = 0; k < P9; k++) z[k] = (k == 3 || k == 6 || k == 8) ? T(1) : T(0);
  chol_solve9<T>(G, z);
  return ratio;
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
  gram<double>(nb, mm, g, crd, ntot, G);
  if (!(cholesky9<double>(G) >= APC_TAU_RANK)) m[t] = 0;
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
// rows take the canonical constants (the same fit on the canonical stencil) and
// are flagged by their level in rkind; the SpMV reads no weights for them.
//
// Assembly runs in three passes: k_classify (integer test for the uniform
// 2-ring, canonical rows written), the sliced layout (sell.hip), then k_fit_sell
// with one wavefront per slice, so that cheap uniform slices and general slices
// never share a wavefront and the solver's copy is written coalesced.
__global__ void k_canon24(const int32_t *__restrict__ crd, double *__restrict__ tc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t ntot = 25;
  int32_t nb[24];
  for (int j = 0; j < 24; j++) nb[j] = j + 1;
  const NodeGeom g = node_geom(nb, 24, crd, ntot, 0);
  double z[P9];
  lap_fit<double>(nb, 24, g, crd, ntot, z);
  const double hp = (double)g.h; // spacing 1, unit 1
  const int pick[3] = {0, 6, 18};
  for (int k = 0; k < 3; k++) {
    double vv[P9];
    const double w2 = row_w2<double>(g, crd, ntot, nb[pick[k]], vv);
    double dotv = 0.0;
    for (int q = 0; q < P9; q++) dotv += vv[q] * z[q];
    tc[k] = w2 * dotv / (hp * hp);
  }
}

// Structural test run at build time: is the stencil the full uniform 2-ring of
// the node's own level?  rkind = level if so, else -1.
__global__ void __launch_bounds__(APC_BLOCK)
    k_classify(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
               const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
               int D, int8_t *__restrict__ rkind) {
  int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int32_t a = st_off[y];
  const int m = st_off[y + 1] - a;
  const int l = level[y];
  bool tmpl = (m == 24);
  if (tmpl) {
    const int32_t sp = 1 << (D - l + 1);
    const int32_t c0 = crd[y], c1 = crd[ntot + y], c2 = crd[2 * ntot + y], S = crd[3 * ntot];
    for (int j = 0; j < 24 && tmpl; j++) {
      const int32_t v = st_idx[a + j];
      const int32_t d[3] = {abs(apc_doff(crd[v], c0, S)), abs(apc_doff(crd[ntot + v], c1, S)),
                            abs(apc_doff(crd[2 * ntot + v], c2, S))};
      int32_t l1 = 0;
      for (int k = 0; k < 3; k++) {
        tmpl = tmpl && (d[k] == 0 || d[k] == sp || d[k] == 2 * sp);
        l1 += d[k];
      }
      tmpl = tmpl && l1 <= 2 * sp;
    }
  }
  rkind[y] = tmpl ? (int8_t)l : (int8_t)-1;
}

__global__ void k_zero_u64(unsigned long long *p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

// FP64 fit of a general row: weights into the CSR copy and the slice (FP32 storage
// in the mixed modes), diagonal; returns the R-diagonal ratio.
template <bool MIXED>
__device__ inline double fit64_row(int32_t row, int64_t off, const int32_t *__restrict__ st_off,
                                   const int32_t *__restrict__ st_idx, const int32_t *__restrict__ crd,
                                   int64_t ntot, double unit, double *__restrict__ w64,
                                   float *__restrict__ w32, double *__restrict__ sw64,
                                   float *__restrict__ sw32, double *__restrict__ diag,
                                   double *__restrict__ inv_diag, double &asum) {
  const int32_t a = st_off[row];
  const int m = st_off[row + 1] - a;
  const int32_t *nb = st_idx + a;
  const NodeGeom g = node_geom(nb, m, crd, ntot, row);
  const double hp = (double)g.h * unit;
  const double inv_h2 = 1.0 / (hp * hp);
  double z[P9];
  const double ratio = lap_fit<double>(nb, m, g, crd, ntot, z);
  double sum = 0.0;
  asum = 0.0;
#pragma unroll 4
  for (int j = 0; j < m; j++) {
    double vv[P9];
    const double w2 = row_w2<double>(g, crd, ntot, nb[j], vv);
    double dotv = 0.0;
#pragma unroll
    for (int k = 0; k < P9; k++) dotv += vv[k] * z[k];
    const double w = w2 * dotv * inv_h2;
    const int64_t e = off + (int64_t)j * APC_SLICE;
    if (MIXED) {
      const float wf = (float)w;
      w32[a + j] = wf;
      sw32[e] = wf;
      sum += (double)wf;
      asum += fabs((double)wf);
    } else {
      w64[a + j] = w;
      sw64[e] = w;
      sum += w;
      asum += fabs(w);
    }
  }
  diag[row] = -sum;
  inv_diag[row] = -1.0 / sum;
  return ratio;
}

// Density row of a node whose CIC / TSC kernel reaches past a wall (eq.
// density_linear_system with the moments over Omega, divided by a_0): the FP64 fit
// of the functional sum_alpha (a_alpha / a_0) d^alpha, b_j = W_j^2 (v_j . z), into
// dwx (CSR order).  Returns whether the row meets the stability bound
// sum |b_j| <= theta (1 - sum b_j) (else the caller takes the identity row).
__device__ inline bool density_explicit(int32_t row, int kernel, double hc, double unit,
                                        const double tlo[3], const double thi[3],
                                        const int32_t *__restrict__ st_off,
                                        const int32_t *__restrict__ st_idx,
                                        const int32_t *__restrict__ crd, int64_t ntot,
                                        double *__restrict__ dwx) {
  const int32_t a = st_off[row];
  const int m = st_off[row + 1] - a;
  const int32_t *nb = st_idx + a;
  const NodeGeom g = node_geom(nb, m, crd, ntot, row);
  const double hp = (double)g.h * unit;
  const double a0 = apc_kernel_a0(kernel, tlo, thi);
  // unknowns in the order of mono9: x, y, z, xx, xy, xz, yy, yz, zz
  constexpr int AX[P9] = {1, 0, 0, 2, 1, 1, 0, 0, 0}, AY[P9] = {0, 1, 0, 0, 1, 0, 2, 1, 0},
                AZ[P9] = {0, 0, 1, 0, 0, 1, 0, 1, 2};
  double G[G45], z[P9];
  gram<double>(nb, m, g, crd, ntot, G);
  cholesky9<double>(G);
#pragma unroll
  for (int k = 0; k < P9; k++) z[k] = apc_dens_coef(kernel, AX[k], AY[k], AZ[k], hc, hp, tlo, thi, a0);
  chol_solve9<double>(G, z);
  double sum = 0.0, asum = 0.0;
  for (int j = 0; j < m; j++) {
    double vv[P9];
    const double w2 = row_w2<double>(g, crd, ntot, nb[j], vv);
    double dotv = 0.0;
#pragma unroll
    for (int k = 0; k < P9; k++) dotv += vv[k] * z[k];
    const double b = w2 * dotv;
    dwx[a + j] = b;
    sum += b;
    asum += fabs(b);
  }
  return asum <= APC_THETA_B * (1.0 - sum);
}

// One wavefront per slice of the sliced layout (indices were laid out at build).
// Uniform slices: the rows' diagonal from the canonical shell constants (their
// CSR weights are implied by rkind and are not stored).  General slices: fit
// each row (FP64, or FP32 in the mixed modes), write its weights to the CSR copy
// and to the slice (entry-major, coalesced); padding entries keep weight 0.  In
// the mixed modes a row whose FP32 Cholesky gives min|R_ii|/max|R_ii| <
// APC_TAU_FP32 is refitted in FP64 right away, while its neighbours'
// coordinates are still in cache (a separate refit kernel over a list of such
// rows measured slower: 339 against 284 us on 1.01e6 nodes).
template <bool MIXED>
__global__ void __launch_bounds__(APC_BLOCK)
    k_fit_sell(int64_t nsl, const int32_t *__restrict__ sl_rows, const int32_t *__restrict__ sl_len,
               const int64_t *__restrict__ sl_off, const int32_t *__restrict__ sl_tmpl,
               const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
               const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
               double unit, double L, const double *__restrict__ tc, double *__restrict__ w64,
               float *__restrict__ w32, double *__restrict__ diag, double *__restrict__ inv_diag,
               double *__restrict__ hscale, int8_t *__restrict__ dorder,
               double *__restrict__ sw64, float *__restrict__ sw32,
               int *__restrict__ err, unsigned long long *__restrict__ nfp64, int kernel,
               double S2, double *__restrict__ dwx) {
  const int64_t s = (int64_t)blockIdx.x * (APC_BLOCK / 64) + (threadIdx.x >> 6);
  if (s >= nsl) return;
  const int lane = threadIdx.x & 63;
  const int32_t row = sl_rows[s * APC_SLICE + lane];
  if (row < 0) return;
  const int64_t off = sl_off[s] + lane;
  const double hc = L / (double)(1 << level[row]);
  // a_2 = h_c^2 mu_2 / 2 per axis: mu_2 = 1/12 (NGP), 1/6 (CIC), 1/4 (TSC)
  const double hs = kernel == APC_KERNEL_CIC ? hc * hc / 12.0
                                             : (kernel == APC_KERNEL_TSC ? hc * hc / 8.0 : hc * hc / 24.0);
  double tlo[3], thi[3];
  apc_node_trunc(crd[row], crd[ntot + row], crd[2 * ntot + row], hc / unit, S2, tlo, thi);
  const bool trunc = apc_truncated(kernel, tlo, thi);
  // density row b = hs w (eq. density_linear_system at k = 2), diagonal 1 - hs sum w:
  // kept when hs sum |w| <= theta (1 - hs sum w), else the identity row (hs = 0).
  // A kernel that reaches past a wall has odd and mixed moments: that row is the
  // FP64 fit of its own functional, stored in dwx (hs = -1 marks it).
  auto density_row = [&](double sum, double asum) {
    if (trunc) {
      const bool ok = density_explicit(row, kernel, hc, unit, tlo, thi, st_off, st_idx, crd,
                                       ntot, dwx);
      hscale[row] = ok ? -1.0 : 0.0;
      if (dorder) dorder[row] = ok ? 2 : 0;
      return;
    }
    const bool ok = hs * asum <= APC_THETA_B * (1.0 - hs * sum);
    hscale[row] = ok ? hs : 0.0;
    if (dorder) dorder[row] = ok ? 2 : 0;
  };
  if (sl_tmpl[s]) {
    const double ih2 = 1.0 / (hc * hc);
    double sum = 0.0;
    for (int k = 0; k < 3; k++) {
      const int cnt = k == 1 ? 12 : 6;
      const double w = tc[k] * ih2;
      sum += cnt * (MIXED ? (double)(float)w : w);
    }
    diag[row] = -sum;
    inv_diag[row] = -1.0 / sum;
    density_row(sum, sum); // the shell constants are positive
    return;
  }
  if (!MIXED) {
    double asum;
    const double ratio = fit64_row<false>(row, off, st_off, st_idx, crd, ntot, unit, w64, w32,
                                          sw64, sw32, diag, inv_diag, asum);
    if (!(ratio >= APC_TAU_RANK)) atomicOr(err, 1);
    density_row(-diag[row], asum);
    return;
  }
  const int32_t a = st_off[row];
  const int m = st_off[row + 1] - a;
  const int32_t *nb = st_idx + a;
  const NodeGeom g = node_geom(nb, m, crd, ntot, row);
  const double hp = (double)g.h * unit;
  const double inv_h2 = 1.0 / (hp * hp);
  float z[P9];
  const float ratio = lap_fit<float>(nb, m, g, crd, ntot, z);
  if (!(ratio >= (float)APC_TAU_FP32)) {
    atomicAdd(nfp64, 1ull);
    double asum;
    const double r64 = fit64_row<true>(row, off, st_off, st_idx, crd, ntot, unit, w64, w32, sw64,
                                       sw32, diag, inv_diag, asum);
    if (!(r64 >= APC_TAU_RANK)) atomicOr(err, 1);
    density_row(-diag[row], asum);
    return;
  }
  double sum = 0.0, asum = 0.0;
#pragma unroll 4
  for (int j = 0; j < m; j++) {
    float vv[P9];
    const float w2 = row_w2<float>(g, crd, ntot, nb[j], vv);
    float dotv = 0.f;
#pragma unroll
    for (int k = 0; k < P9; k++) dotv += vv[k] * z[k];
    const float wf = (float)((double)(w2 * dotv) * inv_h2);
    w32[a + j] = wf;
    sw32[off + (int64_t)j * APC_SLICE] = wf;
    sum += (double)wf;
    asum += fabs((double)wf);
  }
  diag[row] = -sum;
  inv_diag[row] = -1.0 / sum;
  density_row(sum, asum);
}

// FP64 reference residual of the mixed modes: r_i = b_i - sum_j w_ij (x_j - x_i)
// with w the FP64 fit of row i (refitted here, the FP32 weights are not used):
// general rows by the FP64 normal equations of the assembly, uniform 2-ring rows
// by the FP64 shell constants (CSR order: 6, 12 and 6 entries at r^2 = 1, 2, 4
// cells).  One thread per row.
__global__ void __launch_bounds__(APC_BLOCK)
    k_resid64(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
              const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
              const int8_t *__restrict__ rkind, double unit, double L,
              const double *__restrict__ tc, const double *__restrict__ b,
              const double *__restrict__ x, double *__restrict__ r) {
  const int64_t row = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (row >= n) return;
  const int32_t a = st_off[row];
  const int m = st_off[row + 1] - a;
  const int32_t *nb = st_idx + a;
  const double xi = x[row];
  double t = 0.0;
  if (rkind[row] >= 0) {
    const double hc = L / (double)(1 << level[row]);
    const double ih2 = 1.0 / (hc * hc);
    for (int j = 0; j < 24; j++) t += tc[j < 6 ? 0 : (j < 18 ? 1 : 2)] * ih2 * (x[nb[j]] - xi);
  } else {
    const NodeGeom g = node_geom(nb, m, crd, ntot, (int32_t)row);
    const double hp = (double)g.h * unit;
    const double inv_h2 = 1.0 / (hp * hp);
    double z[P9];
    lap_fit<double>(nb, m, g, crd, ntot, z);
    for (int j = 0; j < m; j++) {
      double vv[P9];
      const double w2 = row_w2<double>(g, crd, ntot, nb[j], vv);
      double dotv = 0.0;
#pragma unroll
      for (int k = 0; k < P9; k++) dotv += vv[k] * z[k];
      t += w2 * dotv * inv_h2 * (x[nb[j]] - xi);
    }
  }
  r[row] = b[row] - t;
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
    const double w2 = row_w2<double>(g, crd, ntot, v, vv);
    const double df = w2 * (f[v] - f0);
#pragma unroll
    for (int p = 0; p < P9; p++) {
      const double wa = w2 * vv[p];
      rhs[p] += vv[p] * df;
#pragma unroll
      for (int q = 0; q <= p; q++) G[tri(p, q)] += wa * vv[q];
    }
  }
  cholesky9<double>(G);
  chol_solve9<double>(G, rhs);
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
  mono9<double>(x, y, z, mv);
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

// Rank test of candidate stencils: k = 2 clouds by the per-thread Cholesky of the
// 9x9 normal equations; k = 4 clouds (order-4 rows and their order-2 fallback
// rows) by the column-parallel Householder QR (one wavefront per candidate
// stencil), the oracle's algorithm.
int apc_rank_check(apc_cloud *c, int order, const int32_t *pending, int64_t np,
                   const int32_t *cand, int32_t *m, hipStream_t s) {
  if (c->P.order == 4) return apc_rank_check4(c, order == 4 ? 34 : 9, pending, np, cand, m, s);
  hipLaunchKernelGGL(k_rank9, dim3(grid_for(np)), dim3(APC_BLOCK), 0, s, pending, np, cand, m,
                     c->crd, c->n + c->nb);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

// Structural part of the assembly, run by build_cloud: uniform-row flags, the
// sliced layout and every array the assembly writes (so that assembly allocates
// nothing), plus the canonical stencil for the shell constants.
int apc_prepare_operator(apc_cloud *c, hipStream_t s) {
  const int64_t n = c->n, ntot = c->n + c->nb;
  const bool mixed = c->P.precision != APC_FP64;
  HIPCHK(apc_dev_alloc((void **)&c->diag, (size_t)n * sizeof(double)));
  HIPCHK(apc_dev_alloc((void **)&c->inv_diag, (size_t)n * sizeof(double)));
  HIPCHK(apc_dev_alloc((void **)&c->hscale, (size_t)n * sizeof(double)));
  HIPCHK(apc_dev_alloc((void **)&c->dorder, (size_t)(n > 0 ? n : 1) * sizeof(int8_t)));
  HIPCHK(apc_dev_alloc((void **)&c->rkind, (size_t)n * sizeof(int8_t)));
  if (mixed)
    HIPCHK(apc_dev_alloc((void **)&c->w32, (size_t)(c->nnz > 0 ? c->nnz : 1) * sizeof(float)));
  else
    HIPCHK(apc_dev_alloc((void **)&c->w64, (size_t)(c->nnz > 0 ? c->nnz : 1) * sizeof(double)));
  if (c->P.order == 2 && c->P.kernel != APC_KERNEL_NGP) // explicit density rows beside walls
    HIPCHK(apc_dev_alloc((void **)&c->dwx, (size_t)(c->nnz > 0 ? c->nnz : 1) * sizeof(double)));
  if (c->P.order == 2) {
    hipLaunchKernelGGL(k_classify, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, n, c->st_off,
                       c->st_idx, c->crd, ntot, c->level, c->P.max_depth, c->rkind);
    HIPCHK(hipGetLastError());
  } else {
    // k = 4: no uniform 2-ring rows; the uniform 56-node rows are flagged in rkind4
    HIPCHK(hipMemsetAsync(c->rkind, 0xff, (size_t)(n > 0 ? n : 1), s));
    APCCHK(apc_prepare_uniform4(c, s));
  }
  APCCHK(apc_build_sell(c, s));
  if (c->P.order == 4) {
    HIPCHK(apc_dev_alloc((void **)&c->fb_list, (size_t)(n > 0 ? n : 1) * sizeof(int32_t)));
    const size_t nz = (size_t)(c->nnz > 0 ? c->nnz : 1), ne = (size_t)(c->sl_entries > 0 ? c->sl_entries : 1);
    if (mixed) {
      HIPCHK(apc_dev_alloc((void **)&c->bw32, nz * sizeof(float)));
      HIPCHK(apc_dev_alloc((void **)&c->sl_bw32, ne * sizeof(float)));
      HIPCHK(hipMemsetAsync(c->sl_bw32, 0, ne * sizeof(float), s));
    } else {
      HIPCHK(apc_dev_alloc((void **)&c->bw64, nz * sizeof(double)));
      HIPCHK(apc_dev_alloc((void **)&c->sl_bw64, ne * sizeof(double)));
      HIPCHK(hipMemsetAsync(c->sl_bw64, 0, ne * sizeof(double), s));
    }
  }
  // canonical uniform 2-ring (spacing 1) around (4,4,4), sorted by r^2
  int32_t hcrd[3 * 25];
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
  HIPCHK(apc_dev_alloc((void **)&c->scratch, sizeof(apc_asm_scratch)));
  HIPCHK(hipMemsetAsync(c->scratch, 0, sizeof(apc_asm_scratch), s));
  HIPCHK(hipMemcpyAsync(c->scratch->crd, hcrd, sizeof(hcrd), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_canon24, dim3(1), dim3(64), 0, s, c->scratch->crd, c->scratch->tc);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->tmpl, c->scratch->tc, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return APC_OK;
}

// The assembly proper: one kernel, no allocation, no synchronisation.
int apc_assemble_impl(apc_cloud *c, hipStream_t s) {
  const int64_t ntot = c->n + c->nb;
  const bool mixed = c->P.precision != APC_FP64;
  const unsigned gsl = (unsigned)((c->nsl + (APC_BLOCK / 64) - 1) / (APC_BLOCK / 64));
  c->learned = false; // M depends on the assembled rows: install it again
  if (c->P.order == 4) {
    APCCHK(apc_assemble4(c, s));
    c->assembled = true;
    return APC_OK;
  }
  // the counter is cleared by a kernel (a memset node of a captured graph is what a
  // batch pipeline would record here)
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, &c->scratch->nfp64);
  if (c->nsl > 0) {
    if (mixed) {
      hipLaunchKernelGGL(k_fit_sell<true>, dim3(gsl), dim3(APC_BLOCK), 0, s, c->nsl, c->sl_rows,
                         c->sl_len, c->sl_off, c->sl_tmpl, c->st_off, c->st_idx, c->crd, ntot,
                         c->level, c->unit, c->P.L, c->scratch->tc, c->w64, c->w32, c->diag,
                         c->inv_diag, c->hscale, c->dorder, c->sl_w64, c->sl_w32,
                         &c->scratch->err, &c->scratch->nfp64, c->P.kernel,
                         c->P.periodic ? 0.0 : c->P.L / c->unit, c->dwx);
    } else {
      hipLaunchKernelGGL(k_fit_sell<false>, dim3(gsl), dim3(APC_BLOCK), 0, s, c->nsl, c->sl_rows,
                         c->sl_len, c->sl_off, c->sl_tmpl, c->st_off, c->st_idx, c->crd, ntot,
                         c->level, c->unit, c->P.L, c->scratch->tc, c->w64, c->w32, c->diag,
                         c->inv_diag, c->hscale, c->dorder, c->sl_w64, c->sl_w32,
                         &c->scratch->err, &c->scratch->nfp64, c->P.kernel,
                         c->P.periodic ? 0.0 : c->P.L / c->unit, c->dwx);
    }
    HIPCHK(hipGetLastError());
  }
  c->assembled = true;
  return APC_OK;
}

int apc_resid64_rows(apc_cloud *c, const double *b, const double *x, double *r, hipStream_t s) {
  if (c->n > 0)
    hipLaunchKernelGGL(k_resid64, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->st_off,
                       c->st_idx, c->crd, c->n + c->nb, c->level, c->rkind, c->unit, c->P.L,
                       (const double *)c->scratch->tc, b, x, r);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_node_derivs_impl(apc_cloud *c, const double *f, double *D, hipStream_t s) {
  if (c->P.order == 4) return apc_node_derivs4(c, f, D, s);
  hipLaunchKernelGGL(k_node_derivs, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->st_off,
                     c->st_idx, c->crd, c->n + c->nb, c->unit, f, D);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

// Interpolation with the caller's derivative buffer D (n x p doubles, p = 9 or
// 34): every row of D is written by the derivative kernel before the particle
// kernel reads it, so D needs no clearing.
int apc_interp_with(apc_cloud *c, const double *phi, double *phi_p, double *grad_p, double *D,
                    hipStream_t s) {
  if (c->P.order == 4) return apc_interp4_with(c, phi, phi_p, grad_p, D, s);
  APCCHK(apc_node_derivs_impl(c, phi, D, s));
  hipLaunchKernelGGL(k_interp, dim3(grid_for(c->N)), dim3(APC_BLOCK), 0, s, c->N, c->sxyz, c->perm,
                     c->pnode, c->crd, c->n + c->nb, c->P.lo[0], c->P.lo[1], c->P.lo[2], c->unit,
                     phi, D, phi_p, grad_p);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_interp_impl(apc_cloud *c, const double *phi, double *phi_p, double *grad_p,
                    hipStream_t s) {
  if (c->P.order == 4) return apc_interp4(c, phi, phi_p, grad_p, s);
  double *D = nullptr;
  HIPCHK(apc_malloc_async((void **)&D, (size_t)(c->n > 0 ? c->n : 1) * P9 * sizeof(double), s));
  APCCHK(apc_interp_with(c, phi, phi_p, grad_p, D, s));
  HIPCHK(apc_free_async(D, s));
  return APC_OK;
}

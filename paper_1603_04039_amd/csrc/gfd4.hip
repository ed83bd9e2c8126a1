// Fourth-order GFD (k = 4, p = 34 unknowns) on gfx950 (Sec. 3.1).  Rows that
// fall back to order 2 (no acceptable order-4 stencil) use the first 9 unknowns,
// which are the order-2 unknowns in the same order.
//
// A 34-unknown fit does not fit one thread's registers, so every k = 4 kernel
// here runs one wavefront per node: lane j holds row j of W V0 (the stencil has
// at most 64 nodes; lanes beyond it hold zero rows), the matrix lives in LDS as
// 34 columns of 64 doubles, and the Householder QR of W V0 reduces each column
// product across the wavefront.  This is the oracle's algorithm (Householder QR,
// rank ratio min|R_ii| / max|R_ii|), so both sides take the same rank decisions.
// The fit stays in FP64 in every precision mode (k = 4 systems are less well
// conditioned); the mixed modes store FP32 weights.
//
// From one factorisation W V0 = Q R:
//   Laplacian row   w_j = W_j (Q R^-T c)_j / h^2,  c = e_xx + e_yy + e_zz
//   density row     b_j = W_j (Q R^-T c_B)_j,       c_B = cell moments a_alpha / h^|alpha|
//                   (eq. density_linear_system; B row sums are 1, so the diagonal
//                   is 1 - sum b and B is applied in difference form)
//   derivatives     h^|alpha| d^alpha f = R^-1 Q^T (W (f_j - f_0))
#include <hip/hip_runtime.h>

#include <cmath>

#include "apc_internal.h"

namespace {

constexpr int P4 = 34;
constexpr int WPB4 = 4; // wavefronts per block
constexpr int LCOL = 64; // LDS column length (one entry per lane)

struct Wave4 {
  double A[P4 * LCOL]; // column-major: A[c * 64 + j]; after QR: R on and above the
                       // diagonal, reflector entries below it
  double vd[P4];       // diagonal entries of the reflectors
  double beta[P4];
  double y[P4];
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wmax_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wmax_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wmin_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
// LDS ordering between lanes of one wavefront
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// multi-index of unknown k in the oracle's order: degree 1..4, then the x power
// descending, then the y power descending
__device__ __forceinline__ void alpha4(int k, int &a, int &b, int &c) {
  int d = 1, base = 0;
  while (base + (d + 1) * (d + 2) / 2 <= k) {
    base += (d + 1) * (d + 2) / 2;
    d++;
  }
  int r = k - base;
  a = d;
  while (r > d - a) { // number of (b, c) pairs for this a is d - a + 1
    r -= d - a + 1;
    a--;
  }
  b = d - a - r;
  c = d - a - b;
}

__device__ __forceinline__ double fact(int a) {
  double f = 1.0;
  for (int i = 2; i <= a; i++) f *= (double)i;
  return f;
}

// xi^alpha / alpha! for the 34 unknowns into column-major LDS (row `lane`), times W
__device__ inline void fill_row(double *A, int lane, double x, double y, double z, double W) {
  double px[5], py[5], pz[5];
  px[0] = py[0] = pz[0] = 1.0;
  for (int e = 1; e <= 4; e++) {
    px[e] = px[e - 1] * x;
    py[e] = py[e - 1] * y;
    pz[e] = pz[e - 1] * z;
  }
  int k = 0;
  for (int d = 1; d <= 4; d++)
    for (int a = d; a >= 0; a--)
      for (int b = d - a; b >= 0; b--) {
        const int c = d - a - b;
        A[k * LCOL + lane] = W * (px[a] / fact(a) * py[b] / fact(b) * pz[c] / fact(c));
        k++;
      }
}

// Geometry of node y's stencil (lane j < m: neighbour j), rows of W V0 into LDS.
// Returns h (integer units); W of the lane's row in *Wl (0 beyond the stencil).
__device__ inline int stencil_rows(Wave4 &S, int lane, const int32_t *nb, int m,
                                   const int32_t *__restrict__ crd, int64_t ntot, int64_t y,
                                   double *Wl) {
  int32_t d0 = 0, d1 = 0, d2 = 0;
  if (lane < m) {
    const int32_t v = nb[lane];
    d0 = crd[v] - crd[y];
    d1 = crd[ntot + v] - crd[ntot + y];
    d2 = crd[2 * ntot + v] - crd[2 * ntot + y];
  }
  const int h = wmax_i(max(abs(d0), max(abs(d1), abs(d2))));
  const double r2 = (double)((int64_t)d0 * d0 + (int64_t)d1 * d1 + (int64_t)d2 * d2);
  const double r2max = wmax_d(r2);
  double W = 0.0;
  if (lane < m) {
    const double e4 = exp(-4.0);
    W = (exp(-r2 / r2max) - e4) / (1.0 - e4);
  }
  *Wl = W;
  const double hd = (double)h;
  if (lane < m)
    fill_row(S.A, lane, (double)d0 / hd, (double)d1 / hd, (double)d2 / hd, W);
  else
    for (int k = 0; k < P4; k++) S.A[k * LCOL + lane] = 0.0;
  wsync();
  return h;
}

// Householder QR of the first pc columns (34, or 9 for an order-2 row) of the
// 64 x 34 matrix in S.A; returns min|R_ii| / max|R_ii|
__device__ inline double wave_qr(Wave4 &S, int lane, int pc) {
  double rmin = INFINITY, rmax = 0.0;
  for (int c = 0; c < pc; c++) {
    double *col = S.A + c * LCOL;
    const double x = lane >= c ? col[lane] : 0.0;
    const double nrm = sqrt(wsum(x * x));
    const double acc = __shfl(x, c, 64);
    double alpha = 0.0, bt = 0.0, v = 0.0;
    if (nrm > 0.0) {
      alpha = acc >= 0.0 ? -nrm : nrm;
      v = lane == c ? x - alpha : x;
      const double vn2 = wsum(v * v);
      bt = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      for (int c2 = c + 1; c2 < pc; c2++) {
        double *cc = S.A + c2 * LCOL;
        const double s = wsum(v * cc[lane]) * bt;
        if (lane >= c) cc[lane] -= s * v;
      }
    }
    if (lane == c) {
      col[lane] = alpha;
      S.vd[c] = v;
      S.beta[c] = bt;
    } else if (lane > c) {
      col[lane] = v;
    }
    rmin = fmin(rmin, fabs(alpha));
    rmax = fmax(rmax, fabs(alpha));
    wsync();
  }
  return rmax > 0.0 ? rmin / rmax : 0.0;
}

// reflector c's entry for this lane
__device__ __forceinline__ double refl(const Wave4 &S, int c, int lane) {
  return lane == c ? S.vd[c] : (lane > c ? S.A[c * LCOL + lane] : 0.0);
}

// u <- Q^T u (forward order of the reflectors); u held one entry per lane
__device__ inline double apply_qt(const Wave4 &S, int lane, int pc, double u) {
  for (int c = 0; c < pc; c++) {
    const double v = refl(S, c, lane);
    const double s = wsum(v * u) * S.beta[c];
    u -= s * v;
  }
  return u;
}
// z <- Q z (reverse order)
__device__ inline double apply_q(const Wave4 &S, int lane, int pc, double z) {
  for (int c = pc - 1; c >= 0; c--) {
    const double v = refl(S, c, lane);
    const double s = wsum(v * z) * S.beta[c];
    z -= s * v;
  }
  return z;
}

// solve R^T y = rhs (lane i < pc holds rhs_i); returns y_i in lane i
__device__ inline double solve_rt(const Wave4 &S, int lane, int pc, double rhs) {
  double ym = 0.0;
  for (int i = 0; i < pc; i++) {
    // R_ki = A[i * 64 + k] for k < i, held in column i
    const double t = wsum(lane < i ? S.A[i * LCOL + lane] * ym : 0.0);
    if (lane == i) ym = (rhs - t) / S.A[i * LCOL + i];
  }
  return ym;
}
// solve R a = u (lane i < pc holds u_i); returns a_i in lane i
__device__ inline double solve_r(const Wave4 &S, int lane, int pc, double u) {
  double am = 0.0;
  for (int i = pc - 1; i >= 0; i--) {
    // R_ik = A[k * 64 + i] for k > i, held in column k
    const double t = wsum((lane > i && lane < pc) ? S.A[lane * LCOL + i] * am : 0.0);
    if (lane == i) am = (u - t) / S.A[i * LCOL + i];
  }
  return am;
}

// ---------------------------------------------------------------- rank test (build)
__global__ void __launch_bounds__(WPB4 * 64)
    k_rank_qr(int pc, const int32_t *__restrict__ pending, int64_t np, const int32_t *__restrict__ cand,
              int32_t *__restrict__ m, const int32_t *__restrict__ crd, int64_t ntot) {
  __shared__ Wave4 SH[WPB4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * WPB4 + wv;
  if (t >= np) return;
  const int mm = m[t];
  if (mm <= 0) return;
  double W;
  stencil_rows(SH[wv], lane, cand + t * APC_MAXM, mm, crd, ntot, pending[t], &W);
  const double ratio = wave_qr(SH[wv], lane, pc);
  bool ok = ratio >= APC_TAU_RANK;
  if (ok && pc == P4) {
    // stability of the order-4 Laplacian row: negative diagonal and off-diagonal
    // weights of total magnitude <= APC_TAU_DOM times it (scale-free, h cancels)
    const double cl = (lane == 3 || lane == 6 || lane == 8) ? 1.0 : 0.0;
    const double yl = solve_rt(SH[wv], lane, pc, cl);
    const double zl = apply_q(SH[wv], lane, pc, lane < pc ? yl : 0.0);
    const double sv = lane < mm ? W * zl : 0.0;
    const double s1 = wsum(sv), s2 = wsum(fabs(sv));
    ok = s1 > 0.0 && s2 <= APC_TAU_DOM * s1;
  }
  if (lane == 0 && !ok) m[t] = 0;
}

// ---------------------------------------------------------------- assembly
// Laplacian and density rows of every node (CSR order); one wavefront per node
template <bool MIXED>
__global__ void __launch_bounds__(WPB4 * 64)
    k_fit4(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
           const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
           const int8_t *__restrict__ rorder, double unit, double L, double *__restrict__ w64,
           float *__restrict__ w32,
           double *__restrict__ bw64, float *__restrict__ bw32, double *__restrict__ diag,
           double *__restrict__ inv_diag, double *__restrict__ hscale, int *__restrict__ err) {
  __shared__ Wave4 SH[WPB4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t y = (int64_t)blockIdx.x * WPB4 + wv;
  if (y >= n) return;
  Wave4 &S = SH[wv];
  const int32_t a0 = st_off[y];
  const int m = st_off[y + 1] - a0;
  double W;
  const int pc = rorder[y] == 4 ? P4 : 9;
  const int h = stencil_rows(S, lane, st_idx + a0, m, crd, ntot, y, &W);
  const double ratio = wave_qr(S, lane, pc);
  if (!(ratio >= APC_TAU_RANK)) {
    if (lane == 0) *err = 1;
    return;
  }
  const double hp = (double)h * unit;
  const double hc = L / (double)(1 << level[y]);
  // right-hand sides: Laplacian (unknowns xx = 3, yy = 6, zz = 8) and the cell moments
  double cl = 0.0, cb = 0.0;
  if (lane < pc) {
    int ax, ay, az;
    alpha4(lane, ax, ay, az);
    cl = (lane == 3 || lane == 6 || lane == 8) ? 1.0 : 0.0;
    if (((ax | ay | az) & 1) == 0) {
      double mom = 1.0;
      const int e[3] = {ax, ay, az};
      for (int d = 0; d < 3; d++) {
        double pw = 1.0;
        for (int q = 0; q < e[d]; q++) pw *= hc / 2.0;
        mom *= pw / (double)(e[d] + 1) / fact(e[d]);
      }
      double hk = 1.0;
      for (int q = 0; q < ax + ay + az; q++) hk *= hp;
      cb = mom / hk;
    }
  }
  const double yl = solve_rt(S, lane, pc, cl);
  const double zl = apply_q(S, lane, pc, lane < pc ? yl : 0.0);
  const double yb = solve_rt(S, lane, pc, cb);
  const double zb = apply_q(S, lane, pc, lane < pc ? yb : 0.0);
  const double wl = lane < m ? W * zl / (hp * hp) : 0.0;
  const double wb = lane < m ? W * zb : 0.0;
  const double sw = wsum(wl);
  if (lane < m) {
    if (MIXED) {
      w32[a0 + lane] = (float)wl;
      bw32[a0 + lane] = (float)wb;
    } else {
      w64[a0 + lane] = wl;
      bw64[a0 + lane] = wb;
    }
  }
  if (lane == 0) {
    diag[y] = -sw;
    inv_diag[y] = -1.0 / sw;
    hscale[y] = hc * hc / 24.0;
  }
}

// CSR weights -> the sliced layout (entry-major; padding entries 0)
template <typename T>
__global__ void __launch_bounds__(APC_BLOCK)
    k_sell_copy(int64_t nsl, const int32_t *__restrict__ sl_rows, const int32_t *__restrict__ sl_len,
                const int64_t *__restrict__ sl_off, const int32_t *__restrict__ st_off,
                const T *__restrict__ w, T *__restrict__ sw) {
  const int64_t s = (int64_t)blockIdx.x * (APC_BLOCK / 64) + (threadIdx.x >> 6);
  if (s >= nsl) return;
  const int lane = threadIdx.x & 63;
  const int32_t row = sl_rows[s * APC_SLICE + lane];
  const int len = sl_len[s];
  const int64_t off = sl_off[s] + lane;
  const int32_t a = row >= 0 ? st_off[row] : 0;
  const int m = row >= 0 ? st_off[row + 1] - a : 0;
  for (int k = 0; k < len; k++) sw[off + (int64_t)k * APC_SLICE] = k < m ? w[a + k] : T(0);
}

// ---------------------------------------------------------------- derivatives
__global__ void __launch_bounds__(WPB4 * 64)
    k_node_derivs4(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
                   const int32_t *__restrict__ crd, int64_t ntot, const int8_t *__restrict__ rorder,
                   double unit,
                   const double *__restrict__ f, double *__restrict__ D) {
  __shared__ Wave4 SH[WPB4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t y = (int64_t)blockIdx.x * WPB4 + wv;
  if (y >= n) return;
  Wave4 &S = SH[wv];
  const int32_t a0 = st_off[y];
  const int m = st_off[y + 1] - a0;
  double W;
  const int pc = rorder[y] == 4 ? P4 : 9;
  const int h = stencil_rows(S, lane, st_idx + a0, m, crd, ntot, y, &W);
  wave_qr(S, lane, pc);
  const double u = lane < m ? W * (f[st_idx[a0 + lane]] - f[y]) : 0.0;
  const double qu = apply_qt(S, lane, pc, u);
  const double ai = solve_r(S, lane, pc, lane < pc ? qu : 0.0);
  if (lane >= pc && lane < P4) D[y * P4 + lane] = 0.0; // order-2 fallback row
  if (lane < pc) {
    int ax, ay, az;
    alpha4(lane, ax, ay, az);
    double hk = 1.0;
    const double hp = (double)h * unit;
    for (int q = 0; q < ax + ay + az; q++) hk *= hp;
    D[y * P4 + lane] = ai / hk;
  }
}

// ---------------------------------------------------------------- interpolation
// phi(p) = phi_j + sum_alpha d^alpha phi_j delta^alpha / alpha!, and its gradient
__global__ void __launch_bounds__(APC_BLOCK)
    k_interp4(int64_t N, const double *__restrict__ sxyz, const int32_t *__restrict__ perm,
              const int32_t *__restrict__ pnode, const int32_t *__restrict__ crd, int64_t ntot,
              double lo0, double lo1, double lo2, double unit, const double *__restrict__ phi,
              const double *__restrict__ D, double *__restrict__ phi_p, double *__restrict__ grad) {
  const int64_t s = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (s >= N) return;
  const int32_t j = pnode[s];
  const double x = sxyz[s] - (lo0 + unit * (double)crd[j]);
  const double y = sxyz[N + s] - (lo1 + unit * (double)crd[ntot + j]);
  const double z = sxyz[2 * N + s] - (lo2 + unit * (double)crd[2 * ntot + j]);
  // q[e] = t^e / e! per coordinate
  double qx[5], qy[5], qz[5];
  qx[0] = qy[0] = qz[0] = 1.0;
  for (int e = 1; e <= 4; e++) {
    qx[e] = qx[e - 1] * x / (double)e;
    qy[e] = qy[e - 1] * y / (double)e;
    qz[e] = qz[e - 1] * z / (double)e;
  }
  const double *d = D + (int64_t)j * P4;
  double v = phi[j], gx = 0.0, gy = 0.0, gz = 0.0;
  int k = 0;
  for (int deg = 1; deg <= 4; deg++)
    for (int a = deg; a >= 0; a--)
      for (int b = deg - a; b >= 0; b--) {
        const int c = deg - a - b;
        const double dk = d[k++];
        v += dk * qx[a] * qy[b] * qz[c];
        // d/dx (x^a / a!) = x^(a-1) / (a-1)!
        if (a > 0) gx += dk * qx[a - 1] * qy[b] * qz[c];
        if (b > 0) gy += dk * qx[a] * qy[b - 1] * qz[c];
        if (c > 0) gz += dk * qx[a] * qy[b] * qz[c - 1];
      }
  const int64_t i = perm[s];
  phi_p[i] = v;
  grad[i] = gx;
  grad[N + i] = gy;
  grad[2 * N + i] = gz;
}

inline unsigned grid4(int64_t count) {
  const int64_t g = (count + WPB4 - 1) / WPB4;
  return (unsigned)(g < 1 ? 1 : g);
}

} // namespace

int apc_rank_check4(const apc_cloud *c, int pk, const int32_t *pending, int64_t np,
                    const int32_t *cand, int32_t *m, hipStream_t s) {
  if (np <= 0) return APC_OK;
  hipLaunchKernelGGL(k_rank_qr, dim3(grid4(np)), dim3(WPB4 * 64), 0, s, pk, pending, np, cand, m,
                     c->crd, c->n + c->nb);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_assemble4(apc_cloud *c, hipStream_t s) {
  const int64_t n = c->n, ntot = c->n + c->nb;
  const bool mixed = c->P.precision != APC_FP64;
  HIPCHK(hipMemsetAsync(&c->scratch->err, 0, sizeof(int), s));
  HIPCHK(hipMemsetAsync(&c->scratch->nfp64, 0, sizeof(unsigned long long), s));
  if (n > 0) {
    if (mixed)
      hipLaunchKernelGGL(k_fit4<true>, dim3(grid4(n)), dim3(WPB4 * 64), 0, s, n, c->st_off, c->st_idx,
                         c->crd, ntot, c->level, c->rorder, c->unit, c->P.L, c->w64, c->w32, c->bw64, c->bw32,
                         c->diag, c->inv_diag, c->hscale, &c->scratch->err);
    else
      hipLaunchKernelGGL(k_fit4<false>, dim3(grid4(n)), dim3(WPB4 * 64), 0, s, n, c->st_off, c->st_idx,
                         c->crd, ntot, c->level, c->rorder, c->unit, c->P.L, c->w64, c->w32, c->bw64, c->bw32,
                         c->diag, c->inv_diag, c->hscale, &c->scratch->err);
    HIPCHK(hipGetLastError());
  }
  if (c->nsl > 0) {
    const unsigned g = (unsigned)((c->nsl + (APC_BLOCK / 64) - 1) / (APC_BLOCK / 64));
    if (mixed) {
      hipLaunchKernelGGL(k_sell_copy<float>, dim3(g), dim3(APC_BLOCK), 0, s, c->nsl, c->sl_rows,
                         c->sl_len, c->sl_off, c->st_off, (const float *)c->w32, c->sl_w32);
      hipLaunchKernelGGL(k_sell_copy<float>, dim3(g), dim3(APC_BLOCK), 0, s, c->nsl, c->sl_rows,
                         c->sl_len, c->sl_off, c->st_off, (const float *)c->bw32, c->sl_bw32);
    } else {
      hipLaunchKernelGGL(k_sell_copy<double>, dim3(g), dim3(APC_BLOCK), 0, s, c->nsl, c->sl_rows,
                         c->sl_len, c->sl_off, c->st_off, (const double *)c->w64, c->sl_w64);
      hipLaunchKernelGGL(k_sell_copy<double>, dim3(g), dim3(APC_BLOCK), 0, s, c->nsl, c->sl_rows,
                         c->sl_len, c->sl_off, c->st_off, (const double *)c->bw64, c->sl_bw64);
    }
    HIPCHK(hipGetLastError());
  }
  return APC_OK;
}

int apc_node_derivs4(apc_cloud *c, const double *f, double *D, hipStream_t s) {
  if (c->n > 0)
    hipLaunchKernelGGL(k_node_derivs4, dim3(grid4(c->n)), dim3(WPB4 * 64), 0, s, c->n, c->st_off,
                       c->st_idx, c->crd, c->n + c->nb, (const int8_t *)c->rorder, c->unit, f, D);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_interp4(apc_cloud *c, const double *phi, double *phi_p, double *grad_p, hipStream_t s) {
  double *D = nullptr;
  HIPCHK(hipMallocAsync((void **)&D, (size_t)(c->n > 0 ? c->n : 1) * P4 * sizeof(double), s));
  APCCHK(apc_node_derivs4(c, phi, D, s));
  hipLaunchKernelGGL(k_interp4, dim3(grid_for(c->N)), dim3(APC_BLOCK), 0, s, c->N, c->sxyz, c->perm,
                     c->pnode, c->crd, c->n + c->nb, c->P.lo[0], c->P.lo[1], c->P.lo[2], c->unit,
                     phi, D, phi_p, grad_p);
  HIPCHK(hipGetLastError());
  HIPCHK(hipFreeAsync(D, s));
  return APC_OK;
}

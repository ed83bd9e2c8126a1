// Fourth-order GFD (k = 4, p = 34 unknowns) on gfx950 (Sec. 3.1).  Rows that
// fall back to order 2 (no acceptable order-4 stencil) use the first 9 unknowns,
// which are the order-2 unknowns in the same order.
//
// A 34-unknown fit does not fit one thread's registers, so every k = 4 kernel
// here runs one wavefront per node (the stencil has at most 64 nodes).  Lane j
// builds row j of W V0 and stores it into LDS column-major; then lane c takes
// column c into registers and the Householder QR runs column-parallel: at step
// k lane k forms the reflector of its column and publishes it in LDS, and every
// lane c > k applies it to its own column with a lane-local dot product, so the
// factorisation needs no cross-lane reduction.  This is the oracle's algorithm
// (Householder QR, rank ratio min|R_ii| / max|R_ii|), so both sides take the
// same rank decisions; the lane-local sums run as four interleaved partial sums
// to shorten the FP64 dependency chains.  The fit
// stays in FP64 in every precision mode (k = 4 systems are less well
// conditioned); the mixed modes store FP32 weights.
//
// From one factorisation W V0 = Q R and u = R^-1 R^-T c (two triangular solves,
// one lane per unknown, each solved value broadcast with readlane):
//   Laplacian row   w_j = W_j (W V0 u)_j / h^2 = W_j (Q R^-T c)_j / h^2,
//                   c = e_xx + e_yy + e_zz
//   density row     b_j = W_j (W V0 u_B)_j,  c_B = cell moments a_alpha / h^|alpha|
//                   (eq. density_linear_system; B row sums are 1, so the diagonal
//                   is 1 - sum b and B is applied in difference form)
//   derivatives     h^|alpha| d^alpha f = R^-1 Q^T (W (f_j - f_0)): the vector
//                   W (f_j - f_0) rides along as one more column of the QR and
//                   comes out multiplied by Q^T.
// (W V0) R^-1 is Q, so the rows need no reflector after the factorisation; the
// triangular solves are backward stable, which keeps the rows within
// kappa(W V0) eps of the Q form.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "apc_internal.h"

namespace {

constexpr int P4 = 34;
constexpr int WPB4 = 4;      // wavefronts per block; the kernels ask for 2 blocks per CU
                             // (2 waves per SIMD, as the LDS allows): measured on the
                             // 8.8e6-node assembly, 0.58 s against 0.81 s at the
                             // register count the compiler picks alone
constexpr int MR = APC_MAXM; // rows of a column held per lane (the stencil cap)
constexpr int LD = 66;       // LDS column stride in doubles (16-byte aligned columns)
constexpr int RC = 8;        // rows per LDS read chunk in the QR update
constexpr int RLD = P4 + 1;  // row stride of R in LDS (odd: conflict-free both ways)

struct Wave4 {
  double A[(P4 + 1) * LD]; // the rows of W V0 column-major (and one extra column)
                           // for the column loads; then R row-major (stride RLD)
  double v[MR];            // the current step's reflector
  double u[2 * P4];        // two solved vectors, broadcast to every lane
  double beta;
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
// x of lane l, in every lane (l is the same in all lanes)
__device__ __forceinline__ double rdlane(double x, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
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

// xi^alpha / alpha! of the 34 unknowns, in the order of alpha4
__device__ __forceinline__ void monos(double x, double y, double z, double (&mo)[P4]) {
  double px[5], py[5], pz[5];
  px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
  for (int e = 1; e <= 4; e++) {
    px[e] = px[e - 1] * x;
    py[e] = py[e - 1] * y;
    pz[e] = pz[e - 1] * z;
  }
  int k = 0;
#pragma unroll
  for (int d = 1; d <= 4; d++)
#pragma unroll
    for (int a = d; a >= 0; a--)
#pragma unroll
      for (int b = d - a; b >= 0; b--) {
        const int c = d - a - b;
        mo[k++] = px[a] / fact(a) * py[b] / fact(b) * pz[c] / fact(c);
      }
}

// Geometry of the lane's stencil node: offset scaled by h, WLS weight W (0 beyond
// the stencil), h in integer units
struct Geo {
  double x, y, z, W;
  int h;
};

// Node y's stencil (lane j < m: neighbour j): rows of W V0 into LDS columns 0..33
// (zero rows beyond the stencil).  The caller synchronises.
__device__ __forceinline__ Geo stencil_rows(Wave4 &S, int lane, const int32_t *nb, int m,
                                   const int32_t *__restrict__ crd, int64_t ntot, int64_t y) {
  int32_t d0 = 0, d1 = 0, d2 = 0;
  if (lane < m) {
    const int32_t v = nb[lane];
    const int32_t S = crd[3 * ntot]; // periodic side (0: none)
    d0 = apc_doff(crd[v], crd[y], S);
    d1 = apc_doff(crd[ntot + v], crd[ntot + y], S);
    d2 = apc_doff(crd[2 * ntot + v], crd[2 * ntot + y], S);
  }
  Geo g;
  g.h = wmax_i(max(abs(d0), max(abs(d1), abs(d2))));
  const double r2 = (double)((int64_t)d0 * d0 + (int64_t)d1 * d1 + (int64_t)d2 * d2);
  const double r2max = wmax_d(r2);
  g.W = 0.0;
  if (lane < m) {
    const double e4 = exp(-4.0);
    g.W = (exp(-r2 / r2max) - e4) / (1.0 - e4);
  }
  const double hd = (double)g.h;
  g.x = (double)d0 / hd;
  g.y = (double)d1 / hd;
  g.z = (double)d2 / hd;
  double mo[P4];
  monos(g.x, g.y, g.z, mo);
#pragma unroll
  for (int k = 0; k < P4; k++) S.A[k * LD + lane] = lane < m ? g.W * mo[k] : 0.0;
  return g;
}

// One Householder step of col_qr on the first LEN rows of the lane's column: the
// rows below are zero after the earlier steps' shifts, so the sums skip exact
// zeros only and the arithmetic (the partial sum of row r is r % 4) is that of a
// step over all rows.
template <int MR, int LEN>
__device__ __forceinline__ void qr_step(Wave4 &S, int lane, int k, int ncol, double (&a)[MR],
                                        double &rd) {
  // a[] = rows k..k+LEN-1 of the lane's column; lane k's reflector:
  // v = a - alpha e_0, alpha = -sign(a_0) ||a||
  double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < LEN; r++) q[r & 3] += a[r] * a[r];
  if (lane == k) {
    const double nrm = sqrt((q[0] + q[1]) + (q[2] + q[3]));
    double alpha = 0.0, bt = 0.0;
    if (nrm > 0.0) {
      alpha = a[0] >= 0.0 ? -nrm : nrm;
      double e[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < LEN; r++) {
        const double v = r == 0 ? a[0] - alpha : a[r];
        e[r & 3] += v * v;
        S.v[r] = v;
      }
      const double vn2 = (e[0] + e[1]) + (e[2] + e[3]);
      bt = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    } else {
#pragma unroll
      for (int r = 0; r < LEN; r++) S.v[r] = 0.0;
    }
    S.beta = bt;
    S.A[k * RLD + k] = alpha;
    rd = alpha;
  }
  wsync();
  // every later column: a -= beta (v . a) v; its new pivot entry is R_k,lane
  if (lane > k && lane < ncol) {
    double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r0 = 0; r0 < LEN; r0 += RC) {
#pragma unroll
      for (int r = r0; r < r0 + RC; r++) d[r & 3] += S.v[r] * a[r];
      __asm__ volatile("" ::: "memory");
    }
    const double sc = ((d[0] + d[1]) + (d[2] + d[3])) * S.beta;
#pragma unroll
    for (int r0 = 0; r0 < LEN; r0 += RC) {
#pragma unroll
      for (int r = r0; r < r0 + RC; r++) a[r] -= sc * S.v[r];
      __asm__ volatile("" ::: "memory");
    }
    S.A[k * RLD + lane] = a[0];
  }
#pragma unroll
  for (int r = 0; r < LEN - 1; r++) a[r] = a[r + 1];
  a[LEN - 1] = 0.0;
  wsync(); // the reflector reads are done before the next step rewrites it
}

// Column-parallel Householder QR of the first pc columns in LDS (column-major,
// stride LD), with columns pc..ncol-1 carried along (they receive Q^T).  Lane
// c < ncol holds column c (its first MR rows: MR >= the stencil size); after step
// k it drops the finished row k, so a[0] is always the pivot row and no step needs
// a row predicate, and steps 8p .. 8p+7 work on the first MR - 8p rows only (the
// rest are zero).  On return R is in LDS row-major with stride RLD (R_ij at
// A[i * RLD + j], i <= j < pc) and row i of Q^T times the extra column c at
// A[i * RLD + c].  Returns min|R_ii| / max|R_ii|.
template <int MR>
__device__ __forceinline__ double col_qr(Wave4 &S, int lane, int pc, int ncol) {
  static_assert(MR % RC == 0 && MR - 32 >= RC, "row chunks");
  double a[MR];
#pragma unroll
  for (int r = 0; r < MR; r++) a[r] = lane < ncol ? S.A[lane * LD + r] : 0.0;
  wsync(); // every column is in registers before R reuses the buffer
  double rd = 0.0;
  int k = 0;
  for (; k < pc && k < 8; k++) qr_step<MR, MR>(S, lane, k, ncol, a, rd);
  for (; k < pc && k < 16; k++) qr_step<MR, MR - 8>(S, lane, k, ncol, a, rd);
  for (; k < pc && k < 24; k++) qr_step<MR, MR - 16>(S, lane, k, ncol, a, rd);
  for (; k < pc && k < 32; k++) qr_step<MR, MR - 24>(S, lane, k, ncol, a, rd);
  for (; k < pc; k++) qr_step<MR, MR - 32>(S, lane, k, ncol, a, rd);
  const double rmin = wmin_d(lane < pc ? fabs(rd) : INFINITY);
  const double rmax = wmax_d(lane < pc ? fabs(rd) : 0.0);
  return rmax > 0.0 ? rmin / rmax : 0.0;
}

// u = R^-1 R^-T rhs for two right-hand sides (lane i < pc holds rhs_i); R in LDS
// row-major.  Returns u_i in lane i (0 in lanes >= pc).
__device__ __forceinline__ void solve_rrt(const Wave4 &S, int lane, int pc, double r1, double r2,
                                          double &u1, double &u2) {
  const double rinv = lane < pc ? 1.0 / S.A[lane * RLD + lane] : 1.0;
  double a1 = r1, a2 = r2, y1 = 0.0, y2 = 0.0;
  // R^T y = rhs: y_i = (rhs_i - sum_{k<i} R_ki y_k) / R_ii
  for (int i = 0; i < pc; i++) {
    const double d = rdlane(rinv, i);
    const double t1 = rdlane(a1, i) * d, t2 = rdlane(a2, i) * d;
    if (lane == i) {
      y1 = t1;
      y2 = t2;
    }
    if (lane > i && lane < pc) {
      const double rij = S.A[i * RLD + lane];
      a1 -= rij * t1;
      a2 -= rij * t2;
    }
  }
  // R u = y: u_j = (y_j - sum_{k>j} R_jk u_k) / R_jj
  a1 = y1;
  a2 = y2;
  u1 = u2 = 0.0;
  for (int j = pc - 1; j >= 0; j--) {
    const double d = rdlane(rinv, j);
    const double t1 = rdlane(a1, j) * d, t2 = rdlane(a2, j) * d;
    if (lane == j) {
      u1 = t1;
      u2 = t2;
    }
    if (lane < j) {
      const double rij = S.A[lane * RLD + j];
      a1 -= rij * t1;
      a2 -= rij * t2;
    }
  }
}

// R u = g (lane i < pc holds g_i); returns u_i in lane i
__device__ __forceinline__ double solve_r(const Wave4 &S, int lane, int pc, double g) {
  const double rinv = lane < pc ? 1.0 / S.A[lane * RLD + lane] : 1.0;
  double a = g, u = 0.0;
  for (int j = pc - 1; j >= 0; j--) {
    const double t = rdlane(a, j) * rdlane(rinv, j);
    if (lane == j) u = t;
    if (lane < j) a -= S.A[lane * RLD + j] * t;
  }
  return u;
}

// (W V0 u)_j of the lane's row j for two vectors u (u_c in lane c < pc), the
// u broadcast through LDS
__device__ __forceinline__ void wv0_times(Wave4 &S, const Geo &g, int lane, int pc, double u1,
                                          double u2, double &z1, double &z2) {
  if (lane < pc) {
    S.u[lane] = u1;
    S.u[P4 + lane] = u2;
  }
  wsync();
  // recompute the monomials here rather than keep the 34 values of the row build
  // live across the factorisation (the asm statements hide that they are equal)
  double x = g.x, y = g.y, z = g.z;
  __asm__ volatile("" : "+v"(x), "+v"(y), "+v"(z));
  double mo[P4];
  monos(x, y, z, mo);
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int c = 0; c < P4; c++)
    if (c < pc) {
      const double a0 = g.W * mo[c];
      s1 += a0 * S.u[c];
      s2 += a0 * S.u[P4 + c];
    }
  z1 = s1;
  z2 = s2;
}

// r^2 (in cells) of entry j of a uniform 56-node stencil in (r^2, index) order
__device__ __forceinline__ int shell4_r2(int j) {
  return j < 6 ? 1 : (j < 18 ? 2 : (j < 26 ? 3 : (j < 32 ? 4 : 5)));
}

// ---------------------------------------------------------------- rank test (build)
// uni >= 0 (order-4 test only): a candidate that is the uniform 56-node stencil
// (entry j at a lattice offset of spacing h/2 with r^2 = shell4_r2(j) spacings;
// the stencil lists candidates by (r^2, index)) takes the decision `uni` of the
// canonical stencil without a QR: its QR inputs (offsets over h, weights) equal the
// canonical ones exactly, up to the order of rows within a shell.  diag (the
// canonical run): ratio, s1, s2 of candidate 0.
template <int MR>
__global__ void __launch_bounds__(WPB4 * 64, 2)
    k_rank_qr(int pc, double tau, const int32_t *__restrict__ pending, int64_t np,
              const int32_t *__restrict__ cand, int32_t *__restrict__ m,
              const int32_t *__restrict__ crd, int64_t ntot, int uni, double *__restrict__ diag) {
  __shared__ Wave4 SH[WPB4];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * WPB4 + wv;
  if (t >= np) return;
  const int mm = m[t];
  if (mm <= 0) return;
  if (uni >= 0 && pc == P4 && mm == 56) {
    const int32_t y = pending[t];
    int32_t d[3] = {0, 0, 0};
    if (lane < 56) {
      const int32_t v = cand[t * APC_MAXM + lane];
      const int32_t S = crd[3 * ntot];
      for (int k = 0; k < 3; k++) d[k] = abs(apc_doff(crd[k * ntot + v], crd[k * ntot + y], S));
    }
    const int32_t h = wmax_i(max(d[0], max(d[1], d[2])));
    const int32_t sp = h >> 1;
    bool ok = true;
    if (lane < 56) {
      int q2 = 0;
      for (int k = 0; k < 3; k++) {
        ok = ok && (d[k] == 0 || d[k] == sp || d[k] == h);
        const int q = d[k] == 0 ? 0 : (d[k] == sp ? 1 : 2);
        q2 += q * q;
      }
      ok = ok && sp > 0 && (h & 1) == 0 && q2 == shell4_r2(lane);
    }
    if (wmax_i(ok ? 0 : 1) == 0) {
      if (lane == 0 && uni == 0) m[t] = 0;
      return;
    }
  }
  Wave4 &S = SH[wv];
  const Geo g = stencil_rows(S, lane, cand + t * APC_MAXM, mm, crd, ntot, pending[t]);
  wsync();
  const double ratio = col_qr<MR>(S, lane, pc, pc);
  bool ok = ratio >= APC_TAU_RANK;
  if (ok && pc == P4) {
    // stability of the order-4 Laplacian row: negative diagonal and off-diagonal
    // weights of total magnitude <= tau times it (scale-free, h cancels)
    const double cl = (lane == 3 || lane == 6 || lane == 8) ? 1.0 : 0.0;
    double u1, u2, z1, z2;
    solve_rrt(S, lane, pc, cl, 0.0, u1, u2);
    wv0_times(S, g, lane, pc, u1, u2, z1, z2);
    const double sv = lane < mm ? g.W * z1 : 0.0;
    const double s1 = wsum(sv), s2 = wsum(fabs(sv));
    ok = s1 > 0.0 && s2 <= tau * s1;
    if (diag && lane == 0) {
      diag[1] = s1;
      diag[2] = s2;
    }
  }
  if (diag && lane == 0) diag[0] = ratio;
  if (lane == 0 && !ok) m[t] = 0;
}

// ---------------------------------------------------------------- assembly
// Kernel moments (eq. density_linear_system) over h^|alpha| for unknown `lane` --
// of the node's own cell (NGP), or of the CIC / TSC kernel over its support inside
// Omega ([tlo, thi] per axis) divided by the mass a0 there -- and the Laplacian's
// right-hand side (unknowns xx = 3, yy = 6, zz = 8)
__device__ __forceinline__ void fit_rhs(int lane, int pc, double hc, double hp, int kernel,
                                        const double *tlo, const double *thi, double a0,
                                        double &cl, double &cb) {
  cl = 0.0;
  cb = 0.0;
  if (lane < pc) {
    int ax, ay, az;
    alpha4(lane, ax, ay, az);
    cl = (lane == 3 || lane == 6 || lane == 8) ? 1.0 : 0.0;
    cb = apc_dens_coef(kernel, ax, ay, az, hc, hp, tlo, thi, a0);
  }
}

// the kernel's support inside Omega for node y (S2 = 0: no walls)
struct Trunc {
  double lo[3], hi[3], a0;
};
__device__ __forceinline__ Trunc node_trunc4(int kernel, const int32_t *__restrict__ crd,
                                             int64_t ntot, int64_t y, double hc, double unit,
                                             double S2) {
  Trunc t;
  apc_node_trunc(crd[y], crd[ntot + y], crd[2 * ntot + y], hc / unit, S2, t.lo, t.hi);
  t.a0 = kernel == APC_KERNEL_NGP ? 1.0 : apc_kernel_a0(kernel, t.lo, t.hi);
  return t;
}

// Writes one node's Laplacian and density rows (lane j: stencil entry j) and its
// diagonal; the density row goes through the stability rule: kept when
// sum |b_j| <= theta (1 - sum b_j), else the order-2 row of the same stencil
// (computed by order2(), which returns it per lane), else the identity row.
template <bool MIXED, typename Order2>
__device__ __forceinline__ void write_rows(int lane, int64_t y, int32_t a0, int m, int pc,
                                           double wl, double wb, double hc, Order2 order2,
                                           double *__restrict__ w64, float *__restrict__ w32,
                                           double *__restrict__ bw64, float *__restrict__ bw32,
                                           double *__restrict__ diag, double *__restrict__ inv_diag,
                                           double *__restrict__ hscale, int8_t *__restrict__ dorder,
                                           double *__restrict__ w64ref) {
  const double sw = wsum(wl);
  auto row_ok = [&](double v) { return wsum(fabs(v)) <= APC_THETA_B * (1.0 - wsum(v)); };
  int dord = pc == P4 ? 4 : 2;
  if (!row_ok(wb)) {
    dord = 0;
    if (pc == P4) {
      wb = order2();
      if (row_ok(wb)) dord = 2;
    }
    if (dord == 0) wb = 0.0;
  }
  if (lane < m) {
    if (MIXED) {
      w32[a0 + lane] = (float)wl;
      bw32[a0 + lane] = (float)wb;
      if (w64ref) w64ref[a0 + lane] = wl; // FP64 rows kept for the reference residual
    } else {
      w64[a0 + lane] = wl;
      bw64[a0 + lane] = wb;
    }
  }
  if (lane == 0) {
    diag[y] = -sw;
    inv_diag[y] = -1.0 / sw;
    hscale[y] = hc * hc / 24.0;
    dorder[y] = (int8_t)dord;
  }
}

// Laplacian and density rows by Householder QR (the oracle's algorithm); one
// wavefront per node.  Runs over the nodes listed in list[0 .. *cnt) (the nodes
// whose normal-equation fit did not converge, see k_fit4n), grid-stride.
template <bool MIXED, int MR>
__global__ void __launch_bounds__(WPB4 * 64, 2)
    k_fit4(const int32_t *__restrict__ list, const unsigned *__restrict__ cnt,
           const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
           const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
           const int8_t *__restrict__ rorder, double unit, double L, double *__restrict__ w64,
           float *__restrict__ w32,
           double *__restrict__ bw64, float *__restrict__ bw32, double *__restrict__ diag,
           double *__restrict__ inv_diag, double *__restrict__ hscale, int8_t *__restrict__ dorder,
           double *__restrict__ w64ref, int *__restrict__ err, int kernel, double S2) {
  __shared__ Wave4 SH[WPB4];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  Wave4 &S = SH[wv];
  const int64_t total = *cnt;
  for (int64_t t = (int64_t)blockIdx.x * WPB4 + wv; t < total; t += (int64_t)gridDim.x * WPB4) {
    const int64_t y = list[t];
    const int32_t a0 = st_off[y];
    const int m = st_off[y + 1] - a0;
    const int pc = rorder[y] == 4 ? P4 : 9;
    const Geo g = stencil_rows(S, lane, st_idx + a0, m, crd, ntot, y);
    wsync();
    const double ratio = col_qr<MR>(S, lane, pc, pc);
    if (!(ratio >= APC_TAU_RANK)) {
      if (lane == 0) *err = 1;
      continue;
    }
    const double hp = (double)g.h * unit;
    const double hc = L / (double)(1 << level[y]);
    const Trunc tr = node_trunc4(kernel, crd, ntot, y, hc, unit, S2);
    double cl, cb;
    fit_rhs(lane, pc, hc, hp, kernel, tr.lo, tr.hi, tr.a0, cl, cb);
    double ul, ub, zl, zb;
    solve_rrt(S, lane, pc, cl, cb, ul, ub);
    wv0_times(S, g, lane, pc, ul, ub, zl, zb);
    const double wl = lane < m ? g.W * zl / (hp * hp) : 0.0;
    const double wb = lane < m ? g.W * zb : 0.0;
    // the order-2 row of the same stencil: the leading 9 columns of the same
    // factorisation, moments of order <= 2 only
    auto order2 = [&]() {
      const double cb2 = lane < 9 ? cb : 0.0;
      double u2, u0, z2, z0;
      solve_rrt(S, lane, 9, cb2, 0.0, u2, u0);
      wv0_times(S, g, lane, 9, u2, u0, z2, z0);
      return lane < m ? g.W * z2 : 0.0;
    };
    write_rows<MIXED>(lane, y, a0, m, pc, wl, wb, hc, order2, w64, w32, bw64, bw32, diag,
                      inv_diag, hscale, dorder, w64ref);
    wsync(); // the next node's rows reuse the LDS
  }
}

// the count of nodes refitted by the QR, as the assembly's n_fp64_rows
__global__ void k_fb_report(const unsigned *cnt, unsigned long long *nfp64) {
  if (threadIdx.x == 0) *nfp64 = *cnt;
}

// ---------------------------------------------------------------- normal equations on MFMA
// The same rows from the normal equations G z = c, G = (W V0)^T (W V0), with
// iterative refinement: A = W V0 (m x pc, one stencil row per lane) is staged in
// LDS column-major; G is formed on the matrix cores (v_mfma_f64_16x16x4f64, 16 x 16
// blocks of G, 4 stencil rows per step; lane l of a block product holds entries
// ((l >> 4) + 4 e, l & 15), e < 4); G = L L^T by Cholesky with one row of G per lane;
// z = G^-1 c, then twice r = c - A^T (A z) (the product A^T y again on the matrix
// cores) and z += G^-1 r.  The rows are w_j = W_j (A z)_j, as from the QR, since
// A G^-1 = Q R^-T.  The normal equations square the condition number of A, the
// refinement brings the rows back to the accuracy of the QR (their error is that
// of the residual, kappa(A) eps); a node whose last correction is not below 1e-13
// of the solution, or whose Cholesky meets a pivot that is not positive, is
// listed for the Householder kernel above instead.
typedef double v4d __attribute__((ext_vector_type(4)));
// wavefronts per block: as many as the 160 KB of LDS per compute unit hold (7 x 21.7 KB
// for stencils of up to 56 nodes, 6 x 24.5 KB up to 64)
template <int MR> constexpr int wpbn() { return MR <= 56 ? 7 : 6; }
constexpr int NREF = 1; // refinement steps

template <int MR>
struct WaveN {
  static constexpr int LDA = MR + 1; // column stride of A (odd: spreads the banks)
  double A[P4 * LDA];                // W V0 column-major; rows m .. MR-1 are zero
  double L[P4 * (P4 + 1) / 2];       // G, then its Cholesky factor: packed lower, row-major
  double y[2 * MR];                  // two stencil-row vectors
  double z[2 * P4];                  // two unknown-space vectors
  double cb[64];                     // one column of L, broadcast
};

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// xi^alpha / alpha! of the 34 unknowns (the order of alpha4), with the factorials
// as constant reciprocals
__device__ __forceinline__ void monos_n(double x, double y, double z, double (&mo)[P4]) {
  constexpr double rf[5] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0};
  double px[5], py[5], pz[5];
  px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
  for (int e = 1; e <= 4; e++) {
    px[e] = px[e - 1] * x;
    py[e] = py[e - 1] * y;
    pz[e] = pz[e - 1] * z;
  }
#pragma unroll
  for (int e = 2; e <= 4; e++) {
    px[e] *= rf[e];
    py[e] *= rf[e];
    pz[e] *= rf[e];
  }
  int k = 0;
#pragma unroll
  for (int d = 1; d <= 4; d++)
#pragma unroll
    for (int a = d; a >= 0; a--)
#pragma unroll
      for (int b = d - a; b >= 0; b--)
        mo[k++] = px[a] * py[b] * pz[d - a - b];
}

// Node y's stencil: rows of W V0 into S.A (lanes < MR)
template <int MR>
__device__ __forceinline__ Geo stencil_rows_n(WaveN<MR> &S, int lane, const int32_t *nb, int m,
                                              const int32_t *__restrict__ crd, int64_t ntot,
                                              int64_t y) {
  int32_t d0 = 0, d1 = 0, d2 = 0;
  if (lane < m) {
    const int32_t v = nb[lane];
    const int32_t S = crd[3 * ntot]; // periodic side (0: none)
    d0 = apc_doff(crd[v], crd[y], S);
    d1 = apc_doff(crd[ntot + v], crd[ntot + y], S);
    d2 = apc_doff(crd[2 * ntot + v], crd[2 * ntot + y], S);
  }
  Geo g;
  g.h = wmax_i(max(abs(d0), max(abs(d1), abs(d2))));
  const double r2 = (double)((int64_t)d0 * d0 + (int64_t)d1 * d1 + (int64_t)d2 * d2);
  const double r2max = wmax_d(r2);
  g.W = 0.0;
  if (lane < m) {
    const double e4 = exp(-4.0);
    g.W = (exp(-r2 / r2max) - e4) / (1.0 - e4);
  }
  const double hd = (double)g.h;
  g.x = (double)d0 / hd;
  g.y = (double)d1 / hd;
  g.z = (double)d2 / hd;
  double mo[P4];
  monos_n(g.x, g.y, g.z, mo);
  if (lane < MR) {
#pragma unroll
    for (int k = 0; k < P4; k++) S.A[k * WaveN<MR>::LDA + lane] = lane < m ? g.W * mo[k] : 0.0;
  }
  return g;
}

// G = A^T A over the first PC columns into S.L (packed lower)
template <int MR, int PC>
__device__ __forceinline__ void gram_mfma(WaveN<MR> &S, int lane) {
  constexpr int NB = (PC + 15) / 16, NP = NB * (NB + 1) / 2, LDA = WaveN<MR>::LDA;
  const int i16 = lane & 15, k4 = lane >> 4;
  v4d acc[NP];
#pragma unroll
  for (int q = 0; q < NP; q++) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (int r0 = 0; r0 < MR; r0 += 4) {
    double a[NB];
#pragma unroll
    for (int I = 0; I < NB; I++) {
      const int col = 16 * I + i16;
      a[I] = col < PC ? S.A[col * LDA + r0 + k4] : 0.0;
    }
    int q = 0;
#pragma unroll
    for (int I = 0; I < NB; I++)
#pragma unroll
      for (int J = I; J < NB; J++, q++)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], a[J], acc[q], 0, 0, 0);
  }
  int q = 0;
#pragma unroll
  for (int I = 0; I < NB; I++)
#pragma unroll
    for (int J = I; J < NB; J++, q++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int row = 16 * I + k4 + 4 * e, col = 16 * J + i16; // entry (row, col) of G
        if (row < PC && col < PC && col >= row) S.L[tri(col, row)] = acc[q][e];
      }
}

// Cholesky G = L L^T with row `lane` of G in g (lanes < PC); on return g holds row
// `lane` of L, rd = 1 / L_lane,lane, S.L the packed factor.  False when a pivot is
// not positive.
template <int MR, int PC>
__device__ __forceinline__ bool cholesky_n(WaveN<MR> &S, int lane, double (&g)[P4], double &rd) {
#pragma unroll
  for (int j = 0; j < P4; j++) g[j] = (j < PC && lane < PC && j <= lane) ? S.L[tri(lane, j)] : 0.0;
  bool ok = true;
  rd = 1.0;
#pragma unroll
  for (int k = 0; k < PC; k++) {
    const double pk = rdlane(g[k], k);
    ok = ok && pk > 0.0;
    const double d = sqrt(pk), inv = 1.0 / d;
    if (lane == k) {
      g[k] = d;
      rd = inv;
    } else if (lane > k) {
      g[k] *= inv;
    }
    S.cb[lane] = g[k];
    wsync();
#pragma unroll
    for (int j = k + 1; j < PC; j++)
      if (lane >= j) g[j] -= g[k] * S.cb[j];
    wsync();
  }
  if (lane < PC)
#pragma unroll
    for (int j = 0; j < PC; j++)
      if (j <= lane) S.L[tri(lane, j)] = g[j];
  wsync();
  return ok;
}

// G z = c for two right-hand sides (lane i < PC holds c0_i, c1_i); returns z in place
template <int MR, int PC>
__device__ __forceinline__ void chol_solve_n(const WaveN<MR> &S, int lane, const double (&g)[P4],
                                             double rd, double &c0, double &c1) {
  // L y = c (columns of L in the lanes' rows)
#pragma unroll
  for (int k = 0; k < PC; k++) {
    const double ik = rdlane(rd, k);
    const double y0 = rdlane(c0, k) * ik, y1 = rdlane(c1, k) * ik;
    if (lane == k) {
      c0 = y0;
      c1 = y1;
    } else if (lane > k) {
      c0 -= g[k] * y0;
      c1 -= g[k] * y1;
    }
  }
  // L^T z = y (row k of L from LDS)
#pragma unroll
  for (int k = PC - 1; k >= 0; k--) {
    const double ik = rdlane(rd, k);
    const double z0 = rdlane(c0, k) * ik, z1 = rdlane(c1, k) * ik;
    if (lane == k) {
      c0 = z0;
      c1 = z1;
    } else if (lane < k) {
      const double lki = S.L[tri(k, lane)];
      c0 -= lki * z0;
      c1 -= lki * z1;
    }
  }
}

// y = A z for two vectors (z in lanes < PC); y into S.y and returned in the lanes
template <int MR, int PC>
__device__ __forceinline__ void a_times_n(WaveN<MR> &S, int lane, double z0, double z1,
                                          double &y0, double &y1) {
  constexpr int LDA = WaveN<MR>::LDA;
  if (lane < PC) {
    S.z[lane] = z0;
    S.z[P4 + lane] = z1;
  }
  wsync();
  double s0 = 0.0, s1 = 0.0;
  if (lane < MR) {
#pragma unroll
    for (int c = 0; c < PC; c++) {
      const double a = S.A[c * LDA + lane];
      s0 += a * S.z[c];
      s1 += a * S.z[P4 + c];
    }
    S.y[lane] = s0;
    S.y[MR + lane] = s1;
  }
  y0 = s0;
  y1 = s1;
  wsync();
}

// A^T y for the two vectors in S.y, on the matrix cores; returned in lanes < PC
template <int MR, int PC>
__device__ __forceinline__ void at_times_n(WaveN<MR> &S, int lane, double &t0, double &t1) {
  constexpr int NB = (PC + 15) / 16, LDA = WaveN<MR>::LDA;
  const int i16 = lane & 15, k4 = lane >> 4;
  v4d acc[NB];
#pragma unroll
  for (int I = 0; I < NB; I++) acc[I] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (int r0 = 0; r0 < MR; r0 += 4) {
    const double b = i16 < 2 ? S.y[i16 * MR + r0 + k4] : 0.0;
#pragma unroll
    for (int I = 0; I < NB; I++) {
      const int col = 16 * I + i16;
      const double a = col < PC ? S.A[col * LDA + r0 + k4] : 0.0;
      acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[I], 0, 0, 0);
    }
  }
#pragma unroll
  for (int I = 0; I < NB; I++)
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int row = 16 * I + k4 + 4 * e; // unknown; the column i16 is the vector
      if (i16 < 2 && row < PC) S.z[i16 * P4 + row] = acc[I][e];
    }
  wsync();
  t0 = lane < PC ? S.z[lane] : 0.0;
  t1 = lane < PC ? S.z[P4 + lane] : 0.0;
  wsync();
}

// z = G^-1 c with NREF refinement steps.  Refinement contracts the error by about
// rho = kappa(G) eps per step, and the last correction d estimates the error it
// removed, so the error left is about rho |d| with rho ~ |d| / |z|: the solve is
// accepted (true) when |d| <= 1e-7 |z| for each right-hand side, which leaves an
// error of at most about 1e-14 |z|.
template <int MR, int PC>
__device__ __forceinline__ bool solve_refined(WaveN<MR> &S, int lane, const double (&g)[P4],
                                              double rd, double c0, double c1, double &z0,
                                              double &z1) {
  z0 = c0;
  z1 = c1;
  chol_solve_n<MR, PC>(S, lane, g, rd, z0, z1);
  bool ok = true;
  for (int it = 0; it < NREF; it++) {
    double y0, y1, t0, t1;
    a_times_n<MR, PC>(S, lane, z0, z1, y0, y1);
    at_times_n<MR, PC>(S, lane, t0, t1);
    double r0 = lane < PC ? c0 - t0 : 0.0, r1 = lane < PC ? c1 - t1 : 0.0;
    chol_solve_n<MR, PC>(S, lane, g, rd, r0, r1);
    if (lane < PC) {
      z0 += r0;
      z1 += r1;
    }
    if (it == NREF - 1) {
      const double d0 = wmax_d(fabs(r0)), d1 = wmax_d(fabs(r1));
      const double m0 = wmax_d(lane < PC ? fabs(z0) : 0.0), m1 = wmax_d(lane < PC ? fabs(z1) : 0.0);
      ok = d0 <= 1e-7 * m0 && d1 <= 1e-7 * m1;
    }
  }
  return ok;
}

// Runs over the rows list[0 .. n) (list null: rows 0 .. n-1), one wavefront per row.
template <bool MIXED, int MR>
__global__ void __launch_bounds__(wpbn<MR>() * 64)
    k_fit4n(int64_t n, const int32_t *__restrict__ list, const int32_t *__restrict__ st_off,
            const int32_t *__restrict__ st_idx,
            const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
            const int8_t *__restrict__ rorder, double unit, double L, double *__restrict__ w64,
            float *__restrict__ w32, double *__restrict__ bw64, float *__restrict__ bw32,
            double *__restrict__ diag, double *__restrict__ inv_diag, double *__restrict__ hscale,
            int8_t *__restrict__ dorder, double *__restrict__ w64ref, int32_t *__restrict__ fb_list,
            unsigned *__restrict__ fb_cnt, int kernel, double S2) {
  constexpr int WPB = wpbn<MR>();
  __shared__ WaveN<MR> SH[WPB];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * WPB + wv;
  if (t >= n) return;
  const int64_t y = list ? (int64_t)list[t] : t;
  WaveN<MR> &S = SH[wv];
  const int32_t a0 = st_off[y];
  const int m = st_off[y + 1] - a0;
  const int pc = rorder[y] == 4 ? P4 : 9;
  const Geo g = stencil_rows_n<MR>(S, lane, st_idx + a0, m, crd, ntot, y);
  wsync();
  const double hp = (double)g.h * unit;
  const double hc = L / (double)(1 << level[y]);
  const Trunc tr = node_trunc4(kernel, crd, ntot, y, hc, unit, S2);
  double cl, cb;
  fit_rhs(lane, pc, hc, hp, kernel, tr.lo, tr.hi, tr.a0, cl, cb);
  double lrow[P4], rd, zl, zb;
  bool ok;
  if (pc == P4) {
    gram_mfma<MR, P4>(S, lane);
    wsync();
    ok = cholesky_n<MR, P4>(S, lane, lrow, rd);
    if (ok) ok = solve_refined<MR, P4>(S, lane, lrow, rd, cl, cb, zl, zb);
  } else {
    gram_mfma<MR, 9>(S, lane);
    wsync();
    ok = cholesky_n<MR, 9>(S, lane, lrow, rd);
    if (ok) ok = solve_refined<MR, 9>(S, lane, lrow, rd, cl, cb, zl, zb);
  }
  if (!ok) { // the Householder kernel takes this node
    if (lane == 0) fb_list[atomicAdd(fb_cnt, 1u)] = (int32_t)y;
    return;
  }
  double yl, yb;
  if (pc == P4)
    a_times_n<MR, P4>(S, lane, zl, zb, yl, yb);
  else
    a_times_n<MR, 9>(S, lane, zl, zb, yl, yb);
  const double wl = lane < m ? g.W * yl / (hp * hp) : 0.0;
  const double wb = lane < m ? g.W * yb : 0.0;
  // the order-2 row of the same stencil: the leading 9 x 9 block of the same
  // Cholesky factor (G's leading block), moments of order <= 2 only
  bool ok2 = true;
  auto order2 = [&]() {
    const double cb2 = lane < 9 ? cb : 0.0;
    double z2, z0, y2, y0;
    ok2 = solve_refined<MR, 9>(S, lane, lrow, rd, cb2, 0.0, z2, z0);
    a_times_n<MR, 9>(S, lane, z2, z0, y2, y0);
    return lane < m ? g.W * y2 : 0.0;
  };
  write_rows<MIXED>(lane, y, a0, m, pc, wl, wb, hc, order2, w64, w32, bw64, bw32, diag, inv_diag,
                    hscale, dorder, w64ref);
  if (!ok2 && lane == 0) fb_list[atomicAdd(fb_cnt, 1u)] = (int32_t)y;
}

// CSR weights -> the sliced layout (entry-major; padding entries 0), one wavefront
// per slice, through an LDS tile of 16 entries x 64 rows: a load instruction reads
// 16 consecutive entries of each of 4 rows (coalesced along the CSR rows), a store
// instruction writes one entry of all 64 rows (coalesced along the slice).
template <typename T>
__global__ void __launch_bounds__(APC_BLOCK)
    k_sell_copy(int64_t nsl, const int32_t *__restrict__ sl_rows, const int32_t *__restrict__ sl_len,
                const int64_t *__restrict__ sl_off, const int32_t *__restrict__ st_off,
                const T *__restrict__ w, T *__restrict__ sw) {
  __shared__ T tile[APC_BLOCK / 64][16][APC_SLICE + 1];
  const int wv = threadIdx.x >> 6;
  const int64_t s = (int64_t)blockIdx.x * (APC_BLOCK / 64) + wv;
  if (s >= nsl) return; // whole wavefronts
  const int lane = threadIdx.x & 63;
  const int kk = lane & 15, rr = lane >> 4;
  // the lane's own row (for the 4 x 16 loads: rows r0 + rr read by shuffles)
  const int32_t row = sl_rows[s * APC_SLICE + lane];
  const int32_t a = row >= 0 ? st_off[row] : 0;
  const int m = row >= 0 ? st_off[row + 1] - a : 0;
  const int len = sl_len[s];
  const int64_t off = sl_off[s];
  for (int k0 = 0; k0 < len; k0 += 16) {
    for (int r0 = 0; r0 < APC_SLICE; r0 += 4) {
      const int r = r0 + rr;
      const int32_t ar = __shfl(a, r, 64), mr = __shfl(m, r, 64);
      const int k = k0 + kk;
      tile[wv][kk][r] = k < mr ? w[ar + k] : T(0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int kn = len - k0 < 16 ? len - k0 : 16;
    for (int q = 0; q < kn; q++) sw[off + (int64_t)(k0 + q) * APC_SLICE + lane] = tile[wv][q][lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---------------------------------------------------------------- uniform 56-node rows

// Structural test run at build time: is the node's stencil (an order-4 row) the
// uniform 56-node stencil of its own level, i.e. the nodes at lattice offsets of
// one cell spacing with r^2 = 1 .. 5 cells (6, 12, 8, 6 and 24 of them, every
// offset with |q_d| <= 2 and |q|_1 <= 3)?  The stencil lists distinct nodes by
// (r^2, index), so shell counts and offsets fix the set.  rkind4 = level if so,
// else -1.
__global__ void __launch_bounds__(APC_BLOCK)
    k_classify4(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
                const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
                const int8_t *__restrict__ rorder, int D, int8_t *__restrict__ rkind4) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int32_t a = st_off[y];
  const int l = level[y];
  bool ok = st_off[y + 1] - a == 56 && rorder[y] == 4;
  if (ok) {
    const int32_t sp = 1 << (D - l + 1);
    const int32_t c0 = crd[y], c1 = crd[ntot + y], c2 = crd[2 * ntot + y], S = crd[3 * ntot];
    for (int j = 0; j < 56 && ok; j++) {
      const int32_t v = st_idx[a + j];
      const int32_t d[3] = {abs(apc_doff(crd[v], c0, S)), abs(apc_doff(crd[ntot + v], c1, S)),
                            abs(apc_doff(crd[2 * ntot + v], c2, S))};
      int q2 = 0;
      for (int k = 0; k < 3; k++) {
        ok = ok && (d[k] == 0 || d[k] == sp || d[k] == 2 * sp);
        const int q = d[k] == 0 ? 0 : (d[k] == sp ? 1 : 2);
        q2 += q * q;
      }
      ok = ok && q2 == shell4_r2(j);
    }
  }
  rkind4[y] = ok ? (int8_t)l : (int8_t)-1;
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_gen_flag(const int8_t *__restrict__ rkind4, int64_t n, int32_t *__restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) f[i] = rkind4[i] < 0 ? 1 : 0;
}
__global__ void __launch_bounds__(APC_BLOCK)
    k_gen_list(const int8_t *__restrict__ rkind4, const int32_t *__restrict__ pos, int64_t n,
               int32_t *__restrict__ list) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n && rkind4[i] < 0) list[pos[i]] = (int32_t)i;
}

// shell constants of the uniform 56-node rows
struct Tmpl4 {
  double tl[5]; // Laplacian at h_c = 1
  double tb[5]; // density row (scale-free)
  double sl;    // sum of the 56 Laplacian weights at h_c = 1
  int dord;     // order of the density row
};
__device__ __forceinline__ double pick5(const double (&t)[5], int k) {
  return k == 0 ? t[0] : (k == 1 ? t[1] : (k == 2 ? t[2] : (k == 3 ? t[3] : t[4])));
}

// Rows of the uniform 56-node nodes from the shell constants (what the fit gives
// them up to rounding): Laplacian weight tl / h_c^2, density weight tb, into the
// CSR copies the fitted rows go to; one wavefront per node.
template <bool MIXED>
__global__ void __launch_bounds__(APC_BLOCK)
    k_fill4(int64_t n, const int8_t *__restrict__ rkind4, const int32_t *__restrict__ st_off,
            Tmpl4 T, double L, double *__restrict__ w64, float *__restrict__ w32,
            double *__restrict__ bw64, float *__restrict__ bw32, double *__restrict__ diag,
            double *__restrict__ inv_diag, double *__restrict__ hscale,
            int8_t *__restrict__ dorder, double *__restrict__ w64ref) {
  const int64_t y = (int64_t)blockIdx.x * (APC_BLOCK / 64) + (threadIdx.x >> 6);
  if (y >= n) return;
  const int l = rkind4[y];
  if (l < 0) return;
  const int lane = threadIdx.x & 63;
  const double hc = L / (double)(1 << l);
  const double ih2 = 1.0 / (hc * hc);
  if (lane < 56) {
    const int k = shell4_r2(lane) - 1;
    const double wl = pick5(T.tl, k) * ih2, wb = pick5(T.tb, k);
    const int64_t e = (int64_t)st_off[y] + lane;
    if (MIXED) {
      w32[e] = (float)wl;
      bw32[e] = (float)wb;
      if (w64ref) w64ref[e] = wl;
    } else {
      w64[e] = wl;
      bw64[e] = wb;
    }
  }
  if (lane == 0) {
    const double sw = T.sl * ih2;
    diag[y] = -sw;
    inv_diag[y] = -1.0 / sw;
    hscale[y] = hc * hc / 24.0;
    dorder[y] = (int8_t)T.dord;
  }
}

// the canonical uniform 56-node stencil: node 0 at (4, 4, 4), nodes 1 .. 56 at the
// offsets of spacing 1 sorted by r^2, one cell of size 1 (L = 1, level 0)
struct Canon4 {
  int32_t crd[3 * 57 + 1]; // then S = 0
  int32_t st_off[2], st_idx[56], level[1], fb_list[1];
  int8_t rorder[1], dorder[1];
  unsigned fb_cnt;
  int err;
  double w64[56], bw64[56], diag[1], inv_diag[1], hscale[1];
};

// the canonical stencil (host): node 0 at (4, 4, 4), nodes 1 .. 56 at the 56
// offsets in (r^2, enumeration) order
static inline void canon4_stencil(Canon4 &h) {
  memset(&h, 0, sizeof(h));
  int k = 1;
  for (int a = 0; a < 3; a++) h.crd[57 * a] = 4;
  for (int r2 = 1; r2 <= 5; r2++)
    for (int dx = -2; dx <= 2; dx++)
      for (int dy = -2; dy <= 2; dy++)
        for (int dz = -2; dz <= 2; dz++) {
          if (dx * dx + dy * dy + dz * dz != r2 || abs(dx) + abs(dy) + abs(dz) > 3) continue;
          h.crd[k] = 4 + dx;
          h.crd[57 + k] = 4 + dy;
          h.crd[114 + k] = 4 + dz;
          k++;
        }
  h.st_off[0] = 0;
  h.st_off[1] = 56;
  for (int j = 0; j < 56; j++) h.st_idx[j] = j + 1;
  h.rorder[0] = 4;
}

// ---------------------------------------------------------------- derivatives
// The least-squares derivatives by the normal equations on the matrix cores: G = A^T
// A (A = W V0, PC columns), c = A^T b with b = W (f_j - f_0), z = G^-1 c, then one
// refinement step with the residual of the least-squares problem itself, z += G^-1
// A^T (b - A z) (semi-normal equations: the step contracts the error of z by about
// kappa(G) eps).  True when the Cholesky pivots are positive and the last correction
// is at most 1e-7 of z.
template <int MR, int PC>
__device__ __forceinline__ bool derivs_ne(WaveN<MR> &S, int lane, double b, double &z) {
  gram_mfma<MR, PC>(S, lane);
  wsync();
  double g[P4], rd;
  if (!cholesky_n<MR, PC>(S, lane, g, rd)) return false;
  if (lane < MR) {
    S.y[lane] = b;
    S.y[MR + lane] = 0.0;
  }
  wsync();
  double c0, c1;
  at_times_n<MR, PC>(S, lane, c0, c1);
  double z0 = c0, z1 = 0.0;
  chol_solve_n<MR, PC>(S, lane, g, rd, z0, z1);
  double y0, y1;
  a_times_n<MR, PC>(S, lane, lane < PC ? z0 : 0.0, 0.0, y0, y1);
  if (lane < MR) {
    S.y[lane] = b - y0;
    S.y[MR + lane] = 0.0;
  }
  wsync();
  double d0, d1;
  at_times_n<MR, PC>(S, lane, d0, d1);
  double e0 = lane < PC ? d0 : 0.0, e1 = 0.0;
  chol_solve_n<MR, PC>(S, lane, g, rd, e0, e1);
  if (lane < PC) z0 += e0;
  const double dm = wmax_d(lane < PC ? fabs(e0) : 0.0);
  const double zm = wmax_d(lane < PC ? fabs(z0) : 0.0);
  z = z0;
  return dm <= 1e-7 * zm;
}

// Derivatives of the rows listed (list null: rows 0 .. n-1), one wavefront per row,
// by derivs_ne; a row it does not accept gets a NaN as its first derivative and is
// taken by k_node_derivs4 (flagged = 1).
template <int MR>
__global__ void __launch_bounds__(wpbn<MR>() * 64)
    k_node_derivs4n(int64_t n, const int32_t *__restrict__ list, const int32_t *__restrict__ st_off,
                    const int32_t *__restrict__ st_idx, const int32_t *__restrict__ crd,
                    int64_t ntot, const int8_t *__restrict__ rorder, double unit,
                    const double *__restrict__ f, double *__restrict__ D) {
  constexpr int WPB = wpbn<MR>();
  __shared__ WaveN<MR> SH[WPB];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * WPB + wv;
  if (t >= n) return;
  const int64_t y = list ? (int64_t)list[t] : t;
  WaveN<MR> &S = SH[wv];
  const int32_t a0 = st_off[y];
  const int m = st_off[y + 1] - a0;
  const int pc = rorder[y] == 4 ? P4 : 9;
  const Geo g = stencil_rows_n<MR>(S, lane, st_idx + a0, m, crd, ntot, y);
  const double b = lane < m ? g.W * (f[st_idx[a0 + lane]] - f[y]) : 0.0;
  wsync();
  double z;
  const bool ok = pc == P4 ? derivs_ne<MR, P4>(S, lane, b, z) : derivs_ne<MR, 9>(S, lane, b, z);
  if (!ok) {
    if (lane == 0) D[y * P4] = __builtin_nan("");
    return;
  }
  if (lane >= pc && lane < P4) D[y * P4 + lane] = 0.0; // order-2 fallback row
  if (lane < pc) {
    int ax, ay, az;
    alpha4(lane, ax, ay, az);
    double hk = 1.0;
    const double hp = (double)g.h * unit;
    for (int q = 0; q < ax + ay + az; q++) hk *= hp;
    D[y * P4 + lane] = z / hk;
  }
}

// The same derivatives by the Householder QR of W V0 (the oracle's route), for the
// rows listed; flagged: only those whose first derivative k_node_derivs4n left NaN.
template <int MR>
__global__ void __launch_bounds__(WPB4 * 64, 2)
    k_node_derivs4(int64_t n, const int32_t *__restrict__ list, const int32_t *__restrict__ st_off,
                   const int32_t *__restrict__ st_idx, const int32_t *__restrict__ crd, int64_t ntot,
                   const int8_t *__restrict__ rorder, double unit,
                   const double *__restrict__ f, double *__restrict__ D, int flagged) {
  __shared__ Wave4 SH[WPB4];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * WPB4 + wv;
  if (t >= n) return;
  const int64_t y = list ? (int64_t)list[t] : t;
  if (flagged && !isnan(D[y * P4])) return;
  Wave4 &S = SH[wv];
  const int32_t a0 = st_off[y];
  const int m = st_off[y + 1] - a0;
  const int pc = rorder[y] == 4 ? P4 : 9;
  const Geo g = stencil_rows(S, lane, st_idx + a0, m, crd, ntot, y);
  // W (f_j - f_0) as column pc, transformed by the QR into Q^T W (f_j - f_0)
  S.A[pc * LD + lane] = lane < m ? g.W * (f[st_idx[a0 + lane]] - f[y]) : 0.0;
  wsync();
  col_qr<MR>(S, lane, pc, pc + 1);
  const double ai = solve_r(S, lane, pc, lane < pc ? S.A[lane * RLD + pc] : 0.0);
  if (lane >= pc && lane < P4) D[y * P4 + lane] = 0.0; // order-2 fallback row
  if (lane < pc) {
    int ax, ay, az;
    alpha4(lane, ax, ay, az);
    double hk = 1.0;
    const double hp = (double)g.h * unit;
    for (int q = 0; q < ax + ay + az; q++) hk *= hp;
    D[y * P4 + lane] = ai / hk;
  }
}

// Derivative operator of the canonical 56-node stencil: C[j][a] = the unknown a of
// the fit of f = e_j (the same QR steps as k_node_derivs4), so that at a uniform
// node d_a = sum_j C[j][a] (f_j - f_0) / hp^|alpha_a|.  One wavefront per j.
__global__ void __launch_bounds__(WPB4 * 64, 2)
    k_canon_derivs4(const int32_t *__restrict__ st_idx, const int32_t *__restrict__ crd,
                    double *__restrict__ C) {
  __shared__ Wave4 SH[WPB4];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int j = blockIdx.x * WPB4 + wv;
  if (j >= 56) return;
  Wave4 &S = SH[wv];
  const Geo g = stencil_rows(S, lane, st_idx, 56, crd, 57, 0);
  S.A[P4 * LD + lane] = lane == j ? g.W : 0.0;
  wsync();
  col_qr<56>(S, lane, P4, P4 + 1);
  const double ai = solve_r(S, lane, P4, lane < P4 ? S.A[lane * RLD + P4] : 0.0);
  if (lane < P4) C[j * P4 + lane] = ai;
}

// Derivatives of the uniform 56-node nodes from the canonical operator, tabulated
// by lattice offset: T[o][a] with o = 25 (q_x + 2) + 5 (q_y + 2) + (q_z + 2) for the
// offset q (in spacings) of a stencil node (the shells' order by node index differs
// from node to node; the offset names the canonical entry).  One thread per node,
// T in LDS; hp = 2 spacings.
__global__ void __launch_bounds__(APC_BLOCK)
    k_derivs_u4(int64_t n, const int8_t *__restrict__ rkind4, const int32_t *__restrict__ st_off,
                const int32_t *__restrict__ st_idx, const int32_t *__restrict__ crd, int64_t ntot,
                int Dmax, double unit, const double *__restrict__ T, const double *__restrict__ f,
                double *__restrict__ D) {
  __shared__ double Ts[125 * P4];
  for (int q = threadIdx.x; q < 125 * P4; q += APC_BLOCK) Ts[q] = T[q];
  __syncthreads();
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int l = rkind4[y];
  if (l < 0) return;
  const int sh = Dmax - l + 1; // spacing 2^sh integer units
  const int32_t a0 = st_off[y];
  const double f0 = f[y];
  const int32_t c0 = crd[y], c1 = crd[ntot + y], c2 = crd[2 * ntot + y], S = crd[3 * ntot];
  double acc[P4];
#pragma unroll
  for (int a = 0; a < P4; a++) acc[a] = 0.0;
  for (int j = 0; j < 56; j++) {
    const int32_t v = st_idx[a0 + j];
    const int o = 25 * ((apc_doff(crd[v], c0, S) >> sh) + 2) +
                  5 * ((apc_doff(crd[ntot + v], c1, S) >> sh) + 2) +
                  ((apc_doff(crd[2 * ntot + v], c2, S) >> sh) + 2);
    const double df = f[v] - f0;
    const double *t = Ts + o * P4;
#pragma unroll
    for (int a = 0; a < P4; a++) acc[a] += t[a] * df;
  }
  const double hp = ldexp(unit, sh + 1);
  double hk[5];
  hk[0] = 1.0;
  for (int q = 1; q <= 4; q++) hk[q] = hk[q - 1] * hp;
#pragma unroll
  for (int a = 0; a < P4; a++) {
    const int deg = a < 3 ? 1 : (a < 9 ? 2 : (a < 19 ? 3 : 4));
    D[y * P4 + a] = acc[a] / hk[deg];
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

// The canonical stencil's order-4 rank and stability test (the same kernel, on the
// canonical stencil): c->uni4_rank = its decision when both margins are wide
// (ratio at least twice the rank bound, s2 / (tau s1) outside [1 - 1e-9, 1 + 1e-9]),
// else -1 (every candidate takes the QR).  Synchronises.
static int rank_uniform4(apc_cloud *c, double tau, hipStream_t s) {
  Canon4 h;
  canon4_stencil(h);
  struct Buf {
    Canon4 cn;
    int32_t pend, m;
    double diag[3];
  };
  Buf hb;
  memset(&hb, 0, sizeof(hb));
  hb.cn = h;
  hb.pend = 0;
  hb.m = 56;
  Buf *d = nullptr;
  HIPCHK(apc_malloc_async((void **)&d, sizeof(Buf), s));
  HIPCHK(hipMemcpyAsync(d, &hb, sizeof(Buf), hipMemcpyHostToDevice, s));
  // the canonical candidate list: nodes 1 .. 56 (cand has the APC_MAXM stride; one row)
  int32_t *cand = nullptr;
  HIPCHK(apc_malloc_async((void **)&cand, APC_MAXM * sizeof(int32_t), s));
  int32_t hc[APC_MAXM];
  for (int j = 0; j < APC_MAXM; j++) hc[j] = j < 56 ? j + 1 : 0;
  HIPCHK(hipMemcpyAsync(cand, hc, sizeof(hc), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_rank_qr<56>, dim3(1), dim3(WPB4 * 64), 0, s, P4, tau,
                     (const int32_t *)&d->pend, (int64_t)1, (const int32_t *)cand, &d->m,
                     (const int32_t *)d->cn.crd, (int64_t)57, -1, d->diag);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(&hb, d, sizeof(Buf), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(apc_free_async(d, s));
  HIPCHK(apc_free_async(cand, s));
  const double ratio = hb.diag[0], s1 = hb.diag[1], s2 = hb.diag[2];
  const bool wide_rank = ratio >= 2.0 * APC_TAU_RANK;
  const double q = s1 > 0.0 ? s2 / (tau * s1) : 0.0;
  const bool wide_dom = s1 > 0.0 && (q < 1.0 - 1e-9 || q > 1.0 + 1e-9);
  c->uni4_rank = (wide_rank && wide_dom) ? (hb.m == 56 ? 1 : 0) : -1;
  return APC_OK;
}

int apc_rank_check4(apc_cloud *c, int pk, const int32_t *pending, int64_t np,
                    const int32_t *cand, int32_t *m, hipStream_t s) {
  if (np <= 0) return APC_OK;
  // stencils hold at most m_cap rows (order-2 fallback: 40): QR over 56 or 64 rows
  const double tau = c->P.tau_dom > 0.0 ? c->P.tau_dom : APC_TAU_DOM;
  if (pk == P4 && c->uni4_rank == -2) APCCHK(rank_uniform4(c, tau, s));
  const int uni = pk == P4 ? c->uni4_rank : -1;
  if (c->P.m_cap <= 56)
    hipLaunchKernelGGL(k_rank_qr<56>, dim3(grid4(np)), dim3(WPB4 * 64), 0, s, pk, tau, pending,
                       np, cand, m, c->crd, c->n + c->nb, uni, (double *)nullptr);
  else
    hipLaunchKernelGGL(k_rank_qr<APC_MAXM>, dim3(grid4(np)), dim3(WPB4 * 64), 0, s, pk, tau,
                       pending, np, cand, m, c->crd, c->n + c->nb, uni, (double *)nullptr);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

// The shell constants of the uniform 56-node rows are the assembly's own fit (FP64
// normal equations, Householder QR if they do not converge) of the canonical
// stencil; by the stencil's cubic symmetry every shell then holds one value (up to
// rounding: checked, the shell mean is kept).  Then the rows are classified and
// the other rows listed for the assembly.  Synchronises.
int apc_prepare_uniform4(apc_cloud *c, hipStream_t s) {
  const int64_t n = c->n;
  HIPCHK(apc_dev_alloc((void **)&c->rkind4, (size_t)(n > 0 ? n : 1)));
  HIPCHK(apc_dev_alloc((void **)&c->gen4, (size_t)(n > 0 ? n : 1) * sizeof(int32_t)));
  c->n_uniform4 = 0;
  c->n_gen4 = n;
  for (double &v : c->tmpl4) v = 0.0;
  c->dorder4 = 0;
  Canon4 h;
  canon4_stencil(h);
  Canon4 *d = nullptr;
  HIPCHK(apc_malloc_async((void **)&d, sizeof(Canon4), s));
  HIPCHK(hipMemcpyAsync(d, &h, sizeof(Canon4), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL((k_fit4n<false, 56>), dim3(1), dim3(wpbn<56>() * 64), 0, s, (int64_t)1,
                     (const int32_t *)nullptr, d->st_off, d->st_idx, d->crd, (int64_t)57, d->level,
                     d->rorder, 1.0, 1.0, d->w64, (float *)nullptr, d->bw64, (float *)nullptr,
                     d->diag, d->inv_diag, d->hscale, d->dorder, (double *)nullptr, d->fb_list,
                     &d->fb_cnt, c->P.kernel, 0.0);
  hipLaunchKernelGGL((k_fit4<false, 56>), dim3(1), dim3(WPB4 * 64), 0, s,
                     (const int32_t *)d->fb_list, (const unsigned *)&d->fb_cnt, d->st_off,
                     d->st_idx, d->crd, (int64_t)57, d->level, d->rorder, 1.0, 1.0, d->w64,
                     (float *)nullptr, d->bw64, (float *)nullptr, d->diag, d->inv_diag, d->hscale,
                     d->dorder, (double *)nullptr, &d->err, c->P.kernel, 0.0);
  // the canonical derivative operator (56 x 34), then tabulated by offset (125 x 34)
  HIPCHK(apc_dev_alloc((void **)&c->cder4, 125 * P4 * sizeof(double)));
  double *cj = nullptr;
  HIPCHK(apc_malloc_async((void **)&cj, 56 * P4 * sizeof(double), s));
  hipLaunchKernelGGL(k_canon_derivs4, dim3((56 + WPB4 - 1) / WPB4), dim3(WPB4 * 64), 0, s,
                     (const int32_t *)d->st_idx, (const int32_t *)d->crd, cj);
  HIPCHK(hipGetLastError());
  std::vector<double> hcj(56 * P4), tab(125 * P4, 0.0);
  HIPCHK(hipMemcpyAsync(hcj.data(), cj, hcj.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&h, d, sizeof(Canon4), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(apc_free_async(d, s));
  HIPCHK(apc_free_async(cj, s));
  for (int j = 0; j < 56; j++) {
    const int o = 25 * (h.crd[j + 1] - 2) + 5 * (h.crd[57 + j + 1] - 2) + (h.crd[114 + j + 1] - 2);
    for (int a = 0; a < P4; a++) tab[o * P4 + a] = hcj[j * P4 + a];
  }
  HIPCHK(hipMemcpyAsync(c->cder4, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  const int lo[6] = {0, 6, 18, 26, 32, 56};
  double tl[5], tb[5], dev = 0.0, wmax = 0.0, bmax = 0.0;
  bool ok = h.err == 0;
  for (int q = 0; q < 5; q++) {
    double sl = 0.0, sb = 0.0;
    for (int j = lo[q]; j < lo[q + 1]; j++) {
      sl += h.w64[j];
      sb += h.bw64[j];
      wmax = fmax(wmax, fabs(h.w64[j]));
      bmax = fmax(bmax, fabs(h.bw64[j]));
    }
    tl[q] = sl / (lo[q + 1] - lo[q]);
    tb[q] = sb / (lo[q + 1] - lo[q]);
  }
  for (int q = 0; q < 5; q++)
    for (int j = lo[q]; j < lo[q + 1]; j++) {
      dev = fmax(dev, fabs(h.w64[j] - tl[q]) / wmax);
      if (bmax > 0.0) dev = fmax(dev, fabs(h.bw64[j] - tb[q]) / bmax);
    }
  ok = ok && wmax > 0.0 && dev <= 1e-12 && std::isfinite(dev);
  if (ok) {
    double sw = 0.0;
    for (int q = 0; q < 5; q++) sw += (double)(lo[q + 1] - lo[q]) * tl[q];
    for (int q = 0; q < 5; q++) {
      c->tmpl4[q] = tl[q];
      c->tmpl4[5 + q] = tb[q];
    }
    c->tmpl4_sum = sw;
    c->dorder4 = h.dorder[0];
  }
  if (n <= 0) return APC_OK;
  const int64_t ntot = c->n + c->nb;
  if (ok) {
    hipLaunchKernelGGL(k_classify4, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, n, c->st_off,
                       c->st_idx, c->crd, ntot, c->level, c->rorder, c->P.max_depth, c->rkind4);
  } else {
    HIPCHK(hipMemsetAsync(c->rkind4, 0xff, (size_t)n, s));
  }
  HIPCHK(hipGetLastError());
  int32_t *f = nullptr, *pos = nullptr;
  HIPCHK(apc_malloc_async((void **)&f, (size_t)n * sizeof(int32_t), s));
  HIPCHK(apc_malloc_async((void **)&pos, (size_t)n * sizeof(int32_t), s));
  hipLaunchKernelGGL(k_gen_flag, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, (const int8_t *)c->rkind4,
                     n, f);
  APCCHK(apc_scan_i32(f, pos, n, s));
  hipLaunchKernelGGL(k_gen_list, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, (const int8_t *)c->rkind4,
                     (const int32_t *)pos, n, c->gen4);
  HIPCHK(hipGetLastError());
  int32_t lastf = 0, lastp = 0;
  HIPCHK(hipMemcpyAsync(&lastf, f + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&lastp, pos + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(apc_free_async(f, s));
  HIPCHK(apc_free_async(pos, s));
  c->n_gen4 = (int64_t)lastp + lastf;
  c->n_uniform4 = n - c->n_gen4;
  return APC_OK;
}

int apc_assemble4(apc_cloud *c, hipStream_t s) {
  const int64_t n = c->n, ntot = c->n + c->nb;
  const bool mixed = c->P.precision != APC_FP64;
  HIPCHK(hipMemsetAsync(&c->scratch->err, 0, sizeof(int), s));
  HIPCHK(hipMemsetAsync(&c->scratch->nfp64, 0, sizeof(unsigned long long), s));
  HIPCHK(hipMemsetAsync(&c->scratch->fb_count, 0, sizeof(unsigned), s));
  if (n > 0) {
    const bool m56 = c->P.m_cap <= 56;
    double *ref = mixed ? c->w64ref : nullptr;
    // the fitted rows: every row but the uniform 56-node ones
    const int64_t nfit = c->n_uniform4 > 0 ? c->n_gen4 : n;
    const int32_t *fit_list = c->n_uniform4 > 0 ? c->gen4 : nullptr;
    const double s2 = c->P.periodic ? 0.0 : c->P.L / c->unit; // walls for the kernel moments
    // normal equations on the matrix cores for every node, then the Householder QR
    // for the nodes listed by it (grid-stride over the list; the count stays on
    // the device)
#define APC_FIT4N(MX, R)                                                                       \
  if (nfit > 0)                                                                                \
  hipLaunchKernelGGL((k_fit4n<MX, R>), dim3((unsigned)((nfit + wpbn<R>() - 1) / wpbn<R>())),  \
                     dim3(wpbn<R>() * 64), 0, s, nfit, fit_list, c->st_off, c->st_idx, c->crd, ntot, \
                     c->level, c->rorder, c->unit, c->P.L, c->w64, c->w32, c->bw64, c->bw32,   \
                     c->diag, c->inv_diag, c->hscale, c->dorder, ref, c->fb_list,              \
                     &c->scratch->fb_count, c->P.kernel, s2)
#define APC_FIT4(MX, R)                                                                        \
  hipLaunchKernelGGL((k_fit4<MX, R>), dim3(1024), dim3(WPB4 * 64), 0, s,                       \
                     (const int32_t *)c->fb_list, (const unsigned *)&c->scratch->fb_count,     \
                     c->st_off, c->st_idx, c->crd, ntot, c->level, c->rorder, c->unit, c->P.L, \
                     c->w64, c->w32, c->bw64, c->bw32, c->diag, c->inv_diag, c->hscale,        \
                     c->dorder, ref, &c->scratch->err, c->P.kernel, s2)
    if (mixed && m56) {
      APC_FIT4N(true, 56);
      APC_FIT4(true, 56);
    } else if (mixed) {
      APC_FIT4N(true, APC_MAXM);
      APC_FIT4(true, APC_MAXM);
    } else if (m56) {
      APC_FIT4N(false, 56);
      APC_FIT4(false, 56);
    } else {
      APC_FIT4N(false, APC_MAXM);
      APC_FIT4(false, APC_MAXM);
    }
#undef APC_FIT4
#undef APC_FIT4N
    hipLaunchKernelGGL(k_fb_report, dim3(1), dim3(64), 0, s, (const unsigned *)&c->scratch->fb_count,
                       &c->scratch->nfp64);
    if (c->n_uniform4 > 0) {
      Tmpl4 T;
      for (int q = 0; q < 5; q++) {
        T.tl[q] = c->tmpl4[q];
        T.tb[q] = c->tmpl4[5 + q];
      }
      T.sl = c->tmpl4_sum;
      T.dord = c->dorder4;
      const unsigned g = grid_for(n, APC_BLOCK / 64);
      if (mixed)
        hipLaunchKernelGGL(k_fill4<true>, dim3(g), dim3(APC_BLOCK), 0, s, n,
                           (const int8_t *)c->rkind4, c->st_off, T, c->P.L, c->w64, c->w32, c->bw64,
                           c->bw32, c->diag, c->inv_diag, c->hscale, c->dorder, ref);
      else
        hipLaunchKernelGGL(k_fill4<false>, dim3(g), dim3(APC_BLOCK), 0, s, n,
                           (const int8_t *)c->rkind4, c->st_off, T, c->P.L, c->w64, c->w32, c->bw64,
                           c->bw32, c->diag, c->inv_diag, c->hscale, c->dorder, ref);
    }
    HIPCHK(hipGetLastError());
  }
  c->w64_mixed = mixed && c->w64ref != nullptr;
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

// The general nodes by the normal equations on the matrix cores (k_node_derivs4n),
// the few it does not accept by the Householder QR; the uniform 56-node nodes
// through the canonical derivative operator.
int apc_node_derivs4(apc_cloud *c, const double *f, double *D, hipStream_t s) {
  const bool uni = c->n_uniform4 > 0 && c->cder4;
  const int64_t cnt = uni ? c->n_gen4 : c->n;
  const int32_t *list = uni ? c->gen4 : nullptr;
  if (cnt > 0 && c->P.m_cap <= 56) {
    hipLaunchKernelGGL(k_node_derivs4n<56>, dim3((unsigned)((cnt + wpbn<56>() - 1) / wpbn<56>())),
                       dim3(wpbn<56>() * 64), 0, s, cnt, list, c->st_off, c->st_idx, c->crd,
                       c->n + c->nb, (const int8_t *)c->rorder, c->unit, f, D);
    hipLaunchKernelGGL(k_node_derivs4<56>, dim3(grid4(cnt)), dim3(WPB4 * 64), 0, s, cnt, list,
                       c->st_off, c->st_idx, c->crd, c->n + c->nb, (const int8_t *)c->rorder,
                       c->unit, f, D, 1);
  } else if (cnt > 0) {
    hipLaunchKernelGGL(k_node_derivs4n<APC_MAXM>,
                       dim3((unsigned)((cnt + wpbn<APC_MAXM>() - 1) / wpbn<APC_MAXM>())),
                       dim3(wpbn<APC_MAXM>() * 64), 0, s, cnt, list, c->st_off, c->st_idx, c->crd,
                       c->n + c->nb, (const int8_t *)c->rorder, c->unit, f, D);
    hipLaunchKernelGGL(k_node_derivs4<APC_MAXM>, dim3(grid4(cnt)), dim3(WPB4 * 64), 0, s, cnt,
                       list, c->st_off, c->st_idx, c->crd, c->n + c->nb, (const int8_t *)c->rorder,
                       c->unit, f, D, 1);
  }
  if (uni)
    hipLaunchKernelGGL(k_derivs_u4, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n,
                       (const int8_t *)c->rkind4, c->st_off, c->st_idx, c->crd, c->n + c->nb,
                       c->P.max_depth, c->unit, (const double *)c->cder4, f, D);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

// Interpolation with the caller's derivative buffer D (n x 34 doubles): every row
// of D is written by the derivative kernel before the particle kernel reads it.
int apc_interp4_with(apc_cloud *c, const double *phi, double *phi_p, double *grad_p, double *D,
                     hipStream_t s) {
  APCCHK(apc_node_derivs4(c, phi, D, s));
  hipLaunchKernelGGL(k_interp4, dim3(grid_for(c->N)), dim3(APC_BLOCK), 0, s, c->N, c->sxyz, c->perm,
                     c->pnode, c->crd, c->n + c->nb, c->P.lo[0], c->P.lo[1], c->P.lo[2], c->unit,
                     phi, D, phi_p, grad_p);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_interp4(apc_cloud *c, const double *phi, double *phi_p, double *grad_p, hipStream_t s) {
  double *D = nullptr;
  HIPCHK(apc_malloc_async((void **)&D, (size_t)(c->n > 0 ? c->n : 1) * P4 * sizeof(double), s));
  APCCHK(apc_interp4_with(c, phi, phi_p, grad_p, D, s));
  HIPCHK(apc_free_async(D, s));
  return APC_OK;
}

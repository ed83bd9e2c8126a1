// Charge deposit and Krylov solves on gfx950.
//
// Operators are applied in difference form, (A x)_i = a_i x_i + s_i sum_j w_ij (x_j - x_i)
// with (a, s) = (0, 1) for the GFD Laplacian and (1, h_c^2/24) for the k = 2
// density operator B = I + diag(h_c^2/24) L.  Row sums of L are zero by
// construction (the constant is removed by differencing in the GFD fit), so this
// form never forms the large diagonal and stays accurate when x is smooth, also
// with FP32 weights.  Krylov vectors have n + nb entries; the boundary tail stays
// zero, boundary data enter through the right-hand side.
//
// BiCGSTAB runs as 8 kernels per iteration: 2 SpMV with fused dot products, 3
// fused vector updates and 3 one-block finalize kernels.  Dot products are
// reduced deterministically (per-block partials, then a fixed-order sum) and the
// solver scalars live on the device, so the host only polls a status word every
// few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstring>
#include <vector>

#include "apc_internal.h"
#include "spmv_core.h"
#include "prec_core.h"

namespace {

struct Scal {
  double rho, alpha, omega, beta;
  double bnorm, rnorm, rtrue;
  double rv, ts, tt;
  double tol;
  int it, maxit, done, pad;
};

// Reductions: kernels that produce dot products run on a capped grid of GRED
// blocks (grid-stride) and store one partial per block; a one-block finalize
// kernel sums the partials in a fixed order and updates the solver scalars.  No
// atomics or device-scope fences inside kernels: kernel boundaries order
// everything.  (Finalizing in the last block to finish, behind a device-scope
// release fence in every block, was measured: the fence writes back the XCD's L2
// each time and the iteration ran 3x slower.)
constexpr unsigned GRED = 2048;

template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *part) {
  __shared__ double sh[NV][APC_BLOCK / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; k++) {
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
      double s = 0.0;
      for (int q = 0; q < APC_BLOCK / 64; q++) s += sh[k][q];
      part[(size_t)k * gridDim.x + blockIdx.x] = s;
    }
  }
}

// Sum of partials part[k*G .. k*G+G) in one block of FIN_T threads, fixed order;
// valid in thread 0.  Each thread first issues all its loads (G <= 4 FIN_T), so the
// finalize kernels cost one memory round trip.
constexpr int FIN_T = 1024;
template <int NV>
__device__ __forceinline__ void fin_sum(const double *part, unsigned G, double (&out)[NV]) {
  __shared__ double sh[NV][FIN_T / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; k++) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const unsigned q = threadIdx.x + u * FIN_T;
      v[u] = q < G ? part[(size_t)k * G + q] : 0.0;
    }
    double s = (v[0] + v[1]) + (v[2] + v[3]);
    s = wave_sum(s);
    if (lane == 0) sh[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
      double t = 0.0;
      for (int q = 0; q < FIN_T / 64; q++) t += sh[k][q];
      out[k] = t;
    }
  }
}

static inline unsigned vec_grid(int64_t n) {
  const unsigned g = grid_for(n);
  return g < GRED ? g : GRED;
}

// ---------------------------------------------------------------- BiCGSTAB kernels
// v = A ph ; partial (rh, v)
template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    k_spmv_v(Op op, const double *__restrict__ ph, double *__restrict__ v,
             const double *__restrict__ rh, double *part, const Scal *sc) {
  if (sc->done) return;
  double val[1] = {0.0};
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    int32_t i;
    const double y = sell_apply<MODE>(op, ph, it.s, i);
    if (i >= 0) {
      v[i] = y;
      val[0] += rh[i] * y;
    }
  }
  block_partials<1>(val, part);
}

// t = A sh ; partials (t, s), (t, t)
template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    k_spmv_t(Op op, const double *__restrict__ sh, const double *__restrict__ s,
             double *__restrict__ t, double *part, const Scal *sc) {
  if (sc->done) return;
  double val[2] = {0.0, 0.0};
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    int32_t i;
    const double y = sell_apply<MODE>(op, sh, it.s, i);
    if (i >= 0) {
      t[i] = y;
      val[0] += y * s[i];
      val[1] += y * y;
    }
  }
  block_partials<2>(val, part);
}

// alpha = rho / (rh, v)
__global__ void __launch_bounds__(FIN_T) k_fin_alpha(const double *part, unsigned G, Scal *sc) {
  if (sc->done) return;
  double out[1];
  fin_sum<1>(part, G, out);
  if (threadIdx.x == 0) {
    sc->rv = out[0];
    const double al = sc->rho / out[0];
    if (out[0] == 0.0 || !isfinite(al))
      sc->done = 2;
    else
      sc->alpha = al;
  }
}

// omega = (t, s) / (t, t)
__global__ void __launch_bounds__(FIN_T) k_fin_omega(const double *part, unsigned G, Scal *sc) {
  if (sc->done) return;
  double out[2];
  fin_sum<2>(part, G, out);
  if (threadIdx.x == 0) {
    sc->ts = out[0];
    sc->tt = out[1];
    sc->omega = out[1] > 0.0 ? out[0] / out[1] : 0.0;
  }
}

// p = r + beta (p - omega v); ph = M p
template <bool JAC>
__global__ void __launch_bounds__(APC_BLOCK)
    k_upd_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
            const double *__restrict__ v, double *__restrict__ ph,
            const double *__restrict__ invd, const Scal *sc) {
  if (sc->done) return;
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double pi = r[i] + sc->beta * (p[i] - sc->omega * v[i]);
  p[i] = pi;
  if (JAC) ph[i] = pi * invd[i];
}

// s = r - alpha v; sh = M s
template <bool JAC>
__global__ void __launch_bounds__(APC_BLOCK)
    k_upd_s(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
            double *__restrict__ s, double *__restrict__ sh, const double *__restrict__ invd,
            const Scal *sc) {
  if (sc->done) return;
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double si = r[i] - sc->alpha * v[i];
  s[i] = si;
  if (JAC) sh[i] = si * invd[i];
}

// out = M in over the rows of every slice (the learned preconditioner); launched
// with op_lds(op) bytes of dynamic LDS
__global__ void __launch_bounds__(APC_BLOCK)
    k_prec_apply(Op op, MOp M, const double *__restrict__ in, double *__restrict__ out,
                 const Scal *sc) {
  if (sc && sc->done) return;
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    const int s = __builtin_amdgcn_readfirstlane(it.s);
    const int u = op.sl_un ? op.sl_un[s] : 0;
    if (u > 0)
      prec_slice<false, true>(op, M, in, out, s, u);
    else if (op.sl_top4)
      prec_slice<true, false>(op, M, in, out, s, 0);
    else
      prec_slice<false, false>(op, M, in, out, s, 0);
  }
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_scale_copy(int64_t n, const double *__restrict__ in, const double *__restrict__ invd,
                 double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) out[i] = invd ? in[i] * invd[i] : in[i];
}

// x += alpha ph + omega sh; r = s - omega t; partials (rh, r), (r, r)
__global__ void __launch_bounds__(APC_BLOCK)
    k_upd_xr(int64_t n, double *__restrict__ x, const double *__restrict__ ph,
             const double *__restrict__ sh, const double *__restrict__ s,
             const double *__restrict__ t, double *__restrict__ r,
             const double *__restrict__ rh, double *part, const Scal *sc) {
  if (sc->done) return;
  const double al = sc->alpha, om = sc->omega;
  double val[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * APC_BLOCK) {
    // x, t and rh are not read again before the next iteration's update: they
    // bypass the caches, which keep p, s and r for the next operator applies
    // (same arithmetic: x + (alpha ph + omega sh))
    const double dx = al * ph[i] + om * sh[i];
    __builtin_nontemporal_store(__builtin_nontemporal_load(&x[i]) + dx, &x[i]);
    const double ri = s[i] - om * __builtin_nontemporal_load(&t[i]);
    r[i] = ri;
    val[0] += __builtin_nontemporal_load(&rh[i]) * ri;
    val[1] += ri * ri;
  }
  block_partials<2>(val, part);
}

// rho' = (rh, r): convergence test, beta for the next iteration
__global__ void __launch_bounds__(FIN_T) k_fin_rho(const double *part, unsigned G, Scal *sc) {
  if (sc->done) return;
  double out[2];
  fin_sum<2>(part, G, out);
  if (threadIdx.x == 0) {
    const double rho_new = out[0];
    const double al = sc->alpha, om = sc->omega;
    sc->rnorm = sqrt(out[1]);
    sc->it += 1;
    if (sc->rnorm <= sc->tol * sc->bnorm) {
      sc->done = 1;
    } else if (rho_new == 0.0 || om == 0.0 || !isfinite(rho_new)) {
      sc->done = 2;
    } else if (sc->it >= sc->maxit) {
      sc->done = 3;
    } else {
      sc->beta = (rho_new / sc->rho) * (al / om);
      sc->rho = rho_new;
    }
  }
}

// (re)start from x: r = b - A x (true residual, arithmetic MODE), rh = r, p = v = 0;
// partials (r, r), (b, b)
template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    k_restart(Op op, const double *__restrict__ b, const double *__restrict__ x,
              double *__restrict__ r, double *__restrict__ rh, double *__restrict__ p,
              double *__restrict__ v, double *part, int first) {
  double val[2] = {0.0, 0.0};
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    int32_t i = op.sl_rows[(int64_t)it.s * SL + (threadIdx.x & 63)];
    double y = 0.0;
    if (!first) y = sell_apply<MODE>(op, x, it.s, i);
    if (i >= 0) {
      const double ri = b[i] - y;
      r[i] = ri;
      rh[i] = ri;
      p[i] = 0.0;
      v[i] = 0.0;
      val[0] += ri * ri;
      val[1] += b[i] * b[i];
    }
  }
  block_partials<2>(val, part);
}

__global__ void __launch_bounds__(FIN_T)
    k_fin_restart(const double *part, unsigned G, Scal *sc, int first) {
  double out[2];
  fin_sum<2>(part, G, out);
  if (threadIdx.x == 0) {
    if (first) sc->bnorm = sqrt(out[1]);
    sc->rho = out[0];
    sc->rnorm = sqrt(out[0]);
    sc->rtrue = sc->bnorm > 0.0 ? sc->rnorm / sc->bnorm : 0.0;
    sc->beta = 0.0;
    sc->alpha = 1.0;
    sc->omega = 1.0;
    sc->done = (sc->bnorm == 0.0 || sc->rnorm <= sc->tol * sc->bnorm) ? 1 : 0;
  }
}

// ---------------------------------------------------------------- right-hand sides
// Poisson: b_i = c rho_i - sum_{j boundary} w_ij g_j
// Density: b_i = rhoM_i - hs_i sum_{j boundary} w_ij rhoM_j
template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    k_rhs(Op op, int64_t n, const double *__restrict__ src, double srcscale,
          const double *__restrict__ bval, double *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const bool ex = op.hs && op.hs[i] < 0.0; // explicit density row
  double acc = 0.0;
  if (bval) {
    for (int32_t e = op.off[i]; e < op.off[i + 1]; e++) {
      const int32_t j = op.idx[e];
      if (j >= n)
        acc += (ex ? op.dwx[e] : ((MODE == V64) ? op.w64[e] : (double)op.w32[e])) * bval[j - n];
    }
  }
  b[i] = srcscale * src[i] - ((op.hs && !ex) ? op.hs[i] * acc : acc);
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_write_out(int64_t n, int64_t nb, const double *__restrict__ x,
                const double *__restrict__ bval, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n)
    out[i] = x[i];
  else if (i < n + nb)
    out[i] = bval ? bval[i - n] : 0.0;
}

template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    k_apply(Op op, const double *__restrict__ x, double *__restrict__ y) {
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    int32_t i;
    const double v = sell_apply<MODE>(op, x, it.s, i);
    if (i >= 0) y[i] = v;
  }
}

// NGP deposit: rho_M_j = (sum of the charges in cell j) / h_j^3
__global__ void __launch_bounds__(APC_BLOCK)
    k_deposit(int64_t n, int64_t N, const int32_t *__restrict__ first,
              const int32_t *__restrict__ count, const int32_t *__restrict__ level,
              const int32_t *__restrict__ perm, const double *__restrict__ q, double L,
              double *__restrict__ rho) {
  const int64_t j = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (j >= n) return;
  double sum;
  if (q) {
    sum = 0.0;
    const int32_t a = first[j], b = a + count[j];
    for (int32_t s = a; s < b; s++) sum += q[perm[s]];
  } else {
    sum = (double)count[j] * (1.0 / (double)N);
  }
  const double hc = L / (double)(1 << level[j]);
  rho[j] = sum / (hc * hc * hc);
}

// last node whose code (Morton key of its cell's minimum corner) is <= key; the
// leaves tile Omega, so that node's cell holds the key
__device__ __forceinline__ int64_t leaf_of(const uint64_t *__restrict__ code, int64_t n,
                                           uint64_t key) {
  int64_t lo = 0, hi = n; // code[lo] <= key < code[hi] (code[0] = 0)
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (code[mid] <= key) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Leaf lookup table of level L0 (<= max_depth): tab[k] = the leaf that holds the
// lowest corner of level-L0 cell k (a coarser leaf covers all its level-L0 cells);
// -1 where no leaf lies (cells outside Omega).  The leaf holding a key then lies
// between the entries of the key's cell and of the next cell.
__global__ void __launch_bounds__(APC_BLOCK)
    k_leaf_table(int64_t n, const uint64_t *__restrict__ code, const int32_t *__restrict__ level,
                 int D, int L0, int32_t *__restrict__ tab) {
  const int64_t j = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (j >= n) return;
  const int sh = 3 * (D - L0);
  const uint64_t cc = code[j] >> sh;
  const int l = level[j];
  if (l >= L0) {
    if (j == 0 || (code[j - 1] >> sh) != cc) tab[cc] = (int32_t)j;
  } else {
    const uint64_t m = 1ull << (3 * (L0 - l));
    for (uint64_t k = 0; k < m; k++) tab[cc + k] = (int32_t)j;
  }
}

// the last leaf with code <= key, searched between the table entries of the key's
// level-L0 cell and of the next one (the whole list where the table has no entry)
__device__ __forceinline__ int64_t leaf_of_tab(const uint64_t *__restrict__ code, int64_t n,
                                               const int32_t *__restrict__ tab, int64_t ncell,
                                               int sh, uint64_t key) {
  const int64_t cc = (int64_t)(key >> sh);
  const int32_t t0 = tab[cc];
  if (t0 < 0) return leaf_of(code, n, key);
  int64_t hi = n;
  for (int64_t k = cc + 1; k < ncell; k++) // the next cell with an entry
    if (tab[k] >= 0) {
      hi = tab[k];
      break;
    }
  int64_t lo = t0; // code[lo] <= key < code[hi]
  if (hi <= lo) return lo;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (code[mid] <= key) lo = mid;
    else hi = mid;
  }
  return lo;
}

// CIC / TSC deposit (eq. density_apcloud): rho_M_j = sum_i q_i Phi((p_i - y_j) / h_j)
// / (a_0 h_j^3), one wavefront per node.  The kernel's support lies in the 3 x 3 x 3
// block of cells of the node's size around it; each such region R (an aligned cube,
// so a contiguous range of Morton keys and of sorted particles) is either inside
// one leaf (a coarser or equal cell: its particles are visited once, from the
// region of the block that holds the leaf's lowest corner in it) or the union of
// the leaves whose keys fall in R.  Lane t < 27 finds region t's particle range;
// the ranges are then walked as one list, 64 consecutive particles at a time (each
// lane its own particle: coalesced loads), and the lanes' partial sums are reduced
// in a fixed order.  Minimum-image offsets on a periodic domain.
__global__ void __launch_bounds__(APC_BLOCK)
    k_deposit_kern(int64_t n, int64_t N, int kernel, int D, const uint64_t *__restrict__ code,
                   const int32_t *__restrict__ level, const int32_t *__restrict__ first,
                   const int32_t *__restrict__ count, const int32_t *__restrict__ crd,
                   int64_t ntot, const double *__restrict__ sxyz, const int32_t *__restrict__ perm,
                   const double *__restrict__ q, double lo0, double lo1, double lo2, double L,
                   double unit, const int32_t *__restrict__ tab, int L0,
                   double *__restrict__ rho) {
  __shared__ int32_t s_end[APC_BLOCK / 64][32], s_off[APC_BLOCK / 64][32];
  const int tsh = 3 * (D - L0);
  const int64_t ncell = (int64_t)1 << (3 * L0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * (APC_BLOCK / 64) + w;
  if (j >= n) return; // whole wavefronts
  const int32_t side = 1 << D, S = crd[3 * ntot];
  const bool per = S != 0;
  const int l = level[j];
  const int32_t E = 1 << (D - l); // cell edge in units L / 2^D
  const int32_t c[3] = {crd[j], crd[ntot + j], crd[2 * ntot + j]};
  const int32_t o[3] = {(c[0] - E) >> 1, (c[1] - E) >> 1, (c[2] - E) >> 1};
  const double hc = L / (double)(1 << l);
  const double yc[3] = {lo0 + unit * (double)c[0], lo1 + unit * (double)c[1],
                        lo2 + unit * (double)c[2]};
  const double q0 = 1.0 / (double)N;
  // region coordinate along an axis (-1 when outside a bounded domain)
  auto rc = [&](int d, int t) -> int32_t {
    int32_t r = o[d] + t * E;
    if (per) return (r + side) & (side - 1);
    return (r < 0 || r >= side) ? -1 : r;
  };
  int32_t ps = 0, pe = 0;
  if (lane < 27) {
    const int t[3] = {lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1};
    int32_t r[3];
    bool valid = true;
    for (int d = 0; d < 3; d++) {
      r[d] = rc(d, t[d]);
      valid = valid && r[d] >= 0;
    }
    if (valid) {
      const uint64_t k0 = apc_morton((uint32_t)r[0], (uint32_t)r[1], (uint32_t)r[2]);
      const int64_t a = leaf_of_tab(code, n, tab, ncell, tsh, k0);
      const int32_t Ea = 1 << (D - level[a]);
      if (Ea >= E) {
        // R lies in leaf a: only the block's first region in that leaf (per axis
        // the smallest offset t whose region is inside it) takes its particles
        const int32_t oa[3] = {(crd[a] - Ea) >> 1, (crd[ntot + a] - Ea) >> 1,
                               (crd[2 * ntot + a] - Ea) >> 1};
        bool firstr = true;
        for (int d = 0; d < 3 && firstr; d++)
          for (int u = -1; u < t[d]; u++) {
            const int32_t rr = rc(d, u);
            if (rr >= 0 && ((rr - oa[d] + side) & (side - 1)) < Ea) firstr = false;
          }
        if (firstr) {
          ps = first[a];
          pe = ps + count[a];
        }
      } else {
        const uint64_t e3 = (uint64_t)E * (uint64_t)E * (uint64_t)E;
        const int64_t b = leaf_of_tab(code, n, tab, ncell, tsh, k0 + e3 - 1);
        ps = first[a];
        pe = first[b] + count[b];
      }
    }
  }
  // the ranges as one list: region t holds list positions [end_t - len_t, end_t)
  const int32_t len = pe - ps;
  int32_t incl = len;
#pragma unroll
  for (int sh = 1; sh < 64; sh <<= 1) {
    const int32_t v = __shfl_up(incl, sh, 64);
    if (lane >= sh) incl += v;
  }
  const int32_t T = __shfl(incl, 63, 64);
  if (lane < 32) {
    s_end[w][lane] = lane < 27 ? incl : INT32_MAX;
    s_off[w][lane] = ps - (incl - len); // particle = list position + off
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double sum = 0.0;
  for (int32_t i = lane; i < T; i += 64) {
    int lo = 0, hi = 26; // the first region with end > i
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_end[w][mid] > i) hi = mid;
      else lo = mid + 1;
    }
    const int32_t sp = i + s_off[w][lo];
    double wgt = 1.0;
    for (int d = 0; d < 3 && wgt != 0.0; d++) {
      double dx = sxyz[(int64_t)d * N + sp] - yc[d];
      if (per) {
        if (dx >= 0.5 * L) dx -= L;
        else if (dx < -0.5 * L) dx += L;
      }
      wgt *= apc_kernel_phi(kernel, dx / hc);
    }
    if (wgt != 0.0) sum += (q ? q[perm[sp]] : q0) * wgt;
  }
#pragma unroll
  for (int sh = 32; sh > 0; sh >>= 1) sum += __shfl_xor(sum, sh, 64);
  if (lane == 0) {
    double tlo[3], thi[3];
    apc_node_trunc(c[0], c[1], c[2], (double)(2 * E), per ? 0.0 : (double)(2 * side), tlo, thi);
    rho[j] = sum / (apc_kernel_a0(kernel, tlo, thi) * (hc * hc * hc));
  }
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_bnd_copy(int64_t n, int64_t nb, const int32_t *__restrict__ bowner, double *__restrict__ v) {
  const int64_t b = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (b < nb) v[n + b] = v[bowner[b]];
}

// FP64 reference residual, fourth order: r_i = b_i - sum_j w_ij (x_j - x_i) over
// the CSR rows of the FP64 weights (x has a zero boundary tail, so boundary
// columns contribute -w_ij x_i as in the interior operator); one wavefront per
// row (at most 64 entries); partial sums of r^2 per block.
__global__ void __launch_bounds__(APC_BLOCK)
    k_resid_csr(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
                const double *__restrict__ w64, const double *__restrict__ b,
                const double *__restrict__ x, double *part) {
  double val[1] = {0.0};
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (APC_BLOCK / 64);
  for (int64_t i = (int64_t)blockIdx.x * (APC_BLOCK / 64) + (threadIdx.x >> 6); i < n; i += nw) {
    const int32_t a = st_off[i], m = st_off[i + 1] - a;
    const double xi = x[i];
    double t = lane < m ? w64[a + lane] * (x[st_idx[a + lane]] - xi) : 0.0;
    t = wave_sum(t);
    if (lane == 0) {
      const double r = b[i] - t;
      val[0] += r * r;
    }
  }
  block_partials<1>(val, part);
}

// sum of r^2 over rows (r given), partials per block
__global__ void __launch_bounds__(APC_BLOCK)
    k_sumsq(int64_t n, const double *__restrict__ r, double *part) {
  double val[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * APC_BLOCK)
    val[0] += r[i] * r[i];
  block_partials<1>(val, part);
}

} // namespace

// ---------------------------------------------------------------- workspace
struct apc_solver_ws {
  int64_t n = 0, ntot = 0;
  double *x = nullptr, *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr,
         *t = nullptr, *ph = nullptr, *sh = nullptr, *b = nullptr;
  double *part = nullptr;
  Scal *sc = nullptr;
  Scal *sc_host = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // kernel timing (apc_set_diagnostics): start/stop events of the two SpMVs of
  // every iteration of a chunk (at most 32 iterations between host polls)
  hipEvent_t kev[4 * 32] = {};
  bool kev_made = false;
  double spmv_ms = 0.0;
  int64_t spmv_launches = 0;
};

void apc_free_solver(apc_cloud *c) {
  apc_solver_ws *w = c->ws;
  if (!w) return;
  double *vs[] = {w->x, w->r, w->rh, w->p, w->v, w->s, w->t, w->ph, w->sh, w->b, w->part};
  for (double *q : vs)
    if (q) (void)apc_dev_free(q);
  if (w->sc) (void)apc_dev_free(w->sc);
  if (w->sc_host) (void)hipHostFree(w->sc_host);
  if (w->e0) (void)hipEventDestroy(w->e0);
  if (w->e1) (void)hipEventDestroy(w->e1);
  if (w->kev_made)
    for (hipEvent_t e : w->kev) (void)hipEventDestroy(e);
  delete w;
  c->ws = nullptr;
}

static int ensure_ws(apc_cloud *c) {
  if (c->ws) return APC_OK;
  apc_solver_ws *w = new apc_solver_ws();
  c->ws = w;
  w->n = c->n;
  w->ntot = c->n + c->nb;
  const size_t bytes = (size_t)w->ntot * sizeof(double);
  double **vs[] = {&w->x, &w->r, &w->rh, &w->p, &w->v, &w->s, &w->t, &w->ph, &w->sh, &w->b};
  for (double **q : vs) {
    HIPCHK(apc_dev_alloc((void **)q, bytes));
    HIPCHK(hipMemset(*q, 0, bytes)); // boundary tails stay zero for good
  }
  HIPCHK(apc_dev_alloc((void **)&w->part, 2 * (size_t)GSPMV * sizeof(double)));
  HIPCHK(apc_dev_alloc((void **)&w->sc, sizeof(Scal)));
  HIPCHK(hipMemset(w->sc, 0, sizeof(Scal)));
  HIPCHK(hipHostMalloc((void **)&w->sc_host, sizeof(Scal), hipHostMallocDefault));
  HIPCHK(hipEventCreate(&w->e0));
  HIPCHK(hipEventCreate(&w->e1));
  return APC_OK;
}

static int read_sc(apc_solver_ws *w, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(w->sc_host, w->sc, sizeof(Scal), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return APC_OK;
}

template <int MODE>
static int launch_restart(apc_solver_ws *w, const Op &op, const double *b, const double *x,
                          int first, unsigned g, hipStream_t s) {
  hipLaunchKernelGGL(k_restart<MODE>, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, b, x, w->r, w->rh, w->p,
                     w->v, w->part, first);
  hipLaunchKernelGGL(k_fin_restart, dim3(1), dim3(FIN_T), 0, s, w->part, g, w->sc, first);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

// ev (may be null): four events recorded around the iteration's two SpMVs
template <int MODE>
static void launch_iteration(apc_solver_ws *w, const Op &op, double *x, const double *invd,
                             const MOp &mw, int prec, unsigned gs, hipStream_t s,
                             hipEvent_t *ev) {
  const int64_t n = w->n;
  const unsigned gv = grid_for(n), gr = vec_grid(n);
  const bool jac = prec == APC_PRECOND_JACOBI, lrn = prec == APC_PRECOND_LEARNED;
  double *ph = (jac || lrn) ? w->ph : w->p;
  double *sh = (jac || lrn) ? w->sh : w->s;
  if (jac)
    hipLaunchKernelGGL(k_upd_p<true>, dim3(gv), dim3(APC_BLOCK), 0, s, n, w->r, w->p, w->v, ph,
                       invd, w->sc);
  else
    hipLaunchKernelGGL(k_upd_p<false>, dim3(gv), dim3(APC_BLOCK), 0, s, n, w->r, w->p, w->v, ph,
                       invd, w->sc);
  if (lrn) hipLaunchKernelGGL(k_prec_apply, dim3(gs), dim3(APC_BLOCK), op_lds(op), s, op, mw, w->p, ph, w->sc);
  if (ev) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(k_spmv_v<MODE>, dim3(gs), dim3(APC_BLOCK), op_lds(op), s, op, ph, w->v, w->rh, w->part,
                     w->sc);
  if (ev) (void)hipEventRecord(ev[1], s);
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(FIN_T), 0, s, w->part, gs, w->sc);
  if (jac)
    hipLaunchKernelGGL(k_upd_s<true>, dim3(gv), dim3(APC_BLOCK), 0, s, n, w->r, w->v, w->s, sh,
                       invd, w->sc);
  else
    hipLaunchKernelGGL(k_upd_s<false>, dim3(gv), dim3(APC_BLOCK), 0, s, n, w->r, w->v, w->s, sh,
                       invd, w->sc);
  if (lrn) hipLaunchKernelGGL(k_prec_apply, dim3(gs), dim3(APC_BLOCK), op_lds(op), s, op, mw, w->s, sh, w->sc);
  if (ev) (void)hipEventRecord(ev[2], s);
  hipLaunchKernelGGL(k_spmv_t<MODE>, dim3(gs), dim3(APC_BLOCK), op_lds(op), s, op, sh, w->s, w->t, w->part,
                     w->sc);
  if (ev) (void)hipEventRecord(ev[3], s);
  hipLaunchKernelGGL(k_fin_omega, dim3(1), dim3(FIN_T), 0, s, w->part, gs, w->sc);
  hipLaunchKernelGGL(k_upd_xr, dim3(gr), dim3(APC_BLOCK), 0, s, n, x, ph, sh, w->s, w->t, w->r,
                     w->rh, w->part, w->sc);
  hipLaunchKernelGGL(k_fin_rho, dim3(1), dim3(FIN_T), 0, s, w->part, gr, w->sc);
}

// BiCGSTAB on A x = b from x = 0.  MODE is the SpMV of the iteration, TMODE the
// one of the true residual; when the recursive residual meets tol (or the method
// breaks down) the true residual b - A x is recomputed and, if it does not meet
// tol, the iteration restarts from it.  With FP32 iteration arithmetic and FP64
// true residuals this restart is the iterative refinement of the mixed mode.
template <int MODE, int TMODE>
static int bicgstab(apc_cloud *c, const Op &op, const double *invd, const double *b, double *x,
                    double tol, int maxit, int prec, apc_stats *st, hipStream_t s) {
  apc_solver_ws *w = c->ws;
  const int64_t n = w->n;
  const unsigned gs = spmv_grid(c);
  Scal init;
  memset(&init, 0, sizeof(init));
  init.tol = tol;
  init.maxit = maxit;
  HIPCHK(hipMemcpyAsync(w->sc, &init, sizeof(Scal), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s));
  APCCHK(launch_restart<TMODE>(w, op, b, x, 1, gs, s));
  const bool timed = (c->diag_flags & APC_DIAG_KERNEL_TIMES) != 0;
  if (timed && !w->kev_made) {
    // timing-only events: no system-scope fence (the default event's cache write-back
    // and invalidate would slow the SpMV it brackets; the chunk's read of the
    // solver scalars synchronises before the times are read)
    for (hipEvent_t &e : w->kev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    w->kev_made = true;
  }
  int chunk = 8, nrest = 0, status = APC_ENOCONV, it0 = 0;
  for (;;) {
    for (int k = 0; k < chunk; k++)
      launch_iteration<MODE>(w, op, x, invd, MOp{c->m_diag, c->m_sell, c->m_tmpl, c->P.order == 4 ? 42 : 26}, prec,
                             gs, s, timed ? &w->kev[4 * k] : nullptr);
    HIPCHK(hipGetLastError());
    APCCHK(read_sc(w, s));
    Scal &h = *w->sc_host;
    if (timed) {
      // SpMVs of the iterations that completed (later launches of the chunk return
      // at once once the solver has stopped, and are not counted)
      for (int k = 0; k < chunk && it0 + k < h.it; k++)
        for (int q = 0; q < 2; q++) {
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, w->kev[4 * k + 2 * q], w->kev[4 * k + 2 * q + 1]));
          w->spmv_ms += ms;
          w->spmv_launches++;
        }
    }
    it0 = h.it;
    if (!h.done) {
      if (chunk < 32) chunk *= 2;
      continue;
    }
    const int reason = h.done;
    APCCHK(launch_restart<TMODE>(w, op, b, x, 0, gs, s));
    APCCHK(read_sc(w, s));
    if (h.rtrue <= tol) {
      status = APC_OK;
      break;
    }
    if (reason == 3 || h.it >= maxit || nrest >= 50) break;
    nrest++;
    chunk = 8;
  }
  const Scal &h = *w->sc_host;
  if (st) {
    st->spmv_ms = w->spmv_ms;
    st->spmv_launches = w->spmv_launches;
    st->iters = h.it;
    st->restarts = nrest;
    st->sweeps = 1 + nrest;
    st->status = status;
    st->rel_resid = h.bnorm > 0.0 ? h.rnorm / h.bnorm : 0.0;
    st->rel_resid_true = h.rtrue;
    st->precond_used = prec;
  }
  return status;
}

// FP64: FP64 weights and arithmetic throughout.  Mixed: FP32 weights (half the
// matrix bytes), FP64 SpMV accumulation, FP64 vectors and dot products, FP64
// true residuals deciding convergence.  Mixed with FP32 accumulation: FP32 SpMV
// arithmetic in the iteration, the FP64 true residual restarting it (iterative
// refinement) until it meets tol.
static int run_once(apc_cloud *c, const Op &op, const double *invd, const double *b, double *x,
                    double tol, int maxit, int prec, apc_stats *st, hipStream_t s) {
  if (c->P.precision == APC_MIXED_F32ACC)
    return bicgstab<V32A32, V32A64>(c, op, invd, b, x, tol, maxit, prec, st, s);
  if (c->P.precision == APC_MIXED)
    return bicgstab<V32A64, V32A64>(c, op, invd, b, x, tol, maxit, prec, st, s);
  return bicgstab<V64, V64>(c, op, invd, b, x, tol, maxit, prec, st, s);
}

// The learned preconditioner only changes the iteration; the true residual decides.
// When the learned solve does not reach tol, the solve is repeated with Jacobi.
static int run_solve(apc_cloud *c, bool density, const double *b, double *x, double tol, int maxit,
                     int prec, apc_stats *st, hipStream_t s) {
  Op op = make_op(c, density);
  op.pin = (!density && c->P.periodic) ? 1 : 0;
  c->ws->spmv_ms = 0.0;
  c->ws->spmv_launches = 0;
  const double *invd = density ? nullptr : c->inv_diag; // the density solve is plain
  int rc = run_once(c, op, invd, b, x, tol, maxit, prec, st, s);
  if (rc == APC_ENOCONV && prec == APC_PRECOND_LEARNED) {
    const int it = st ? st->iters : 0;
    rc = run_once(c, op, invd, b, x, tol, maxit, APC_PRECOND_JACOBI, st, s);
    if (st) st->iters += it;
  }
  return rc;
}

int apc_deposit_impl(apc_cloud *c, const double *q, double *rho_M, hipStream_t s) {
  if (c->P.kernel == APC_KERNEL_NGP) {
    hipLaunchKernelGGL(k_deposit, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->N,
                       c->first, c->count, c->level, c->perm, q, c->P.L, rho_M);
  } else if (c->n > 0) {
    const int D = c->P.max_depth, L0 = D < 7 ? D : 7; // table of 8^L0 entries (8 MiB at most)
    const size_t ncell = (size_t)1 << (3 * L0);
    int32_t *tab = nullptr;
    HIPCHK(apc_malloc_async((void **)&tab, ncell * sizeof(int32_t), s));
    HIPCHK(hipMemsetAsync(tab, 0xff, ncell * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_leaf_table, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n,
                       (const uint64_t *)c->code, c->level, D, L0, tab);
    hipLaunchKernelGGL(k_deposit_kern, dim3(grid_for(c->n, APC_BLOCK / 64)), dim3(APC_BLOCK), 0, s,
                       c->n, c->N, c->P.kernel, D, (const uint64_t *)c->code, c->level, c->first,
                       c->count, c->crd, c->n + c->nb, c->sxyz, c->perm, q, c->P.lo[0],
                       c->P.lo[1], c->P.lo[2], c->P.L, c->unit, (const int32_t *)tab, L0, rho_M);
    HIPCHK(hipGetLastError());
    HIPCHK(apc_free_async(tab, s));
  }
  if (c->nb > 0)
    hipLaunchKernelGGL(k_bnd_copy, dim3(grid_for(c->nb)), dim3(APC_BLOCK), 0, s, c->n, c->nb,
                       c->bowner, rho_M);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_density_solve_impl(apc_cloud *c, const double *rho_M, double *rho_t, double tol,
                           int maxit, apc_stats *st, hipStream_t s) {
  if (!c->assembled) return APC_EINVAL;
  APCCHK(ensure_ws(c));
  apc_solver_ws *w = c->ws;
  const Op op = make_op(c, true);
  HIPCHK(hipEventRecord(w->e0, s));
  if (c->P.precision != APC_FP64)
    hipLaunchKernelGGL(k_rhs<V32A64>, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, op, c->n, rho_M,
                       1.0, rho_M + c->n, w->b);
  else
    hipLaunchKernelGGL(k_rhs<V64>, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, op, c->n, rho_M,
                       1.0, rho_M + c->n, w->b);
  HIPCHK(hipGetLastError());
  // plain BiCGSTAB: B is the identity plus a local perturbation.  (For k = 4
  // the rows of coarse nodes beside finer ones have diagonals far from 1, of
  // either sign; right Jacobi scaling of the other rows changed the iteration
  // count at 8.8e6 nodes by -17% to +18% depending on the cut-off, and scaling
  // all rows stalled.)
  int rc = run_solve(c, true, w->b, w->x, tol, maxit, APC_PRECOND_NONE, st, s);
  if (rc < 0) return rc;
  if (st) st->rel_resid_fp64ref = c->P.precision == APC_FP64 ? w->sc_host->rtrue : -1.0;
  hipLaunchKernelGGL(k_write_out, dim3(grid_for(c->n + c->nb)), dim3(APC_BLOCK), 0, s, c->n, c->nb,
                     w->x, rho_M + c->n, rho_t);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(w->e1, s));
  HIPCHK(hipEventSynchronize(w->e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, w->e0, w->e1));
  if (st) {
    st->ms = ms;
    unsigned long long nf = 0;
    HIPCHK(hipMemcpy(&nf, &c->scratch->nfp64, sizeof(nf), hipMemcpyDeviceToHost));
    c->n_fp64_rows = (int64_t)nf;
    st->n_fp64_rows = c->n_fp64_rows;
  }
  return rc;
}

// ---------------------------------------------------------------- periodic domains
// per-block partial sums of v_j h_j^3 and h_j^3 (cell volumes), PV blocks
constexpr int PV = 1024;
__global__ void __launch_bounds__(APC_BLOCK)
    k_vol_part(int64_t n, const int32_t *__restrict__ level, double L, const double *__restrict__ v,
               double *__restrict__ part) {
  double q = 0.0, vol = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * APC_BLOCK) {
    const double h = ldexp(L, -level[i]);
    const double h3 = h * h * h;
    q += v[i] * h3;
    vol += h3;
  }
  __shared__ double sq[APC_BLOCK / 64], sv[APC_BLOCK / 64];
  q = wave_sum(q);
  vol = wave_sum(vol);
  if ((threadIdx.x & 63) == 0) {
    sq[threadIdx.x >> 6] = q;
    sv[threadIdx.x >> 6] = vol;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < APC_BLOCK / 64; k++) {
      a += sq[k];
      b += sv[k];
    }
    part[blockIdx.x] = a;
    part[PV + blockIdx.x] = b;
  }
}
// the volume-weighted mean from the partials (one block, fixed order)
__global__ void __launch_bounds__(APC_BLOCK) k_vol_mean(const double *__restrict__ part, int nblk,
                                                        double *__restrict__ mean) {
  __shared__ double sq[APC_BLOCK], sv[APC_BLOCK];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblk; k += APC_BLOCK) {
    a += part[k];
    b += part[PV + k];
  }
  sq[threadIdx.x] = a;
  sv[threadIdx.x] = b;
  __syncthreads();
  for (int w = APC_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sq[threadIdx.x] += sq[threadIdx.x + w];
      sv[threadIdx.x] += sv[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *mean = sv[0] > 0.0 ? sq[0] / sv[0] : 0.0;
}
// b = c (rho~ - mean), with the equation of node 0 replaced by phi_0 = 0
__global__ void __launch_bounds__(APC_BLOCK)
    k_rhs_periodic(int64_t n, const double *__restrict__ rho, double c,
                   const double *__restrict__ mean, double *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) b[i] = i == 0 ? 0.0 : c * (rho[i] - *mean);
}
__global__ void __launch_bounds__(APC_BLOCK)
    k_sub_mean(int64_t n, const double *__restrict__ mean, double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) x[i] -= *mean;
}

static int vol_mean(apc_cloud *c, const double *v, hipStream_t s) {
  const unsigned g = std::min(grid_for(c->n), (unsigned)PV);
  hipLaunchKernelGGL(k_vol_part, dim3(g), dim3(APC_BLOCK), 0, s, c->n, c->level, c->P.L, v,
                     c->ws->part);
  hipLaunchKernelGGL(k_vol_mean, dim3(1), dim3(APC_BLOCK), 0, s, (const double *)c->ws->part,
                     (int)g, &c->scratch->pmean);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_solve_impl(apc_cloud *c, const double *rho_t, const double *g, double *phi, double tol,
                   int maxit, int precond, apc_stats *st, hipStream_t s) {
  if (!c->assembled) return APC_EINVAL;
  if (precond != APC_PRECOND_NONE && precond != APC_PRECOND_JACOBI &&
      precond != APC_PRECOND_LEARNED)
    return APC_EINVAL;
  if (precond == APC_PRECOND_LEARNED && !c->learned) return APC_EINVAL;
  APCCHK(ensure_ws(c));
  apc_solver_ws *w = c->ws;
  const Op op = make_op(c, false);
  HIPCHK(hipEventRecord(w->e0, s));
  if (c->P.periodic) {
    // Delta phi = c (rho~ - mean rho~); phi_0 = 0 in place of node 0's equation
    APCCHK(vol_mean(c, rho_t, s));
    hipLaunchKernelGGL(k_rhs_periodic, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, rho_t,
                       c->P.poisson_c, (const double *)&c->scratch->pmean, w->b);
  } else if (c->P.precision != APC_FP64) {
    hipLaunchKernelGGL(k_rhs<V32A64>, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, op, c->n, rho_t,
                       c->P.poisson_c, g, w->b);
  } else {
    hipLaunchKernelGGL(k_rhs<V64>, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, op, c->n, rho_t,
                       c->P.poisson_c, g, w->b);
  }
  HIPCHK(hipGetLastError());
  int rc = run_solve(c, false, w->b, w->x, tol, maxit, precond, st, s);
  if (rc < 0) return rc;
  double fp64ref = -1.0;
  if (c->P.precision == APC_FP64) {
    fp64ref = w->sc_host->rtrue;
  } else if ((c->diag_flags & APC_DIAG_FP64_RESIDUAL) && !c->P.periodic) {
    // (not for periodic domains: the FP64 rows below do not hold the pinned row)
    // ||b - A64 x|| / ||b|| with the FP64 fit of the same stencils (the mixed
    // modes iterate on FP32 weights); w->t is free after the solve
    const unsigned gr = vec_grid(c->n);
    if (c->P.order == 4 && !c->w64_mixed) {
      fp64ref = -1.0; // assembled before the flag was set: no FP64 rows kept
    } else if (c->P.order == 4) {
      hipLaunchKernelGGL(k_resid_csr, dim3(gr), dim3(APC_BLOCK), 0, s, c->n, c->st_off, c->st_idx,
                         (const double *)c->w64ref, (const double *)w->b, (const double *)w->x,
                         w->part);
    } else {
      APCCHK(apc_resid64_rows(c, w->b, w->x, w->t, s));
      hipLaunchKernelGGL(k_sumsq, dim3(gr), dim3(APC_BLOCK), 0, s, c->n, (const double *)w->t,
                         w->part);
    }
    if (c->P.order == 2 || c->w64_mixed) {
      HIPCHK(hipGetLastError());
      std::vector<double> part(gr);
      HIPCHK(hipMemcpyAsync(part.data(), w->part, gr * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double ss = 0.0;
      for (double v : part) ss += v;
      const double bn = w->sc_host->bnorm;
      fp64ref = bn > 0.0 ? sqrt(ss) / bn : 0.0;
    }
  }
  if (st) st->rel_resid_fp64ref = fp64ref;
  if (c->P.periodic) { // phi of volume-weighted mean 0
    APCCHK(vol_mean(c, w->x, s));
    hipLaunchKernelGGL(k_sub_mean, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n,
                       (const double *)&c->scratch->pmean, w->x);
  }
  hipLaunchKernelGGL(k_write_out, dim3(grid_for(c->n + c->nb)), dim3(APC_BLOCK), 0, s, c->n, c->nb,
                     w->x, g, phi);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(w->e1, s));
  HIPCHK(hipEventSynchronize(w->e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, w->e0, w->e1));
  if (st) {
    st->ms = ms;
    unsigned long long nf = 0;
    HIPCHK(hipMemcpy(&nf, &c->scratch->nfp64, sizeof(nf), hipMemcpyDeviceToHost));
    c->n_fp64_rows = (int64_t)nf;
    st->n_fp64_rows = c->n_fp64_rows;
  }
  return rc;
}

int apc_apply_impl(apc_cloud *c, const double *f, double *out, hipStream_t s) {
  if (!c->assembled) return APC_EINVAL;
  const Op op = make_op(c, false);
  // f has n+nb entries: boundary values take part as given (no zero tail here)
  if (c->P.precision != APC_FP64)
    hipLaunchKernelGGL(k_apply<V32A64>, dim3(spmv_grid(c)), dim3(APC_BLOCK), op_lds(op), s, op, f, out);
  else
    hipLaunchKernelGGL(k_apply<V64>, dim3(spmv_grid(c)), dim3(APC_BLOCK), op_lds(op), s, op, f, out);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_apply_precond_impl(apc_cloud *c, int precond, const double *in, double *out,
                           hipStream_t s) {
  if (!c->assembled) return APC_EINVAL;
  if (precond == APC_PRECOND_LEARNED) {
    if (!c->learned) return APC_EINVAL;
    if (c->nsl > 0) {
      const Op op = make_op(c, false);
      hipLaunchKernelGGL(k_prec_apply, dim3(spmv_grid(c)), dim3(APC_BLOCK), op_lds(op), s, op,
                         MOp{c->m_diag, c->m_sell, c->m_tmpl, c->P.order == 4 ? 42 : 26}, in, out, (const Scal *)nullptr);
    }
  } else if (precond == APC_PRECOND_JACOBI || precond == APC_PRECOND_NONE) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, in,
                       precond == APC_PRECOND_JACOBI ? (const double *)c->inv_diag : nullptr, out);
  } else {
    return APC_EINVAL;
  }
  HIPCHK(hipGetLastError());
  return APC_OK;
}

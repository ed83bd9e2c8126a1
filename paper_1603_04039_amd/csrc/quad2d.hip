// Two-dimensional AP-Cloud field solve (the quadtree variant of Sec. 5.1), k = 2:
// quadtree node selection (Sec. 4: error balance, 2:1 face balance, boundary face
// nodes), quadrant-criterion stencils (Sec. 3.1), second-order least squares with
// 5 unknowns, NGP deposit and density rows (Sec. 3.2), Poisson rows, BiCGSTAB,
// derivatives and Taylor interpolation.  Clouds of this variant are small (the
// paper's reach 1e4 - 1e5 nodes), so the kernels are one thread per node or
// particle, and the solver keeps its scalars on the device (one read of the
// state per chunk of iterations).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "apc_internal.h"

namespace {

constexpr int Q5 = 5;        // unknowns: x, y, x^2/2, xy, y^2/2
constexpr int Q15 = 15;      // packed lower triangle of the 5 x 5 Gram matrix
constexpr int M2MAX = 64;    // stencil size cap
constexpr int RING2 = 1024;  // ring list capacity per node (an R <= 5 ring holds far fewer)
constexpr int HASH2 = 2048;  // its hash set
constexpr int64_t CHUNK2 = 16384;

__host__ __device__ inline uint64_t spread2(uint64_t v) {
  v &= 0xffffffffull;
  v = (v | (v << 16)) & 0x0000ffff0000ffffull;
  v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
  v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}
__host__ __device__ inline uint32_t compact2(uint64_t v) {
  v &= 0x5555555555555555ull;
  v = (v | (v >> 1)) & 0x3333333333333333ull;
  v = (v | (v >> 2)) & 0x0f0f0f0f0f0f0f0full;
  v = (v | (v >> 4)) & 0x00ff00ff00ff00ffull;
  v = (v | (v >> 8)) & 0x0000ffff0000ffffull;
  v = (v | (v >> 16)) & 0x00000000ffffffffull;
  return (uint32_t)v;
}
// x bit above the y bit at every level
__host__ __device__ inline uint64_t morton2(uint32_t x, uint32_t y) {
  return (spread2(x) << 1) | spread2(y);
}

template <typename T>
int dalloc2(T **p, int64_t n, hipStream_t s) {
  HIPCHK(apc_malloc_async((void **)p, (size_t)(n > 0 ? n : 1) * sizeof(T), s));
  return APC_OK;
}
template <typename T>
int dfree2(T *&p, hipStream_t s) {
  if (p) HIPCHK(apc_free_async(p, s));
  p = nullptr;
  return APC_OK;
}

// ---------------------------------------------------------------- build kernels
__global__ void __launch_bounds__(APC_BLOCK)
    q_keys(const double *__restrict__ xy, int64_t N, double lo0, double lo1, double L, double s,
           int D, uint64_t *__restrict__ keys, int32_t *__restrict__ vals, int *__restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= N) return;
  const double lo[2] = {lo0, lo1};
  const uint32_t top = (1u << D) - 1u;
  uint32_t u[2];
  int e = 0;
  for (int d = 0; d < 2; d++) {
    const double x = xy[(int64_t)d * N + i];
    if (isnan(x)) e |= 1;
    if (x < lo[d] || x > lo[d] + L) e |= 2;
    double q = floor((x - lo[d]) * s);
    if (!(q >= 0.0)) q = 0.0;
    if (q > (double)top) q = (double)top;
    u[d] = (uint32_t)q;
  }
  if (e) atomicOr(err, e);
  keys[i] = morton2(u[0], u[1]);
  vals[i] = (int32_t)i;
}

__global__ void __launch_bounds__(APC_BLOCK)
    q_gather(const double *__restrict__ xy, const int32_t *__restrict__ perm, int64_t N,
             double *__restrict__ sxy) {
  const int64_t s = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (s >= N) return;
  const int64_t i = perm[s];
  sxy[s] = xy[i];
  sxy[N + s] = xy[N + i];
}

struct QCells {
  uint64_t *pre = nullptr; // key prefix at the cell's level
  int32_t *lev = nullptr, *fst = nullptr, *cnt = nullptr, *flag = nullptr;
  int64_t n = 0;
};
int qcells_alloc(QCells &c, int64_t n, hipStream_t s) {
  c.n = n;
  APCCHK(dalloc2(&c.pre, n, s));
  APCCHK(dalloc2(&c.lev, n, s));
  APCCHK(dalloc2(&c.fst, n, s));
  APCCHK(dalloc2(&c.cnt, n, s));
  APCCHK(dalloc2(&c.flag, n, s));
  return APC_OK;
}
int qcells_free(QCells &c, hipStream_t s) {
  APCCHK(dfree2(c.pre, s));
  APCCHK(dfree2(c.lev, s));
  APCCHK(dfree2(c.fst, s));
  APCCHK(dfree2(c.cnt, s));
  APCCHK(dfree2(c.flag, s));
  c.n = 0;
  return APC_OK;
}

struct Thr2 {
  double T[24];
};

__global__ void __launch_bounds__(APC_BLOCK) q_sizes(const int32_t *flag, int64_t n, int32_t *sz) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) sz[i] = flag[i] ? 4 : 1;
}

// every flagged cell is replaced by its 4 children (Morton order keeps the list
// sorted), each with the sub-range of its parent's sorted particles carrying its
// prefix; with `criterion` a child is flagged when below max_depth with N' >= T_l
__global__ void __launch_bounds__(APC_BLOCK)
    q_expand(QCells in, const int32_t *__restrict__ off, const uint64_t *__restrict__ keys, int D,
             Thr2 thr, int criterion, QCells out) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= in.n) return;
  const int64_t o = off[i];
  if (!in.flag[i]) {
    out.pre[o] = in.pre[i];
    out.lev[o] = in.lev[i];
    out.fst[o] = in.fst[i];
    out.cnt[o] = in.cnt[i];
    out.flag[o] = 0;
    return;
  }
  const int l = in.lev[i] + 1, sh = 2 * (D - l);
  const int64_t a1 = (int64_t)in.fst[i] + in.cnt[i];
  int64_t a = in.fst[i];
  for (int c = 0; c < 4; c++) {
    const uint64_t cp = in.pre[i] * 4ull + (uint64_t)c;
    const int64_t b = apc_lower_bound(keys, a, a1, (cp + 1ull) << sh);
    out.pre[o + c] = cp;
    out.lev[o + c] = l;
    out.fst[o + c] = (int32_t)a;
    out.cnt[o + c] = (int32_t)(b - a);
    out.flag[o + c] = criterion ? (l < D && (double)(b - a) >= thr.T[l]) : 0;
    a = b;
  }
}

int q_expand_all(QCells &c, const uint64_t *keys, int D, const Thr2 &thr, int criterion,
                 hipStream_t s) {
  int32_t *sz = nullptr, *off = nullptr;
  APCCHK(dalloc2(&sz, c.n, s));
  APCCHK(dalloc2(&off, c.n, s));
  hipLaunchKernelGGL(q_sizes, dim3(grid_for(c.n)), dim3(APC_BLOCK), 0, s, c.flag, c.n, sz);
  APCCHK(apc_scan_i32(sz, off, c.n, s));
  int32_t last[2];
  HIPCHK(hipMemcpyAsync(&last[0], off + c.n - 1, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&last[1], sz + c.n - 1, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  QCells o;
  APCCHK(qcells_alloc(o, (int64_t)last[0] + last[1], s));
  hipLaunchKernelGGL(q_expand, dim3(grid_for(c.n)), dim3(APC_BLOCK), 0, s, c, off, keys, D, thr,
                     criterion, o);
  HIPCHK(hipGetLastError());
  APCCHK(dfree2(sz, s));
  APCCHK(dfree2(off, s));
  APCCHK(qcells_free(c, s));
  c = o;
  return APC_OK;
}

__global__ void __launch_bounds__(APC_BLOCK)
    q_mincorner(const uint64_t *pre, const int32_t *lev, int64_t n, int D, uint64_t *mc) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) mc[i] = pre[i] << (2 * (D - lev[i]));
}

// the same-level cell across face f of cell (t, l); false on the domain boundary
__device__ inline bool q_across(const uint32_t t0[2], int l, int f, uint32_t t[2]) {
  const int d = f >> 1;
  const uint32_t top = (1u << l) - 1u;
  t[0] = t0[0];
  t[1] = t0[1];
  if (f & 1) {
    if (t[d] == top) return false;
    t[d]++;
  } else {
    if (t[d] == 0u) return false;
    t[d]--;
  }
  return true;
}

// 2:1 balance: a leaf of level l marks every face-neighbouring leaf coarser than
// l - 1 (the leaf holding the minimum corner of the same-level cell across)
__global__ void __launch_bounds__(APC_BLOCK)
    q_balance_mark(const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev,
                   const uint64_t *__restrict__ mc, int64_t n, int D, int32_t *__restrict__ mark) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int l = lev[y];
  if (l < 2) return;
  const uint32_t t0[2] = {compact2(pre[y] >> 1), compact2(pre[y])};
  for (int f = 0; f < 4; f++) {
    uint32_t t[2];
    if (!q_across(t0, l, f, t)) continue;
    const int sh = D - l;
    const int64_t z = apc_last_le(mc, n, morton2(t[0] << sh, t[1] << sh));
    if (lev[z] < l - 1) mark[z] = 1;
  }
}

__global__ void __launch_bounds__(APC_BLOCK)
    q_bcount(const uint64_t *pre, const int32_t *lev, int64_t n, int32_t *bc) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const uint32_t t0[2] = {compact2(pre[y] >> 1), compact2(pre[y])};
  int k = 0;
  for (int f = 0; f < 4; f++) {
    uint32_t t[2];
    k += !q_across(t0, lev[y], f, t);
  }
  bc[y] = k;
}

// node coordinates in units of L 2^-(D+1): a level-l cell of index i is centred at
// (2i+1) 2^(D-l); boundary nodes at the centre of their owner's boundary face
__global__ void __launch_bounds__(APC_BLOCK)
    q_nodes(const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev,
            const int32_t *__restrict__ bstart, int64_t n, int64_t ntot, int D,
            int32_t *__restrict__ crd, int32_t *__restrict__ bowner, int32_t *__restrict__ bface) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int l = lev[y];
  const uint32_t t0[2] = {compact2(pre[y] >> 1), compact2(pre[y])};
  const int32_t sz = 1 << (D - l);
  const int32_t c[2] = {(int32_t)(2u * t0[0] + 1u) * sz, (int32_t)(2u * t0[1] + 1u) * sz};
  crd[y] = c[0];
  crd[ntot + y] = c[1];
  int64_t b = n + bstart[y];
  for (int f = 0; f < 4; f++) {
    uint32_t t[2];
    if (q_across(t0, l, f, t)) continue;
    const int d = f >> 1;
    crd[b] = c[0];
    crd[ntot + b] = c[1];
    crd[(int64_t)d * ntot + b] = c[d] + ((f & 1) ? sz : -sz);
    bowner[b - n] = (int32_t)y;
    bface[b - n] = f;
    b++;
  }
}

// 1-ring: per face the neighbouring leaf if not finer, else the 2 leaves of level
// l + 1 on the shared face; a boundary face gives the boundary node
__global__ void __launch_bounds__(APC_BLOCK)
    q_ring1(const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev,
            const uint64_t *__restrict__ mc, const int32_t *__restrict__ bstart, int64_t n, int D,
            int32_t *__restrict__ r1cnt, int32_t *__restrict__ r1, int *__restrict__ err) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int l = lev[y];
  const uint32_t t0[2] = {compact2(pre[y] >> 1), compact2(pre[y])};
  int32_t *out = r1 + y * 8;
  int k = 0, kb = 0;
  for (int f = 0; f < 4; f++) {
    uint32_t t[2];
    if (!q_across(t0, l, f, t)) {
      out[k++] = (int32_t)(n + bstart[y] + kb++);
      continue;
    }
    const int sh = D - l;
    const int64_t z = apc_last_le(mc, n, morton2(t[0] << sh, t[1] << sh));
    if (lev[z] <= l) {
      out[k++] = (int32_t)z;
      continue;
    }
    if (l + 1 > D) {
      atomicOr(err, 4);
      continue;
    }
    const int d = f >> 1, side = (f & 1) ? 0 : 1;
    for (int a = 0; a < 2; a++) {
      uint32_t u[2];
      u[d] = 2u * t[d] + (uint32_t)side;
      u[1 - d] = 2u * t[1 - d] + (uint32_t)a;
      const int sh1 = D - l - 1;
      const uint64_t pc = morton2(u[0] << sh1, u[1] << sh1);
      const int64_t zc = apc_last_le(mc, n, pc);
      if (lev[zc] != l + 1 || mc[zc] != pc) atomicOr(err, 4);
      out[k++] = (int32_t)zc;
    }
  }
  r1cnt[y] = k;
}

__global__ void __launch_bounds__(APC_BLOCK)
    q_pnode(int64_t n, const int32_t *__restrict__ first, const int32_t *__restrict__ count,
            int32_t *__restrict__ pnode) {
  const int64_t j = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (j >= n) return;
  for (int32_t s = first[j]; s < first[j] + count[j]; s++) pnode[s] = (int32_t)j;
}

// ---------------------------------------------------------------- the fit
__device__ __forceinline__ int tri5(int i, int j) { return i * (i + 1) / 2 + j; } // j <= i

struct Geo2 {
  int32_t c0, c1;
  double h, r2max;
};
__device__ inline Geo2 geo2(const int32_t *nb, int m, const int32_t *__restrict__ crd,
                            int64_t ntot, int64_t y) {
  Geo2 g;
  g.c0 = crd[y];
  g.c1 = crd[ntot + y];
  int64_t h = 0, r2 = 0;
  for (int j = 0; j < m; j++) {
    const int64_t d0 = (int64_t)crd[nb[j]] - g.c0, d1 = (int64_t)crd[ntot + nb[j]] - g.c1;
    h = max(h, max(d0 < 0 ? -d0 : d0, d1 < 0 ? -d1 : d1));
    r2 = max(r2, d0 * d0 + d1 * d1);
  }
  g.h = (double)h;
  g.r2max = (double)r2;
  return g;
}
// monomial row and squared weight of neighbour v
__device__ inline double row2(const Geo2 &g, const int32_t *__restrict__ crd, int64_t ntot,
                              int32_t v, double r[Q5]) {
  const int64_t d0 = (int64_t)crd[v] - g.c0, d1 = (int64_t)crd[ntot + v] - g.c1;
  const double x = (double)d0 / g.h, y = (double)d1 / g.h;
  r[0] = x;
  r[1] = y;
  r[2] = 0.5 * x * x;
  r[3] = x * y;
  r[4] = 0.5 * y * y;
  const double e4 = 0.018315638888734179; // exp(-4)
  const double W = (exp(-(double)(d0 * d0 + d1 * d1) / g.r2max) - e4) / (1.0 - e4);
  return W * W;
}
// normal equations G = sum W^2 v v^T, Cholesky in place; min/max diag(L) (0 if not SPD)
__device__ inline double gram_chol5(const int32_t *nb, int m, const Geo2 &g,
                                    const int32_t *__restrict__ crd, int64_t ntot, double G[Q15]) {
  for (int k = 0; k < Q15; k++) G[k] = 0.0;
  for (int j = 0; j < m; j++) {
    double r[Q5];
    const double w2 = row2(g, crd, ntot, nb[j], r);
    for (int a = 0; a < Q5; a++)
      for (int b = 0; b <= a; b++) G[tri5(a, b)] += w2 * r[a] * r[b];
  }
  double dmin = 1e300, dmax = 0.0;
  bool ok = true;
  for (int i = 0; i < Q5; i++)
    for (int j = 0; j <= i; j++) {
      double s = G[tri5(i, j)];
      for (int k = 0; k < j; k++) s -= G[tri5(i, k)] * G[tri5(j, k)];
      if (i == j) {
        ok = ok && s > 0.0;
        const double d = sqrt(s > 0.0 ? s : 0.0);
        G[tri5(i, i)] = d;
        dmin = fmin(dmin, d);
        dmax = fmax(dmax, d);
      } else {
        const double dj = G[tri5(j, j)];
        G[tri5(i, j)] = dj > 0.0 ? s / dj : 0.0;
      }
    }
  return (ok && dmax > 0.0) ? dmin / dmax : 0.0;
}
__device__ inline void chol_solve5(const double L[Q15], double z[Q5]) {
  for (int i = 0; i < Q5; i++) {
    double s = z[i];
    for (int k = 0; k < i; k++) s -= L[tri5(i, k)] * z[k];
    z[i] = s / L[tri5(i, i)];
  }
  for (int i = Q5 - 1; i >= 0; i--) {
    double s = z[i];
    for (int k = i + 1; k < Q5; k++) s -= L[tri5(k, i)] * z[k];
    z[i] = s / L[tri5(i, i)];
  }
}

// ---------------------------------------------------------------- stencils
__device__ inline bool in_quad2(int q, int64_t dx, int64_t dy) {
  const int sx = (q >> 1) & 1 ? 1 : -1, sy = q & 1 ? 1 : -1;
  return sx * dx >= 0 && sy * dy >= 0;
}
__device__ inline bool key_less(int64_t r2a, int32_t ia, int64_t r2b, int32_t ib) {
  return r2a < r2b || (r2a == r2b && ia < ib);
}

// One thread per node of a chunk: the R-ring (R from ring_min up) by a BFS over the
// 1-ring (boundary nodes hang off their owner) in the thread's scratch (list and an
// open-addressing set, element-major), then the quadrant criterion: per closed
// quadrant its two nearest candidates by (r^2, index), then the nearest remaining
// ones up to min(count, m_cap); accepted when every closed quadrant holds a chosen
// node, m >= 6 and the normal equations' Cholesky has min/max diag >= 1e-6.  The
// chosen nodes go out in (r^2, index) order.  err: 8 ring too large, 16 no stencil.
__global__ void __launch_bounds__(APC_BLOCK)
    q_stencil(int64_t y0, int64_t cnt, int64_t n, const int32_t *__restrict__ r1off,
              const int32_t *__restrict__ r1, const int32_t *__restrict__ bowner,
              const int32_t *__restrict__ crd, int64_t ntot, int ring_min, int ring_max,
              int m_cap, int32_t *__restrict__ lst_all, int32_t *__restrict__ hash_all,
              int32_t *__restrict__ mout, int32_t *__restrict__ sout, int32_t *__restrict__ rout,
              int *__restrict__ err) {
  const int64_t t = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (t >= cnt) return;
  const int64_t y = y0 + t;
  const int64_t stride = cnt;
  int32_t *lst = lst_all + t;
  int32_t *tab = hash_all + t;
#define LST2(k) lst[(int64_t)(k) * stride]
#define TAB2(k) tab[(int64_t)(k) * stride]
  const int64_t cy0 = crd[y], cy1 = crd[ntot + y];
  for (int R = ring_min; R <= ring_max; R++) {
    for (int k = 0; k < HASH2; k++) TAB2(k) = -1;
    auto insert = [&](int32_t v) -> bool {
      uint32_t hh = ((uint32_t)v * 2654435761u) & (HASH2 - 1);
      for (;;) {
        const int32_t e = TAB2(hh);
        if (e < 0) {
          TAB2(hh) = v;
          return true;
        }
        if (e == v) return false;
        hh = (hh + 1) & (HASH2 - 1);
      }
    };
    int nf = 0, lo = 0;
    insert((int32_t)y);
    LST2(nf++) = (int32_t)y;
    bool over = false;
    for (int depth = 1; depth <= R && !over; depth++) {
      const int hi = nf;
      for (int q = lo; q < hi && !over; q++) {
        const int32_t u = LST2(q);
        auto visit = [&](int32_t v) {
          if (insert(v)) {
            if (nf >= RING2 || nf >= HASH2 / 2) over = true;
            else LST2(nf++) = v;
          }
        };
        if (u >= n) {
          visit(bowner[u - n]);
        } else {
          for (int32_t a = r1off[u]; a < r1off[u + 1] && !over; a++) visit(r1[a]);
        }
      }
      lo = hi;
    }
    if (over) {
      atomicOr(err, 8);
      mout[y] = 0;
      return;
    }
    // candidates: list entries 1 .. nf-1
    const int want = (nf - 1) < m_cap ? (nf - 1) : m_cap;
    int32_t pick[M2MAX];
    int got = 0;
    auto picked = [&](int32_t v) {
      for (int k = 0; k < got; k++)
        if (pick[k] == v) return true;
      return false;
    };
    auto r2of = [&](int32_t v) {
      const int64_t d0 = (int64_t)crd[v] - cy0, d1 = (int64_t)crd[ntot + v] - cy1;
      return d0 * d0 + d1 * d1;
    };
    for (int q = 0; q < 4; q++) {
      // the two nearest candidates in the closed quadrant
      int32_t b1 = -1, b2 = -1;
      int64_t k1 = 0, k2 = 0;
      for (int i = 1; i < nf; i++) {
        const int32_t v = LST2(i);
        if (!in_quad2(q, (int64_t)crd[v] - cy0, (int64_t)crd[ntot + v] - cy1)) continue;
        const int64_t r2 = r2of(v);
        if (b1 < 0 || key_less(r2, v, k1, b1)) {
          b2 = b1;
          k2 = k1;
          b1 = v;
          k1 = r2;
        } else if (b2 < 0 || key_less(r2, v, k2, b2)) {
          b2 = v;
          k2 = r2;
        }
      }
      if (b1 >= 0 && got < want && !picked(b1)) pick[got++] = b1;
      if (b2 >= 0 && got < want && !picked(b2)) pick[got++] = b2;
    }
    while (got < want) { // the nearest remaining candidate
      int32_t best = -1;
      int64_t kb = 0;
      for (int i = 1; i < nf; i++) {
        const int32_t v = LST2(i);
        if (picked(v)) continue;
        const int64_t r2 = r2of(v);
        if (best < 0 || key_less(r2, v, kb, best)) {
          best = v;
          kb = r2;
        }
      }
      if (best < 0) break;
      pick[got++] = best;
    }
    // in (r^2, index) order
    for (int a = 1; a < got; a++) {
      const int32_t v = pick[a];
      const int64_t rv = r2of(v);
      int b = a - 1;
      while (b >= 0 && key_less(rv, v, r2of(pick[b]), pick[b])) {
        pick[b + 1] = pick[b];
        b--;
      }
      pick[b + 1] = v;
    }
    bool ok = got >= Q5 + 1;
    for (int q = 0; q < 4 && ok; q++) {
      bool any = false;
      for (int k = 0; k < got; k++)
        any = any || in_quad2(q, (int64_t)crd[pick[k]] - cy0, (int64_t)crd[ntot + pick[k]] - cy1);
      ok = any;
    }
    if (ok) {
      const Geo2 g = geo2(pick, got, crd, ntot, y);
      double G[Q15];
      ok = gram_chol5(pick, got, g, crd, ntot, G) >= 1e-6;
    }
    if (ok) {
      for (int k = 0; k < got; k++) sout[y * M2MAX + k] = pick[k];
      mout[y] = got;
      rout[y] = R;
      return;
    }
  }
  atomicOr(err, 16);
  mout[y] = 0;
#undef LST2
#undef TAB2
}

__global__ void __launch_bounds__(APC_BLOCK)
    q_st_copy(int64_t n, const int32_t *__restrict__ sout, const int32_t *__restrict__ off,
              const int32_t *__restrict__ m, int32_t *__restrict__ st_idx) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  for (int k = 0; k < m[y]; k++) st_idx[off[y] + k] = sout[y * M2MAX + k];
}

// ---------------------------------------------------------------- assembly
// Laplacian row: z = G^-1 (e_xx + e_yy), w_j = W_j^2 (v_j . z) / (h unit)^2, diagonal
// -sum w; density row b = hs w with hs = h_c^2 / 24 (the NGP cell average of the
// fitted quadratic), kept when hs sum |w| <= (1 - hs sum w) / 2, else the identity
// row (hs = 0)
__global__ void __launch_bounds__(APC_BLOCK)
    q_fit(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
          const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
          double unit, double L, double *__restrict__ w, double *__restrict__ diag,
          double *__restrict__ hs, int8_t *__restrict__ dord, int *__restrict__ err) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int32_t a = st_off[y];
  const int m = st_off[y + 1] - a;
  const int32_t *nb = st_idx + a;
  const Geo2 g = geo2(nb, m, crd, ntot, y);
  double G[Q15];
  if (!(gram_chol5(nb, m, g, crd, ntot, G) > 0.0)) atomicOr(err, 1);
  double z[Q5] = {0.0, 0.0, 1.0, 0.0, 1.0};
  chol_solve5(G, z);
  const double hp = g.h * unit, ih2 = 1.0 / (hp * hp);
  double sum = 0.0, asum = 0.0;
  for (int j = 0; j < m; j++) {
    double r[Q5];
    const double w2 = row2(g, crd, ntot, nb[j], r);
    double dv = 0.0;
    for (int k = 0; k < Q5; k++) dv += r[k] * z[k];
    const double v = w2 * dv * ih2;
    w[a + j] = v;
    sum += v;
    asum += fabs(v);
  }
  diag[y] = -sum;
  const double hc = L / (double)(1 << level[y]);
  const double h = hc * hc / 24.0;
  const bool ok = h * asum <= 0.5 * (1.0 - h * sum);
  hs[y] = ok ? h : 0.0;
  dord[y] = ok ? 2 : 0;
}

// derivatives of the fitted quadratic (physical units): phi_x, phi_y, phi_xx,
// phi_xy, phi_yy
__global__ void __launch_bounds__(APC_BLOCK)
    q_derivs(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
             const int32_t *__restrict__ crd, int64_t ntot, double unit,
             const double *__restrict__ f, double *__restrict__ D) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int32_t a = st_off[y];
  const int m = st_off[y + 1] - a;
  const int32_t *nb = st_idx + a;
  const Geo2 g = geo2(nb, m, crd, ntot, y);
  double G[Q15], z[Q5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  gram_chol5(nb, m, g, crd, ntot, G);
  const double f0 = f[y];
  for (int j = 0; j < m; j++) {
    double r[Q5];
    const double w2 = row2(g, crd, ntot, nb[j], r);
    const double df = w2 * (f[nb[j]] - f0);
    for (int k = 0; k < Q5; k++) z[k] += r[k] * df;
  }
  chol_solve5(G, z);
  const double hp = g.h * unit;
  for (int k = 0; k < Q5; k++) D[y * Q5 + k] = z[k] / (k < 2 ? hp : hp * hp);
}

__global__ void __launch_bounds__(APC_BLOCK)
    q_interp(int64_t N, const double *__restrict__ sxy, const int32_t *__restrict__ perm,
             const int32_t *__restrict__ pnode, const int32_t *__restrict__ crd, int64_t ntot,
             double lo0, double lo1, double unit, const double *__restrict__ phi,
             const double *__restrict__ D, double *__restrict__ phi_p, double *__restrict__ grad) {
  const int64_t s = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (s >= N) return;
  const int32_t j = pnode[s];
  const double x = sxy[s] - (lo0 + unit * (double)crd[j]);
  const double y = sxy[N + s] - (lo1 + unit * (double)crd[ntot + j]);
  const double *d = D + (int64_t)j * Q5;
  const int64_t i = perm[s];
  phi_p[i] = phi[j] + d[0] * x + d[1] * y + d[2] * (0.5 * x * x) + d[3] * (x * y) +
             d[4] * (0.5 * y * y);
  grad[i] = d[0] + d[2] * x + d[3] * y;
  grad[N + i] = d[1] + d[3] * x + d[4] * y;
}

__global__ void __launch_bounds__(APC_BLOCK)
    q_deposit(int64_t n, int64_t N, const int32_t *__restrict__ first,
              const int32_t *__restrict__ count, const int32_t *__restrict__ level,
              const int32_t *__restrict__ perm, const double *__restrict__ q, double L,
              const int32_t *__restrict__ bowner, int64_t nb, double *__restrict__ rho) {
  const int64_t j = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (j < n) {
    double sum;
    if (q) {
      sum = 0.0;
      for (int32_t s = first[j]; s < first[j] + count[j]; s++) sum += q[perm[s]];
    } else {
      sum = (double)count[j] * (1.0 / (double)N);
    }
    const double hc = L / (double)(1 << level[j]);
    rho[j] = sum / (hc * hc);
  }
}
__global__ void __launch_bounds__(APC_BLOCK)
    q_bnd_copy(int64_t n, int64_t nb, const int32_t *__restrict__ bowner, double *__restrict__ v) {
  const int64_t b = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (b < nb) v[n + b] = v[bowner[b]];
}

// ---------------------------------------------------------------- solver
// y = A x over the interior rows, x with a zero boundary tail: Poisson
// sum_j w_ij (x_j - x_i); density (hs != null) x_i + hs_i sum_j w_ij (x_j - x_i)
__global__ void __launch_bounds__(APC_BLOCK)
    q_apply(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
            const double *__restrict__ w, const double *__restrict__ hs,
            const double *__restrict__ x, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i];
  double s = 0.0;
  for (int32_t e = st_off[i]; e < st_off[i + 1]; e++) s += w[e] * (x[st_idx[e]] - xi);
  y[i] = hs ? xi + hs[i] * s : s;
}
// b = c src - (hs) sum over boundary columns w_ij bval_j
__global__ void __launch_bounds__(APC_BLOCK)
    q_rhs(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
          const double *__restrict__ w, const double *__restrict__ hs,
          const double *__restrict__ src, double c, const double *__restrict__ bval,
          double *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  if (bval)
    for (int32_t e = st_off[i]; e < st_off[i + 1]; e++)
      if (st_idx[e] >= n) acc += w[e] * bval[st_idx[e] - n];
  b[i] = c * src[i] - (hs ? hs[i] * acc : acc);
}
// per-block partial sums of a . b
__global__ void __launch_bounds__(APC_BLOCK)
    q_dot(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
          double *__restrict__ part) {
  __shared__ double sh[APC_BLOCK];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * APC_BLOCK)
    s += a[i] * b[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = APC_BLOCK / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
// y = a x + b y (element-wise, optional scaling by 1/d)
__global__ void __launch_bounds__(APC_BLOCK)
    q_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
__global__ void __launch_bounds__(APC_BLOCK)
    q_pupdate(int64_t n, const double *__restrict__ r, double beta, double omega,
              const double *__restrict__ v, double *__restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}
__global__ void __launch_bounds__(APC_BLOCK)
    q_scale(int64_t n, const double *__restrict__ x, const double *__restrict__ dinv,
            double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) y[i] = dinv ? x[i] * dinv[i] : x[i];
}
__global__ void __launch_bounds__(APC_BLOCK)
    q_inv(int64_t n, const double *__restrict__ d, double *__restrict__ dinv) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) dinv[i] = 1.0 / d[i];
}
__global__ void __launch_bounds__(APC_BLOCK)
    q_write_out(int64_t n, int64_t nb, const double *__restrict__ x,
                const double *__restrict__ bval, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) out[i] = x[i];
  else if (i < n + nb) out[i] = bval ? bval[i - n] : 0.0;
}

// ---- BiCGSTAB with its scalars on the device: each step is a kernel that returns
// at once when the solve has stopped, so the host launches iterations in chunks
// and reads the state once per chunk.  done: 0 running, 1 recursive residual
// below tol (or omega = 0), 2 breakdown (rho or (rh, v) zero or not finite),
// 3 iteration limit.
struct Scal2 {
  double rho, alpha, omega, beta, bnorm, tol, rnorm;
  int it, maxit, done;
};
constexpr unsigned G2 = 1024; // blocks of the reducing kernels (partials per value)

template <int K>
__device__ __forceinline__ void q_partials(double (&v)[K], double *part) {
  __shared__ double sh[K][APC_BLOCK / 64];
#pragma unroll
  for (int k = 0; k < K; k++) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double x = 0.0;
    for (int w = 0; w < APC_BLOCK / 64; w++) x += sh[threadIdx.x][w];
    part[threadIdx.x * G2 + blockIdx.x] = x;
  }
}
template <int K>
__device__ __forceinline__ void q_fin(const double *part, unsigned G, double (&out)[K]) {
  __shared__ double sh[K][APC_BLOCK];
#pragma unroll
  for (int k = 0; k < K; k++) {
    double x = 0.0;
    for (unsigned b = threadIdx.x; b < G; b += APC_BLOCK) x += part[k * G2 + b];
    sh[k][threadIdx.x] = x;
  }
  __syncthreads();
  for (int h = APC_BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int k = 0; k < K; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + h];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < K; k++) out[k] = sh[k][0];
}

// partials of (a, b) over n
__global__ void __launch_bounds__(APC_BLOCK)
    q_dotp(int64_t n, const double *__restrict__ a, const double *__restrict__ b, double *part) {
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * APC_BLOCK)
    v[0] += a[i] * b[i];
  q_partials<1>(v, part);
}
// (re)start from r (rh = r, p = v = 0 before this): rho = (r, r); first call sets
// the norm of b from the same sum (r = b there)
__global__ void __launch_bounds__(APC_BLOCK)
    q_fin_start(const double *part, unsigned G, Scal2 *sc, double tol, int maxit, int first) {
  double o[1];
  q_fin<1>(part, G, o);
  if (threadIdx.x == 0) {
    if (first) {
      sc->bnorm = sqrt(o[0]);
      sc->tol = tol;
      sc->maxit = maxit;
      sc->it = 0;
    }
    sc->rho = o[0];
    sc->alpha = sc->omega = 1.0;
    sc->beta = 0.0;
    sc->rnorm = sqrt(o[0]);
    sc->done = (o[0] == 0.0 || !isfinite(o[0])) ? 2 : (sc->it >= sc->maxit ? 3 : 0);
  }
}
// p = r + beta (p - omega v); ph = dinv p (when scaled)
__global__ void __launch_bounds__(APC_BLOCK)
    q_upd_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
            const double *__restrict__ v, const double *__restrict__ dinv, double *__restrict__ ph,
            const Scal2 *sc) {
  if (sc->done) return;
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double pi = r[i] + sc->beta * (p[i] - sc->omega * v[i]);
  p[i] = pi;
  if (dinv) ph[i] = pi * dinv[i];
}
// y = A x and partials (a, y) [, (y, y)]
template <int K>
__global__ void __launch_bounds__(APC_BLOCK)
    q_spmv_dot(int64_t n, const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
               const double *__restrict__ w, const double *__restrict__ hs,
               const double *__restrict__ x, double *__restrict__ y, const double *__restrict__ a,
               double *part, const Scal2 *sc) {
  if (sc->done) return;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; k++) v[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * APC_BLOCK) {
    const double xi = x[i];
    double acc = 0.0;
    for (int32_t e = st_off[i]; e < st_off[i + 1]; e++) acc += w[e] * (x[st_idx[e]] - xi);
    const double yi = hs ? xi + hs[i] * acc : acc;
    y[i] = yi;
    v[0] += a[i] * yi;
    if (K > 1) v[K - 1] += yi * yi;
  }
  q_partials<K>(v, part);
}
// alpha = rho / (rh, v)
__global__ void __launch_bounds__(APC_BLOCK) q_fin_alpha(const double *part, unsigned G, Scal2 *sc) {
  if (sc->done) return;
  double o[1];
  q_fin<1>(part, G, o);
  if (threadIdx.x == 0) {
    const double al = sc->rho / o[0];
    if (o[0] == 0.0 || !isfinite(al)) {
      sc->done = 2;
      sc->it += 1; // the iteration that broke down counts
    } else {
      sc->alpha = al;
    }
  }
}
// s = r - alpha v; sh = dinv s (when scaled)
__global__ void __launch_bounds__(APC_BLOCK)
    q_upd_s(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
            double *__restrict__ sv, const double *__restrict__ dinv, double *__restrict__ sh,
            const Scal2 *sc) {
  if (sc->done) return;
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double si = r[i] - sc->alpha * v[i];
  sv[i] = si;
  if (dinv) sh[i] = si * dinv[i];
}
// omega = (t, s) / (t, t)
__global__ void __launch_bounds__(APC_BLOCK) q_fin_omega(const double *part, unsigned G, Scal2 *sc) {
  if (sc->done) return;
  double o[2];
  q_fin<2>(part, G, o);
  if (threadIdx.x == 0) sc->omega = o[1] > 0.0 ? o[0] / o[1] : 0.0;
}
// x += alpha ph + omega sh; r = s - omega t; partials (rh, r), (r, r)
__global__ void __launch_bounds__(APC_BLOCK)
    q_upd_xr(int64_t n, double *__restrict__ x, const double *__restrict__ ph,
             const double *__restrict__ sh, const double *__restrict__ sv,
             const double *__restrict__ t, double *__restrict__ r, const double *__restrict__ rh,
             double *part, const Scal2 *sc) {
  if (sc->done) return;
  const double al = sc->alpha, om = sc->omega;
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * APC_BLOCK) {
    x[i] += al * ph[i] + om * sh[i];
    const double ri = sv[i] - om * t[i];
    r[i] = ri;
    v[0] += rh[i] * ri;
    v[1] += ri * ri;
  }
  q_partials<2>(v, part);
}
// rho' = (rh, r), ||r||: convergence test, then beta for the next iteration
__global__ void __launch_bounds__(APC_BLOCK) q_fin_rho(const double *part, unsigned G, Scal2 *sc) {
  if (sc->done) return;
  double o[2];
  q_fin<2>(part, G, o);
  if (threadIdx.x == 0) {
    const double rho_new = o[0], om = sc->omega;
    sc->it += 1;
    sc->rnorm = sqrt(o[1]);
    if (sc->rnorm <= sc->tol * sc->bnorm || om == 0.0) {
      sc->done = 1;
    } else if (rho_new == 0.0 || !isfinite(rho_new)) {
      sc->done = 2;
    } else if (sc->it >= sc->maxit) {
      sc->done = 3;
    } else {
      sc->beta = (rho_new / sc->rho) * (sc->alpha / om);
      sc->rho = rho_new;
    }
  }
}

} // namespace

struct apc2_cloud {
  apc_params P;
  int device = 0;
  int64_t N = 0, n = 0, nb = 0, nnz = 0, n_opened = 0;
  double T[24];
  double unit = 0.0;
  int32_t *perm = nullptr, *pnode = nullptr;
  double *sxy = nullptr;
  uint64_t *code = nullptr;
  int32_t *level = nullptr, *first = nullptr, *count = nullptr;
  int32_t *crd = nullptr, *bowner = nullptr, *bface = nullptr;
  int32_t *st_off = nullptr, *st_idx = nullptr;
  double *w = nullptr, *diag = nullptr, *hs = nullptr, *dinv = nullptr;
  int8_t *dord = nullptr;
  bool assembled = false;
  // solver vectors (n + nb long; the tail stays 0)
  double *vx = nullptr, *vr = nullptr, *vrh = nullptr, *vp = nullptr, *vv = nullptr,
         *vs = nullptr, *vt = nullptr, *vph = nullptr, *vsh = nullptr, *vb = nullptr,
         *part = nullptr;
  Scal2 *sc = nullptr;
};

namespace {

void free2(apc2_cloud *c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  void *ps[] = {c->perm, c->pnode, c->sxy, c->code, c->level, c->first, c->count, c->crd,
                c->bowner, c->bface, c->st_off, c->st_idx, c->w, c->diag, c->hs, c->dinv,
                c->dord, c->vx, c->vr, c->vrh, c->vp, c->vv, c->vs, c->vt, c->vph, c->vsh,
                c->vb, c->part, c->sc};
  for (void *q : ps)
    if (q) (void)apc_dev_free(q);
  delete c;
}

template <typename T>
int palloc(T **p, int64_t n) {
  HIPCHK(apc_dev_alloc((void **)p, (size_t)(n > 0 ? n : 1) * sizeof(T)));
  return APC_OK;
}

int build2(apc2_cloud *c, const double *xy, hipStream_t s) {
  const apc_params &P = c->P;
  const int D = P.max_depth;
  const int64_t N = c->N;
  Thr2 thr;
  for (int l = 0; l < 24; l++) thr.T[l] = c->T[l];
  uint64_t *keys = nullptr;
  int *err = nullptr;
  APCCHK(dalloc2(&keys, N, s));
  APCCHK(palloc(&c->perm, N));
  APCCHK(dalloc2(&err, 1, s));
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
  hipLaunchKernelGGL(q_keys, dim3(grid_for(N)), dim3(APC_BLOCK), 0, s, xy, N, P.lo[0], P.lo[1],
                     P.L, ldexp(1.0, D) / P.L, D, keys, c->perm, err);
  HIPCHK(hipGetLastError());
  int herr = 0;
  HIPCHK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (herr & 1) {
    apc_set_error_msg("non-finite particle coordinate");
    return APC_EINVAL;
  }
  if (herr & 2) {
    apc_set_error_msg("particle outside the domain");
    return APC_EDOMAIN;
  }
  APCCHK(apc_radix_sort(keys, c->perm, N, 2 * D, s));
  APCCHK(palloc(&c->sxy, 2 * N));
  hipLaunchKernelGGL(q_gather, dim3(grid_for(N)), dim3(APC_BLOCK), 0, s, xy, c->perm, N, c->sxy);
  // criterion, level by level
  QCells cl;
  APCCHK(qcells_alloc(cl, 1, s));
  {
    const uint64_t z = 0;
    const int32_t zi = 0, n32 = (int32_t)N;
    const int32_t op = (0 < D && (double)N >= c->T[0]) ? 1 : 0;
    HIPCHK(hipMemcpyAsync(cl.pre, &z, 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cl.lev, &zi, 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cl.fst, &zi, 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cl.cnt, &n32, 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cl.flag, &op, 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  int64_t opened = 0;
  for (;;) {
    int64_t nf = 0;
    APCCHK(apc_sum_i32(cl.flag, cl.n, &nf, s));
    if (nf == 0) break;
    opened += nf;
    APCCHK(q_expand_all(cl, keys, D, thr, 1, s));
  }
  // balance to its fixed point
  uint64_t *mc = nullptr;
  for (;;) {
    APCCHK(dfree2(mc, s));
    APCCHK(dalloc2(&mc, cl.n, s));
    hipLaunchKernelGGL(q_mincorner, dim3(grid_for(cl.n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev,
                       cl.n, D, mc);
    HIPCHK(hipMemsetAsync(cl.flag, 0, (size_t)cl.n * 4, s));
    hipLaunchKernelGGL(q_balance_mark, dim3(grid_for(cl.n)), dim3(APC_BLOCK), 0, s, cl.pre,
                       cl.lev, mc, cl.n, D, cl.flag);
    HIPCHK(hipGetLastError());
    int64_t nm = 0;
    APCCHK(apc_sum_i32(cl.flag, cl.n, &nm, s));
    if (nm == 0) break;
    opened += nm;
    APCCHK(q_expand_all(cl, keys, D, thr, 0, s));
  }
  const int64_t n = cl.n;
  c->n = n;
  c->n_opened = opened;
  APCCHK(palloc(&c->code, n));
  APCCHK(palloc(&c->level, n));
  APCCHK(palloc(&c->first, n));
  APCCHK(palloc(&c->count, n));
  HIPCHK(hipMemcpyAsync(c->code, mc, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->level, cl.lev, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->first, cl.fst, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->count, cl.cnt, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  APCCHK(palloc(&c->pnode, N));
  hipLaunchKernelGGL(q_pnode, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, n, c->first, c->count,
                     c->pnode);
  // boundary nodes
  int32_t *bcnt = nullptr, *bstart = nullptr;
  APCCHK(dalloc2(&bcnt, n, s));
  APCCHK(dalloc2(&bstart, n, s));
  hipLaunchKernelGGL(q_bcount, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev, n, bcnt);
  APCCHK(apc_scan_i32(bcnt, bstart, n, s));
  int32_t last[2];
  HIPCHK(hipMemcpyAsync(&last[0], bstart + n - 1, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&last[1], bcnt + n - 1, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t nb = (int64_t)last[0] + last[1];
  c->nb = nb;
  const int64_t ntot = n + nb;
  APCCHK(palloc(&c->crd, 2 * ntot));
  APCCHK(palloc(&c->bowner, nb));
  APCCHK(palloc(&c->bface, nb));
  hipLaunchKernelGGL(q_nodes, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev, bstart, n,
                     ntot, D, c->crd, c->bowner, c->bface);
  // 1-ring
  int32_t *r1cnt = nullptr, *r1off = nullptr, *r1 = nullptr;
  APCCHK(dalloc2(&r1cnt, n + 1, s));
  APCCHK(dalloc2(&r1off, n + 1, s));
  APCCHK(dalloc2(&r1, 8 * n, s));
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
  HIPCHK(hipMemsetAsync(r1cnt + n, 0, 4, s));
  hipLaunchKernelGGL(q_ring1, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev, mc, bstart,
                     n, D, r1cnt, r1, err);
  HIPCHK(hipGetLastError());
  // the 1-ring in CSR (8 slots per node, compacted by the scan of the counts)
  APCCHK(apc_scan_i32(r1cnt, r1off, n + 1, s));
  int32_t *r1c = nullptr;
  APCCHK(dalloc2(&r1c, 8 * n, s));
  {
    std::vector<int32_t> cnt(n), off(n + 1), slot((size_t)8 * n), out((size_t)8 * n);
    HIPCHK(hipMemcpyAsync(cnt.data(), r1cnt, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(off.data(), r1off, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(slot.data(), r1, (size_t)8 * n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (herr) {
      apc_set_error_msg("2:1 balance violated after the balance phase");
      return APC_EINVAL;
    }
    for (int64_t j = 0; j < n; j++)
      for (int k = 0; k < cnt[j]; k++) out[(size_t)off[j] + k] = slot[(size_t)8 * j + k];
    HIPCHK(hipMemcpyAsync(r1c, out.data(), (size_t)8 * n * 4, hipMemcpyHostToDevice, s));
  }
  // stencils, in chunks of nodes
  int32_t *mnode = nullptr, *sout = nullptr, *rnode = nullptr, *lst = nullptr, *tab = nullptr;
  APCCHK(dalloc2(&mnode, n, s));
  APCCHK(dalloc2(&rnode, n, s));
  APCCHK(dalloc2(&sout, (int64_t)M2MAX * n, s));
  const int64_t ch = std::min<int64_t>(n, CHUNK2);
  APCCHK(dalloc2(&lst, (int64_t)RING2 * ch, s));
  APCCHK(dalloc2(&tab, (int64_t)HASH2 * ch, s));
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
  for (int64_t y0 = 0; y0 < n; y0 += ch) {
    const int64_t cnt = std::min<int64_t>(ch, n - y0);
    hipLaunchKernelGGL(q_stencil, dim3(grid_for(cnt)), dim3(APC_BLOCK), 0, s, y0, cnt, n,
                       (const int32_t *)r1off, (const int32_t *)r1c, (const int32_t *)c->bowner,
                       (const int32_t *)c->crd, ntot, P.ring_min, P.ring_max, P.m_cap, lst, tab,
                       mnode, sout, rnode, err);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (herr & 8) {
    apc_set_error_msg("stencil ring larger than the search capacity");
    return APC_ESTENCIL;
  }
  if (herr & 16) {
    apc_set_error_msg("no acceptable stencil up to ring_max");
    return APC_ESTENCIL;
  }
  APCCHK(palloc(&c->st_off, n + 1));
  HIPCHK(hipMemsetAsync(c->st_off + n, 0, 4, s));
  HIPCHK(hipMemcpyAsync(r1cnt, mnode, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(r1cnt + n, 0, 4, s));
  APCCHK(apc_scan_i32(r1cnt, c->st_off, n + 1, s));
  int32_t nnz32 = 0;
  HIPCHK(hipMemcpyAsync(&nnz32, c->st_off + n, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c->nnz = nnz32;
  APCCHK(palloc(&c->st_idx, c->nnz));
  hipLaunchKernelGGL(q_st_copy, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, n, sout, c->st_off, mnode,
                     c->st_idx);
  HIPCHK(hipGetLastError());
  for (void *q : {(void *)keys, (void *)err, (void *)mc, (void *)bcnt, (void *)bstart, (void *)r1cnt,
                  (void *)r1off, (void *)r1, (void *)r1c, (void *)mnode, (void *)rnode,
                  (void *)sout, (void *)lst, (void *)tab})
    HIPCHK(apc_free_async(q, s));
  APCCHK(qcells_free(cl, s));
  // operator and solver arrays
  APCCHK(palloc(&c->w, c->nnz));
  APCCHK(palloc(&c->diag, n));
  APCCHK(palloc(&c->hs, n));
  APCCHK(palloc(&c->dinv, n));
  APCCHK(palloc(&c->dord, n));
  for (double **v : {&c->vx, &c->vr, &c->vrh, &c->vp, &c->vv, &c->vs, &c->vt, &c->vph, &c->vsh,
                     &c->vb}) {
    APCCHK(palloc(v, ntot));
    HIPCHK(hipMemsetAsync(*v, 0, (size_t)ntot * 8, s));
  }
  APCCHK(palloc(&c->part, 2 * (int64_t)G2));
  APCCHK(palloc(&c->sc, 1));
  HIPCHK(hipStreamSynchronize(s));
  return APC_OK;
}

double dot2(apc2_cloud *c, const double *a, const double *b, hipStream_t s, int *rc) {
  const unsigned g = std::min<unsigned>(grid_for(c->n), 1024u);
  hipLaunchKernelGGL(q_dot, dim3(g), dim3(APC_BLOCK), 0, s, c->n, a, b, c->part);
  std::vector<double> h(g);
  if (hipMemcpyAsync(h.data(), c->part, g * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    *rc = APC_EHIP;
  double t = 0.0;
  for (double v : h) t += v;
  return t;
}

// BiCGSTAB (x0 = 0, shadow residual r0, right Jacobi scaling with dinv when given)
// with its scalars on the device; stops when the recursive ||r|| / ||b|| <= tol and
// the true residual agrees, else restarts from the true residual (also after a
// breakdown)
int bicgstab2(apc2_cloud *c, const double *hs, const double *dinv, double tol, int maxit,
              apc_stats *st, hipStream_t s) {
  const int64_t n = c->n;
  const unsigned g = grid_for(n), gr = std::min<unsigned>(g, G2);
  constexpr int CHUNK = 16; // iterations launched between reads of the state
  int rc = APC_OK;
  double *ph = dinv ? c->vph : c->vp, *sh = dinv ? c->vsh : c->vs;
  HIPCHK(hipMemsetAsync(c->vx, 0, (size_t)n * 8, s));
  HIPCHK(hipMemcpyAsync(c->vr, c->vb, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
  int it = 0, status = APC_ENOCONV;
  double bn = 0.0, rel = 0.0, relt = 0.0;
  Scal2 h{};
  for (int first = 1;; first = 0) {
    // (re)start: rh = r, p = v = 0, rho = (r, r)
    HIPCHK(hipMemcpyAsync(c->vrh, c->vr, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(c->vp, 0, (size_t)n * 8, s));
    HIPCHK(hipMemsetAsync(c->vv, 0, (size_t)n * 8, s));
    hipLaunchKernelGGL(q_dotp, dim3(gr), dim3(APC_BLOCK), 0, s, n, (const double *)c->vr,
                       (const double *)c->vr, c->part);
    hipLaunchKernelGGL(q_fin_start, dim3(1), dim3(APC_BLOCK), 0, s, (const double *)c->part, gr,
                       c->sc, tol, maxit, first);
    HIPCHK(hipGetLastError());
    if (first) {
      HIPCHK(hipMemcpyAsync(&h, c->sc, sizeof(Scal2), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      bn = h.bnorm;
      if (bn == 0.0) {
        status = APC_OK;
        break;
      }
    }
    const int it0 = it;
    do {
      for (int k = 0; k < CHUNK; k++) {
        hipLaunchKernelGGL(q_upd_p, dim3(g), dim3(APC_BLOCK), 0, s, n, (const double *)c->vr, c->vp,
                           (const double *)c->vv, dinv, c->vph, (const Scal2 *)c->sc);
        hipLaunchKernelGGL(q_spmv_dot<1>, dim3(gr), dim3(APC_BLOCK), 0, s, n, c->st_off, c->st_idx,
                           c->w, hs, (const double *)ph, c->vv, (const double *)c->vrh, c->part,
                           (const Scal2 *)c->sc);
        hipLaunchKernelGGL(q_fin_alpha, dim3(1), dim3(APC_BLOCK), 0, s, (const double *)c->part, gr,
                           c->sc);
        hipLaunchKernelGGL(q_upd_s, dim3(g), dim3(APC_BLOCK), 0, s, n, (const double *)c->vr,
                           (const double *)c->vv, c->vs, dinv, c->vsh, (const Scal2 *)c->sc);
        hipLaunchKernelGGL(q_spmv_dot<2>, dim3(gr), dim3(APC_BLOCK), 0, s, n, c->st_off, c->st_idx,
                           c->w, hs, (const double *)sh, c->vt, (const double *)c->vs, c->part,
                           (const Scal2 *)c->sc);
        hipLaunchKernelGGL(q_fin_omega, dim3(1), dim3(APC_BLOCK), 0, s, (const double *)c->part, gr,
                           c->sc);
        hipLaunchKernelGGL(q_upd_xr, dim3(gr), dim3(APC_BLOCK), 0, s, n, c->vx, (const double *)ph,
                           (const double *)sh, (const double *)c->vs, (const double *)c->vt, c->vr,
                           (const double *)c->vrh, c->part, (const Scal2 *)c->sc);
        hipLaunchKernelGGL(q_fin_rho, dim3(1), dim3(APC_BLOCK), 0, s, (const double *)c->part, gr,
                           c->sc);
      }
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(&h, c->sc, sizeof(Scal2), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    } while (h.done == 0);
    it = h.it;
    rel = h.rnorm / bn;
    // true residual
    hipLaunchKernelGGL(q_apply, dim3(g), dim3(APC_BLOCK), 0, s, n, c->st_off, c->st_idx, c->w, hs,
                       (const double *)c->vx, c->vt);
    HIPCHK(hipMemcpyAsync(c->vr, c->vb, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(q_axpby, dim3(g), dim3(APC_BLOCK), 0, s, n, -1.0, (const double *)c->vt, 1.0,
                       c->vr);
    relt = sqrt(dot2(c, c->vr, c->vr, s, &rc)) / bn;
    if (rc != APC_OK) break;
    if (relt <= tol) {
      status = APC_OK;
      break;
    }
    if (it >= maxit || it == it0) break; // the limit, or a restart that made no step
  }
  HIPCHK(hipGetLastError());
  if (rc != APC_OK) return rc;
  if (st) {
    memset(st, 0, sizeof(*st));
    st->iters = it;
    st->status = status;
    st->sweeps = 1;
    st->rel_resid = rel;
    st->rel_resid_true = relt;
    st->rel_resid_fp64ref = relt;
    st->precond_used = dinv ? APC_PRECOND_JACOBI : APC_PRECOND_NONE;
  }
  return status;
}

} // namespace

// ---------------------------------------------------------------- entry points
extern "C" {

int apc2_build_cloud(const apc_params *p, const double *xy, int64_t N, hipStream_t stream,
                     apc2_cloud **out) {
  if (!out) return APC_EINVAL;
  *out = nullptr;
  if (!p || !xy || N < 1 || N > INT32_MAX || p->order != 2 || p->max_depth < 1 ||
      p->max_depth > 20 || !(p->L > 0.0) || !(p->c > 0.0) || p->ring_min < 1 ||
      p->ring_max < p->ring_min || p->m_cap < Q5 + 1 || p->m_cap > M2MAX ||
      p->criterion_pow < 0 || p->criterion_pow > 16 || !std::isfinite(p->poisson_c) ||
      !std::isfinite(p->lo[0]) || !std::isfinite(p->lo[1]))
    return APC_EINVAL;
  apc2_cloud *c = new apc2_cloud();
  c->P = *p;
  c->P.mask = nullptr;
  HIPCHK(hipGetDevice(&c->device));
  c->N = N;
  c->unit = p->L / ldexp(1.0, p->max_depth + 1);
  // T_l = (c 2^l / L)^e by repeated multiplication, e = 2 (k = 2) or criterion_pow
  const int pw = p->criterion_pow > 0 ? p->criterion_pow : 2;
  for (int l = 0; l < 24; l++) {
    const double t = (p->c * ldexp(1.0, l)) / p->L;
    double v = 1.0;
    for (int e = 0; e < pw; e++) v *= t;
    c->T[l] = v;
  }
  const int rc = build2(c, xy, stream);
  if (rc != APC_OK) {
    (void)hipStreamSynchronize(stream);
    free2(c);
    return rc;
  }
  *out = c;
  return APC_OK;
}

void apc2_destroy(apc2_cloud *c) { free2(c); }

int apc2_cloud_info(const apc2_cloud *c, int64_t *n, int64_t *nb, int64_t *nnz,
                    int64_t *n_opened) {
  if (!c) return APC_EINVAL;
  if (n) *n = c->n;
  if (nb) *nb = c->nb;
  if (nnz) *nnz = c->nnz;
  if (n_opened) *n_opened = c->n_opened;
  return APC_OK;
}

int apc2_get_nodes(const apc2_cloud *c, int32_t *perm, uint64_t *code, int32_t *level,
                   int32_t *first, int32_t *count, int32_t *bowner, int32_t *bface,
                   int32_t *st_off, int32_t *st_idx, int32_t *ixy) {
  if (!c) return APC_EINVAL;
  HIPCHK(hipDeviceSynchronize());
  const int64_t n = c->n, nb = c->nb, nt = n + nb;
  if (perm) HIPCHK(hipMemcpy(perm, c->perm, (size_t)c->N * 4, hipMemcpyDeviceToHost));
  if (code && n) HIPCHK(hipMemcpy(code, c->code, (size_t)n * 8, hipMemcpyDeviceToHost));
  if (level && n) HIPCHK(hipMemcpy(level, c->level, (size_t)n * 4, hipMemcpyDeviceToHost));
  if (first && n) HIPCHK(hipMemcpy(first, c->first, (size_t)n * 4, hipMemcpyDeviceToHost));
  if (count && n) HIPCHK(hipMemcpy(count, c->count, (size_t)n * 4, hipMemcpyDeviceToHost));
  if (bowner && nb) HIPCHK(hipMemcpy(bowner, c->bowner, (size_t)nb * 4, hipMemcpyDeviceToHost));
  if (bface && nb) HIPCHK(hipMemcpy(bface, c->bface, (size_t)nb * 4, hipMemcpyDeviceToHost));
  if (st_off) HIPCHK(hipMemcpy(st_off, c->st_off, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost));
  if (st_idx && c->nnz)
    HIPCHK(hipMemcpy(st_idx, c->st_idx, (size_t)c->nnz * 4, hipMemcpyDeviceToHost));
  if (ixy) HIPCHK(hipMemcpy(ixy, c->crd, (size_t)2 * nt * 4, hipMemcpyDeviceToHost));
  return APC_OK;
}

int apc2_assemble(apc2_cloud *c, hipStream_t s) {
  if (!c) return APC_EINVAL;
  int *err = nullptr;
  APCCHK(dalloc2(&err, 1, s));
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
  hipLaunchKernelGGL(q_fit, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->st_off, c->st_idx,
                     c->crd, c->n + c->nb, c->level, c->unit, c->P.L, c->w, c->diag, c->hs, c->dord,
                     err);
  hipLaunchKernelGGL(q_inv, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n,
                     (const double *)c->diag, c->dinv);
  HIPCHK(hipGetLastError());
  int herr = 0;
  HIPCHK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(apc_free_async(err, s));
  if (herr) {
    apc_set_error_msg("a stencil lost rank in the assembly");
    return APC_ESTENCIL;
  }
  c->assembled = true;
  return APC_OK;
}

int apc2_get_operator(const apc2_cloud *c, double *w_host, double *diag_host, double *bw_host,
                      double *bdiag_host, int8_t *order_host) {
  if (!c || !c->assembled) return APC_EINVAL;
  HIPCHK(hipDeviceSynchronize());
  const int64_t n = c->n, nnz = c->nnz;
  std::vector<double> w((size_t)(nnz > 0 ? nnz : 1)), d((size_t)(n > 0 ? n : 1)),
      hs((size_t)(n > 0 ? n : 1));
  std::vector<int32_t> off((size_t)n + 1);
  if (nnz) HIPCHK(hipMemcpy(w.data(), c->w, (size_t)nnz * 8, hipMemcpyDeviceToHost));
  if (n) {
    HIPCHK(hipMemcpy(d.data(), c->diag, (size_t)n * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hs.data(), c->hs, (size_t)n * 8, hipMemcpyDeviceToHost));
  }
  HIPCHK(hipMemcpy(off.data(), c->st_off, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost));
  if (w_host && nnz) memcpy(w_host, w.data(), (size_t)nnz * 8);
  if (diag_host && n) memcpy(diag_host, d.data(), (size_t)n * 8);
  if (order_host && n) HIPCHK(hipMemcpy(order_host, c->dord, (size_t)n, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; i++) {
    double sum = 0.0;
    for (int32_t e = off[i]; e < off[i + 1]; e++) {
      const double b = hs[i] * w[e];
      if (bw_host) bw_host[e] = b;
      sum += b;
    }
    if (bdiag_host) bdiag_host[i] = 1.0 - sum;
  }
  return APC_OK;
}

int apc2_deposit(apc2_cloud *c, const double *q, double *rho_M, hipStream_t s) {
  if (!c || !rho_M) return APC_EINVAL;
  hipLaunchKernelGGL(q_deposit, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->N, c->first,
                     c->count, c->level, c->perm, q, c->P.L, c->bowner, c->nb, rho_M);
  if (c->nb > 0)
    hipLaunchKernelGGL(q_bnd_copy, dim3(grid_for(c->nb)), dim3(APC_BLOCK), 0, s, c->n, c->nb,
                       c->bowner, rho_M);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc2_density_solve(apc2_cloud *c, const double *rho_M, double *rho_t, double tol, int maxit,
                       apc_stats *st, hipStream_t s) {
  if (!c || !c->assembled || !rho_M || !rho_t || !(tol > 0.0) || maxit < 1) return APC_EINVAL;
  hipLaunchKernelGGL(q_rhs, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->st_off, c->st_idx,
                     c->w, (const double *)c->hs, rho_M, 1.0, rho_M + c->n, c->vb);
  HIPCHK(hipGetLastError());
  const int rc = bicgstab2(c, c->hs, nullptr, tol, maxit, st, s);
  if (rc < 0) return rc;
  hipLaunchKernelGGL(q_write_out, dim3(grid_for(c->n + c->nb)), dim3(APC_BLOCK), 0, s, c->n, c->nb,
                     (const double *)c->vx, rho_M + c->n, rho_t);
  HIPCHK(hipStreamSynchronize(s));
  return rc;
}

int apc2_solve(apc2_cloud *c, const double *rho_t, const double *g, double *phi, double tol,
               int maxit, int precond, apc_stats *st, hipStream_t s) {
  if (!c || !c->assembled || !rho_t || !phi || !(tol > 0.0) || maxit < 1 ||
      (precond != APC_PRECOND_NONE && precond != APC_PRECOND_JACOBI))
    return APC_EINVAL;
  hipLaunchKernelGGL(q_rhs, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->st_off, c->st_idx,
                     c->w, (const double *)nullptr, rho_t, c->P.poisson_c, g, c->vb);
  HIPCHK(hipGetLastError());
  const int rc = bicgstab2(c, nullptr, precond == APC_PRECOND_JACOBI ? c->dinv : nullptr, tol,
                           maxit, st, s);
  if (rc < 0) return rc;
  hipLaunchKernelGGL(q_write_out, dim3(grid_for(c->n + c->nb)), dim3(APC_BLOCK), 0, s, c->n, c->nb,
                     (const double *)c->vx, g, phi);
  HIPCHK(hipStreamSynchronize(s));
  return rc;
}

int apc2_node_derivs(apc2_cloud *c, const double *f, double *D, hipStream_t s) {
  if (!c || !f || !D) return APC_EINVAL;
  hipLaunchKernelGGL(q_derivs, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->st_off,
                     c->st_idx, c->crd, c->n + c->nb, c->unit, f, D);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc2_interpolate_force(apc2_cloud *c, const double *phi, double *phi_p, double *grad_p,
                           hipStream_t s) {
  if (!c || !phi || !phi_p || !grad_p) return APC_EINVAL;
  double *D = nullptr;
  APCCHK(dalloc2(&D, (int64_t)Q5 * c->n, s));
  hipLaunchKernelGGL(q_derivs, dim3(grid_for(c->n)), dim3(APC_BLOCK), 0, s, c->n, c->st_off,
                     c->st_idx, c->crd, c->n + c->nb, c->unit, phi, D);
  hipLaunchKernelGGL(q_interp, dim3(grid_for(c->N)), dim3(APC_BLOCK), 0, s, c->N, c->sxy, c->perm,
                     c->pnode, c->crd, c->n + c->nb, c->P.lo[0], c->P.lo[1], c->unit, phi,
                     (const double *)D, phi_p, grad_p);
  HIPCHK(hipGetLastError());
  HIPCHK(apc_free_async(D, s));
  return APC_OK;
}

} // extern "C"

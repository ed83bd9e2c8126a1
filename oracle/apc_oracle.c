/*
 * apc_oracle.c -- FP64 CPU oracle of the AP-Cloud field solve.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  Plain, serial,
 * deliberately unoptimised C that follows the paper's steps in order:
 *
 *   Sec. 4      particles sorted by Morton key; pointer octree whose cells keep
 *               (first particle, particle count)
 *   Sec. 4.1    error-balance criterion h < c N'^(-1/(2k-2)) tested over the
 *               queue Q (eq. errorbalance_implementation)
 *   Sec. 4.2-3  2:1 face balance, processed from the deepest level upward, with
 *               the face-neighbour definition of Sec. 4.3
 *   Sec. 4.3    boundary nodes; k-ring neighbour search up to the 5-ring
 *   Sec. 3.1    weighted least squares GFD fit (scaled Vandermonde V0, Gaussian
 *               weight with c = 4) solved by Householder QR
 *   Sec. 3.2    density rows B = a^T V^+ C (eq. density_linear_system), GFD
 *               Poisson rows, Taylor interpolation of phi and grad phi
 *   Sec. 5      BiCGSTAB (the paper leaves the sparse solver open) and a dense
 *               LU cross-check
 *   Sec. 1      leapfrog particle push of the Vlasov-Poisson loop, with
 *               specular walls (the paper leaves the integrator open)
 *
 * Readings of points the paper leaves open are stated where they are used.
 */
#include "apc_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXP 34
#define MAXM 64

/* ------------------------------------------------------------------ */
/* Monomials: fitted unknowns are d^alpha f for 1 <= |alpha| <= k (the constant
   term is removed by differencing, eq. gfd); columns are ordered by degree and,
   within a degree, by descending exponent tuple (x first), as in the 2-D
   example matrix of Sec. 3.1. */

int apco_num_unknowns(int order) {
  if (order < 1 || order > 4) return APCO_EINVAL;
  return (order + 1) * (order + 2) * (order + 3) / 6 - 1;
}

int apco_monomials(int order, int32_t *al) {
  int p = apco_num_unknowns(order);
  if (p < 0) return p;
  int c = 0;
  for (int d = 1; d <= order; d++)
    for (int a = d; a >= 0; a--)
      for (int b = d - a; b >= 0; b--) {
        al[3 * c + 0] = a;
        al[3 * c + 1] = b;
        al[3 * c + 2] = d - a - b;
        c++;
      }
  return 0;
}

static double factorial(int a) {
  double f = 1.0;
  for (int i = 2; i <= a; i++) f *= (double)i;
  return f;
}

static double ipow(double x, int a) {
  double r = 1.0;
  for (int i = 0; i < a; i++) r *= x;
  return r;
}

/* xi^alpha / alpha! */
static double mono(const int32_t *a, double x, double y, double z) {
  return ipow(x, a[0]) / factorial(a[0]) * ipow(y, a[1]) / factorial(a[1]) * ipow(z, a[2]) /
         factorial(a[2]);
}

/* ------------------------------------------------------------------ */
/* Weighted least squares fit (Sec. 3.1).
   delta_j = y^j - y^0, h = max_{d,j} |delta_d^j|, xi = delta / h,
   V0 row j = [xi_j^alpha / alpha!], W_j = (exp(-r_j^2/r_max^2) - e^-4)/(1 - e^-4).
   Reading: rows are scaled by W (minimise sum_j (W_j (V0 a - df)_j)^2).
   X = (W V0)^+ W = R^{-1} Q^T W via Householder QR of W V0, so that the scaled
   derivatives h^{|alpha|} d^alpha f(y0) are X (f_j - f_0). */
static int wls_core(int order, int m, const double *dx, const double *dy, const double *dz,
                    double *X, double *hout, double *ratio) {
  int p = apco_num_unknowns(order);
  int32_t al[3 * MAXP];
  apco_monomials(order, al);
  if (m < 1 || m > MAXM) return APCO_EINVAL;
  double h = 0.0, r2max = 0.0;
  double r2[MAXM], W[MAXM];
  for (int j = 0; j < m; j++) {
    if (fabs(dx[j]) > h) h = fabs(dx[j]);
    if (fabs(dy[j]) > h) h = fabs(dy[j]);
    if (fabs(dz[j]) > h) h = fabs(dz[j]);
    r2[j] = dx[j] * dx[j] + dy[j] * dy[j] + dz[j] * dz[j];
    if (r2[j] > r2max) r2max = r2[j];
  }
  *hout = h;
  if (h == 0.0 || m < p) {
    *ratio = 0.0;
    return 0;
  }
  const double e4 = exp(-4.0);
  for (int j = 0; j < m; j++) W[j] = (exp(-r2[j] / r2max) - e4) / (1.0 - e4);

  /* A = W V0, column-major m x p */
  static double A[MAXP * MAXM], V[MAXP * MAXM], Q[MAXP * MAXM];
  double beta[MAXP], R[MAXP * MAXP];
  for (int c = 0; c < p; c++)
    for (int j = 0; j < m; j++)
      A[c * m + j] = W[j] * mono(&al[3 * c], dx[j] / h, dy[j] / h, dz[j] / h);

  /* Householder QR */
  for (int c = 0; c < p; c++) {
    double nrm2 = 0.0;
    for (int j = c; j < m; j++) nrm2 += A[c * m + j] * A[c * m + j];
    double nrm = sqrt(nrm2);
    for (int j = 0; j < m; j++) V[c * m + j] = 0.0;
    if (nrm == 0.0) {
      beta[c] = 0.0;
      continue;
    }
    double alpha = A[c * m + c] >= 0.0 ? -nrm : nrm;
    for (int j = c; j < m; j++) V[c * m + j] = A[c * m + j];
    V[c * m + c] -= alpha;
    double vn2 = 0.0;
    for (int j = c; j < m; j++) vn2 += V[c * m + j] * V[c * m + j];
    beta[c] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    for (int c2 = c + 1; c2 < p; c2++) {
      double s = 0.0;
      for (int j = c; j < m; j++) s += V[c * m + j] * A[c2 * m + j];
      s *= beta[c];
      for (int j = c; j < m; j++) A[c2 * m + j] -= s * V[c * m + j];
    }
    A[c * m + c] = alpha;
    for (int j = c + 1; j < m; j++) A[c * m + j] = 0.0;
  }
  double rmin = INFINITY, rmax = 0.0;
  for (int c = 0; c < p; c++) {
    for (int i = 0; i < p; i++) R[i * p + c] = (i <= c) ? A[c * m + i] : 0.0;
    double d = fabs(R[c * p + c]);
    if (d < rmin) rmin = d;
    if (d > rmax) rmax = d;
  }
  *ratio = rmax > 0.0 ? rmin / rmax : 0.0;
  if (rmin == 0.0) return 0;

  /* thin Q = H_0 ... H_{p-1} [I_p; 0], column-major m x p */
  for (int c = 0; c < p; c++)
    for (int j = 0; j < m; j++) Q[c * m + j] = (j == c) ? 1.0 : 0.0;
  for (int c = p - 1; c >= 0; c--)
    for (int q = 0; q < p; q++) {
      double s = 0.0;
      for (int j = c; j < m; j++) s += V[c * m + j] * Q[q * m + j];
      s *= beta[c];
      for (int j = c; j < m; j++) Q[q * m + j] -= s * V[c * m + j];
    }
  /* X[:, j] = R^{-1} (Q[j, :]^T W_j) by back substitution */
  for (int j = 0; j < m; j++) {
    double x[MAXP];
    for (int i = p - 1; i >= 0; i--) {
      double s = Q[i * m + j] * W[j];
      for (int k = i + 1; k < p; k++) s -= R[i * p + k] * x[k];
      x[i] = s / R[i * p + i];
    }
    for (int i = 0; i < p; i++) X[i * m + j] = x[i];
  }
  return 0;
}

int apco_wls_fit(int order, int m, const double *delta, double *X, double *h, double *ratio) {
  if (apco_num_unknowns(order) < 0 || m < 1 || m > MAXM) return APCO_EINVAL;
  double dx[MAXM], dy[MAXM], dz[MAXM];
  for (int j = 0; j < m; j++) {
    dx[j] = delta[3 * j];
    dy[j] = delta[3 * j + 1];
    dz[j] = delta[3 * j + 2];
  }
  return wls_core(order, m, dx, dy, dz, X, h, ratio);
}

/* ------------------------------------------------------------------ */
/* Octree (Sec. 4).  Reading of the Morton key: 3 bits per level, the x bit
   highest in each triple; particles are quantised at the deepest level
   max_depth: u_d = floor((x_d - lo_d) * (2^max_depth / L)), clamped into
   [0, 2^max_depth - 1]. */

typedef struct {
  int32_t level, ix, iy, iz;
  int64_t child;  /* index of the first of 8 children, -1 for a leaf */
  int64_t first, count;
  int32_t opened; /* 0 leaf, 1 criterion, 2 balance */
} ocell;

struct apco_cloud {
  apco_params P;
  int64_t N;
  int p;
  double T[32];
  double unit;
  int64_t *perm;
  uint64_t *skey;
  ocell *cells;
  int64_t ncells, capcells, nopened;
  int64_t n, nb;
  int64_t *node_cell;
  int64_t *cell_node;
  int32_t *crd; /* 3*(n+nb), node-major */
  int32_t *bowner, *bface;
  int32_t *bidx; /* 6*n: boundary node index of (node, face) or -1 */
  int32_t *r1off, *r1;
  int32_t *st_off, *st, *st_ring;
  int8_t *node_order; /* GFD order of each node's row: the cloud's k, or 2 (fallback) */
  uint8_t *pyr;       /* irregular domain: state of every cell of levels 0 .. mask_level
                         (0 inside Omega, 1 excluded, 2 mixed), level l at pyr_off[l],
                         index x + 2^l (y + 2^l z) */
  int64_t pyr_off[8];
};

static uint64_t morton(uint64_t x, uint64_t y, uint64_t z, int bits) {
  uint64_t k = 0;
  for (int b = 0; b < bits; b++) {
    k |= ((x >> b) & 1ull) << (3 * b + 2);
    k |= ((y >> b) & 1ull) << (3 * b + 1);
    k |= ((z >> b) & 1ull) << (3 * b);
  }
  return k;
}

typedef struct {
  uint64_t key;
  int64_t idx;
} kpair;

/* Offset between two integer coordinates along one axis: the plain difference, or
   on a periodic domain (side S = 2^(D+1) integer units) the minimum image in
   [-S/2, S/2). */
static int64_t doff(const apco_params *P, int64_t a, int64_t b) {
  int64_t d = a - b;
  if (P->periodic) {
    const int64_t S = (int64_t)1 << (P->max_depth + 1);
    if (d >= S / 2) d -= S;
    else if (d < -(S / 2)) d += S;
  }
  return d;
}

/* State of the level-l cell (ix, iy, iz) on an irregular domain: 0 inside Omega,
   1 excluded, 2 partly excluded (levels below mask_level only). */
static int cell_state(const apco_cloud *C, int l, int64_t ix, int64_t iy, int64_t iz) {
  const int ml = C->P.mask_level;
  if (ml <= 0) return 0;
  if (l > ml) {
    ix >>= (l - ml);
    iy >>= (l - ml);
    iz >>= (l - ml);
    l = ml;
  }
  const int64_t s = (int64_t)1 << l;
  return C->pyr[C->pyr_off[l] + ix + s * (iy + s * iz)];
}

static int cmp_kpair(const void *a, const void *b) {
  const kpair *x = a, *y = b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

/* first position in [lo,hi) with skey >= v */
static int64_t lower_bound(const uint64_t *a, int64_t lo, int64_t hi, uint64_t v) {
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

int apco_thresholds(const apco_params *P, double *T) {
  /* T_l = t^(2k-2), t = c 2^l / L: the criterion h < c N'^(-1/(2k-2)) with
     h = L 2^-l (cell edge, as in the worked example of Sec. 4.3) is N' < T_l;
     a cell is opened when N' >= T_l.  Evaluated as t = (c * 2^l) / L and then
     repeated multiplication from 1.0.  For k = 2 the supraconvergent bound of
     Sec. 3.3, with the optimal h of Sec. 3.4, balances with h ~ N'^(-1/4) instead:
     exponent 4 (criterion_pow). */
  const int pw = P->criterion_pow > 0 ? P->criterion_pow : 2 * P->order - 2;
  for (int l = 0; l <= P->max_depth; l++) {
    double t = (P->c * ldexp(1.0, l)) / P->L;
    double v = 1.0;
    for (int e = 0; e < pw; e++) v *= t;
    T[l] = v;
  }
  /* periodic: levels 0 and 1 always open, so that every leaf sees distinct cells
     across its faces */
  if (P->periodic)
    for (int l = 0; l < 2 && l <= P->max_depth; l++) T[l] = 0.0;
  return 0;
}

static int push_cell(apco_cloud *C, ocell c) {
  if (C->ncells == C->capcells) {
    int64_t nc = C->capcells ? 2 * C->capcells : 1024;
    ocell *q = realloc(C->cells, (size_t)nc * sizeof(ocell));
    if (!q) return APCO_ENOMEM;
    C->cells = q;
    C->capcells = nc;
  }
  C->cells[C->ncells++] = c;
  return 0;
}

/* "open" a cell (Sec. 4.3): mark it non-node and append its 8 children to Q;
   each child's particle range is the sub-range of its parent's sorted range
   carrying the child's key prefix. */
static int open_cell(apco_cloud *C, int64_t i, int why) {
  int D = C->P.max_depth;
  ocell par = C->cells[i];
  int64_t first = C->ncells;
  int lv = par.level + 1;
  int sh = 3 * (D - lv);
  for (int c = 0; c < 8; c++) {
    ocell ch;
    ch.level = lv;
    ch.ix = 2 * par.ix + ((c >> 2) & 1);
    ch.iy = 2 * par.iy + ((c >> 1) & 1);
    ch.iz = 2 * par.iz + (c & 1);
    ch.child = -1;
    ch.opened = 0;
    uint64_t pre = morton((uint64_t)ch.ix, (uint64_t)ch.iy, (uint64_t)ch.iz, lv);
    int64_t a = lower_bound(C->skey, par.first, par.first + par.count, pre << sh);
    int64_t b = lower_bound(C->skey, par.first, par.first + par.count, (pre + 1) << sh);
    ch.first = a;
    ch.count = b - a;
    int rc = push_cell(C, ch);
    if (rc) return rc;
  }
  C->cells[i].child = first;
  C->cells[i].opened = why;
  C->nopened++;
  return 0;
}

/* Face neighbour of cell i across face f (Sec. 4.3), read as the deepest cell of
   Q with level <= level(i) that shares face f with cell i (the paper's wording
   "no ancestor" is read as "no descendant": the neighbour's level only grows as
   cells open).  -1 if the face lies on the domain boundary (never on a periodic
   domain). */
static int64_t face_nb(const apco_cloud *C, int64_t i, int f) {
  const ocell *y = &C->cells[i];
  int32_t t[3] = {y->ix, y->iy, y->iz};
  int d = f / 2;
  t[d] += (f & 1) ? 1 : -1;
  if (C->P.periodic) /* the face across the domain boundary meets the opposite cell */
    t[d] = (t[d] + (1 << y->level)) % (1 << y->level);
  else if (t[d] < 0 || t[d] >= (1 << y->level))
    return -1;
  /* irregular domain: a face onto an excluded cell is a wall */
  if (cell_state(C, y->level, t[0], t[1], t[2]) == 1) return -1;
  int64_t cur = 0;
  while (C->cells[cur].child >= 0 && C->cells[cur].level < y->level) {
    int sh = y->level - C->cells[cur].level - 1;
    int c = (((t[0] >> sh) & 1) << 2) | (((t[1] >> sh) & 1) << 1) | ((t[2] >> sh) & 1);
    cur = C->cells[cur].child + c;
  }
  return cur;
}

typedef struct {
  uint64_t code;
  int64_t cell;
} lpair;

static int cmp_lpair(const void *a, const void *b) {
  const lpair *x = a, *y = b;
  return (x->code > y->code) - (x->code < y->code);
}

typedef struct {
  int64_t r2;
  int32_t idx;
} cand_t;

static int cmp_cand(const void *a, const void *b) {
  const cand_t *x = a, *y = b;
  if (x->r2 != y->r2) return x->r2 < y->r2 ? -1 : 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Octant membership with closed octants (a zero offset counts on both sides). */
static int in_octant(int o, int64_t d0, int64_t d1, int64_t d2) {
  int sx = (o >> 2) & 1 ? 1 : -1, sy = (o >> 1) & 1 ? 1 : -1, sz = o & 1 ? 1 : -1;
  return sx * d0 >= 0 && sy * d1 >= 0 && sz * d2 >= 0;
}

/* Stencil choice from a candidate ring sorted by (r^2, index) -- the quadrant
   criterion of Sec. 3.1 read for 3-D octants: first the two nearest candidates of
   every closed octant, then (order 4 only) for each axis in turn the nearest
   candidates with a new offset along that axis until the axis has 5 distinct
   offsets counting the centre's 0 (on fewer planes a degree-4 polynomial
   vanishes on the whole stencil), then the nearest remaining candidates, until
   min(count, m_cap) nodes are chosen; the chosen set is kept in candidate order.
   It is accepted when (i) every closed octant holds at least one chosen node --
   with relax set, every closed octant in which the ring holds a candidate at all
   (on an irregular domain at ring_max: at a convex corner of the voxel staircase
   an octant can hold no node of any ring, and the rule asks for a neighbour in
   each octant where the domain has one) --, (ii) m >= p + 1, (iii) the weighted V0 has full column rank:
   min|R_ii| / max|R_ii| >= 1e-6, and (iv, order 4) its Laplacian row has a
   negative diagonal d and sum |w_j| <= 10 |d|.  Returns m (>0) on acceptance, 0
   otherwise; the chosen candidates are compacted to the front of cd. */
#define TAU_RANK 1e-6
#define TAU_DOM_DEFAULT 10.0
static int choose_stencil(const apco_cloud *C, int32_t y, cand_t *cd, int64_t cnt, int m_cap,
                          int order, int relax) {
  const int32_t *c0 = &C->crd[3 * y];
  int64_t want = cnt < m_cap ? cnt : m_cap;
  static unsigned char pick[1 << 20];
  if (cnt > (int64_t)sizeof(pick)) return 0;
  memset(pick, 0, (size_t)cnt);
  int64_t got = 0;
  int populated[8];
  for (int o = 0; o < 8; o++) {
    int taken = 0;
    for (int64_t j = 0; j < cnt && taken < 2; j++) {
      const int32_t *c1 = &C->crd[3 * cd[j].idx];
      if (!in_octant(o, doff(&C->P, c1[0], c0[0]), doff(&C->P, c1[1], c0[1]),
                     doff(&C->P, c1[2], c0[2])))
        continue;
      taken++;
      if (!pick[j] && got < want) {
        pick[j] = 1;
        got++;
      }
    }
    populated[o] = taken > 0;
  }
  for (int d = 0; order == 4 && d < 3; d++) {
    for (;;) {
      int64_t vals[MAXM + 1];
      int nv = 1;
      vals[0] = 0;
      for (int64_t j = 0; j < cnt; j++) {
        if (!pick[j]) continue;
        int64_t o = doff(&C->P, C->crd[3 * cd[j].idx + d], c0[d]);
        int seen = 0;
        for (int q = 0; q < nv; q++) seen |= vals[q] == o;
        if (!seen && nv <= MAXM) vals[nv++] = o;
      }
      if (nv >= 5 || got >= want) break;
      int64_t add = -1;
      for (int64_t j = 0; j < cnt && add < 0; j++) {
        if (pick[j]) continue;
        int64_t o = doff(&C->P, C->crd[3 * cd[j].idx + d], c0[d]);
        int seen = 0;
        for (int q = 0; q < nv; q++) seen |= vals[q] == o;
        if (!seen) add = j;
      }
      if (add < 0) break;
      pick[add] = 1;
      got++;
    }
  }
  for (int64_t j = 0; j < cnt && got < want; j++)
    if (!pick[j]) {
      pick[j] = 1;
      got++;
    }
  int m = 0;
  for (int64_t j = 0; j < cnt; j++)
    if (pick[j]) cd[m++] = cd[j];
  if (m < apco_num_unknowns(order) + 1 || m > MAXM) return 0;
  int oct[8] = {0};
  double dx[MAXM], dy[MAXM], dz[MAXM];
  for (int j = 0; j < m; j++) {
    const int32_t *c1 = &C->crd[3 * cd[j].idx];
    int64_t d0 = doff(&C->P, c1[0], c0[0]), d1 = doff(&C->P, c1[1], c0[1]),
            d2 = doff(&C->P, c1[2], c0[2]);
    dx[j] = (double)d0;
    dy[j] = (double)d1;
    dz[j] = (double)d2;
    for (int o = 0; o < 8; o++) oct[o] += in_octant(o, d0, d1, d2);
  }
  for (int o = 0; o < 8; o++)
    if (oct[o] < 1 && (populated[o] || !relax)) return 0;
  static double X[MAXP * MAXM];
  double h, ratio;
  wls_core(order, m, dx, dy, dz, X, &h, &ratio);
  if (!(ratio >= TAU_RANK)) return 0;
  if (order == 4) {
    /* stability of the order-4 Laplacian row: a negative diagonal and off-diagonal
       weights of total magnitude at most tau_dom times the diagonal's (scale-free:
       h cancels); otherwise the node falls back to an order-2 row */
    double s = 0.0, sa = 0.0;
    for (int j = 0; j < m; j++) {
      double v = X[3 * m + j] + X[6 * m + j] + X[8 * m + j];
      s += v;
      sa += fabs(v);
    }
    const double tau = C->P.tau_dom > 0.0 ? C->P.tau_dom : TAU_DOM_DEFAULT;
    if (!(s > 0.0 && sa <= tau * s)) return 0;
  }
  return m;
}

void apco_destroy(apco_cloud *C) {
  if (!C) return;
  free(C->perm);
  free(C->skey);
  free(C->cells);
  free(C->node_cell);
  free(C->cell_node);
  free(C->crd);
  free(C->bowner);
  free(C->bface);
  free(C->bidx);
  free(C->r1off);
  free(C->r1);
  free(C->st_off);
  free(C->st);
  free(C->st_ring);
  free(C->node_order);
  free(C->pyr);
  free(C);
}

#define CHECK_ALLOC(p)       \
  do {                       \
    if (!(p)) {              \
      apco_destroy(C);       \
      return APCO_ENOMEM;    \
    }                        \
  } while (0)

int apco_build_cloud(const apco_params *P, const double *xyz, int64_t N, apco_cloud **out) {
  *out = NULL;
  int p = apco_num_unknowns(P->order);
  if (!(P->order == 2 || P->order == 4) || P->max_depth < 1 || P->max_depth > 20 ||
      !(P->L > 0.0) || !(P->c > 0.0) || P->ring_min < 1 || P->ring_max < P->ring_min ||
      P->m_cap > MAXM || P->m_cap < p + 1 || N < 1 || P->criterion_pow < 0 ||
      P->criterion_pow > 16 || !(P->tau_dom >= 0.0) || P->periodic < 0 || P->periodic > 1 ||
      (P->periodic && P->max_depth < 2) || P->kernel < APCO_KERNEL_NGP ||
      P->kernel > APCO_KERNEL_TSC || P->mask_level < 0 || P->mask_level > 6 ||
      P->mask_level > P->max_depth ||
      (P->mask_level > 0 && (!P->mask || P->periodic || P->kernel != APCO_KERNEL_NGP)))
    return APCO_EINVAL;
  apco_cloud *C = calloc(1, sizeof(apco_cloud));
  if (!C) return APCO_ENOMEM;
  C->P = *P;
  C->N = N;
  C->p = p;
  const int D = P->max_depth;
  apco_thresholds(P, C->T);
  C->unit = P->L / ldexp(1.0, D + 1);

  /* Irregular domain: the state pyramid of the mask, level mask_level from the
     mask, each coarser cell from its 8 children (0 all inside, 1 all excluded,
     2 mixed).  Omega must keep at least one cell. */
  const int ml = P->mask_level;
  if (ml > 0) {
    int64_t tot = 0;
    for (int l = 0; l <= ml; l++) {
      C->pyr_off[l] = tot;
      tot += (int64_t)1 << (3 * l);
    }
    C->pyr = malloc((size_t)tot);
    CHECK_ALLOC(C->pyr);
    const int64_t sm = (int64_t)1 << ml;
    int64_t inside = 0;
    for (int64_t q = 0; q < sm * sm * sm; q++) {
      C->pyr[C->pyr_off[ml] + q] = P->mask[q] ? 1 : 0;
      inside += P->mask[q] ? 0 : 1;
    }
    if (inside == 0) {
      apco_destroy(C);
      return APCO_EINVAL;
    }
    for (int l = ml - 1; l >= 0; l--) {
      const int64_t s = (int64_t)1 << l;
      for (int64_t z = 0; z < s; z++)
        for (int64_t y = 0; y < s; y++)
          for (int64_t x = 0; x < s; x++) {
            int n0 = 0, n1 = 0;
            for (int c = 0; c < 8; c++) {
              const int st = cell_state(C, l + 1, 2 * x + ((c >> 2) & 1), 2 * y + ((c >> 1) & 1),
                                        2 * z + (c & 1));
              n0 += st == 0;
              n1 += st == 1;
            }
            C->pyr[C->pyr_off[l] + x + s * (y + s * z)] = n0 == 8 ? 0 : (n1 == 8 ? 1 : 2);
          }
    }
  }

  /* Morton keys and sort (Sec. 4): stable by (key, original index) */
  kpair *kp = malloc((size_t)N * sizeof(kpair));
  CHECK_ALLOC(kp);
  const double s = ldexp(1.0, D) / P->L;
  const int64_t top = ((int64_t)1 << D) - 1;
  for (int64_t i = 0; i < N; i++) {
    int64_t u[3];
    for (int d = 0; d < 3; d++) {
      double x = xyz[d * N + i];
      if (isnan(x)) {
        free(kp);
        apco_destroy(C);
        return APCO_EINVAL;
      }
      if (x < P->lo[d] || x > P->lo[d] + P->L) {
        free(kp);
        apco_destroy(C);
        return APCO_EDOMAIN;
      }
      double q = floor((x - P->lo[d]) * s);
      int64_t v = (int64_t)q;
      if (v < 0) v = 0;
      if (v > top) v = top;
      u[d] = v;
    }
    if (ml > 0 && cell_state(C, D, u[0], u[1], u[2]) == 1) { /* in an excluded cell */
      free(kp);
      apco_destroy(C);
      return APCO_EDOMAIN;
    }
    kp[i].key = morton((uint64_t)u[0], (uint64_t)u[1], (uint64_t)u[2], D);
    kp[i].idx = i;
  }
  qsort(kp, (size_t)N, sizeof(kpair), cmp_kpair);
  C->perm = malloc((size_t)N * sizeof(int64_t));
  C->skey = malloc((size_t)N * sizeof(uint64_t));
  if (!C->perm || !C->skey) {
    free(kp);
    apco_destroy(C);
    return APCO_ENOMEM;
  }
  for (int64_t i = 0; i < N; i++) {
    C->perm[i] = kp[i].idx;
    C->skey[i] = kp[i].key;
  }
  free(kp);

  /* Node selection (Sec. 4.3).  Step 1: Q = {root}. */
  ocell root = {0, 0, 0, 0, -1, 0, N, 0};
  if (push_cell(C, root)) {
    apco_destroy(C);
    return APCO_ENOMEM;
  }
  /* Step 2: traverse Q (children appended during the traversal are visited too);
     open every cell violating the error-balance criterion, below max_depth.  On an
     irregular domain excluded cells are never opened, and every other cell of a
     level below mask_level is (so no leaf straddles a wall). */
  for (int64_t i = 0; i < C->ncells; i++) {
    const ocell *c = &C->cells[i];
    const int st = cell_state(C, c->level, c->ix, c->iy, c->iz);
    if (c->level < D && st != 1 && (c->level < ml || (double)c->count >= C->T[c->level]))
      if (open_cell(C, i, 1)) {
        apco_destroy(C);
        return APCO_ENOMEM;
      }
  }
  int lq = 0;
  for (int64_t i = 0; i < C->ncells; i++)
    if (C->cells[i].level > lq) lq = C->cells[i].level;
  /* Steps 3-4: from the deepest level up, every leaf at level l opens each face
     neighbour that is a leaf more than one level coarser (re-resolving the
     neighbour after each opening). */
  for (int l = lq; l >= 1; l--) {
    for (int64_t i = 0; i < C->ncells; i++) {
      if (C->cells[i].child >= 0 || C->cells[i].level != l) continue;
      if (cell_state(C, l, C->cells[i].ix, C->cells[i].iy, C->cells[i].iz) == 1) continue;
      for (int f = 0; f < 6; f++) {
        for (;;) {
          int64_t z = face_nb(C, i, f);
          if (z < 0) break;
          if (C->cells[z].child < 0 && C->cells[z].level < l - 1) {
            if (open_cell(C, z, 2)) {
              apco_destroy(C);
              return APCO_ENOMEM;
            }
          } else {
            break;
          }
        }
      }
    }
  }

  /* Nodes: every leaf (node candidate) inside Omega, ordered by the Morton code of
     its minimum corner at max_depth. */
  int64_t n = 0;
  for (int64_t i = 0; i < C->ncells; i++) {
    const ocell *c = &C->cells[i];
    n += c->child < 0 && cell_state(C, c->level, c->ix, c->iy, c->iz) != 1;
  }
  lpair *lp = malloc((size_t)(n > 0 ? n : 1) * sizeof(lpair));
  CHECK_ALLOC(lp);
  int64_t k = 0;
  for (int64_t i = 0; i < C->ncells; i++) {
    const ocell *c = &C->cells[i];
    if (c->child >= 0 || cell_state(C, c->level, c->ix, c->iy, c->iz) == 1) continue;
    int sh = D - c->level;
    lp[k].code = morton((uint64_t)c->ix << sh, (uint64_t)c->iy << sh, (uint64_t)c->iz << sh, D);
    lp[k].cell = i;
    k++;
  }
  if (k != n) {
    free(lp);
    apco_destroy(C);
    return APCO_EINVAL;
  }
  qsort(lp, (size_t)n, sizeof(lpair), cmp_lpair);
  C->n = n;
  C->node_cell = malloc((size_t)n * sizeof(int64_t));
  C->cell_node = malloc((size_t)C->ncells * sizeof(int64_t));
  C->bidx = malloc((size_t)n * 6 * sizeof(int32_t));
  if (!C->node_cell || !C->cell_node || !C->bidx) {
    free(lp);
    apco_destroy(C);
    return APCO_ENOMEM;
  }
  for (int64_t i = 0; i < C->ncells; i++) C->cell_node[i] = -1;
  for (int64_t j = 0; j < n; j++) {
    C->node_cell[j] = lp[j].cell;
    C->cell_node[lp[j].cell] = j;
  }
  free(lp);

  /* Boundary nodes (Sec. 4.3 "add additional nodes on the boundary"): read as one
     node at the centre of every leaf face lying on the domain boundary (a box face,
     or on an irregular domain a face onto an excluded cell). */
  int64_t nb = 0;
  for (int64_t j = 0; j < n; j++) {
    for (int f = 0; f < 6; f++) {
      int on = face_nb(C, C->node_cell[j], f) < 0;
      C->bidx[6 * j + f] = on ? (int32_t)(n + nb++) : -1;
    }
  }
  C->nb = nb;
  C->crd = malloc((size_t)3 * (n + nb) * sizeof(int32_t));
  C->bowner = malloc((size_t)(nb + 1) * sizeof(int32_t));
  C->bface = malloc((size_t)(nb + 1) * sizeof(int32_t));
  CHECK_ALLOC(C->crd);
  CHECK_ALLOC(C->bowner);
  CHECK_ALLOC(C->bface);
  for (int64_t j = 0; j < n; j++) {
    const ocell *c = &C->cells[C->node_cell[j]];
    int32_t sz = 1 << (D - c->level);
    C->crd[3 * j + 0] = (2 * c->ix + 1) * sz;
    C->crd[3 * j + 1] = (2 * c->iy + 1) * sz;
    C->crd[3 * j + 2] = (2 * c->iz + 1) * sz;
    for (int f = 0; f < 6; f++) {
      int32_t b = C->bidx[6 * j + f];
      if (b < 0) continue;
      int d = f / 2;
      for (int e = 0; e < 3; e++) C->crd[3 * b + e] = C->crd[3 * j + e];
      C->crd[3 * b + d] += (f & 1) ? sz : -sz; /* the centre of face f */
      C->bowner[b - n] = (int32_t)j;
      C->bface[b - n] = f;
    }
  }

  /* 1-ring (Sec. 4.3): for each face, the neighbour if it is a node, else the 4
     children of the neighbour sharing that face (nodes by 2:1 balance); a face on
     the domain boundary contributes its boundary node. */
  C->r1off = malloc((size_t)(n + 1) * sizeof(int32_t));
  C->r1 = malloc((size_t)n * 24 * sizeof(int32_t));
  CHECK_ALLOC(C->r1off);
  CHECK_ALLOC(C->r1);
  int64_t e = 0;
  for (int64_t j = 0; j < n; j++) {
    C->r1off[j] = (int32_t)e;
    int64_t ci = C->node_cell[j];
    for (int f = 0; f < 6; f++) {
      int64_t z = face_nb(C, ci, f);
      if (z < 0) {
        C->r1[e++] = C->bidx[6 * j + f];
        continue;
      }
      if (C->cells[z].child < 0) {
        C->r1[e++] = (int32_t)C->cell_node[z];
        continue;
      }
      int d = f / 2;
      int side = (f & 1) ? 0 : 1; /* children of z on the face shared with cell j */
      for (int c = 0; c < 8; c++) {
        int bit = (c >> (2 - d)) & 1;
        if (bit != side) continue;
        int64_t ch = C->cells[z].child + c;
        if (C->cells[ch].child >= 0) { /* cannot happen in a 2:1-balanced tree */
          apco_destroy(C);
          return APCO_EINVAL;
        }
        C->r1[e++] = (int32_t)C->cell_node[ch];
      }
    }
  }
  C->r1off[n] = (int32_t)e;

  /* Stencils (Sec. 4.3): the R-ring = nodes within R face-adjacency steps
     (boundary nodes hang off their owner), sorted by (integer squared distance,
     node index); a stencil is chosen from ring_min upward until one is accepted.
     Order fallback (k = 4 only): a node with no acceptable order-4 stencil up to
     ring_max takes an order-2 row, chosen by the order-2 rule from ring 2 with
     m_cap 40.  Past ring_max at order 2 the build fails.  On an irregular domain the
     last ring (ring_max) does not ask for the octants in which it holds no node. */
  int64_t ntot = n + nb;
  int32_t *stamp = malloc((size_t)ntot * sizeof(int32_t));
  int32_t *front = malloc((size_t)ntot * sizeof(int32_t));
  cand_t *cand = malloc((size_t)ntot * sizeof(cand_t));
  C->st_off = malloc((size_t)(n + 1) * sizeof(int32_t));
  C->st_ring = malloc((size_t)(n + 1) * sizeof(int32_t));
  C->node_order = malloc((size_t)(n + 1));
  int64_t stcap = n * 32 + 64;
  C->st = malloc((size_t)stcap * sizeof(int32_t));
  if (!stamp || !front || !cand || !C->st_off || !C->st_ring || !C->st || !C->node_order) {
    free(stamp);
    free(front);
    free(cand);
    apco_destroy(C);
    return APCO_ENOMEM;
  }
  for (int64_t i = 0; i < ntot; i++) stamp[i] = -1;
  int64_t ne = 0;
  int rc = 0;
  for (int64_t y = 0; y < n && !rc; y++) {
    C->st_off[y] = (int32_t)ne;
    int done = 0;
    for (int att = 0; att < 2 && !done; att++) {
    const int ko = att == 0 ? P->order : 2;
    if (att == 1 && P->order != 4) break;
    const int rmin = att == 0 ? P->ring_min : 2, mcap = att == 0 ? P->m_cap : 40;
    for (int R = rmin; R <= P->ring_max && !done; R++) {
      /* depth-limited BFS */
      int64_t nf = 0, cnt = 0;
      stamp[y] = (int32_t)y;
      front[nf++] = (int32_t)y;
      int64_t lo = 0;
      for (int depth = 1; depth <= R; depth++) {
        int64_t hi = nf;
        for (int64_t t = lo; t < hi; t++) {
          int32_t u = front[t];
          if (u >= n) { /* boundary node: adjacent to its owner only */
            int32_t v = C->bowner[u - n];
            if (stamp[v] != (int32_t)y) {
              stamp[v] = (int32_t)y;
              front[nf++] = v;
            }
            continue;
          }
          for (int32_t a = C->r1off[u]; a < C->r1off[u + 1]; a++) {
            int32_t v = C->r1[a];
            if (stamp[v] != (int32_t)y) {
              stamp[v] = (int32_t)y;
              front[nf++] = v;
            }
          }
        }
        lo = hi;
      }
      for (int64_t t = 1; t < nf; t++) {
        int32_t v = front[t];
        int64_t d0 = doff(P, C->crd[3 * v], C->crd[3 * y]);
        int64_t d1 = doff(P, C->crd[3 * v + 1], C->crd[3 * y + 1]);
        int64_t d2 = doff(P, C->crd[3 * v + 2], C->crd[3 * y + 2]);
        cand[cnt].r2 = d0 * d0 + d1 * d1 + d2 * d2;
        cand[cnt].idx = v;
        cnt++;
      }
      /* reset stamps for the next ring size of this node */
      for (int64_t t = 0; t < nf; t++) stamp[front[t]] = -1;
      qsort(cand, (size_t)cnt, sizeof(cand_t), cmp_cand);
      int m = choose_stencil(C, (int32_t)y, cand, cnt, mcap, ko,
                             P->mask_level > 0 && R == P->ring_max);
      if (m > 0) {
        if (ne + m > stcap) {
          stcap = 2 * stcap + m;
          int32_t *q = realloc(C->st, (size_t)stcap * sizeof(int32_t));
          if (!q) {
            rc = APCO_ENOMEM;
            break;
          }
          C->st = q;
        }
        for (int j = 0; j < m; j++) C->st[ne++] = cand[j].idx;
        C->st_ring[y] = R;
        C->node_order[y] = (int8_t)ko;
        done = 1;
      }
    }
    }
    if (!done && !rc) rc = APCO_ESTENCIL;
  }
  C->st_off[n] = (int32_t)ne;
  free(stamp);
  free(front);
  free(cand);
  if (rc) {
    apco_destroy(C);
    return rc;
  }
  *out = C;
  return 0;
}

int apco_info(const apco_cloud *C, int64_t *n, int64_t *nb, int64_t *nnz, int64_t *n_opened,
              int64_t *ncells) {
  if (n) *n = C->n;
  if (nb) *nb = C->nb;
  if (nnz) *nnz = C->st_off[C->n];
  if (n_opened) *n_opened = C->nopened;
  if (ncells) *ncells = C->ncells;
  return 0;
}

int apco_get_nodes(const apco_cloud *C, int64_t *perm, uint64_t *code, int32_t *level,
                   int64_t *first, int64_t *count, int32_t *bowner, int32_t *bface,
                   int32_t *st_off, int32_t *st_idx, int32_t *st_ring) {
  const int D = C->P.max_depth;
  if (perm) memcpy(perm, C->perm, (size_t)C->N * sizeof(int64_t));
  for (int64_t j = 0; j < C->n; j++) {
    const ocell *c = &C->cells[C->node_cell[j]];
    int sh = D - c->level;
    if (code)
      code[j] = morton((uint64_t)c->ix << sh, (uint64_t)c->iy << sh, (uint64_t)c->iz << sh, D);
    if (level) level[j] = c->level;
    if (first) first[j] = c->first;
    if (count) count[j] = c->count;
    if (st_ring) st_ring[j] = C->st_ring[j];
  }
  if (bowner) memcpy(bowner, C->bowner, (size_t)C->nb * sizeof(int32_t));
  if (bface) memcpy(bface, C->bface, (size_t)C->nb * sizeof(int32_t));
  if (st_off) memcpy(st_off, C->st_off, (size_t)(C->n + 1) * sizeof(int32_t));
  if (st_idx) memcpy(st_idx, C->st, (size_t)C->st_off[C->n] * sizeof(int32_t));
  return 0;
}

int apco_node_coords(const apco_cloud *C, int32_t *ixyz) {
  int64_t nt = C->n + C->nb;
  for (int64_t j = 0; j < nt; j++)
    for (int d = 0; d < 3; d++) ixyz[d * nt + j] = C->crd[3 * j + d];
  return 0;
}

int apco_get_cells(const apco_cloud *C, int32_t *level, int32_t *ijk, int64_t *count,
                   int32_t *opened) {
  for (int64_t i = 0; i < C->ncells; i++) {
    const ocell *c = &C->cells[i];
    if (level) level[i] = c->level;
    if (ijk) {
      ijk[3 * i] = c->ix;
      ijk[3 * i + 1] = c->iy;
      ijk[3 * i + 2] = c->iz;
    }
    if (count) count[i] = c->count;
    if (opened) opened[i] = c->opened;
  }
  return 0;
}

int apco_ring1(const apco_cloud *C, int32_t *off, int32_t *idx, int64_t cap) {
  if (C->r1off[C->n] > cap) return APCO_EINVAL;
  memcpy(off, C->r1off, (size_t)(C->n + 1) * sizeof(int32_t));
  memcpy(idx, C->r1, (size_t)C->r1off[C->n] * sizeof(int32_t));
  return 0;
}

/* ------------------------------------------------------------------ */
/* Per-node fit on the cloud's stencil, in integer units. */
static int node_fit(const apco_cloud *C, int64_t y, double *X, int *m, double *hphys, int *pk) {
  int32_t a = C->st_off[y], b = C->st_off[y + 1];
  *m = b - a;
  double dx[MAXM], dy[MAXM], dz[MAXM];
  for (int j = 0; j < *m; j++) {
    int32_t v = C->st[a + j];
    dx[j] = (double)doff(&C->P, C->crd[3 * v], C->crd[3 * y]);
    dy[j] = (double)doff(&C->P, C->crd[3 * v + 1], C->crd[3 * y + 1]);
    dz[j] = (double)doff(&C->P, C->crd[3 * v + 2], C->crd[3 * y + 2]);
  }
  double h, ratio;
  const int ko = C->node_order[y];
  *pk = apco_num_unknowns(ko);
  int rc = wls_core(ko, *m, dx, dy, dz, X, &h, &ratio);
  if (rc) return rc;
  if (ratio < TAU_RANK) return APCO_ESTENCIL;
  *hphys = h * C->unit;
  return 0;
}

static int find_alpha(const int32_t *al, int p, int a, int b, int c) {
  for (int i = 0; i < p; i++)
    if (al[3 * i] == a && al[3 * i + 1] == b && al[3 * i + 2] == c) return i;
  return -1;
}

/* GFD Poisson row (Sec. 3.2 step 2): Delta f(y0) = sum_d d^{2 e_d} f(y0)
   = h^-2 sum_d X[2e_d] (f - f_0); off-diagonal weights w_j and diagonal -sum w_j. */
int apco_assemble(const apco_cloud *C, double *w, double *diag) {
  int p = C->p;
  int32_t al[3 * MAXP];
  apco_monomials(C->P.order, al);
  int ixx = find_alpha(al, p, 2, 0, 0), iyy = find_alpha(al, p, 0, 2, 0),
      izz = find_alpha(al, p, 0, 0, 2);
  static double X[MAXP * MAXM];
  for (int64_t y = 0; y < C->n; y++) {
    int m, pk;
    double hp;
    int rc = node_fit(C, y, X, &m, &hp, &pk);
    if (rc) return rc;
    double s = 0.0;
    int32_t a = C->st_off[y];
    for (int j = 0; j < m; j++) {
      double v = (X[ixx * m + j] + X[iyy * m + j] + X[izz * m + j]) / (hp * hp);
      w[a + j] = v;
      s += v;
    }
    diag[y] = -s;
  }
  return 0;
}

/* Charge-assignment kernels Phi(u) = phi(u_x) phi(u_y) phi(u_z) of eq.
   density_apcloud, u = (x - y) / h: each 1-D phi is a piecewise polynomial
   c0 + c1 u + c2 u^2 on up to three pieces [a, b].  NGP: the characteristic
   function of [-1/2, 1/2] (the node's own cell).  CIC: the tent 1 - |u| on
   [-1, 1].  TSC: the quadratic B-spline, 3/4 - u^2 on [-1/2, 1/2] and
   (3/2 - |u|)^2 / 2 on 1/2 <= |u| <= 3/2.  Each integrates to 1. */
typedef struct {
  int np;
  double a[3], b[3], c[3][3];
} kpieces;

static kpieces kernel_pieces(int kernel) {
  kpieces K;
  memset(&K, 0, sizeof(K));
  if (kernel == APCO_KERNEL_NGP) {
    K.np = 1;
    K.a[0] = -0.5; K.b[0] = 0.5; K.c[0][0] = 1.0;
  } else if (kernel == APCO_KERNEL_CIC) {
    K.np = 2;
    K.a[0] = -1.0; K.b[0] = 0.0; K.c[0][0] = 1.0; K.c[0][1] = 1.0;
    K.a[1] = 0.0; K.b[1] = 1.0; K.c[1][0] = 1.0; K.c[1][1] = -1.0;
  } else {
    K.np = 3;
    /* (3/2 + u)^2 / 2 = 9/8 + 3/2 u + 1/2 u^2 */
    K.a[0] = -1.5; K.b[0] = -0.5; K.c[0][0] = 1.125; K.c[0][1] = 1.5; K.c[0][2] = 0.5;
    K.a[1] = -0.5; K.b[1] = 0.5; K.c[1][0] = 0.75; K.c[1][2] = -1.0;
    K.a[2] = 0.5; K.b[2] = 1.5; K.c[2][0] = 1.125; K.c[2][1] = -1.5; K.c[2][2] = 0.5;
  }
  return K;
}

/* phi(u) evaluated as defined (the expanded coefficients above serve the moment
   integrals; near the edge of the support they would cancel) */
static double kernel_phi(int kernel, double u) {
  const double a = fabs(u);
  if (kernel == APCO_KERNEL_CIC) return a <= 1.0 ? 1.0 - a : 0.0;
  if (kernel == APCO_KERNEL_TSC) {
    if (a <= 0.5) return 0.75 - a * a;
    return a <= 1.5 ? 0.5 * (1.5 - a) * (1.5 - a) : 0.0;
  }
  return a <= 0.5 ? 1.0 : 0.0;
}

static double kernel_halfsupport(int kernel) {
  return kernel == APCO_KERNEL_NGP ? 0.5 : (kernel == APCO_KERNEL_CIC ? 1.0 : 1.5);
}

double apco_kernel_moment(int kernel, int k, double tlo, double thi) {
  kpieces K = kernel_pieces(kernel);
  const double hs = kernel_halfsupport(kernel);
  /* a kernel symmetric about 0 has vanishing odd moments over its whole support */
  if ((k & 1) && tlo <= -hs && thi >= hs) return 0.0;
  double m = 0.0;
  for (int q = 0; q < K.np; q++) {
    const double lo = tlo > K.a[q] ? tlo : K.a[q], hi = thi < K.b[q] ? thi : K.b[q];
    if (!(hi > lo)) continue;
    for (int e = 0; e < 3; e++) {
      if (K.c[q][e] == 0.0) continue;
      const int r = k + e + 1;
      m += K.c[q][e] * (ipow(hi, r) - ipow(lo, r)) / (double)r;
    }
  }
  return m;
}

/* Truncation of node y's kernel by the walls, per axis: the kernel's argument
   u = (x - y) / h runs over [tlo, thi] inside Omega (unbounded on a periodic
   domain). */
static void node_trunc(const apco_cloud *C, int64_t y, double *tlo, double *thi) {
  const int l = C->cells[C->node_cell[y]].level;
  const double hs = ldexp(1.0, C->P.max_depth + 1 - l); /* cell edge, integer units */
  const double S = ldexp(1.0, C->P.max_depth + 1);
  for (int d = 0; d < 3; d++) {
    if (C->P.periodic) {
      tlo[d] = -INFINITY;
      thi[d] = INFINITY;
    } else {
      tlo[d] = -(double)C->crd[3 * y + d] / hs;
      thi[d] = (S - (double)C->crd[3 * y + d]) / hs;
    }
  }
}

/* a_0(y): the kernel's mass inside Omega */
static double node_a0(const apco_cloud *C, int64_t y) {
  double tlo[3], thi[3], a0 = 1.0;
  node_trunc(C, y, tlo, thi);
  for (int d = 0; d < 3; d++) a0 *= apco_kernel_moment(C->P.kernel, 0, tlo[d], thi[d]);
  return a0;
}

/* Density row (eq. density_linear_system): b = a^T V^+ C, with the kernel moments
   a_alpha = (1/h_c^3) int_cell (x - y)^alpha dx / alpha! of the NGP kernel (the
   characteristic function of the node's own cell, edge h_c).  Reading: the
   Taylor terms carry 1/alpha!, so a^T d rho~ is the cell average of the Taylor
   polynomial; odd moments vanish and a_alpha = prod_d mu(alpha_d) / alpha! with
   mu(e) = (h_c/2)^e / (e + 1).  The row is b_j = sum_alpha a_alpha X_alpha,j / h^|alpha|
   over the unknowns of the fit of order ko (moments of order <= ko); the
   diagonal is 1 - sum_j b_j (the row reproduces constants). */
static void density_row(const double *X, int m, int ko, double hc, double hp, int kernel,
                        const double *tlo, const double *thi, double *b, double *bdiag) {
  int32_t al[3 * MAXP];
  int pk = apco_num_unknowns(ko);
  apco_monomials(ko, al);
  double coef[MAXP];
  double a0 = 1.0;
  if (kernel != APCO_KERNEL_NGP)
    for (int d = 0; d < 3; d++) a0 *= apco_kernel_moment(kernel, 0, tlo[d], thi[d]);
  for (int i = 0; i < pk; i++) {
    const int32_t *a = &al[3 * i];
    coef[i] = 0.0;
    double mom = 1.0;
    if (kernel == APCO_KERNEL_NGP) {
      if ((a[0] | a[1] | a[2]) & 1) continue;
      for (int d = 0; d < 3; d++) mom *= ipow(hc / 2.0, a[d]) / (double)(a[d] + 1) / factorial(a[d]);
    } else {
      /* a_alpha / a_0 = prod_d h^a_d mu_a_d / a_d! / a_0, mu over the truncated
         support (odd and mixed moments appear beside the walls) */
      for (int d = 0; d < 3; d++)
        mom *= ipow(hc, a[d]) * apco_kernel_moment(kernel, a[d], tlo[d], thi[d]) / factorial(a[d]);
      mom /= a0;
    }
    coef[i] = mom / ipow(hp, a[0] + a[1] + a[2]);
  }
  double s = 0.0;
  for (int j = 0; j < m; j++) {
    double v = 0.0;
    for (int i = 0; i < pk; i++) v += coef[i] * X[i * m + j];
    b[j] = v;
    s += v;
  }
  *bdiag = 1.0 - s;
}

/* Stability bound of a density row (reading; the paper states none): the row is
   strictly diagonally dominant with sum_j |b_j| <= THETA_B * b_ii.  Then B has
   a positive diagonal and the Jacobi iteration matrix of B has infinity norm at
   most THETA_B, so the density solve converges at a rate independent of n. */
#define THETA_B 0.5
static int density_row_ok(const double *b, int m, double bdiag) {
  double sa = 0.0;
  for (int j = 0; j < m; j++) sa += fabs(b[j]);
  return sa <= THETA_B * bdiag;
}

/* Density rows of every interior node, with the stability rule (reading): the
   row of the node's own fit order k_y is kept when it meets the bound; else, for
   an order-4 row, the order-2 row of the same stencil (the fit restricted to the
   9 unknowns of order 1 and 2, moments a_{2 e_d} only); else the identity row
   (rho~ = rho_M at that node: the cell average read as the centre value, which
   the vanishing odd moments make second-order accurate).  ord (may be NULL)
   receives the order of each row kept: k_y, 2 or 0. */
static int density_rows_ord(const apco_cloud *C, double *bw, double *bdiag, int8_t *ord) {
  static double X[MAXP * MAXM];
  double b[MAXM];
  for (int64_t y = 0; y < C->n; y++) {
    int m, pk;
    double hp;
    int rc = node_fit(C, y, X, &m, &hp, &pk);
    if (rc) return rc;
    double hc = C->P.L / ldexp(1.0, C->cells[C->node_cell[y]].level);
    int ko = C->node_order[y];
    double bd, tlo[3], thi[3];
    node_trunc(C, y, tlo, thi);
    density_row(X, m, ko, hc, hp, C->P.kernel, tlo, thi, b, &bd);
    if (!density_row_ok(b, m, bd) && ko == 4) {
      /* the order-2 fit of the same stencil */
      int32_t a = C->st_off[y];
      double dx[MAXM], dy[MAXM], dz[MAXM], h2, ratio2;
      for (int j = 0; j < m; j++) {
        int32_t v = C->st[a + j];
        dx[j] = (double)doff(&C->P, C->crd[3 * v], C->crd[3 * y]);
        dy[j] = (double)doff(&C->P, C->crd[3 * v + 1], C->crd[3 * y + 1]);
        dz[j] = (double)doff(&C->P, C->crd[3 * v + 2], C->crd[3 * y + 2]);
      }
      rc = wls_core(2, m, dx, dy, dz, X, &h2, &ratio2);
      if (rc) return rc;
      ko = 2;
      density_row(X, m, 2, hc, hp, C->P.kernel, tlo, thi, b, &bd);
    }
    if (!density_row_ok(b, m, bd)) {
      ko = 0;
      for (int j = 0; j < m; j++) b[j] = 0.0;
      bd = 1.0;
    }
    int32_t a0 = C->st_off[y];
    for (int j = 0; j < m; j++) bw[a0 + j] = b[j];
    bdiag[y] = bd;
    if (ord) ord[y] = (int8_t)ko;
  }
  return 0;
}

int apco_density_rows(const apco_cloud *C, double *bw, double *bdiag) {
  return density_rows_ord(C, bw, bdiag, NULL);
}

int apco_density_orders(const apco_cloud *C, int8_t *ord) {
  int64_t nnz = C->st_off[C->n];
  double *bw = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  double *bd = malloc(sizeof(double) * (size_t)(C->n > 0 ? C->n : 1));
  if (!bw || !bd) {
    free(bw);
    free(bd);
    return APCO_ENOMEM;
  }
  int rc = density_rows_ord(C, bw, bd, ord);
  free(bw);
  free(bd);
  return rc;
}

/* rho_M(y_j) = (1/h_c^3) sum_{particles in cell j} q_i (eq. density_apcloud with
   the NGP kernel); summed in sorted order.  q == NULL: each particle carries 1/N
   (total charge 1, Sec. 2) and the sum is count * (1/N). */
int apco_deposit(const apco_cloud *C, const double *q, double *rho_M) {
  double q0 = 1.0 / (double)C->N;
  for (int64_t j = 0; j < C->n; j++) {
    const ocell *c = &C->cells[C->node_cell[j]];
    double sum = 0.0;
    if (q) {
      for (int64_t s = c->first; s < c->first + c->count; s++) sum += q[C->perm[s]];
    } else {
      sum = (double)c->count * q0;
    }
    double hc = C->P.L / ldexp(1.0, c->level);
    rho_M[j] = sum / (hc * hc * hc);
  }
  /* boundary nodes carry their owner's value (reading: boundary density is not
     solved for; it enters the rhs) */
  for (int64_t b = 0; b < C->nb; b++) rho_M[C->n + b] = rho_M[C->bowner[b]];
  return 0;
}

/* eq. density_apcloud's right-hand side with a CIC or TSC kernel: every particle
   against every node (the kernel vanishes outside its support), in sorted
   particle order.  Reading: the moments a(y) integrate over Omega, so beside a
   wall the kernel's mass a_0(y) inside Omega is below 1; each row of the density
   system is divided by a_0 (so that it reproduces constants with unit weight) and
   so is rho_M here.  Offsets are minimum images on a periodic domain. */
int apco_deposit_xyz(const apco_cloud *C, const double *xyz, const double *q, double *rho_M) {
  if (C->P.kernel == APCO_KERNEL_NGP) return apco_deposit(C, q, rho_M);
  if (!xyz) return APCO_EINVAL;
  const int64_t N = C->N;
  const double q0 = 1.0 / (double)N, L = C->P.L;
  for (int64_t j = 0; j < C->n; j++) {
    const double h = L / ldexp(1.0, C->cells[C->node_cell[j]].level);
    double yc[3];
    for (int d = 0; d < 3; d++) yc[d] = C->P.lo[d] + C->unit * (double)C->crd[3 * j + d];
    double sum = 0.0;
    for (int64_t s = 0; s < N; s++) {
      const int64_t i = C->perm[s];
      double w = 1.0;
      for (int d = 0; d < 3 && w != 0.0; d++) {
        double dx = xyz[d * N + i] - yc[d];
        if (C->P.periodic) {
          if (dx >= 0.5 * L) dx -= L;
          else if (dx < -0.5 * L) dx += L;
        }
        w *= kernel_phi(C->P.kernel, dx / h);
      }
      if (w != 0.0) sum += (q ? q[i] : q0) * w;
    }
    rho_M[j] = sum / (node_a0(C, j) * h * h * h);
  }
  for (int64_t b = 0; b < C->nb; b++) rho_M[C->n + b] = rho_M[C->bowner[b]];
  return 0;
}

/* ------------------------------------------------------------------ */
/* Krylov solver on rows (diag, w) over the interior unknowns. */

static void rows_matvec(const apco_cloud *C, const double *diag, const double *w,
                        const double *x, double *y) {
  for (int64_t i = 0; i < C->n; i++) {
    double s = diag[i] * x[i];
    for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++) {
      int32_t j = C->st[e];
      if (j < C->n) s += w[e] * x[j];
    }
    y[i] = s;
  }
}

static double dot(const double *a, const double *b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

/* BiCGSTAB (van der Vorst), x0 = 0, shadow residual r^ = r0, optional right
   Jacobi preconditioning; stops when the recursive ||r||/||b|| <= tol and the
   recomputed true residual agrees; restarts from the true residual on
   breakdown or disagreement. */
static int bicgstab(const apco_cloud *C, const double *diag, const double *w, const double *b,
                    double *x, double tol, int maxit, int precond, apco_stats *st) {
  int64_t n = C->n;
  double *r = calloc((size_t)n, sizeof(double)), *rh = calloc((size_t)n, sizeof(double)),
         *pv = calloc((size_t)n, sizeof(double)), *v = calloc((size_t)n, sizeof(double)),
         *s = calloc((size_t)n, sizeof(double)), *t = calloc((size_t)n, sizeof(double)),
         *ph = calloc((size_t)n, sizeof(double)), *sh = calloc((size_t)n, sizeof(double));
  if (!r || !rh || !pv || !v || !s || !t || !ph || !sh) {
    free(r); free(rh); free(pv); free(v); free(s); free(t); free(ph); free(sh);
    return APCO_ENOMEM;
  }
  for (int64_t i = 0; i < n; i++) x[i] = 0.0;
  double bn = sqrt(dot(b, b, n));
  int it = 0, status = APCO_ENOCONV;
  double rel = 0.0, relt = 0.0;
  if (bn == 0.0) {
    status = 0;
    goto done;
  }
  memcpy(r, b, (size_t)n * sizeof(double));
  for (;;) {
    /* (re)start */
    memcpy(rh, r, (size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; i++) pv[i] = v[i] = 0.0;
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    int restart = 0;
    while (it < maxit && !restart) {
      it++;
      double rho = dot(rh, r, n);
      if (rho == 0.0 || !isfinite(rho)) {
        restart = 1;
        break;
      }
      double beta = (rho / rho_old) * (alpha / omega);
      for (int64_t i = 0; i < n; i++) pv[i] = r[i] + beta * (pv[i] - omega * v[i]);
      for (int64_t i = 0; i < n; i++) ph[i] = precond ? pv[i] / diag[i] : pv[i];
      rows_matvec(C, diag, w, ph, v);
      double rv = dot(rh, v, n);
      if (rv == 0.0 || !isfinite(rv)) {
        restart = 1;
        break;
      }
      alpha = rho / rv;
      for (int64_t i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
      for (int64_t i = 0; i < n; i++) sh[i] = precond ? s[i] / diag[i] : s[i];
      rows_matvec(C, diag, w, sh, t);
      double tt = dot(t, t, n);
      omega = tt > 0.0 ? dot(t, s, n) / tt : 0.0;
      for (int64_t i = 0; i < n; i++) x[i] += alpha * ph[i] + omega * sh[i];
      for (int64_t i = 0; i < n; i++) r[i] = s[i] - omega * t[i];
      rho_old = rho;
      rel = sqrt(dot(r, r, n)) / bn;
      if (rel <= tol || omega == 0.0) {
        /* true residual */
        rows_matvec(C, diag, w, x, t);
        for (int64_t i = 0; i < n; i++) r[i] = b[i] - t[i];
        relt = sqrt(dot(r, r, n)) / bn;
        if (relt <= tol) {
          status = 0;
          goto done;
        }
        restart = 1;
      }
    }
    if (it >= maxit) break;
    if (restart) {
      rows_matvec(C, diag, w, x, t);
      for (int64_t i = 0; i < n; i++) r[i] = b[i] - t[i];
    }
  }
done:
  if (bn != 0.0) {
    rows_matvec(C, diag, w, x, t);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - t[i];
    relt = sqrt(dot(r, r, n)) / bn;
  }
  if (st) {
    st->iters = it;
    st->status = status;
    st->rel_resid = rel;
    st->rel_resid_true = relt;
  }
  free(r); free(rh); free(pv); free(v); free(s); free(t); free(ph); free(sh);
  return 0;
}

static void bnd_rhs(const apco_cloud *C, const double *w, const double *bval, double *rhs) {
  for (int64_t i = 0; i < C->n; i++)
    for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++) {
      int32_t j = C->st[e];
      if (j >= C->n) rhs[i] -= w[e] * bval[j - C->n];
    }
}

int apco_density_solve(const apco_cloud *C, const double *rho_M, double *rho_t, double tol,
                       int maxit, int precond, apco_stats *st) {
  int64_t n = C->n, nnz = C->st_off[n];
  double *bw = malloc((size_t)(nnz + 1) * sizeof(double));
  double *bd = malloc((size_t)(n + 1) * sizeof(double));
  double *rhs = malloc((size_t)(n + 1) * sizeof(double));
  if (!bw || !bd || !rhs) {
    free(bw); free(bd); free(rhs);
    return APCO_ENOMEM;
  }
  int rc = apco_density_rows(C, bw, bd);
  if (!rc) {
    for (int64_t i = 0; i < n; i++) rhs[i] = rho_M[i];
    bnd_rhs(C, bw, rho_M + n, rhs);
    rc = bicgstab(C, bd, bw, rhs, rho_t, tol, maxit, precond, st);
    for (int64_t b = 0; b < C->nb; b++) rho_t[n + b] = rho_M[n + b];
  }
  free(bw); free(bd); free(rhs);
  return rc;
}

static int poisson_system(const apco_cloud *C, const double *rho_t, const double *g, double **w,
                          double **diag, double **rhs) {
  int64_t n = C->n, nnz = C->st_off[n];
  *w = malloc((size_t)(nnz + 1) * sizeof(double));
  *diag = malloc((size_t)(n + 1) * sizeof(double));
  *rhs = malloc((size_t)(n + 1) * sizeof(double));
  if (!*w || !*diag || !*rhs) return APCO_ENOMEM;
  int rc = apco_assemble(C, *w, *diag);
  if (rc) return rc;
  if (C->P.periodic) {
    /* Delta phi = c (rho~ - rhobar), rhobar the volume-weighted mean of rho~ (the
       neutralising background without which no periodic potential exists); the
       operator's constant null space is removed by replacing the equation of node
       0 with phi_0 = 0, and the solution is shifted to mean 0 afterwards */
    double vol = 0.0, q = 0.0;
    for (int64_t i = 0; i < n; i++) {
      const double h = C->P.L / ldexp(1.0, C->cells[C->node_cell[i]].level);
      vol += h * h * h;
      q += rho_t[i] * h * h * h;
    }
    const double rbar = q / vol;
    for (int64_t i = 0; i < n; i++) (*rhs)[i] = C->P.poisson_c * (rho_t[i] - rbar);
    if (n > 0) {
      (*rhs)[0] = 0.0;
      (*diag)[0] = 1.0;
      for (int32_t e = C->st_off[0]; e < C->st_off[1]; e++) (*w)[e] = 0.0;
    }
    return 0;
  }
  for (int64_t i = 0; i < n; i++) (*rhs)[i] = C->P.poisson_c * rho_t[i];
  if (g) bnd_rhs(C, *w, g, *rhs);
  return 0;
}

/* periodic: phi shifted to volume-weighted mean 0 */
static void zero_mean(const apco_cloud *C, double *phi) {
  if (!C->P.periodic) return;
  double vol = 0.0, q = 0.0;
  for (int64_t i = 0; i < C->n; i++) {
    const double h = C->P.L / ldexp(1.0, C->cells[C->node_cell[i]].level);
    vol += h * h * h;
    q += phi[i] * h * h * h;
  }
  const double m = q / vol;
  for (int64_t i = 0; i < C->n; i++) phi[i] -= m;
}

int apco_poisson_solve(const apco_cloud *C, const double *rho_t, const double *g, double *phi,
                       double tol, int maxit, int precond, apco_stats *st) {
  double *w = NULL, *diag = NULL, *rhs = NULL;
  int rc = poisson_system(C, rho_t, g, &w, &diag, &rhs);
  if (!rc) rc = bicgstab(C, diag, w, rhs, phi, tol, maxit, precond, st);
  if (!rc) zero_mean(C, phi);
  if (!rc)
    for (int64_t b = 0; b < C->nb; b++) phi[C->n + b] = g ? g[b] : 0.0;
  free(w); free(diag); free(rhs);
  return rc;
}

/* BiCGSTAB on rows the caller assembled (apco_assemble or apco_density_rows) and
   an interior right-hand side: the solver of apco_poisson_solve without the
   assembly, so that the two can be timed apart. */
int apco_bicgstab_rows(const apco_cloud *C, const double *w, const double *diag,
                       const double *rhs, double *x, double tol, int maxit, int precond,
                       apco_stats *st) {
  return bicgstab(C, diag, w, rhs, x, tol, maxit, precond, st);
}

int apco_poisson_lu(const apco_cloud *C, const double *rho_t, const double *g, double *phi) {
  int64_t n = C->n;
  double *w = NULL, *diag = NULL, *rhs = NULL;
  int rc = poisson_system(C, rho_t, g, &w, &diag, &rhs);
  double *A = rc ? NULL : calloc((size_t)(n * n), sizeof(double));
  if (!rc && !A) rc = APCO_ENOMEM;
  if (!rc) {
    for (int64_t i = 0; i < n; i++) {
      A[i * n + i] = diag[i];
      for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++)
        if (C->st[e] < n) A[i * n + C->st[e]] += w[e];
    }
    /* Gaussian elimination with partial pivoting */
    for (int64_t k = 0; k < n && !rc; k++) {
      int64_t piv = k;
      for (int64_t i = k + 1; i < n; i++)
        if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
      if (A[piv * n + k] == 0.0) {
        rc = APCO_EINVAL;
        break;
      }
      if (piv != k) {
        for (int64_t j = 0; j < n; j++) {
          double t = A[k * n + j];
          A[k * n + j] = A[piv * n + j];
          A[piv * n + j] = t;
        }
        double t = rhs[k];
        rhs[k] = rhs[piv];
        rhs[piv] = t;
      }
      for (int64_t i = k + 1; i < n; i++) {
        double f = A[i * n + k] / A[k * n + k];
        if (f == 0.0) continue;
        for (int64_t j = k; j < n; j++) A[i * n + j] -= f * A[k * n + j];
        rhs[i] -= f * rhs[k];
      }
    }
    for (int64_t i = n - 1; i >= 0 && !rc; i--) {
      double s = rhs[i];
      for (int64_t j = i + 1; j < n; j++) s -= A[i * n + j] * phi[j];
      phi[i] = s / A[i * n + i];
    }
    if (!rc) zero_mean(C, phi);
    for (int64_t b = 0; b < C->nb; b++) phi[n + b] = g ? g[b] : 0.0;
  }
  free(A); free(w); free(diag); free(rhs);
  return rc;
}

int apco_apply_laplacian(const apco_cloud *C, const double *f, double *out) {
  int64_t n = C->n, nnz = C->st_off[n];
  double *w = malloc((size_t)(nnz + 1) * sizeof(double));
  double *diag = malloc((size_t)(n + 1) * sizeof(double));
  if (!w || !diag) {
    free(w); free(diag);
    return APCO_ENOMEM;
  }
  int rc = apco_assemble(C, w, diag);
  if (!rc)
    for (int64_t i = 0; i < n; i++) {
      double s = diag[i] * f[i];
      for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++) s += w[e] * f[C->st[e]];
      out[i] = s;
    }
  free(w); free(diag);
  return rc;
}

/* d^alpha f(y_j) = h^{-|alpha|} sum_i X[alpha][i] (f_i - f_j)  (Sec. 3.1) */
int apco_node_derivs(const apco_cloud *C, const double *f, double *Dout) {
  int p = C->p;
  int32_t al[3 * MAXP];
  apco_monomials(C->P.order, al);
  static double X[MAXP * MAXM];
  for (int64_t y = 0; y < C->n; y++) {
    int m, pk;
    double hp;
    int rc = node_fit(C, y, X, &m, &hp, &pk);
    if (rc) return rc;
    int32_t a = C->st_off[y];
    for (int i = pk; i < p; i++) Dout[y * p + i] = 0.0; /* order-2 fallback rows */
    for (int i = 0; i < pk; i++) {
      double s = 0.0;
      for (int j = 0; j < m; j++) s += X[i * m + j] * (f[C->st[a + j]] - f[y]);
      Dout[y * p + i] = s / ipow(hp, al[3 * i] + al[3 * i + 1] + al[3 * i + 2]);
    }
  }
  return 0;
}

/* Taylor interpolation (Sec. 3.2 step 3): a particle in leaf j takes
   phi(p) = phi_j + sum_alpha d^alpha phi_j delta^alpha / alpha!  and its gradient,
   delta = p - y_j (reading: the leaf containing the particle interpolates it). */
int apco_interpolate(const apco_cloud *C, const double *phi, const double *xyz, double *phi_p,
                     double *grad_p) {
  int p = C->p;
  int64_t n = C->n, N = C->N;
  int32_t al[3 * MAXP];
  apco_monomials(C->P.order, al);
  double *Dv = malloc((size_t)n * p * sizeof(double));
  if (!Dv) return APCO_ENOMEM;
  int rc = apco_node_derivs(C, phi, Dv);
  if (rc) {
    free(Dv);
    return rc;
  }
  for (int64_t j = 0; j < n; j++) {
    const ocell *c = &C->cells[C->node_cell[j]];
    double yc[3];
    for (int d = 0; d < 3; d++) yc[d] = C->P.lo[d] + C->unit * (double)C->crd[3 * j + d];
    const double *Dj = &Dv[j * p];
    for (int64_t s = c->first; s < c->first + c->count; s++) {
      int64_t i = C->perm[s];
      double dl[3];
      for (int d = 0; d < 3; d++) dl[d] = xyz[d * N + i] - yc[d];
      double v = phi[j], g[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < p; a++) {
        const int32_t *A = &al[3 * a];
        v += Dj[a] * mono(A, dl[0], dl[1], dl[2]);
        for (int d = 0; d < 3; d++) {
          if (A[d] == 0) continue;
          int32_t B[3] = {A[0], A[1], A[2]};
          B[d] -= 1;
          g[d] += Dj[a] * mono(B, dl[0], dl[1], dl[2]);
        }
      }
      phi_p[i] = v;
      for (int d = 0; d < 3; d++) grad_p[d * N + i] = g[d];
    }
  }
  free(Dv);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Learned preconditioner: training data, loss gradient, forward (plain loops). */

#define LIN 48
#define LHID 64
#define LOUT 41              /* {i} + up to 40 stencil entries */
#define LQQ (LOUT * (LOUT + 1) / 2)
#define LQ (LQQ + LOUT + 1)
#define LNW 40

int apco_learn_data(const apco_cloud *C, const double *Z, int K, double *feat, double *quad) {
  int64_t n = C->n, ntot = C->n + C->nb, nnz = C->st_off[n];
  double *w = malloc((size_t)(nnz + 1) * sizeof(double));
  double *d = malloc((size_t)(n + 1) * sizeof(double));
  double *U = (Z && K > 0) ? malloc((size_t)K * n * sizeof(double)) : NULL;
  if (!w || !d || (Z && K > 0 && !U)) {
    free(w); free(d); free(U);
    return APCO_ENOMEM;
  }
  int rc = apco_assemble(C, w, d);
  if (rc) {
    free(w); free(d); free(U);
    return rc;
  }
  /* U_k = A z_k over the interior unknowns (boundary values of z taken as 0) */
  for (int k = 0; U && k < K; k++) {
    const double *z = Z + (int64_t)k * ntot;
    for (int64_t i = 0; i < n; i++) {
      double s = d[i] * z[i];
      for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++)
        if (C->st[e] < n) s += w[e] * z[C->st[e]];
      U[(int64_t)k * n + i] = s;
    }
  }
  for (int64_t i = 0; i < n; i++) {
    int32_t a = C->st_off[i];
    int m = C->st_off[i + 1] - a;
    int li = C->cells[C->node_cell[i]].level;
    double *f = feat + i * LIN;
    for (int j = 0; j < LNW; j++) f[j] = j < m ? w[a + j] / fabs(d[i]) : 0.0;
    for (int k = 0; k < 6; k++) {
      int32_t v = C->st[a + k];
      f[LNW + k] = v < n ? (double)(C->cells[C->node_cell[v]].level - li) : 0.0;
    }
    int nbnd = 0;
    for (int j = 0; j < m; j++) nbnd += C->st[a + j] >= n;
    f[46] = (double)m / (double)LNW;
    f[47] = (double)nbnd / (double)m;
    if (!U) continue;
    /* pattern of row i of M: J_0 = i, J_p = the p-th stencil node (p <= min(m, 40)) */
    int32_t J[LOUT];
    for (int p = 0; p < LOUT; p++) J[p] = p == 0 ? (int32_t)i : (p - 1 < m ? C->st[a + p - 1] : -1);
    double *q = quad + i * LQ;
    for (int t = 0; t < LQ; t++) q[t] = 0.0;
    for (int k = 0; k < K; k++) {
      double u[LOUT];
      for (int p = 0; p < LOUT; p++)
        u[p] = (J[p] >= 0 && J[p] < n) ? U[(int64_t)k * n + J[p]] / d[i] : 0.0;
      double zi = Z[(int64_t)k * ntot + i];
      int t = 0;
      for (int p = 0; p < LOUT; p++) {
        for (int r = 0; r <= p; r++) q[t++] += u[p] * u[r] / K;
        q[LQQ + p] += u[p] * zi / K;
      }
      q[LQ - 1] += zi * zi / K;
    }
  }
  free(w); free(d); free(U);
  return 0;
}

int apco_mlp_loss_grad(const double *P, const double *feat, const double *quad,
                       const int32_t *rows, int B, double *loss, double *grad) {
  const double *W1 = P, *b1 = W1 + LIN * LHID, *W2 = b1 + LHID, *b2 = W2 + LHID * LHID,
               *W3 = b2 + LHID, *b3 = W3 + LHID * LOUT;
  int np = LIN * LHID + LHID + LHID * LHID + LHID + LHID * LOUT + LOUT;
  double *gW1 = grad, *gb1 = gW1 + LIN * LHID, *gW2 = gb1 + LHID, *gb2 = gW2 + LHID * LHID,
         *gW3 = gb2 + LHID, *gb3 = gW3 + LHID * LOUT;
  for (int t = 0; t < np; t++) grad[t] = 0.0;
  double total = 0.0;
  for (int bi = 0; bi < B; bi++) {
    const double *x = feat + (int64_t)rows[bi] * LIN;
    const double *q = quad + (int64_t)rows[bi] * LQ;
    double h1[LHID], h2[LHID], o[LOUT];
    for (int j = 0; j < LHID; j++) {
      double s = b1[j];
      for (int i = 0; i < LIN; i++) s += x[i] * W1[i * LHID + j];
      h1[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < LHID; j++) {
      double s = b2[j];
      for (int i = 0; i < LHID; i++) s += h1[i] * W2[i * LHID + j];
      h2[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < LOUT; j++) {
      double s = b3[j];
      for (int i = 0; i < LHID; i++) s += h2[i] * W3[i * LOUT + j];
      o[j] = s;
    }
    /* L = m^T Q m - 2 b^T m + c with Q symmetric from its packed lower triangle */
    double m[LOUT], Qm[LOUT], dO[LOUT];
    for (int k = 0; k < LOUT; k++) m[k] = o[k] + (k == 0 ? 1.0 : 0.0);
    for (int p = 0; p < LOUT; p++) {
      Qm[p] = 0.0;
      for (int r = 0; r < LOUT; r++) {
        int hi = p > r ? p : r, lo = p > r ? r : p;
        Qm[p] += q[hi * (hi + 1) / 2 + lo] * m[r];
      }
    }
    double L = q[LQ - 1];
    for (int p = 0; p < LOUT; p++) {
      L += m[p] * Qm[p] - 2.0 * q[LQQ + p] * m[p];
      dO[p] = 2.0 * (Qm[p] - q[LQQ + p]) / B;
    }
    total += L;
    /* back-propagation */
    double dh2[LHID], dh1[LHID];
    for (int j = 0; j < LOUT; j++) {
      gb3[j] += dO[j];
      for (int i = 0; i < LHID; i++) gW3[i * LOUT + j] += h2[i] * dO[j];
    }
    for (int i = 0; i < LHID; i++) {
      double s = 0.0;
      for (int j = 0; j < LOUT; j++) s += dO[j] * W3[i * LOUT + j];
      dh2[i] = h2[i] > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < LHID; j++) {
      gb2[j] += dh2[j];
      for (int i = 0; i < LHID; i++) gW2[i * LHID + j] += h1[i] * dh2[j];
    }
    for (int i = 0; i < LHID; i++) {
      double s = 0.0;
      for (int j = 0; j < LHID; j++) s += dh2[j] * W2[i * LHID + j];
      dh1[i] = h1[i] > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < LHID; j++) {
      gb1[j] += dh1[j];
      for (int i = 0; i < LIN; i++) gW1[i * LHID + j] += x[i] * dh1[j];
    }
  }
  *loss = total / B;
  return 0;
}

int apco_mlp_forward(const double *P, const double *feat, int64_t nrow, double *out) {
  const double *W1 = P, *b1 = W1 + LIN * LHID, *W2 = b1 + LHID, *b2 = W2 + LHID * LHID,
               *W3 = b2 + LHID, *b3 = W3 + LHID * LOUT;
  for (int64_t r = 0; r < nrow; r++) {
    const double *x = feat + r * LIN;
    double h1[LHID], h2[LHID];
    for (int j = 0; j < LHID; j++) {
      double s = b1[j];
      for (int i = 0; i < LIN; i++) s += x[i] * W1[i * LHID + j];
      h1[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < LHID; j++) {
      double s = b2[j];
      for (int i = 0; i < LHID; i++) s += h1[i] * W2[i * LHID + j];
      h2[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < LOUT; j++) {
      double s = b3[j];
      for (int i = 0; i < LHID; i++) s += h2[i] * W3[i * LOUT + j];
      out[r * LOUT + j] = s;
    }
  }
  return 0;
}

/* Rows of M: the network output on every row (m_i = (e_0 + o_i) / d_i on the
   operator's pattern, boundary columns 0), then, with probes, the safeguard
   m_i <- j_i + alpha_i (m_i - j_i) on every row, alpha_i in [0, 1] minimising the
   row's probe loss.  Rows longer than 40 stencil nodes (fourth order) keep their
   first 40, the nearest. */
int apco_learned_m(const apco_cloud *C, const double *params, const double *Z, int K,
                   double *mdiag, double *mw) {
  int64_t n = C->n, ntot = C->n + C->nb, nnz = C->st_off[n];
  double *w = malloc((size_t)(nnz + 1) * sizeof(double));
  double *d = malloc((size_t)(n + 1) * sizeof(double));
  double *feat = malloc((size_t)(n + 1) * LIN * sizeof(double));
  double *o = malloc((size_t)(n + 1) * LOUT * sizeof(double));
  double *U = (Z && K > 0) ? malloc((size_t)K * n * sizeof(double)) : NULL;
  int rc = (!w || !d || !feat || !o || (Z && K > 0 && !U)) ? APCO_ENOMEM : 0;
  if (!rc) rc = apco_assemble(C, w, d);
  if (!rc) rc = apco_learn_data(C, NULL, 0, feat, NULL);
  if (!rc) rc = apco_mlp_forward(params, feat, n, o);
  if (rc) {
    free(w); free(d); free(feat); free(o); free(U);
    return rc;
  }
  for (int64_t i = 0; i < n; i++) {
    int32_t a = C->st_off[i];
    int m = C->st_off[i + 1] - a;
    mdiag[i] = (1.0 + o[i * LOUT]) / d[i];
    for (int p = 1; p <= m; p++) {
      int32_t v = C->st[a + p - 1];
      mw[a + p - 1] = (v < n && p < LOUT) ? o[i * LOUT + p] / d[i] : 0.0;
    }
  }
  for (int k = 0; U && k < K; k++) {
    const double *z = Z + (int64_t)k * ntot;
    for (int64_t i = 0; i < n; i++) {
      double s = d[i] * z[i];
      for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++)
        if (C->st[e] < n) s += w[e] * z[C->st[e]];
      U[(int64_t)k * n + i] = s;
    }
  }
  for (int64_t i = 0; U && i < n; i++) {
    int32_t a = C->st_off[i];
    int m = C->st_off[i + 1] - a;
    double jd = 1.0 / d[i], st = 0.0, tt = 0.0;
    for (int k = 0; k < K; k++) {
      const double *Uk = U + (int64_t)k * n;
      double sk = Uk[i] * jd - Z[(int64_t)k * ntot + i];
      double tk = (mdiag[i] - jd) * Uk[i];
      for (int p = 1; p <= m; p++) {
        int32_t v = C->st[a + p - 1];
        if (v < n) tk += mw[a + p - 1] * Uk[v];
      }
      st += sk * tk;
      tt += tk * tk;
    }
    double al = tt > 0.0 ? -st / tt : 1.0;
    al = al < 0.0 ? 0.0 : (al > 1.0 ? 1.0 : al);
    mdiag[i] = jd + al * (mdiag[i] - jd);
    for (int p = 1; p <= m; p++) mw[a + p - 1] *= al;
  }
  free(w); free(d); free(feat); free(o); free(U);
  return 0;
}

int apco_node_orders(const apco_cloud *C, int8_t *ord) {
  memcpy(ord, C->node_order, (size_t)C->n);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Particle push of the Vlasov-Poisson time loop (Sec. 1: particles move in the
   field that the three steps of Sec. 3.2 compute from their own positions).  The
   paper does not name its time integrator; the reading here is the leapfrog
   scheme in kick-drift form, velocities staggered half a step behind positions:
       v <- v + kick * grad phi(x),     x <- x + dt * v,
   kick being dt times the caller's charge-to-mass coupling.  Every product and
   every sum is rounded on its own (the library is built without contraction).
   Walls: a particle that ends outside Omega is reflected specularly.  Per axis,
   u = (x - lo) / L is outside [0, 1]; with f = floor(u) whole lengths and
   r = u - f, the position after f wall crossings is r (f even) or 1 - r (f odd),
   x = lo + u L, and the velocity component flips sign when f is odd.  A particle
   inside Omega keeps x + dt v as computed.  On a periodic domain a particle that
   leaves through one face re-enters through the opposite one: u = r, velocity
   unchanged. */
int apco_push(const apco_params *P, int64_t N, double *xyz, double *vel, const double *grad,
              double kick, double dt) {
  if (!P || N < 0 || !(P->L > 0.0) || !isfinite(kick) || !isfinite(dt)) return APCO_EINVAL;
  if (N > 0 && (!xyz || !vel || !grad)) return APCO_EINVAL;
  for (int d = 0; d < 3; d++) {
    const double lo = P->lo[d], hi = P->lo[d] + P->L;
    for (int64_t i = 0; i < N; i++) {
      double v = vel[d * N + i] + kick * grad[d * N + i];
      double x = xyz[d * N + i] + dt * v;
      if (x < lo || x > hi) {
        double u = (x - lo) / P->L;
        const double f = floor(u);
        const double r = u - f;
        const int odd = !P->periodic && fmod(f, 2.0) != 0.0;
        u = odd ? 1.0 - r : r;
        if (odd) v = -v;
        x = lo + u * P->L;
      }
      xyz[d * N + i] = x;
      vel[d * N + i] = v;
    }
  }
  return 0;
}

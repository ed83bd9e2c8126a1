/*
 * apc_oracle2d.c -- the two-dimensional AP-Cloud oracle (quadtree, k = 2).
 * TEST INFRASTRUCTURE ONLY (see apc_oracle2d.h).  Plain loops in FP64, in the
 * order of the paper's steps: quadtree and node selection (Sec. 4: error balance,
 * 2:1 balance, boundary nodes), GFD stencils and least squares (Sec. 3.1), density
 * rows and deposit (Sec. 3.2, eq. density_apcloud / density_linear_system),
 * Poisson rows (eq. Poisson), BiCGSTAB, derivatives and Taylor interpolation
 * (Sec. 3.2 step 3).
 */
#include "apc_oracle2d.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define P2 5   /* unknowns of the second-order fit: x, y, xx, xy, yy */
#define MAXM2 64

typedef struct {
  int32_t level, ix, iy;
  int64_t child; /* first of 4 children, -1 for a leaf */
  int64_t first, count;
} qcell;

struct apco2_cloud {
  apco_params P;
  int64_t N;
  double T[32];
  double unit;
  int64_t *perm;
  uint64_t *skey;
  qcell *cells;
  int64_t ncells, capcells, nopened;
  int64_t n, nb;
  int64_t *node_cell, *cell_node;
  int32_t *crd; /* 2 (n + nb), node-major */
  int32_t *bowner, *bface, *bidx;
  int32_t *r1off, *r1;
  int32_t *st_off, *st, *st_ring;
};

static uint64_t morton2(uint64_t x, uint64_t y, int bits) {
  uint64_t k = 0;
  for (int b = 0; b < bits; b++) {
    k |= ((x >> b) & 1ull) << (2 * b + 1);
    k |= ((y >> b) & 1ull) << (2 * b);
  }
  return k;
}

typedef struct {
  uint64_t key;
  int64_t idx;
} kp2;

static int cmp_kp2(const void *a, const void *b) {
  const kp2 *x = a, *y = b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

static int64_t lower_bound2(const uint64_t *a, int64_t lo, int64_t hi, uint64_t v) {
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

void apco2_destroy(apco2_cloud *C) {
  if (!C) return;
  free(C->perm); free(C->skey); free(C->cells); free(C->node_cell); free(C->cell_node);
  free(C->crd); free(C->bowner); free(C->bface); free(C->bidx); free(C->r1off); free(C->r1);
  free(C->st_off); free(C->st); free(C->st_ring);
  free(C);
}

static int push2(apco2_cloud *C, qcell c) {
  if (C->ncells == C->capcells) {
    int64_t nc = C->capcells ? 2 * C->capcells : 1024;
    qcell *q = realloc(C->cells, (size_t)nc * sizeof(qcell));
    if (!q) return APCO_ENOMEM;
    C->cells = q;
    C->capcells = nc;
  }
  C->cells[C->ncells++] = c;
  return 0;
}

/* open a cell: its 4 children (child c: x bit c >> 1, y bit c & 1) go to the end of
   Q with the sub-ranges of the parent's sorted particles carrying their key prefix */
static int open2(apco2_cloud *C, int64_t i) {
  const int D = C->P.max_depth;
  qcell par = C->cells[i];
  int64_t first = C->ncells;
  int lv = par.level + 1, sh = 2 * (D - lv);
  for (int c = 0; c < 4; c++) {
    qcell ch;
    ch.level = lv;
    ch.ix = 2 * par.ix + ((c >> 1) & 1);
    ch.iy = 2 * par.iy + (c & 1);
    ch.child = -1;
    uint64_t pre = morton2((uint64_t)ch.ix, (uint64_t)ch.iy, lv);
    int64_t a = lower_bound2(C->skey, par.first, par.first + par.count, pre << sh);
    int64_t b = lower_bound2(C->skey, par.first, par.first + par.count, (pre + 1) << sh);
    ch.first = a;
    ch.count = b - a;
    int rc = push2(C, ch);
    if (rc) return rc;
  }
  C->cells[i].child = first;
  C->nopened++;
  return 0;
}

/* face neighbour (Sec. 4.3): the deepest cell of Q of level <= level(i) sharing
   face f of cell i; -1 on the domain boundary */
static int64_t face_nb2(const apco2_cloud *C, int64_t i, int f) {
  const qcell *y = &C->cells[i];
  int32_t t[2] = {y->ix, y->iy};
  t[f / 2] += (f & 1) ? 1 : -1;
  if (t[f / 2] < 0 || t[f / 2] >= (1 << y->level)) return -1;
  int64_t cur = 0;
  while (C->cells[cur].child >= 0 && C->cells[cur].level < y->level) {
    int sh = y->level - C->cells[cur].level - 1;
    int c = (((t[0] >> sh) & 1) << 1) | ((t[1] >> sh) & 1);
    cur = C->cells[cur].child + c;
  }
  return cur;
}

typedef struct {
  int64_t r2;
  int32_t idx;
} cand2;

static int cmp_cand2(const void *a, const void *b) {
  const cand2 *x = a, *y = b;
  if (x->r2 != y->r2) return x->r2 < y->r2 ? -1 : 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

/* closed quadrant q (sign bits x = q >> 1, y = q & 1): a zero offset counts on both
   sides */
static int in_quad(int q, int64_t dx, int64_t dy) {
  int sx = (q >> 1) & 1 ? 1 : -1, sy = q & 1 ? 1 : -1;
  return sx * dx >= 0 && sy * dy >= 0;
}

/* Weighted least squares of the second-order Taylor fit (Sec. 3.1) over the m
   offsets (dx, dy): W_j = (exp(-r_j^2/r_max^2) - e^-4) / (1 - e^-4), V0 rows
   (x, y, x^2/2, xy, y^2/2) in units of h = max |offset|; X (5 x m) = R^-1 Q^T W,
   so that the scaled derivatives (h f_x, h f_y, h^2 f_xx, h^2 f_xy, h^2 f_yy) of
   the fit are X (f_j - f_0).  ratio = min|R_ii| / max|R_ii| (Householder QR). */
static void wls2(int m, const double *dx, const double *dy, double *X, double *hout,
                 double *ratio) {
  double h = 0.0, r2max = 0.0, r2[MAXM2], W[MAXM2];
  for (int j = 0; j < m; j++) {
    if (fabs(dx[j]) > h) h = fabs(dx[j]);
    if (fabs(dy[j]) > h) h = fabs(dy[j]);
    r2[j] = dx[j] * dx[j] + dy[j] * dy[j];
    if (r2[j] > r2max) r2max = r2[j];
  }
  *hout = h;
  *ratio = 0.0;
  if (h == 0.0 || m < P2) return;
  const double e4 = exp(-4.0);
  for (int j = 0; j < m; j++) W[j] = (exp(-r2[j] / r2max) - e4) / (1.0 - e4);
  double A[P2 * MAXM2], V[P2 * MAXM2], beta[P2];
  for (int j = 0; j < m; j++) {
    const double x = dx[j] / h, y = dy[j] / h;
    const double row[P2] = {x, y, 0.5 * x * x, x * y, 0.5 * y * y};
    for (int c = 0; c < P2; c++) A[c * m + j] = W[j] * row[c];
  }
  for (int c = 0; c < P2; c++) {
    double nrm2 = 0.0;
    for (int j = c; j < m; j++) nrm2 += A[c * m + j] * A[c * m + j];
    const double nrm = sqrt(nrm2);
    for (int j = 0; j < m; j++) V[c * m + j] = 0.0;
    if (nrm == 0.0) {
      beta[c] = 0.0;
      continue;
    }
    const double alpha = A[c * m + c] >= 0.0 ? -nrm : nrm;
    for (int j = c; j < m; j++) V[c * m + j] = A[c * m + j];
    V[c * m + c] -= alpha;
    double vn2 = 0.0;
    for (int j = c; j < m; j++) vn2 += V[c * m + j] * V[c * m + j];
    beta[c] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    for (int c2 = c + 1; c2 < P2; c2++) {
      double s = 0.0;
      for (int j = c; j < m; j++) s += V[c * m + j] * A[c2 * m + j];
      s *= beta[c];
      for (int j = c; j < m; j++) A[c2 * m + j] -= s * V[c * m + j];
    }
    A[c * m + c] = alpha;
  }
  double rmin = INFINITY, rmax = 0.0;
  for (int c = 0; c < P2; c++) {
    const double d = fabs(A[c * m + c]);
    if (d < rmin) rmin = d;
    if (d > rmax) rmax = d;
  }
  *ratio = rmax > 0.0 ? rmin / rmax : 0.0;
  if (!(*ratio > 0.0)) return;
  /* X = R^-1 Q^T W: for each j, Q^T e_j by the reflectors, times W_j, then back
     substitution */
  for (int j = 0; j < m; j++) {
    double e[MAXM2];
    for (int i = 0; i < m; i++) e[i] = i == j ? W[j] : 0.0;
    for (int c = 0; c < P2; c++) {
      double s = 0.0;
      for (int i = c; i < m; i++) s += V[c * m + i] * e[i];
      s *= beta[c];
      for (int i = c; i < m; i++) e[i] -= s * V[c * m + i];
    }
    for (int c = P2 - 1; c >= 0; c--) {
      double s = e[c];
      for (int c2 = c + 1; c2 < P2; c2++) s -= A[c2 * m + c] * X[c2 * m + j];
      X[c * m + j] = s / A[c * m + c];
    }
  }
}

/* stencil choice from candidates sorted by (r^2, index): per closed quadrant its
   two nearest candidates, then the nearest remaining ones up to min(count, m_cap);
   kept in candidate order.  Returns m on acceptance, 0 otherwise. */
static int choose2(const apco2_cloud *C, int32_t y, cand2 *cd, int64_t cnt, int m_cap) {
  const int32_t *c0 = &C->crd[2 * y];
  int64_t want = cnt < m_cap ? cnt : m_cap, got = 0;
  unsigned char *pick = calloc((size_t)(cnt > 0 ? cnt : 1), 1);
  if (!pick) return 0;
  for (int q = 0; q < 4; q++) {
    int taken = 0;
    for (int64_t j = 0; j < cnt && taken < 2; j++) {
      const int32_t *c1 = &C->crd[2 * cd[j].idx];
      if (!in_quad(q, (int64_t)c1[0] - c0[0], (int64_t)c1[1] - c0[1])) continue;
      taken++;
      if (!pick[j] && got < want) {
        pick[j] = 1;
        got++;
      }
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
  free(pick);
  if (m < P2 + 1 || m > MAXM2) return 0;
  int quad[4] = {0, 0, 0, 0};
  double dx[MAXM2], dy[MAXM2], X[P2 * MAXM2], h, ratio;
  for (int j = 0; j < m; j++) {
    const int32_t *c1 = &C->crd[2 * cd[j].idx];
    dx[j] = (double)((int64_t)c1[0] - c0[0]);
    dy[j] = (double)((int64_t)c1[1] - c0[1]);
    for (int q = 0; q < 4; q++) quad[q] += in_quad(q, (int64_t)dx[j], (int64_t)dy[j]);
  }
  for (int q = 0; q < 4; q++)
    if (quad[q] < 1) return 0;
  wls2(m, dx, dy, X, &h, &ratio);
  if (!(ratio >= 1e-6)) return 0;
  return m;
}

typedef struct {
  uint64_t code;
  int64_t cell;
} lp2;

static int cmp_lp2(const void *a, const void *b) {
  const lp2 *x = a, *y = b;
  return (x->code > y->code) - (x->code < y->code);
}

#define FAIL(rc_)      \
  do {                 \
    apco2_destroy(C);  \
    return (rc_);      \
  } while (0)

int apco2_build_cloud(const apco_params *P, const double *xy, int64_t N, apco2_cloud **out) {
  *out = NULL;
  if (!P || !xy || N < 1 || P->order != 2 || P->max_depth < 1 || P->max_depth > 20 ||
      !(P->L > 0.0) || !(P->c > 0.0) || P->ring_min < 1 || P->ring_max < P->ring_min ||
      P->m_cap < P2 + 1 || P->m_cap > MAXM2 || P->criterion_pow < 0 || P->criterion_pow > 16)
    return APCO_EINVAL;
  apco2_cloud *C = calloc(1, sizeof(apco2_cloud));
  if (!C) return APCO_ENOMEM;
  C->P = *P;
  C->N = N;
  const int D = P->max_depth;
  C->unit = P->L / ldexp(1.0, D + 1);
  const int pw = P->criterion_pow > 0 ? P->criterion_pow : 2;
  for (int l = 0; l <= D; l++) {
    const double t = (P->c * ldexp(1.0, l)) / P->L;
    double v = 1.0;
    for (int e = 0; e < pw; e++) v *= t;
    C->T[l] = v;
  }
  /* Morton keys at max_depth (u = floor((x - lo) 2^D / L), clamped) and a stable sort */
  kp2 *kp = malloc((size_t)N * sizeof(kp2));
  if (!kp) FAIL(APCO_ENOMEM);
  const double s = ldexp(1.0, D) / P->L;
  const int64_t top = ((int64_t)1 << D) - 1;
  for (int64_t i = 0; i < N; i++) {
    int64_t u[2];
    for (int d = 0; d < 2; d++) {
      const double x = xy[d * N + i];
      if (isnan(x)) {
        free(kp);
        FAIL(APCO_EINVAL);
      }
      if (x < P->lo[d] || x > P->lo[d] + P->L) {
        free(kp);
        FAIL(APCO_EDOMAIN);
      }
      int64_t v = (int64_t)floor((x - P->lo[d]) * s);
      u[d] = v < 0 ? 0 : (v > top ? top : v);
    }
    kp[i].key = morton2((uint64_t)u[0], (uint64_t)u[1], D);
    kp[i].idx = i;
  }
  qsort(kp, (size_t)N, sizeof(kp2), cmp_kp2);
  C->perm = malloc((size_t)N * sizeof(int64_t));
  C->skey = malloc((size_t)N * sizeof(uint64_t));
  if (!C->perm || !C->skey) {
    free(kp);
    FAIL(APCO_ENOMEM);
  }
  for (int64_t i = 0; i < N; i++) {
    C->perm[i] = kp[i].idx;
    C->skey[i] = kp[i].key;
  }
  free(kp);
  /* node selection: Q = {root}; open every cell with N' >= T_l below max_depth
     (children appended are visited too) */
  qcell root = {0, 0, 0, -1, 0, N};
  if (push2(C, root)) FAIL(APCO_ENOMEM);
  for (int64_t i = 0; i < C->ncells; i++) {
    const qcell *c = &C->cells[i];
    if (c->level < D && (double)c->count >= C->T[c->level])
      if (open2(C, i)) FAIL(APCO_ENOMEM);
  }
  int lq = 0;
  for (int64_t i = 0; i < C->ncells; i++)
    if (C->cells[i].level > lq) lq = C->cells[i].level;
  /* 2:1 balance from the deepest level up: each leaf at level l opens every face
     neighbour that is a leaf more than one level coarser */
  for (int l = lq; l >= 1; l--)
    for (int64_t i = 0; i < C->ncells; i++) {
      if (C->cells[i].child >= 0 || C->cells[i].level != l) continue;
      for (int f = 0; f < 4; f++)
        for (;;) {
          const int64_t z = face_nb2(C, i, f);
          if (z < 0 || C->cells[z].child >= 0 || C->cells[z].level >= l - 1) break;
          if (open2(C, z)) FAIL(APCO_ENOMEM);
        }
    }
  /* nodes: the leaves in Morton order of their minimum corner */
  const int64_t n = C->ncells - C->nopened;
  lp2 *lp = malloc((size_t)n * sizeof(lp2));
  if (!lp) FAIL(APCO_ENOMEM);
  int64_t k = 0;
  for (int64_t i = 0; i < C->ncells; i++) {
    const qcell *c = &C->cells[i];
    if (c->child >= 0) continue;
    const int sh = D - c->level;
    lp[k].code = morton2((uint64_t)c->ix << sh, (uint64_t)c->iy << sh, D);
    lp[k].cell = i;
    k++;
  }
  qsort(lp, (size_t)n, sizeof(lp2), cmp_lp2);
  C->n = n;
  C->node_cell = malloc((size_t)n * sizeof(int64_t));
  C->cell_node = malloc((size_t)C->ncells * sizeof(int64_t));
  C->bidx = malloc((size_t)n * 4 * sizeof(int32_t));
  if (!C->node_cell || !C->cell_node || !C->bidx) {
    free(lp);
    FAIL(APCO_ENOMEM);
  }
  for (int64_t i = 0; i < C->ncells; i++) C->cell_node[i] = -1;
  for (int64_t j = 0; j < n; j++) {
    C->node_cell[j] = lp[j].cell;
    C->cell_node[lp[j].cell] = j;
  }
  free(lp);
  /* boundary nodes at the centre of every leaf face on the boundary */
  int64_t nb = 0;
  for (int64_t j = 0; j < n; j++)
    for (int f = 0; f < 4; f++)
      C->bidx[4 * j + f] = face_nb2(C, C->node_cell[j], f) < 0 ? (int32_t)(n + nb++) : -1;
  C->nb = nb;
  C->crd = malloc((size_t)2 * (n + nb) * sizeof(int32_t));
  C->bowner = malloc((size_t)(nb + 1) * sizeof(int32_t));
  C->bface = malloc((size_t)(nb + 1) * sizeof(int32_t));
  if (!C->crd || !C->bowner || !C->bface) FAIL(APCO_ENOMEM);
  for (int64_t j = 0; j < n; j++) {
    const qcell *c = &C->cells[C->node_cell[j]];
    const int32_t sz = 1 << (D - c->level);
    C->crd[2 * j] = (2 * c->ix + 1) * sz;
    C->crd[2 * j + 1] = (2 * c->iy + 1) * sz;
    for (int f = 0; f < 4; f++) {
      const int32_t b = C->bidx[4 * j + f];
      if (b < 0) continue;
      C->crd[2 * b] = C->crd[2 * j];
      C->crd[2 * b + 1] = C->crd[2 * j + 1];
      C->crd[2 * b + f / 2] += (f & 1) ? sz : -sz;
      C->bowner[b - n] = (int32_t)j;
      C->bface[b - n] = f;
    }
  }
  /* 1-ring: per face the neighbour if it is a leaf, else its 2 children on the
     shared face; a boundary face gives its boundary node */
  C->r1off = malloc((size_t)(n + 1) * sizeof(int32_t));
  C->r1 = malloc((size_t)n * 8 * sizeof(int32_t));
  if (!C->r1off || !C->r1) FAIL(APCO_ENOMEM);
  int64_t e = 0;
  for (int64_t j = 0; j < n; j++) {
    C->r1off[j] = (int32_t)e;
    for (int f = 0; f < 4; f++) {
      const int64_t z = face_nb2(C, C->node_cell[j], f);
      if (z < 0) {
        C->r1[e++] = C->bidx[4 * j + f];
        continue;
      }
      if (C->cells[z].child < 0) {
        C->r1[e++] = (int32_t)C->cell_node[z];
        continue;
      }
      const int d = f / 2, side = (f & 1) ? 0 : 1;
      for (int c = 0; c < 4; c++) {
        const int bit = d == 0 ? (c >> 1) & 1 : c & 1;
        if (bit != side) continue;
        const int64_t ch = C->cells[z].child + c;
        if (C->cells[ch].child >= 0) FAIL(APCO_EINVAL); /* not 2:1 balanced */
        C->r1[e++] = (int32_t)C->cell_node[ch];
      }
    }
  }
  C->r1off[n] = (int32_t)e;
  /* stencils: the R-ring by face adjacency (boundary nodes hang off their owner)
     sorted by (r^2, index), from ring_min up until one is accepted */
  const int64_t ntot = n + nb;
  int32_t *stamp = malloc((size_t)ntot * sizeof(int32_t));
  int32_t *front = malloc((size_t)ntot * sizeof(int32_t));
  cand2 *cand = malloc((size_t)ntot * sizeof(cand2));
  C->st_off = malloc((size_t)(n + 1) * sizeof(int32_t));
  C->st_ring = malloc((size_t)(n + 1) * sizeof(int32_t));
  int64_t stcap = n * (int64_t)P->m_cap + 16;
  C->st = malloc((size_t)stcap * sizeof(int32_t));
  if (!stamp || !front || !cand || !C->st_off || !C->st_ring || !C->st) {
    free(stamp); free(front); free(cand);
    FAIL(APCO_ENOMEM);
  }
  for (int64_t i = 0; i < ntot; i++) stamp[i] = -1;
  int64_t ne = 0;
  int rc = 0;
  for (int64_t y = 0; y < n && !rc; y++) {
    C->st_off[y] = (int32_t)ne;
    int done = 0;
    for (int R = P->ring_min; R <= P->ring_max && !done; R++) {
      int64_t nf = 0, lo = 0, cnt = 0;
      stamp[y] = (int32_t)y;
      front[nf++] = (int32_t)y;
      for (int depth = 1; depth <= R; depth++) {
        const int64_t hi = nf;
        for (int64_t t = lo; t < hi; t++) {
          const int32_t u = front[t];
          if (u >= n) {
            const int32_t v = C->bowner[u - n];
            if (stamp[v] != (int32_t)y) {
              stamp[v] = (int32_t)y;
              front[nf++] = v;
            }
            continue;
          }
          for (int32_t a = C->r1off[u]; a < C->r1off[u + 1]; a++) {
            const int32_t v = C->r1[a];
            if (stamp[v] != (int32_t)y) {
              stamp[v] = (int32_t)y;
              front[nf++] = v;
            }
          }
        }
        lo = hi;
      }
      for (int64_t t = 1; t < nf; t++) {
        const int32_t v = front[t];
        const int64_t d0 = (int64_t)C->crd[2 * v] - C->crd[2 * y];
        const int64_t d1 = (int64_t)C->crd[2 * v + 1] - C->crd[2 * y + 1];
        cand[cnt].r2 = d0 * d0 + d1 * d1;
        cand[cnt].idx = v;
        cnt++;
      }
      for (int64_t t = 0; t < nf; t++) stamp[front[t]] = -1;
      qsort(cand, (size_t)cnt, sizeof(cand2), cmp_cand2);
      const int m = choose2(C, (int32_t)y, cand, cnt, P->m_cap);
      if (m > 0) {
        for (int j = 0; j < m; j++) C->st[ne++] = cand[j].idx;
        C->st_ring[y] = R;
        done = 1;
      }
    }
    if (!done) rc = APCO_ESTENCIL;
  }
  C->st_off[n] = (int32_t)ne;
  free(stamp); free(front); free(cand);
  if (rc) FAIL(rc);
  *out = C;
  return 0;
}

int apco2_info(const apco2_cloud *C, int64_t *n, int64_t *nb, int64_t *nnz, int64_t *n_opened) {
  if (n) *n = C->n;
  if (nb) *nb = C->nb;
  if (nnz) *nnz = C->st_off[C->n];
  if (n_opened) *n_opened = C->nopened;
  return 0;
}

int apco2_get_nodes(const apco2_cloud *C, int64_t *perm, uint64_t *code, int32_t *level,
                    int64_t *first, int64_t *count, int32_t *bowner, int32_t *bface,
                    int32_t *st_off, int32_t *st_idx) {
  const int D = C->P.max_depth;
  if (perm) memcpy(perm, C->perm, (size_t)C->N * sizeof(int64_t));
  for (int64_t j = 0; j < C->n; j++) {
    const qcell *c = &C->cells[C->node_cell[j]];
    const int sh = D - c->level;
    if (code) code[j] = morton2((uint64_t)c->ix << sh, (uint64_t)c->iy << sh, D);
    if (level) level[j] = c->level;
    if (first) first[j] = c->first;
    if (count) count[j] = c->count;
  }
  if (bowner) memcpy(bowner, C->bowner, (size_t)C->nb * sizeof(int32_t));
  if (bface) memcpy(bface, C->bface, (size_t)C->nb * sizeof(int32_t));
  if (st_off) memcpy(st_off, C->st_off, (size_t)(C->n + 1) * sizeof(int32_t));
  if (st_idx) memcpy(st_idx, C->st, (size_t)C->st_off[C->n] * sizeof(int32_t));
  return 0;
}

int apco2_node_coords(const apco2_cloud *C, int32_t *ixy) {
  const int64_t nt = C->n + C->nb;
  for (int64_t j = 0; j < nt; j++) {
    ixy[j] = C->crd[2 * j];
    ixy[nt + j] = C->crd[2 * j + 1];
  }
  return 0;
}

int apco2_ring1(const apco2_cloud *C, int32_t *off, int32_t *idx, int64_t cap) {
  if (C->r1off[C->n] > cap) return APCO_EINVAL;
  memcpy(off, C->r1off, (size_t)(C->n + 1) * sizeof(int32_t));
  memcpy(idx, C->r1, (size_t)C->r1off[C->n] * sizeof(int32_t));
  return 0;
}

/* the fit of node y: X (5 x m) and the scale h (physical units) */
static void node_fit2(const apco2_cloud *C, int64_t y, double *X, int *m, double *hp) {
  const int32_t a = C->st_off[y];
  *m = C->st_off[y + 1] - a;
  double dx[MAXM2], dy[MAXM2], h, ratio;
  for (int j = 0; j < *m; j++) {
    const int32_t v = C->st[a + j];
    dx[j] = (double)((int64_t)C->crd[2 * v] - C->crd[2 * y]);
    dy[j] = (double)((int64_t)C->crd[2 * v + 1] - C->crd[2 * y + 1]);
  }
  wls2(*m, dx, dy, X, &h, &ratio);
  *hp = h * C->unit;
}

/* Laplacian row: w_j = (X_xx,j + X_yy,j) / h^2, diagonal -sum_j w_j */
int apco2_assemble(const apco2_cloud *C, double *w, double *diag) {
  double X[P2 * MAXM2], hp;
  int m;
  for (int64_t y = 0; y < C->n; y++) {
    node_fit2(C, y, X, &m, &hp);
    const int32_t a = C->st_off[y];
    double s = 0.0;
    for (int j = 0; j < m; j++) {
      const double v = (X[2 * m + j] + X[4 * m + j]) / (hp * hp);
      w[a + j] = v;
      s += v;
    }
    diag[y] = -s;
  }
  return 0;
}

/* Density row (eq. density_linear_system, NGP): the cell average of the fitted
   quadratic, a_{2 e_d} = (h_c/2)^2 / 3 / 2! per axis, b_j = a (X_xx,j + X_yy,j) /
   h^2 and diagonal 1 - sum_j b_j; kept when sum |b_j| <= (1 - sum b_j) / 2, else
   the identity row (order 0). */
int apco2_density_rows(const apco2_cloud *C, double *bw, double *bdiag, int8_t *ord) {
  double X[P2 * MAXM2], hp;
  int m;
  for (int64_t y = 0; y < C->n; y++) {
    node_fit2(C, y, X, &m, &hp);
    const double hc = C->P.L / ldexp(1.0, C->cells[C->node_cell[y]].level);
    const double a2 = (hc / 2.0) * (hc / 2.0) / 3.0 / 2.0;
    const int32_t a = C->st_off[y];
    double s = 0.0, sa = 0.0;
    for (int j = 0; j < m; j++) {
      const double v = a2 * (X[2 * m + j] + X[4 * m + j]) / (hp * hp);
      bw[a + j] = v;
      s += v;
      sa += fabs(v);
    }
    const int ok = sa <= 0.5 * (1.0 - s);
    if (!ok) {
      for (int j = 0; j < m; j++) bw[a + j] = 0.0;
      s = 0.0;
    }
    bdiag[y] = 1.0 - s;
    if (ord) ord[y] = ok ? 2 : 0;
  }
  return 0;
}

int apco2_deposit(const apco2_cloud *C, const double *q, double *rho_M) {
  const double q0 = 1.0 / (double)C->N;
  for (int64_t j = 0; j < C->n; j++) {
    const qcell *c = &C->cells[C->node_cell[j]];
    double sum = 0.0;
    if (q) {
      for (int64_t s = c->first; s < c->first + c->count; s++) sum += q[C->perm[s]];
    } else {
      sum = (double)c->count * q0;
    }
    const double hc = C->P.L / ldexp(1.0, c->level);
    rho_M[j] = sum / (hc * hc);
  }
  for (int64_t b = 0; b < C->nb; b++) rho_M[C->n + b] = rho_M[C->bowner[b]];
  return 0;
}

/* ---- BiCGSTAB on rows (diag, w) over the interior unknowns ---- */
static void matvec2(const apco2_cloud *C, const double *diag, const double *w, const double *x,
                    double *y) {
  for (int64_t i = 0; i < C->n; i++) {
    double s = diag[i] * x[i];
    for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++)
      if (C->st[e] < C->n) s += w[e] * x[C->st[e]];
    y[i] = s;
  }
}

static double dot2(const double *a, const double *b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

/* van der Vorst's BiCGSTAB, x0 = 0, shadow residual r0, optional right Jacobi
   preconditioning; stops when the recursive ||r|| / ||b|| <= tol and the true
   residual agrees, else restarts from the true residual */
static int bicgstab2(const apco2_cloud *C, const double *diag, const double *w, const double *b,
                     double *x, double tol, int maxit, int precond, apco_stats *st) {
  const int64_t n = C->n;
  double *r = calloc((size_t)n + 1, 8), *rh = calloc((size_t)n + 1, 8), *pv = calloc((size_t)n + 1, 8),
         *v = calloc((size_t)n + 1, 8), *s = calloc((size_t)n + 1, 8), *t = calloc((size_t)n + 1, 8),
         *ph = calloc((size_t)n + 1, 8), *sh = calloc((size_t)n + 1, 8);
  if (!r || !rh || !pv || !v || !s || !t || !ph || !sh) {
    free(r); free(rh); free(pv); free(v); free(s); free(t); free(ph); free(sh);
    return APCO_ENOMEM;
  }
  for (int64_t i = 0; i < n; i++) x[i] = 0.0;
  const double bn = sqrt(dot2(b, b, n));
  int it = 0, status = APCO_ENOCONV;
  double rel = 0.0, relt = 0.0;
  if (bn == 0.0) {
    status = 0;
  } else {
    memcpy(r, b, (size_t)n * 8);
    while (status != 0 && it < maxit) {
      memcpy(rh, r, (size_t)n * 8);
      for (int64_t i = 0; i < n; i++) pv[i] = v[i] = 0.0;
      double rho_old = 1.0, alpha = 1.0, omega = 1.0;
      int restart = 0;
      while (it < maxit && !restart) {
        it++;
        const double rho = dot2(rh, r, n);
        if (rho == 0.0 || !isfinite(rho)) break;
        const double beta = (rho / rho_old) * (alpha / omega);
        for (int64_t i = 0; i < n; i++) pv[i] = r[i] + beta * (pv[i] - omega * v[i]);
        for (int64_t i = 0; i < n; i++) ph[i] = precond ? pv[i] / diag[i] : pv[i];
        matvec2(C, diag, w, ph, v);
        const double rv = dot2(rh, v, n);
        if (rv == 0.0 || !isfinite(rv)) break;
        alpha = rho / rv;
        for (int64_t i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
        for (int64_t i = 0; i < n; i++) sh[i] = precond ? s[i] / diag[i] : s[i];
        matvec2(C, diag, w, sh, t);
        const double tt = dot2(t, t, n);
        omega = tt > 0.0 ? dot2(t, s, n) / tt : 0.0;
        for (int64_t i = 0; i < n; i++) x[i] += alpha * ph[i] + omega * sh[i];
        for (int64_t i = 0; i < n; i++) r[i] = s[i] - omega * t[i];
        rho_old = rho;
        rel = sqrt(dot2(r, r, n)) / bn;
        if (rel <= tol || omega == 0.0) restart = 1;
      }
      matvec2(C, diag, w, x, t);
      for (int64_t i = 0; i < n; i++) r[i] = b[i] - t[i];
      relt = sqrt(dot2(r, r, n)) / bn;
      if (relt <= tol) status = 0;
    }
  }
  if (st) {
    st->iters = it;
    st->status = status;
    st->rel_resid = rel;
    st->rel_resid_true = relt;
  }
  free(r); free(rh); free(pv); free(v); free(s); free(t); free(ph); free(sh);
  return status;
}

int apco2_density_solve(const apco2_cloud *C, const double *rho_M, double *rho_t, double tol,
                        int maxit, apco_stats *st) {
  const int64_t n = C->n, nnz = C->st_off[n];
  double *bw = malloc((size_t)(nnz + 1) * 8), *bd = malloc((size_t)(n + 1) * 8),
         *rhs = malloc((size_t)(n + 1) * 8);
  if (!bw || !bd || !rhs) {
    free(bw); free(bd); free(rhs);
    return APCO_ENOMEM;
  }
  apco2_density_rows(C, bw, bd, NULL);
  /* boundary columns carry their owner's rho_M and move to the right-hand side */
  for (int64_t i = 0; i < n; i++) {
    double s = rho_M[i];
    for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++)
      if (C->st[e] >= n) s -= bw[e] * rho_M[C->st[e]];
    rhs[i] = s;
  }
  int rc = bicgstab2(C, bd, bw, rhs, rho_t, tol, maxit, 0, st);
  for (int64_t b = 0; b < C->nb; b++) rho_t[n + b] = rho_M[n + b];
  free(bw); free(bd); free(rhs);
  return rc < 0 ? rc : 0;
}

int apco2_poisson_solve(const apco2_cloud *C, const double *rho_t, const double *g, double *phi,
                        double tol, int maxit, int precond, apco_stats *st) {
  const int64_t n = C->n, nnz = C->st_off[n];
  double *w = malloc((size_t)(nnz + 1) * 8), *d = malloc((size_t)(n + 1) * 8),
         *rhs = malloc((size_t)(n + 1) * 8);
  if (!w || !d || !rhs) {
    free(w); free(d); free(rhs);
    return APCO_ENOMEM;
  }
  apco2_assemble(C, w, d);
  for (int64_t i = 0; i < n; i++) {
    double s = C->P.poisson_c * rho_t[i];
    for (int32_t e = C->st_off[i]; e < C->st_off[i + 1]; e++)
      if (C->st[e] >= n && g) s -= w[e] * g[C->st[e] - n];
    rhs[i] = s;
  }
  int rc = bicgstab2(C, d, w, rhs, phi, tol, maxit, precond, st);
  for (int64_t b = 0; b < C->nb; b++) phi[n + b] = g ? g[b] : 0.0;
  free(w); free(d); free(rhs);
  return rc < 0 ? rc : 0;
}

/* derivatives of the fitted quadratic at each node, physical units */
int apco2_node_derivs(const apco2_cloud *C, const double *f, double *Dv) {
  double X[P2 * MAXM2], hp;
  int m;
  for (int64_t y = 0; y < C->n; y++) {
    node_fit2(C, y, X, &m, &hp);
    const int32_t a = C->st_off[y];
    for (int c = 0; c < P2; c++) {
      double s = 0.0;
      for (int j = 0; j < m; j++) s += X[c * m + j] * (f[C->st[a + j]] - f[y]);
      Dv[y * P2 + c] = s / (c < 2 ? hp : hp * hp);
    }
  }
  return 0;
}

/* Taylor polynomial of each particle's leaf node at the particle:
   phi_p = phi + f_x dx + f_y dy + f_xx dx^2/2 + f_xy dx dy + f_yy dy^2/2, and its
   gradient */
int apco2_interpolate(const apco2_cloud *C, const double *phi, const double *xy, double *phi_p,
                      double *grad) {
  const int64_t n = C->n, N = C->N;
  double *Dv = malloc((size_t)(n + 1) * P2 * 8);
  if (!Dv) return APCO_ENOMEM;
  apco2_node_derivs(C, phi, Dv);
  for (int64_t j = 0; j < n; j++) {
    const qcell *c = &C->cells[C->node_cell[j]];
    const double y0 = C->P.lo[0] + C->unit * (double)C->crd[2 * j];
    const double y1 = C->P.lo[1] + C->unit * (double)C->crd[2 * j + 1];
    const double *d = &Dv[j * P2];
    for (int64_t s = c->first; s < c->first + c->count; s++) {
      const int64_t i = C->perm[s];
      const double x = xy[i] - y0, y = xy[N + i] - y1;
      phi_p[i] = phi[j] + d[0] * x + d[1] * y + d[2] * (0.5 * x * x) + d[3] * (x * y) +
                 d[4] * (0.5 * y * y);
      grad[i] = d[0] + d[2] * x + d[3] * y;
      grad[N + i] = d[1] + d[3] * x + d[4] * y;
    }
  }
  free(Dv);
  return 0;
}

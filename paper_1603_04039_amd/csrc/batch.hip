// Batches of independent clouds on gfx950.
//
// A batch is held as one union cloud: the disjoint union of the clouds' node
// sets, interior nodes of cloud 0, 1, ... first, then their boundary nodes, with
// particle, node, stencil and sliced-layout arrays concatenated and re-indexed.
// Its operator is block diagonal, so the union's assembly, deposit, right-hand
// side, SpMV and interpolation are single launches over every cloud at once.
// What must stay per cloud is the Krylov iteration: each cloud runs its own
// BiCGSTAB (own scalars, own convergence test against its own right-hand side),
// so the batched solver keeps one scalar record per cloud and reduces dot
// products per cloud: SpMV products per slice (a slice never spans two clouds),
// vector products per row block (a block never spans two clouds), both summed
// in a fixed order by one workgroup per cloud.  Converged clouds skip their
// rows.  The 8 kernels of an iteration are recorded once in a HIP graph of C
// iterations and replayed until every cloud has stopped; the launch shape of the
// SpMV and C are picked by measurement (apc_batch_tune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>
#include <cstring>
#include <vector>

#include "apc_internal.h"
#include "spmv_core.h"
#include "prec_core.h"

void apc_free_cloud(apc_cloud *c);

namespace {

constexpr int RB = APC_BLOCK; // rows per row block of the vector kernels
constexpr int FB = 256;       // threads of a per-cloud finalize workgroup

struct BScal {
  double rho, alpha, omega, beta;
  double bnorm, rnorm, rtrue, tol;
  int it, maxit, done, fin; // done: iteration stopped (1 conv, 2 breakdown, 3 maxit); fin: 1 ok, 2 failed
  int nrest, reason, pad0, pad1;
};

// ---------------------------------------------------------------- merge kernels
// dst[i] = src[i] + (src[i] < thr ? add_lo : add_hi); negative entries kept when keep_neg
__global__ void __launch_bounds__(APC_BLOCK)
    k_map_i32(const int32_t *__restrict__ src, int64_t cnt, int32_t *__restrict__ dst,
              int32_t thr, int32_t add_lo, int32_t add_hi, int keep_neg) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= cnt) return;
  const int32_t v = src[i];
  dst[i] = (keep_neg && v < 0) ? v : v + (v < thr ? add_lo : add_hi);
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_add_i64(const int64_t *__restrict__ src, int64_t cnt, int64_t *__restrict__ dst, int64_t add) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < cnt) dst[i] = src[i] + add;
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_fill_i32v(int32_t *__restrict__ dst, int64_t cnt, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < cnt) dst[i] = v;
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_fill_f64(double *__restrict__ dst, int64_t cnt, double v) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < cnt) dst[i] = v;
}

// ---------------------------------------------------------------- batched BiCGSTAB
struct BDesc {
  const int32_t *sl_cloud;  // nsl: cloud of each slice
  const int32_t *rb_cloud;  // nrb: cloud of each row block
  const int32_t *rb_row0;   // nrb: first row of each row block
  const int32_t *rb_row1;   // nrb: one past the last row
  const int64_t *c_sl0, *c_nsl, *c_rb0, *c_nrb; // per cloud: slice / row-block ranges
  int64_t nsl, nrb;
  int count;
};

__device__ __forceinline__ double wsum(double v) { return wave_sum(v); }

// v = A ph ; per-slice partial (rh, v)
template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    kb_spmv_v(Op op, BDesc B, const BScal *__restrict__ sc, const double *__restrict__ ph,
              double *__restrict__ v, const double *__restrict__ rh, double *__restrict__ part) {
  const int lane = threadIdx.x & 63;
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    const int s = __builtin_amdgcn_readfirstlane(it.s);
    if (sc[B.sl_cloud[s]].done) continue;
    int32_t i;
    const double y = sell_apply<MODE>(op, ph, s, i);
    double val = 0.0;
    if (i >= 0) {
      v[i] = y;
      val = rh[i] * y;
    }
    val = wsum(val);
    if (lane == 0) part[s] = val;
  }
}

// t = A sh ; per-slice partials (t, s), (t, t)
template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    kb_spmv_t(Op op, BDesc B, const BScal *__restrict__ sc, const double *__restrict__ sh,
              const double *__restrict__ s_, double *__restrict__ t, double *__restrict__ part) {
  const int lane = threadIdx.x & 63;
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    const int s = __builtin_amdgcn_readfirstlane(it.s);
    if (sc[B.sl_cloud[s]].done) continue;
    int32_t i;
    const double y = sell_apply<MODE>(op, sh, s, i);
    double a = 0.0, b = 0.0;
    if (i >= 0) {
      t[i] = y;
      a = y * s_[i];
      b = y * y;
    }
    a = wsum(a);
    b = wsum(b);
    if (lane == 0) {
      part[s] = a;
      part[B.nsl + s] = b;
    }
  }
}

// out = M in (the learned preconditioner of the union) over the slices of the clouds
// still iterating; launched with op_lds(op) bytes of dynamic LDS
__global__ void __launch_bounds__(APC_BLOCK)
    kb_prec(Op op, MOp M, BDesc B, const BScal *__restrict__ sc, const double *__restrict__ in,
            double *__restrict__ out) {
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    const int s = __builtin_amdgcn_readfirstlane(it.s);
    if (sc[B.sl_cloud[s]].done) continue;
    const int u = op.sl_un ? op.sl_un[s] : 0;
    if (u > 0)
      prec_slice<false, true>(op, M, in, out, s, u);
    else if (op.sl_top4)
      prec_slice<true, false>(op, M, in, out, s, 0);
    else
      prec_slice<false, false>(op, M, in, out, s, 0);
  }
}

// restart from x (first: x = 0): r = b - A x, rh = r, p = v = 0; partials (r, r), (b, b)
template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    kb_restart(Op op, BDesc B, const BScal *__restrict__ sc, const double *__restrict__ b,
               const double *__restrict__ x, double *__restrict__ r, double *__restrict__ rh,
               double *__restrict__ p, double *__restrict__ v, double *__restrict__ part, int first) {
  const int lane = threadIdx.x & 63;
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    const int s = __builtin_amdgcn_readfirstlane(it.s);
    if (!first && sc[B.sl_cloud[s]].fin) continue;
    int32_t i = op.sl_rows[(int64_t)s * SL + lane];
    double y = 0.0;
    if (!first) y = sell_apply<MODE>(op, x, s, i);
    double rr = 0.0, bb = 0.0;
    if (i >= 0) {
      const double ri = b[i] - y;
      r[i] = ri;
      rh[i] = ri;
      p[i] = 0.0;
      v[i] = 0.0;
      rr = ri * ri;
      bb = b[i] * b[i];
    }
    rr = wsum(rr);
    bb = wsum(bb);
    if (lane == 0) {
      part[s] = rr;
      part[B.nsl + s] = bb;
    }
  }
}

// row-block reduction of NV values into part[k * nrb + blk]
template <int NV>
__device__ __forceinline__ void rb_partials(double (&v)[NV], double *part, int64_t nrb, int64_t blk) {
  __shared__ double sh[NV][RB / 64];
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
      for (int q = 0; q < RB / 64; q++) s += sh[k][q];
      part[(int64_t)k * nrb + blk] = s;
    }
  }
}

// p = r + beta (p - omega v); ph = D^-1 p (Jacobi) or p
template <bool JAC>
__global__ void __launch_bounds__(RB)
    kb_upd_p(BDesc B, const BScal *__restrict__ sc, const double *__restrict__ r,
             double *__restrict__ p, const double *__restrict__ v, double *__restrict__ ph,
             const double *__restrict__ invd) {
  const int64_t blk = blockIdx.x;
  const BScal &c = sc[B.rb_cloud[blk]];
  if (c.done) return;
  const int64_t i = B.rb_row0[blk] + threadIdx.x;
  if (i >= B.rb_row1[blk]) return;
  const double pi = r[i] + c.beta * (p[i] - c.omega * v[i]);
  p[i] = pi;
  if (JAC) ph[i] = pi * invd[i];
}

// s = r - alpha v; sh = D^-1 s (Jacobi) or s
template <bool JAC>
__global__ void __launch_bounds__(RB)
    kb_upd_s(BDesc B, const BScal *__restrict__ sc, const double *__restrict__ r,
             const double *__restrict__ v, double *__restrict__ s, double *__restrict__ sh,
             const double *__restrict__ invd) {
  const int64_t blk = blockIdx.x;
  const BScal &c = sc[B.rb_cloud[blk]];
  if (c.done) return;
  const int64_t i = B.rb_row0[blk] + threadIdx.x;
  if (i >= B.rb_row1[blk]) return;
  const double si = r[i] - c.alpha * v[i];
  s[i] = si;
  if (JAC) sh[i] = si * invd[i];
}

// x += alpha ph + omega sh; r = s - omega t; row-block partials (rh, r), (r, r)
__global__ void __launch_bounds__(RB)
    kb_upd_xr(BDesc B, const BScal *__restrict__ sc, double *__restrict__ x,
              const double *__restrict__ ph, const double *__restrict__ sh,
              const double *__restrict__ s, const double *__restrict__ t, double *__restrict__ r,
              const double *__restrict__ rh, double *__restrict__ part) {
  const int64_t blk = blockIdx.x;
  const BScal &c = sc[B.rb_cloud[blk]];
  if (c.done) return; // block-uniform: the whole block belongs to this cloud
  const int64_t i = B.rb_row0[blk] + threadIdx.x;
  double val[2] = {0.0, 0.0};
  if (i < B.rb_row1[blk]) {
    x[i] += c.alpha * ph[i] + c.omega * sh[i];
    const double ri = s[i] - c.omega * t[i];
    r[i] = ri;
    val[0] = rh[i] * ri;
    val[1] = ri * ri;
  }
  rb_partials<2>(val, part, B.nrb, blk);
}

// per-cloud fixed-order sum of part[k * stride + a .. a + cnt) for k < NV (valid in thread 0)
template <int NV>
__device__ __forceinline__ void cloud_sum(const double *part, int64_t stride, int64_t a, int64_t cnt,
                                          double (&out)[NV]) {
  __shared__ double sh[NV][FB];
#pragma unroll
  for (int k = 0; k < NV; k++) {
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < cnt; q += FB) s += part[(int64_t)k * stride + a + q];
    sh[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = FB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < NV; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; k++) out[k] = sh[k][0];
}

__global__ void __launch_bounds__(FB) kb_fin_alpha(BDesc B, const double *part, BScal *sc) {
  const int c = blockIdx.x;
  if (sc[c].done) return;
  double out[1];
  cloud_sum<1>(part, B.nsl, B.c_sl0[c], B.c_nsl[c], out);
  if (threadIdx.x == 0) {
    const double al = sc[c].rho / out[0];
    if (out[0] == 0.0 || !isfinite(al))
      sc[c].done = 2;
    else
      sc[c].alpha = al;
  }
}

__global__ void __launch_bounds__(FB) kb_fin_omega(BDesc B, const double *part, BScal *sc) {
  const int c = blockIdx.x;
  if (sc[c].done) return;
  double out[2];
  cloud_sum<2>(part, B.nsl, B.c_sl0[c], B.c_nsl[c], out);
  if (threadIdx.x == 0) sc[c].omega = out[1] > 0.0 ? out[0] / out[1] : 0.0;
}

__global__ void __launch_bounds__(FB) kb_fin_rho(BDesc B, const double *part, BScal *sc) {
  const int c = blockIdx.x;
  if (sc[c].done) return;
  double out[2];
  cloud_sum<2>(part, B.nrb, B.c_rb0[c], B.c_nrb[c], out);
  if (threadIdx.x == 0) {
    BScal &q = sc[c];
    const double rho_new = out[0];
    q.rnorm = sqrt(out[1]);
    q.it += 1;
    if (q.rnorm <= q.tol * q.bnorm)
      q.done = 1;
    else if (rho_new == 0.0 || q.omega == 0.0 || !isfinite(rho_new))
      q.done = 2;
    else if (q.it >= q.maxit)
      q.done = 3;
    else {
      q.beta = (rho_new / q.rho) * (q.alpha / q.omega);
      q.rho = rho_new;
    }
  }
}

// after a (re)start: norms; on a check (first == 0) decide per cloud whether it
// has converged for good (true residual), failed, or iterates again
__global__ void __launch_bounds__(FB) kb_fin_restart(BDesc B, const double *part, BScal *sc, int first) {
  const int c = blockIdx.x;
  if (!first && sc[c].fin) return;
  double out[2];
  cloud_sum<2>(part, B.nsl, B.c_sl0[c], B.c_nsl[c], out);
  if (threadIdx.x == 0) {
    BScal &q = sc[c];
    if (first) q.bnorm = sqrt(out[1]);
    q.rho = out[0];
    q.rnorm = sqrt(out[0]);
    q.rtrue = q.bnorm > 0.0 ? q.rnorm / q.bnorm : 0.0;
    q.beta = 0.0;
    q.alpha = 1.0;
    q.omega = 1.0;
    const bool conv = q.bnorm == 0.0 || q.rnorm <= q.tol * q.bnorm;
    if (first) {
      q.done = conv ? 1 : 0;
      return;
    }
    if (conv) {
      q.fin = 1;
      q.done = 1;
    } else if (q.reason == 3 || q.it >= q.maxit || q.nrest >= 50) {
      q.fin = 2;
      q.done = 3;
    } else {
      q.nrest += 1;
      q.done = 0;
    }
  }
}

template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    k_apply_batch(Op op, const double *__restrict__ x, double *__restrict__ y) {
  for (SlIter it = sl_iter(op); it.s < it.end; it.s += it.step) {
    int32_t i;
    const double v = sell_apply<MODE>(op, x, it.s, i);
    if (i >= 0) y[i] = v;
  }
}

// NGP deposit of the union (the single-cloud formula; without charges every
// particle of cloud c carries 1 / N_c, applied per node as count * (1 / N_c))
__global__ void __launch_bounds__(APC_BLOCK)
    kb_deposit(int64_t n, const int32_t *__restrict__ first, const int32_t *__restrict__ count,
               const int32_t *__restrict__ level, const int32_t *__restrict__ perm,
               const double *__restrict__ q, const double *__restrict__ invN, double L,
               double *__restrict__ rho) {
  const int64_t j = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (j >= n) return;
  double sum;
  if (q) {
    sum = 0.0;
    const int32_t a = first[j], b = a + count[j];
    for (int32_t s = a; s < b; s++) sum += q[perm[s]];
  } else {
    sum = (double)count[j] * invN[j];
  }
  const double hc = L / (double)(1 << level[j]);
  rho[j] = sum / (hc * hc * hc);
}

__global__ void __launch_bounds__(APC_BLOCK)
    kb_bnd_copy(int64_t n, int64_t nb, const int32_t *__restrict__ bowner, double *__restrict__ v) {
  const int64_t b = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (b < nb) v[n + b] = v[bowner[b]];
}

// fresh solver records (a kernel, so that a captured graph holds no host copy)
__global__ void kb_init_sc(BScal *sc, int count, double tol, int maxit) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= count) return;
  BScal q;
  q.rho = q.alpha = q.omega = q.beta = 0.0;
  q.bnorm = q.rnorm = q.rtrue = 0.0;
  q.tol = tol;
  q.it = 0;
  q.maxit = maxit;
  q.done = q.fin = q.nrest = q.reason = q.pad0 = q.pad1 = 0;
  sc[c] = q;
}

// remember why each cloud stopped before the check overwrites done
__global__ void kb_mark_reason(BScal *sc, int count) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < count && !sc[c].fin) sc[c].reason = sc[c].done;
}

} // namespace

// ---------------------------------------------------------------- the batch
struct apc_batch {
  apc_params P;
  int device = 0;
  int count = 0;
  std::vector<int64_t> N, n, nb, nnz, nsl, pbase, ibase, bbase, sbase, rbbase, nrb;
  apc_cloud *u = nullptr;
  // device tables
  int32_t *sl_cloud = nullptr, *rb_cloud = nullptr, *rb_row0 = nullptr, *rb_row1 = nullptr;
  int64_t *c_tab = nullptr; // 4 x count: sl0, nsl, rb0, nrb
  int64_t nrb_all = 0;
  double *invN = nullptr; // n: 1 / N_c of the node's cloud (default charges)
  // workspace
  double *x = nullptr, *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr,
         *t = nullptr, *ph = nullptr, *sh = nullptr, *b = nullptr, *part_sl = nullptr,
         *part_rb = nullptr;
  BScal *sc = nullptr, *sc_host = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t cap = nullptr; // private stream for graph capture
  // launch shape and graphs
  int use_graph = 1, chunk = 8, spmv_div = 1;
  // [density][mode][preconditioner: none, Jacobi, learned] for the current chunk
  hipGraphExec_t gexec[2][3][3] = {};
  hipGraph_t graph[2][3][3] = {};
  int gchunk[2][3][3] = {};
  int gdiv[2][3][3] = {};
  // pipeline graph (apc_batch_pipeline): its own solver records (density, then
  // Poisson), rho_M and the derivative workspace, the iteration budgets and what
  // the graph was recorded with
  BScal *sc_pipe = nullptr, *scp_host = nullptr;
  double *rhoM = nullptr, *Dw = nullptr;
  int budget_d = 0, budget_p = 0;
  hipGraph_t pgraph = nullptr;
  hipGraphExec_t pexec = nullptr;
  struct Key {
    const void *ptr[7];
    double tol_d, tol;
    int maxit, precond, budget_d, budget_p, div;
  } pkey = {};
};

namespace {

BDesc make_desc(const apc_batch *b) {
  BDesc d;
  d.sl_cloud = b->sl_cloud;
  d.rb_cloud = b->rb_cloud;
  d.rb_row0 = b->rb_row0;
  d.rb_row1 = b->rb_row1;
  d.c_sl0 = b->c_tab;
  d.c_nsl = b->c_tab + b->count;
  d.c_rb0 = b->c_tab + 2 * b->count;
  d.c_nrb = b->c_tab + 3 * b->count;
  d.nsl = b->u->nsl;
  d.nrb = b->nrb_all;
  d.count = b->count;
  return d;
}

unsigned batch_spmv_grid(const apc_batch *b) {
  unsigned g = spmv_grid(b->u) / (unsigned)b->spmv_div;
  g &= ~7u; // a multiple of the 8 XCDs
  return g < 8 ? 8 : g;
}

template <typename T>
int dmalloc(T **p, int64_t cnt) {
  HIPCHK(hipMalloc((void **)p, (size_t)(cnt > 0 ? cnt : 1) * sizeof(T)));
  return APC_OK;
}

int map_i32(const int32_t *src, int64_t cnt, int32_t *dst, int32_t thr, int32_t lo, int32_t hi,
            int keep_neg, hipStream_t s) {
  if (cnt <= 0) return APC_OK;
  hipLaunchKernelGGL(k_map_i32, dim3(grid_for(cnt)), dim3(APC_BLOCK), 0, s, src, cnt, dst, thr, lo,
                     hi, keep_neg);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int cpy(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  return APC_OK;
}

// union of the built clouds
int merge(apc_batch *B, std::vector<apc_cloud *> &cl, hipStream_t s) {
  const int C = B->count;
  int64_t Nall = 0, nall = 0, nball = 0, nnzall = 0, nslall = 0, entall = 0, nopen = 0, ntmpl = 0;
  std::vector<int64_t> ebase(C), slbase(C);
  for (int c = 0; c < C; c++) {
    B->pbase[c] = Nall;
    B->ibase[c] = nall;
    B->bbase[c] = nball;
    B->sbase[c] = nslall;
    ebase[c] = nnzall;
    slbase[c] = entall;
    Nall += cl[c]->N;
    nall += cl[c]->n;
    nball += cl[c]->nb;
    nnzall += cl[c]->nnz;
    nslall += cl[c]->nsl;
    entall += cl[c]->sl_entries;
    nopen += cl[c]->n_opened;
    ntmpl += cl[c]->n_template;
  }
  if (nall + nball >= INT32_MAX || nnzall >= INT32_MAX || Nall >= INT32_MAX) return APC_EINVAL;
  apc_cloud *u = new apc_cloud();
  B->u = u;
  u->P = B->P;
  u->device = B->device;
  u->p = cl[0]->p;
  u->N = Nall;
  u->n = nall;
  u->nb = nball;
  u->nnz = nnzall;
  u->n_opened = nopen;
  u->unit = cl[0]->unit;
  memcpy(u->T, cl[0]->T, sizeof(u->T));
  u->n_template = ntmpl;
  for (int k = 0; k < 3; k++) u->tmpl[k] = cl[0]->tmpl[k];
  const int64_t ntot = nall + nball;
  const bool mixed = B->P.precision != APC_FP64;
  APCCHK(dmalloc(&u->perm, Nall));
  APCCHK(dmalloc(&u->sxyz, 3 * Nall));
  APCCHK(dmalloc(&u->pnode, Nall));
  APCCHK(dmalloc(&u->code, nall));
  APCCHK(dmalloc(&u->level, nall));
  APCCHK(dmalloc(&u->first, nall));
  APCCHK(dmalloc(&u->count, nall));
  APCCHK(dmalloc(&u->crd, 3 * ntot + 1)); // + the periodic side slot (0: bounded)
  HIPCHK(hipMemsetAsync(u->crd + 3 * ntot, 0, sizeof(int32_t), s));
  APCCHK(dmalloc(&u->bowner, nball));
  APCCHK(dmalloc(&u->bface, nball));
  APCCHK(dmalloc(&u->st_off, nall + 1));
  APCCHK(dmalloc(&u->st_idx, nnzall));
  APCCHK(dmalloc(&u->rkind, nall));
  APCCHK(dmalloc(&u->diag, nall));
  APCCHK(dmalloc(&u->inv_diag, nall));
  APCCHK(dmalloc(&u->hscale, nall));
  if (mixed)
    APCCHK(dmalloc(&u->w32, nnzall));
  else
    APCCHK(dmalloc(&u->w64, nnzall));
  u->nsl = nslall;
  u->sl_entries = entall;
  APCCHK(dmalloc(&u->sl_rows, nslall * APC_SLICE));
  APCCHK(dmalloc(&u->sl_len, nslall));
  APCCHK(dmalloc(&u->sl_tmpl, nslall));
  APCCHK(dmalloc(&u->sl_off, nslall));
  APCCHK(dmalloc(&u->sl_idx, entall));
  if (mixed)
    APCCHK(dmalloc(&u->sl_w32, entall));
  else
    APCCHK(dmalloc(&u->sl_w64, entall));
  APCCHK(dmalloc(&u->scratch, 1));
  APCCHK(cpy(u->scratch, cl[0]->scratch, sizeof(apc_asm_scratch), s));
  APCCHK(dmalloc(&B->sl_cloud, nslall));
  APCCHK(dmalloc(&B->invN, nall));
  for (int c = 0; c < C; c++) {
    const apc_cloud *k = cl[c];
    const int64_t pb = B->pbase[c], ib = B->ibase[c], bb = B->bbase[c];
    const int64_t kt = k->n + k->nb;
    // a node j of cloud c: interior j < n_c -> ib + j; boundary -> nall + bb + (j - n_c)
    const int32_t lo = (int32_t)ib, hi = (int32_t)(nall + bb - k->n), thr = (int32_t)k->n;
    APCCHK(map_i32(k->perm, k->N, u->perm + pb, INT32_MAX, (int32_t)pb, 0, 0, s));
    for (int d = 0; d < 3; d++) {
      APCCHK(cpy(u->sxyz + d * Nall + pb, k->sxyz + d * k->N, (size_t)k->N * 8, s));
      APCCHK(cpy(u->crd + d * ntot + ib, k->crd + d * kt, (size_t)k->n * 4, s));
      APCCHK(cpy(u->crd + d * ntot + nall + bb, k->crd + d * kt + k->n, (size_t)k->nb * 4, s));
    }
    APCCHK(map_i32(k->pnode, k->N, u->pnode + pb, INT32_MAX, lo, 0, 0, s));
    APCCHK(cpy(u->code + ib, k->code, (size_t)k->n * 8, s));
    APCCHK(cpy(u->level + ib, k->level, (size_t)k->n * 4, s));
    APCCHK(map_i32(k->first, k->n, u->first + ib, INT32_MAX, (int32_t)pb, 0, 0, s));
    APCCHK(cpy(u->count + ib, k->count, (size_t)k->n * 4, s));
    APCCHK(map_i32(k->bowner, k->nb, u->bowner + bb, INT32_MAX, lo, 0, 0, s));
    APCCHK(cpy(u->bface + bb, k->bface, (size_t)k->nb * 4, s));
    APCCHK(map_i32(k->st_off, k->n, u->st_off + ib, INT32_MAX, (int32_t)ebase[c], 0, 0, s));
    APCCHK(map_i32(k->st_idx, k->nnz, u->st_idx + ebase[c], thr, lo, hi, 0, s));
    APCCHK(cpy(u->rkind + ib, k->rkind, (size_t)k->n, s));
    const int64_t sb = B->sbase[c];
    APCCHK(map_i32(k->sl_rows, k->nsl * APC_SLICE, u->sl_rows + sb * APC_SLICE, INT32_MAX, lo, 0, 1, s));
    APCCHK(cpy(u->sl_len + sb, k->sl_len, (size_t)k->nsl * 4, s));
    APCCHK(cpy(u->sl_tmpl + sb, k->sl_tmpl, (size_t)k->nsl * 4, s));
    if (k->nsl > 0) {
      hipLaunchKernelGGL(k_add_i64, dim3(grid_for(k->nsl)), dim3(APC_BLOCK), 0, s, k->sl_off, k->nsl,
                         u->sl_off + sb, slbase[c]);
      hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(k->nsl)), dim3(APC_BLOCK), 0, s,
                         B->sl_cloud + sb, k->nsl, (int32_t)c);
    }
    APCCHK(map_i32(k->sl_idx, k->sl_entries, u->sl_idx + slbase[c], thr, lo, hi, 0, s));
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(k->n)), dim3(APC_BLOCK), 0, s, B->invN + ib, k->n,
                       1.0 / (double)k->N);
    HIPCHK(hipGetLastError());
  }
  const int32_t nnz32 = (int32_t)nnzall;
  HIPCHK(hipMemcpyAsync(u->st_off + nall, &nnz32, 4, hipMemcpyHostToDevice, s));
  if (u->sl_w32) HIPCHK(hipMemsetAsync(u->sl_w32, 0, (size_t)(entall > 0 ? entall : 1) * 4, s));
  if (u->sl_w64) HIPCHK(hipMemsetAsync(u->sl_w64, 0, (size_t)(entall > 0 ? entall : 1) * 8, s));
  APCCHK(apc_pack_sell_idx(u, s)); // the operator kernels' copy of the union's column indices
  // 8 contiguous slice ranges, one per XCD, balanced by slice count
  for (int k = 0; k <= 8; k++) u->sl_cs[k] = (int64_t)k * nslall / 8;
  // row blocks of the vector kernels: each inside one cloud
  std::vector<int32_t> rbc, r0, r1;
  std::vector<int64_t> tab(4 * (size_t)C);
  for (int c = 0; c < C; c++) {
    const int64_t nb_c = (cl[c]->n + RB - 1) / RB;
    B->rbbase[c] = (int64_t)rbc.size();
    B->nrb[c] = nb_c;
    for (int64_t q = 0; q < nb_c; q++) {
      rbc.push_back(c);
      r0.push_back((int32_t)(B->ibase[c] + q * RB));
      r1.push_back((int32_t)std::min(B->ibase[c] + cl[c]->n, B->ibase[c] + (q + 1) * RB));
    }
    tab[c] = B->sbase[c];
    tab[C + c] = cl[c]->nsl;
    tab[2 * C + c] = B->rbbase[c];
    tab[3 * C + c] = nb_c;
  }
  B->nrb_all = (int64_t)rbc.size();
  APCCHK(dmalloc(&B->rb_cloud, B->nrb_all));
  APCCHK(dmalloc(&B->rb_row0, B->nrb_all));
  APCCHK(dmalloc(&B->rb_row1, B->nrb_all));
  APCCHK(dmalloc(&B->c_tab, 4 * (int64_t)C));
  HIPCHK(hipMemcpyAsync(B->rb_cloud, rbc.data(), rbc.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(B->rb_row0, r0.data(), r0.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(B->rb_row1, r1.data(), r1.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(B->c_tab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s)); // the host tables above are freed on return
  return APC_OK;
}

int ensure_bws(apc_batch *B) {
  if (B->x) return APC_OK;
  const int64_t ntot = B->u->n + B->u->nb;
  double **vs[] = {&B->x, &B->r, &B->rh, &B->p, &B->v, &B->s, &B->t, &B->ph, &B->sh, &B->b};
  for (double **q : vs) {
    APCCHK(dmalloc(q, ntot));
    HIPCHK(hipMemset(*q, 0, (size_t)(ntot > 0 ? ntot : 1) * 8)); // boundary tails stay zero
  }
  APCCHK(dmalloc(&B->part_sl, 2 * B->u->nsl));
  APCCHK(dmalloc(&B->part_rb, 2 * B->nrb_all));
  APCCHK(dmalloc(&B->sc, B->count));
  HIPCHK(hipHostMalloc((void **)&B->sc_host, (size_t)B->count * sizeof(BScal), hipHostMallocDefault));
  HIPCHK(hipEventCreate(&B->e0));
  HIPCHK(hipEventCreate(&B->e1));
  HIPCHK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
  return APC_OK;
}

template <int MODE>
void launch_restart(apc_batch *B, const Op &op, const BDesc &D, int first, hipStream_t s) {
  const unsigned g = batch_spmv_grid(B);
  hipLaunchKernelGGL(kb_restart<MODE>, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, D, (const BScal *)B->sc,
                     (const double *)B->b, (const double *)B->x, B->r, B->rh, B->p, B->v, B->part_sl,
                     first);
  hipLaunchKernelGGL(kb_fin_restart, dim3(B->count), dim3(FB), 0, s, D, (const double *)B->part_sl,
                     B->sc, first);
}

// one iteration; PC: 0 no preconditioner, 1 Jacobi (invd), 2 the learned M of the
// union (ph = M p and sh = M s by kb_prec)
template <int MODE, int PC>
void launch_iteration(apc_batch *B, const Op &op, const BDesc &D, const double *invd, hipStream_t s) {
  constexpr bool JAC = PC == 1;
  const unsigned g = batch_spmv_grid(B);
  const unsigned gr = (unsigned)(B->nrb_all > 0 ? B->nrb_all : 1);
  const BScal *sc = B->sc;
  double *ph = PC ? B->ph : B->p;
  double *sh = PC ? B->sh : B->s;
  const MOp M{B->u->m_diag, B->u->m_sell, B->u->m_tmpl, 26};
  hipLaunchKernelGGL(kb_upd_p<JAC>, dim3(gr), dim3(RB), 0, s, D, sc, (const double *)B->r, B->p,
                     (const double *)B->v, ph, invd);
  if (PC == 2)
    hipLaunchKernelGGL(kb_prec, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, M, D, sc,
                       (const double *)B->p, B->ph);
  hipLaunchKernelGGL(kb_spmv_v<MODE>, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, D, sc, (const double *)ph,
                     B->v, (const double *)B->rh, B->part_sl);
  hipLaunchKernelGGL(kb_fin_alpha, dim3(B->count), dim3(FB), 0, s, D, (const double *)B->part_sl,
                     B->sc);
  hipLaunchKernelGGL(kb_upd_s<JAC>, dim3(gr), dim3(RB), 0, s, D, sc, (const double *)B->r,
                     (const double *)B->v, B->s, sh, invd);
  if (PC == 2)
    hipLaunchKernelGGL(kb_prec, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, M, D, sc,
                       (const double *)B->s, B->sh);
  hipLaunchKernelGGL(kb_spmv_t<MODE>, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, D, sc, (const double *)sh,
                     (const double *)B->s, B->t, B->part_sl);
  hipLaunchKernelGGL(kb_fin_omega, dim3(B->count), dim3(FB), 0, s, D, (const double *)B->part_sl,
                     B->sc);
  hipLaunchKernelGGL(kb_upd_xr, dim3(gr), dim3(RB), 0, s, D, sc, B->x, (const double *)ph,
                     (const double *)sh, (const double *)B->s, (const double *)B->t, B->r,
                     (const double *)B->rh, B->part_rb);
  hipLaunchKernelGGL(kb_fin_rho, dim3(B->count), dim3(FB), 0, s, D, (const double *)B->part_rb,
                     B->sc);
}

template <int MODE, int PC>
int run_chunk(apc_batch *B, const Op &op, const BDesc &D, const double *invd, bool density,
              hipStream_t s) {
  if (!B->use_graph) {
    for (int k = 0; k < B->chunk; k++) launch_iteration<MODE, PC>(B, op, D, invd, s);
    HIPCHK(hipGetLastError());
    return APC_OK;
  }
  const int di = density ? 1 : 0, ji = PC;
  hipGraphExec_t &ex = B->gexec[di][MODE][ji];
  if (ex && (B->gchunk[di][MODE][ji] != B->chunk || B->gdiv[di][MODE][ji] != B->spmv_div)) {
    HIPCHK(hipGraphExecDestroy(ex));
    HIPCHK(hipGraphDestroy(B->graph[di][MODE][ji]));
    ex = nullptr;
  }
  if (!ex) {
    // record C iterations once on the private stream; kernel arguments (device
    // pointers of the batch's own workspace) stay valid for the batch's life
    HIPCHK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < B->chunk; k++) launch_iteration<MODE, PC>(B, op, D, invd, B->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap, &g);
    HIPCHK(e);
    B->graph[di][MODE][ji] = g;
    HIPCHK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    B->gchunk[di][MODE][ji] = B->chunk;
    B->gdiv[di][MODE][ji] = B->spmv_div;
  }
  HIPCHK(hipGraphLaunch(ex, s));
  return APC_OK;
}

int read_sc(apc_batch *B, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(B->sc_host, B->sc, (size_t)B->count * sizeof(BScal), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return APC_OK;
}

template <int MODE, int PC>
int bicgstab(apc_batch *B, bool density, double tol, int maxit, apc_stats *st, hipStream_t s) {
  const Op op = make_op(B->u, density);
  const BDesc D = make_desc(B);
  std::vector<BScal> init((size_t)B->count);
  memset(init.data(), 0, init.size() * sizeof(BScal));
  for (auto &q : init) {
    q.tol = tol;
    q.maxit = maxit;
  }
  HIPCHK(hipMemcpyAsync(B->sc, init.data(), init.size() * sizeof(BScal), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(B->x, 0, (size_t)B->u->n * sizeof(double), s));
  launch_restart<MODE>(B, op, D, 1, s);
  HIPCHK(hipGetLastError());
  const double *invd = B->u->inv_diag;
  for (int guard = 0;; guard++) {
    APCCHK(read_sc(B, s));
    bool all_fin = true, all_stopped = true;
    for (int c = 0; c < B->count; c++) {
      all_fin = all_fin && B->sc_host[c].fin != 0;
      all_stopped = all_stopped && (B->sc_host[c].fin != 0 || B->sc_host[c].done != 0);
    }
    if (all_fin) break;
    if (all_stopped) {
      hipLaunchKernelGGL(kb_mark_reason, dim3((B->count + 255) / 256), dim3(256), 0, s, B->sc, B->count);
      launch_restart<MODE>(B, op, D, 0, s);
      HIPCHK(hipGetLastError());
      continue;
    }
    APCCHK((run_chunk<MODE, PC>(B, op, D, invd, density, s)));
    if (guard > 4 * (maxit + 64)) return APC_EHIP; // cannot happen: every chunk advances it
  }
  int status = APC_OK;
  for (int c = 0; c < B->count; c++) {
    const BScal &q = B->sc_host[c];
    const int sc_status = q.fin == 1 ? APC_OK : APC_ENOCONV;
    if (sc_status != APC_OK) status = APC_ENOCONV;
    if (st) {
      st[c].iters = q.it;
      st[c].restarts = q.nrest;
      st[c].sweeps = 1 + q.nrest;
      st[c].status = sc_status;
      st[c].rel_resid = q.bnorm > 0.0 ? q.rnorm / q.bnorm : 0.0;
      st[c].rel_resid_true = q.rtrue;
      st[c].n_fp64_rows = 0;
      st[c].precond_used = PC == 2 ? APC_PRECOND_LEARNED : (PC == 1 ? APC_PRECOND_JACOBI : APC_PRECOND_NONE);
    }
  }
  return status;
}

int run_bsolve(apc_batch *B, bool density, double tol, int maxit, int prec, apc_stats *st,
               hipStream_t s) {
  auto run = [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
    return prec == APC_PRECOND_LEARNED  ? bicgstab<MODE, 2>(B, density, tol, maxit, st, s)
           : prec == APC_PRECOND_JACOBI ? bicgstab<MODE, 1>(B, density, tol, maxit, st, s)
                                        : bicgstab<MODE, 0>(B, density, tol, maxit, st, s);
  };
  switch (B->P.precision) {
  case APC_MIXED_F32ACC: return run(std::integral_constant<int, V32A32>{});
  case APC_MIXED: return run(std::integral_constant<int, V32A64>{});
  default: return run(std::integral_constant<int, V64>{});
  }
}

// k_rhs / k_write_out of the single-cloud path, restated for the union (same formulas)
template <int MODE>
__global__ void __launch_bounds__(APC_BLOCK)
    kb_rhs(Op op, int64_t n, const double *__restrict__ src, double srcscale,
           const double *__restrict__ bval, double *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  if (bval) {
    for (int32_t e = op.off[i]; e < op.off[i + 1]; e++) {
      const int32_t j = op.idx[e];
      if (j >= n) acc += ((MODE == V64) ? op.w64[e] : (double)op.w32[e]) * bval[j - n];
    }
  }
  b[i] = srcscale * src[i] - (op.hs ? op.hs[i] * acc : acc);
}

__global__ void __launch_bounds__(APC_BLOCK)
    kb_write_out(int64_t n, int64_t nb, const double *__restrict__ x, const double *__restrict__ bval,
                 double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n)
    out[i] = x[i];
  else if (i < n + nb)
    out[i] = bval ? bval[i - n] : 0.0;
}

int rhs(apc_batch *B, bool density, const double *src, double scale, const double *bval,
        hipStream_t s) {
  const Op op = make_op(B->u, density);
  if (B->P.precision == APC_FP64)
    hipLaunchKernelGGL(kb_rhs<V64>, dim3(grid_for(B->u->n)), dim3(APC_BLOCK), 0, s, op, B->u->n, src,
                       scale, bval, B->b);
  else
    hipLaunchKernelGGL(kb_rhs<V32A64>, dim3(grid_for(B->u->n)), dim3(APC_BLOCK), 0, s, op, B->u->n,
                       src, scale, bval, B->b);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

void set_stats_ms(apc_batch *B, apc_stats *st, float ms) {
  if (!st) return;
  for (int c = 0; c < B->count; c++) st[c].ms = ms;
}

} // namespace

// ---------------------------------------------------------------- entry points (impl)
int apc_build_batch_impl(const apc_params *P, int count, const double *const *xyz,
                         const int64_t *N, hipStream_t s, apc_batch **out) {
  apc_batch *B = new apc_batch();
  B->P = *P;
  B->count = count;
  HIPCHK(hipGetDevice(&B->device));
  for (auto *v : {&B->N, &B->n, &B->nb, &B->nnz, &B->nsl, &B->pbase, &B->ibase, &B->bbase, &B->sbase,
                  &B->rbbase, &B->nrb})
    v->assign((size_t)count, 0);
  std::vector<apc_cloud *> cl((size_t)count, nullptr);
  int rc = APC_OK;
  for (int c = 0; c < count && rc == APC_OK; c++) {
    rc = apc_build_impl(P, xyz[c], N[c], s, &cl[c]);
    if (rc == APC_OK) {
      B->N[c] = cl[c]->N;
      B->n[c] = cl[c]->n;
      B->nb[c] = cl[c]->nb;
      B->nnz[c] = cl[c]->nnz;
      B->nsl[c] = cl[c]->nsl;
    }
  }
  if (rc == APC_OK) rc = merge(B, cl, s);
  for (apc_cloud *c : cl)
    if (c) apc_free_cloud(c);
  if (rc != APC_OK) {
    apc_destroy_batch_impl(B);
    return rc;
  }
  *out = B;
  return APC_OK;
}

void apc_destroy_batch_impl(apc_batch *B) {
  if (!B) return;
  if (B->pexec) (void)hipGraphExecDestroy(B->pexec);
  if (B->pgraph) (void)hipGraphDestroy(B->pgraph);
  for (void *q : {(void *)B->sc_pipe, (void *)B->rhoM, (void *)B->Dw})
    if (q) (void)hipFree(q);
  if (B->scp_host) (void)hipHostFree(B->scp_host);
  for (int a = 0; a < 2; a++)
    for (int m = 0; m < 3; m++)
      for (int j = 0; j < 3; j++) {
        if (B->gexec[a][m][j]) (void)hipGraphExecDestroy(B->gexec[a][m][j]);
        if (B->graph[a][m][j]) (void)hipGraphDestroy(B->graph[a][m][j]);
      }
  void *ptrs[] = {B->sl_cloud, B->rb_cloud, B->rb_row0, B->rb_row1, B->c_tab, B->invN, B->x, B->r,
                  B->rh, B->p, B->v, B->s, B->t, B->ph, B->sh, B->b, B->part_sl, B->part_rb, B->sc};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  if (B->sc_host) (void)hipHostFree(B->sc_host);
  if (B->e0) (void)hipEventDestroy(B->e0);
  if (B->e1) (void)hipEventDestroy(B->e1);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  if (B->u) apc_free_cloud(B->u);
  delete B;
}

apc_cloud *apc_batch_union(apc_batch *B) { return B->u; }

// The learned preconditioner of every cloud, installed on the union: a row's
// features and M row are local to its stencil, and the uniform 2-ring rows of one
// level (identical in every cloud of the batch) share one row of M.
int apc_batch_set_learned_impl(apc_batch *B, const float *params, const double *Z, int K,
                               hipStream_t s) {
  if (!B->u->assembled || B->P.order != 2) return APC_EINVAL;
  return apc_set_learned_impl(B->u, params, Z, K, s);
}

int apc_batch_info_impl(const apc_batch *B, apc_batch_info_t *info, int64_t *cN, int64_t *cn,
                        int64_t *cnb) {
  if (info) {
    info->count = B->count;
    info->N = B->u->N;
    info->n = B->u->n;
    info->nb = B->u->nb;
    info->nnz = B->u->nnz;
    info->nsl = B->u->nsl;
    info->use_graph = B->use_graph;
    info->chunk = B->chunk;
    info->spmv_blocks = (int)batch_spmv_grid(B);
    info->pad = 0;
  }
  for (int c = 0; c < B->count; c++) {
    if (cN) cN[c] = B->N[c];
    if (cn) cn[c] = B->n[c];
    if (cnb) cnb[c] = B->nb[c];
  }
  return APC_OK;
}

int apc_batch_configure_impl(apc_batch *B, int use_graph, int chunk, int spmv_div) {
  if (use_graph >= 0) B->use_graph = use_graph ? 1 : 0;
  if (chunk > 0) B->chunk = chunk;
  if (spmv_div > 0) B->spmv_div = spmv_div;
  return APC_OK;
}

int apc_batch_deposit_impl(apc_batch *B, const double *q, double *rho_M, double *rho_t, double tol,
                           int maxit, apc_stats *st, hipStream_t s) {
  if (!B->u->assembled) return APC_EINVAL;
  APCCHK(ensure_bws(B));
  HIPCHK(hipEventRecord(B->e0, s));
  apc_cloud *u = B->u;
  hipLaunchKernelGGL(kb_deposit, dim3(grid_for(u->n)), dim3(APC_BLOCK), 0, s, u->n, u->first, u->count,
                     u->level, u->perm, q, (const double *)B->invN, u->P.L, rho_M);
  if (u->nb > 0)
    hipLaunchKernelGGL(kb_bnd_copy, dim3(grid_for(u->nb)), dim3(APC_BLOCK), 0, s, u->n, u->nb,
                       u->bowner, rho_M);
  HIPCHK(hipGetLastError());
  APCCHK(rhs(B, true, rho_M, 1.0, rho_M + B->u->n, s));
  int rc = run_bsolve(B, true, tol, maxit, APC_PRECOND_NONE, st, s);
  if (rc < 0) return rc;
  // boundary nodes keep their owner's rho_M
  hipLaunchKernelGGL(kb_write_out, dim3(grid_for(B->u->n + B->u->nb)), dim3(APC_BLOCK), 0, s,
                     B->u->n, B->u->nb, (const double *)B->x, (const double *)(rho_M + B->u->n),
                     rho_t);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(B->e1, s));
  HIPCHK(hipEventSynchronize(B->e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, B->e0, B->e1));
  set_stats_ms(B, st, ms);
  return rc;
}

int apc_batch_solve_impl(apc_batch *B, const double *rho_t, const double *g, double *phi,
                         double tol, int maxit, int precond, apc_stats *st, hipStream_t s) {
  if (!B->u->assembled) return APC_EINVAL;
  if (precond != APC_PRECOND_NONE && precond != APC_PRECOND_JACOBI &&
      !(precond == APC_PRECOND_LEARNED && B->u->learned))
    return APC_EINVAL;
  APCCHK(ensure_bws(B));
  HIPCHK(hipEventRecord(B->e0, s));
  APCCHK(rhs(B, false, rho_t, B->P.poisson_c, g, s));
  int rc = run_bsolve(B, false, tol, maxit, precond, st, s);
  if (rc < 0) return rc;
  hipLaunchKernelGGL(kb_write_out, dim3(grid_for(B->u->n + B->u->nb)), dim3(APC_BLOCK), 0, s,
                     B->u->n, B->u->nb, (const double *)B->x, g, phi);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(B->e1, s));
  HIPCHK(hipEventSynchronize(B->e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, B->e0, B->e1));
  set_stats_ms(B, st, ms);
  return rc;
}

// Autotuner: SpMV grid divisor by timing the batched operator apply, then the
// graph chunk length by timing whole Jacobi solves of the batch's own deposit.
int apc_batch_tune_impl(apc_batch *B, double tol, int *out_div, int *out_chunk, hipStream_t s) {
  if (!B->u->assembled) return APC_EINVAL;
  APCCHK(ensure_bws(B));
  const int64_t ntot = B->u->n + B->u->nb;
  double *f = nullptr, *y = nullptr, *rhoM = nullptr, *rhot = nullptr, *phi = nullptr;
  HIPCHK(apc_malloc_async((void **)&f, (size_t)ntot * 8, s));
  HIPCHK(apc_malloc_async((void **)&y, (size_t)ntot * 8, s));
  HIPCHK(apc_malloc_async((void **)&rhoM, (size_t)ntot * 8, s));
  HIPCHK(apc_malloc_async((void **)&rhot, (size_t)ntot * 8, s));
  HIPCHK(apc_malloc_async((void **)&phi, (size_t)ntot * 8, s));
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(ntot)), dim3(APC_BLOCK), 0, s, f, ntot, 1.0);
  const Op op = make_op(B->u, false);
  float best = 1e30f;
  int best_div = 1;
  for (int div : {1, 2, 4, 8}) {
    B->spmv_div = div;
    const unsigned g = batch_spmv_grid(B);
    for (int rep = 0; rep < 3; rep++)
      if (B->P.precision == APC_FP64)
        hipLaunchKernelGGL(k_apply_batch<V64>, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, (const double *)f, y);
      else
        hipLaunchKernelGGL(k_apply_batch<V32A64>, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, (const double *)f, y);
    HIPCHK(hipEventRecord(B->e0, s));
    for (int rep = 0; rep < 20; rep++)
      if (B->P.precision == APC_FP64)
        hipLaunchKernelGGL(k_apply_batch<V64>, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, (const double *)f, y);
      else
        hipLaunchKernelGGL(k_apply_batch<V32A64>, dim3(g), dim3(APC_BLOCK), op_lds(op), s, op, (const double *)f, y);
    HIPCHK(hipEventRecord(B->e1, s));
    HIPCHK(hipEventSynchronize(B->e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, B->e0, B->e1));
    if (ms < best) {
      best = ms;
      best_div = div;
    }
  }
  B->spmv_div = best_div;
  std::vector<apc_stats> st((size_t)B->count);
  int rc = apc_batch_deposit_impl(B, nullptr, rhoM, rhot, 1e-10, 4000, st.data(), s);
  int best_chunk = B->chunk;
  if (rc >= 0) {
    best = 1e30f;
    for (int ch : {4, 8, 16, 32}) {
      B->chunk = ch;
      for (int rep = 0; rep < 2; rep++) { // the first run records the graph
        rc = apc_batch_solve_impl(B, rhot, nullptr, phi, tol, 20000, APC_PRECOND_JACOBI, st.data(), s);
        if (rc < 0) break;
      }
      if (rc < 0) break;
      if (st[0].ms < best) {
        best = (float)st[0].ms;
        best_chunk = ch;
      }
    }
  }
  B->chunk = best_chunk;
  HIPCHK(apc_free_async(f, s));
  HIPCHK(apc_free_async(y, s));
  HIPCHK(apc_free_async(rhoM, s));
  HIPCHK(apc_free_async(rhot, s));
  HIPCHK(apc_free_async(phi, s));
  HIPCHK(hipStreamSynchronize(s));
  if (out_div) *out_div = B->spmv_div;
  if (out_chunk) *out_chunk = B->chunk;
  return rc < 0 ? rc : APC_OK;
}

// ---------------------------------------------------------------- pipeline graph
namespace {

// one batched BiCGSTAB recorded into the capture stream: fresh records, x = 0, the
// start, `budget` iterations (clouds that stop skip their rows), then one
// true-residual check; sc: the solve's own records
template <int MODE, int PC>
void record_solve(apc_batch *B, bool density, BScal *sc, double tol, int maxit, int budget,
                  hipStream_t cs) {
  const Op op = make_op(B->u, density);
  const BDesc D = make_desc(B);
  BScal *save = B->sc;
  B->sc = sc;
  hipLaunchKernelGGL(kb_init_sc, dim3((B->count + 63) / 64), dim3(64), 0, cs, sc, B->count, tol,
                     maxit);
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(B->u->n)), dim3(APC_BLOCK), 0, cs, B->x, B->u->n, 0.0);
  launch_restart<MODE>(B, op, D, 1, cs);
  for (int k = 0; k < budget; k++) launch_iteration<MODE, PC>(B, op, D, B->u->inv_diag, cs);
  hipLaunchKernelGGL(kb_mark_reason, dim3((B->count + 255) / 256), dim3(256), 0, cs, sc, B->count);
  launch_restart<MODE>(B, op, D, 0, cs);
  B->sc = save;
}

template <int MODE>
void record_solve_any(apc_batch *B, bool density, BScal *sc, double tol, int maxit, int budget,
                      int pc, hipStream_t cs) {
  if (pc == APC_PRECOND_LEARNED)
    record_solve<MODE, 2>(B, density, sc, tol, maxit, budget, cs);
  else if (pc == APC_PRECOND_JACOBI)
    record_solve<MODE, 1>(B, density, sc, tol, maxit, budget, cs);
  else
    record_solve<MODE, 0>(B, density, sc, tol, maxit, budget, cs);
}

// assembly, deposit and density solve, Poisson solve and interpolation, recorded
// on the batch's capture stream
int record_pipeline(apc_batch *B, const double *q, const double *g, double tol_d, double tol,
                    int maxit, int precond, double *rho_t, double *phi, double *phi_p,
                    double *grad_p, hipStream_t cs) {
  apc_cloud *u = B->u;
  const bool keep = u->learned; // same rows every assembly: an installed M stays valid
  APCCHK(apc_assemble_impl(u, cs));
  u->learned = keep;
  hipLaunchKernelGGL(kb_deposit, dim3(grid_for(u->n)), dim3(APC_BLOCK), 0, cs, u->n, u->first,
                     u->count, u->level, u->perm, q, (const double *)B->invN, u->P.L, B->rhoM);
  if (u->nb > 0)
    hipLaunchKernelGGL(kb_bnd_copy, dim3(grid_for(u->nb)), dim3(APC_BLOCK), 0, cs, u->n, u->nb,
                       u->bowner, B->rhoM);
  APCCHK(rhs(B, true, B->rhoM, 1.0, B->rhoM + u->n, cs));
  auto solve = [&](bool density, BScal *sc, double t, int budget, int j) {
    switch (B->P.precision) {
    case APC_MIXED_F32ACC: record_solve_any<V32A32>(B, density, sc, t, maxit, budget, j, cs); break;
    case APC_MIXED: record_solve_any<V32A64>(B, density, sc, t, maxit, budget, j, cs); break;
    default: record_solve_any<V64>(B, density, sc, t, maxit, budget, j, cs);
    }
  };
  solve(true, B->sc_pipe, tol_d, B->budget_d, APC_PRECOND_NONE);
  hipLaunchKernelGGL(kb_write_out, dim3(grid_for(u->n + u->nb)), dim3(APC_BLOCK), 0, cs, u->n, u->nb,
                     (const double *)B->x, (const double *)(B->rhoM + u->n), rho_t);
  APCCHK(rhs(B, false, rho_t, B->P.poisson_c, g, cs));
  solve(false, B->sc_pipe + B->count, tol, B->budget_p, precond);
  hipLaunchKernelGGL(kb_write_out, dim3(grid_for(u->n + u->nb)), dim3(APC_BLOCK), 0, cs, u->n, u->nb,
                     (const double *)B->x, g, phi);
  APCCHK(apc_interp_with(u, phi, phi_p, grad_p, B->Dw, cs));
  HIPCHK(hipGetLastError());
  return APC_OK;
}

void pipe_stats(const BScal &q, int precond, float ms, apc_stats *st) {
  st->iters = q.it;
  st->restarts = q.nrest;
  st->sweeps = 1 + q.nrest;
  st->status = q.fin == 1 ? APC_OK : APC_ENOCONV;
  st->rel_resid = q.bnorm > 0.0 ? q.rnorm / q.bnorm : 0.0;
  st->rel_resid_true = q.rtrue;
  st->n_fp64_rows = 0;
  st->precond_used = precond;
  st->ms = ms;
}

} // namespace

int apc_batch_pipeline_impl(apc_batch *B, const double *q, const double *g, double tol_d,
                            double tol, int maxit, int precond, double *rho_t, double *phi,
                            double *phi_p, double *grad_p, apc_stats *st_d, apc_stats *st,
                            int *graph_used, hipStream_t s) {
  if (precond != APC_PRECOND_NONE && precond != APC_PRECOND_JACOBI &&
      !(precond == APC_PRECOND_LEARNED && B->u->learned))
    return APC_EINVAL;
  if (B->P.order != 2) return APC_EINVAL;
  APCCHK(ensure_bws(B));
  apc_cloud *u = B->u;
  const int64_t ntot = u->n + u->nb;
  if (!B->sc_pipe) {
    APCCHK(dmalloc(&B->sc_pipe, 2 * B->count));
    APCCHK(dmalloc(&B->rhoM, ntot));
    APCCHK(dmalloc(&B->Dw, u->n * 9)); // k = 2: 9 derivatives a node
    HIPCHK(hipHostMalloc((void **)&B->scp_host, (size_t)2 * B->count * sizeof(BScal),
                         hipHostMallocDefault));
  }
  if (graph_used) *graph_used = 0;
  std::vector<apc_stats> sd((size_t)B->count), sp((size_t)B->count);
  // the separate entry points: the first call (it sets the budgets) and any call
  // whose graph left a cloud unfinished
  auto separate = [&]() -> int {
    // the union's rows come out of its assembly the same every time, so an
    // installed M stays valid across it
    const bool keep = u->learned;
    APCCHK(apc_assemble_impl(u, s));
    u->learned = keep;
    int rc = apc_batch_deposit_impl(B, q, B->rhoM, rho_t, tol_d, maxit, sd.data(), s);
    if (rc < 0) return rc;
    const int rc2 = apc_batch_solve_impl(B, rho_t, g, phi, tol, maxit, precond, sp.data(), s);
    if (rc2 < 0) return rc2;
    APCCHK(apc_interp_with(u, phi, phi_p, grad_p, B->Dw, s));
    HIPCHK(hipStreamSynchronize(s));
    int md = 0, mp = 0;
    for (int c = 0; c < B->count; c++) {
      md = std::max(md, sd[c].iters);
      mp = std::max(mp, sp[c].iters);
    }
    // budgets: the largest count with a quarter (at least 4) to spare, raised
    // when a graph fell short
    B->budget_d = std::max(B->budget_d, md + std::max(4, md / 4));
    B->budget_p = std::max(B->budget_p, mp + std::max(4, mp / 4));
    if (st_d) memcpy(st_d, sd.data(), sd.size() * sizeof(apc_stats));
    if (st) memcpy(st, sp.data(), sp.size() * sizeof(apc_stats));
    return rc != APC_OK ? rc : rc2;
  };
  if (B->budget_d == 0 || B->budget_p == 0) return separate();
  apc_batch::Key key;
  memset(&key, 0, sizeof(key)); // compared bytewise, padding included
  const void *ptrs[7] = {q, g, rho_t, phi, phi_p, grad_p, nullptr};
  for (int k = 0; k < 7; k++) key.ptr[k] = ptrs[k];
  key.tol_d = tol_d;
  key.tol = tol;
  key.maxit = maxit;
  key.precond = precond;
  key.budget_d = B->budget_d;
  key.budget_p = B->budget_p;
  key.div = B->spmv_div;
  if (B->pexec && memcmp(&key, &B->pkey, sizeof(key)) != 0) {
    HIPCHK(hipGraphExecDestroy(B->pexec));
    HIPCHK(hipGraphDestroy(B->pgraph));
    B->pexec = nullptr;
    B->pgraph = nullptr;
  }
  if (!B->pexec) {
    HIPCHK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    const int rc = record_pipeline(B, q, g, tol_d, tol, maxit, precond, rho_t, phi, phi_p, grad_p,
                                   B->cap);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap, &gr);
    if (rc < 0) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    HIPCHK(e);
    B->pgraph = gr;
    HIPCHK(hipGraphInstantiate(&B->pexec, gr, nullptr, nullptr, 0));
    B->pkey = key;
  }
  HIPCHK(hipEventRecord(B->e0, s));
  HIPCHK(hipGraphLaunch(B->pexec, s));
  HIPCHK(hipEventRecord(B->e1, s));
  HIPCHK(hipMemcpyAsync(B->scp_host, B->sc_pipe, (size_t)2 * B->count * sizeof(BScal),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, B->e0, B->e1));
  bool all = true;
  for (int c = 0; c < 2 * B->count; c++) all = all && B->scp_host[c].fin != 0;
  if (!all) {
    // a cloud needed more iterations or a restart: enlarge the budgets, record
    // again on the next call, and run this one through the separate entry points
    B->budget_d += std::max(4, B->budget_d / 2);
    B->budget_p += std::max(4, B->budget_p / 2);
    return separate();
  }
  int status = APC_OK;
  for (int c = 0; c < B->count; c++) {
    if (B->scp_host[c].fin != 1 || B->scp_host[B->count + c].fin != 1) status = APC_ENOCONV;
    if (st_d) pipe_stats(B->scp_host[c], APC_PRECOND_NONE, ms, &st_d[c]);
    if (st) pipe_stats(B->scp_host[B->count + c], precond, ms, &st[c]);
  }
  if (graph_used) *graph_used = 1;
  return status;
}

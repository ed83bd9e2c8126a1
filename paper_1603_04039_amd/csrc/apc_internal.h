// Internal declarations of the gfx950 AP-Cloud library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/apcloud.h"

#define APC_BLOCK 256
#define APC_MAXM 64      // hard stencil cap: one wavefront
// density-row stability bound: a row of B is kept when sum_j |b_ij| <= APC_THETA_B b_ii
#define APC_THETA_B 0.5
#define APC_RING_CAP 16384 // per-node candidate capacity of the ring search
#define APC_TAU_RANK 1e-6 // min|R_ii| / max|R_ii| below this => rank deficient
#define APC_TAU_DOM 10.0  // default of apc_params.tau_dom: order-4 rows need sum |w_j| <= tau |diag|
// window of the length sort of general rows in the sliced layout (SELL-C-sigma;
// a multiple of the 64-row slice, 64 = no sort)
#ifndef APC_SELL_SIGMA
#define APC_SELL_SIGMA 256
#endif
// most distinct neighbour columns of a slice staged in LDS (per wavefront; a
// slice with more gathers directly).  1008 doubles a wave keep a 256-thread
// block at 32,256 bytes, five blocks per 160 KB compute unit.
#ifndef APC_UCAP_MAX
#define APC_UCAP_MAX 1008
#endif
// default tile cap (stage_cap = 0): 768 doubles a wave keep a 256-thread block at
// 24,576 bytes, six blocks per compute unit (the register limit of the operator
// kernels); on the 1e8-particle k = 4 cloud the apply ran 352-360 us against
// 372-375 us at 1008 (same build, interleaved runs), 366 at 640, 425 at 544
#define APC_UCAP_DEFAULT 768
#define APC_SLICE 64      // rows per sliced-ELL slice: one wavefront
// box of a boxed slice: cell (x, y, z) of the 8 x 8 x 8 box at x + 8 y + 64 z;
// APC_BOX_N positions.  (A z stride of 68, 4 mod 32, halves the LDS bank conflicts
// of the neighbour reads but ran slower: 443 against 423 us per apply on the 1e8
// k = 4 cloud, and strides of 66 and 68 staged in one batch still ran 1.5% slower.)
#define APC_BOX_SZ 64
#define APC_BOX_N (7 + 8 * 7 + APC_BOX_SZ * 7 + 1)
#define APC_TAU_FP32 0.1  // mixed modes: FP32 fit kept when min|R_ii| / max|R_ii| >= this
#define APC_MAX_LEVELS 24 // > max_depth (<= 20): per-level tables

void apc_set_hip_error(hipError_t e, const char *what, const char *file, int line);

#define HIPCHK(x)                                          \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) {                                \
      apc_set_hip_error(e_, #x, __FILE__, __LINE__);       \
      return e_ == hipErrorOutOfMemory ? APC_ENOMEM : APC_EHIP; \
    }                                                      \
  } while (0)

#define APCCHK(x)        \
  do {                   \
    int r_ = (x);        \
    if (r_ < 0) return r_; \
  } while (0)

static inline unsigned grid_for(int64_t n, int per_block = APC_BLOCK) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------- Morton codes
// 3 bits per level, x highest in each triple; bits spread with magic masks.
__host__ __device__ inline uint64_t apc_spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
__host__ __device__ inline uint32_t apc_compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return (uint32_t)v;
}
// Node coordinates are held as crd[3 (n + nb) + 1]: x, y and z of every node, then
// one int32 S, the domain side in integer units on a periodic domain (0 on the
// Dirichlet box).  Offsets between nodes are minimum images in [-S/2, S/2) then.
__host__ __device__ inline int32_t apc_doff(int32_t a, int32_t b, int32_t S) {
  int32_t d = a - b;
  if (S) {
    if (d >= (S >> 1)) d -= S;
    else if (d < -(S >> 1)) d += S;
  }
  return d;
}

// ---- charge-assignment kernels of eq. density_apcloud (APC_KERNEL_*), per axis
__host__ __device__ inline double apc_kernel_reach(int kernel) {
  return kernel == APC_KERNEL_CIC ? 1.0 : (kernel == APC_KERNEL_TSC ? 1.5 : 0.5);
}
// phi(u) of CIC (tent) and TSC (quadratic B-spline)
__host__ __device__ inline double apc_kernel_phi(int kernel, double u) {
  const double a = fabs(u);
  if (kernel == APC_KERNEL_CIC) return a < 1.0 ? 1.0 - a : 0.0;
  if (a <= 0.5) return 0.75 - u * u;
  if (a < 1.5) {
    const double t = 1.5 - a;
    return 0.5 * t * t;
  }
  return 0.0;
}
// u^k as a product of k factors
__host__ __device__ inline double apc_powi(double u, int k) {
  double r = 1.0;
  for (int i = 0; i < k; i++) r *= u;
  return r;
}
// int_lo^hi u^k phi(u) du, the integral of u^k (c0 + c1 u + c2 u^2) term by term
__host__ __device__ inline double apc_piece_int(int k, double c0, double c1, double c2, double lo,
                                                double hi) {
  auto F = [&](double u) {
    return c0 * apc_powi(u, k + 1) / (k + 1) + c1 * apc_powi(u, k + 2) / (k + 2) +
           c2 * apc_powi(u, k + 3) / (k + 3);
  };
  return F(hi) - F(lo);
}
// 1-D moment int u^k phi(u) du over [lo, hi] intersected with the kernel's support
// (lo, hi may be infinite).  Over the whole support odd moments vanish (phi is
// even).  NGP: phi = 1 on [-1/2, 1/2].
__host__ __device__ inline double apc_kernel_moment(int kernel, int k, double lo, double hi) {
  const double r = apc_kernel_reach(kernel);
  if ((k & 1) && lo <= -r && hi >= r) return 0.0;
  double m = 0.0;
  auto piece = [&](double a, double b, double c0, double c1, double c2) {
    const double l = fmax(a, lo), h = fmin(b, hi);
    if (h > l) m += apc_piece_int(k, c0, c1, c2, l, h);
  };
  if (kernel == APC_KERNEL_NGP) {
    piece(-0.5, 0.5, 1.0, 0.0, 0.0);
  } else if (kernel == APC_KERNEL_CIC) {
    piece(-1.0, 0.0, 1.0, 1.0, 0.0);
    piece(0.0, 1.0, 1.0, -1.0, 0.0);
  } else { // (3/2 -+ u)^2 / 2 = 9/8 -+ 3/2 u + u^2 / 2 outside, 3/4 - u^2 inside
    piece(-1.5, -0.5, 1.125, 1.5, 0.5);
    piece(-0.5, 0.5, 0.75, 0.0, -1.0);
    piece(0.5, 1.5, 1.125, -1.5, 0.5);
  }
  return m;
}
// Range [tlo, thi] of the kernel argument u = (x - y) / h_c inside Omega along
// each axis for the node at integer coordinates c (units L / 2^(D+1)), cell edge E
// in those units, domain side S2 = 2^(D+1) units; S2 = 0: no walls (periodic).
__host__ __device__ inline void apc_node_trunc(int32_t c0, int32_t c1, int32_t c2, double E,
                                               double S2, double tlo[3], double thi[3]) {
  const int32_t c[3] = {c0, c1, c2};
  for (int d = 0; d < 3; d++) {
    tlo[d] = S2 > 0.0 ? -(double)c[d] / E : -INFINITY;
    thi[d] = S2 > 0.0 ? (S2 - (double)c[d]) / E : INFINITY;
  }
}
__host__ __device__ inline bool apc_truncated(int kernel, const double tlo[3], const double thi[3]) {
  const double r = apc_kernel_reach(kernel);
  return kernel != APC_KERNEL_NGP &&
         (tlo[0] > -r || tlo[1] > -r || tlo[2] > -r || thi[0] < r || thi[1] < r || thi[2] < r);
}
// a_0: the kernel's mass inside Omega
__host__ __device__ inline double apc_kernel_a0(int kernel, const double tlo[3], const double thi[3]) {
  double a0 = 1.0;
  for (int d = 0; d < 3; d++) a0 *= apc_kernel_moment(kernel, 0, tlo[d], thi[d]);
  return a0;
}
// Density-row coefficient of the fitted unknown hp^|alpha| d^alpha f: (a_alpha / a_0)
// / hp^|alpha|, a_alpha = prod_d hc^a_d mu_a_d / a_d! (the Taylor terms carry
// 1/alpha!).  NGP: mu_e = (1/2)^e / (e + 1) for even e, 0 for odd.
__host__ __device__ inline double apc_dens_coef(int kernel, int ax, int ay, int az, double hc,
                                                double hp, const double tlo[3],
                                                const double thi[3], double a0) {
  const int e[3] = {ax, ay, az};
  double mom = 1.0;
  if (kernel == APC_KERNEL_NGP) {
    if ((ax | ay | az) & 1) return 0.0;
    for (int d = 0; d < 3; d++) {
      double pw = 1.0, f = 1.0;
      for (int q = 0; q < e[d]; q++) pw *= hc / 2.0;
      for (int q = 2; q <= e[d]; q++) f *= q;
      mom *= pw / (double)(e[d] + 1) / f;
    }
  } else {
    for (int d = 0; d < 3; d++) {
      double f = 1.0;
      for (int q = 2; q <= e[d]; q++) f *= q;
      mom *= apc_powi(hc, e[d]) * apc_kernel_moment(kernel, e[d], tlo[d], thi[d]) / f;
    }
    mom /= a0;
  }
  return mom / apc_powi(hp, ax + ay + az);
}

__host__ __device__ inline uint64_t apc_morton(uint32_t x, uint32_t y, uint32_t z) {
  return (apc_spread3(x) << 2) | (apc_spread3(y) << 1) | apc_spread3(z);
}

// first index in [lo, hi) with a[i] >= v
__device__ inline int64_t apc_lower_bound(const uint64_t *a, int64_t lo, int64_t hi, uint64_t v) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
// last index in [0, n) with a[i] <= v (a[0] <= v assumed)
__device__ inline int64_t apc_last_le(const uint64_t *a, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo - 1;
}

// ---------------------------------------------------------------- cloud handle
struct apc_solver_ws;

// small device block used by the assembly: canonical stencil, its shell
// constants, error flag and the count of rows refitted in FP64
struct apc_asm_scratch {
  int32_t crd[3 * 25 + 1]; // canonical 2-ring, then S = 0
  double tc[3];
  int err;
  unsigned fb_count; // k = 4 assembly: nodes handed from the normal equations to the QR
  unsigned long long nfp64;
  double pmean; // periodic solve: the volume-weighted mean being removed
};

struct apc_cloud {
  apc_params P;
  int device = 0;
  int diag_flags = 0; // apc_set_diagnostics: APC_DIAG_KERNEL_TIMES | APC_DIAG_FP64_RESIDUAL
  bool w64_mixed = false; // k = 4 mixed modes: the last assembly also wrote FP64 rows to w64ref
  double *w64ref = nullptr; // nnz: those FP64 rows (allocated by apc_set_diagnostics)
  int p = 9;
  int64_t N = 0, n = 0, nb = 0, nnz = 0, n_opened = 0;
  double unit = 0.0; // L / 2^(max_depth+1)
  double T[24];
  // particles (sorted by key)
  int32_t *perm = nullptr;  // N: sorted position -> original index
  double *sxyz = nullptr;   // 3 x N sorted positions
  int32_t *pnode = nullptr; // N: sorted position -> leaf
  // leaves
  uint64_t *code = nullptr; // n
  int32_t *level = nullptr, *first = nullptr, *count = nullptr;
  int32_t *crd = nullptr; // 3 x (n+nb) SoA integer coordinates
  int32_t *bowner = nullptr, *bface = nullptr;
  int32_t *st_off = nullptr, *st_idx = nullptr; // stencil CSR
  int8_t *rorder = nullptr; // n: GFD order of each row (k, or 2 for a k = 4 fallback row)
  // operator
  bool assembled = false;
  double *w64 = nullptr; // nnz (APC_FP64)
  float *w32 = nullptr;  // nnz (APC_MIXED)
  double *diag = nullptr, *inv_diag = nullptr; // n
  double *dwx = nullptr;    // nnz (k = 2, CIC / TSC): explicit density rows (hscale < 0)
  double *hscale = nullptr;                    // n: h_c^2 / 24 (density operator, k = 2;
                                               // 0 for an identity density row)
  int32_t *fb_list = nullptr;                  // n (k = 4): nodes the assembly refits by QR
  int8_t *dorder = nullptr;                    // n: order of each density row: the row's
                                               // fit order, 2 (order-4 row replaced by the
                                               // order-2 row of the same stencil) or 0
                                               // (identity row)
  // k = 4: density operator rows (B has its own weights; row sums are 1)
  double *bw64 = nullptr, *sl_bw64 = nullptr;
  float *bw32 = nullptr, *sl_bw32 = nullptr;
  int64_t n_fp64_rows = 0;
  apc_asm_scratch *scratch = nullptr;
  // learned preconditioner M: diagonal per row, off-diagonal weights in the
  // operator's sliced layout (general slices), and per-level rows of the uniform
  // 2-ring rows (APC_MAX_LEVELS x 25: diagonal, then the 24 stencil entries)
  float *m_diag = nullptr, *m_sell = nullptr, *m_tmpl = nullptr;
  bool learned = false;
  // rows whose stencil is the uniform 24-node 2-ring of their own level share one
  // set of weights c_shell / h_c^2 (shells r^2 = s^2, 2 s^2, 4 s^2): rkind[i] is
  // the level of such a row, -1 for a general row
  int8_t *rkind = nullptr;
  double tmpl[3] = {0.0, 0.0, 0.0};
  int64_t n_template = 0;
  // k = 4: rows whose stencil is the uniform 56-node lattice stencil of their own
  // level (6, 12, 8, 6 and 24 nodes at r^2 = 1 .. 5 cells, in that order in the
  // (r^2, index) order of the stencil) share one Laplacian row c_shell / h_c^2 and
  // one density row (scale-free).  rkind4[i] is the level of such a row, -1
  // otherwise; tmpl4 holds the 5 Laplacian shell weights at h_c = 1, then the 5
  // density shell weights; dorder4 the order of that density row.  Their CSR rows
  // are written from the constants; the SpMV reads no weights for them.  gen4
  // lists the other rows (the ones the assembly fits).
  int8_t *rkind4 = nullptr;
  double tmpl4[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double tmpl4_sum = 0.0; // sum of the 56 Laplacian weights at h_c = 1
  int dorder4 = 0;
  int64_t n_uniform4 = 0;
  int32_t *gen4 = nullptr;
  int64_t n_gen4 = 0;
  double *cder4 = nullptr; // 125 x 34: derivative operator of the canonical stencil by
                           // lattice offset (25 (q_x+2) + 5 (q_y+2) + q_z+2), 0 off-stencil
  // build: decision of the order-4 rank and stability test on the canonical 56-node
  // stencil, taken by every uniform candidate (1 accept, 0 reject; -1 none: every
  // candidate takes the QR; -2 not yet computed)
  int uni4_rank = -2;
  // sliced-ELL copy of the operator used by the SpMV (see sell.hip)
  int64_t nsl = 0, sl_entries = 0;
  int64_t sl_cs[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}; // slice range of each XCD chunk
  int32_t *sl_rows = nullptr;  // nsl * 64 row ids (-1 = padding lane)
  int32_t *sl_len = nullptr;   // entries per row in the slice
  int32_t *sl_tmpl = nullptr;  // 1: uniform 2-ring slice (k = 2), 2: uniform 56-node slice
                               // (k = 4; the SpMV reads no weights), 3 | (box << 2): boxed
                               // slice (below), 0: general; 32-bit: scalar loads
  int64_t *sl_off = nullptr;   // first entry of the slice (a multiple of 4 x 64: slices
                               // hold a multiple of 4 entries per row)
  int32_t *sl_idx = nullptr;   // column indices, entry-major within a slice
  // compact copy of sl_idx read by the operator kernels: low 16 bits two entries per
  // word, bits 16..23 four entries per word, bits 24..31 likewise (only when the
  // cloud has 2^24 nodes or more); entry k of lane r of the slice at entry offset o
  // is in word o/2 + 64 (k/2) + r (low) and o/4 + 64 (k/4) + r (high, top)
  uint32_t *sl_lo2 = nullptr, *sl_hi4 = nullptr, *sl_top4 = nullptr;
  // neighbour staging: slice s with sl_un[s] > 0 first gathers its sl_un[s]
  // distinct columns, listed ascending in sl_uq[sl_off[s] ..], into an LDS tile of
  // ucap doubles per wavefront; entry k of lane r then reads tile slot
  // (sl_lx2[o/2 + 64 (k/2) + r] >> 16 (k%2)) & 0xffff.  sl_un[s] = 0: the slice
  // gathers through sl_lo2 / sl_hi4 / sl_top4.  ucap = 0: no slice is staged.
  int32_t *sl_un = nullptr;
  int32_t *sl_uq = nullptr;
  uint32_t *sl_lx2 = nullptr;
  int ucap = 0;
  // boxed slices (k = 4): a slice whose 64 rows are one Morton-aligned 4 x 4 x 4
  // block of uniform 56-node rows of one level (lane = Morton index within the
  // block) has sl_tmpl = 3 | (box << 2); box b is sl_box[APC_BOX_N b ..]: the node
  // of every cell of the 8 x 8 x 8 box around the block that a stencil of the block
  // reaches, at (x + 2) + 8 (y + 2) + APC_BOX_SZ (z + 2) for the cell's local
  // coordinates (-1 elsewhere).  The operator kernels find every neighbour's box position from
  // the lane and the offset and read no per-entry index.
  int64_t n_boxes = 0;
  int32_t *sl_box = nullptr;
  double *sl_w64 = nullptr;    // weights (general slices), APC_FP64
  float *sl_w32 = nullptr;     // weights (general slices), mixed modes
  apc_solver_ws *ws = nullptr;
};

// ---------------------------------------------------------------- host utilities
// text returned by apc_last_error for the calling thread
void apc_set_error_msg(const char *msg);
int apc_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s);  // exclusive
int apc_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s);  // exclusive
int apc_sum_i32(const int32_t *in, int64_t n, int64_t *host_out, hipStream_t s);
int apc_radix_sort(uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s);
// Stream-ordered temporaries through a cache: a block freed on stream s goes to
// a free list of (device, s) and serves the next allocation of a fitting size on
// that same stream (stream order makes the reuse safe) without a HIP call; the
// HIP stream-ordered allocator is called only on a miss, and blocks beyond a
// 16 GiB cache go back to it.  Same signatures as hipMallocAsync / hipFreeAsync.
hipError_t apc_malloc_async(void **p, size_t bytes, hipStream_t s);
hipError_t apc_free_async(void *p, hipStream_t s);
// Arrays a cloud keeps for its lifetime: a device-wide cache of freed blocks of
// the same size classes; apc_dev_free requires that no queued work uses the block.
hipError_t apc_dev_alloc(void **p, size_t bytes);
hipError_t apc_dev_free(void *p);

int apc_build_impl(const apc_params *p, const double *xyz, int64_t N, hipStream_t s,
                   apc_cloud **out);
int apc_assemble_impl(apc_cloud *c, hipStream_t s);
int apc_prepare_operator(apc_cloud *c, hipStream_t s);
int apc_learn_data_impl(apc_cloud *c, const double *Z, int K, float *feat, float *quad,
                        hipStream_t s);
int apc_mlp_loss_grad_impl(const float *P, const float *feat, const float *quad,
                           const int32_t *rows, int B, float *loss, float *grad, hipStream_t s);
int apc_mlp_adam_impl(float *P, float *m, float *v, const float *g, int step, float lr,
                      hipStream_t s);
int apc_mlp_infer_impl(apc_cloud *c, const float *P, const float *feat, int bf16, float *out,
                       hipStream_t s);
int apc_set_learned_impl(apc_cloud *c, const float *P, const double *Z, int K, hipStream_t s);
int apc_apply_precond_impl(apc_cloud *c, int precond, const double *in, double *out,
                           hipStream_t s);
int apc_node_derivs_impl(apc_cloud *c, const double *f, double *D, hipStream_t s);
// k = 4 (gfd4.hip)
int apc_rank_check4(apc_cloud *c, int pk, const int32_t *pending, int64_t np,
                    const int32_t *cand, int32_t *m, hipStream_t s);
int apc_assemble4(apc_cloud *c, hipStream_t s);
// uniform 56-node rows: canonical constants, rkind4 and the list of the other rows
int apc_prepare_uniform4(apc_cloud *c, hipStream_t s);
int apc_node_derivs4(apc_cloud *c, const double *f, double *D, hipStream_t s);
int apc_interp4(apc_cloud *c, const double *phi, double *phi_p, double *grad_p, hipStream_t s);
int apc_interp4_with(apc_cloud *c, const double *phi, double *phi_p, double *grad_p, double *D,
                     hipStream_t s);
int apc_interp_with(apc_cloud *c, const double *phi, double *phi_p, double *grad_p, double *D,
                    hipStream_t s);
int apc_resid64_rows(apc_cloud *c, const double *b, const double *x, double *r, hipStream_t s);
int apc_interp_noalloc_impl(apc_cloud *c, const double *phi, double *phi_p, double *grad_p,
                            hipStream_t s);
int apc_interp_impl(apc_cloud *c, const double *phi, double *phi_p, double *grad_p,
                    hipStream_t s);
int apc_deposit_impl(apc_cloud *c, const double *q, double *rho_M, hipStream_t s);
int apc_density_solve_impl(apc_cloud *c, const double *rho_M, double *rho_t, double tol,
                           int maxit, apc_stats *st, hipStream_t s);
int apc_solve_impl(apc_cloud *c, const double *rho_t, const double *g, double *phi,
                   double tol, int maxit, int precond, apc_stats *st, hipStream_t s);
int apc_apply_impl(apc_cloud *c, const double *f, double *out, hipStream_t s);
// time loop (push.hip)
int apc_push_impl(const apc_params *p, int64_t N, double *xyz, double *vel, const double *grad,
                  double kick, double dt, hipStream_t s);
int apc_step_impl(const apc_params *p, double *xyz, double *vel, const double *q, int64_t N,
                  double kick, double dt, double tol_density, double tol, int maxit, int precond,
                  double *phi_p, double *grad_p, apc_step_stats *st, hipStream_t s);

// batches (batch.hip)
int apc_build_batch_impl(const apc_params *P, int count, const double *const *xyz,
                         const int64_t *N, hipStream_t s, apc_batch **out);
void apc_destroy_batch_impl(apc_batch *B);
apc_cloud *apc_batch_union(apc_batch *B);
int apc_batch_set_learned_impl(apc_batch *B, const float *params, const double *Z, int K,
                               hipStream_t s);
int apc_batch_info_impl(const apc_batch *B, apc_batch_info_t *info, int64_t *cN, int64_t *cn,
                        int64_t *cnb);
int apc_batch_configure_impl(apc_batch *B, int use_graph, int chunk, int spmv_div);
int apc_batch_deposit_impl(apc_batch *B, const double *q, double *rho_M, double *rho_t, double tol,
                           int maxit, apc_stats *st, hipStream_t s);
int apc_batch_solve_impl(apc_batch *B, const double *rho_t, const double *g, double *phi,
                         double tol, int maxit, int precond, apc_stats *st, hipStream_t s);
int apc_batch_tune_impl(apc_batch *B, double tol, int *out_div, int *out_chunk, hipStream_t s);
int apc_batch_pipeline_impl(apc_batch *B, const double *q, const double *g, double tol_d,
                            double tol, int maxit, int precond, double *rho_t, double *phi,
                            double *phi_p, double *grad_p, apc_stats *st_d, apc_stats *st,
                            int *graph_used, hipStream_t s);
void apc_free_solver(apc_cloud *c);
int apc_build_sell(apc_cloud *c, hipStream_t s);
// (re)build sl_lo2 / sl_hi4 / sl_top4 and the neighbour staging from sl_idx
// (allocates them)
int apc_pack_sell_idx(apc_cloud *c, hipStream_t s);
void apc_free_sell(apc_cloud *c);
// stencil rank test of pending nodes (k = 2); clears m[y] of rejected nodes
int apc_rank_check(apc_cloud *c, int order, const int32_t *pending, int64_t np,
                   const int32_t *cand, int32_t *m, hipStream_t s);

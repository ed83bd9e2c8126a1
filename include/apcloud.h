/*
 * apcloud.h -- C ABI of the MI355X (gfx950) AP-Cloud field-solve library.
 *
 * AP-Cloud (Wang, Samulyak, Jiao, Yu, "AP-Cloud: Adaptive Particle-in-Cloud
 * Method for Optimal Solutions to Vlasov-Poisson Equation") replaces the PIC
 * mesh by an adaptive octree node cloud.  Given N charged particles it computes,
 * in three steps (Sec. 3.2):
 *   1. the node density rho~ from the WLS charge assignment B rho~ = rho_M
 *      (eq. density_apcloud, eq. density_linear_system), NGP kernel (Sec. 5.1);
 *   2. phi at the nodes from the GFD discretisation of Delta phi = c rho
 *      (eq. Poisson, Sec. 3.1), solved by a Krylov method;
 *   3. phi and E = grad phi at the particles by Taylor expansion from GFD
 *      derivatives (Sec. 3.2 step 3).
 * The node cloud itself comes from the error-balance criterion and 2:1 face
 * balance on a Morton-sorted octree (Sec. 4).
 *
 * Conventions
 *  - Every array argument is a DEVICE pointer unless the name ends in _host.
 *    The caller owns every buffer it passes; the library never frees them.
 *  - Every call is ordered on the given HIP stream.  Calls that report solver
 *    statistics (apc_deposit, apc_density_solve, apc_solve) synchronise that
 *    stream before returning; the others return without synchronising.
 *  - A cloud handle owns its internal device workspaces; apc_destroy frees
 *    them.  A handle is bound to the device that was current at build time and
 *    must not be used from two host threads at once.
 *  - Particle positions are a 3 x N structure of arrays of float64
 *    (x[0..N), y[0..N), z[0..N)).  Node numbering: interior nodes (octree
 *    leaves) 0..n-1 in ascending Morton order of their minimum corner, then
 *    boundary nodes n..n+nb-1 by (owner node, face), faces -x,+x,-y,+y,-z,+z.
 *  - Return value: APC_OK (0) on success, a negative APC_E* code on failure
 *    (outputs then undefined), APC_ENOCONV (+1) when a solve stopped at maxit
 *    (outputs hold the last iterate; stats say how far it got).
 */
#ifndef APCLOUD_H
#define APCLOUD_H

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define APC_OK 0
#define APC_EINVAL (-1)   /* bad parameter, NaN input, wrong call order */
#define APC_ENOMEM (-2)   /* device allocation failed */
#define APC_EHIP (-3)     /* a HIP runtime call failed (apc_last_error has text) */
#define APC_EDOMAIN (-4)  /* a particle lies outside the domain */
#define APC_ESTENCIL (-5) /* a node found no acceptable stencil up to ring_max */
#define APC_ENOCONV 1     /* solver hit maxit (warning) */

#define APC_FP64 0  /* FP64 stencil fit, FP64 matrix values, FP64 Krylov */
#define APC_MIXED 1 /* FP32 matrix values, FP64 SpMV accumulation, FP64 dots + refinement */
#define APC_MIXED_F32ACC 2 /* as APC_MIXED with FP32 SpMV arithmetic in the iteration */

#define APC_PRECOND_NONE 0
#define APC_PRECOND_JACOBI 1
#define APC_PRECOND_LEARNED 2 /* needs apc_set_learned_precond; Jacobi is the fallback */

/* Learned preconditioner network: a 3-layer MLP APC_MLP_IN -> 64 -> 64 -> APC_MLP_OUT
   (ReLU), parameters as one float array [W1 (IN x 64, row-major), b1, W2 (64 x 64),
   b2, W3 (64 x OUT), b3], APC_MLP_NPARAM floats. */
#define APC_MLP_IN 48
#define APC_MLP_HID 64
#define APC_MLP_OUT 41 /* row i of M: the diagonal and up to 40 stencil entries */
#define APC_MLP_NPARAM (48 * 64 + 64 + 64 * 64 + 64 + 64 * 41 + 41)
#define APC_LEARN_QUAD 903 /* per row: 861 (packed lower 41x41 Q), 41 (b), 1 (c) */

typedef struct apc_cloud apc_cloud;

typedef struct {
  double lo[3];     /* domain Omega = [lo, lo + L]^3 */
  double L;         /* domain edge, > 0 */
  int order;        /* GFD order k (Sec. 3.1): 2 or 4 */
  double c;         /* error-balance constant (Sec. 4.3, eq. errorbalance_implementation), > 0 */
  int max_depth;    /* deepest octree level, 1..20 */
  int ring_min;     /* first k-ring searched for a stencil (Sec. 4.3); 2 for k = 2 */
  int ring_max;     /* last ring searched; the paper finds 5 always enough */
  int m_cap;        /* stencil size cap (<= 64); 40 for k = 2 */
  double poisson_c; /* c in Delta phi = c rho (eq. Poisson); 1 */
  int precision;    /* APC_FP64, APC_MIXED or APC_MIXED_F32ACC, fixed at build time */
  int stage_cap;    /* operator kernels: a 64-row slice with at most this many distinct
                       neighbour columns gathers them once into LDS (performance only,
                       same results bit for bit); 0 = default (768), at most 1008,
                       -1 = never */
  int criterion_pow; /* exponent e of the criterion thresholds T_l = (c 2^l / L)^e:
                        0 = 2k - 2 (eq. errorbalance_implementation, the default);
                        4 with k = 2 is the balance of the supraconvergent
                        second-order error bound (Sec. 3.3; its optimal h, Sec. 3.4),
                        h = c N'^(-1/4);
                        1..16 accepted */
  int ring_lds;      /* order-2 stencil search (performance only, same stencils bit
                        for bit): 0 = default, rings of up to 63 candidates with one
                        wavefront per node and up to 255 with one block per node,
                        both in LDS, the rest per thread; 1 = the wavefront tier
                        only; -1 = every ring per thread */
  int ring_first_cap; /* per-thread stencil search (performance only, same stencils
                        bit for bit): ring capacity of its first pass; a node whose
                        R-ring holds more candidates is searched again with the full
                        capacity (16384).  0 = default, 2 (2R+1)^3 for ring R;
                        1..16384 accepted */
  double tau_dom;     /* stability bound of an order-4 Laplacian row (k = 4; the paper
                        states none, a reading): the row is accepted when its diagonal
                        d is negative and sum_j |w_j| <= tau_dom |d|, else the node
                        searches a larger ring and finally takes an order-2 row;
                        0 = default 10 */
  int periodic;       /* 1: Omega is periodic in x, y and z (Sec. 4.3 speaks of "a
                        non-periodic region"; this is the other case): face neighbours
                        wrap around, there are no boundary nodes (nb = 0, g ignored),
                        stencil offsets are minimum images, levels 0 and 1 are always
                        opened (max_depth >= 2), and apc_solve solves
                        Delta phi = c (rho~ - mean rho~) with the equation of node 0
                        replaced by phi_0 = 0, then shifts phi to mean 0 (means
                        weighted by cell volume); the FP64 residual diagnostic of
                        the mixed modes is not computed (-1).  0 (default): the
                        Dirichlet box */
  int kernel;         /* charge-assignment kernel Phi of eq. density_apcloud, per axis of
                        u = (x - y) / h_c: APC_KERNEL_NGP (0, default: the node's own
                        cell), APC_KERNEL_CIC (1: the tent 1 - |u|, |u| <= 1) or
                        APC_KERNEL_TSC (2: the quadratic B-spline, |u| <= 3/2).  CIC and
                        TSC gather every particle within reach of the node, neighbour
                        cells included; their moments a(y) integrate over Omega, so a
                        node whose kernel reaches past a wall has a_0 < 1 (the kernel's
                        mass inside Omega) and odd and mixed moments: its density row
                        and rho_M are divided by a_0.  Batches take NGP only. */
  int mask_level;     /* irregular domain (0, default: the whole box): Omega is the box
                        minus the cells of the uniform level-mask_level grid (1 ..
                        min(6, max_depth)) that `mask` excludes, its walls the box faces
                        and the faces between included and excluded cells (a reading of
                        the method's independence of the domain's shape, Sec. 5.1).
                        Cells of a level below mask_level are opened unless wholly
                        excluded, excluded cells never; leaves in excluded cells are not
                        nodes; every node face on a wall carries a boundary node at its
                        centre (Dirichlet data g as on the box).  A particle in an
                        excluded cell is outside Omega (APC_EDOMAIN).  Not with periodic,
                        a CIC / TSC kernel, batches or apc_step (whose push knows the
                        box's walls only): APC_EINVAL. */
  const uint8_t *mask; /* host array of (2^mask_level)^3 bytes, index x + s (y + s z),
                          s = 2^mask_level; nonzero excludes the cell.  Read by
                          apc_build_cloud only (not kept by the cloud). */
} apc_params;

#define APC_KERNEL_NGP 0
#define APC_KERNEL_CIC 1
#define APC_KERNEL_TSC 2

typedef struct {
  int iters;             /* Krylov iterations (summed over refinement sweeps) */
  int restarts;          /* BiCGSTAB restarts (breakdown or residual disagreement) */
  int sweeps;            /* iterative-refinement sweeps (APC_MIXED), else 1 */
  int status;            /* APC_OK or APC_ENOCONV */
  double rel_resid;      /* recursive ||r|| / ||b|| at exit */
  double rel_resid_true; /* ||b - A x|| / ||b|| recomputed in FP64 at exit */
  int64_t n_fp64_rows;   /* k = 2, APC_MIXED: stencils refitted in FP64 (R-diagonal test);
                            k = 4: nodes whose normal-equation fit was handed to the
                            Householder QR */
  double ms;             /* device time of the call, milliseconds */
  int precond_used;      /* preconditioner of the final iteration (Jacobi after a fallback) */
  int pad;
  double rel_resid_fp64ref; /* apc_solve: ||b - A64 x|| / ||b|| with A64 the FP64 fit of the
                               same stencils.  FP64 mode: rel_resid_true.  Mixed modes: computed
                               at exit when APC_DIAG_FP64_RESIDUAL is set, else -1 */
  double spmv_ms;        /* APC_DIAG_KERNEL_TIMES: summed device time of the operator
                            SpMV launches of the iterations (HIP events on the call's
                            stream), else 0 */
  int64_t spmv_launches; /* number of SpMV launches summed in spmv_ms */
} apc_stats;

#define APC_DIAG_KERNEL_TIMES 1  /* time every operator SpMV of the solves with HIP events */
#define APC_DIAG_FP64_RESIDUAL 2 /* mixed modes: FP64 reference residual at the end of apc_solve */

/* Fill *p with the defaults above for order k (domain [0,1]^3, c, max_depth left
   as given by the caller afterwards). */
void apc_default_params(apc_params *p, int order);

/* Build the node cloud (Sec. 4): Morton keys and a stable radix sort of the
   particles, the error-balance criterion opening cells with N' >= T_l where
   T_l = t^(2k-2) (or t^criterion_pow), t = (c 2^l) / L evaluated in FP64 by
   repeated multiplication,
   level-by-level 2:1 face balance to the unique minimal balanced refinement,
   boundary face nodes, and per-node GFD stencils from the R-ring (Sec. 3.1,
   4.3).  Stencil rule: the ring's nodes sorted by (squared distance, index); the
   two nearest of every closed octant (a zero offset counts on both sides), for
   k = 4 then per axis the nearest with a new offset until the axis has 5
   distinct offsets, then the nearest remaining, up to m_cap nodes.  Accepted when
   every closed octant holds a chosen node, m >= p + 1, the weighted V0 has
   min|R_ii| / max|R_ii| >= 1e-6, and (k = 4) the Laplacian row has a negative
   diagonal d with sum |w_j| <= tau_dom |d|; otherwise R grows from ring_min to
   ring_max.  A k = 4 node with no acceptable stencil takes an order-2 row (ring
   2, m_cap 40); past ring_max at order 2 the build fails (APC_ESTENCIL).
   xyz: 3 x N float64, read during the call and copied (sorted) into the
   handle.  Errors: APC_EINVAL (parameters, NaN), APC_EDOMAIN (a particle outside
   Omega), APC_ESTENCIL, APC_ENOMEM, APC_EHIP.  Synchronises the stream. */
int apc_build_cloud(const apc_params *p, const double *xyz, int64_t N, hipStream_t stream,
                    apc_cloud **out);

/* Sizes: interior nodes n, boundary nodes nb, stencil entries nnz (off-diagonal),
   cells opened by the criterion or the balance (n = 1 + 7 n_opened). */
int apc_cloud_info(const apc_cloud *c, int64_t *n, int64_t *nb, int64_t *nnz,
                   int64_t *n_opened);

/* Host copies of the cloud structure (any pointer may be NULL): perm_host[N]
   (sorted position -> original particle index), code_host[n] (Morton code of the
   minimum corner at max_depth), level_host[n], first_host[n], count_host[n]
   (sorted particle range of each leaf), bowner_host[nb], bface_host[nb],
   st_off_host[n+1], st_idx_host[nnz] (stencil CSR), ixyz_host[3*(n+nb)]
   (integer node coordinates in units of L 2^-(max_depth+1), SoA).
   Synchronises the handle's build stream. */
int apc_get_nodes(const apc_cloud *c, int32_t *perm_host, uint64_t *code_host,
                  int32_t *level_host, int32_t *first_host, int32_t *count_host,
                  int32_t *bowner_host, int32_t *bface_host, int32_t *st_off_host,
                  int32_t *st_idx_host, int32_t *ixyz_host);

/* Assemble the GFD Poisson operator (Sec. 3.1, 3.2 step 2): per node the weighted
   least-squares fit of the scaled Taylor Vandermonde V0 over its stencil
   (h = max |delta|, Gaussian weight with c = 4), giving the off-diagonal weights
   w_ij of Delta at node i; the diagonal is -sum_j w_ij.  k = 2: normal equations
   and Cholesky per node (FP32 with an FP64 refit of ill-conditioned rows in the
   mixed modes, FP64 otherwise).  k = 4: Householder QR in FP64 in every mode,
   also giving the rows of the density operator B.  Must follow apc_build_cloud.
   Does not synchronise. */
int apc_assemble_gfd(apc_cloud *c, hipStream_t stream);

/* Host copy of the assembled operator: w_host[nnz] aligned with the stencil
   CSR, diag_host[n].  In APC_MIXED the FP32 values are widened exactly. */
int apc_get_operator(const apc_cloud *c, double *w_host, double *diag_host);

/* Layout of the assembled operator as the solver streams it: n_uniform rows have
   the uniform stencil of their own level -- k = 2: the 24-node 2-ring, k = 4: the
   56 nodes at lattice offsets with r^2 = 1 .. 5 cells -- (their weights are the
   shared shell constants and are not read; at k = 4 the CSR rows returned by
   apc_get_operator and apc_get_density_operator hold those constants),
   nnz_general entries belong to the other rows, sell_entries is the padded entry
   count of the sliced layout,
   m_entries the off-diagonal entries the learned M stores for the other rows
   (min(m, APC_MLP_OUT - 1) per row).  staged[4], if not NULL, receives the
   neighbour staging of the operator kernels: the number of 64-row slices whose
   distinct neighbour columns are gathered once into LDS, the sum of those
   distinct-column counts, the entries those slices read (row length x 64 each),
   and the LDS tile in doubles per wavefront (0: no slice staged).  Any output may
   be NULL; m_entries and staged copy device arrays to the host and synchronise
   the device. */
int apc_operator_info(const apc_cloud *c, int64_t *n_uniform, int64_t *nnz_general,
                      int64_t *sell_entries, int64_t *m_entries, int64_t *staged);

/* Boxed slices of the operator layout (k = 4; 0 at k = 2): 64-row slices that are
   one Morton-aligned 4 x 4 x 4 block of same-level rows with the uniform 56-node
   stencil; the operator kernels address their neighbours through the block's
   8 x 8 x 8 box of node ids (512 int32 per slice) and read no per-entry column
   index.  *n_boxed receives their count.  APC_EINVAL on NULL arguments. */
int apc_operator_boxes(const apc_cloud *c, int64_t *n_boxed);

/* WLS charge assignment (Sec. 3.2 step 1): rho_M_j = (1/h_j^3) sum_{i in cell j} q_i
   (NGP kernel: the node's own octree cell, edge h_j), then B rho~ = rho_M with
   B = I + sum_alpha a_alpha D^alpha over the even derivatives up to order k (eq.
   density_linear_system; a_alpha the kernel moments of the cell): for k = 2
   B = I + diag(h_j^2 / 24) L, for k = 4 B has rows of its own from the same
   fit.  Boundary nodes carry their owner's rho_M.  q: N charges in the
   caller's particle order, or NULL for 1/N each (total charge 1, Sec. 2).
   rho_M (may be NULL) and rho_t: n+nb.  Requires apc_assemble_gfd.  BiCGSTAB to
   relative residual tol (maxit iterations), no preconditioner.  Synchronises
   the stream. */
int apc_deposit(apc_cloud *c, const double *q, double *rho_M, double *rho_t, double tol,
                int maxit, apc_stats *st, hipStream_t stream);

/* The density solve of apc_deposit on a caller-supplied rho_M (n+nb). */
int apc_density_solve(apc_cloud *c, const double *rho_M, double *rho_t, double tol, int maxit,
                      apc_stats *st, hipStream_t stream);

/* GFD Poisson solve (Sec. 3.2 step 2): L phi = poisson_c rho~ at interior nodes,
   phi = g at boundary nodes (Dirichlet; g: nb values or NULL for 0).  rho_t: n
   (or n+nb, tail ignored); phi: n+nb out.  BiCGSTAB with optional right Jacobi
   preconditioning to recursive relative residual tol, confirmed by the true
   FP64 residual.  precond APC_PRECOND_LEARNED uses the installed learned M and
   falls back to Jacobi when that solve does not reach tol.  APC_MIXED: FP32
   weights inside FP64 iterative refinement (the
   true residual, with the FP32 weights widened exactly, restarts the iteration
   until it meets tol).
   Requires apc_assemble_gfd.  Synchronises the stream. */
int apc_solve(apc_cloud *c, const double *rho_t, const double *g, double *phi, double tol,
              int maxit, int precond, apc_stats *st, hipStream_t stream);

/* Interpolation (Sec. 3.2 step 3): GFD derivatives of phi at every node, then
   for each particle the k-th order Taylor polynomial of its leaf's node
   evaluated at the particle: phi_p[N], grad_p[3 x N] (= grad phi, the paper's E),
   both in the caller's original particle order.  phi: n+nb.  Does not
   synchronise. */
int apc_interpolate_force(apc_cloud *c, const double *phi, double *phi_p, double *grad_p,
                          hipStream_t stream);

/* apc_interpolate_force without allocation, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc).  Same arguments, kernels and results (bit for bit) as
   apc_interpolate_force; its n x p derivative buffer (p = 9 for k = 2, 34 for
   k = 4) lives in a fixed device array of APC_NOALLOC_BYTES that each GPU holds
   until the process ends, so the call makes no hipMalloc or hipFree.  Clouds with
   n p 8 > APC_NOALLOC_BYTES are rejected with APC_EINVAL (apc_last_error says
   so): k = 2 clouds up to 466,033 nodes, k = 4 up to 123,361.  Every call on a
   GPU shares that GPU's array: calls that overlap on one GPU (two streams, two
   host threads) race and must be ordered by the caller.  Does not synchronise. */
#define APC_NOALLOC_BYTES (32LL << 20)
int apc_interpolate_force_noalloc(apc_cloud *c, const double *phi, double *phi_p,
                                  double *grad_p, hipStream_t stream);

/* Scaled-back GFD derivatives d^alpha f at every interior node (n x p row-major,
   p = 9 for k = 2, columns x,y,z,xx,xy,xz,yy,yz,zz).  f: n+nb. */
int apc_node_derivs(apc_cloud *c, const double *f, double *D, hipStream_t stream);

/* Apply the assembled operator: out[i] = (L f)_i for interior i; f: n+nb. */
int apc_apply_operator(apc_cloud *c, const double *f, double *out, hipStream_t stream);

/* Host copy of the density operator B of the WLS charge assignment (eq.
   density_linear_system), as the density solve applies it: bw_host[nnz] aligned
   with the stencil CSR, bdiag_host[n], so that (B f)_i = bdiag_i f_i +
   sum_j bw_ij f_j, and order_host[n] (int8) the order of each row.  Stability
   rule (the paper states no bound; a reading): a row of the node's fit order is
   kept when sum_j |b_ij| <= 0.5 b_ii; an order-4 row that fails is replaced by
   the order-2 row of the same stencil (the fit on the 9 unknowns of order 1 and
   2, moments a_(2 e_d) = h_c^2 / 24 only), and a row that still fails by the
   identity row (rho~_i = rho_M,i, order 0).  Every row of B then meets the bound,
   so the density solve converges at a rate independent of n.  k = 2 rows are
   b = (h_c^2 / 24) w with diagonal 1 + (h_c^2 / 24) d (w, d the Poisson row);
   APC_MIXED widens the stored FP32 values exactly.  Any pointer may be NULL.
   Requires apc_assemble_gfd.  Synchronises the device. */
int apc_get_density_operator(const apc_cloud *c, double *bw_host, double *bdiag_host,
                             int8_t *order_host);

/* GFD order of every interior node's row into host memory (n int8): the cloud's
   k, or 2 where a k = 4 cloud found no acceptable order-4 stencil up to ring_max
   and the node took an order-2 row instead (order fallback, Sec. 4.3 reading). */
int apc_get_node_orders(const apc_cloud *c, int8_t *order_host);

/* ---- learned preconditioner (a grown form beside the paper's method) ----
   Row i of M has the pattern of row i of the Poisson operator: J_0 = i and J_p the
   p-th stencil node (p = 1..min(m, 40); boundary nodes carry weight 0), and is
   written as m_i = (e_0 + o_i) / d_i, d_i the operator's diagonal: o_i = 0 is
   Jacobi.  k = 2 stencils hold at most 40 nodes, so M has the whole pattern of
   the row; k = 4 rows (up to 56 nodes) keep their 40 nearest.  One parameter
   set serves one order: the operators of k = 2 and k = 4 differ in kind.  The network maps row features to o_i (APC_MLP_OUT entries, those
   beyond m unused).  Training minimises the left approximate-inverse loss
   ||m_i^T A - e_i^T||^2 per row, estimated with K probe vectors z ~ N(0, I):
   E (m_i^T A z - z_i)^2.  Per row this is the quadratic
   L_i(o) = m~^T Q m~ - 2 b^T m~ + c in m~ = e_0 + o.

   Features and quadratic data of every interior row for K probes Z (K x (n+nb)
   float64, boundary entries ignored): feat n x APC_MLP_IN float32, quad
   n x APC_LEARN_QUAD float32 (Q packed lower row-major, then b, then c).
   Features: the row's Poisson weights divided by |d_i| in stencil order (the
   first 40, zero padded); level(J_p) - level(i) of the first 6 stencil nodes (0
   for boundary nodes); m / 40; the fraction of boundary nodes in the stencil.  All
   are scale-free, so clouds of any depth share one network.  Z may be NULL (K
   ignored, quad untouched): features only.  Requires
   apc_assemble_gfd.  Does not synchronise. */
int apc_learn_data(apc_cloud *c, const double *Z, int K, float *feat, float *quad,
                   hipStream_t stream);

/* Mean loss over the rows listed in rows[B] (indices into feat/quad) and its
   gradient with respect to the parameters (FP32, own forward/backward kernels).
   loss: 1 float, grad: APC_MLP_NPARAM floats (overwritten).  Does not synchronise. */
int apc_mlp_loss_grad(const float *params, const float *feat, const float *quad,
                      const int32_t *rows, int B, float *loss, float *grad, hipStream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step >= 1) on params with the
   gradient of apc_mlp_loss_grad; m and v are the Adam moments (APC_MLP_NPARAM
   floats each, zero before the first step). */
int apc_mlp_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                 hipStream_t stream);

/* Network output o for every interior row of the cloud (n x APC_MLP_OUT float32)
   from feat (n x APC_MLP_IN, as written by apc_learn_data).  bf16 = 0: FP32
   arithmetic throughout; bf16 = 1: the inference that apc_set_learned_precond
   runs (weights and activations rounded to bfloat16, MFMA products, FP32
   accumulation, FP32 biases).  Does not synchronise. */
int apc_mlp_infer(apc_cloud *c, const float *params, const float *feat, int bf16, float *out,
                  hipStream_t stream);

/* Install the learned preconditioner of the cloud: features, then BF16 MFMA
   inference with FP32 accumulation, then M stored in the solver's sliced layout
   (FP32).  Rows whose stencil is the uniform same-level 2-ring have identical
   features at a given level; M keeps one row per level for them (the network's
   output for the first such row of that level) and each such row's safeguard
   weight alpha_i below.
   Safeguard (Z != NULL): K probe vectors Z (K x (n+nb) float64, boundary
   entries ignored).  Every row becomes m_i = j_i + alpha_i (m_i - j_i),
   j_i the Jacobi row, with alpha_i in [0, 1] minimising the probe estimate
   sum_k ((j_i + alpha (m_i - j_i))^T A z_k - z_ki)^2 (alpha_i = 1 when the two
   rows agree), so that rows the network does not know fall back towards
   Jacobi.  Z = NULL: alpha = 1 everywhere.  Requires apc_assemble_gfd (and again
   after every re-assembly, which drops M).  Synchronises. */
int apc_set_learned_precond(apc_cloud *c, const float *params, const double *Z, int K,
                            hipStream_t stream);

/* Apply a preconditioner: out = M in over the interior rows.  precond
   APC_PRECOND_NONE: out = in; APC_PRECOND_JACOBI: out_i = in_i / d_i;
   APC_PRECOND_LEARNED: the installed M (boundary entries of in are ignored).
   in: n+nb, out: n, device.  Requires apc_assemble_gfd.  Does not synchronise. */
int apc_apply_precond(apc_cloud *c, int precond, const double *in, double *out,
                      hipStream_t stream);

/* ---- batches of independent clouds (a grown form beside the paper's method) ----
   count clouds built with the same parameters are held as one union: node
   vectors of the batch (n_total + nb_total) carry the interior nodes of cloud 0,
   1, ... first (cloud c at [ibase_c, ibase_c + n_c), ibase_c = sum of n before c,
   its nodes in the order of a single cloud), then the boundary nodes in the same
   cloud order; particle arrays (N_total) carry cloud c's particles, in the
   caller's order, at [pbase_c, pbase_c + N_c).  Assembly, deposit, right-hand
   sides, operator applies and interpolation run as single launches over all
   clouds; every cloud keeps its own BiCGSTAB (own scalars and convergence test,
   so its iterates are those of a single-cloud solve up to rounding), replayed
   from a HIP graph of `chunk` iterations until every cloud has stopped. */
typedef struct apc_batch apc_batch;
typedef struct {
  int64_t count, N, n, nb, nnz, nsl; /* clouds; totals over the batch; slices */
  int use_graph, chunk;               /* solver replay: HIP graph on/off, iterations per replay */
  int spmv_blocks, pad;               /* workgroups of the batched SpMV */
} apc_batch_info_t;

/* Build count clouds (xyz[c]: device pointer of cloud c's 3 x N[c] SoA particles;
   xyz and N are host arrays), then their union.  Same errors as
   apc_build_cloud, for the first cloud that fails; APC_EINVAL for order 4, a
   periodic domain or a CIC / TSC kernel (a batch holds bounded order-2 clouds
   with the NGP deposit).  Synchronises. */
int apc_build_batch(const apc_params *p, int count, const double *const *xyz, const int64_t *N,
                    hipStream_t stream, apc_batch **out);
/* Totals and launch shape; per-cloud sizes into host arrays (each may be NULL). */
int apc_batch_info(const apc_batch *b, apc_batch_info_t *info, int64_t *cloud_N,
                   int64_t *cloud_n, int64_t *cloud_nb);
/* Solver launch shape: use_graph 0/1 (-1 keeps), chunk iterations per replay
   (<= 0 keeps), SpMV workgroup divisor 1, 2, 4 or 8 (<= 0 keeps). */
int apc_batch_configure(apc_batch *b, int use_graph, int chunk, int spmv_div);
/* Autotuner: times the batched SpMV for each workgroup divisor and whole Jacobi
   solves (to tol, right-hand side from the batch's own deposit) for chunk 4, 8,
   16 and 32; keeps the fastest of each and returns them (host ints, may be
   NULL).  Requires apc_batch_assemble.  Synchronises. */
int apc_batch_tune(apc_batch *b, double tol, int *spmv_div, int *chunk, hipStream_t stream);
/* The operator of every cloud (apc_assemble_gfd on each), one launch. */
int apc_batch_assemble(apc_batch *b, hipStream_t stream);
/* apc_deposit for every cloud: q (N_total, or NULL for 1/N_c per particle of
   cloud c), rho_M (may be NULL) and rho_t (n_total + nb_total); st: count
   host records (may be NULL; ms is the batch's time).  Synchronises. */
int apc_batch_deposit(apc_batch *b, const double *q, double *rho_M, double *rho_t, double tol,
                      int maxit, apc_stats *st, hipStream_t stream);
/* apc_solve for every cloud: rho_t (n_total, or longer), g (nb_total or NULL),
   phi (n_total + nb_total), precond APC_PRECOND_NONE, APC_PRECOND_JACOBI or
   APC_PRECOND_LEARNED (after apc_batch_set_learned_precond; APC_EINVAL
   otherwise); st: count host records (may be NULL).  Returns APC_ENOCONV if any
   cloud did not converge (see its record).  Synchronises. */
int apc_batch_solve(apc_batch *b, const double *rho_t, const double *g, double *phi, double tol,
                    int maxit, int precond, apc_stats *st, hipStream_t stream);
/* apc_set_learned_precond for every cloud of a second-order batch, on the union
   (features and M rows are local to a row's stencil, so each cloud's rows of M
   are those of a single-cloud install; the uniform 2-ring rows of one level share
   one row of M across the batch).  params: APC_MLP_NPARAM floats (device); Z: K
   probe vectors of n_total + nb_total float64 for the safeguard (device, or NULL
   for none).  Requires apc_batch_assemble (APC_EINVAL otherwise, and for order
   4).  Synchronises. */
int apc_batch_set_learned_precond(apc_batch *b, const float *params, const double *Z, int K,
                                  hipStream_t stream);
/* apc_interpolate_force for every cloud: phi (n_total + nb_total), phi_p
   (N_total), grad_p (3 x N_total SoA).  Does not synchronise. */
int apc_batch_interpolate_force(apc_batch *b, const double *phi, double *phi_p, double *grad_p,
                                hipStream_t stream);
/* One field solve of every cloud of the batch -- assembly, NGP deposit and density
   solve, Poisson solve, interpolation -- replayed as one HIP graph with no host work
   inside.  Each of the two BiCGSTAB solves runs a fixed budget of iterations in the
   graph: every cloud tests its own convergence on the device and skips its rows
   once it has stopped, and one true-residual check on the device closes each
   solve.  The first call runs the separate entry points (apc_batch_assemble,
   apc_batch_deposit, apc_batch_solve, apc_batch_interpolate_force) and sets the
   budgets from every cloud's iteration counts (the largest, plus a quarter, at
   least 4); later calls replay the graph, which is recorded again when a pointer,
   a tolerance, maxit, the preconditioner or the SpMV launch shape changes.  A
   replay that leaves a cloud unfinished (more iterations or a restart needed)
   enlarges the budgets and runs that call through the separate entry points.
   q (N_total or NULL), g (nb_total or NULL), rho_t (n_total + nb_total), phi
   (n_total + nb_total), phi_p (N_total), grad_p (3 x N_total) as in those entry
   points; precond APC_PRECOND_NONE, APC_PRECOND_JACOBI or APC_PRECOND_LEARNED
   (after apc_batch_set_learned_precond; the density solve runs without).
   st_density, st: count host records each (may be NULL; ms is the
   graph's time when it ran); *graph_used (may be NULL): 1 when this call replayed
   the graph.  Returns APC_ENOCONV if a cloud did not converge.  Synchronises.
   The graph holds the batch's workspace: calls on one batch must not overlap. */
int apc_batch_pipeline(apc_batch *b, const double *q, const double *g, double tol_density,
                       double tol, int maxit, int precond, double *rho_t, double *phi,
                       double *phi_p, double *grad_p, apc_stats *st_density, apc_stats *st,
                       int *graph_used, hipStream_t stream);
void apc_batch_destroy(apc_batch *b);

/* ---- Vlasov-Poisson time loop (Sec. 1) ----
   The particles move in the field the three steps of Sec. 3.2 compute from their
   own positions; the node cloud is re-selected from the current positions every
   step (Sec. 4).  The paper leaves the time integrator open: this is the
   leapfrog scheme in kick-drift form, velocities half a step behind positions. */

/* Particle push: per particle and axis v <- v + kick grad, then x <- x + dt v,
   each product and sum rounded on its own (no fused multiply-add).  kick is dt
   times the caller's charge-to-mass coupling (its sign is the caller's: grad is
   grad phi); kick = coupling dt / 2 on the first step staggers the velocities.
   A particle that ends outside Omega = [p->lo, p->lo + p->L]^3 is reflected
   specularly: per axis u = (x - lo) / L, f = floor(u) wall crossings,
   r = u - f, u <- r (f even) or 1 - r (f odd), x = lo + u L, and the velocity
   component changes sign for odd f; a particle inside keeps x + dt v.  With
   p->periodic the particle re-enters through the opposite face instead (u <- r,
   velocity unchanged).  Only p->lo, p->L and p->periodic are read.  xyz, vel: 3 x N float64, updated in place; grad:
   3 x N (as apc_interpolate_force writes it).  Errors: APC_EINVAL (N < 0,
   L <= 0, a non-finite lo, L, kick or dt, NULL arrays with N > 0).  Does not
   synchronise. */
int apc_push(const apc_params *p, int64_t N, double *xyz, double *vel, const double *grad,
             double kick, double dt, hipStream_t stream);

typedef struct {
  int64_t n, nb, nnz;    /* the step's node cloud */
  int density_iters;     /* BiCGSTAB iterations of the density solve */
  int iters;             /* BiCGSTAB iterations of the Poisson solve */
  int status;            /* APC_OK, or APC_ENOCONV if a solve stopped at maxit */
  int pad;
  double rel_resid_true; /* Poisson solve: ||b - A x|| / ||b|| */
  double ms[6];          /* device time of build, assemble, deposit (with the density
                            solve), Poisson solve, interpolation, push */
} apc_step_stats;

/* One time step: apc_build_cloud(p, xyz), apc_assemble_gfd, apc_deposit(q,
   tol_density), apc_solve (phi = 0 on the boundary, tol, precond
   APC_PRECOND_NONE or APC_PRECOND_JACOBI), apc_interpolate_force into phi_p[N]
   and grad_p[3 x N] (the field at the positions the step started from), then
   apc_push(kick, dt) of xyz and vel.  maxit bounds both solves.  The node cloud
   and its buffers live for the call only.  st_host (may be NULL) receives the
   cloud's sizes, iteration counts and per-phase device times.  Returns APC_OK,
   APC_ENOCONV when a solve stopped at maxit (the step still completes with the
   last iterate), or the first error of a phase (xyz and vel are then unchanged
   unless the push itself ran).  Synchronises the stream. */
int apc_step(const apc_params *p, double *xyz, double *vel, const double *q, int64_t N,
             double kick, double dt, double tol_density, double tol, int maxit, int precond,
             double *phi_p, double *grad_p, apc_step_stats *st_host, hipStream_t stream);

/* Diagnostics of the cloud's solves (flags, a combination of APC_DIAG_*; 0 = off,
   the default).  APC_DIAG_KERNEL_TIMES records HIP events on the solve's stream
   around the two operator SpMVs (k_spmv_v, k_spmv_t) of every iteration and
   reports their summed device time and count in apc_stats.spmv_ms /
   spmv_launches (iterations that ran after the solver stopped are not counted);
   the events add marker packets between kernels.  APC_DIAG_FP64_RESIDUAL makes
   apc_solve in the mixed modes compute rel_resid_fp64ref once at exit (an FP64
   refit of every k = 2 row, or the FP64 copy of the k = 4 rows that assembly
   then also keeps), outside the iteration. */
int apc_set_diagnostics(apc_cloud *c, int flags);

void apc_destroy(apc_cloud *c);

/* ---- the two-dimensional variant (quadtree nodes, k = 2; Sec. 5.1) ----
   The method of the calls above with one dimension fewer: Omega = [lo[0], lo[0] +
   L] x [lo[1], lo[1] + L]; cells open when N' >= (c 2^l / L)^2 (eq.
   errorbalance_implementation) below max_depth, then the 2:1 balance across the 4
   faces; nodes are the leaves in Morton order (x bit above y), boundary nodes sit
   at the centre of every leaf face on the boundary (faces 0..3 = -x, +x, -y, +y),
   ordered by (owner, face); stencils by the quadrant criterion (Sec. 3.1: the two
   nearest candidates of every closed quadrant, then the nearest remaining ones up
   to m_cap, 8 being the paper's choice) from the R-ring (R = ring_min ..
   ring_max), accepted when every closed quadrant holds a chosen node, m >= 6 and
   the weighted normal equations have min/max Cholesky diagonal >= 1e-6; the
   second-order fit has the 5 unknowns of x, y, x^2/2, xy, y^2/2; NGP deposit onto
   the node's cell (area h^2); density rows b = (h_c^2 / 24) w with the stability
   rule of the three-dimensional k = 2 rows; FP64 throughout.  Integer node
   coordinates are in units of L 2^-(max_depth+1) from lo. */
typedef struct apc2_cloud apc2_cloud;
/* xy: device pointer, 2 x N float64 (SoA).  Reads lo[0..1], L, order (must be 2),
   c, max_depth (1..20), ring_min, ring_max, m_cap (6..64), poisson_c and
   criterion_pow.  Errors: APC_EINVAL (parameters, NaN), APC_EDOMAIN (a particle
   outside Omega), APC_ESTENCIL (no acceptable stencil up to ring_max, or a ring
   beyond 1024 nodes).  Synchronises. */
int apc2_build_cloud(const apc_params *p, const double *xy, int64_t N, hipStream_t stream,
                     apc2_cloud **out);
int apc2_cloud_info(const apc2_cloud *c, int64_t *n, int64_t *nb, int64_t *nnz,
                    int64_t *n_opened);
/* Host arrays (each may be NULL): perm[N] (sorted position -> caller's index),
   code/level/first/count [n], bowner/bface [nb], st_off [n+1], st_idx [nnz] (the
   stencils in (r^2, index) order), ixy [2 x (n + nb)].  Synchronises. */
int apc2_get_nodes(const apc2_cloud *c, int32_t *perm, uint64_t *code, int32_t *level,
                   int32_t *first, int32_t *count, int32_t *bowner, int32_t *bface,
                   int32_t *st_off, int32_t *st_idx, int32_t *ixy);
/* Laplacian and density rows of every node (Sec. 3.1, eq. density_linear_system).
   APC_ESTENCIL if a stencil lost rank.  Synchronises. */
int apc2_assemble(apc2_cloud *c, hipStream_t stream);
/* Host copies (each may be NULL): Laplacian w [nnz] (difference form) and diagonal
   [n]; density rows bw [nnz], diagonal [n], order [n] (2, or 0 for the identity
   row).  APC_EINVAL before apc2_assemble.  Synchronises. */
int apc2_get_operator(const apc2_cloud *c, double *w_host, double *diag_host, double *bw_host,
                      double *bdiag_host, int8_t *order_host);
/* rho_M [n + nb] (device): the charge in each node's cell over h^2 (q: device
   array of N charges in the caller's order, or NULL for 1/N each); boundary nodes
   take their owner's value.  Does not synchronise. */
int apc2_deposit(apc2_cloud *c, const double *q, double *rho_M, hipStream_t stream);
/* B rho~ = rho_M (eq. density_linear_system), plain BiCGSTAB to tol; rho_t [n + nb]
   (boundary values copied).  Returns APC_OK, APC_ENOCONV, or an error.
   Synchronises. */
int apc2_density_solve(apc2_cloud *c, const double *rho_M, double *rho_t, double tol, int maxit,
                       apc_stats *st, hipStream_t stream);
/* Delta phi = poisson_c rho~ (eq. Poisson) with phi = g on the boundary nodes (g:
   device [nb] or NULL for 0); precond APC_PRECOND_NONE or APC_PRECOND_JACOBI.
   phi [n + nb].  Synchronises. */
int apc2_solve(apc2_cloud *c, const double *rho_t, const double *g, double *phi, double tol,
               int maxit, int precond, apc_stats *st, hipStream_t stream);
/* Derivatives of each node's fitted quadratic, D [n x 5] (device): phi_x, phi_y,
   phi_xx, phi_xy, phi_yy.  Does not synchronise. */
int apc2_node_derivs(apc2_cloud *c, const double *f, double *D, hipStream_t stream);
/* Taylor interpolation (Sec. 3.2 step 3) of phi [n + nb] to the particles, in the
   caller's order: phi_p [N] and grad_p [2 x N] (device).  Does not synchronise. */
int apc2_interpolate_force(apc2_cloud *c, const double *phi, double *phi_p, double *grad_p,
                           hipStream_t stream);
void apc2_destroy(apc2_cloud *c);

const char *apc_strerror(int code);
/* Text of the last HIP error seen by the calling thread (empty if none). */
const char *apc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

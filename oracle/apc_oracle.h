/*
 * apc_oracle.h -- plain, slow, FP64 CPU oracle of the AP-Cloud field solve
 * (Wang, Samulyak, Jiao, Yu, "AP-Cloud: Adaptive Particle-in-Cloud Method for
 * Optimal Solutions to Vlasov-Poisson Equation").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source
 * with the HIP library (no headers, helpers or tables); the two agree only
 * through the paper and the readings written down beside each function.
 *
 * All pointers are host pointers.  All functions return 0 on success and a
 * negative APCO_E* code on failure.  Node numbering: interior nodes (octree
 * leaves) 0..n-1 in ascending Morton order of their minimum corner, then
 * boundary nodes n..n+nb-1 ordered by (owner node, face id), face ids
 * 0..5 = -x,+x,-y,+y,-z,+z.  Integer node coordinates are in units of
 * L * 2^-(max_depth+1) measured from lo (cell centres are odd multiples).
 */
#ifndef APC_ORACLE_H
#define APC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define APCO_OK 0
#define APCO_EINVAL (-1)
#define APCO_ENOMEM (-2)
#define APCO_EDOMAIN (-4)
#define APCO_ESTENCIL (-5)
#define APCO_ENOCONV 1

typedef struct {
  double lo[3];   /* domain Omega = [lo, lo+L]^3 */
  double L;
  int order;      /* GFD order k: 2 or 4 */
  double c;       /* error-balance tuning constant (Sec. 4.3, eq. errorbalance_implementation) */
  int max_depth;  /* deepest octree level, <= 20 */
  int ring_min;   /* first ring searched for a stencil (2 for k=2, 3 for k=4) */
  int ring_max;   /* last ring searched (5, Sec. 4.3) */
  int m_cap;      /* stencil size cap (40 for k=2, 56 for k=4); hard cap 64 */
  double poisson_c; /* Delta phi = c rho (eq. Poisson) */
  int criterion_pow; /* exponent e of T_l = (c 2^l / L)^e: 0 = 2k - 2 (eq.
                        errorbalance_implementation); 4 with k = 2 is the balance
                        of the supraconvergent second-order error bound (Sec. 3.3;
                        its optimal h, Sec. 3.4), h = c N'^(-1/4) */
  double tau_dom; /* stability bound of order-4 Laplacian rows: accepted when the
                     diagonal is negative and sum_j |w_j| <= tau_dom |diag|;
                     0 = the default 10 */
  int periodic;   /* 1: Omega is periodic in x, y and z (Sec. 4.3 "non-periodic region"
                     read the other way): face neighbours wrap around, no boundary
                     nodes, stencil offsets are minimum images, levels 0 and 1 are
                     always opened (max_depth >= 2), and the Poisson problem is
                     Delta phi = c (rho~ - mean rho~) with phi of mean 0 (means
                     weighted by cell volume); 0: the Dirichlet box */
  int kernel;     /* charge-assignment kernel Phi of eq. density_apcloud: APCO_KERNEL_NGP
                     (0, the node's own cell), APCO_KERNEL_CIC (1, the tent, support
                     |u| <= 1 per axis) or APCO_KERNEL_TSC (2, the quadratic B-spline,
                     |u| <= 3/2), u = (x - y) / h with h the node's cell edge */
  int mask_level; /* irregular domain (0: none): Omega is the box minus the cells of
                     the uniform level-mask_level grid that mask excludes (1 ..
                     min(6, max_depth)); the walls are the box faces and the faces
                     between included and excluded cells.  Cells of a level below
                     mask_level are always opened unless wholly excluded, excluded
                     cells never; leaves in excluded cells are not nodes; a node's
                     face on a wall carries a boundary node at its centre.  The
                     stencil rule's last ring (ring_max) does not ask for an octant
                     in which it holds no node (a convex corner of the staircase).
                     Not with periodic or a CIC / TSC kernel. */
  const uint8_t *mask; /* (2^mask_level)^3 bytes, index x + s (y + s z), s = 2^mask_level;
                          nonzero: excluded.  Read during apco_build_cloud only. */
} apco_params;

#define APCO_KERNEL_NGP 0
#define APCO_KERNEL_CIC 1
#define APCO_KERNEL_TSC 2

typedef struct {
  int iters;
  int status;           /* 0 converged, APCO_ENOCONV otherwise */
  double rel_resid;     /* recursive ||r||/||b|| at exit */
  double rel_resid_true;/* ||b - A x|| / ||b|| recomputed at exit */
} apco_stats;

typedef struct apco_cloud apco_cloud;

/* Number of fitted derivative unknowns p = C(k+3,3) - 1 (9 for k=2, 34 for k=4). */
int apco_num_unknowns(int order);
/* Multi-index table of the fitted unknowns in column order (p x 3 ints). */
int apco_monomials(int order, int32_t *alpha);
/* Refinement thresholds T_l = (c 2^l / L)^e, l = 0..max_depth, e = 2k-2 or criterion_pow. */
int apco_thresholds(const apco_params *P, double *T);

/* Build octree, node set, boundary nodes and GFD stencils from N particles
   (xyz: 3 x N structure of arrays). */
int apco_build_cloud(const apco_params *P, const double *xyz, int64_t N, apco_cloud **out);
void apco_destroy(apco_cloud *C);
int apco_info(const apco_cloud *C, int64_t *n, int64_t *nb, int64_t *nnz, int64_t *n_opened,
              int64_t *ncells);
/* perm[N] (sorted position -> original index), node codes/levels/particle ranges,
   boundary owner/face, stencil CSR (off-diagonal neighbours only). Any pointer may be NULL. */
int apco_get_nodes(const apco_cloud *C, int64_t *perm, uint64_t *code, int32_t *level,
                   int64_t *first, int64_t *count, int32_t *bowner, int32_t *bface,
                   int32_t *st_off, int32_t *st_idx, int32_t *st_ring);
/* GFD order of each interior node's row (n int8): the cloud's k, or 2 where a
   k = 4 cloud found no acceptable order-4 stencil (order fallback). */
int apco_node_orders(const apco_cloud *C, int8_t *ord);
/* Integer coordinates of all n+nb nodes, 3 x (n+nb) SoA. */
int apco_node_coords(const apco_cloud *C, int32_t *ixyz);
/* All cells of the queue Q in creation order: level, integer index (3), particle count,
   opened flag (0 leaf, 1 opened by the criterion, 2 opened for 2:1 balance). */
int apco_get_cells(const apco_cloud *C, int32_t *level, int32_t *ijk, int64_t *count,
                   int32_t *opened);
/* 1-ring adjacency of interior nodes (incl. their boundary nodes): offsets n+1, idx. */
int apco_ring1(const apco_cloud *C, int32_t *off, int32_t *idx, int64_t cap);

/* Weighted least-squares GFD fit on an explicit stencil (Sec. 3.1): delta is m x 3
   (row-major) of neighbour offsets; returns X (p x m, row-major) with
   h^{|alpha|} d^alpha f(y0) ~= sum_j X[alpha][j] (f_j - f_0), the stencil scale
   h = max |delta| and the R-diagonal ratio min|R_ii| / max|R_ii|. */
int apco_wls_fit(int order, int m, const double *delta, double *X, double *h, double *ratio);

/* Poisson rows: off-diagonal weights w (nnz, aligned with the stencil CSR) and the
   diagonal (n), so that (L f)_i = diag_i f_i + sum_j w_ij f_j. */
int apco_assemble(const apco_cloud *C, double *w, double *diag);
/* BiCGSTAB (the solver of apco_poisson_solve) on caller-assembled rows w/diag and
   an interior right-hand side rhs (n); x (n) receives the solution. */
int apco_bicgstab_rows(const apco_cloud *C, const double *w, const double *diag,
                       const double *rhs, double *x, double tol, int maxit, int precond,
                       apco_stats *st);
/* Density rows B (eq. density_linear_system), same layout, with the stability
   rule: a row is kept when sum_j |b_j| <= 0.5 b_ii; an order-4 row that fails
   is replaced by the order-2 row of the same stencil, and a row that still fails
   by the identity row. */
int apco_density_rows(const apco_cloud *C, double *bw, double *bdiag);
/* Order of every interior node's density row (n int8): the node's fit order, 2
   (order-4 row replaced by the order-2 row of the same stencil) or 0 (identity). */
int apco_density_orders(const apco_cloud *C, int8_t *ord);
/* NGP deposit (Sec. 5.1 kernel choice): rho_M for all n+nb nodes (boundary node takes
   its owner's value).  q may be NULL: every particle then carries 1/N. */
int apco_deposit(const apco_cloud *C, const double *q, double *rho_M);
/* eq. density_apcloud's right-hand side with the cloud's kernel, from the
   particle positions xyz (3 x N, the order the cloud was built from):
   rho_M(y_j) = sum_i q_i Phi((p_i - y_j) / h_j) / (a_0(y_j) h_j^3), a_0 the
   kernel's mass inside Omega (1 away from the walls).  The NGP kernel gives
   apco_deposit's values.  q NULL: 1/N each. */
int apco_deposit_xyz(const apco_cloud *C, const double *xyz, const double *q, double *rho_M);
/* 1-D kernel moment int_{max(tlo,-s)}^{min(thi,s)} u^k phi(u) du of kernel
   (APCO_KERNEL_*), s its half-support; tlo/thi may be +-INFINITY. */
double apco_kernel_moment(int kernel, int k, double tlo, double thi);
/* Solve B rho~ = rho_M over interior nodes (boundary values moved to the rhs).
   rho_M, rho_t: n+nb. precond: 0 none, 1 Jacobi (right). */
int apco_density_solve(const apco_cloud *C, const double *rho_M, double *rho_t, double tol,
                       int maxit, int precond, apco_stats *st);
/* Solve the GFD Poisson system for phi at interior nodes with phi = g on boundary
   nodes (g may be NULL: zero).  rho_t: n (or n+nb); phi: n+nb out. */
int apco_poisson_solve(const apco_cloud *C, const double *rho_t, const double *g, double *phi,
                       double tol, int maxit, int precond, apco_stats *st);
/* Same system solved by dense LU with partial pivoting (small n only). */
int apco_poisson_lu(const apco_cloud *C, const double *rho_t, const double *g, double *phi);
/* Apply the Poisson operator: out_i = (L f)_i for interior i, f over n+nb nodes. */
int apco_apply_laplacian(const apco_cloud *C, const double *f, double *out);
/* Scaled-back derivatives d^alpha f at every interior node (n x p, row-major). */
int apco_node_derivs(const apco_cloud *C, const double *f, double *D);
/* Taylor interpolation of phi and grad phi to the particles, original order.
   grad: 3 x N SoA. */
int apco_interpolate(const apco_cloud *C, const double *phi, const double *xyz, double *phi_p,
                     double *grad_p);

/* Leapfrog push of the Vlasov-Poisson loop: per particle and axis
   v <- v + kick grad, then x <- x + dt v (each product and sum rounded on its own),
   and a particle that leaves Omega is reflected specularly at its faces (velocity
   component negated once per wall crossing).  xyz, vel: 3 x N in/out; grad: 3 x N. */
int apco_push(const apco_params *P, int64_t N, double *xyz, double *vel, const double *grad,
              double kick, double dt);

/* ---- learned preconditioner (checks of the training data and gradients) ----
   Row i of M has the pattern J_0 = i, J_p = the p-th stencil node (p = 1..m,
   m <= 40) and is m_i = (e_0 + o_i) / d_i with o_i (41) the network output.
   Row features (n x 48): Poisson weights / |d_i| in stencil order (40 slots, zero
   padded); level(J_p) - level(i) of the first 6 stencil nodes (0 for boundary
   nodes); m / 40; the fraction of boundary nodes in the stencil.
   Quadratic data (n x 903) from K probes Z (K x (n+nb), boundary entries
   ignored): with U = A Z over the interior unknowns and u_p = U[J_p] / d_i (0 for
   boundary or absent J_p): Q = u u^T / K (packed lower, 861), b = u z_i / K (41),
   c = z_i^2 / K. */
int apco_learn_data(const apco_cloud *C, const double *Z, int K, double *feat, double *quad);
/* Mean over rows[B] of L(o) = m^T Q m - 2 b^T m + c, m = e_0 + o, o = MLP(feat) with
   the 48 -> 64 -> 64 -> 41 ReLU network, params laid out [W1 (48x64), b1, W2 (64x64),
   b2, W3 (64x41), b3]; the gradient of that mean with respect to params. */
int apco_mlp_loss_grad(const double *params, const double *feat, const double *quad,
                       const int32_t *rows, int B, double *loss, double *grad);
/* Network output o (nrow x 41) of every feature row (nrow x 48), same layout. */
int apco_mlp_forward(const double *params, const double *feat, int64_t nrow, double *out);
/* Rows of the learned M: diagonal mdiag (n) and off-diagonal weights mw aligned
   with the stencil CSR (boundary columns 0), m_i = (e_0 + o_i) / d_i.  With K
   probes Z (K x (n+nb), boundary entries ignored), every row that is not a
   uniform 2-ring row (24 stencil nodes at offsets, in cells of the row's level,
   with components in {0, 1, 2} and L1 norm <= 2) becomes j_i + alpha (m_i - j_i),
   j_i the Jacobi row, alpha in [0, 1] minimising sum_k ((.)^T A z_k - z_ki)^2
   (alpha = 1 when t = 0). */
int apco_learned_m(const apco_cloud *C, const double *params, const double *Z, int K,
                   double *mdiag, double *mw);

#ifdef __cplusplus
}
#endif
#endif

/*
 * apc_oracle2d.h -- plain, slow, FP64 CPU oracle of the two-dimensional AP-Cloud
 * field solve (quadtree nodes, second-order GFD), the variant of Sec. 5.1.
 *
 * TEST INFRASTRUCTURE ONLY, like apc_oracle.h: only the test suite, the smoke
 * check and the CPU baseline leg of the benchmark may load it, and it shares no
 * source with the HIP library.
 *
 * The readings are those of the three-dimensional oracle with one dimension
 * fewer: Omega = [lo, lo + L]^2; Morton keys with 2 bits per level (x bit
 * higher); cells open when N' >= T_l = (c 2^l / L)^2 (eq.
 * errorbalance_implementation, k = 2) below max_depth, then the 2:1 balance
 * across faces from the deepest level up; nodes are the leaves in Morton order,
 * boundary nodes sit at the centre of every leaf face on the boundary (faces 0..3 =
 * -x, +x, -y, +y), ordered by (owner, face); the R-ring is the R-step face
 * adjacency (boundary nodes hang off their owner); the stencil is the two nearest
 * candidates of every closed quadrant (Sec. 3.1's quadrant criterion), then the
 * nearest remaining ones up to m_cap (8 by default: the paper's 8 neighbours in
 * two dimensions), accepted when every closed quadrant holds a chosen node, m >= 6
 * and the weighted Vandermonde matrix has min|R_ii| / max|R_ii| >= 1e-6.  Integer
 * node coordinates are in units of L 2^-(max_depth+1) from lo.
 */
#ifndef APC_ORACLE2D_H
#define APC_ORACLE2D_H
#include <stdint.h>

#include "apc_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct apco2_cloud apco2_cloud;

/* Reads lo[0..1], L, order (2), c, max_depth (1..20), ring_min, ring_max, m_cap
   (6..64), poisson_c and criterion_pow of P.  xy: 2 x N (structure of arrays). */
int apco2_build_cloud(const apco_params *P, const double *xy, int64_t N, apco2_cloud **out);
void apco2_destroy(apco2_cloud *C);
int apco2_info(const apco2_cloud *C, int64_t *n, int64_t *nb, int64_t *nnz, int64_t *n_opened);
/* perm[N], code[n] (Morton key of the cell's minimum corner at max_depth),
   level, first, count [n], bowner/bface [nb], st_off [n+1], st_idx [nnz]. */
int apco2_get_nodes(const apco2_cloud *C, int64_t *perm, uint64_t *code, int32_t *level,
                    int64_t *first, int64_t *count, int32_t *bowner, int32_t *bface,
                    int32_t *st_off, int32_t *st_idx);
/* integer coordinates 2 x (n + nb) */
int apco2_node_coords(const apco2_cloud *C, int32_t *ixy);
/* 1-ring CSR (off[n+1], idx[cap]) */
int apco2_ring1(const apco2_cloud *C, int32_t *off, int32_t *idx, int64_t cap);
/* Laplacian rows w[nnz] (difference form) and diagonals (Sec. 3.1). */
int apco2_assemble(const apco2_cloud *C, double *w, double *diag);
/* Density rows (eq. density_linear_system with the NGP cell of area h^2) and
   their orders (2, or 0 for the identity row of the stability rule). */
int apco2_density_rows(const apco2_cloud *C, double *bw, double *bdiag, int8_t *ord);
/* rho_M = (charge in the node's cell) / h^2; q NULL: 1/N each. */
int apco2_deposit(const apco2_cloud *C, const double *q, double *rho_M);
int apco2_density_solve(const apco2_cloud *C, const double *rho_M, double *rho_t, double tol,
                        int maxit, apco_stats *st);
/* Delta phi = c rho~ with phi = g on the boundary nodes (g may be NULL: 0). */
int apco2_poisson_solve(const apco2_cloud *C, const double *rho_t, const double *g, double *phi,
                        double tol, int maxit, int precond, apco_stats *st);
/* node derivatives n x 5: phi_x, phi_y, phi_xx, phi_xy, phi_yy */
int apco2_node_derivs(const apco2_cloud *C, const double *f, double *D);
/* Taylor interpolation to the particles (xy 2 x N, the build's order):
   phi_p[N], grad[2 x N] */
int apco2_interpolate(const apco2_cloud *C, const double *phi, const double *xy, double *phi_p,
                      double *grad);

#ifdef __cplusplus
}
#endif
#endif

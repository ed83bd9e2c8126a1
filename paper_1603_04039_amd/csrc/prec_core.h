// Learned preconditioner apply on the operator's sliced layout: the device code
// shared by the single-cloud and the batched solvers.
#pragma once
#include <hip/hip_runtime.h>

#include "apc_internal.h"
#include "spmv_core.h"

namespace {

// out = M in for the learned preconditioner.  Row i of M has the operator's
// pattern: m_ii in_i + sum_k m_ik in_{J_k}.  Uniform 2-ring slices read the
// per-level row of M (25 floats: diagonal, then the 24 entries in slice order)
// and no weights; general slices, and the uniform 56-node slices of k = 4, read
// their own weights, stored like the operator's (entry-major; padding and
// boundary columns carry weight 0).
struct MOp {
  const float *diag, *sell, *tmpl;
  int nt; // floats per level row of tmpl: 26 (k = 2), 42 (k = 4)
};
template <bool TOP, bool STG, bool NT>
__device__ __forceinline__ void prec_slice_nt(const Op &op, const MOp &M,
                                              const double *__restrict__ in,
                                              double *__restrict__ out, int s, int u) {
  const int lane = threadIdx.x & 63;
  const int64_t o = op.sl_off[s];
  const int64_t off = o + lane, lb = (o >> 1) + lane, hb = (o >> 2) + lane;
  double *tile = STG ? stage_tile(op) : nullptr;
  if (op.sl_tmpl[s] == 1) {
    int32_t jj[24];
    if (STG) {
      uint32_t wq[12];
#pragma unroll
      for (int k = 0; k < 12; k++) wq[k] = ld_layout<NT>(&op.sl_lx2[lb + (int64_t)SL * k]);
      stage_fill<NT>(tile, op.sl_uq + o, u, in);
#pragma unroll
      for (int k = 0; k < 24; k++) jj[k] = (int32_t)((wq[k >> 1] >> (16 * (k & 1))) & 0xffffu);
    } else {
#pragma unroll
      for (int k = 0; k < 24; k++) jj[k] = sl_col<TOP, NT>(op, lb, hb, k);
    }
    const int32_t row = op.sl_rows[(int64_t)s * SL + lane];
    if (row < 0) return;
    // the level's row T of M (diagonal, 24 entries, then 1 / d) and the row's
    // safeguard weight alpha: M_i = alpha T + (1 - alpha) e_i / d
    const float *__restrict__ T = M.tmpl + M.nt * (int)op.rk[row];
    double acc = (double)T[0] * in[row];
#pragma unroll
    for (int k = 0; k < 24; k++) acc += (double)T[k + 1] * (STG ? tile[jj[k]] : in[jj[k]]);
    const float a = M.diag[row];
    out[row] = a == 1.0f ? acc : (double)a * acc + (1.0 - (double)a) * ((double)T[25] * in[row]);
  } else if (op.sl_tmpl[s] != 0) {
    // uniform 56-node row (k = 4, boxed or not): the level's row T of M on the first
    // 40 stencil entries (the slice's order), like the 2-ring rows above
    if (STG) stage_fill<NT>(tile, op.sl_uq + o, u, in);
    const int32_t row = op.sl_rows[(int64_t)s * SL + lane];
    if (row < 0) return;
    const float *__restrict__ T = M.tmpl + M.nt * (int)op.rk[row];
    double acc = (double)T[0] * in[row];
#pragma unroll 8
    for (int k = 0; k < APC_MLP_OUT - 1; k++)
      acc += (double)T[k + 1] * (STG ? tile[stage_slot<NT>(op, lb, k)] : in[sl_col<TOP, NT>(op, lb, hb, k)]);
    const float a = M.diag[row];
    out[row] = a == 1.0f ? acc : (double)a * acc + (1.0 - (double)a) * ((double)T[M.nt - 1] * in[row]);
  } else {
    // M holds the first APC_MLP_OUT - 1 stencil entries of a row (all of them
    // for k = 2; the nearest 40 of the up to 56 of k = 4)
    const int len = min(op.sl_len[s], APC_MLP_OUT - 1);
    if (STG) stage_fill<NT>(tile, op.sl_uq + o, u, in);
    const int32_t row = op.sl_rows[(int64_t)s * SL + lane];
    if (row < 0) return;
    const float *__restrict__ wv = M.sell + off;
    double acc = (double)M.diag[row] * in[row];
#pragma unroll 8
    for (int k = 0; k < len; k++)
      acc += (double)ld_layout<NT>(&wv[k * SL]) * (STG ? tile[stage_slot<NT>(op, lb, k)] : in[sl_col<TOP, NT>(op, lb, hb, k)]);
    out[row] = acc;
  }
}

// the layout's loads non-temporal or not (see ld_layout)
template <bool TOP, bool STG>
__device__ __forceinline__ void prec_slice(const Op &op, const MOp &M, const double *__restrict__ in,
                                           double *__restrict__ out, int s, int u) {
  if (op.nt)
    prec_slice_nt<TOP, STG, true>(op, M, in, out, s, u);
  else
    prec_slice_nt<TOP, STG, false>(op, M, in, out, s, u);
}

} // namespace

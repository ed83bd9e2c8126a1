// Device core of the sliced-ELL operator apply, shared by the single-cloud and
// the batched solvers: operator descriptor, slice iteration and the row apply.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "apc_internal.h"

namespace {

enum { V64 = 0, V32A32 = 1, V32A64 = 2 }; // value type / arithmetic of the SpMV

struct Op {
  const int32_t *off;
  const int32_t *idx;
  const double *w64;
  const float *w32;
  const double *hs; // k = 2 density operator: x_i + hs_i (L x)_i; hs_i < 0: an explicit
                    // row x_i + sum_j dwx_ij (x_j - x_i) in CSR order (a kernel reaching
                    // past a wall)
  const double *dwx;
  int unit_diag;    // k = 4 density operator: x_i + (sum_j b_ij (x_j - x_i)) with its own weights
  const int8_t *rk; // level of a uniform row (2-ring, k = 2; 56-node, k = 4), else -1
  double tc[3];     // shell weights of the uniform 2-ring at h_c = 1
  double t4[5];     // shell weights of the uniform 56-node row (Laplacian at h_c = 1,
                    // or the density row)
  int t4_scaled;    // 1: Laplacian (t4 scaled like tc), 0: density row (scale-free)
  int pin;          // periodic Poisson solve: row 0 is the identity (phi_0 = 0 is imposed)
  double invL2;     // 1 / L^2: a level-l row scales tc by 4^l / L^2
  int64_t n;
  // sliced-ELL copy (the SpMV reads only this); column indices from the compact
  // 24-bit copy (plus the top byte for clouds of 2^24 nodes or more)
  const int32_t *sl_rows, *sl_len, *sl_tmpl;
  const uint32_t *sl_lo2, *sl_hi4, *sl_top4;
  const int64_t *sl_off;
  const double *sl_w64;
  const float *sl_w32;
  // neighbour staging (null / 0 when no slice is staged)
  const int32_t *sl_un, *sl_uq;
  const uint32_t *sl_lx2;
  int ucap;
  const int32_t *sl_box; // boxes of the boxed slices (APC_BOX_N node ids each, -1 unused)
  int64_t cs[9];
  int nt; // layout read with non-temporal loads (see ld_layout)
};

// Dynamic LDS of a kernel that applies the operator through sell_apply or
// prec_slice: one tile of ucap doubles per wavefront of the block.
static inline size_t op_lds(const Op &op) {
  return op.sl_un ? (size_t)(APC_BLOCK / 64) * (size_t)op.ucap * sizeof(double) : 0;
}


__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Slices (64 rows, one per wavefront) are grouped in 8 contiguous row chunks, one
// per XCD (workgroups are dealt round-robin over the 8 XCDs): block b works on
// chunk b mod 8, so neighbour gathers reuse that XCD's own L2.  Within a chunk
// the XCD's wavefronts stride over its slices.  The slice index is made
// wave-uniform (readfirstlane) so that the slice's offset, kind and length come
// from scalar loads and its column-index loads issue at once.
constexpr int SL = APC_SLICE;
constexpr unsigned GSPMV = 4096; // <= 4 FIN_T (one load batch per finalize thread)
struct SlIter {
  int s, end, step;
};
__device__ __forceinline__ SlIter sl_iter(const Op &op) {
  const int xcd = blockIdx.x & 7u, j = blockIdx.x >> 3;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  SlIter it;
  it.s = (int)op.cs[xcd] + j * (APC_BLOCK / 64) + wv;
  it.end = (int)op.cs[xcd + 1];
  it.step = (int)(gridDim.x >> 3) * (APC_BLOCK / 64);
  return it;
}
static inline unsigned spmv_grid(const apc_cloud *c) {
  int64_t mx = 0;
  for (int k = 0; k < 8; k++) mx = (c->sl_cs[k + 1] - c->sl_cs[k]) > mx ? (c->sl_cs[k + 1] - c->sl_cs[k]) : mx;
  int64_t per = (mx + (APC_BLOCK / 64) - 1) / (APC_BLOCK / 64);
  if (per < 1) per = 1;
  const int64_t g = 8 * per;
  return (unsigned)(g < (int64_t)GSPMV ? g : (int64_t)GSPMV);
}
// The layout arrays (packed column indices, staging lists and slots, box ids,
// weights) are read once per apply.  When they are far larger than the 256 MB
// Infinity Cache (op.nt) they go through non-temporal loads, so that the caches
// keep the gathered vector instead (same values; 408 -> 365 us per FP64 solver
// SpMV on the 1e8-particle fourth-order cloud); a smaller layout stays cached from
// one apply to the next, which non-temporal loads would defeat (42 -> 51 us on the
// 1e7-particle second-order cloud).  The choice is made once per slice call
// (sell_apply, prec_slice); a run-time select at each load let the compiler merge
// the two loads into a plain one.
template <bool NT, typename T>
__device__ __forceinline__ T ld_layout(const T *p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
//
// Column index of entry k of the lane's row: lb = o/2 + lane and hb = o/4 + lane
// for the slice at entry offset o.  Three bytes per entry (four with TOP): two
// 32-bit loads cover two and four entries, so a uniform row's 24 indices take 18
// loads instead of 24.
template <bool TOP, bool NT>
__device__ __forceinline__ int32_t sl_col(const Op &op, int64_t lb, int64_t hb, int k) {
  const uint32_t lo = (ld_layout<NT>(&op.sl_lo2[lb + (int64_t)SL * (k >> 1)]) >> (16 * (k & 1))) & 0xffffu;
  const uint32_t hi = (ld_layout<NT>(&op.sl_hi4[hb + (int64_t)SL * (k >> 2)]) >> (8 * (k & 3))) & 0xffu;
  uint32_t j = lo | (hi << 16);
  if (TOP) j |= ((ld_layout<NT>(&op.sl_top4[hb + (int64_t)SL * (k >> 2)]) >> (8 * (k & 3))) & 0xffu) << 24;
  return (int32_t)j;
}

// Tile of the calling wavefront in the block's dynamic LDS.
__device__ __forceinline__ double *stage_tile(const Op &op) {
  extern __shared__ double apc_stage_lds[];
  return apc_stage_lds + (threadIdx.x >> 6) * op.ucap;
}

// Orders the wavefront's LDS accesses before and after this point (the lanes of
// one wavefront read what other lanes wrote).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Gathers x at the slice's u distinct columns (ascending, so that neighbouring
// lanes read neighbouring addresses) into the tile: PER loads a lane in flight
// (all PER column loads, then all PER gathers).  Every lane of the wavefront takes
// part.
template <bool NT, int PER = 4>
__device__ __forceinline__ void stage_fill(double *tile, const int32_t *__restrict__ uq, int u,
                                           const double *__restrict__ x) {
  const int lane = threadIdx.x & 63;
  wave_lds_sync();
  for (int b = 0; b < u; b += PER * SL) {
    int32_t q[PER];
    double v[PER];
#pragma unroll
    for (int h = 0; h < PER; h++) q[h] = b + SL * h + lane < u ? ld_layout<NT>(&uq[b + SL * h + lane]) : -1;
#pragma unroll
    for (int h = 0; h < PER; h++) v[h] = q[h] >= 0 ? x[q[h]] : 0.0;
#pragma unroll
    for (int h = 0; h < PER; h++)
      if (q[h] >= 0) tile[b + SL * h + lane] = v[h];
  }
  wave_lds_sync();
}

// tile slot of entry k of the lane (lb = o/2 + lane)
template <bool NT>
__device__ __forceinline__ int stage_slot(const Op &op, int64_t lb, int k) {
  return (int)((ld_layout<NT>(&op.sl_lx2[lb + (int64_t)SL * (k >> 1)]) >> (16 * (k & 1))) & 0xffffu);
}

// (A x)_row for the lane's row of slice s (row = -1 on padding lanes, result 0).
// Uniform 2-ring slices hold 24 entries ordered by shell (6 at r = 1 cell, 12 at
// sqrt 2, 6 at 2) and no weights: their index loads go out before the row id.
// Uniform 56-node slices (k = 4) hold 6, 12, 8, 6 and 24 entries at r^2 = 1 .. 5
// cells and no weights: they run the general loop with the weight of entry k taken
// from the shell constants (k is wave-uniform, so the choice is scalar) and the
// level's scale applied once.
// General slices run their entry loop unrolled by 8 so that 8 index/weight loads
// and then 8 gathers are in flight together.  STG: the slice's u distinct
// neighbour values are staged in the wavefront's LDS tile first, and each entry
// reads its slot there (same values, same arithmetic, so the result is the same
// bit for bit); otherwise every entry gathers from x.
template <int MODE, bool TOP, bool STG, bool NT>
__device__ __forceinline__ double sell_apply_t(const Op &op, const double *__restrict__ x, int s,
                                               int u, int32_t &row) {
  const int lane = threadIdx.x & 63;
  const int64_t o = op.sl_off[s];
  const int64_t off = o + lane, lb = (o >> 1) + lane, hb = (o >> 2) + lane;
  double *tile = STG ? stage_tile(op) : nullptr;
  double acc;
  double xi;
  const int kind = op.sl_tmpl[s];
  if (STG && kind == 2) {
    // staged uniform 56-node slice: all 56 slots are loaded before the staging
    // gathers so that their latency overlaps; same arithmetic, in the same order,
    // as the unstaged loop below
    uint32_t wq[28];
#pragma unroll
    for (int k = 0; k < 28; k++) wq[k] = ld_layout<NT>(&op.sl_lx2[lb + (int64_t)SL * k]);
    stage_fill<NT>(tile, op.sl_uq + o, u, x);
    row = op.sl_rows[(int64_t)s * SL + lane];
    if (row < 0) return 0.0;
    xi = x[row];
    const double scale = op.t4_scaled ? ldexp(op.invL2, 2 * (int)op.rk[row]) : 1.0;
#define APC_TS(k) tile[(wq[(k) >> 1] >> (16 * ((k) & 1))) & 0xffffu]
#define APC_T4(c, k) ((k) < 6 ? c[0] : ((k) < 18 ? c[1] : ((k) < 26 ? c[2] : ((k) < 32 ? c[3] : c[4]))))
    if (MODE == V32A32) {
      float cf[5];
#pragma unroll
      for (int k = 0; k < 5; k++) cf[k] = (float)op.t4[k];
      float af = 0.f;
#pragma unroll
      for (int k = 0; k < 56; k++) af += APC_T4(cf, k) * (float)(APC_TS(k) - xi);
      acc = (double)af * scale;
    } else {
      double cd[5];
#pragma unroll
      for (int k = 0; k < 5; k++) cd[k] = MODE == V64 ? op.t4[k] : (double)(float)op.t4[k];
      double ad = 0.0;
#pragma unroll
      for (int k = 0; k < 56; k++) ad += APC_T4(cd, k) * (APC_TS(k) - xi);
      acc = ad * scale;
    }
#undef APC_T4
#undef APC_TS
  } else if (kind == 1) {
    int32_t jj[24];
    if (STG) {
      uint32_t wq[12];
#pragma unroll
      for (int k = 0; k < 12; k++) wq[k] = ld_layout<NT>(&op.sl_lx2[lb + (int64_t)SL * k]);
      stage_fill<NT>(tile, op.sl_uq + o, u, x);
#pragma unroll
      for (int k = 0; k < 24; k++) jj[k] = (int32_t)((wq[k >> 1] >> (16 * (k & 1))) & 0xffffu);
    } else {
#pragma unroll
      for (int k = 0; k < 24; k++) jj[k] = sl_col<TOP, NT>(op, lb, hb, k);
    }
    row = op.sl_rows[(int64_t)s * SL + lane];
    if (row < 0) return 0.0;
    xi = x[row];
    const double scale = ldexp(op.invL2, 2 * (int)op.rk[row]);
    if (MODE == V32A32) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
      for (int k = 0; k < 24; k++) {
        const float d = (float)((STG ? tile[jj[k]] : x[jj[k]]) - xi);
        if (k < 6) a0 += d; else if (k < 18) a1 += d; else a2 += d;
      }
      acc = (double)((float)op.tc[0] * a0 + (float)op.tc[1] * a1 + (float)op.tc[2] * a2) * scale;
    } else {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
      for (int k = 0; k < 24; k++) {
        const double d = (STG ? tile[jj[k]] : x[jj[k]]) - xi;
        if (k < 6) a0 += d; else if (k < 18) a1 += d; else a2 += d;
      }
      const double c0 = MODE == V64 ? op.tc[0] : (double)(float)op.tc[0];
      const double c1 = MODE == V64 ? op.tc[1] : (double)(float)op.tc[1];
      const double c2 = MODE == V64 ? op.tc[2] : (double)(float)op.tc[2];
      acc = (c0 * a0 + c1 * a1 + c2 * a2) * scale;
    }
  } else {
    const int len = op.sl_len[s];
    if (STG) stage_fill<NT>(tile, op.sl_uq + o, u, x);
    row = op.sl_rows[(int64_t)s * SL + lane];
    if (row < 0) return 0.0;
    xi = x[row];
#define APC_NB(k) (STG ? tile[stage_slot<NT>(op, lb, k)] : x[sl_col<TOP, NT>(op, lb, hb, k)])
#define APC_T4(c, k) ((k) < 6 ? c[0] : ((k) < 18 ? c[1] : ((k) < 26 ? c[2] : ((k) < 32 ? c[3] : c[4]))))
    if (kind == 2) {
      const double scale = op.t4_scaled ? ldexp(op.invL2, 2 * (int)op.rk[row]) : 1.0;
      if (MODE == V32A32) {
        float cf[5];
#pragma unroll
        for (int k = 0; k < 5; k++) cf[k] = (float)op.t4[k];
        float af = 0.f;
#pragma unroll 8
        for (int k = 0; k < 56; k++) af += APC_T4(cf, k) * (float)(APC_NB(k) - xi);
        acc = (double)af * scale;
      } else {
        double cd[5];
#pragma unroll
        for (int k = 0; k < 5; k++) cd[k] = MODE == V64 ? op.t4[k] : (double)(float)op.t4[k];
        double ad = 0.0;
#pragma unroll 8
        for (int k = 0; k < 56; k++) ad += APC_T4(cd, k) * (APC_NB(k) - xi);
        acc = ad * scale;
      }
    } else if (MODE == V32A32) {
      const float *__restrict__ wv = op.sl_w32 + off;
      float af = 0.f;
#pragma unroll 8
      for (int k = 0; k < len; k++) af += ld_layout<NT>(&wv[k * SL]) * (float)(APC_NB(k) - xi);
      acc = (double)af;
    } else if (MODE == V64) {
      const double *__restrict__ wv = op.sl_w64 + off;
      double ad = 0.0;
#pragma unroll 8
      for (int k = 0; k < len; k++) ad += ld_layout<NT>(&wv[k * SL]) * (APC_NB(k) - xi);
      acc = ad;
    } else {
      const float *__restrict__ wv = op.sl_w32 + off;
      double ad = 0.0;
#pragma unroll 8
      for (int k = 0; k < len; k++) ad += (double)ld_layout<NT>(&wv[k * SL]) * (APC_NB(k) - xi);
      acc = ad;
    }
#undef APC_T4
#undef APC_NB
  }
  if (op.hs) {
    const double hv = op.hs[row];
    if (hv < 0.0) {
      double e = 0.0;
      for (int32_t k = op.off[row]; k < op.off[row + 1]; k++) e += op.dwx[k] * (x[op.idx[k]] - xi);
      return xi + e;
    }
    return xi + hv * acc;
  }
  return op.unit_diag ? xi + acc : acc;
}
// Offsets (x + 8 y + APC_BOX_SZ z, in box positions) of the 56 nodes of the uniform stencil:
// r^2 = 1 .. 5 cells, each shell in the enumeration order (dx, then dy, then dz
// ascending).
struct Box56 {
  int off[56];
  constexpr Box56() : off() {
    int k = 0;
    for (int r2 = 1; r2 <= 5; r2++)
      for (int dx = -2; dx <= 2; dx++)
        for (int dy = -2; dy <= 2; dy++)
          for (int dz = -2; dz <= 2; dz++) {
            const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy, az = dz < 0 ? -dz : dz;
            if (dx * dx + dy * dy + dz * dz != r2 || ax + ay + az > 3) continue;
            off[k++] = dx + 8 * dy + APC_BOX_SZ * dz;
          }
  }
};
constexpr Box56 kBox56{};

// (A x)_row for the lane's row of a boxed slice (tk = its sl_tmpl): the lane's cell
// sits at box position b = (lx + 2) + 8 (ly + 2) + APC_BOX_SZ (lz + 2), its
// neighbour at offset q at b + q_x + 8 q_y + APC_BOX_SZ q_z.  STG: the box's x values are gathered into
// the wavefront's LDS tile first (positions without a node are skipped); otherwise
// each entry reads x through the box's node id.  Both sum the 56 entries in the
// order of kBox56 with the shell weights, then scale once (same arithmetic, so the
// same result bit for bit).
template <int MODE, bool STG, bool NT>
__device__ __forceinline__ double box_apply(const Op &op, const double *__restrict__ x, int s,
                                            int tk, int32_t &row) {
  const int lane = threadIdx.x & 63;
  const int32_t *__restrict__ bx = op.sl_box + (int64_t)(tk >> 2) * APC_BOX_N;
  const int lx = ((lane >> 2) & 1) | (((lane >> 5) & 1) << 1);
  const int ly = ((lane >> 1) & 1) | (((lane >> 4) & 1) << 1);
  const int lz = (lane & 1) | (((lane >> 3) & 1) << 1);
  const int b = (lx + 2) + 8 * (ly + 2) + APC_BOX_SZ * (lz + 2);
  double *tile = STG ? stage_tile(op) : nullptr;
  if (STG) stage_fill<NT, APC_BOX_N / SL>(tile, bx, APC_BOX_N, x); // one batch: 8 per lane
  row = op.sl_rows[(int64_t)s * SL + lane];
  const double xi = x[row];
  const double scale = op.t4_scaled ? ldexp(op.invL2, 2 * (int)op.rk[row]) : 1.0;
#define APC_BV(k) (STG ? tile[b + kBox56.off[k]] : x[bx[b + kBox56.off[k]]])
#define APC_T4(c, k) ((k) < 6 ? c[0] : ((k) < 18 ? c[1] : ((k) < 26 ? c[2] : ((k) < 32 ? c[3] : c[4]))))
  double acc;
  if (MODE == V32A32) {
    float cf[5];
#pragma unroll
    for (int k = 0; k < 5; k++) cf[k] = (float)op.t4[k];
    float af = 0.f;
#pragma unroll 8
    for (int k = 0; k < 56; k++) af += APC_T4(cf, k) * (float)(APC_BV(k) - xi);
    acc = (double)af * scale;
  } else {
    double cd[5];
#pragma unroll
    for (int k = 0; k < 5; k++) cd[k] = MODE == V64 ? op.t4[k] : (double)(float)op.t4[k];
    double ad = 0.0;
#pragma unroll 8
    for (int k = 0; k < 56; k++) ad += APC_T4(cd, k) * (APC_BV(k) - xi);
    acc = ad * scale;
  }
#undef APC_T4
#undef APC_BV
  return op.unit_diag ? xi + acc : acc;
}

template <int MODE, bool NT>
__device__ __forceinline__ double sell_apply_nt(const Op &op, const double *__restrict__ x, int s,
                                                int32_t &row) {
  const int tk = op.sl_tmpl[s];
  double v;
  if ((tk & 3) == 3) {
    v = (op.sl_un && op.ucap >= APC_BOX_N) ? box_apply<MODE, true, NT>(op, x, s, tk, row)
                                          : box_apply<MODE, false, NT>(op, x, s, tk, row);
  } else {
    const int u = op.sl_un ? op.sl_un[s] : 0;
    if (u > 0)
      v = sell_apply_t<MODE, false, true, NT>(op, x, s, u, row);
    else
      v = op.sl_top4 ? sell_apply_t<MODE, true, false, NT>(op, x, s, 0, row)
                     : sell_apply_t<MODE, false, false, NT>(op, x, s, 0, row);
  }
  if (op.pin && row == 0) v = x[0];
  return v;
}

// Kernels that call this are launched with op_lds(op) bytes of dynamic LDS.
template <int MODE>
__device__ __forceinline__ double sell_apply(const Op &op, const double *__restrict__ x, int s_in,
                                             int32_t &row) {
  const int s = __builtin_amdgcn_readfirstlane(s_in);
  return op.nt ? sell_apply_nt<MODE, true>(op, x, s, row) : sell_apply_nt<MODE, false>(op, x, s, row);
}

static inline Op make_op(const apc_cloud *c, bool density) {
  Op op;
  op.off = c->st_off;
  op.idx = c->st_idx;
  const bool b4 = density && c->P.order == 4;
  op.w64 = b4 ? c->bw64 : c->w64;
  op.w32 = b4 ? c->bw32 : c->w32;
  op.hs = (density && !b4) ? c->hscale : nullptr;
  op.dwx = (density && !b4) ? c->dwx : nullptr;
  op.unit_diag = b4 ? 1 : 0;
  op.rk = c->P.order == 4 ? c->rkind4 : c->rkind;
  for (int k = 0; k < 3; k++) op.tc[k] = c->tmpl[k];
  for (int k = 0; k < 5; k++) op.t4[k] = b4 ? c->tmpl4[5 + k] : c->tmpl4[k];
  op.t4_scaled = b4 ? 0 : 1;
  op.pin = 0; // set by the periodic Poisson solve
  op.invL2 = 1.0 / (c->P.L * c->P.L);
  op.n = c->n;
  op.sl_rows = c->sl_rows;
  op.sl_len = c->sl_len;
  op.sl_lo2 = c->sl_lo2;
  op.sl_hi4 = c->sl_hi4;
  op.sl_top4 = c->sl_top4;
  op.sl_tmpl = c->sl_tmpl;
  op.sl_off = c->sl_off;
  op.sl_w64 = b4 ? c->sl_bw64 : c->sl_w64;
  op.sl_w32 = b4 ? c->sl_bw32 : c->sl_w32;
  op.ucap = c->ucap;
  op.sl_un = c->ucap > 0 ? c->sl_un : nullptr;
  op.sl_uq = c->sl_uq;
  op.sl_lx2 = c->sl_lx2;
  op.sl_box = c->sl_box;
  // non-temporal layout loads past 64M stored entries (about 0.5 GB of layout)
  op.nt = c->sl_entries > ((int64_t)64 << 20) ? 1 : 0;
  for (int k = 0; k < 9; k++) op.cs[k] = c->sl_cs[k];
  return op;
}

} // namespace

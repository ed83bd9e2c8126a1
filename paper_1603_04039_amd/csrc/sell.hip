// Sliced-ELL layout of the assembled operator for the solver's SpMV.
//
// Rows are cut into 8 contiguous chunks (one per XCD; the XCDs' L2s then each
// hold the x-vector neighbourhood of one chunk).  Inside a chunk the uniform rows
// (the 2-ring rows of k = 2, the 56-node rows of k = 4) and the general rows each
// form slices of 64 rows (one wavefront, one thread per row) in ascending row
// order.  A slice stores its column indices
// entry-major (entry k of lane r at off + 64 k + r), so every index/weight load
// of a wavefront is one contiguous 256-byte (or 512-byte) request and every lane
// has all its neighbour gathers independent of each other.  Uniform slices have
// exactly 24 entries (k = 2) or 56 (k = 4) and the SpMV reads no weights for them
// (the weights are the shell constants); general slices are padded to their
// longest row with (own index, weight 0).
// This file builds the layout and the column indices at build time; the weights
// are written by the assembly (k_fit_sell for k = 2, k_sell_copy for k = 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "apc_internal.h"

namespace {

constexpr int SL = APC_SLICE;

// row classes of the layout: 0 boxed (a row of a complete 4 x 4 x 4 block of
// uniform 56-node rows, k = 4), 1 uniform (the other uniform rows), 2 general
__global__ void __launch_bounds__(APC_BLOCK)
    k_cflag(const int8_t *__restrict__ rk, const int8_t *__restrict__ inblk, int64_t n,
            int32_t *__restrict__ f0, int32_t *__restrict__ f1) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const bool b = inblk && inblk[i];
  f0[i] = b ? 1 : 0;
  f1[i] = (!b && rk[i] >= 0) ? 1 : 0;
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_split(const int32_t *__restrict__ f0, const int32_t *__restrict__ f1,
            const int32_t *__restrict__ p0, const int32_t *__restrict__ p1, int64_t n,
            int32_t *__restrict__ srow_b, int32_t *__restrict__ srow_t,
            int32_t *__restrict__ srow_g) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  if (f0[i])
    srow_b[p0[i]] = (int32_t)i;
  else if (f1[i])
    srow_t[p1[i]] = (int32_t)i;
  else
    srow_g[i - p0[i] - p1[i]] = (int32_t)i;
}

// Complete blocks (k = 4): 64 consecutive rows that are the 4 x 4 x 4 cells of one
// Morton-aligned block of their level, all uniform 56-node rows, inside one XCD
// chunk.  Pass 1 (one thread per row) flags the rows whose cell starts such a
// block; pass 2 marks the block's rows.  cell = leaf code >> 3 (D - level): the
// cell's Morton index at its own level.
struct Chunks {
  int64_t lo[9];
};
__global__ void __launch_bounds__(APC_BLOCK)
    k_block_start(int64_t n, const uint64_t *__restrict__ code, const int32_t *__restrict__ level,
                  const int8_t *__restrict__ rk4, int D, Chunks C, int8_t *__restrict__ bst) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int l = level[y];
  const uint64_t cell = code[y] >> (3 * (D - l));
  bool ok = rk4[y] >= 0 && (cell & 63u) == 0 && y + 64 <= n;
  if (ok) {
    int c = 0;
    while (c < 7 && y >= C.lo[c + 1]) c++;
    ok = y + 64 <= C.lo[c + 1];
  }
  for (int j = 1; j < 64 && ok; j++)
    ok = rk4[y + j] >= 0 && level[y + j] == l && (code[y + j] >> (3 * (D - l))) == cell + j;
  bst[y] = ok ? 1 : 0;
}
__global__ void __launch_bounds__(APC_BLOCK)
    k_block_rows(int64_t n, const uint64_t *__restrict__ code, const int32_t *__restrict__ level,
                 const int8_t *__restrict__ bst, int D, int8_t *__restrict__ inblk) {
  const int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int k = (int)((code[y] >> (3 * (D - level[y]))) & 63u);
  inblk[y] = (y - k >= 0 && bst[y - k]) ? 1 : 0;
}

// The 8 x 8 x 8 box of a block (one wavefront per boxed slice, lane = row of the
// block, whose cell has local coordinates (lx, ly, lz) from the 6 Morton bits of
// the lane): every stencil node of every row at box position
// (lx + 2 + q_x) + 8 (ly + 2 + q_y) + APC_BOX_SZ (lz + 2 + q_z), q its lattice
// offset in spacings, and the row itself at q = 0 (rows of one block write the
// same node to a shared position).  Positions no stencil reaches keep -1.
__global__ void __launch_bounds__(SL)
    k_box_fill(const int32_t *__restrict__ sl_tmpl, const int32_t *__restrict__ sl_rows,
               const int32_t *__restrict__ st_off, const int32_t *__restrict__ st_idx,
               const int32_t *__restrict__ crd, int64_t ntot, const int32_t *__restrict__ level,
               int D, int32_t *__restrict__ box) {
  const int64_t s = blockIdx.x;
  const int tk = sl_tmpl[s];
  if ((tk & 3) != 3) return;
  const int lane = threadIdx.x;
  const int32_t row = sl_rows[s * SL + lane];
  int32_t *bx = box + (int64_t)(tk >> 2) * APC_BOX_N;
  const int lx = ((lane >> 2) & 1) | (((lane >> 5) & 1) << 1);
  const int ly = ((lane >> 1) & 1) | (((lane >> 4) & 1) << 1);
  const int lz = (lane & 1) | (((lane >> 3) & 1) << 1);
  const int sh = D - level[row] + 1;
  const int32_t c0 = crd[row], c1 = crd[ntot + row], c2 = crd[2 * ntot + row], S = crd[3 * ntot];
  const int32_t a = st_off[row];
  bx[(lx + 2) + 8 * (ly + 2) + APC_BOX_SZ * (lz + 2)] = row;
  for (int j = 0; j < 56; j++) {
    const int32_t v = st_idx[a + j];
    const int qx = apc_doff(crd[v], c0, S) >> sh, qy = apc_doff(crd[ntot + v], c1, S) >> sh,
              qz = apc_doff(crd[2 * ntot + v], c2, S) >> sh;
    bx[(lx + 2 + qx) + 8 * (ly + 2 + qy) + APC_BOX_SZ * (lz + 2 + qz)] = v;
  }
}

// slice groups g = 3 * chunk + (0 boxed, 1 uniform, 2 general)
constexpr int NGRP = 24;
struct Groups {
  int64_t sl0[NGRP], nsl[NGRP], r0[NGRP], nr[NGRP];
};

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// SELL-C-sigma: the general rows of each chunk are sorted by descending stencil
// length (stably) within windows of APC_SELL_SIGMA consecutive rows, so that the
// 64 rows of a slice have nearly equal lengths and padding stays small, while a
// window keeps the Morton locality of its rows.  Key: chunk (3 bits) | window |
// 255 - m (8 bits); the radix sort permutes srow_g in place.
__global__ void __launch_bounds__(APC_BLOCK)
    k_sigma_keys(Groups G, const int32_t *__restrict__ srow_g, const int32_t *__restrict__ st_off,
                 int64_t ng, uint64_t *__restrict__ key) {
  const int64_t q = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (q >= ng) return;
  int c = 7;
  while (c > 0 && q < G.r0[3 * c + 2]) c--;
  const int64_t win = (q - G.r0[3 * c + 2]) / APC_SELL_SIGMA;
  const int32_t row = srow_g[q];
  const int m = min(st_off[row + 1] - st_off[row], 255);
  key[q] = ((uint64_t)c << 33) | ((uint64_t)win << 8) | (uint64_t)(255 - m);
}

// one 64-thread block per slice
__global__ void __launch_bounds__(SL)
    k_slices(Groups G, int tkind, const int32_t *__restrict__ srow_b,
             const int32_t *__restrict__ srow_t, const int32_t *__restrict__ srow_g,
             const int32_t *__restrict__ st_off, int32_t *__restrict__ sl_rows,
             int32_t *__restrict__ sl_len, int32_t *__restrict__ sl_tmpl,
             int64_t *__restrict__ sl_ent) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  int g = 0;
  while (g < NGRP - 1 && !(s >= G.sl0[g] && s < G.sl0[g] + G.nsl[g])) g++;
  const int type = g % 3;
  const int64_t k = s - G.sl0[g];
  const int64_t q = k * SL + lane;
  const bool valid = q < G.nr[g];
  const int32_t *src = type == 0 ? srow_b : (type == 1 ? srow_t : srow_g);
  const int32_t row = valid ? src[G.r0[g] + q] : -1;
  sl_rows[s * SL + lane] = row;
  const int m = valid ? st_off[row + 1] - st_off[row] : 0;
  const int len = type == 2 ? wave_max_i(m) : (tkind == 1 ? 24 : 56);
  if (lane == 0) {
    sl_len[s] = len;
    // boxed slice: kind 3 and, above it, the box number (blocks numbered in row order)
    sl_tmpl[s] = type == 0 ? (int32_t)(3 | ((G.r0[g] / SL + k) << 2)) : (type == 1 ? tkind : 0);
    sl_ent[s] = (int64_t)((len + 3) & ~3) * SL; // storage padded to a multiple of 4 entries
  }
}

// column indices of every slice (structure only), storage padding included;
// weights start at 0 so that padding entries contribute nothing
__global__ void __launch_bounds__(SL)
    k_sell_idx(const int32_t *__restrict__ sl_rows, const int32_t *__restrict__ sl_len,
               const int64_t *__restrict__ sl_off, const int32_t *__restrict__ st_off,
               const int32_t *__restrict__ st_idx, int32_t *__restrict__ idx) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t row = sl_rows[s * SL + lane];
  const int len = sl_len[s];
  const int64_t off = sl_off[s] + lane;
  const int32_t a = row >= 0 ? st_off[row] : 0;
  const int m = row >= 0 ? st_off[row + 1] - a : 0;
  const int len4 = (len + 3) & ~3;
  for (int k = 0; k < len4; k++) idx[off + (int64_t)k * SL] = k < m ? st_idx[a + k] : (row >= 0 ? row : 0);
}

// the compact copy of the column indices (layout in apc_cloud::sl_lo2)
__global__ void __launch_bounds__(SL)
    k_pack_idx(const int32_t *__restrict__ sl_len, const int64_t *__restrict__ sl_off,
               const int32_t *__restrict__ idx, uint32_t *__restrict__ lo2,
               uint32_t *__restrict__ hi4, uint32_t *__restrict__ top4) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const int len4 = (sl_len[s] + 3) & ~3;
  const int64_t o = sl_off[s];
  for (int k = 0; k < len4; k += 4) {
    uint32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = (uint32_t)idx[o + (int64_t)(k + q) * SL + lane];
    lo2[o / 2 + (int64_t)SL * (k / 2) + lane] = (v[0] & 0xffffu) | (v[1] << 16);
    lo2[o / 2 + (int64_t)SL * (k / 2 + 1) + lane] = (v[2] & 0xffffu) | (v[3] << 16);
    uint32_t h = 0, t = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      h |= ((v[q] >> 16) & 0xffu) << (8 * q);
      t |= (v[q] >> 24) << (8 * q);
    }
    hi4[o / 4 + (int64_t)SL * (k / 4) + lane] = h;
    if (top4) top4[o / 4 + (int64_t)SL * (k / 4) + lane] = t;
  }
}

// Distinct neighbour columns of one slice (one 256-thread block per slice, at most
// 4096 entries: k < len on lanes with a row): the entries' columns go into an LDS
// hash set (each new column appended to a list), only the distinct columns are
// sorted (bitonic), and every entry finds its slot by binary search in the sorted
// list.  Entries of padding rows keep slot 0.  Writes the count (un), the columns
// in ascending order at the slice's entry offset (uq) and the 16-bit slots (lx2, as
// uint16: entry k of lane r at 2 (o/2 + 64 (k/2) + r) + k%2).
constexpr int UQ_T = 256, UQ_MAX = 4096, UQ_HASH = 8192; // hash at most half full
__global__ void __launch_bounds__(UQ_T)
    k_uniq(const int32_t *__restrict__ sl_rows, const int32_t *__restrict__ sl_len,
           const int64_t *__restrict__ sl_off, const int32_t *__restrict__ idx,
           int32_t *__restrict__ un, int32_t *__restrict__ uq, uint16_t *__restrict__ lx) {
  __shared__ int32_t hk[UQ_HASH];
  __shared__ int32_t lst[UQ_MAX];
  __shared__ int32_t nd;
  const int64_t s = blockIdx.x;
  const int t = threadIdx.x;
  const int len = sl_len[s];
  const int ne = len * SL;
  if (ne > UQ_MAX || ne <= 0) {
    if (t == 0) un[s] = 0;
    return;
  }
  const int64_t o = sl_off[s];
  for (int k = t; k < UQ_HASH; k += UQ_T) hk[k] = -1;
  if (t == 0) nd = 0;
  __syncthreads();
  for (int e = t; e < ne; e += UQ_T) {
    if (sl_rows[s * SL + (e & (SL - 1))] < 0) continue;
    const int32_t col = idx[o + e];
    uint32_t h = ((uint32_t)col * 2654435761u) & (UQ_HASH - 1);
    for (;;) {
      const int32_t old = atomicCAS(&hk[h], -1, col);
      if (old == -1) {
        lst[atomicAdd(&nd, 1)] = col;
        break;
      }
      if (old == col) break;
      h = (h + 1) & (UQ_HASH - 1);
    }
  }
  __syncthreads();
  const int n_d = nd;
  int np = 1;
  while (np < n_d) np <<= 1;
  for (int k = n_d + t; k < np; k += UQ_T) lst[k] = 0x7fffffff;
  __syncthreads();
  for (int kk = 2; kk <= np; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int e = t; e < np; e += UQ_T) {
        const int q = e ^ j;
        if (q > e) {
          const int32_t a = lst[e], b = lst[q];
          if ((a > b) == ((e & kk) == 0)) {
            lst[e] = b;
            lst[q] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int r = t; r < n_d; r += UQ_T) uq[o + r] = lst[r];
  for (int e = t; e < ne; e += UQ_T) {
    if (sl_rows[s * SL + (e & (SL - 1))] < 0) continue;
    const int32_t col = idx[o + e];
    int lo = 0, hi = n_d; // first position with lst[pos] >= col
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (lst[mid] < col) lo = mid + 1;
      else hi = mid;
    }
    const int k = e >> 6, lane = e & (SL - 1);
    lx[2 * ((o >> 1) + (int64_t)SL * (k >> 1) + lane) + (k & 1)] = (uint16_t)lo;
  }
  if (t == 0) un[s] = n_d;
}

// slices with more distinct columns than the tile holds gather directly
__global__ void __launch_bounds__(APC_BLOCK) k_cap_un(int32_t *un, int64_t ns, int cap) {
  const int64_t s = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (s < ns && un[s] > cap) un[s] = 0;
}

} // namespace

int apc_build_sell(apc_cloud *c, hipStream_t s) {
  const int64_t n = c->n;
  int32_t *f0 = nullptr, *f1 = nullptr, *p0 = nullptr, *p1 = nullptr;
  int32_t *srow_b = nullptr, *srow_t = nullptr, *srow_g = nullptr;
  int8_t *bst = nullptr, *inblk = nullptr;
  const size_t n1 = (size_t)(n > 0 ? n : 1);
  for (int32_t **q : {&f0, &f1, &p0, &p1, &srow_b, &srow_t, &srow_g})
    HIPCHK(apc_malloc_async((void **)q, n1 * sizeof(int32_t), s));
  // uniform rows: the 2-ring rows of k = 2 or the 56-node rows of k = 4
  const int8_t *rk = c->P.order == 4 ? c->rkind4 : c->rkind;
  const int tkind = c->P.order == 4 ? 2 : 1;
  int64_t lo[9];
  for (int k = 0; k <= 8; k++) lo[k] = (int64_t)k * n / 8;
  if (c->P.order == 4 && n > 0) {
    // complete 4 x 4 x 4 blocks of uniform rows (boxed slices)
    HIPCHK(apc_malloc_async((void **)&bst, n1, s));
    HIPCHK(apc_malloc_async((void **)&inblk, n1, s));
    Chunks C;
    for (int k = 0; k <= 8; k++) C.lo[k] = lo[k];
    hipLaunchKernelGGL(k_block_start, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, n, c->code,
                       c->level, rk, c->P.max_depth, C, bst);
    hipLaunchKernelGGL(k_block_rows, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, n, c->code,
                       c->level, (const int8_t *)bst, c->P.max_depth, inblk);
    HIPCHK(hipGetLastError());
  }
  int32_t B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, T[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (n > 0) {
    hipLaunchKernelGGL(k_cflag, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, rk,
                       (const int8_t *)inblk, n, f0, f1);
    APCCHK(apc_scan_i32(f0, p0, n, s));
    APCCHK(apc_scan_i32(f1, p1, n, s));
    hipLaunchKernelGGL(k_split, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, (const int32_t *)f0,
                       (const int32_t *)f1, (const int32_t *)p0, (const int32_t *)p1, n, srow_b,
                       srow_t, srow_g);
    HIPCHK(hipGetLastError());
    // class prefix counts at the 8 chunk boundaries
    for (int k = 0; k < 8; k++) {
      HIPCHK(hipMemcpyAsync(&B[k], p0 + lo[k], sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(&T[k], p1 + lo[k], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    int32_t lf[2] = {0, 0}, lp[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&lf[0], f0 + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&lf[1], f1 + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&lp[0], p0 + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&lp[1], p1 + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    B[8] = lp[0] + lf[0];
    T[8] = lp[1] + lf[1];
  }
  c->n_template = tkind == 1 ? T[8] : 0;
  c->n_boxes = B[8] / SL;
  Groups G;
  int64_t ns = 0;
  for (int k = 0; k < 8; k++) {
    const int64_t nb = B[k + 1] - B[k], nt = T[k + 1] - T[k];
    const int64_t g0 = lo[k] - B[k] - T[k];
    const int64_t ng = (lo[k + 1] - B[k + 1] - T[k + 1]) - g0;
    const int64_t nr[3] = {nb, nt, ng}, r0[3] = {B[k], T[k], g0};
    c->sl_cs[k] = ns;
    for (int t = 0; t < 3; t++) {
      G.sl0[3 * k + t] = ns;
      G.nsl[3 * k + t] = (nr[t] + SL - 1) / SL;
      G.r0[3 * k + t] = r0[t];
      G.nr[3 * k + t] = nr[t];
      ns += G.nsl[3 * k + t];
    }
  }
  c->sl_cs[8] = ns;
  c->nsl = ns;
  const int64_t ng = n - B[8] - T[8];
  if (APC_SELL_SIGMA > SL && ng > 1) {
    uint64_t *key = nullptr;
    HIPCHK(apc_malloc_async((void **)&key, (size_t)ng * sizeof(uint64_t), s));
    hipLaunchKernelGGL(k_sigma_keys, dim3(grid_for(ng)), dim3(APC_BLOCK), 0, s, G, srow_g, c->st_off,
                       ng, key);
    HIPCHK(hipGetLastError());
    APCCHK(apc_radix_sort(key, srow_g, ng, 36, s));
    HIPCHK(apc_free_async(key, s));
  }
  const size_t nsz = (size_t)(ns > 0 ? ns : 1);
  HIPCHK(apc_dev_alloc((void **)&c->sl_rows, nsz * SL * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->sl_len, nsz * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->sl_tmpl, nsz * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->sl_off, nsz * sizeof(int64_t)));
  int64_t *ent = nullptr;
  HIPCHK(apc_malloc_async((void **)&ent, nsz * sizeof(int64_t), s));
  if (ns > 0) {
    hipLaunchKernelGGL(k_slices, dim3((unsigned)ns), dim3(SL), 0, s, G, tkind, srow_b, srow_t,
                       srow_g, c->st_off, c->sl_rows, c->sl_len, c->sl_tmpl, ent);
    HIPCHK(hipGetLastError());
    APCCHK(apc_scan_i64(ent, c->sl_off, ns, s));
    int64_t lasto = 0, laste = 0;
    HIPCHK(hipMemcpyAsync(&lasto, c->sl_off + ns - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&laste, ent + ns - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    c->sl_entries = lasto + laste;
  }
  const size_t ne = (size_t)(c->sl_entries > 0 ? c->sl_entries : 1);
  HIPCHK(apc_dev_alloc((void **)&c->sl_idx, ne * sizeof(int32_t)));
  if (c->P.precision == APC_FP64)
    HIPCHK(apc_dev_alloc((void **)&c->sl_w64, ne * sizeof(double)));
  else
    HIPCHK(apc_dev_alloc((void **)&c->sl_w32, ne * sizeof(float)));
  if (ns > 0) {
    hipLaunchKernelGGL(k_sell_idx, dim3((unsigned)ns), dim3(SL), 0, s, c->sl_rows, c->sl_len,
                       c->sl_off, c->st_off, c->st_idx, c->sl_idx);
    HIPCHK(hipGetLastError());
  }
  if (c->sl_w64) HIPCHK(hipMemsetAsync(c->sl_w64, 0, ne * sizeof(double), s));
  if (c->sl_w32) HIPCHK(hipMemsetAsync(c->sl_w32, 0, ne * sizeof(float), s));
  APCCHK(apc_pack_sell_idx(c, s));
  // boxes of the boxed slices
  if (c->n_boxes > 0) {
    const size_t nbx = (size_t)c->n_boxes * APC_BOX_N;
    HIPCHK(apc_dev_alloc((void **)&c->sl_box, nbx * sizeof(int32_t)));
    HIPCHK(hipMemsetAsync(c->sl_box, 0xff, nbx * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_box_fill, dim3((unsigned)ns), dim3(SL), 0, s, (const int32_t *)c->sl_tmpl,
                       (const int32_t *)c->sl_rows, c->st_off, c->st_idx, c->crd, c->n + c->nb,
                       c->level, c->P.max_depth, c->sl_box);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(apc_free_async(ent, s));
  for (void *q : {(void *)f0, (void *)f1, (void *)p0, (void *)p1, (void *)srow_b, (void *)srow_t,
                  (void *)srow_g, (void *)bst, (void *)inblk})
    if (q) HIPCHK(apc_free_async(q, s));
  return APC_OK;
}

// Neighbour staging (layout in apc_cloud::sl_un): the distinct columns of every
// slice, then the tile size ucap = the largest count (at least a box when there
// are boxed slices), rounded up to 16 and capped at the cloud's stage_cap (0:
// APC_UCAP_DEFAULT; APC_UCAP_MAX at most); slices above the cap keep the direct
// gathers, boxed slices read through their box when the tile cannot hold it.
static int build_staging(apc_cloud *c, hipStream_t s) {
  const size_t ne = (size_t)(c->sl_entries > 0 ? c->sl_entries : 4);
  const size_t nsz = (size_t)(c->nsl > 0 ? c->nsl : 1);
  const int cap = c->P.stage_cap == 0 ? APC_UCAP_DEFAULT : std::min(c->P.stage_cap, APC_UCAP_MAX);
  c->ucap = 0;
  if (cap <= 0) return APC_OK;
  HIPCHK(apc_dev_alloc((void **)&c->sl_un, nsz * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->sl_uq, ne * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->sl_lx2, ne / 2 * sizeof(uint32_t)));
  HIPCHK(hipMemsetAsync(c->sl_lx2, 0, ne / 2 * sizeof(uint32_t), s));
  if (c->nsl <= 0) return APC_OK;
  hipLaunchKernelGGL(k_uniq, dim3((unsigned)c->nsl), dim3(UQ_T), 0, s, c->sl_rows, c->sl_len,
                     c->sl_off, c->sl_idx, c->sl_un, c->sl_uq, (uint16_t *)c->sl_lx2);
  HIPCHK(hipGetLastError());
  std::vector<int32_t> un((size_t)c->nsl);
  HIPCHK(hipMemcpyAsync(un.data(), c->sl_un, un.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int mx = 0;
  for (int32_t v : un) mx = v > mx ? v : mx;
  if (c->n_boxes > 0) mx = std::max(mx, APC_BOX_N); // a boxed slice stages its box
  c->ucap = std::min((mx + 15) & ~15, cap);
  hipLaunchKernelGGL(k_cap_un, dim3(grid_for(c->nsl)), dim3(APC_BLOCK), 0, s, c->sl_un, c->nsl,
                     c->ucap);
  HIPCHK(hipGetLastError());
  return APC_OK;
}

int apc_pack_sell_idx(apc_cloud *c, hipStream_t s) {
  const size_t ne = (size_t)(c->sl_entries > 0 ? c->sl_entries : 4);
  void *old[] = {c->sl_lo2, c->sl_hi4, c->sl_top4, c->sl_un, c->sl_uq, c->sl_lx2};
  bool any = false;
  for (void *q : old) any = any || q;
  if (any) HIPCHK(hipDeviceSynchronize()); // queued work may still read the old arrays
  for (void *q : old)
    if (q) HIPCHK(apc_dev_free(q));
  c->sl_lo2 = c->sl_hi4 = c->sl_top4 = c->sl_lx2 = nullptr;
  c->sl_un = c->sl_uq = nullptr;
  HIPCHK(apc_dev_alloc((void **)&c->sl_lo2, ne / 2 * sizeof(uint32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->sl_hi4, ne / 4 * sizeof(uint32_t)));
  if (c->n + c->nb >= ((int64_t)1 << 24))
    HIPCHK(apc_dev_alloc((void **)&c->sl_top4, ne / 4 * sizeof(uint32_t)));
  if (c->nsl > 0) {
    hipLaunchKernelGGL(k_pack_idx, dim3((unsigned)c->nsl), dim3(SL), 0, s, c->sl_len, c->sl_off,
                       c->sl_idx, c->sl_lo2, c->sl_hi4, c->sl_top4);
    HIPCHK(hipGetLastError());
  }
  return build_staging(c, s);
}

void apc_free_sell(apc_cloud *c) {
  void *ptrs[] = {c->sl_rows, c->sl_len, c->sl_tmpl, c->sl_off, c->sl_idx, c->sl_w64, c->sl_w32,
                  c->sl_lo2, c->sl_hi4, c->sl_top4, c->sl_un, c->sl_uq, c->sl_lx2, c->sl_box};
  for (void *q : ptrs)
    if (q) (void)apc_dev_free(q);
  c->sl_lo2 = c->sl_hi4 = c->sl_top4 = c->sl_lx2 = nullptr;
  c->sl_un = c->sl_uq = nullptr;
  c->ucap = 0;
  c->sl_rows = c->sl_len = c->sl_idx = c->sl_tmpl = c->sl_box = nullptr;
  c->n_boxes = 0;
  c->sl_off = nullptr;
  c->sl_w64 = nullptr;
  c->sl_w32 = nullptr;
}

// Node-cloud build on the GPU (Sec. 4): Morton keys, stable radix sort, the
// error-balance criterion expanded level by level, 2:1 face balance to its
// unique minimal fixed point, boundary face nodes, face adjacency (1-ring) and
// per-node k-ring stencil choice.  All geometry is integer, so the result is
// independent of evaluation order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "apc_internal.h"

namespace {

struct Thr {
  double T[24];
};

// Irregular domain: the state of every cell of levels 0 .. ml in Morton order
// (level l at off[l] + its key prefix): 0 inside Omega, 1 excluded, 2 mixed.
// ml = 0: no mask, every cell inside.
struct Mask {
  const uint8_t *pyr;
  int ml;
  int64_t off[8];
};
__device__ __forceinline__ int mask_state(const Mask &M, uint64_t pre, int l) {
  if (M.ml <= 0) return 0;
  if (l > M.ml) {
    pre >>= 3 * (l - M.ml);
    l = M.ml;
  }
  return M.pyr[M.off[l] + (int64_t)pre];
}

// ---------------------------------------------------------------- keys
__global__ void __launch_bounds__(APC_BLOCK)
    k_keys(const double *__restrict__ xyz, int64_t N, double lo0, double lo1, double lo2, double L,
           double s, int D, Mask M, uint64_t *__restrict__ keys, int32_t *__restrict__ vals,
           int *__restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= N) return;
  const double lo[3] = {lo0, lo1, lo2};
  const uint32_t top = (1u << D) - 1u;
  uint32_t u[3];
  int e = 0;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const double x = xyz[(int64_t)d * N + i];
    if (isnan(x)) e |= 1;
    if (x < lo[d] || x > lo[d] + L) e |= 2;
    double q = floor((x - lo[d]) * s);
    if (!(q >= 0.0)) q = 0.0;
    if (q > (double)top) q = (double)top;
    u[d] = (uint32_t)q;
  }
  const uint64_t k = apc_morton(u[0], u[1], u[2]);
  if (mask_state(M, k, D) == 1) e |= 2; // in an excluded cell: outside Omega
  if (e) atomicOr(err, e);
  keys[i] = k;
  vals[i] = (int32_t)i;
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_gather_xyz(const double *__restrict__ xyz, const int32_t *__restrict__ perm, int64_t N,
                 double *__restrict__ sxyz) {
  int64_t s = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (s >= N) return;
  const int64_t i = perm[s];
  sxyz[s] = xyz[i];
  sxyz[N + s] = xyz[N + i];
  sxyz[2 * N + s] = xyz[2 * N + i];
}

// ---------------------------------------------------------------- cell lists
struct Cells {
  uint64_t *pre = nullptr; // key prefix at the cell's own level
  int32_t *lev = nullptr, *fst = nullptr, *cnt = nullptr, *flag = nullptr;
  int64_t n = 0;
};

int cells_alloc(Cells &c, int64_t n, hipStream_t s) {
  c.n = n;
  size_t m = (size_t)(n > 0 ? n : 1);
  HIPCHK(apc_malloc_async((void **)&c.pre, m * sizeof(uint64_t), s));
  HIPCHK(apc_malloc_async((void **)&c.lev, m * sizeof(int32_t), s));
  HIPCHK(apc_malloc_async((void **)&c.fst, m * sizeof(int32_t), s));
  HIPCHK(apc_malloc_async((void **)&c.cnt, m * sizeof(int32_t), s));
  HIPCHK(apc_malloc_async((void **)&c.flag, m * sizeof(int32_t), s));
  return APC_OK;
}
int cells_free(Cells &c, hipStream_t s) {
  if (c.pre) HIPCHK(apc_free_async(c.pre, s));
  if (c.lev) HIPCHK(apc_free_async(c.lev, s));
  if (c.fst) HIPCHK(apc_free_async(c.fst, s));
  if (c.cnt) HIPCHK(apc_free_async(c.cnt, s));
  if (c.flag) HIPCHK(apc_free_async(c.flag, s));
  c = Cells();
  return APC_OK;
}

__global__ void __launch_bounds__(APC_BLOCK) k_sizes(const int32_t *flag, int64_t n, int32_t *sz) {
  int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) sz[i] = flag[i] ? 8 : 1;
}

// Replace every flagged cell by its 8 children (Morton child order keeps the list
// sorted); each child's particle range is the sub-range of its parent carrying the
// child's key prefix.  With `criterion`, a child is flagged for the next pass when
// it lies above max_depth and holds N' >= T_l particles; on an irregular domain
// excluded children never, other children of a level below the mask's always.
__global__ void __launch_bounds__(APC_BLOCK)
    k_expand(const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev,
             const int32_t *__restrict__ fst, const int32_t *__restrict__ cnt,
             const int32_t *__restrict__ flag, const int32_t *__restrict__ off, int64_t n,
             const uint64_t *__restrict__ keys, int D, Thr thr, Mask M, int criterion,
             uint64_t *__restrict__ opre, int32_t *__restrict__ olev, int32_t *__restrict__ ofst,
             int32_t *__restrict__ ocnt, int32_t *__restrict__ oflag) {
  int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int64_t o = off[i];
  if (!flag[i]) {
    opre[o] = pre[i];
    olev[o] = lev[i];
    ofst[o] = fst[i];
    ocnt[o] = cnt[i];
    oflag[o] = 0;
    return;
  }
  const int l = lev[i] + 1;
  const int sh = 3 * (D - l);
  const int64_t a0 = fst[i], a1 = (int64_t)fst[i] + cnt[i];
  int64_t a = a0;
  for (int c = 0; c < 8; c++) {
    const uint64_t cp = pre[i] * 8ull + (uint64_t)c;
    const int64_t b = apc_lower_bound(keys, a, a1, (cp + 1ull) << sh);
    const int32_t k = (int32_t)(b - a);
    opre[o + c] = cp;
    olev[o + c] = l;
    ofst[o + c] = (int32_t)a;
    ocnt[o + c] = k;
    oflag[o + c] = criterion ? (l < D && mask_state(M, cp, l) != 1 &&
                                (l < M.ml || (double)k >= thr.T[l]))
                             : 0;
    a = b;
  }
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_mincorner(const uint64_t *pre, const int32_t *lev, int64_t n, int D, uint64_t *mc) {
  int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) mc[i] = pre[i] << (3 * (D - lev[i]));
}

__device__ inline void cell_index(uint64_t pre, uint32_t t[3]) {
  t[0] = apc_compact3(pre >> 2);
  t[1] = apc_compact3(pre >> 1);
  t[2] = apc_compact3(pre);
}

// 2:1 face balance: a leaf at level l marks every face-neighbouring leaf coarser
// than l - 1.  The neighbour across a face is the leaf containing the minimum
// corner of the same-level cell across it.
__global__ void __launch_bounds__(APC_BLOCK)
    k_balance_mark(const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev,
                   const uint64_t *__restrict__ mc, int64_t n, int D, int periodic, Mask M,
                   int32_t *__restrict__ mark) {
  int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int l = lev[y];
  if (l < 2) return;
  if (mask_state(M, pre[y], l) == 1) return; // excluded leaves are not nodes
  uint32_t t0[3];
  cell_index(pre[y], t0);
  const int sh = D - l;
  for (int f = 0; f < 6; f++) {
    const int d = f >> 1;
    uint32_t t[3] = {t0[0], t0[1], t0[2]};
    const uint32_t side = 1u << l;
    if (f & 1) {
      if (t[d] + 1u >= side && !periodic) continue;
      t[d] = (t[d] + 1u) & (side - 1u); // periodic: the face across the domain boundary
    } else {
      if (t[d] == 0u && !periodic) continue;
      t[d] = (t[d] + side - 1u) & (side - 1u);
    }
    if (mask_state(M, apc_morton(t[0], t[1], t[2]), l) == 1) continue; // a wall
    const uint64_t pc = apc_morton(t[0] << sh, t[1] << sh, t[2] << sh);
    const int64_t z = apc_last_le(mc, n, pc);
    if (lev[z] < l - 1) mark[z] = 1;
  }
}

// Face f of leaf y lies on a wall: a face of the box (not periodic), or on an
// irregular domain a face onto an excluded cell.
__device__ inline bool wall_face(const Mask &M, const uint32_t t0[3], int l, int f, int periodic) {
  const int d = f >> 1;
  const uint32_t top = (1u << l) - 1u;
  const bool box = (f & 1) ? (t0[d] == top) : (t0[d] == 0u);
  if (box) return !periodic;
  if (M.ml <= 0) return false;
  uint32_t t[3] = {t0[0], t0[1], t0[2]};
  t[d] = (f & 1) ? t[d] + 1u : t[d] - 1u;
  return mask_state(M, apc_morton(t[0], t[1], t[2]), l) == 1;
}

// number of faces of each leaf lying on a wall
__global__ void __launch_bounds__(APC_BLOCK)
    k_bcount(const uint64_t *pre, const int32_t *lev, int64_t n, int periodic, Mask M, int32_t *bc) {
  int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  uint32_t t[3];
  cell_index(pre[y], t);
  int k = 0;
  for (int f = 0; f < 6; f++) k += wall_face(M, t, lev[y], f, periodic);
  bc[y] = k;
}

// Node coordinates (units of L 2^-(D+1)): centre of a level-l cell with index i is
// (2i+1) 2^(D-l); boundary nodes sit at the centre of their owner's face.
__global__ void __launch_bounds__(APC_BLOCK)
    k_nodes(const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev,
            const int32_t *__restrict__ bstart, int64_t n, int64_t ntot, int D, int periodic,
            Mask M, int32_t *__restrict__ crd, int32_t *__restrict__ bowner,
            int32_t *__restrict__ bface) {
  int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y == 0) crd[3 * ntot] = periodic ? (1 << (D + 1)) : 0; // the side S
  if (y >= n) return;
  const int l = lev[y];
  uint32_t t[3];
  cell_index(pre[y], t);
  const int32_t sz = 1 << (D - l);
  int32_t c[3];
  for (int d = 0; d < 3; d++) {
    c[d] = (int32_t)(2u * t[d] + 1u) * sz;
    crd[(int64_t)d * ntot + y] = c[d];
  }
  int64_t b = n + bstart[y];
  for (int f = 0; f < 6; f++) {
    const int d = f >> 1;
    if (!wall_face(M, t, l, f, periodic)) continue;
    for (int e = 0; e < 3; e++) crd[(int64_t)e * ntot + b] = c[e];
    crd[(int64_t)d * ntot + b] = c[d] + ((f & 1) ? sz : -sz); // the centre of face f
    bowner[b - n] = (int32_t)y;
    bface[b - n] = f;
    b++;
  }
}

// 1-ring (Sec. 4.3): per face, the neighbouring leaf if it is not finer, else the
// 4 level-(l+1) leaves touching the face; boundary faces give the boundary node.
__global__ void __launch_bounds__(APC_BLOCK)
    k_ring1(const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev,
            const uint64_t *__restrict__ mc, const int32_t *__restrict__ bstart, int64_t n, int D,
            int periodic, Mask M, int32_t *__restrict__ r1cnt, int32_t *__restrict__ r1,
            int *__restrict__ err) {
  int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  const int l = lev[y];
  uint32_t t0[3];
  cell_index(pre[y], t0);
  const uint32_t top = (1u << l) - 1u;
  int32_t *out = r1 + y * 24;
  int k = 0, kb = 0;
  for (int f = 0; f < 6; f++) {
    const int d = f >> 1;
    if (wall_face(M, t0, l, f, periodic)) {
      out[k++] = (int32_t)(n + bstart[y] + kb++);
      continue;
    }
    uint32_t t[3] = {t0[0], t0[1], t0[2]};
    t[d] = ((f & 1) ? t[d] + 1u : t[d] + top) & top; // wraps across a periodic boundary
    const int sh = D - l;
    const uint64_t pc = apc_morton(t[0] << sh, t[1] << sh, t[2] << sh);
    const int64_t z = apc_last_le(mc, n, pc);
    if (lev[z] <= l) {
      out[k++] = (int32_t)z;
      continue;
    }
    if (l + 1 > D) {
      atomicOr(err, 4);
      continue;
    }
    const int side = (f & 1) ? 0 : 1;
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++) {
        uint32_t u[3];
        int q = 0;
        for (int e = 0; e < 3; e++) {
          if (e == d) {
            u[e] = 2u * t[e] + (uint32_t)side;
          } else {
            u[e] = 2u * t[e] + (uint32_t)(q == 0 ? a : b);
            q++;
          }
        }
        const int sh1 = D - l - 1;
        const uint64_t pc1 = apc_morton(u[0] << sh1, u[1] << sh1, u[2] << sh1);
        const int64_t zc = apc_last_le(mc, n, pc1);
        if (lev[zc] != l + 1 || mc[zc] != pc1) atomicOr(err, 4);
        out[k++] = (int32_t)zc;
      }
  }
  r1cnt[y] = k;
}

// Stencil of node y from its R-ring (nodes within R face-adjacency steps, boundary
// nodes hanging off their owner): candidates sorted by (squared integer distance,
// node index); the two nearest of every closed octant are chosen first; for an
// order-4 row then, axis by axis, the nearest candidates with a new offset along
// the axis until it spans 5 distinct offsets (the centre's 0 included; on fewer
// planes a quartic vanishes on the whole stencil); then the nearest remaining ones
// up to min(count, m_cap).  Accepted (m > 0) when every closed octant holds a
// chosen node (relax: every closed octant in which the ring holds a candidate; set
// for the last ring of an irregular domain, where at a convex corner of the voxel
// staircase an octant holds no node of any ring) and m >= p + 1; the rank test
// follows in a separate kernel.
//
// One thread per pending node (thread t works on position pos = tmap ? tmap[t] : t
// of the chunk and writes mout[pos], cand[pos]).  The ring lives in per-thread
// global scratch laid out element-major (element k of thread t at k * stride + t,
// so that the lanes of a wavefront walking their lists in step touch neighbouring
// words): the BFS list (node ids), the sort keys, and an open-addressing hash set
// of the nodes seen (entries gen << 32 | node; an entry of another generation is
// empty, so the table is never cleared).  The list holds at most cap nodes: past
// that the thread reports -1 (the host reruns it with the full APC_RING_CAP), or,
// when cap is already APC_RING_CAP (full), flags error 8.  The result does not
// depend on cap.
// A ring-search sort key holds r2 in bits 0-47 (r2 < 3 * 2^42 at max_depth 20, whose
// integer coordinates stay below 2^21) and the closed-octant mask in bits 48-55, so
// bits 56-63 of every key are zero.
constexpr int KEY_MASK_SHIFT = 48;
constexpr int64_t KEY_R2 = ((int64_t)1 << KEY_MASK_SHIFT) - 1;

__device__ __forceinline__ uint32_t ring_hash(int32_t v, uint32_t mask) {
  return ((uint32_t)v * 2654435761u) & mask;
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_stencil(const int32_t *__restrict__ pending, const int32_t *__restrict__ tmap, int64_t np,
              int R, int m_cap, int p, int order, const int32_t *__restrict__ crd, int64_t ntot,
              int64_t n, const int32_t *__restrict__ r1cnt, const int32_t *__restrict__ r1,
              const int32_t *__restrict__ bowner, int cap, int64_t stride, uint32_t hmask,
              uint32_t gen, int32_t *__restrict__ lst_all, int64_t *__restrict__ key_all,
              uint64_t *__restrict__ hash_all, int full, int32_t *__restrict__ cand,
              int32_t *__restrict__ mout, int *__restrict__ err, int relax) {
  const int64_t t = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (t >= np) return;
  const int64_t pos = tmap ? tmap[t] : t;
  const int32_t y = pending[pos];
  int32_t *lst = lst_all + t;
  int64_t *key = key_all + t;
  uint64_t *tab = hash_all + t;
#define LST(k) lst[(int64_t)(k) * stride]
#define KEY(k) key[(int64_t)(k) * stride]
  // Tag of this launch: bit 31 of the upper half set, so no stale word of the
  // scratch can match it.  The same scratch is carved anew for each ring radius,
  // so a hash slot may hold words of an earlier launch's list or keys.  A list
  // word is a pair of node ids: an upper half below 2^31, or -(v+1) for a picked
  // node, which equals the tag only for v = 2^31 - gen - 1 >= ntot (the host keeps
  // gen < 2^16 and ntot <= 2^31 - 2^16).  A key word has bits 56-63 clear, so its
  // upper half is below 2^24.
  const uint64_t g = (uint64_t)(gen | 0x80000000u) << 32;
  // true when v was not in the set (and is now)
  auto insert = [&](int32_t v) -> bool {
    uint32_t h = ring_hash(v, hmask);
    for (;;) {
      const uint64_t e = tab[(int64_t)h * stride];
      if ((e & 0xffffffff00000000ull) != g) {
        tab[(int64_t)h * stride] = g | (uint32_t)v;
        return true;
      }
      if ((int32_t)(uint32_t)e == v) return false;
      h = (h + 1) & hmask;
    }
  };
  int cnt = 0;
  LST(cnt++) = y;
  insert(y);
  int lo = 0;
  bool overflow = false;
  for (int depth = 1; depth <= R && !overflow; depth++) {
    const int hi = cnt;
    for (int q = lo; q < hi && !overflow; q++) {
      const int32_t u = LST(q);
      const bool bnd = u >= n; // a boundary node's only neighbour is its owner
      const int na = bnd ? 1 : r1cnt[u];
      for (int a = 0; a < na; a++) {
        const int32_t v = bnd ? bowner[u - n] : r1[(int64_t)u * 24 + a];
        if (!insert(v)) continue;
        if (cnt == cap) {
          overflow = true;
          break;
        }
        LST(cnt++) = v;
      }
    }
    lo = hi;
  }
  if (overflow) {
    if (full) atomicOr(err, 8);
    mout[pos] = full ? 0 : -1;
    return;
  }
  const int32_t cy0 = crd[y], cy1 = crd[ntot + y], cy2 = crd[2 * ntot + y];
  const int32_t S = crd[3 * ntot]; // periodic side (0: none): minimum-image offsets
  // candidates = list positions 1 .. cnt-1, heap-sorted by (r2, index).  Each key
  // carries the candidate's closed-octant mask in bits 48-55 (bit o: the offset lies
  // in octant o, a zero component counting on both sides); r2 < 2^44 below them.
  for (int j = 1; j < cnt; j++) {
    const int32_t v = LST(j);
    const int64_t d0 = apc_doff(crd[v], cy0, S), d1 = apc_doff(crd[ntot + v], cy1, S),
                  d2 = apc_doff(crd[2 * ntot + v], cy2, S);
    const uint32_t mx = (d0 >= 0 ? 0xF0u : 0u) | (d0 <= 0 ? 0x0Fu : 0u);
    const uint32_t my = (d1 >= 0 ? 0xCCu : 0u) | (d1 <= 0 ? 0x33u : 0u);
    const uint32_t mz = (d2 >= 0 ? 0xAAu : 0u) | (d2 <= 0 ? 0x55u : 0u);
    KEY(j) = (int64_t)((uint64_t)(d0 * d0 + d1 * d1 + d2 * d2) |
                       ((uint64_t)(mx & my & mz) << KEY_MASK_SHIFT));
  }
  {
    const int m = cnt - 1;
    auto less = [&](int a, int b) -> bool { // heap positions 0..m-1 = list positions 1..m
      const int64_t ka = KEY(a + 1) & KEY_R2, kb = KEY(b + 1) & KEY_R2;
      return ka < kb || (ka == kb && LST(a + 1) < LST(b + 1));
    };
    auto swp = [&](int a, int b) {
      const int64_t k = KEY(a + 1);
      KEY(a + 1) = KEY(b + 1);
      KEY(b + 1) = k;
      const int32_t v = LST(a + 1);
      LST(a + 1) = LST(b + 1);
      LST(b + 1) = v;
    };
    auto sift = [&](int root, int end) {
      for (;;) {
        int c = 2 * root + 1;
        if (c >= end) break;
        if (c + 1 < end && less(c, c + 1)) c++;
        if (!less(root, c)) break;
        swp(root, c);
        root = c;
      }
    };
    for (int st = m / 2 - 1; st >= 0; st--) sift(st, m);
    for (int e = m - 1; e > 0; e--) {
      swp(0, e);
      sift(0, e);
    }
  }
  const int nc = cnt - 1;
  const int want = nc < m_cap ? nc : m_cap;
  int got = 0;
  // picked candidates are marked by storing -(v+1).  Octant by octant, the two
  // nearest candidates in the octant are taken and picked unless picked already:
  // one pass over the sorted list finds each octant's two nearest.
  uint32_t popm = 0; // octants in which the ring holds a candidate
  {
    int f0[8], f1[8], nf[8];
#pragma unroll
    for (int o = 0; o < 8; o++) nf[o] = 0, f0[o] = f1[o] = 0;
    uint32_t open = 0xFFu; // octants still short of two
    for (int j = 1; j < cnt && open; j++) {
      const uint32_t msk = (uint32_t)((uint64_t)KEY(j) >> KEY_MASK_SHIFT) & open;
#pragma unroll
      for (int o = 0; o < 8; o++)
        if ((msk >> o) & 1u) {
          if (nf[o] == 0) f0[o] = j;
          else f1[o] = j;
          if (++nf[o] == 2) open &= ~(1u << o);
        }
    }
#pragma unroll
    for (int o = 0; o < 8; o++)
      if (nf[o] > 0) popm |= 1u << o;
#pragma unroll
    for (int o = 0; o < 8; o++)
#pragma unroll
      for (int t = 0; t < 2; t++) {
        if (t >= nf[o]) continue;
        const int j = t == 0 ? f0[o] : f1[o];
        const int32_t v = LST(j);
        if (v >= 0 && got < want) {
          LST(j) = -v - 1;
          got++;
        }
      }
  }
  for (int d = 0; order == 4 && d < 3; d++) {
    const int32_t *cd = crd + (int64_t)d * ntot;
    const int64_t c0 = d == 0 ? cy0 : (d == 1 ? cy1 : cy2);
    for (;;) {
      int64_t vals[5];
      int nv = 1;
      vals[0] = 0;
      for (int j = 1; j < cnt && nv < 5; j++) {
        if (LST(j) >= 0) continue;
        const int64_t o = apc_doff(cd[-LST(j) - 1], (int32_t)c0, S);
        bool seen = false;
        for (int q = 0; q < nv; q++) seen = seen || vals[q] == o;
        if (!seen) vals[nv++] = o;
      }
      if (nv >= 5 || got >= want) break;
      int add = -1;
      for (int j = 1; j < cnt && add < 0; j++) {
        if (LST(j) < 0) continue;
        const int64_t o = apc_doff(cd[LST(j)], (int32_t)c0, S);
        bool seen = false;
        for (int q = 0; q < nv; q++) seen = seen || vals[q] == o;
        if (!seen) add = j;
      }
      if (add < 0) break;
      LST(add) = -LST(add) - 1;
      got++;
    }
  }
  for (int j = 1; j < cnt && got < want; j++)
    if (LST(j) >= 0) {
      LST(j) = -LST(j) - 1;
      got++;
    }
  int m = 0;
  int oct[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int32_t *out = cand + pos * APC_MAXM;
  for (int j = 1; j < cnt; j++) {
    if (LST(j) >= 0) continue;
    const int32_t v = -LST(j) - 1;
    if (m < APC_MAXM) out[m] = v;
    m++;
    const uint32_t msk = (uint32_t)((uint64_t)KEY(j) >> KEY_MASK_SHIFT) & 0xFFu;
#pragma unroll
    for (int o = 0; o < 8; o++) oct[o] += (msk >> o) & 1u;
  }
#undef LST
#undef KEY
  bool ok = m >= p + 1 && m <= APC_MAXM;
  for (int o = 0; o < 8; o++) ok = ok && (oct[o] >= 1 || (relax && !((popm >> o) & 1u)));
  mout[pos] = ok ? m : 0;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The order-2 stencil search of k_stencil with one wavefront per node, for rings
// of at most 63 candidates (the node itself and 63 others fill the 64 lanes).
// Lanes expand the BFS frontier in parallel (lane q takes frontier node q and its
// up to 24 face neighbours) into a hash set in LDS; the members, in any order,
// are then sorted across the lanes by (r2, index) with a bitonic network, so lane
// j holds the j-th nearest candidate; the selection of k_stencil (per octant the
// two nearest, then the nearest remaining up to m_cap) runs on lane masks.  The
// set, the order and so the stencil are those of k_stencil.  A larger ring gets
// m = -1 and is searched again by k_stencil.
constexpr int WV_HASH = 256; // > 2 x 128: at most 64 + 64 members before the overflow test
__global__ void __launch_bounds__(APC_BLOCK)
    k_stencil_wave(const int32_t *__restrict__ pending, int64_t np, int R, int m_cap, int p,
                   const int32_t *__restrict__ crd, int64_t ntot, int64_t n,
                   const int32_t *__restrict__ r1cnt, const int32_t *__restrict__ r1,
                   const int32_t *__restrict__ bowner, int32_t *__restrict__ cand,
                   int32_t *__restrict__ mout, int relax) {
  __shared__ int32_t sh_h[APC_BLOCK / 64][WV_HASH];
  __shared__ int32_t sh_l[APC_BLOCK / 64][64];
  __shared__ int32_t sh_c[APC_BLOCK / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t pos = (int64_t)blockIdx.x * (APC_BLOCK / 64) + w;
  if (pos >= np) return; // whole wavefronts
  int32_t *H = sh_h[w], *Ls = sh_l[w];
  int32_t *cnt = &sh_c[w];
  for (int k = lane; k < WV_HASH; k += 64) H[k] = -1;
  if (lane == 0) *cnt = 0;
  const int32_t y = pending[pos];
  wave_sync();
  auto insert = [&](int32_t v) {
    uint32_t h = ring_hash(v, WV_HASH - 1);
    for (;;) {
      const int32_t old = atomicCAS(&H[h], -1, v);
      if (old == -1) {
        const int slot = atomicAdd(cnt, 1);
        if (slot < 64) Ls[slot] = v;
        return;
      }
      if (old == v) return;
      h = (h + 1) & (WV_HASH - 1);
    }
  };
  if (lane == 0) insert(y);
  wave_sync();
  int lo = 0, hi = 1;
  bool ovf = false;
  for (int depth = 1; depth <= R && !ovf; depth++) {
    const int q = lo + lane;
    int32_t nb[24];
    int na = 0;
    if (q < hi) {
      const int32_t u = Ls[q];
      if (u >= n) { // a boundary node's only neighbour is its owner
        na = 1;
        nb[0] = bowner[u - n];
      } else {
        na = r1cnt[u];
#pragma unroll
        for (int a = 0; a < 24; a++) nb[a] = a < na ? r1[(int64_t)u * 24 + a] : -1;
      }
    }
#pragma unroll
    for (int a = 0; a < 24; a++) {
      if (a < na) insert(nb[a]);
      wave_sync();
      if (*cnt > 64) {
        ovf = true;
        break;
      }
    }
    lo = hi;
    hi = *cnt;
  }
  const int total = *cnt;
  if (ovf || total > 64) {
    if (lane == 0) mout[pos] = -1;
    return;
  }
  const int nc = total - 1; // candidates: the members other than y
  int32_t v = 0x7fffffff;
  int64_t r2 = INT64_MAX;
  uint32_t msk = 0;
  if (lane < nc) {
    const int32_t cy0 = crd[y], cy1 = crd[ntot + y], cy2 = crd[2 * ntot + y];
    const int32_t S = crd[3 * ntot]; // periodic side (0: none)
    v = Ls[lane + 1]; // slot 0 holds y
    const int64_t d0 = apc_doff(crd[v], cy0, S), d1 = apc_doff(crd[ntot + v], cy1, S),
                  d2 = apc_doff(crd[2 * ntot + v], cy2, S);
    r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const uint32_t mx = (d0 >= 0 ? 0xF0u : 0u) | (d0 <= 0 ? 0x0Fu : 0u);
    const uint32_t my = (d1 >= 0 ? 0xCCu : 0u) | (d1 <= 0 ? 0x33u : 0u);
    const uint32_t mz = (d2 >= 0 ? 0xAAu : 0u) | (d2 <= 0 ? 0x55u : 0u);
    msk = mx & my & mz;
  }
  // bitonic sort of (r2, v) ascending over the 64 lanes; idle lanes hold the maximum
  for (int k = 2; k <= 64; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int64_t r2o = __shfl_xor(r2, j);
      const int32_t vo = __shfl_xor(v, j);
      const uint32_t mo = (uint32_t)__shfl_xor((int)msk, j);
      const bool lower = (lane & j) == 0, up = (lane & k) == 0;
      const bool o_less = r2o < r2 || (r2o == r2 && vo < v);
      const bool o_more = r2o > r2 || (r2o == r2 && vo > v);
      if (up == lower ? o_less : o_more) {
        r2 = r2o;
        v = vo;
        msk = mo;
      }
    }
  const int want = nc < m_cap ? nc : m_cap;
  uint64_t inO[8];
#pragma unroll
  for (int o = 0; o < 8; o++) inO[o] = __ballot(lane < nc && ((msk >> o) & 1u));
  uint64_t P = 0;
#pragma unroll
  for (int o = 0; o < 8; o++) {
    uint64_t b = inO[o];
#pragma unroll
    for (int t = 0; t < 2; t++) {
      if (!b) break;
      const uint64_t low = b & (~b + 1ull);
      b &= b - 1ull;
      if (!(P & low) && __popcll(P) < want) P |= low;
    }
  }
  uint64_t rem = (nc >= 64 ? ~0ull : ((1ull << nc) - 1ull)) & ~P;
  while (__popcll(P) < want && rem) {
    P |= rem & (~rem + 1ull);
    rem &= rem - 1ull;
  }
  const int m = __popcll(P);
  bool ok = m >= p + 1 && m <= APC_MAXM;
#pragma unroll
  for (int o = 0; o < 8; o++) ok = ok && ((P & inO[o]) != 0 || (relax && inO[o] == 0));
  if ((P >> lane) & 1ull)
    cand[pos * APC_MAXM + __popcll(P & ((1ull << lane) - 1ull))] = v;
  if (lane == 0) mout[pos] = ok ? m : 0;
}

// The same search with one block per node for rings of 64 to 255 candidates
// (the rings k_stencil_wave leaves open): threads expand the frontier into an LDS
// hash set, a bitonic network in LDS sorts the members by (r2, index), and thread
// 0 runs the selection on the 256-bit masks of the four wavefronts' ballots.
// Larger rings keep m = -1 and go to k_stencil.  tmap lists the chunk positions
// of the nodes to search (one block each).
constexpr int BK_HASH = 1024; // > 2 x 512: at most 256 + 256 members before the overflow test
__global__ void __launch_bounds__(APC_BLOCK)
    k_stencil_block(const int32_t *__restrict__ pending, const int32_t *__restrict__ tmap,
                    int64_t np, int R, int m_cap, int p, const int32_t *__restrict__ crd,
                    int64_t ntot, int64_t n, const int32_t *__restrict__ r1cnt,
                    const int32_t *__restrict__ r1, const int32_t *__restrict__ bowner,
                    int32_t *__restrict__ cand, int32_t *__restrict__ mout, int relax) {
  __shared__ int32_t H[BK_HASH];
  __shared__ int32_t Ls[APC_BLOCK];
  __shared__ int64_t Kr[APC_BLOCK];
  __shared__ int32_t Kv[APC_BLOCK];
  __shared__ uint32_t Km[APC_BLOCK];
  __shared__ uint64_t inO[8][APC_BLOCK / 64];
  __shared__ uint64_t Pm[APC_BLOCK / 64];
  __shared__ int32_t cnt, mres;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t t = blockIdx.x;
  if (t >= np) return; // whole blocks
  const int64_t pos = tmap[t];
  const int32_t y = pending[pos];
  for (int k = tid; k < BK_HASH; k += APC_BLOCK) H[k] = -1;
  if (tid == 0) cnt = 0;
  __syncthreads();
  auto insert = [&](int32_t v) {
    uint32_t h = ring_hash(v, BK_HASH - 1);
    for (;;) {
      const int32_t old = atomicCAS(&H[h], -1, v);
      if (old == -1) {
        const int slot = atomicAdd(&cnt, 1);
        if (slot < APC_BLOCK) Ls[slot] = v;
        return;
      }
      if (old == v) return;
      h = (h + 1) & (BK_HASH - 1);
    }
  };
  if (tid == 0) insert(y);
  __syncthreads();
  int lo = 0, hi = 1;
  bool ovf = false;
  for (int depth = 1; depth <= R && !ovf; depth++) {
    const int q = lo + tid;
    int32_t u = -1;
    int na = 0;
    if (q < hi) {
      u = Ls[q];
      na = u >= n ? 1 : r1cnt[u];
    }
    for (int a = 0; a < 24; a++) {
      if (a < na) insert(u >= n ? bowner[u - n] : r1[(int64_t)u * 24 + a]);
      __syncthreads();
      const int c_now = cnt;
      __syncthreads(); // every thread has read cnt before the next round changes it
      if (c_now > APC_BLOCK) {
        ovf = true;
        break;
      }
    }
    lo = hi;
    hi = cnt;
    __syncthreads();
  }
  const int total = cnt;
  if (ovf || total > APC_BLOCK) {
    if (tid == 0) mout[pos] = -1;
    return;
  }
  const int nc = total - 1;
  {
    int32_t v = 0x7fffffff;
    int64_t r2 = INT64_MAX;
    uint32_t msk = 0;
    if (tid < nc) {
      v = Ls[tid + 1]; // slot 0 holds y
      const int32_t S = crd[3 * ntot]; // periodic side (0: none)
      const int64_t d0 = apc_doff(crd[v], crd[y], S), d1 = apc_doff(crd[ntot + v], crd[ntot + y], S),
                    d2 = apc_doff(crd[2 * ntot + v], crd[2 * ntot + y], S);
      r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const uint32_t mx = (d0 >= 0 ? 0xF0u : 0u) | (d0 <= 0 ? 0x0Fu : 0u);
      const uint32_t my = (d1 >= 0 ? 0xCCu : 0u) | (d1 <= 0 ? 0x33u : 0u);
      const uint32_t mz = (d2 >= 0 ? 0xAAu : 0u) | (d2 <= 0 ? 0x55u : 0u);
      msk = mx & my & mz;
    }
    Kr[tid] = r2;
    Kv[tid] = v;
    Km[tid] = msk;
  }
  __syncthreads();
  // bitonic sort of (r2, v) ascending over the block
  for (int k = 2; k <= APC_BLOCK; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int o = tid ^ j;
      int64_t r2 = Kr[tid];
      int32_t v = Kv[tid];
      uint32_t msk = Km[tid];
      const int64_t r2o = Kr[o];
      const int32_t vo = Kv[o];
      const uint32_t mo = Km[o];
      const bool lower = (tid & j) == 0, up = (tid & k) == 0;
      const bool o_less = r2o < r2 || (r2o == r2 && vo < v);
      const bool o_more = r2o > r2 || (r2o == r2 && vo > v);
      const bool take = up == lower ? o_less : o_more;
      __syncthreads();
      if (take) {
        Kr[tid] = r2o;
        Kv[tid] = vo;
        Km[tid] = mo;
      }
      __syncthreads();
    }
  const uint32_t msk = Km[tid];
#pragma unroll
  for (int o = 0; o < 8; o++) {
    const uint64_t b = __ballot(tid < nc && ((msk >> o) & 1u));
    if (lane == 0) inO[o][w] = b;
  }
  __syncthreads();
  if (tid == 0) {
    const int want = nc < m_cap ? nc : m_cap;
    uint64_t P[APC_BLOCK / 64] = {0, 0, 0, 0};
    int got = 0;
    for (int o = 0; o < 8; o++) {
      int taken = 0;
      for (int q = 0; q < APC_BLOCK / 64 && taken < 2; q++) {
        uint64_t b = inO[o][q];
        while (b && taken < 2) {
          const uint64_t low = b & (~b + 1ull);
          b &= b - 1ull;
          taken++;
          if (!(P[q] & low) && got < want) {
            P[q] |= low;
            got++;
          }
        }
      }
    }
    for (int q = 0; q < APC_BLOCK / 64 && got < want; q++) {
      const int base = 64 * q;
      const int lim = nc - base;
      if (lim <= 0) break;
      uint64_t rem = (lim >= 64 ? ~0ull : ((1ull << lim) - 1ull)) & ~P[q];
      while (got < want && rem) {
        P[q] |= rem & (~rem + 1ull);
        rem &= rem - 1ull;
        got++;
      }
    }
    bool ok = got >= p + 1 && got <= APC_MAXM;
    for (int o = 0; o < 8; o++) {
      bool any = false, pop = false;
      for (int q = 0; q < APC_BLOCK / 64; q++) {
        any = any || (P[q] & inO[o][q]) != 0;
        pop = pop || inO[o][q] != 0;
      }
      ok = ok && (any || (relax && !pop));
    }
    for (int q = 0; q < APC_BLOCK / 64; q++) Pm[q] = P[q];
    mres = ok ? got : 0;
  }
  __syncthreads();
  if ((Pm[w] >> lane) & 1ull) {
    int idx = __popcll(Pm[w] & ((1ull << lane) - 1ull));
    for (int q = 0; q < w; q++) idx += __popcll(Pm[q]);
    cand[pos * APC_MAXM + idx] = Kv[tid];
  }
  if (tid == 0) mout[pos] = mres;
}

// 1 where the first pass ran out of ring capacity
__global__ void __launch_bounds__(APC_BLOCK) k_retry_flag(const int32_t *m, int64_t n, int32_t *f) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) f[i] = m[i] < 0 ? 1 : 0;
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_accept(const int32_t *__restrict__ pending, int64_t np, const int32_t *__restrict__ cand,
             const int32_t *__restrict__ m, int32_t *__restrict__ stbuf,
             int32_t *__restrict__ mnode, int32_t *__restrict__ still, int order,
             int8_t *__restrict__ rorder) {
  // one thread per (node, slot): a wavefront copies one node's row of APC_MAXM slots
  const int64_t e = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  const int64_t t = e / APC_MAXM;
  const int j = (int)(e % APC_MAXM);
  if (t >= np) return;
  const int32_t y = pending[t];
  const int mm = m[t];
  if (j == 0) {
    still[t] = mm > 0 ? 0 : 1;
    if (mm > 0) {
      mnode[y] = mm;
      rorder[y] = (int8_t)order;
    }
  }
  if (j < mm) stbuf[(int64_t)y * APC_MAXM + j] = cand[t * APC_MAXM + j];
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_compact_idx(const int32_t *flag, const int32_t *off, const int32_t *src, int64_t n,
                  int32_t *dst) {
  int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n && flag[i]) dst[off[i]] = src ? src[i] : (int32_t)i;
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_csr_fill(const int32_t *__restrict__ stbuf, const int32_t *__restrict__ off, int64_t n,
               int32_t *__restrict__ idx) {
  int64_t e = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  // one thread per (node, slot) pair
  const int64_t y = e / APC_MAXM;
  const int j = (int)(e % APC_MAXM);
  if (y >= n) return;
  const int32_t a = off[y], b = off[y + 1];
  if (j < b - a) idx[a + j] = stbuf[y * APC_MAXM + j];
}

__global__ void __launch_bounds__(APC_BLOCK)
    k_leaf_out(const uint64_t *mc, const int32_t *lev, int64_t n, uint64_t *code, int32_t *level) {
  int64_t y = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (y >= n) return;
  code[y] = mc[y];
  level[y] = lev[y];
}

// leaf of every sorted particle: the last leaf whose range starts at or before it
__global__ void __launch_bounds__(APC_BLOCK)
    k_pnode(const int32_t *__restrict__ first, int64_t n, int64_t N, int32_t *__restrict__ pnode) {
  int64_t s = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (s >= N) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (first[mid] <= s)
      lo = mid + 1;
    else
      hi = mid;
  }
  pnode[s] = (int32_t)(lo - 1);
}

template <typename T>
int dalloc(T **p, int64_t n, hipStream_t s) {
  HIPCHK(apc_malloc_async((void **)p, (size_t)(n > 0 ? n : 1) * sizeof(T), s));
  return APC_OK;
}
template <typename T>
int dfree(T *&p, hipStream_t s) {
  if (p) HIPCHK(apc_free_async(p, s));
  p = nullptr;
  return APC_OK;
}

// flagged cells -> 8 children; returns the new list in `c`
int expand(Cells &c, const uint64_t *keys, int D, const Thr &thr, const Mask &M, int criterion,
           hipStream_t s) {
  int32_t *sz = nullptr, *off = nullptr;
  APCCHK(dalloc(&sz, c.n, s));
  APCCHK(dalloc(&off, c.n, s));
  hipLaunchKernelGGL(k_sizes, dim3(grid_for(c.n)), dim3(APC_BLOCK), 0, s, c.flag, c.n, sz);
  HIPCHK(hipGetLastError());
  APCCHK(apc_scan_i32(sz, off, c.n, s));
  int32_t last[2];
  HIPCHK(hipMemcpyAsync(&last[0], off + c.n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&last[1], sz + c.n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t m = (int64_t)last[0] + last[1];
  Cells o;
  APCCHK(cells_alloc(o, m, s));
  hipLaunchKernelGGL(k_expand, dim3(grid_for(c.n)), dim3(APC_BLOCK), 0, s, c.pre, c.lev, c.fst,
                     c.cnt, c.flag, off, c.n, keys, D, thr, M, criterion, o.pre, o.lev, o.fst, o.cnt,
                     o.flag);
  HIPCHK(hipGetLastError());
  APCCHK(dfree(sz, s));
  APCCHK(dfree(off, s));
  APCCHK(cells_free(c, s));
  c = o;
  return APC_OK;
}

// flag[i] = 1 for the leaves inside Omega
__global__ void __launch_bounds__(APC_BLOCK)
    k_inside(const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev, int64_t n, Mask M,
             int32_t *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i < n) flag[i] = mask_state(M, pre[i], lev[i]) != 1;
}
__global__ void __launch_bounds__(APC_BLOCK)
    k_keep_cells(const int32_t *__restrict__ flag, const int32_t *__restrict__ off, int64_t n,
                 const uint64_t *__restrict__ pre, const int32_t *__restrict__ lev,
                 const int32_t *__restrict__ fst, const int32_t *__restrict__ cnt,
                 uint64_t *__restrict__ opre, int32_t *__restrict__ olev,
                 int32_t *__restrict__ ofst, int32_t *__restrict__ ocnt) {
  const int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const int64_t o = off[i];
  opre[o] = pre[i];
  olev[o] = lev[i];
  ofst[o] = fst[i];
  ocnt[o] = cnt[i];
}

int read_err(int *err, hipStream_t s, int *host) {
  HIPCHK(hipMemcpyAsync(host, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return APC_OK;
}

void free_cloud_arrays(apc_cloud *c) {
  void *ptrs[] = {c->perm, c->sxyz, c->pnode, c->code, c->level, c->first, c->count, c->crd,
                  c->bowner, c->bface, c->st_off, c->st_idx};
  for (void *q : ptrs)
    if (q) (void)apc_dev_free(q);
}

} // namespace

void apc_free_cloud(apc_cloud *c) {
  if (!c) return;
  // once for all arrays: queued work on any stream may still use them
  (void)hipDeviceSynchronize();
  apc_free_solver(c);
  apc_free_sell(c);
  free_cloud_arrays(c);
  void *ops[] = {c->w64, c->w32, c->diag, c->inv_diag, c->hscale, c->dwx, c->rkind, c->scratch,
                 c->m_diag, c->m_sell, c->m_tmpl, c->bw64, c->bw32, c->sl_bw64, c->sl_bw32,
                 c->rorder, c->dorder, c->w64ref, c->fb_list, c->rkind4, c->gen4, c->cder4};
  for (void *q : ops)
    if (q) (void)apc_dev_free(q);
  delete c;
}

static int build_body(apc_cloud *c, const double *xyz, hipStream_t s) {
  const apc_params &P = c->P;
  const int D = P.max_depth;
  const int64_t N = c->N;
  Thr thr;
  for (int l = 0; l < 24; l++) thr.T[l] = 0.0;
  for (int l = 0; l <= D; l++) thr.T[l] = c->T[l];

  // irregular domain: the state pyramid of the mask (host), in Morton order
  Mask M;
  M.pyr = nullptr;
  M.ml = P.mask_level;
  uint8_t *pyr_dev = nullptr;
  if (M.ml > 0) {
    int64_t tot = 0;
    for (int l = 0; l <= M.ml; l++) {
      M.off[l] = tot;
      tot += (int64_t)1 << (3 * l);
    }
    std::vector<uint8_t> h((size_t)tot);
    const uint32_t sm = 1u << M.ml;
    for (uint32_t z = 0; z < sm; z++)
      for (uint32_t y = 0; y < sm; y++)
        for (uint32_t x = 0; x < sm; x++)
          h[(size_t)(M.off[M.ml] + (int64_t)apc_morton(x, y, z))] =
              P.mask[x + (size_t)sm * (y + (size_t)sm * z)] ? 1 : 0;
    for (int l = M.ml - 1; l >= 0; l--)
      for (int64_t q = 0; q < ((int64_t)1 << (3 * l)); q++) {
        int n0 = 0, n1 = 0;
        for (int c8 = 0; c8 < 8; c8++) {
          const uint8_t v = h[(size_t)(M.off[l + 1] + 8 * q + c8)];
          n0 += v == 0;
          n1 += v == 1;
        }
        h[(size_t)(M.off[l] + q)] = n0 == 8 ? 0 : (n1 == 8 ? 1 : 2);
      }
    if (h[0] == 1) {
      apc_set_error_msg("the mask excludes the whole domain");
      return APC_EINVAL;
    }
    APCCHK(dalloc(&pyr_dev, tot, s));
    HIPCHK(hipMemcpyAsync(pyr_dev, h.data(), (size_t)tot, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    M.pyr = pyr_dev;
  }

  // keys + sort
  uint64_t *keys = nullptr;
  int *err = nullptr;
  APCCHK(dalloc(&keys, N, s));
  HIPCHK(apc_dev_alloc((void **)&c->perm, (size_t)N * sizeof(int32_t)));
  APCCHK(dalloc(&err, 1, s));
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
  const double scale = ldexp(1.0, D) / P.L;
  hipLaunchKernelGGL(k_keys, dim3(grid_for(N)), dim3(APC_BLOCK), 0, s, xyz, N, P.lo[0], P.lo[1],
                     P.lo[2], P.L, scale, D, M, keys, c->perm, err);
  HIPCHK(hipGetLastError());
  int herr = 0;
  APCCHK(read_err(err, s, &herr));
  if (herr & 1) {
    apc_set_error_msg("non-finite particle coordinate");
    return APC_EINVAL;
  }
  if (herr & 2) {
    apc_set_error_msg("particle outside the domain");
    return APC_EDOMAIN;
  }
  APCCHK(apc_radix_sort(keys, c->perm, N, 3 * D, s));

  // criterion phase, one level per pass
  Cells cl;
  APCCHK(cells_alloc(cl, 1, s));
  {
    const uint64_t z = 0;
    const int32_t zi = 0, n32 = (int32_t)N;
    const int32_t op = (0 < D && (M.ml > 0 || (double)N >= c->T[0])) ? 1 : 0;
    HIPCHK(hipMemcpyAsync(cl.pre, &z, sizeof(z), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cl.lev, &zi, sizeof(zi), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cl.fst, &zi, sizeof(zi), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cl.cnt, &n32, sizeof(n32), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cl.flag, &op, sizeof(op), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  int64_t opened = 0;
  for (;;) {
    int64_t nf = 0;
    APCCHK(apc_sum_i32(cl.flag, cl.n, &nf, s));
    if (nf == 0) break;
    opened += nf;
    APCCHK(expand(cl, keys, D, thr, M, 1, s));
  }
  // balance phase: mark, expand, repeat until no leaf is marked
  uint64_t *mc = nullptr;
  for (;;) {
    APCCHK(dfree(mc, s));
    APCCHK(dalloc(&mc, cl.n, s));
    hipLaunchKernelGGL(k_mincorner, dim3(grid_for(cl.n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev,
                       cl.n, D, mc);
    HIPCHK(hipMemsetAsync(cl.flag, 0, (size_t)cl.n * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_balance_mark, dim3(grid_for(cl.n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev,
                       mc, cl.n, D, P.periodic, M, cl.flag);
    HIPCHK(hipGetLastError());
    int64_t nm = 0;
    APCCHK(apc_sum_i32(cl.flag, cl.n, &nm, s));
    if (nm == 0) break;
    opened += nm;
    APCCHK(expand(cl, keys, D, thr, M, 0, s));
  }
  if (M.ml > 0) { // the leaves inside Omega become the nodes
    int32_t *off = nullptr;
    APCCHK(dalloc(&off, cl.n, s));
    hipLaunchKernelGGL(k_inside, dim3(grid_for(cl.n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev,
                       cl.n, M, cl.flag);
    APCCHK(apc_scan_i32(cl.flag, off, cl.n, s));
    int32_t last[2];
    HIPCHK(hipMemcpyAsync(&last[0], off + cl.n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&last[1], cl.flag + cl.n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    Cells in;
    APCCHK(cells_alloc(in, (int64_t)last[0] + last[1], s));
    hipLaunchKernelGGL(k_keep_cells, dim3(grid_for(cl.n)), dim3(APC_BLOCK), 0, s, cl.flag, off,
                       cl.n, cl.pre, cl.lev, cl.fst, cl.cnt, in.pre, in.lev, in.fst, in.cnt);
    HIPCHK(hipGetLastError());
    APCCHK(dfree(off, s));
    APCCHK(cells_free(cl, s));
    cl = in;
    APCCHK(dfree(mc, s));
    APCCHK(dalloc(&mc, cl.n, s));
    hipLaunchKernelGGL(k_mincorner, dim3(grid_for(cl.n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev,
                       cl.n, D, mc);
  }
  const int64_t n = cl.n;
  c->n = n;
  c->n_opened = opened;

  // leaves
  HIPCHK(apc_dev_alloc((void **)&c->code, (size_t)n * sizeof(uint64_t)));
  HIPCHK(apc_dev_alloc((void **)&c->level, (size_t)n * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->first, (size_t)n * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->count, (size_t)n * sizeof(int32_t)));
  hipLaunchKernelGGL(k_leaf_out, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, mc, cl.lev, n, c->code,
                     c->level);
  HIPCHK(hipMemcpyAsync(c->first, cl.fst, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->count, cl.cnt, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));

  // boundary nodes
  int32_t *bcnt = nullptr, *bstart = nullptr;
  APCCHK(dalloc(&bcnt, n, s));
  APCCHK(dalloc(&bstart, n, s));
  hipLaunchKernelGGL(k_bcount, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev, n,
                     P.periodic, M, bcnt);
  APCCHK(apc_scan_i32(bcnt, bstart, n, s));
  int32_t last[2];
  HIPCHK(hipMemcpyAsync(&last[0], bstart + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&last[1], bcnt + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t nb = (int64_t)last[0] + last[1];
  c->nb = nb;
  const int64_t ntot = n + nb;
  HIPCHK(apc_dev_alloc((void **)&c->crd, (size_t)(3 * ntot + 1) * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->bowner, (size_t)(nb > 0 ? nb : 1) * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->bface, (size_t)(nb > 0 ? nb : 1) * sizeof(int32_t)));
  hipLaunchKernelGGL(k_nodes, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev, bstart, n,
                     ntot, D, P.periodic, M, c->crd, c->bowner, c->bface);
  HIPCHK(hipGetLastError());

  // 1-ring adjacency
  int32_t *r1cnt = nullptr, *r1 = nullptr;
  APCCHK(dalloc(&r1cnt, n, s));
  APCCHK(dalloc(&r1, n * 24, s));
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_ring1, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, cl.pre, cl.lev, mc, bstart,
                     n, D, P.periodic, M, r1cnt, r1, err);
  HIPCHK(hipGetLastError());
  APCCHK(read_err(err, s, &herr));
  if (herr) { // an unbalanced face: cannot happen after the balance phase
    apc_set_error_msg("2:1 balance violated after the balance phase");
    return APC_EINVAL;
  }
  APCCHK(dfree(bcnt, s));
  APCCHK(dfree(bstart, s));
  APCCHK(dfree(mc, s));
  APCCHK(cells_free(cl, s));
  if (pyr_dev) APCCHK(dfree(pyr_dev, s));

  // stencils, ring by ring over the nodes still pending
  int32_t *stbuf = nullptr, *mnode = nullptr, *pending = nullptr;
  APCCHK(dalloc(&stbuf, n * APC_MAXM, s));
  APCCHK(dalloc(&mnode, n, s));
  APCCHK(dalloc(&pending, n, s));
  HIPCHK(hipMemsetAsync(mnode, 0, (size_t)n * sizeof(int32_t), s));
  {
    std::vector<int32_t> h(0);
    // pending = 0..n-1
    int32_t *ones = nullptr, *offs = nullptr;
    APCCHK(dalloc(&ones, n, s));
    APCCHK(dalloc(&offs, n, s));
    // all flags 1 -> compaction yields the identity list
    hipLaunchKernelGGL(k_sizes, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, mnode, n, ones);
    // k_sizes writes 1 where mnode == 0 (all), 8 otherwise (none)
    APCCHK(apc_scan_i32(ones, offs, n, s));
    hipLaunchKernelGGL(k_compact_idx, dim3(grid_for(n)), dim3(APC_BLOCK), 0, s, ones, offs,
                       (const int32_t *)nullptr, n, pending);
    HIPCHK(hipGetLastError());
    APCCHK(dfree(ones, s));
    APCCHK(dfree(offs, s));
  }
  int64_t np = n;
  // Ring-search scratch of k_stencil, per node of a chunk (element-major): a list
  // of cap nodes, their sort keys and a hash set of 2^k >= 2 cap entries.  First
  // pass with cap = 2 (2R+1)^3 on chunks of up to 8 GiB of scratch; nodes whose
  // ring is larger are rerun with the full APC_RING_CAP in sub-chunks of up to
  // 1 GiB.  (A tighter first cap, four times the ring of a uniform region, sent
  // more fourth-order nodes to the slow rerun: 0.98 -> 1.13 s at 8.8e6 nodes.)
  // apc_params.ring_first_cap > 0 sets the first-pass capacity instead (a smaller
  // value sends more nodes to the full-capacity rerun; the stencils are the same).
  auto ring_cap = [&P](int R) {
    const int64_t w = 2 * (int64_t)R + 1;
    return (int)std::min<int64_t>(APC_RING_CAP, P.ring_first_cap > 0 ? P.ring_first_cap
                                                                     : 2 * w * w * w);
  };
  auto hash_size = [](int cap) {
    int h = 1;
    while (h < 2 * cap) h <<= 1;
    return h;
  };
  auto node_words = [&](int cap) { // 8-byte words per node
    return ((int64_t)cap * 4 + 7) / 8 + (int64_t)cap + (int64_t)hash_size(cap);
  };
  const int64_t W1 = ((int64_t)8 << 30) / 8, W2 = ((int64_t)1 << 30) / 8;
  auto chunk_nodes = [&](int cap, int64_t words) {
    return std::max<int64_t>(1, std::min<int64_t>(np, words / node_words(cap)));
  };
  int64_t CHmax = 1, words1 = 1;
  for (int R = 1; R <= P.ring_max; R++) {
    const int64_t ch = chunk_nodes(ring_cap(R), W1);
    CHmax = std::max(CHmax, ch);
    words1 = std::max(words1, ch * node_words(ring_cap(R)));
  }
  const int64_t CH2 = chunk_nodes(APC_RING_CAP, W2);
  const int64_t words2 = CH2 * node_words(APC_RING_CAP);
  uint64_t *scr1 = nullptr, *scr2 = nullptr;
  int32_t *cand = nullptr, *mch = nullptr, *still = nullptr, *soff = nullptr, *npend = nullptr,
          *rflag = nullptr, *roff = nullptr, *rlist = nullptr;
  // scratch of the per-thread search (k_stencil), allocated on its first use: the
  // wavefront and block searches keep their rings in LDS
  auto scratch = [&]() -> int {
    if (scr1) return APC_OK;
    APCCHK(dalloc(&scr1, words1, s));
    APCCHK(dalloc(&scr2, words2, s));
    // hash entries carry the launch's tag: zero once, never cleared again
    HIPCHK(hipMemsetAsync(scr1, 0, (size_t)words1 * 8, s));
    HIPCHK(hipMemsetAsync(scr2, 0, (size_t)words2 * 8, s));
    return APC_OK;
  };
  uint32_t gen = 0; // launch tag of the hash entries; stays below 2^16 (see k_stencil)
  if (ntot > ((int64_t)1 << 31) - ((int64_t)1 << 16)) {
    apc_set_error_msg("too many nodes for the ring search");
    return APC_EINVAL;
  }
  APCCHK(dalloc(&cand, CHmax * APC_MAXM, s));
  APCCHK(dalloc(&mch, CHmax, s));
  APCCHK(dalloc(&rflag, CHmax, s));
  APCCHK(dalloc(&roff, CHmax, s));
  APCCHK(dalloc(&rlist, CHmax, s));
  APCCHK(dalloc(&still, n, s));
  APCCHK(dalloc(&soff, n, s));
  APCCHK(dalloc(&npend, n, s));
  struct Scr {
    int32_t *lst;
    int64_t *key;
    uint64_t *tab;
    uint32_t mask;
  };
  auto carve = [&](uint64_t *base, int cap, int64_t ch) {
    Scr r;
    r.lst = (int32_t *)base;
    r.key = (int64_t *)(base + (ch * cap * 4 + 7) / 8);
    r.tab = (uint64_t *)(r.key + ch * cap);
    r.mask = (uint32_t)hash_size(cap) - 1u;
    return r;
  };
  // order fallback (k = 4): nodes with no acceptable order-4 stencil up to ring_max
  // take an order-2 row, chosen by the order-2 rule from ring 2 with cap 40
  HIPCHK(apc_dev_alloc((void **)&c->rorder, (size_t)(n > 0 ? n : 1)));
  for (int att = 0; att < 2 && np > 0; att++) {
  if (att == 1 && P.order != 4) break;
  const int ko = att == 0 ? P.order : 2;
  const int pk = ko == 2 ? 9 : 34;
  const int rmin = att == 0 ? P.ring_min : 2, mcap = att == 0 ? P.m_cap : 40;
  for (int R = rmin; R <= P.ring_max && np > 0; R++) {
    // irregular domain, last ring: an octant with no node in the ring is not asked for
    const int relax = P.mask_level > 0 && R == P.ring_max ? 1 : 0;
    HIPCHK(hipMemsetAsync(err, 0, sizeof(int), s));
    const int cap1 = ring_cap(R);
    const int64_t CH = chunk_nodes(cap1, W1);
    for (int64_t c0 = 0; c0 < np; c0 += CH) {
      const int64_t cn = (np - c0) < CH ? (np - c0) : CH;
      if (gen + 2 + (cn + CH2 - 1) / CH2 >= 0xffffu) {
        apc_set_error_msg("ring search: too many launches for the hash tags");
        return APC_EINVAL;
      }
      // the chunk's nodes whose stencil is still open (m < 0) are searched again by
      // k_stencil with capacity capx, in launches of at most per nodes
      // chunk positions with m < 0 into rlist, their count into *nr
      auto compact_open = [&](int64_t *nr) -> int {
        hipLaunchKernelGGL(k_retry_flag, dim3(grid_for(cn)), dim3(APC_BLOCK), 0, s, mch, cn, rflag);
        HIPCHK(hipGetLastError());
        *nr = 0;
        APCCHK(apc_sum_i32(rflag, cn, nr, s));
        if (*nr == 0) return APC_OK;
        APCCHK(apc_scan_i32(rflag, roff, cn, s));
        hipLaunchKernelGGL(k_compact_idx, dim3(grid_for(cn)), dim3(APC_BLOCK), 0, s, rflag, roff,
                           (const int32_t *)nullptr, cn, rlist);
        HIPCHK(hipGetLastError());
        return APC_OK;
      };
      // (scratch 1: capacity cap1, stride CH; scratch 2: the full capacity, stride CH2)
      auto rerun = [&](int capx, int which, int64_t stride, int64_t per, int full) -> int {
        int64_t nr = 0;
        APCCHK(compact_open(&nr));
        if (nr == 0) return APC_OK;
        APCCHK(scratch());
        const Scr S = carve(which == 1 ? scr1 : scr2, capx, stride);
        for (int64_t r0 = 0; r0 < nr; r0 += per) {
          const int64_t rn = (nr - r0) < per ? (nr - r0) : per;
          hipLaunchKernelGGL(k_stencil, dim3(grid_for(rn)), dim3(APC_BLOCK), 0, s, pending + c0,
                             (const int32_t *)(rlist + r0), rn, R, mcap, pk, ko, c->crd, ntot, n,
                             r1cnt, r1, c->bowner, capx, stride, S.mask, ++gen, S.lst, S.key,
                             S.tab, full, cand, mch, err, relax);
          HIPCHK(hipGetLastError());
        }
        return APC_OK;
      };
      if (ko == 2 && P.ring_lds >= 0) {
        // rings of up to 63 candidates: one wavefront per node; up to 255: one
        // block per node; the rest by k_stencil at capacity cap1
        hipLaunchKernelGGL(k_stencil_wave, dim3(grid_for(cn, APC_BLOCK / 64)), dim3(APC_BLOCK), 0,
                           s, pending + c0, cn, R, mcap, pk, c->crd, ntot, n, r1cnt, r1,
                           c->bowner, cand, mch, relax);
        HIPCHK(hipGetLastError());
        int64_t nb = 0;
        if (P.ring_lds == 0) APCCHK(compact_open(&nb));
        if (nb > 0) {
          hipLaunchKernelGGL(k_stencil_block, dim3((unsigned)nb), dim3(APC_BLOCK), 0, s,
                             pending + c0, (const int32_t *)rlist, nb, R, mcap, pk, c->crd, ntot,
                             n, r1cnt, r1, c->bowner, cand, mch, relax);
          HIPCHK(hipGetLastError());
        }
        APCCHK(rerun(cap1, 1, CH, CH, 0));
      } else {
        APCCHK(scratch());
        const Scr S1 = carve(scr1, cap1, CH);
        hipLaunchKernelGGL(k_stencil, dim3(grid_for(cn)), dim3(APC_BLOCK), 0, s, pending + c0,
                           (const int32_t *)nullptr, cn, R, mcap, pk, ko, c->crd, ntot, n, r1cnt,
                           r1, c->bowner, cap1, CH, S1.mask, ++gen, S1.lst, S1.key, S1.tab, 0,
                           cand, mch, err, relax);
        HIPCHK(hipGetLastError());
      }
      // rerun the nodes whose ring outgrew cap1 with the full capacity
      APCCHK(rerun(APC_RING_CAP, 2, CH2, CH2, 1));
      APCCHK(apc_rank_check(c, ko, pending + c0, cn, cand, mch, s));
      hipLaunchKernelGGL(k_accept, dim3(grid_for(cn * APC_MAXM)), dim3(APC_BLOCK), 0, s, pending + c0, cn, cand,
                         mch, stbuf, mnode, still + c0, ko, c->rorder);
      HIPCHK(hipGetLastError());
    }
    APCCHK(read_err(err, s, &herr));
    if (herr) {
      apc_set_error_msg("ring larger than the search capacity (16384 candidates)");
      return APC_EINVAL;
    }
    APCCHK(apc_scan_i32(still, soff, np, s));
    int64_t left = 0;
    APCCHK(apc_sum_i32(still, np, &left, s));
    hipLaunchKernelGGL(k_compact_idx, dim3(grid_for(np)), dim3(APC_BLOCK), 0, s, still, soff,
                       pending, np, npend);
    HIPCHK(hipGetLastError());
    int32_t *tmp = pending;
    pending = npend;
    npend = tmp;
    np = left;
  }
  }
  APCCHK(dfree(scr1, s));
  APCCHK(dfree(scr2, s));
  APCCHK(dfree(rflag, s));
  APCCHK(dfree(roff, s));
  APCCHK(dfree(rlist, s));
  APCCHK(dfree(cand, s));
  APCCHK(dfree(mch, s));
  APCCHK(dfree(still, s));
  APCCHK(dfree(soff, s));
  APCCHK(dfree(npend, s));
  APCCHK(dfree(pending, s));
  APCCHK(dfree(r1cnt, s));
  APCCHK(dfree(r1, s));
  if (np > 0) return APC_ESTENCIL;

  // stencil CSR
  HIPCHK(apc_dev_alloc((void **)&c->st_off, (size_t)(n + 1) * sizeof(int32_t)));
  APCCHK(apc_scan_i32(mnode, c->st_off, n, s));
  int32_t lastm[2];
  HIPCHK(hipMemcpyAsync(&lastm[0], c->st_off + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&lastm[1], mnode + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t nnz = (int64_t)lastm[0] + lastm[1];
  c->nnz = nnz;
  const int32_t nnz32 = (int32_t)nnz;
  HIPCHK(hipMemcpyAsync(c->st_off + n, &nnz32, sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(apc_dev_alloc((void **)&c->st_idx, (size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t)));
  hipLaunchKernelGGL(k_csr_fill, dim3(grid_for(n * APC_MAXM)), dim3(APC_BLOCK), 0, s, stbuf,
                     c->st_off, n, c->st_idx);
  HIPCHK(hipGetLastError());
  APCCHK(dfree(stbuf, s));
  APCCHK(dfree(mnode, s));

  // particles: leaf of each sorted particle, sorted positions
  HIPCHK(apc_dev_alloc((void **)&c->pnode, (size_t)N * sizeof(int32_t)));
  HIPCHK(apc_dev_alloc((void **)&c->sxyz, (size_t)3 * N * sizeof(double)));
  hipLaunchKernelGGL(k_pnode, dim3(grid_for(N)), dim3(APC_BLOCK), 0, s, c->first, n, N, c->pnode);
  hipLaunchKernelGGL(k_gather_xyz, dim3(grid_for(N)), dim3(APC_BLOCK), 0, s, xyz, c->perm, N,
                     c->sxyz);
  HIPCHK(hipGetLastError());
  APCCHK(dfree(keys, s));
  APCCHK(dfree(err, s));
  APCCHK(apc_prepare_operator(c, s));
  HIPCHK(hipStreamSynchronize(s));
  return APC_OK;
}

int apc_build_impl(const apc_params *p, const double *xyz, int64_t N, hipStream_t s,
                   apc_cloud **out) {
  *out = nullptr;
  if (!p || !xyz || N < 1 || N > INT32_MAX) return APC_EINVAL;
  if (p->order != 2 && p->order != 4) return APC_EINVAL;
  if (p->max_depth < 1 || p->max_depth > 20 || !(p->L > 0.0) || !(p->c > 0.0) ||
      p->ring_min < 1 || p->ring_max < p->ring_min || p->m_cap > APC_MAXM || p->m_cap < 10 || p->stage_cap < -1 ||
      p->criterion_pow < 0 || p->criterion_pow > 16 || p->ring_lds < -1 || p->ring_lds > 1 ||
      p->ring_first_cap < 0 || p->ring_first_cap > APC_RING_CAP || !(p->tau_dom >= 0.0) ||
      !(p->precision == APC_FP64 || p->precision == APC_MIXED ||
        p->precision == APC_MIXED_F32ACC) || !std::isfinite(p->poisson_c) ||
      p->periodic < 0 || p->periodic > 1 || (p->periodic && p->max_depth < 2) ||
      p->kernel < APC_KERNEL_NGP || p->kernel > APC_KERNEL_TSC || p->mask_level < 0 ||
      p->mask_level > 6 || p->mask_level > p->max_depth ||
      (p->mask_level > 0 && (!p->mask || p->periodic || p->kernel != APC_KERNEL_NGP)))
    return APC_EINVAL;
  apc_cloud *c = new apc_cloud();
  c->P = *p;
  HIPCHK(hipGetDevice(&c->device));
  c->N = N;
  c->p = p->order == 2 ? 9 : 34;
  c->unit = p->L / ldexp(1.0, p->max_depth + 1);
  // T_l = t^e, t = (c 2^l) / L, by repeated multiplication from 1.0; e = 2k-2,
  // or the caller's exponent (4 for the supraconvergent k = 2 balance)
  const int pw = p->criterion_pow > 0 ? p->criterion_pow : 2 * p->order - 2;
  for (int l = 0; l < 24; l++) {
    double t = (p->c * ldexp(1.0, l)) / p->L;
    double v = 1.0;
    for (int e = 0; e < pw; e++) v *= t;
    c->T[l] = v;
  }
  // periodic: levels 0 and 1 always open, so that every leaf sees distinct cells
  // across its faces
  if (p->periodic) c->T[0] = c->T[1] = 0.0;
  int rc = build_body(c, xyz, s);
  c->P.mask = nullptr; // the caller's mask is read by the build only
  if (rc != APC_OK) {
    (void)hipStreamSynchronize(s);
    apc_free_cloud(c);
    return rc;
  }
  *out = c;
  return APC_OK;
}

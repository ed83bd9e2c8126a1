// Device-wide primitives used by the cloud build: exclusive scan, integer sum and
// a stable LSD radix sort of (64-bit key, 32-bit value) pairs.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "apc_internal.h"

namespace {

constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = APC_BLOCK * SCAN_IPT;

// One tile of 2048 elements per block: per-thread serial sums, wave64 shuffle
// scan of the thread totals, 4 wave totals combined through LDS.
template <typename T>
__global__ void __launch_bounds__(APC_BLOCK) k_scan_tile(const T *in, T *out, T *bsum, int64_t n) {
  __shared__ T wsum[APC_BLOCK / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
  T v[SCAN_IPT];
  T tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; i++) {
    int64_t idx = base + i;
    v[i] = idx < n ? in[idx] : (T)0;
    tot += v[i];
  }
  T x = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  T wpre = 0;
  for (int k = 0; k < w; k++) wpre += wsum[k];
  T run = wpre + x - tot;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; i++) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (threadIdx.x == APC_BLOCK - 1) bsum[blockIdx.x] = wpre + x;
}

template <typename T>
__global__ void __launch_bounds__(APC_BLOCK) k_scan_add(T *out, const T *boff, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  const T add = boff[blockIdx.x];
  for (int i = threadIdx.x; i < SCAN_TILE; i += APC_BLOCK) {
    int64_t idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

template <typename T>
int scan_rec(const T *in, T *out, int64_t n, hipStream_t s) {
  if (n <= 0) return APC_OK;
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  T *bsum = nullptr;
  HIPCHK(apc_malloc_async((void **)&bsum, (size_t)nb * sizeof(T), s));
  hipLaunchKernelGGL(k_scan_tile<T>, dim3((unsigned)nb), dim3(APC_BLOCK), 0, s, in, out, bsum, n);
  HIPCHK(hipGetLastError());
  if (nb > 1) {
    int rc = scan_rec<T>(bsum, bsum, nb, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)nb), dim3(APC_BLOCK), 0, s, out, bsum, n);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(apc_free_async(bsum, s));
  return APC_OK;
}

__global__ void __launch_bounds__(APC_BLOCK) k_sum_i32(const int32_t *in, int64_t n,
                                                       unsigned long long *acc) {
  int64_t i = (int64_t)blockIdx.x * APC_BLOCK + threadIdx.x;
  long long v = 0;
  for (; i < n; i += (int64_t)gridDim.x * APC_BLOCK) v += in[i];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(acc, (unsigned long long)v);
}

// ---------------------------------------------------------------- radix sort
// Each wavefront owns a tile of RS_TILE consecutive keys.  Pass 1 counts the 8-bit
// digit of every tile; the digit-major table of counts is scanned; pass 2 revisits
// each tile in the same order and places every key at its digit's running offset
// plus its rank among equal digits of lower lanes (ballot match), which keeps the
// sort stable.
constexpr int RS_IPT = 16;
constexpr int RS_TILE = 64 * RS_IPT;
constexpr int RS_WAVES = APC_BLOCK / 64;

__global__ void __launch_bounds__(APC_BLOCK) k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                       int64_t ntiles, int32_t *hist) {
  __shared__ int32_t cnt[RS_WAVES][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * RS_WAVES + w;
  for (int d = lane; d < 256; d += 64) cnt[w][d] = 0;
  __syncthreads();
  if (tile < ntiles) {
    for (int r = 0; r < RS_IPT; r++) {
      int64_t idx = tile * RS_TILE + r * 64 + lane;
      if (idx < n) atomicAdd(&cnt[w][(keys[idx] >> shift) & 255u], 1);
    }
  }
  __syncthreads();
  if (tile < ntiles)
    for (int d = lane; d < 256; d += 64) hist[(int64_t)d * ntiles + tile] = cnt[w][d];
}

__global__ void __launch_bounds__(APC_BLOCK) k_rs_scatter(const uint64_t *kin, const int32_t *vin,
                                                          uint64_t *kout, int32_t *vout, int64_t n,
                                                          int shift, int64_t ntiles,
                                                          const int32_t *offs) {
  __shared__ int32_t run[RS_WAVES][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * RS_WAVES + w;
  if (tile < ntiles)
    for (int d = lane; d < 256; d += 64) run[w][d] = offs[(int64_t)d * ntiles + tile];
  __syncthreads();
  if (tile >= ntiles) return;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int r = 0; r < RS_IPT; r++) {
    const int64_t idx = tile * RS_TILE + r * 64 + lane;
    const bool valid = idx < n;
    const uint64_t key = valid ? kin[idx] : 0ull;
    const int32_t val = valid ? vin[idx] : 0;
    const unsigned d = (unsigned)(key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const int bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int32_t base = run[w][d];
    if (valid) {
      const int32_t pos = base + __popcll(peers & below);
      kout[pos] = key;
      vout[pos] = val;
      if ((peers >> lane) == 1ull) run[w][d] = base + __popcll(peers);
    }
  }
}

} // namespace

int apc_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  return scan_rec<int32_t>(in, out, n, s);
}
int apc_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  return scan_rec<int64_t>(in, out, n, s);
}

int apc_sum_i32(const int32_t *in, int64_t n, int64_t *host_out, hipStream_t s) {
  unsigned long long *acc = nullptr;
  HIPCHK(apc_malloc_async((void **)&acc, sizeof(unsigned long long), s));
  HIPCHK(hipMemsetAsync(acc, 0, sizeof(unsigned long long), s));
  unsigned g = grid_for(n);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_sum_i32, dim3(g), dim3(APC_BLOCK), 0, s, in, n, acc);
  HIPCHK(hipGetLastError());
  unsigned long long h = 0;
  HIPCHK(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(apc_free_async(acc, s));
  *host_out = (int64_t)h;
  return APC_OK;
}

int apc_radix_sort(uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s) {
  if (n <= 1 || bits <= 0) return APC_OK;
  const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
  const unsigned nblk = (unsigned)((ntiles + RS_WAVES - 1) / RS_WAVES);
  uint64_t *k2 = nullptr;
  int32_t *v2 = nullptr, *hist = nullptr;
  HIPCHK(apc_malloc_async((void **)&k2, (size_t)n * sizeof(uint64_t), s));
  HIPCHK(apc_malloc_async((void **)&v2, (size_t)n * sizeof(int32_t), s));
  HIPCHK(apc_malloc_async((void **)&hist, (size_t)ntiles * 256 * sizeof(int32_t), s));
  uint64_t *ka = keys, *kb = k2;
  int32_t *va = vals, *vb = v2;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(APC_BLOCK), 0, s, ka, n, shift, ntiles, hist);
    HIPCHK(hipGetLastError());
    int rc = apc_scan_i32(hist, hist, ntiles * 256, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(APC_BLOCK), 0, s, ka, va, kb, vb, n, shift,
                       ntiles, hist);
    HIPCHK(hipGetLastError());
    uint64_t *tk = ka;
    ka = kb;
    kb = tk;
    int32_t *tv = va;
    va = vb;
    vb = tv;
  }
  if (ka != keys) {
    HIPCHK(hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(vals, va, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(apc_free_async(k2, s));
  HIPCHK(apc_free_async(v2, s));
  HIPCHK(apc_free_async(hist, s));
  return APC_OK;
}

// ---------------------------------------------------------------- temporaries
namespace {
struct TmpCache {
  std::mutex mu;
  // (device, stream) -> size class -> free blocks
  std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void *>> free;
  std::unordered_map<void *, size_t> live; // block -> size class
  size_t cached = 0;
};
TmpCache &tmp_cache() {
  static TmpCache *c = new TmpCache(); // never destroyed: blocks live until process exit
  return *c;
}
constexpr size_t TMP_CACHE_MAX = (size_t)16 << 30;
// sizes round up to a power of two below 2 MiB and to 2 MiB steps above
size_t tmp_class(size_t b) {
  if (b <= 256) return 256;
  if (b < ((size_t)2 << 20)) {
    size_t c = 512;
    while (c < b) c <<= 1;
    return c;
  }
  const size_t g = (size_t)2 << 20;
  return (b + g - 1) / g * g;
}
} // namespace

hipError_t apc_malloc_async(void **p, size_t bytes, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t cls = tmp_class(bytes);
  TmpCache &C = tmp_cache();
  {
    std::lock_guard<std::mutex> lock(C.mu);
    auto f = C.free.find({dev, s});
    if (f != C.free.end()) {
      auto it = f->second.lower_bound(cls);
      // a cached block at most twice the request
      if (it != f->second.end() && it->first <= 2 * cls) {
        *p = it->second;
        C.live[it->second] = it->first;
        C.cached -= it->first;
        f->second.erase(it);
        return hipSuccess;
      }
    }
  }
  e = hipMallocAsync(p, cls, s);
  if (e == hipErrorOutOfMemory) {
    // give this device's cached blocks back, then try once more
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lock(C.mu);
    for (auto &kv : C.free) {
      if (kv.first.first != dev) continue;
      for (auto &b : kv.second) {
        (void)hipFreeAsync(b.second, kv.first.second);
        C.cached -= b.first;
      }
      kv.second.clear();
    }
    (void)hipDeviceSynchronize();
    e = hipMallocAsync(p, cls, s);
  }
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(C.mu);
  C.live[*p] = cls;
  return hipSuccess;
}

hipError_t apc_free_async(void *p, hipStream_t s) {
  if (!p) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  TmpCache &C = tmp_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  auto it = C.live.find(p);
  if (it == C.live.end()) return hipFreeAsync(p, s); // not from apc_malloc_async
  const size_t cls = it->second;
  C.live.erase(it);
  if (C.cached + cls > TMP_CACHE_MAX) return hipFreeAsync(p, s);
  C.free[{dev, s}].insert({cls, p});
  C.cached += cls;
  return hipSuccess;
}

// ---------------------------------------------------------------- persistent arrays
// The arrays a cloud keeps (its structure, operators and solver workspace) come
// from a device-wide cache of freed blocks: apc_dev_free keeps a block for the next
// apc_dev_alloc of its size class on that device instead of calling hipFree, which
// waits for the whole device on every call.  The caller of apc_dev_free guarantees
// that no queued work still uses the block (apc_destroy synchronises the device
// once, then frees every array).  Blocks not from apc_dev_alloc go to hipFree.
namespace {
struct DevCache {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void *>> free;       // device -> size class -> blocks
  std::unordered_map<void *, std::pair<int, size_t>> live; // block -> (device, size class)
  size_t cached = 0;
};
DevCache &dev_cache() {
  static DevCache *c = new DevCache(); // never destroyed: blocks live until process exit
  return *c;
}
constexpr size_t DEV_CACHE_MAX = (size_t)32 << 30;
} // namespace

hipError_t apc_dev_alloc(void **p, size_t bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t cls = tmp_class(bytes);
  DevCache &C = dev_cache();
  {
    std::lock_guard<std::mutex> lock(C.mu);
    auto f = C.free.find(dev);
    if (f != C.free.end()) {
      auto it = f->second.lower_bound(cls);
      if (it != f->second.end() && it->first <= 2 * cls) {
        *p = it->second;
        C.live[it->second] = {dev, it->first};
        C.cached -= it->first;
        f->second.erase(it);
        return hipSuccess;
      }
    }
  }
  e = hipMalloc(p, cls);
  if (e == hipErrorOutOfMemory) {
    // give this device's cached blocks back, then try once more
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lock(C.mu);
    auto f = C.free.find(dev);
    if (f != C.free.end()) {
      for (auto &b : f->second) {
        (void)hipFree(b.second);
        C.cached -= b.first;
      }
      f->second.clear();
    }
    e = hipMalloc(p, cls);
  }
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(C.mu);
  C.live[*p] = {dev, cls};
  return hipSuccess;
}

hipError_t apc_dev_free(void *p) {
  if (!p) return hipSuccess;
  DevCache &C = dev_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  auto it = C.live.find(p);
  if (it == C.live.end()) return hipFree(p); // not from apc_dev_alloc
  const int dev = it->second.first;
  const size_t cls = it->second.second;
  C.live.erase(it);
  if (C.cached + cls > DEV_CACHE_MAX) return hipFree(p);
  C.free[dev].insert({cls, p});
  C.cached += cls;
  return hipSuccess;
}

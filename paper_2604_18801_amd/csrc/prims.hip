// Device-wide primitives for gfx950: exclusive scans (reduce-then-scan, fixed
// order, so results are deterministic) and a stable LSD radix sort whose
// in-tile ranks come from wave64 ballots.
#include "pcc_internal.hpp"

#include <algorithm>
#include <cstdio>

namespace pcc {

void hip_fail(hipError_t e, const char *what, const char *file, int line) {
  char buf[512];
  snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  throw Error(e == hipErrorOutOfMemory ? -2 : -3, buf);
}

// ---------------------------------------------------------------------------
// arena
// ---------------------------------------------------------------------------
std::atomic<int64_t> g_alloc_fail_after{-1};

Arena::~Arena() { release(); }

void Arena::release() {
  if (!fixed_)
    for (auto &c : chunks_) hipFree(c.base);
  chunks_.clear();
  used_ = 0;
  fixed_ = false;
}

void Arena::attach(void *base, size_t bytes) {
  release();
  chunks_.push_back({(char *)base, bytes, 0});
  fixed_ = true;
  high_ = 0;
}

void Arena::reset() {
  high_ = 0;
  if (fixed_) {
    chunks_[0].off = 0;
    used_ = 0;
    return;
  }
  size_t total = 0;
  for (auto &c : chunks_) total += c.size;
  // Consolidate into one chunk big enough for the previous call, unless that
  // is huge: freeing and mapping tens of GB again costs seconds, and a call
  // of the same size fills the chunks it left behind in the same order
  // without allocating.
  if (chunks_.size() > 1 && total <= ((size_t)16 << 30)) {
    release();
    void *p = nullptr;
    if (hipMalloc(&p, total) == hipSuccess) chunks_.push_back({(char *)p, total, 0});
  }
  for (auto &c : chunks_) c.off = 0;
  used_ = 0;
}

void *Arena::alloc(size_t bytes) {
  if (g_alloc_fail_after.load() >= 0 && g_alloc_fail_after.fetch_sub(1) == 0)
    throw Error(-2, "device allocation failed (injected by pcc_debug_set)");
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes == 0) bytes = 256;
  for (auto &c : chunks_) {
    if (c.size - c.off >= bytes) {
      void *p = c.base + c.off;
      c.off += bytes;
      used_ += bytes;
      high_ = std::max(high_, used_);
      return p;
    }
  }
  if (fixed_)
    throw Error(-2, "the static scratch buffer is exhausted (" + std::to_string(bytes) +
                        " more bytes needed)");
  size_t last = chunks_.empty() ? 0 : chunks_.back().size;
  size_t sz = std::max(bytes, std::max(last, (size_t)64 << 20));
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (sz > bytes) {
      sz = bytes;
      e = hipMalloc(&p, sz);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(-2, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  chunks_.push_back({(char *)p, sz, bytes});
  used_ += bytes;
  high_ = std::max(high_, used_);
  return p;
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T *p, T v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_iota(uint32_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
  if (n) k_fill<uint32_t><<<blocks_for(n, 256, 65536), 256, 0, s>>>(p, v, n);
}
void fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s) {
  if (n) k_fill<uint64_t><<<blocks_for(n, 256, 65536), 256, 0, s>>>(p, v, n);
}
void fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t s) {
  if (n) k_fill<uint8_t><<<blocks_for(n, 256, 65536), 256, 0, s>>>(p, v, n);
}
void iota_u32(uint32_t *p, size_t n, hipStream_t s) {
  if (n) k_iota<<<blocks_for(n, 256, 65536), 256, 0, s>>>(p, n);
}

// ---------------------------------------------------------------------------
// scans
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr size_t kScanTile = (size_t)kScanThreads * kScanItems;

template <typename T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T u = __shfl_up(v, d, kWave);
    if (lane >= d) v += u;
  }
  return v;
}

// exclusive scan of one value per thread over a 256-thread block
template <typename T>
__device__ inline T block_excl_scan(T v, T &total, T *lds) {
  T inc = wave_incl_scan(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == kWave - 1) lds[w] = inc;
  __syncthreads();
  T woff = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / kWave; ++k) {
    if (k < w) woff += lds[k];
    tot += lds[k];
  }
  total = tot;
  __syncthreads();
  return woff + inc - v;
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const Tin *in, size_t n, Tout *part) {
  __shared__ Tout lds[kScanThreads / kWave];
  const size_t base = (size_t)blockIdx.x * kScanTile;
  Tout acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    size_t idx = base + (size_t)i * kScanThreads + threadIdx.x;
    if (idx < n) acc += (Tout)in[idx];
  }
  Tout tot;
  block_excl_scan<Tout>(acc, tot, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const Tin *in, Tout *out, size_t n,
                                                            const Tout *block_off, Tout *total,
                                                            size_t nblocks) {
  __shared__ Tout lds[kScanThreads / kWave];
  const size_t base = (size_t)blockIdx.x * kScanTile;
  Tout run = block_off ? block_off[blockIdx.x] : (Tout)0;
#pragma unroll 1
  for (int i = 0; i < kScanItems; ++i) {
    size_t idx = base + (size_t)i * kScanThreads + threadIdx.x;
    Tout v = idx < n ? (Tout)in[idx] : (Tout)0;
    Tout tot;
    Tout ex = block_excl_scan<Tout>(v, tot, lds);
    if (idx < n) out[idx] = run + ex;
    run += tot;
  }
  if (total && blockIdx.x == nblocks - 1 && threadIdx.x == 0) *total = run;
}

template <typename Tin, typename Tout>
static void scan_impl(const Tin *in, Tout *out, size_t n, Tout *total, Arena &ar, hipStream_t s) {
  if (n == 0) {
    if (total) k_fill<Tout><<<1, 64, 0, s>>>(total, (Tout)0, 1);
    return;
  }
  size_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    k_scan_down<Tin, Tout><<<1, kScanThreads, 0, s>>>(in, out, n, nullptr, total, 1);
    return;
  }
  Tout *part = ar.get<Tout>(nb);
  k_scan_reduce<Tin, Tout><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, part);
  scan_impl<Tout, Tout>(part, part, nb, (Tout *)nullptr, ar, s);
  k_scan_down<Tin, Tout><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, part, total, nb);
}

void scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, uint64_t *total, Arena &ar,
                  hipStream_t s) {
  scan_impl<uint32_t, uint64_t>(in, out, n, total, ar, s);
}
// Byte counts (flags) to 32-bit offsets, the common case: every thread takes
// 16 consecutive bytes with one 16-byte load and writes their 16 offsets with
// four 16-byte stores, so a block scans 4096 items with one block-wide scan.
constexpr int kScan8Items = 16;
constexpr size_t kScan8Tile = (size_t)kScanThreads * kScan8Items;

__device__ inline void load16(const uint8_t *in, size_t base, size_t n, uint32_t (&b)[16]) {
  if (base + 16 <= n) {
    const uint4 v = *reinterpret_cast<const uint4 *>(in + base);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 16; ++i) b[i] = (w[i >> 2] >> (8 * (i & 3))) & 0xffu;
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) b[i] = base + i < n ? (uint32_t)in[base + i] : 0u;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan8_reduce(const uint8_t *in, size_t n,
                                                               uint32_t *part) {
  __shared__ uint32_t lds[kScanThreads / kWave];
  uint32_t b[16];
  load16(in, (size_t)blockIdx.x * kScan8Tile + (size_t)threadIdx.x * 16, n, b);
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc += b[i];
  uint32_t tot;
  block_excl_scan<uint32_t>(acc, tot, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan8_down(const uint8_t *in, uint32_t *out,
                                                             size_t n, const uint32_t *block_off,
                                                             uint32_t *total, size_t nblocks) {
  __shared__ uint32_t lds[kScanThreads / kWave];
  const size_t base = (size_t)blockIdx.x * kScan8Tile + (size_t)threadIdx.x * 16;
  uint32_t b[16];
  load16(in, base, n, b);
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t v = b[i];
    b[i] = acc;  // exclusive prefix inside the thread's 16
    acc += v;
  }
  uint32_t tot;
  const uint32_t run = (block_off ? block_off[blockIdx.x] : 0u) + block_excl_scan<uint32_t>(acc, tot, lds);
  if (base + 16 <= n) {
    uint4 *o = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      o[i] = make_uint4(run + b[4 * i], run + b[4 * i + 1], run + b[4 * i + 2], run + b[4 * i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (base + i < n) out[base + i] = run + b[i];
  }
  if (total && blockIdx.x == nblocks - 1 && threadIdx.x == kScanThreads - 1)
    *total = (block_off ? block_off[blockIdx.x] : 0u) + tot;
}

void scan_u8_u32(const uint8_t *in, uint32_t *out, size_t n, uint32_t *total, Arena &ar,
                 hipStream_t s) {
  if (n == 0 || ((uintptr_t)in & 15u) || ((uintptr_t)out & 15u)) {
    scan_impl<uint8_t, uint32_t>(in, out, n, total, ar, s);
    return;
  }
  const size_t nb = (n + kScan8Tile - 1) / kScan8Tile;
  if (nb == 1) {
    k_scan8_down<<<1, kScanThreads, 0, s>>>(in, out, n, nullptr, total, 1);
    return;
  }
  uint32_t *part = ar.get<uint32_t>(nb);
  k_scan8_reduce<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, part);
  scan_impl<uint32_t, uint32_t>(part, part, nb, (uint32_t *)nullptr, ar, s);
  k_scan8_down<<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, part, total, nb);
}
void scan_u32_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *total, Arena &ar,
                  hipStream_t s) {
  scan_impl<uint32_t, uint32_t>(in, out, n, total, ar, s);
}
void scan_u64_u64(const uint64_t *in, uint64_t *out, size_t n, uint64_t *total, Arena &ar,
                  hipStream_t s) {
  scan_impl<uint64_t, uint64_t>(in, out, n, total, ar, s);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr size_t kSortTile = (size_t)kSortThreads * kSortItems;
constexpr int kRadix = 256;

__global__ void __launch_bounds__(kSortThreads)
k_sort_hist(const uint32_t *keys, size_t n, int shift, uint32_t mask, uint32_t *counts,
            size_t nblocks) {
  __shared__ uint32_t hist[kRadix];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int i = 0; i < kSortItems; ++i) {
    size_t idx = base + (size_t)i * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&hist[(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  counts[(size_t)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

// Items of a tile are taken in index order (round i, then thread); within a
// round the rank of a key among equal digits is its lane rank inside its
// wave (ballot match) plus the counts of earlier waves, plus the counts of
// earlier rounds: a stable order.  The tile is then reordered by digit in
// LDS and written out in that order, so the items of one digit (a run of
// consecutive output positions) leave in consecutive lanes: whole cache
// lines instead of one scattered word per digit and round.
__global__ void __launch_bounds__(kSortThreads)
k_sort_scatter(const uint32_t *keys, const uint32_t *vals, uint32_t *okeys, uint32_t *ovals,
               size_t n, int shift, int nbits, const uint32_t *offsets, size_t nblocks) {
  __shared__ uint32_t base_off[kRadix];
  __shared__ uint32_t run[kRadix];
  __shared__ uint32_t tstart[kRadix];
  __shared__ uint32_t wcnt[kSortThreads / kWave][kRadix];
  __shared__ uint32_t scan_lds[kSortThreads / kWave];
  __shared__ uint32_t lk[kSortTile], lv[kSortTile];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const uint32_t mask = (1u << nbits) - 1u;
  base_off[t] = offsets[(size_t)t * nblocks + blockIdx.x];
  run[t] = 0;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const size_t base = (size_t)blockIdx.x * kSortTile;
  const uint32_t tile_n = (uint32_t)(n - base < kSortTile ? n - base : kSortTile);
  uint32_t key[kSortItems], val[kSortItems], rk[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const size_t idx = base + (size_t)i * kSortThreads + t;
    key[i] = idx < n ? keys[idx] : 0u;
    val[i] = idx < n ? vals[idx] : 0u;
  }
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
#pragma unroll
    for (int k = 0; k < kSortThreads / kWave; ++k) wcnt[k][t] = 0;
    __syncthreads();
    const bool valid = (uint32_t)(i * kSortThreads + t) < tile_n;
    const uint32_t d = (key[i] >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < nbits; ++bit) {
      const uint64_t bm = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? bm : ~bm;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    const int leader = 63 - __clzll(peers);
    if (valid && lane == leader) wcnt[w][d] = cnt;
    __syncthreads();
    // rank among the tile's items of digit d that come before this one
    uint32_t r = run[d] + rank;
    for (int k = 0; k < w; ++k) r += wcnt[k][d];
    rk[i] = r;
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int k = 0; k < kSortThreads / kWave; ++k) add += wcnt[k][t];
    run[t] += add;
  }
  __syncthreads();
  // first tile slot of each digit
  uint32_t tot;
  tstart[t] = block_excl_scan<uint32_t>(run[t], tot, scan_lds);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    if ((uint32_t)(i * kSortThreads + t) < tile_n) {
      const uint32_t d = (key[i] >> shift) & mask;
      const uint32_t at = tstart[d] + rk[i];
      lk[at] = key[i];
      lv[at] = val[i];
    }
  }
  __syncthreads();
  for (uint32_t at = t; at < tile_n; at += kSortThreads) {
    const uint32_t k2 = lk[at];
    const uint32_t d = (k2 >> shift) & mask;
    const uint32_t pos = base_off[d] + (at - tstart[d]);
    okeys[pos] = k2;
    ovals[pos] = lv[at];
  }
}

void radix_sort_u32(uint32_t *keys, uint32_t *vals, size_t n, int bits, Arena &ar,
                    hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  if (n > 0xffffffffull) throw Error(-6, "radix sort of more than 2^32 - 1 elements");
  size_t nb = (n + kSortTile - 1) / kSortTile;
  uint32_t *k2 = ar.get<uint32_t>(n);
  uint32_t *v2 = ar.get<uint32_t>(n);
  uint32_t *counts = ar.get<uint32_t>(nb * kRadix);
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  for (int shift = 0; shift < bits; shift += 8) {
    int nbits = std::min(8, bits - shift);
    uint32_t mask = (1u << nbits) - 1u;
    k_sort_hist<<<(unsigned)nb, kSortThreads, 0, s>>>(ka, n, shift, mask, counts, nb);
    scan_u32_u32(counts, counts, nb * kRadix, nullptr, ar, s);
    k_sort_scatter<<<(unsigned)nb, kSortThreads, 0, s>>>(ka, va, kb, vb, n, shift, nbits, counts,
                                                         nb);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    PCC_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    PCC_HIP(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace pcc

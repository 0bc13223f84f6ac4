// sort.hip -- device scan and stable LSD radix sort for gfx950 (wave64).
//
// Radix sort: 8-bit digits, one histogram kernel and one scatter kernel per
// pass.  A block owns a tile of rs_tile<K>() consecutive keys (4096 32-bit or
// 2048 64-bit keys).  The scatter keeps the input order of equal digits
// (stability) by ranking the tile's keys round by round (256 keys per round,
// in index order) with wave64 ballots for the within-wave rank and LDS
// counters across the block's waves; the ranked keys are placed in LDS in
// digit order and then written out by consecutive threads to consecutive
// addresses of each digit's output run, so that the global writes are
// coalesced.
#include "internal.h"

namespace ts {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;
constexpr int kWaves = kThreads / 64;
// keys per thread of a radix tile: 16 for 32-bit keys, 8 for 64-bit keys
// (the scatter stages a whole tile of keys and values in LDS)
template <class K>
constexpr int rs_items() { return sizeof(K) == 8 ? 8 : 16; }
template <class K>
constexpr int rs_tile() { return kThreads * rs_items<K>(); }

// ---------------------------------------------------------------- scan

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  // inclusive scan within the wave (wave64)
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int w = 0; w < kWaves; ++w) {
      uint32_t t = lds[w];
      lds[w] = acc;
      acc += t;
    }
    lds[kWaves] = acc;
  }
  __syncthreads();
  const uint32_t res = x - v + lds[wave];
  *total = lds[kWaves];
  __syncthreads();
  return res;
}

__global__ void __launch_bounds__(kThreads) scan_block_sums(const uint32_t* in, size_t n,
                                                            uint32_t* sums) {
  __shared__ uint32_t lds[kWaves + 1];
  const size_t base = size_t(blockIdx.x) * kTile + size_t(threadIdx.x) * kItems;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t total;
  block_exclusive_scan(s, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads) scan_apply(const uint32_t* in, uint32_t* out,
                                                       size_t n, const uint32_t* block_off) {
  __shared__ uint32_t lds[kWaves + 1];
  const size_t base = size_t(blockIdx.x) * kTile + size_t(threadIdx.x) * kItems;
  uint32_t v[kItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t acc = block_exclusive_scan(s, lds, &total) + (block_off ? block_off[blockIdx.x] : 0u);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (base + i < n) out[base + i] = acc;
    acc += v[i];
  }
}

// ---------------------------------------------------------------- radix

template <class K>
__global__ void __launch_bounds__(kThreads) rs_hist(const K* keys, size_t n, int shift,
                                                    uint32_t* hist, int nblocks) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  constexpr int kRsItems = rs_items<K>();
  const size_t base = size_t(blockIdx.x) * rs_tile<K>();
#pragma unroll
  for (int i = 0; i < kRsItems; ++i) {
    const size_t idx = base + size_t(i) * kThreads + threadIdx.x;
    if (idx < n) atomicAdd(&cnt[uint32_t(keys[idx] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[size_t(threadIdx.x) * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// offsets[d * nblocks + b]: first output position of digit d's keys of tile b
template <class K>
__global__ void __launch_bounds__(kThreads) rs_scatter(const K* kin, const uint32_t* vin,
                                                       K* kout, uint32_t* vout, size_t n,
                                                       int shift, const uint32_t* offsets,
                                                       int nblocks) {
  constexpr int kRsItems = rs_items<K>();
  constexpr int kRsTile = rs_tile<K>();
  __shared__ K lk[kRsTile];
  __shared__ uint32_t lv[kRsTile];
  __shared__ uint32_t start[256];    // first tile slot of each digit
  __shared__ uint32_t running[256];  // keys of each digit placed so far
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t scan_tmp[kWaves + 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const size_t base = size_t(blockIdx.x) * kRsTile;
  const int tile_n = int(n - base < size_t(kRsTile) ? n - base : size_t(kRsTile));
  K key[kRsItems];
  uint32_t val[kRsItems];
  running[threadIdx.x] = 0;  // the tile's digit histogram first
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    const size_t idx = base + size_t(r) * kThreads + threadIdx.x;
    key[r] = idx < n ? kin[idx] : K(0);
    val[r] = idx < n ? vin[idx] : 0u;
    if (idx < n) atomicAdd(&running[uint32_t(key[r] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  uint32_t total;
  start[threadIdx.x] = block_exclusive_scan(running[threadIdx.x], scan_tmp, &total);
  running[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const bool valid = r * kThreads + int(threadIdx.x) < tile_n;
    const uint32_t d = uint32_t(key[r] >> shift) & 0xFFu;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank_in_wave = __popcll(peers & lt_mask);
    if (valid && rank_in_wave == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = start[d] + running[d] + rank_in_wave;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      lk[pos] = key[r];
      lv[pos] = val[r];
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) add += wcnt[w][threadIdx.x];
    running[threadIdx.x] += add;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < tile_n; p += kThreads) {
    const K k = lk[p];
    const uint32_t d = uint32_t(k >> shift) & 0xFFu;
    const size_t g = size_t(offsets[size_t(d) * nblocks + blockIdx.x]) + size_t(p - int(start[d]));
    if (g < n) {
      kout[g] = k;
      vout[g] = lv[p];
    }
  }
}

__global__ void copy_u32(const uint32_t* a, uint32_t* b, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}
__global__ void copy_u64(const uint64_t* a, uint64_t* b, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

template <class A>
void scan_impl(A& ws, const uint32_t* in, uint32_t* out, size_t n, hipStream_t s, int depth) {
  if (n == 0) return;
  const size_t nblocks = (n + kTile - 1) / kTile;
  if (nblocks == 1) {
    scan_apply<<<1, kThreads, 0, s>>>(in, out, n, nullptr);
    TS_HIP(hipGetLastError());
    return;
  }
  uint32_t* sums = ws.template get<uint32_t>("scan.sums" + std::to_string(depth), nblocks);
  scan_block_sums<<<unsigned(nblocks), kThreads, 0, s>>>(in, n, sums);
  scan_impl(ws, sums, sums, nblocks, s, depth + 1);
  scan_apply<<<unsigned(nblocks), kThreads, 0, s>>>(in, out, n, sums);
  TS_HIP(hipGetLastError());
}

template <class K, class A>
void radix_sort_impl(A& ws, K* keys, uint32_t* vals, size_t n, int begin_bit,
                     int end_bit, hipStream_t s, const char* tag) {
  if (n <= 1 || end_bit <= begin_bit) return;
  const int nblocks = int((n + rs_tile<K>() - 1) / rs_tile<K>());
  std::string t(tag);
  K* ktmp = ws.template get<K>(t + ".k", n);
  uint32_t* vtmp = ws.template get<uint32_t>(t + ".v", n);
  uint32_t* hist = ws.template get<uint32_t>(t + ".h", size_t(256) * nblocks);
  K* kin = keys;
  uint32_t* vin = vals;
  K* kout = ktmp;
  uint32_t* vout = vtmp;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    rs_hist<K><<<nblocks, kThreads, 0, s>>>(kin, n, shift, hist, nblocks);
    scan_impl(ws, hist, hist, size_t(256) * nblocks, s, 0);
    rs_scatter<K><<<nblocks, kThreads, 0, s>>>(kin, vin, kout, vout, n, shift, hist, nblocks);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  if (kin != keys) {
    const int b = int((n + 255) / 256);
    if (sizeof(K) == 8)
      copy_u64<<<b, 256, 0, s>>>(reinterpret_cast<const uint64_t*>(kin),
                                 reinterpret_cast<uint64_t*>(keys), n);
    else
      copy_u32<<<b, 256, 0, s>>>(reinterpret_cast<const uint32_t*>(kin),
                                 reinterpret_cast<uint32_t*>(keys), n);
    copy_u32<<<b, 256, 0, s>>>(vin, vals, n);
  }
  TS_HIP(hipGetLastError());
}

}  // namespace

void scan_exclusive_u32(Workspace& ws, const uint32_t* in, uint32_t* out, size_t n,
                        hipStream_t s) {
  scan_impl(ws, in, out, n, s, 0);
}

void radix_sort_u64(Workspace& ws, uint64_t* keys, uint32_t* vals, size_t n, int begin_bit,
                    int end_bit, hipStream_t s) {
  radix_sort_impl<uint64_t>(ws, keys, vals, n, begin_bit, end_bit, s, "rs64");
}

void radix_sort_u32(Workspace& ws, uint32_t* keys, uint32_t* vals, size_t n, int begin_bit,
                    int end_bit, hipStream_t s) {
  radix_sort_impl<uint32_t>(ws, keys, vals, n, begin_bit, end_bit, s, "rs32");
}

void radix_sort_u32(Arena& arena, uint32_t* keys, uint32_t* vals, size_t n, int begin_bit,
                    int end_bit, hipStream_t s) {
  radix_sort_impl<uint32_t>(arena, keys, vals, n, begin_bit, end_bit, s, "rs32");
}

}  // namespace ts

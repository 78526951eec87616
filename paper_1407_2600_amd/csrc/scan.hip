// Device-wide exclusive prefix sum of uint32 values (reduce, scan the block
// totals, scan again with the block offsets).  Used for the radix-sort digit
// offsets, the tree-level child offsets, sink-group numbering and the
// interaction-list offsets.
#include "hot_internal.h"

namespace hot {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// exclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total to *tot
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* tot) {
  __shared__ uint32_t wsum[kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t off = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    uint32_t s = wsum[w];
    off += (w < wid) ? s : 0u;
    all += s;
  }
  __syncthreads();
  *tot = all;
  return off + inc - v;
}

__global__ void __launch_bounds__(kThreads) k_reduce(const uint32_t* __restrict__ in, size_t n,
                                                     size_t chunk, uint32_t* __restrict__ bsum) {
  size_t beg = (size_t)blockIdx.x * chunk;
  size_t end = beg + chunk < n ? beg + chunk : n;
  uint32_t s = 0;
  for (size_t i = beg + threadIdx.x; i < end; i += kThreads) s += in[i];
  // block reduction
  __shared__ uint32_t red[kThreads];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) k_top(uint32_t* __restrict__ bsum, int nb,
                                              uint32_t* __restrict__ total) {
  __shared__ uint32_t wsum[16];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  uint32_t v = t < nb ? bsum[t] : 0u;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t off = 0, all = 0;
  for (int w = 0; w < 16; ++w) {
    off += (w < wid) ? wsum[w] : 0u;
    all += wsum[w];
  }
  if (t < nb) bsum[t] = off + inc - v;
  if (t == 0 && total) *total = all;
}

__global__ void __launch_bounds__(kThreads) k_down(const uint32_t* in, uint32_t* out, size_t n,
                                                   size_t chunk,
                                                   const uint32_t* __restrict__ bsum) {
  size_t beg = (size_t)blockIdx.x * chunk;
  size_t end = beg + chunk < n ? beg + chunk : n;
  uint32_t carry = bsum[blockIdx.x];
  for (size_t t0 = beg; t0 < end; t0 += kTile) {
    uint32_t v[kItems];
    uint32_t loc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      size_t i = t0 + (size_t)threadIdx.x * kItems + k;
      v[k] = i < end ? in[i] : 0u;
      loc += v[k];
    }
    uint32_t tot;
    uint32_t pre = block_excl_scan(loc, &tot) + carry;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      size_t i = t0 + (size_t)threadIdx.x * kItems + k;
      if (i < end) out[i] = pre;
      pre += v[k];
    }
    carry += tot;
  }
}

}  // namespace

hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint32_t* total, size_t n,
                    uint32_t* block_sums, hipStream_t s) {
  if (n == 0) {
    if (total) return hipMemsetAsync(total, 0, sizeof(uint32_t), s);
    return hipSuccess;
  }
  int nb = (int)((n + kTile - 1) / kTile);
  if (nb > kScanBlocks) nb = kScanBlocks;
  size_t chunk = (n + nb - 1) / nb;
  chunk = (chunk + kTile - 1) / kTile * kTile;
  nb = (int)((n + chunk - 1) / chunk);
  k_reduce<<<nb, kThreads, 0, s>>>(in, n, chunk, block_sums);
  k_top<<<1, 1024, 0, s>>>(block_sums, nb, total);
  k_down<<<nb, kThreads, 0, s>>>(in, out, n, chunk, block_sums);
  return hipGetLastError();
}

}  // namespace hot

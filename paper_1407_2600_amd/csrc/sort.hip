// Morton keys and the key sort (paper Sec. 2.1: each particle gets a Key from
// Morton ordering, and the domain decomposition is a sort of the keys).
//
// Keys: positions wrap into [0, L) by one add or subtract of L, quantise as
// floor(x * (2^21 / L)) clamped to 2^21 - 1, and interleave with x the most
// significant bit of each octal digit, under a placeholder bit 63 so that a
// cell's key at level l is key >> 3(21 - l), its parent key >> 3 and its
// daughters key << 3 | octant.
//
// Sort: least-significant-digit radix sort of (key, index) with 8-bit digits.
// Each pass builds per-tile digit histograms in LDS, scans them digit-major
// across tiles, and scatters with a stable in-tile rank computed from wave
// ballots, so equal keys keep their original order; each tile is put in
// digit order in LDS first and written out run by run.
#include "hot_internal.h"

namespace hot {

__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  // place bit b of a 21-bit value at bit 3b
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x001f00000000ffffull;
  v = (v | (v << 16)) & 0x001f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ __forceinline__ double wrap_box(double x, double L) {
  if (x < 0.0) x += L;
  if (x >= L) x -= L;
  return x;
}

__device__ __forceinline__ uint32_t quantise(double xw, double S) {
  double t = xw * S;
  uint32_t q = (uint32_t)t;
  return q > 2097151u ? 2097151u : q;
}

__global__ void __launch_bounds__(256) k_keys(const double* __restrict__ pos, size_t n, double L,
                                              double S, uint64_t* __restrict__ key,
                                              uint32_t* __restrict__ idx,
                                              uint32_t* __restrict__ bad) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
  bool ok = (x > -L) && (x < 2.0 * L) && (y > -L) && (y < 2.0 * L) && (z > -L) && (z < 2.0 * L);
  if (!ok) atomicOr(bad, 1u);  // also catches NaN (comparisons are false)
  x = wrap_box(x, L);
  y = wrap_box(y, L);
  z = wrap_box(z, L);
  uint64_t k = (1ull << 63) | (spread3(quantise(x, S)) << 2) | (spread3(quantise(y, S)) << 1) |
               spread3(quantise(z, S));
  key[i] = k;
  idx[i] = (uint32_t)i;
}

// ---------------------------------------------------------------- radix sort
namespace {
constexpr int kT = 256;
constexpr int kRounds = kSortTile / kT;

__global__ void __launch_bounds__(kT) k_hist(const uint64_t* __restrict__ key, size_t n, int shift,
                                             uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t h[kSortBins];
  h[threadIdx.x] = 0;
  __syncthreads();
  size_t beg = (size_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kRounds; ++r) {
    size_t i = beg + (size_t)r * kT + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & (kSortBins - 1)], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one tile: stable tile-local ranks (wave ballots, per-wave digit
// counts) place the tile's keys in LDS in digit order; the tile is then
// written out in that order, so consecutive threads write consecutive
// addresses of each digit's run in the output.
__global__ void __launch_bounds__(kT) k_scatter(const uint64_t* __restrict__ kin,
                                                const uint32_t* __restrict__ vin, size_t n,
                                                int shift, const uint32_t* __restrict__ off,
                                                int nblk, uint64_t* __restrict__ kout,
                                                uint32_t* __restrict__ vout) {
  __shared__ uint32_t base[kSortBins];  // output offset of this tile's digit d
  __shared__ uint32_t loff[kSortBins];  // tile-local offset of digit d, advanced per round
  __shared__ uint32_t lbeg[kSortBins];  // tile-local offset of digit d
  __shared__ uint32_t wcnt[kT / 64][kSortBins];
  __shared__ uint64_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const size_t beg = (size_t)blockIdx.x * kSortTile;
  const uint32_t tn = (uint32_t)(n - beg < (size_t)kSortTile ? n - beg : (size_t)kSortTile);
  // this tile's count of digit t: the next entry of the digit-major scanned
  // histogram (the same digit's next tile, or the next digit's first tile)
  const size_t e = (size_t)t * nblk + blockIdx.x;
  const uint32_t o0 = off[e];
  const uint32_t o1 = (e + 1 < (size_t)kSortBins * nblk) ? off[e + 1] : (uint32_t)n;
  base[t] = o0;
  // exclusive scan of the counts over the 256 digits (one per thread)
  uint32_t c = o1 - o0;
  wcnt[0][t] = c;
  __syncthreads();
  for (int d = 1; d < kSortBins; d <<= 1) {
    const uint32_t u = t >= d ? wcnt[0][t - d] : 0u;
    __syncthreads();
    c += u;
    wcnt[0][t] = c;
    __syncthreads();
  }
  loff[t] = c - (o1 - o0);
  lbeg[t] = c - (o1 - o0);
  for (int w = 0; w < kT / 64; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t li = (uint32_t)(r * kT + t);
    const bool valid = li < tn;
    const uint64_t k = valid ? kin[beg + li] : 0ull;
    const uint32_t v = valid ? vin[beg + li] : 0u;
    const uint32_t d = valid ? (uint32_t)((k >> shift) & (kSortBins - 1)) : 0u;
    // lanes of this wave with the same digit
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kSortBits; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      same &= ((d >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(same & below);
    const bool leader = valid && ((same & below) == 0ull);
    if (leader) wcnt[wid][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pre = loff[d];
      for (int w = 0; w < wid; ++w) pre += wcnt[w][d];
      sk[pre + rank] = k;
      sv[pre + rank] = v;
    }
    __syncthreads();
    // advance the per-digit tile offsets and clear the wave counts
    uint32_t add = 0;
    for (int w = 0; w < kT / 64; ++w) {
      add += wcnt[w][t];
      wcnt[w][t] = 0;
    }
    loff[t] += add;
    __syncthreads();
  }
  for (uint32_t j = (uint32_t)t; j < tn; j += kT) {
    const uint64_t k = sk[j];
    const uint32_t d = (uint32_t)((k >> shift) & (kSortBins - 1));
    const size_t dst = (size_t)base[d] + (j - lbeg[d]);
    kout[dst] = k;
    vout[dst] = sv[j];
  }
}
}  // namespace

// Sort (key, idx) ascending by key, stable.  Buffers a and b alternate; the
// result ends in buffer 0 after an even number of passes (8).
hipError_t radix_sort(uint64_t* key0, uint32_t* idx0, uint64_t* key1, uint32_t* idx1, size_t n,
                      uint32_t* hist, uint32_t* scan_tmp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int nblk = (int)((n + kSortTile - 1) / kSortTile);
  uint64_t* kin = key0;
  uint32_t* vin = idx0;
  uint64_t* kout = key1;
  uint32_t* vout = idx1;
  for (int pass = 0; pass < 8; ++pass) {
    int shift = pass * kSortBits;
    k_hist<<<nblk, kT, 0, s>>>(kin, n, shift, hist, nblk);
    hipError_t e = scan_u32(hist, hist, nullptr, (size_t)kSortBins * nblk, scan_tmp, s);
    if (e != hipSuccess) return e;
    k_scatter<<<nblk, kT, 0, s>>>(kin, vin, n, shift, hist, nblk, kout, vout);
    uint64_t* tk = kin;
    kin = kout;
    kout = tk;
    uint32_t* tv = vin;
    vin = vout;
    vout = tv;
  }
  return hipGetLastError();
}

// sorted, wrapped FP64 positions and FP64 masses
template <typename MT>
__global__ void __launch_bounds__(256) k_gather(const double* __restrict__ pos,
                                                const MT* __restrict__ mass, size_t n, double L,
                                                const uint32_t* __restrict__ idx,
                                                double* __restrict__ spos,
                                                double* __restrict__ smass,
                                                uint32_t* __restrict__ bad) {
  size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t i = idx[s];
  spos[s] = wrap_box(pos[i], L);
  spos[n + s] = wrap_box(pos[n + i], L);
  spos[2 * n + s] = wrap_box(pos[2 * n + i], L);
  double m = (double)mass[i];
  if (!(m >= 0.0) || m == __builtin_inf()) atomicOr(bad, 2u);
  smass[s] = m;
}

hipError_t launch_keys(const double* pos, size_t n, double L, double S, uint64_t* key,
                       uint32_t* idx, uint32_t* bad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(pos, n, L, S, key, idx, bad);
  return hipGetLastError();
}

hipError_t launch_gather(const double* pos, const void* mass, bool fp32, size_t n, double L,
                         const uint32_t* idx, double* spos, double* smass, uint32_t* bad,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  unsigned g = (unsigned)((n + 255) / 256);
  if (fp32)
    k_gather<float><<<g, 256, 0, s>>>(pos, (const float*)mass, n, L, idx, spos, smass, bad);
  else
    k_gather<double><<<g, 256, 0, s>>>(pos, (const double*)mass, n, L, idx, spos, smass, bad);
  return hipGetLastError();
}

}  // namespace hot

// Morton keys and the key sort (paper Sec. 2.1: each particle gets a Key from
// Morton ordering, and the domain decomposition is a sort of the keys).
//
// Keys: positions wrap into [0, L) by one add or subtract of L, quantise as
// floor(x * (2^21 / L)) clamped to 2^21 - 1, and interleave with x the most
// significant bit of each octal digit, under a placeholder bit 63 so that a
// cell's key at level l is key >> 3(21 - l), its parent key >> 3 and its
// daughters key << 3 | octant.
//
// Sort: least-significant-digit radix sort of (key, index) with 9-bit digits
// over bits 0..62 (7 passes; the placeholder bit is the same in every key).
// Each pass builds per-tile digit histograms in LDS, scans them digit-major
// across tiles, and scatters with a stable in-tile rank computed from wave
// ballots and per-wavefront digit counts, so equal keys keep their original
// order; each tile is put in digit order in LDS first and written out run by
// run.
#include "device_math.h"

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
constexpr int kDPT = kSortBins / kT;  // digits per thread, consecutive
// bit 63 (the placeholder) is the same in every key: the passes cover bits
// 0..62
constexpr int kPasses = (63 + kSortBits - 1) / kSortBits;
static_assert(kSortBins % kT == 0, "each thread owns whole digits");
static_assert(kPasses % 2 == 1, "the last pass writes the second buffer pair");

__global__ void __launch_bounds__(kT) k_hist(const uint64_t* __restrict__ key, size_t n, int shift,
                                             uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t h[kSortBins];
  for (int d = threadIdx.x; d < kSortBins; d += kT) h[d] = 0;
  __syncthreads();
  size_t beg = (size_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kRounds; ++r) {
    size_t i = beg + (size_t)r * kT + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & (kSortBins - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kSortBins; d += kT) hist[(size_t)d * nblk + blockIdx.x] = h[d];
}

// Scatter of one tile.  Each wavefront takes a contiguous quarter of the
// tile (16 rounds of 64 keys) and counts its keys per digit in a row of its
// own (wave ballots find the lanes with the same digit; one leader per digit
// adds), with no block barrier between rounds.  The digit offsets within the
// tile (from the scanned histogram) and the rows give each wavefront's
// starting offset per digit; the wavefronts then place their keys in LDS in
// digit order (stable: earlier rounds, then lower lanes, then lower
// wavefronts first), and the tile is written out run by run, so consecutive
// threads write consecutive addresses of each digit's run in the output.
__global__ void __launch_bounds__(kT) k_scatter(const uint64_t* __restrict__ kin,
                                                const uint32_t* __restrict__ vin, size_t n,
                                                int shift, const uint32_t* __restrict__ off,
                                                int nblk, uint64_t* __restrict__ kout,
                                                uint32_t* __restrict__ vout) {
  constexpr int kWaves = kT / 64, kPerWave = kSortTile / kWaves, kWR = kPerWave / 64;
  __shared__ uint32_t base[kSortBins];  // output offset of this tile's digit d
  __shared__ uint32_t lbeg[kSortBins];  // tile-local offset of digit d
  __shared__ uint32_t wrow[kWaves][kSortBins];  // per wavefront: its count, then its offset
  __shared__ uint32_t psum[kT];
  __shared__ uint64_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const size_t beg = (size_t)blockIdx.x * kSortTile;
  const uint32_t tn = (uint32_t)(n - beg < (size_t)kSortTile ? n - beg : (size_t)kSortTile);
  // this tile's count of each of the thread's digits: the next entry of the
  // digit-major scanned histogram (the same digit's next tile, or the next
  // digit's first tile)
  uint32_t cnt[kDPT];
  uint32_t tsum = 0;
#pragma unroll
  for (int j = 0; j < kDPT; ++j) {
    const int d = t * kDPT + j;
    const size_t e = (size_t)d * nblk + blockIdx.x;
    const uint32_t o0 = off[e];
    const uint32_t o1 = (e + 1 < (size_t)kSortBins * nblk) ? off[e + 1] : (uint32_t)n;
    base[d] = o0;
    cnt[j] = o1 - o0;
    tsum += cnt[j];
    for (int w = 0; w < kWaves; ++w) wrow[w][d] = 0;
  }
  // the wavefront's keys and values
  const uint32_t w0 = (uint32_t)wid * kPerWave;
  uint64_t kr[kWR];
  uint32_t vr[kWR];
#pragma unroll
  for (int r = 0; r < kWR; ++r) {
    const uint32_t li = w0 + (uint32_t)(r * 64 + lane);
    kr[r] = li < tn ? kin[beg + li] : 0ull;
    vr[r] = li < tn ? vin[beg + li] : 0u;
  }
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // lanes of this wavefront whose keys have the same digit d
  auto match = [](uint32_t d, bool valid) {
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kSortBits; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      same &= ((d >> b) & 1u) ? bb : ~bb;
    }
    return same;
  };
  auto digit = [&](uint64_t k, bool valid) {
    return valid ? (uint32_t)((k >> shift) & (kSortBins - 1)) : 0u;
  };
  // ---- count per digit in the wavefront's own row; keep per round the
  // digit, the rank among the round's lanes with that digit, their number
  // and whether the lane holds a key: d | rank << 9 | count << 15 | 1 << 22
  static_assert(kSortBits <= 9, "digit field");
  uint32_t info[kWR];
#pragma unroll
  for (int r = 0; r < kWR; ++r) {
    const bool valid = w0 + (uint32_t)(r * 64 + lane) < tn;
    const uint32_t d = digit(kr[r], valid);
    const uint64_t same = match(d, valid);
    const uint32_t rank = (uint32_t)__popcll(same & below), num = (uint32_t)__popcll(same);
    if (valid && rank == 0) wrow[wid][d] += num;
    info[r] = d | rank << 9 | num << 15 | (valid ? 1u << 22 : 0u);
    wave_sync();
  }
  // ---- tile offsets per digit (scan of the threads' counts, digits in
  // thread order), then each wavefront's offset per digit
  uint32_t c = tsum;
  psum[t] = c;
  __syncthreads();
  for (int d = 1; d < kT; d <<= 1) {
    const uint32_t u = t >= d ? psum[t - d] : 0u;
    __syncthreads();
    c += u;
    psum[t] = c;
    __syncthreads();
  }
  uint32_t run = c - tsum;
#pragma unroll
  for (int j = 0; j < kDPT; ++j) {
    const int d = t * kDPT + j;
    lbeg[d] = run;
    uint32_t o = run;
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t k = wrow[w][d];
      wrow[w][d] = o;
      o += k;
    }
    run += cnt[j];
  }
  __syncthreads();
  // ---- place the keys in digit order
#pragma unroll
  for (int r = 0; r < kWR; ++r) {
    const bool valid = (info[r] >> 22) & 1u;
    const uint32_t d = info[r] & (kSortBins - 1), rank = (info[r] >> 9) & 63u,
                   num = (info[r] >> 15) & 127u;
    const uint32_t o = valid ? wrow[wid][d] : 0u;
    wave_sync();
    if (valid) {
      sk[o + rank] = kr[r];
      sv[o + rank] = vr[r];
      if (rank == 0) wrow[wid][d] = o + num;
    }
    wave_sync();
  }
  __syncthreads();
  for (uint32_t j = (uint32_t)t; j < tn; j += kT) {
    const uint64_t k = sk[j];
    const uint32_t d = (uint32_t)((k >> shift) & (kSortBins - 1));
    const size_t dst = (size_t)base[d] + (j - lbeg[d]);
    kout[dst] = k;
    vout[dst] = sv[j];
  }
}
}  // namespace

// Sort (key, idx) ascending by key, stable, from the first buffer pair into
// the second; the passes alternate between the pairs (an odd number of them,
// so the last writes the second pair) and the first pair is overwritten.
hipError_t radix_sort(uint64_t* key_in, uint32_t* idx_in, uint64_t* key_out, uint32_t* idx_out,
                      size_t n, uint32_t* hist, uint32_t* scan_tmp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int nblk = (int)((n + kSortTile - 1) / kSortTile);
  uint64_t* kin = key_in;
  uint32_t* vin = idx_in;
  uint64_t* kout = key_out;
  uint32_t* vout = idx_out;
  for (int pass = 0; pass < kPasses; ++pass) {
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

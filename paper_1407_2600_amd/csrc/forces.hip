// Interaction kernels (paper Sec. 2.1: the gravitational inner loops; direct
// interactions with the particles of nearby leaves and multipole interactions
// with accepted cells, m source cells x n sink particles per list).
//
// One 64-lane wavefront handles one sink group: each lane holds one target
// (tiles of 64 for larger groups) in registers, and the wavefront steps
// through the group's list together, so every source particle or cell record
// is wave-uniform and is read once per wavefront through the scalar cache
// into scalar registers, feeding all 64 targets.
//
// Precision: coordinates are relative to the group's cell centre; positions,
// cell centres and centres of mass are FP64 and are differenced in FP64
// before rounding to the arithmetic type T.  In FP32, per-leaf (direct) and
// per-16-cell (multipole) partial sums are folded into a (hi, lo) pair with
// Knuth's TwoSum, so the long sums keep about twice FP32 precision.
#include "device_math.h"

namespace hot {

constexpr int kForceWaves = 4;

// ------------------------------------------------------------------- direct
// Direct interactions of one sink group per wavefront, targets in lanes, in
// passes of up to 64 targets: first the group's own particles (image 0,
// without the target itself), then every listed leaf with its image shift.
// TAIL selects the passes as in k_m2p: the main launch takes the passes over
// more than 32 targets with wave-uniform sources; the tail launch takes a
// last pass of at most 32 targets and splits the wave into 2 or 4 sub-groups
// that share out the sources and list entries, adding their partial sums at
// the end.  This kernel writes (not adds) the accumulators.
template <typename T, typename T4, bool TAIL>
__global__ void __launch_bounds__(64 * kForceWaves) k_p2p(Cells C, Groups G, uint32_t ngroups,
                                                          double L, T eps2,
                                                          const double* __restrict__ spos,
                                                          const T4* __restrict__ srec, size_t n,
                                                          const uint32_t* __restrict__ list,
                                                          double4* __restrict__ out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t g = __builtin_amdgcn_readfirstlane(xcd_block() * kForceWaves + wid);
  if (g >= ngroups) return;
  const int A = __builtin_amdgcn_readfirstlane(G.cell[g]);
  const uint32_t first = __builtin_amdgcn_readfirstlane(C.first[A]);
  const uint32_t count = __builtin_amdgcn_readfirstlane(C.count[A]);
  const uint32_t tail0 = count - count % 64;
  const bool has_tail = count % 64 != 0 && count % 64 <= 32;
  if (TAIL && !has_tail) return;
  double cA[3];
  center_of(C.key[A], C.level[A], L, cA);
  const uint32_t off = G.off_p2p[g], cnt = G.cnt_p2p[g];
  for (uint32_t t0 = TAIL ? tail0 : 0; t0 < count; t0 += 64) {
    const uint32_t rem = count - t0;
    if (!TAIL && rem <= 32) break;
    const uint32_t split = !TAIL ? 1u : rem <= 16 ? 4u : 2u;  // wave-uniform
    const int width = 64 / (int)split;
    const uint32_t sub = (uint32_t)(lane / width);
    const int tl = lane % width;
    const uint32_t s = first + t0 + tl;
    const bool act = (uint32_t)tl < rem;
    const uint32_t ss = act ? s : first;
    const T tx = (T)(spos[ss] - cA[0]), ty = (T)(spos[n + ss] - cA[1]),
            tz = (T)(spos[2 * n + ss] - cA[2]);
    Acc<T> acc;
    acc.zero();
    // own group (image 0), excluding the target itself
    {
      T part[4] = {0, 0, 0, 0};
      for (uint32_t j = first + sub; j < first + count; j += split) {
        const T sx = (T)(spos[j] - cA[0]), sy = (T)(spos[n + j] - cA[1]),
                sz = (T)(spos[2 * n + j] - cA[2]);
        const T m = srec[j].w;
        const T dx = sx - tx, dy = sy - ty, dz = sz - tz;
        T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
        const bool self = (j == ss);
        r2 = self ? (T)1 : r2;
        const T ri = rsqrt_t(r2);
        const T mr = self ? (T)0 : m * ri;
        const T mr3 = mr * (ri * ri);
        part[0] = fma(dx, mr3, part[0]);
        part[1] = fma(dy, mr3, part[1]);
        part[2] = fma(dz, mr3, part[2]);
        part[3] += mr;
      }
      acc.fold(part);
    }
    for (uint32_t q = sub; q < cnt; q += split) {
      const uint32_t e = list[off + q];
      const int img = (int)(e >> 27);
      const int B = (int)(e & kCellMask);
      double cB[3];
      center_of(C.key[B], C.level[B], L, cB);
      const T shx = (T)(cB[0] + (double)(img / 9 - 1) * L - cA[0]);
      const T shy = (T)(cB[1] + (double)((img / 3) % 3 - 1) * L - cA[1]);
      const T shz = (T)(cB[2] + (double)(img % 3 - 1) * L - cA[2]);
      const uint32_t bf = C.first[B], bc = C.count[B];
      T part[4] = {0, 0, 0, 0};
      for (uint32_t j = bf; j < bf + bc; ++j) {
        const T4 r = srec[j];
        const T dx = (shx + r.x) - tx, dy = (shy + r.y) - ty, dz = (shz + r.z) - tz;
        const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
        const T ri = rsqrt_t(r2);
        const T mr = r.w * ri;
        const T mr3 = mr * (ri * ri);
        part[0] = fma(dx, mr3, part[0]);
        part[1] = fma(dy, mr3, part[1]);
        part[2] = fma(dz, mr3, part[2]);
        part[3] += mr;
      }
      acc.fold(part);
    }
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = acc.get(k);
    for (int w = width; w < 64; w <<= 1)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += __shfl_xor(v[k], w, 64);
    if (act && sub == 0) out[s] = make_double4(v[0], v[1], v[2], v[3]);
  }
}

// one cell's coefficient block into registers with 16-byte loads (blocks are
// padded to a multiple of 4 values and 16-byte aligned)
template <typename T, int N>
__device__ __forceinline__ void load_block(const T* __restrict__ p, T* out) {
  if constexpr (sizeof(T) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const float4 v = q[i];
      out[4 * i] = v.x;
      out[4 * i + 1] = v.y;
      out[4 * i + 2] = v.z;
      out[4 * i + 3] = v.w;
    }
  } else {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      const double2 v = q[i];
      out[2 * i] = v.x;
      out[2 * i + 1] = v.y;
    }
  }
}

// Multipole interactions of one sink group per wavefront, targets in lanes,
// in passes of up to 64 targets.  TAIL = false: the passes over more than 32
// targets, each walking the list once with every entry wave-uniform (scalar
// loads of the record and the cell's coefficients).  TAIL = true: the last
// pass when it has at most 32 targets (the remainder of a group of 65..96,
// or a small group); the wave splits into 2 or 4 sub-groups of 32 or 16 lanes
// that take every 2nd or 4th list entry, and the partial sums are added
// across the sub-groups at the end, so the lanes a short pass would leave
// idle do the work.  Separate launches keep the register budget
// (and occupancy) of the main pass independent of the tail's.
template <int P, typename T, bool TAIL>
__global__ void __launch_bounds__(64 * kForceWaves) k_m2p(Cells C, Groups G, uint32_t ngroups,
                                                          double L, T eps2,
                                                          const double* __restrict__ spos,
                                                          size_t n,
                                                          const uint4* __restrict__ list,
                                                          double4* __restrict__ out) {
  constexpr int STR = coef_stride(P);
  // tail-pass staging: per wave, up to 4 entries' offsets, cells and blocks
  constexpr bool kStage = TAIL && sizeof(T) == 8;
  __shared__ T tail_cf[kStage ? kForceWaves : 1][4][kStage ? STR : 1];
  __shared__ T tail_c[kStage ? kForceWaves : 1][4][4];
  __shared__ int tail_b[kStage ? kForceWaves : 1][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t g = __builtin_amdgcn_readfirstlane(xcd_block() * kForceWaves + wid);
  if (g >= ngroups) return;
  const int A = __builtin_amdgcn_readfirstlane(G.cell[g]);
  const uint32_t first = __builtin_amdgcn_readfirstlane(C.first[A]);
  const uint32_t count = __builtin_amdgcn_readfirstlane(C.count[A]);
  double cA[3];
  center_of(C.key[A], C.level[A], L, cA);
  const uint32_t off = G.off_m2p[g], cnt = G.cnt_m2p[g];
  const T* __restrict__ coef = (const T*)C.coef;
  const uint32_t tail0 = count - count % 64;  // start of a pass of < 64 targets
  const bool has_tail = count % 64 != 0 && count % 64 <= 32;
  if (TAIL && !has_tail) return;
  for (uint32_t t0 = TAIL ? tail0 : 0; t0 < count; t0 += 64) {
    const uint32_t rem = count - t0;
    if (!TAIL && rem <= 32) break;
    const int split = !TAIL ? 1 : rem <= 16 ? 4 : 2;  // wave-uniform
    const int width = 64 / split;
    const int sub = lane / width, tl = lane % width;
    const uint32_t s = first + t0 + tl;
    const bool act = (uint32_t)tl < rem;
    const uint32_t ss = act ? s : first;
    const T tx = (T)(spos[ss] - cA[0]), ty = (T)(spos[n + ss] - cA[1]),
            tz = (T)(spos[2 * n + ss] - cA[2]);
    Acc<T> acc;
    acc.zero();
    T part[4] = {0, 0, 0, 0};
    if (!TAIL) {
      for (uint32_t q = 0; q < cnt; ++q) {
        T c[3];
        const int B = m2p_record<T>(list[off + q], C.walk, L, cA, c);
        T r[4];
        m2p_eval<P, false, T, T>(tx - c[0], ty - c[1], tz - c[2], eps2, coef + (size_t)B * STR,
                                 r);
#pragma unroll
        for (int k = 0; k < 3; ++k) part[k] += r[k];
        // the potential sums many same-signed terms that the far field later
        // cancels almost entirely: fold every term
        acc.fold1(3, r[3]);
        if ((q & 15) == 15) {
          acc.fold(part);
#pragma unroll
          for (int k = 0; k < 3; ++k) part[k] = (T)0;
        }
      }
    } else if constexpr (sizeof(T) == 4) {
      // FP32: each sub-group loads its own entries' records and 288-byte
      // coefficient blocks with 16-byte per-lane loads (measured faster than
      // staging them through LDS for FP32 blocks)
      uint32_t it = 0;
      for (uint32_t q = (uint32_t)sub; q < cnt; q += (uint32_t)split) {
        T c[3];
        const int B = m2p_record<T>(list[off + q], C.walk, L, cA, c);
        T cf[STR];
        load_block<T, STR>(coef + (size_t)B * STR, cf);
        T r[4];
        m2p_eval<P, false, T, T>(tx - c[0], ty - c[1], tz - c[2], eps2, cf, r);
#pragma unroll
        for (int k = 0; k < 3; ++k) part[k] += r[k];
        acc.fold1(3, r[3]);
        if ((++it & 15) == 0) {
          acc.fold(part);
#pragma unroll
          for (int k = 0; k < 3; ++k) part[k] = (T)0;
        }
      }
    } else {
      // FP64: each round stages the next `split` entries' offsets and
      // coefficient blocks in this wave's LDS slots with coalesced loads;
      // every sub-group then reads its own block (a broadcast within it)
      T* cbuf = &tail_cf[wid][0][0];
      uint32_t it = 0;
      for (uint32_t q0 = 0; q0 < cnt; q0 += (uint32_t)split) {
        const uint32_t ne = cnt - q0 < (uint32_t)split ? cnt - q0 : (uint32_t)split;
        if ((uint32_t)lane < ne) {
          T c[3];
          const int B = m2p_record<T>(list[off + q0 + lane], C.walk, L, cA, c);
          tail_c[wid][lane][0] = c[0];
          tail_c[wid][lane][1] = c[1];
          tail_c[wid][lane][2] = c[2];
          tail_b[wid][lane] = B;
        }
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = (uint32_t)lane; i < ne * STR; i += 64) {
          const uint32_t e = i / STR, k = i % STR;
          cbuf[i] = coef[(size_t)tail_b[wid][e] * STR + k];
        }
        __builtin_amdgcn_wave_barrier();
        if (sub < ne) {
          T r[4];
          m2p_eval<P, false, T, T>(tx - tail_c[wid][sub][0], ty - tail_c[wid][sub][1],
                                   tz - tail_c[wid][sub][2], eps2, cbuf + (size_t)sub * STR, r);
#pragma unroll
          for (int k = 0; k < 3; ++k) part[k] += r[k];
          acc.fold1(3, r[3]);
          if ((++it & 15) == 0) {
            acc.fold(part);
#pragma unroll
            for (int k = 0; k < 3; ++k) part[k] = (T)0;
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    acc.fold(part);
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = acc.get(k);
    for (int w = width; w < 64; w <<= 1)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += __shfl_xor(v[k], w, 64);
    if (act && sub == 0) {
      double4 o = out[s];
      o.x += v[0];
      o.y += v[1];
      o.z += v[2];
      o.w += v[3];
      out[s] = o;
    }
  }
}

hipError_t p2p_launch(bool fp32, const Cells& C, const Groups& G, uint32_t ngroups, double L,
                      double eps, const double* spos, const void* srec, size_t n,
                      const uint32_t* list, double4* out, hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  unsigned blocks = (ngroups + kForceWaves - 1) / kForceWaves;
  if (fp32) {
    const float e2 = (float)(eps * eps);
    k_p2p<float, float4, false><<<blocks, 64 * kForceWaves, 0, s>>>(
        C, G, ngroups, L, e2, spos, (const float4*)srec, n, list, out);
    k_p2p<float, float4, true><<<blocks, 64 * kForceWaves, 0, s>>>(
        C, G, ngroups, L, e2, spos, (const float4*)srec, n, list, out);
  } else {
    k_p2p<double, double4, false><<<blocks, 64 * kForceWaves, 0, s>>>(
        C, G, ngroups, L, eps * eps, spos, (const double4*)srec, n, list, out);
    k_p2p<double, double4, true><<<blocks, 64 * kForceWaves, 0, s>>>(
        C, G, ngroups, L, eps * eps, spos, (const double4*)srec, n, list, out);
  }
  return hipGetLastError();
}

template <int P>
static void m2p_launch_p(bool fp32, const Cells& C, const Groups& G, uint32_t ngroups, double L,
                         double eps, const double* spos, size_t n, const uint4* list,
                         double4* out, hipStream_t s) {
  unsigned blocks = (ngroups + kForceWaves - 1) / kForceWaves;
  if (fp32) {
    k_m2p<P, float, false><<<blocks, 64 * kForceWaves, 0, s>>>(C, G, ngroups, L, (float)(eps * eps),
                                                               spos, n, list, out);
    k_m2p<P, float, true><<<blocks, 64 * kForceWaves, 0, s>>>(C, G, ngroups, L, (float)(eps * eps),
                                                              spos, n, list, out);
  } else {
    k_m2p<P, double, false><<<blocks, 64 * kForceWaves, 0, s>>>(C, G, ngroups, L, eps * eps, spos,
                                                                n, list, out);
    k_m2p<P, double, true><<<blocks, 64 * kForceWaves, 0, s>>>(C, G, ngroups, L, eps * eps, spos,
                                                               n, list, out);
  }
}

hipError_t m2p_launch(bool fp32, int order, const Cells& C, const Groups& G, uint32_t ngroups,
                      double L, double eps, const double* spos, size_t n, const uint4* list,
                      double4* out, hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  switch (order) {
    case 0: m2p_launch_p<0>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s); break;
    case 1: m2p_launch_p<1>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s); break;
    case 2: m2p_launch_p<2>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s); break;
    case 3: m2p_launch_p<3>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s); break;
    case 4: m2p_launch_p<4>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hot

// Periodic far field (paper Sec. 2.1: periodic boundary conditions through a
// high-order multipole local expansion; the uniform background is
// subtracted).
//
// With the 27 nearest images walked explicitly, all other images of every
// source contribute Psi(x_i - x_j), Psi = Ewald potential minus the 27 bare
// nearest images, which is smooth inside the box.  It is expanded per pair of
// octants (level-1 cells): for a target in octant t and the sources of octant
// s, about r0 = c_t - c_s with h = x - c_t, s_j = x_j - c_s,
//   Phi_far(x) = sum_q Lam^t_q h^q,
//   Lam^t_q = sum_s sum_k C(q+k, q) (-1)^|k| Tpsi^{c_t-c_s}_{q+k} M^s_k,
//   M^s_k = sum_{j in s} m_j s_j^k,
// |q|, |k| <= far_order, with the 27 Taylor tables Tpsi built on the host.
// Expanding about octant centres instead of the box centre halves the radius
// of the expansions and makes the truncation error orders of magnitude
// smaller at the same order.  Octant s holds a contiguous range of the sorted
// particles (its keys share the top octal digit), found by binary search.
// The moments are a blocked reduction (particles in lanes, moments in
// registers); the local coefficients one wavefront per coefficient; the
// evaluation one thread per particle in FP64, fused with the scaling (-G, G)
// and the scatter back to the caller's particle order.
#include "device_math.h"

namespace hot {

// Octant moments, per block of one octant's particles: each lane takes one
// particle at a time and each of the 4 wavefronts a fixed share of the
// (a, b) exponent pairs, accumulating m x^a y^b z^c for every c of its pairs
// in registers; at the end the lanes' sums are added across the wavefront.
template <int PF, int W>
__device__ __forceinline__ void far_moments_wave(const double* __restrict__ spos,
                                                 const double* __restrict__ smass, size_t n,
                                                 size_t beg, size_t end, const double c[3],
                                                 int lane, double* __restrict__ out) {
  constexpr FarPairs<PF> fp{};
  constexpr int NP = FarPairs<PF>::N;
  constexpr int NA = far_wave_terms<PF>(W);
  if constexpr (NA > 0) {
    double acc[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = 0.0;
    for (size_t s = beg + (size_t)lane; s < end; s += 64) {
      const double dx = spos[s] - c[0], dy = spos[n + s] - c[1], dz = spos[2 * n + s] - c[2];
      const double m = smass[s];
      double px[PF + 1], py[PF + 1], pz[PF + 1];
      px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
      for (int e = 1; e <= PF; ++e) {
        px[e] = px[e - 1] * dx;
        py[e] = py[e - 1] * dy;
        pz[e] = pz[e - 1] * dz;
      }
      int o = 0;
#pragma unroll
      for (int q = W; q < NP; q += kFarWaves) {
        const double w = m * px[fp.a[q]] * py[fp.b[q]];
#pragma unroll
        for (int e = 0; e <= PF - fp.a[q] - fp.b[q]; ++e) {
          acc[o] = fma(w, pz[e], acc[o]);
          ++o;
        }
      }
    }
    int o = 0;
#pragma unroll
    for (int q = W; q < NP; q += kFarWaves) {
#pragma unroll
      for (int e = 0; e <= PF - fp.a[q] - fp.b[q]; ++e) {
        double v = acc[o];
        for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
        if (lane == 0) out[mi_index(fp.a[q], fp.b[q], e)] = v;
        ++o;
      }
    }
  }
}

template <int PF>
__global__ void __launch_bounds__(64 * kFarWaves) k_far_moments(const double* __restrict__ spos,
                                                                const double* __restrict__ smass,
                                                                const uint64_t* __restrict__ skey,
                                                                size_t n, double L, int nblk,
                                                                double* __restrict__ part) {
  constexpr int NQ = nt(PF);
  const int o = blockIdx.y;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  size_t obeg, oend;
  octant_range(skey, n, o, &obeg, &oend);
  const size_t len = oend - obeg;
  const size_t chunk = (len + nblk - 1) / nblk;
  const size_t beg = obeg + (size_t)blockIdx.x * chunk < oend ? obeg + (size_t)blockIdx.x * chunk
                                                              : oend;
  const size_t end = beg + chunk < oend ? beg + chunk : oend;
  double c[3];
  octant_center(o, L, c);
  double* out = part + ((size_t)o * nblk + blockIdx.x) * NQ;
  switch (wid) {
    case 0: far_moments_wave<PF, 0>(spos, smass, n, beg, end, c, lane, out); break;
    case 1: far_moments_wave<PF, 1>(spos, smass, n, beg, end, c, lane, out); break;
    case 2: far_moments_wave<PF, 2>(spos, smass, n, beg, end, c, lane, out); break;
    default: far_moments_wave<PF, 3>(spos, smass, n, beg, end, c, lane, out); break;
  }
}

// octant moments: sum of the per-block partial moments
template <int PF>
__global__ void __launch_bounds__(256) k_far_sum(const double* __restrict__ part, int nblk,
                                                 double* __restrict__ mom) {
  constexpr int NQ = nt(PF);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 8 * NQ) return;
  const int s = i / NQ, k = i % NQ;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += part[((size_t)s * nblk + b) * NQ + k];
  mom[i] = acc;
}

// Local coefficients of target octant t (blockIdx.y), output q (blockIdx.x):
//   Lam_q = sum_s sum_k (-1)^|k| C(q+k, q) Tpsi^(t-s)_(q+k) M^s_k,
// one wavefront per output, the 8 x nt(PF) terms spread over its lanes.
template <int PF>
__global__ void __launch_bounds__(64) k_far_lambda(const double* __restrict__ tpsi,
                                                   const double* __restrict__ mom,
                                                   double* __restrict__ lam) {
  constexpr int NQ = nt(PF);
  constexpr int NT2 = nt(2 * PF);
  const int q = blockIdx.x, t = blockIdx.y, lane = threadIdx.x;
  // decode q's multi-index (degree, then a, b descending)
  int qa = 0, qb = 0, qc = 0;
  {
    int d = 0;
    while (nt(d) <= q) ++d;
    int r = q - nt(d - 1);
    for (qa = d; qa >= 0; --qa) {
      const int cnt = d - qa + 1;
      if (r < cnt) break;
      r -= cnt;
    }
    qb = d - qa - r;
    qc = d - qa - qb;
  }
  double acc = 0.0;
  for (int i = lane; i < 8 * NQ; i += 64) {
    const int s = i / NQ, k = i % NQ;
    int d = 0;
    while (nt(d) <= k) ++d;
    int r = k - nt(d - 1), ka;
    for (ka = d; ka >= 0; --ka) {
      const int cnt = d - ka + 1;
      if (r < cnt) break;
      r -= cnt;
    }
    const int kb = d - ka - r, kc = d - ka - kb;
    const int dx = ((t >> 2) & 1) - ((s >> 2) & 1), dy = ((t >> 1) & 1) - ((s >> 1) & 1),
              dz = (t & 1) - (s & 1);
    const double* Tp = tpsi + (size_t)((dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)) * NT2;
    const double bin = kBinom.v[qa + ka][ka] * kBinom.v[qb + kb][kb] * kBinom.v[qc + kc][kc];
    const double sg = (d & 1) ? -1.0 : 1.0;
    acc += sg * bin * Tp[mi_index(qa + ka, qb + kb, qc + kc)] * mom[(size_t)s * NQ + k];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) lam[(size_t)t * NQ + q] = acc;
}

// One particle per thread.  The block's particles (consecutive in key order)
// almost always lie in one octant: its local coefficients are staged in LDS
// once per block and read from there (broadcast reads), the few particles of
// another octant read theirs from global memory.
template <int PF, typename T>
__global__ void __launch_bounds__(256) k_far_apply(const double* __restrict__ spos,
                                                   const uint64_t* __restrict__ skey,
                                                   const double4* __restrict__ near, size_t n,
                                                   const uint32_t* __restrict__ idx, double L,
                                                   double G, const double* __restrict__ lam,
                                                   int periodic, const uint8_t* __restrict__ rung,
                                                   int rmin, T* __restrict__ acc,
                                                   T* __restrict__ pot) {
  constexpr int NQ = nt(PF);
  __shared__ double cs[NQ];
  const size_t b0 = (size_t)blockIdx.x * blockDim.x;
  const size_t s = b0 + threadIdx.x;
  const int ob = periodic ? (int)((skey[b0] >> 60) & 7ull) : 0;
  if (periodic) {
    for (int i = threadIdx.x; i < NQ; i += blockDim.x) cs[i] = lam[(size_t)ob * NQ + i];
    __syncthreads();
  }
  if (s >= n) return;
  // block timesteps: only the particles whose step ends now get new values
  if (rung && (int)rung[idx[s]] < rmin) return;
  double4 v = near[s];
  double phi = v.w, gx = v.x, gy = v.y, gz = v.z;
  if (periodic) {
    const int o = (int)((skey[s] >> 60) & 7ull);
    double c[3];
    octant_center(o, L, c);
    const double h[3] = {spos[s] - c[0], spos[n + s] - c[1], spos[2 * n + s] - c[2]};
    double r[4];
    if (o == ob)
      local_horner<PF, double>(cs, h[0], h[1], h[2], r);
    else
      local_horner<PF, double>(lam + (size_t)o * NQ, h[0], h[1], h[2], r);
    const double P = r[3], Gx = r[0], Gy = r[1], Gz = r[2];
    phi += P;
    gx += Gx;
    gy += Gy;
    gz += Gz;
  }
  const uint32_t i = idx[s];
  acc[i] = (T)(G * gx);
  acc[n + i] = (T)(G * gy);
  acc[2 * n + i] = (T)(G * gz);
  if (pot) pot[i] = (T)(-G * phi);
}

template <int PF>
static hipError_t far_run(const double* spos, const double* smass, const uint64_t* skey,
                          const double4* near, size_t n, const uint32_t* idx, double box,
                          double G, const double* tpsi, double* part, int nblk_max, double* mom,
                          double* lam, int periodic, const uint8_t* rung, int rmin, bool fp32,
                          void* acc, void* pot, hipStream_t s) {
  if (periodic) {
    int nblk = (int)((n / 8 + 2047) / 2048);
    if (nblk > nblk_max) nblk = nblk_max;
    if (nblk < 1) nblk = 1;
    k_far_moments<PF><<<dim3(nblk, 8), 64 * kFarWaves, 0, s>>>(spos, smass, skey, n, box, nblk,
                                                            part);
    k_far_sum<PF><<<(8 * nt(PF) + 255) / 256, 256, 0, s>>>(part, nblk, mom);
    k_far_lambda<PF><<<dim3(nt(PF), 8), 64, 0, s>>>(tpsi, mom, lam);
  }
  unsigned g = (unsigned)((n + 255) / 256);
  if (fp32)
    k_far_apply<PF, float><<<g, 256, 0, s>>>(spos, skey, near, n, idx, box, G, lam, periodic,
                                              rung, rmin, (float*)acc, (float*)pot);
  else
    k_far_apply<PF, double><<<g, 256, 0, s>>>(spos, skey, near, n, idx, box, G, lam, periodic,
                                               rung, rmin, (double*)acc, (double*)pot);
  return hipGetLastError();
}

template <int PF>
static hipError_t far_prepare_run(const double* spos, const double* smass, const uint64_t* skey,
                                  size_t n, double box, const double* tpsi, double* part,
                                  int nblk_max, double* mom, double* lam, hipStream_t s) {
  int nblk = (int)((n / 8 + 2047) / 2048);
  if (nblk > nblk_max) nblk = nblk_max;
  if (nblk < 1) nblk = 1;
  k_far_moments<PF><<<dim3(nblk, 8), 64 * kFarWaves, 0, s>>>(spos, smass, skey, n, box, nblk, part);
  k_far_sum<PF><<<(8 * nt(PF) + 255) / 256, 256, 0, s>>>(part, nblk, mom);
  k_far_lambda<PF><<<dim3(nt(PF), 8), 64, 0, s>>>(tpsi, mom, lam);
  return hipGetLastError();
}

// octant moments and local coefficients only (the adjoint needs Lam)
hipError_t far_prepare_launch(int far_order, const double* spos, const double* smass,
                              const uint64_t* skey, size_t n, double box, const double* tpsi,
                              double* part, int nblk_max, double* mom, double* lam,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
#define HOT_FARP(PF) \
  case PF:           \
    return far_prepare_run<PF>(spos, smass, skey, n, box, tpsi, part, nblk_max, mom, lam, s);
  switch (far_order) {
    HOT_FARP(0) HOT_FARP(1) HOT_FARP(2) HOT_FARP(3) HOT_FARP(4) HOT_FARP(5) HOT_FARP(6)
    HOT_FARP(7) HOT_FARP(8) HOT_FARP(9) HOT_FARP(10) HOT_FARP(11) HOT_FARP(12)
    default: return hipErrorInvalidValue;
  }
#undef HOT_FARP
}

hipError_t far_launch(int far_order, const double* spos, const double* smass,
                      const uint64_t* skey, const double4* near, size_t n, const uint32_t* idx,
                      double box, double G, const double* tpsi, double* part, int nblk_max,
                      double* mom, double* lam, int periodic, const uint8_t* rung, int rmin,
                      bool fp32, void* acc, void* pot, hipStream_t s) {
  if (n == 0) return hipSuccess;
#define HOT_FAR(PF)                                                                            \
  case PF:                                                                                     \
    return far_run<PF>(spos, smass, skey, near, n, idx, box, G, tpsi, part, nblk_max, mom, lam, \
                       periodic, rung, rmin, fp32, acc, pot, s);
  switch (far_order) {
    HOT_FAR(0) HOT_FAR(1) HOT_FAR(2) HOT_FAR(3) HOT_FAR(4) HOT_FAR(5) HOT_FAR(6)
    HOT_FAR(7) HOT_FAR(8) HOT_FAR(9) HOT_FAR(10) HOT_FAR(11) HOT_FAR(12)
    default: return hipErrorInvalidValue;
  }
#undef HOT_FAR
}

}  // namespace hot

// Adjoint of the periodic far field (exact derivative of the octant local
// expansions used by the forward pass).
//
// Forward: Phi_far(x) = sum_q Lam^t_q h^q, h = x - c_t, t the octant of x,
//   Lam^t_q = sum_s sum_k C(q+k,q) (-1)^|k| Tpsi^{c_t-c_s}_{q+k} M^s_k,
//   M^s_k = sum_{j in s} m_j (x_j - c_s)^k.
// For L = sum_i gacc_i . G grad Phi_far(x_i) - gpot_i G Phi_far(x_i):
//   target side:  xbar_i += G (Hess Phi_far) gacc_i - G gpot_i grad Phi_far
//                 (the Hessian along gacc_i from a dual-number evaluation);
//   source side:  Lbar^t_q = G sum_{i in t} (gacc_i . grad h_i^q - gpot_i h_i^q),
//                 Mbar^s_k = sum_t sum_q Lbar^t_q C(q+k,q) (-1)^|k| Tpsi^{c_t-c_s}_{q+k},
//                 xbar_j += m_j sum_k Mbar^s_k grad s_j^k,  mbar_j += sum_k Mbar^s_k s_j^k.
// The final kernel also adds the near-field adjoint (scaled by G) and writes
// xbar (FP64) and mbar in the caller's particle order.
#include "device_math.h"

namespace hot {

// Target-octant cotangents of the local coefficients,
//   Lbar^t_q = sum_{i in t} (gacc_i . grad h_i^q - gpot_i h_i^q),
// per block of one octant's particles, laid out like the forward moments:
// particles in lanes, each wavefront a fixed share of the (a, b) pairs. For a
// pair, u0 = x^a y^b (-gpot) + a gx x^(a-1) y^b + b gy x^a y^(b-1) and
// u1 = gz x^a y^b give the term of z-exponent c as u0 z^c + u1 c z^(c-1).
template <int PF, int W, typename T4>
__device__ __forceinline__ void far_adj_local_wave(const double* __restrict__ spos,
                                                   const T4* __restrict__ arec, size_t n,
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
      const T4 r = arec[s];
      const double gx = (double)r.x, gy = (double)r.y, gz = (double)r.z, gp = (double)r.w;
      double px[PF + 1], py[PF + 1], pz[PF + 1], dpz[PF + 1];
      px[0] = py[0] = pz[0] = 1.0;
      dpz[0] = 0.0;
#pragma unroll
      for (int e = 1; e <= PF; ++e) {
        px[e] = px[e - 1] * dx;
        py[e] = py[e - 1] * dy;
        pz[e] = pz[e - 1] * dz;
        dpz[e] = (double)e * pz[e - 1];
      }
      int o = 0;
#pragma unroll
      for (int q = W; q < NP; q += kFarWaves) {
        const int qa = fp.a[q], qb = fp.b[q];
        const double xy = px[qa] * py[qb];
        double u0 = -gp * xy;
        if (qa) u0 = fma(gx * (double)qa, px[qa - 1] * py[qb], u0);
        if (qb) u0 = fma(gy * (double)qb, px[qa] * py[qb - 1], u0);
        const double u1 = gz * xy;
#pragma unroll
        for (int e = 0; e <= PF - qa - qb; ++e) {
          acc[o] += fma(u0, pz[e], u1 * dpz[e]);
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

template <int PF, typename T4>
__global__ void __launch_bounds__(64 * kFarWaves) k_far_adj_local(const double* __restrict__ spos,
                                                                  const T4* __restrict__ arec,
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
    case 0: far_adj_local_wave<PF, 0, T4>(spos, arec, n, beg, end, c, lane, out); break;
    case 1: far_adj_local_wave<PF, 1, T4>(spos, arec, n, beg, end, c, lane, out); break;
    case 2: far_adj_local_wave<PF, 2, T4>(spos, arec, n, beg, end, c, lane, out); break;
    default: far_adj_local_wave<PF, 3, T4>(spos, arec, n, beg, end, c, lane, out); break;
  }
}

// one block per source octant s
template <int PF>
__global__ void __launch_bounds__(256) k_far_adj_sum(const double* __restrict__ part, int nblk,
                                                     double G, double* __restrict__ lb) {
  constexpr int NQ = nt(PF);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 8 * NQ) return;
  const int t = i / NQ, q = i % NQ;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += part[((size_t)t * nblk + b) * NQ + q];
  lb[i] = G * acc;
}

__device__ __forceinline__ void mi_decode(int k, int* a, int* b, int* c) {
  int d = 0;
  while (nt(d) <= k) ++d;
  int r = k - nt(d - 1), x;
  for (x = d; x >= 0; --x) {
    const int cnt = d - x + 1;
    if (r < cnt) break;
    r -= cnt;
  }
  *a = x;
  *b = d - x - r;
  *c = d - *a - *b;
}

// Source-octant moment cotangents (the adjoint of the local coefficients):
//   mbar^so_k = (-1)^|k| sum_t sum_q Lb^t_q C(q+k, k) Tpsi^(t-so)_(q+k),
// one wavefront per (so = blockIdx.y, k = blockIdx.x), the 8 x nt(PF) terms
// spread over its lanes.
template <int PF>
__global__ void __launch_bounds__(64) k_far_adj_moments(const double* __restrict__ lb,
                                                        const double* __restrict__ tpsi,
                                                        double* __restrict__ mbar) {
  constexpr int NQ = nt(PF);
  constexpr int NT2 = nt(2 * PF);
  const int k = blockIdx.x, so = blockIdx.y, lane = threadIdx.x;
  int ka, kb, kc;
  mi_decode(k, &ka, &kb, &kc);
  double acc = 0.0;
  for (int i = lane; i < 8 * NQ; i += 64) {
    const int t = i / NQ, q = i % NQ;
    int qa, qb, qc;
    mi_decode(q, &qa, &qb, &qc);
    const int dx = ((t >> 2) & 1) - ((so >> 2) & 1), dy = ((t >> 1) & 1) - ((so >> 1) & 1),
              dz = (t & 1) - (so & 1);
    const double* Tp = tpsi + (size_t)((dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)) * NT2;
    const double bin = kBinom.v[qa + ka][ka] * kBinom.v[qb + kb][kb] * kBinom.v[qc + kc][kc];
    acc += lb[(size_t)t * NQ + q] * bin * Tp[mi_index(qa + ka, qb + kb, qc + kc)];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) mbar[(size_t)so * NQ + k] = (((ka + kb + kc) & 1) ? -1.0 : 1.0) * acc;
}

template <int PF, typename T, typename T4>
__global__ void __launch_bounds__(256) k_far_adj_apply(
    const double* __restrict__ spos, const double* __restrict__ smass,
    const uint64_t* __restrict__ skey, const T4* __restrict__ arec,
    const double4* __restrict__ near, size_t n, const uint32_t* __restrict__ idx, double L,
    double G, const double* __restrict__ lam, const double* __restrict__ mbar, int periodic,
    double* __restrict__ xbar, T* __restrict__ mbar_out) {
  // the block's octant's coefficients in LDS (the block's particles are
  // consecutive in key order, almost always in one octant); particles of
  // another octant read theirs from global memory
  constexpr int NQ = nt(PF);
  __shared__ double cl[NQ], cm[NQ];
  const size_t b0 = (size_t)blockIdx.x * blockDim.x;
  const size_t s = b0 + threadIdx.x;
  const int ob = periodic ? (int)((skey[b0] >> 60) & 7ull) : 0;
  if (periodic) {
    for (int i = threadIdx.x; i < NQ; i += blockDim.x) {
      cl[i] = lam[(size_t)ob * NQ + i];
      cm[i] = mbar[(size_t)ob * NQ + i];
    }
    __syncthreads();
  }
  if (s >= n) return;
  const double4 v = near[s];
  double xb[3] = {G * v.x, G * v.y, G * v.z};
  double mb = G * v.w;
  if (periodic) {
    const int o = (int)((skey[s] >> 60) & 7ull);
    double c[3];
    octant_center(o, L, c);
    const double h[3] = {spos[s] - c[0], spos[n + s] - c[1], spos[2 * n + s] - c[2]};
    const T4 r = arec[s];
    const double ga[3] = {(double)r.x, (double)r.y, (double)r.z};
    const double gp = (double)r.w;
    // target side: gradient and its derivative along gacc; source side
    Dual<double> f[4];
    double sm[4];
    if (o == ob) {
      local_horner<PF, Dual<double>>(cl, Dual<double>(h[0], ga[0]), Dual<double>(h[1], ga[1]),
                                   Dual<double>(h[2], ga[2]), f);
      local_horner<PF, double>(cm, h[0], h[1], h[2], sm);
    } else {
      local_horner<PF, Dual<double>>(lam + (size_t)o * NQ, Dual<double>(h[0], ga[0]),
                                   Dual<double>(h[1], ga[1]), Dual<double>(h[2], ga[2]), f);
      local_horner<PF, double>(mbar + (size_t)o * NQ, h[0], h[1], h[2], sm);
    }
    for (int a = 0; a < 3; ++a) xb[a] += G * f[a].d - G * gp * f[a].v;
    const double m = smass[s];
    for (int a = 0; a < 3; ++a) xb[a] += m * sm[a];
    mb += sm[3];
  }
  const uint32_t i = idx[s];
  xbar[i] = xb[0];
  xbar[n + i] = xb[1];
  xbar[2 * n + i] = xb[2];
  mbar_out[i] = (T)mb;
}

template <int PF>
static hipError_t far_adj_run(const double* spos, const double* smass, const uint64_t* skey,
                              const void* arec, const double4* near, size_t n,
                              const uint32_t* idx, double box, double G, const double* tpsi,
                              double* part, int nblk_max, const double* lam, double* lb,
                              double* mbar, int periodic, bool fp32, double* xbar,
                              void* mbar_out, hipStream_t s) {
  if (periodic) {
    int nblk = (int)((n / 8 + 2047) / 2048);
    if (nblk > nblk_max) nblk = nblk_max;
    if (nblk < 1) nblk = 1;
    if (fp32)
      k_far_adj_local<PF, float4><<<dim3(nblk, 8), 64 * kFarWaves, 0, s>>>(
          spos, (const float4*)arec, skey, n, box, nblk, part);
    else
      k_far_adj_local<PF, double4><<<dim3(nblk, 8), 64 * kFarWaves, 0, s>>>(
          spos, (const double4*)arec, skey, n, box, nblk, part);
    k_far_adj_sum<PF><<<(8 * nt(PF) + 255) / 256, 256, 0, s>>>(part, nblk, G, lb);
    k_far_adj_moments<PF><<<dim3(nt(PF), 8), 64, 0, s>>>(lb, tpsi, mbar);
  }
  unsigned g = (unsigned)((n + 255) / 256);
  if (fp32)
    k_far_adj_apply<PF, float, float4><<<g, 256, 0, s>>>(spos, smass, skey, (const float4*)arec,
                                                         near, n, idx, box, G, lam, mbar,
                                                         periodic, xbar, (float*)mbar_out);
  else
    k_far_adj_apply<PF, double, double4><<<g, 256, 0, s>>>(
        spos, smass, skey, (const double4*)arec, near, n, idx, box, G, lam, mbar, periodic, xbar,
        (double*)mbar_out);
  return hipGetLastError();
}

hipError_t far_adj_launch(int far_order, const double* spos, const double* smass,
                          const uint64_t* skey, const void* arec, const double4* near, size_t n,
                          const uint32_t* idx, double box, double G, const double* tpsi,
                          double* part, int nblk_max, const double* lam, double* lb,
                          double* mbar, int periodic, bool fp32, double* xbar, void* mbar_out,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
#define HOT_FARA(PF)                                                                         \
  case PF:                                                                                   \
    return far_adj_run<PF>(spos, smass, skey, arec, near, n, idx, box, G, tpsi, part,        \
                           nblk_max, lam, lb, mbar, periodic, fp32, xbar, mbar_out, s);
  switch (far_order) {
    HOT_FARA(0) HOT_FARA(1) HOT_FARA(2) HOT_FARA(3) HOT_FARA(4) HOT_FARA(5) HOT_FARA(6)
    HOT_FARA(7) HOT_FARA(8) HOT_FARA(9) HOT_FARA(10) HOT_FARA(11) HOT_FARA(12)
    default: return hipErrorInvalidValue;
  }
#undef HOT_FARA
}

}  // namespace hot

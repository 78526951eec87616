// Fixed-step kick-drift-kick leapfrog (the paper's Sec. 2.1 integrator is an
// adaptive symplectic one; the fixed-step leapfrog is its single-rung case),
// and the interaction counters reported with each force evaluation.
#include <algorithm>

#include "hot_internal.h"

namespace hot {

template <typename T>
__global__ void __launch_bounds__(256) k_kick(T* __restrict__ vel, const T* __restrict__ acc,
                                              size_t m, T h) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) vel[i] = fma(acc[i], h, vel[i]);
}

// x += v dt, then wrap into [0, L) (floor form, robust to any step length)
template <typename T>
__global__ void __launch_bounds__(256) k_drift(double* __restrict__ pos, const T* __restrict__ vel,
                                               size_t m, double dt, double L) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double x = pos[i] + (double)vel[i] * dt;
  x = x - L * floor(x / L);
  if (x >= L) x -= L;
  if (x < 0.0) x = 0.0;
  pos[i] = x;
}

// ---------------------------------------------------------- block timesteps
// Particle i steps dt/2^rung[i] (rungs 0..max_rung), substeps of dt/2^max_rung.
// A particle is due (its step starts or ends at the current substep
// boundary) when rung[i] >= rmin.

// half kick of the due particles over their own step: v += a dt_i / 2
template <typename T>
__global__ void __launch_bounds__(256) k_kick_rung(T* __restrict__ vel, const T* __restrict__ acc,
                                                   const uint8_t* __restrict__ rung, size_t n,
                                                   int rmin, double dt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = rung[i];
  if (r < rmin) return;
  const T h = (T)(0.5 * ldexp(dt, -r));
#pragma unroll
  for (int a = 0; a < 3; ++a) vel[a * n + i] = fma(acc[a * n + i], h, vel[a * n + i]);
}

// rung of the due particles from their accelerations: the largest step
// dt/2^r (r <= max_rung) not above eta sqrt(eps / |a|), but no coarser than
// the rungs whose steps can start at this boundary (r >= rmin)
template <typename T>
__global__ void __launch_bounds__(256) k_rung_assign(const T* __restrict__ acc,
                                                     uint8_t* __restrict__ rung, size_t n,
                                                     int rmin, double dt, int max_rung,
                                                     double eta, double eps) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if ((int)rung[i] < rmin) return;
  const double ax = (double)acc[i], ay = (double)acc[n + i], az = (double)acc[2 * n + i];
  double a2 = ax * ax;
  a2 = a2 + ay * ay;
  a2 = a2 + az * az;
  const double amag = sqrt(a2);
  const double want = eta * sqrt(eps / amag);
  int r = 0;
  while (r < max_rung && ldexp(dt, -r) > want) ++r;
  rung[i] = (uint8_t)(r > rmin ? r : rmin);
}

// largest rung (atomic max into *out, which the caller clears)
__global__ void __launch_bounds__(256) k_rung_max(const uint8_t* __restrict__ rung, size_t n,
                                                  uint32_t* __restrict__ out) {
  uint32_t m = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const uint32_t r = rung[i];
    m = r > m ? r : m;
  }
  for (int d = 32; d > 0; d >>= 1) {
    const uint32_t o = __shfl_down(m, d, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

hipError_t kick_rung_launch(bool fp32, void* vel, const void* acc, const uint8_t* rung, size_t n,
                            int rmin, double dt, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  if (fp32)
    k_kick_rung<float><<<g, 256, 0, s>>>((float*)vel, (const float*)acc, rung, n, rmin, dt);
  else
    k_kick_rung<double><<<g, 256, 0, s>>>((double*)vel, (const double*)acc, rung, n, rmin, dt);
  return hipGetLastError();
}

hipError_t rung_assign_launch(bool fp32, const void* acc, uint8_t* rung, size_t n, int rmin,
                              double dt, int max_rung, double eta, double eps, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  if (fp32)
    k_rung_assign<float><<<g, 256, 0, s>>>((const float*)acc, rung, n, rmin, dt, max_rung, eta,
                                           eps);
  else
    k_rung_assign<double><<<g, 256, 0, s>>>((const double*)acc, rung, n, rmin, dt, max_rung, eta,
                                            eps);
  return hipGetLastError();
}

// groups holding at least one due particle (sorted order; idx = original index)
__global__ void __launch_bounds__(256) k_group_active(Cells C, Groups G, uint32_t ngroups,
                                                      const uint32_t* __restrict__ idx,
                                                      const uint8_t* __restrict__ rung, int rmin,
                                                      uint8_t* __restrict__ act) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  const int A = G.cell[g];
  const uint32_t f = C.first[A], e = f + C.count[A];
  uint8_t a = 0;
  for (uint32_t s = f; s < e && !a; ++s) a = (int)rung[idx[s]] >= rmin;
  act[g] = a;
}

hipError_t group_active_launch(const Cells& C, const Groups& G, uint32_t ngroups,
                               const uint32_t* idx, const uint8_t* rung, int rmin, uint8_t* act,
                               hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  k_group_active<<<(ngroups + 255) / 256, 256, 0, s>>>(C, G, ngroups, idx, rung, rmin, act);
  return hipGetLastError();
}

hipError_t kick_launch(bool fp32, void* vel, const void* acc, size_t n, double h, hipStream_t s) {
  size_t m = 3 * n;
  unsigned g = (unsigned)((m + 255) / 256);
  if (fp32)
    k_kick<float><<<g, 256, 0, s>>>((float*)vel, (const float*)acc, m, (float)h);
  else
    k_kick<double><<<g, 256, 0, s>>>((double*)vel, (const double*)acc, m, h);
  return hipGetLastError();
}

hipError_t drift_launch(bool fp32, double* pos, const void* vel, size_t n, double dt, double L,
                        hipStream_t s) {
  size_t m = 3 * n;
  unsigned g = (unsigned)((m + 255) / 256);
  if (fp32)
    k_drift<float><<<g, 256, 0, s>>>(pos, (const float*)vel, m, dt, L);
  else
    k_drift<double><<<g, 256, 0, s>>>(pos, (const double*)vel, m, dt, L);
  return hipGetLastError();
}

// Reverse sweep of the leapfrog (hot_kdk_vjp).  Between two force
// derivatives the cotangents move through the drift and the kicks:
//   vbar += xbar dt (drift),  gacc = c vbar (kick cotangent of a(x_k)),
// with c = dt/2 at the two ends of the trajectory and dt inside, where the
// closing kick of one step and the opening kick of the next share a(x_k).
template <typename T>
__global__ void __launch_bounds__(256) k_kdk_adj_drift(T* __restrict__ vbar,
                                                       const double* __restrict__ xbar,
                                                       T* __restrict__ gacc, size_t m, double dt,
                                                       double c, int drift) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  T v = vbar[i];
  if (drift) {
    v = (T)((double)v + xbar[i] * dt);
    vbar[i] = v;
  }
  gacc[i] = (T)((double)v * c);
}

// xbar += tx (3 n); mbar (+)= tm (n)
template <typename T>
__global__ void __launch_bounds__(256) k_kdk_adj_accum(double* __restrict__ xbar,
                                                       const double* __restrict__ tx,
                                                       T* __restrict__ mbar,
                                                       const T* __restrict__ tm, size_t n,
                                                       int first) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  xbar[i] += tx[i];
  if (mbar && i < n) mbar[i] = first ? tm[i] : mbar[i] + tm[i];
}

// byte-granular clear by a kernel (safe inside captured graphs)
__global__ void __launch_bounds__(256) k_zero(unsigned char* __restrict__ p, size_t bytes) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < bytes) p[i] = 0;
}

hipError_t zero_launch(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  k_zero<<<(unsigned)((bytes + 255) / 256), 256, 0, s>>>((unsigned char*)p, bytes);
  return hipGetLastError();
}

hipError_t kdk_adj_drift_launch(bool fp32, void* vbar, const double* xbar, void* gacc, size_t n,
                                double dt, double c, bool drift, hipStream_t s) {
  size_t m = 3 * n;
  unsigned g = (unsigned)((m + 255) / 256);
  if (fp32)
    k_kdk_adj_drift<float><<<g, 256, 0, s>>>((float*)vbar, xbar, (float*)gacc, m, dt, c, drift);
  else
    k_kdk_adj_drift<double><<<g, 256, 0, s>>>((double*)vbar, xbar, (double*)gacc, m, dt, c,
                                               drift);
  return hipGetLastError();
}

hipError_t kdk_adj_accum_launch(bool fp32, double* xbar, const double* tx, void* mbar,
                                const void* tm, size_t n, bool first, hipStream_t s) {
  unsigned g = (unsigned)((3 * n + 255) / 256);
  if (fp32)
    k_kdk_adj_accum<float><<<g, 256, 0, s>>>(xbar, tx, (float*)mbar, (const float*)tm, n, first);
  else
    k_kdk_adj_accum<double><<<g, 256, 0, s>>>(xbar, tx, (double*)mbar, (const double*)tm, n,
                                               first);
  return hipGetLastError();
}

// direct pairs = n_A (n_A - 1 + sum of listed leaf counts); multipole pairs =
// n_A x (list length), summed over groups
__global__ void __launch_bounds__(256) k_count_pairs(Cells C, Groups G, uint32_t ngroups,
                                                     int local,
                                                     const uint32_t* __restrict__ list,
                                                     unsigned long long* __restrict__ out,
                                                     unsigned long long* __restrict__ slots) {
  uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long pp = 0, mp = 0, ms = 0, ts = 0, tp = 0, le = 0, lp = 0, lt = 0;
  // the listed leaves' particles of each of the wavefront's 64 groups, one
  // group at a time across the lanes (coalesced list reads); lane j keeps
  // group j's sum
  const int lane = threadIdx.x & 63;
  unsigned long long listed = 0;
  for (int j = 0; j < 64; ++j) {
    const uint32_t gj = g - (uint32_t)lane + (uint32_t)j;  // wave-uniform
    if (gj >= ngroups) break;
    if (G.active && !G.active[gj]) continue;
    const uint32_t off = G.off_p2p[gj], cnt = G.cnt_p2p[gj];
    unsigned long long v = 0;
    for (uint32_t q = (uint32_t)lane; q < cnt; q += 64) v += C.count[list[off + q] & kCellMask];
    for (int d = 1; d < 64; d <<= 1) v += __shfl_xor(v, d, 64);
    if (lane == j) listed = v;
  }
  if (g < ngroups && !(G.active && !G.active[g])) {
    const int A = G.cell[g];
    const unsigned long long na = C.count[A];
    const unsigned long long src = na - 1 + listed;
    pp = na * src;
    const unsigned long long cm = G.cnt_m2p[g];
    mp = na * cm;
    // lane-steps of the multipole kernel: the main pass takes every pass of
    // more than 32 targets on 64 lanes; the tail pass a last pass of at most
    // 32 targets on sub-groups of 32, 16 or 8 lanes
    const unsigned long long rem = na % 64;
    const bool tail = rem != 0 && rem <= 32;
    ms = 64ull * (na / 64 + (rem > 32 ? 1 : 0)) * cm;
    if (tail) {
      ts = (rem <= 8 ? 8ull : rem <= 16 ? 16ull : 32ull) * cm;
      tp = rem * cm;
    }
    // the local route: entries, the sink-cell interactions they stand for,
    // and the sinks that evaluate a local expansion
    if (local) {
      le = G.cnt_m2l[g];
      lp = na * le;
      lt = le > 0 ? na : 0;
    }
  }
  // wave reduction, then one atomic per wave
  for (int d = 32; d > 0; d >>= 1) {
    pp += __shfl_down(pp, d, 64);
    mp += __shfl_down(mp, d, 64);
    ms += __shfl_down(ms, d, 64);
    ts += __shfl_down(ts, d, 64);
    tp += __shfl_down(tp, d, 64);
    le += __shfl_down(le, d, 64);
    lp += __shfl_down(lp, d, 64);
    lt += __shfl_down(lt, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&out[0], pp);
    atomicAdd(&out[1], mp);
    atomicAdd(&slots[0], ms);
    atomicAdd(&slots[1], ts);
    atomicAdd(&slots[2], tp);
    atomicAdd(&slots[3], le);
    atomicAdd(&slots[4], lp);
    atomicAdd(&slots[5], lt);
  }
}

hipError_t count_pairs(const Cells& C, const Groups& G, uint32_t ngroups, bool local,
                       const uint32_t* list, unsigned long long* out, unsigned long long* slots,
                       hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  k_count_pairs<<<(ngroups + 255) / 256, 256, 0, s>>>(C, G, ngroups, local ? 1 : 0, list, out,
                                                      slots);
  return hipGetLastError();
}

hipError_t rung_max_launch(const uint8_t* rung, size_t n, uint32_t* out, hipStream_t s) {
  const unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
  k_zero<<<1, 256, 0, s>>>((unsigned char*)out, 4);
  k_rung_max<<<g, 256, 0, s>>>(rung, n, out);
  return hipGetLastError();
}

}  // namespace hot

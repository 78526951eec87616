// Fixed-step kick-drift-kick leapfrog (the paper's Sec. 2.1 integrator is an
// adaptive symplectic one; the fixed-step leapfrog is its single-rung case),
// and the interaction counters reported with each force evaluation.
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
                                                     const uint32_t* __restrict__ list,
                                                     unsigned long long* __restrict__ out) {
  uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long pp = 0, mp = 0;
  if (g < ngroups) {
    const int A = G.cell[g];
    const unsigned long long na = C.count[A];
    unsigned long long src = na - 1;
    const uint32_t off = G.off_p2p[g], cnt = G.cnt_p2p[g];
    for (uint32_t q = 0; q < cnt; ++q) src += C.count[list[off + q] & kCellMask];
    pp = na * src;
    mp = na * (unsigned long long)G.cnt_m2p[g];
  }
  // wave reduction, then one atomic per wave
  for (int d = 32; d > 0; d >>= 1) {
    pp += __shfl_down(pp, d, 64);
    mp += __shfl_down(mp, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&out[0], pp);
    atomicAdd(&out[1], mp);
  }
}

hipError_t count_pairs(const Cells& C, const Groups& G, uint32_t ngroups, const uint32_t* list,
                       unsigned long long* out, hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  k_count_pairs<<<(ngroups + 255) / 256, 256, 0, s>>>(C, G, ngroups, list, out);
  return hipGetLastError();
}

}  // namespace hot

// libhotref: exact periodic accelerations and potentials of selected target
// particles by direct Ewald summation in FP64 on the GPU.  A measurement
// instrument, not part of the force path: it gives the rms force error of a
// tree evaluation at sizes no CPU reference reaches (one GPU's share of the
// paper's run, Sec. 3), on targets of the caller's choosing.  It shares no
// code, header or table with libhot's tree kernels.
//
// The periodic sum is split the textbook way (Ewald 1921):
//   psi(r) = sum_n erfc(a |r+nL|)/|r+nL|
//          + (1/(pi L)) sum_{h != 0} exp(-pi^2 h^2/(a^2 L^2)) / h^2 cos(2 pi h.r/L)
//          - pi/(a^2 L^3)
// with phi_i = -G sum_j m_j psi(x_i - x_j) (j = i: the regular part, the
// particle's own images) and a_i = -grad phi_i; the last term is the
// neutralising background.  Plummer softening eps replaces 1/|R| by
// (|R|^2+eps^2)^(-1/2) on every image closer than the real-space cut-off.
//
// Split a = 8/L.  Real space: every image of a source within r_c = 0.7 L of
// the target (erfc(5.6) = 1.6e-15; with positions in [0, L) these are among
// the 8 images that shift the minimum-image separation by at most one box
// per axis).  Reciprocal space: all h with pi^2 h^2/(a^2 L^2) <= 32
// (|h| <= 14.4; the first term left out is below 1e-16 of the leading one), half of
// them by the h <-> -h symmetry, through the structure factors
// C(h) = sum_j m_j cos(2 pi h.x_j/L) and S(h) = sum_j m_j sin(2 pi h.x_j/L).
// Softening beyond r_c is left out: there |R| >= 0.7 L and the change of a
// pair term is at most 1.5 eps^2/|R|^2 ~ 3 eps^2/L^2 of it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hotref.h"

namespace {

thread_local std::string g_err;

constexpr double kAlphaL = 8.0;      // split parameter times L
constexpr double kRcutL = 0.7;       // real-space cut-off over L
constexpr double kKcut = 32.0;       // pi^2 h^2 / (a L)^2 <= kKcut
constexpr int kHmax = 14;            // |h_a| <= kHmax covers the sphere
constexpr int kTT = 8;               // targets per real-space block
constexpr int kRB = 256;             // threads per real-space block
constexpr int kKB = 256;             // h vectors per structure-factor block
constexpr int kKP = 32;              // particles per LDS batch (structure factors)
constexpr int kKH = 4;               // h vectors per thread (structure factors)

size_t up(size_t x) { return (x + 255) / 256 * 256; }

struct Sizes {
  size_t nh;        // half-space reciprocal vectors
  size_t rchunk;    // sources per real-space block
  size_t nrc;       // real-space chunks
  size_t kchunk;    // particles per structure-factor block
  size_t nkc;       // structure-factor chunks
  size_t o_h, o_w, o_sf, o_kpart, o_rpart, total;
};

std::vector<int> half_space(double* w_out, double L) {
  // h != 0 with h_x > 0, or h_x = 0 and h_y > 0, or h_x = h_y = 0 and h_z > 0,
  // ordered by (h_x, h_y, h_z) so that neighbouring lanes share h_x and h_y
  std::vector<int> h;
  const double f = M_PI * M_PI / (kAlphaL * kAlphaL);
  for (int x = 0; x <= kHmax; ++x)
    for (int y = -kHmax; y <= kHmax; ++y)
      for (int z = -kHmax; z <= kHmax; ++z) {
        if (x == 0 && (y < 0 || (y == 0 && z <= 0))) continue;
        const int h2 = x * x + y * y + z * z;
        if (f * h2 > kKcut) continue;
        if (w_out) w_out[h.size() / 3] = std::exp(-f * h2) / h2;
        h.push_back(x);
        h.push_back(y);
        h.push_back(z);
      }
  (void)L;
  return h;
}

Sizes plan(size_t n, size_t nt) {
  Sizes z{};
  z.nh = half_space(nullptr, 1.0).size() / 3;
  z.rchunk = std::max<size_t>(65536, (n + 2047) / 2048);
  z.rchunk = (z.rchunk + kRB - 1) / kRB * kRB;
  z.nrc = (n + z.rchunk - 1) / z.rchunk;
  z.kchunk = std::max<size_t>(16384, (n + 1023) / 1024);
  z.kchunk = (z.kchunk + kKP - 1) / kKP * kKP;
  z.nkc = (n + z.kchunk - 1) / z.kchunk;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o += up(b);
    return r;
  };
  z.o_h = take(4 * 3 * z.nh);
  z.o_w = take(8 * z.nh);
  z.o_sf = take(16 * z.nh);
  z.o_kpart = take(std::max<size_t>(16 * z.nh * z.nkc, 8 * 1024));  // also the mass partials
  const size_t ntt = (nt + kTT - 1) / kTT;
  z.o_rpart = take(32 * kTT * ntt * z.nrc);
  z.total = o;
  return z;
}

template <typename M>
__device__ __forceinline__ double mass_at(const M* m, size_t j) {
  return (double)m[j];
}

// real-space part of one block: kTT targets against a chunk of sources
template <typename M>
__global__ void __launch_bounds__(kRB) k_real(const double* __restrict__ pos, const M* __restrict__ mass,
                                              size_t n, const int64_t* __restrict__ tg, size_t nt,
                                              double L, double eps, size_t chunk,
                                              double* __restrict__ part) {
  const size_t t0 = (size_t)blockIdx.x * kTT;
  const size_t c = blockIdx.y;
  const double a = kAlphaL / L;
  const double rc2 = kRcutL * kRcutL * L * L;
  const double two_a_sqrtpi = 2.0 * a / sqrt(M_PI);
  const double e2 = eps * eps;
  double tx[kTT], ty[kTT], tz[kTT];
  int64_t ti[kTT];
  double ax[kTT], ay[kTT], az[kTT], ph[kTT];
#pragma unroll
  for (int k = 0; k < kTT; ++k) {
    const size_t t = t0 + k < nt ? t0 + k : nt - 1;
    ti[k] = (t0 + k < nt) ? tg[t] : -1;
    const int64_t i = tg[t];
    tx[k] = pos[i];
    ty[k] = pos[n + i];
    tz[k] = pos[2 * n + i];
    ax[k] = ay[k] = az[k] = ph[k] = 0.0;
  }
  const size_t j0 = c * chunk, j1 = (j0 + chunk < n) ? j0 + chunk : n;
  const double invL = 1.0 / L;
  for (size_t j = j0 + threadIdx.x; j < j1; j += kRB) {
    const double xj = pos[j], yj = pos[n + j], zj = pos[2 * n + j];
    const double mj = mass_at(mass, j);
#pragma unroll
    for (int k = 0; k < kTT; ++k) {
      // minimum-image separation target - source
      double d[3] = {tx[k] - xj, ty[k] - yj, tz[k] - zj};
      double sh[3];
      int can = 0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        d[q] -= L * rint(d[q] * invL);
        // the image one box the other way is within r_c only if |d| > 0.3 L
        sh[q] = (d[q] > 0.0) ? -L : L;
        if (fabs(d[q]) > (1.0 - kRcutL) * L) can |= 1 << q;
      }
      for (int msk = 0; msk < 8; ++msk) {
        if ((msk & can) != msk) continue;
        const double rx = d[0] + ((msk & 1) ? sh[0] : 0.0);
        const double ry = d[1] + ((msk & 2) ? sh[1] : 0.0);
        const double rz = d[2] + ((msk & 4) ? sh[2] : 0.0);
        const double r2 = rx * rx + ry * ry + rz * rz;
        if (!(r2 < rc2)) continue;
        if (msk == 0 && j == (size_t)ti[k]) continue;  // the self pair
        const double r = sqrt(r2);
        const double ir = 1.0 / r;
        const double ec = erfc(a * r) * ir;
        const double ex = two_a_sqrtpi * exp(-a * a * r2);
        // Ewald real-space term plus the softening correction
        // (g_eps - g_0) and (K_eps - K_0)
        const double is = 1.0 / sqrt(r2 + e2);
        const double f = (ec + ex) * ir * ir + (is * is * is - ir * ir * ir);
        ph[k] -= mj * (ec + (is - ir));
        ax[k] -= mj * f * rx;
        ay[k] -= mj * f * ry;
        az[k] -= mj * f * rz;
      }
    }
  }
  // block reduction, fixed order
  __shared__ double red[kRB];
#pragma unroll 1
  for (int k = 0; k < kTT; ++k) {
    double v[4] = {ax[k], ay[k], az[k], ph[k]};
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      red[threadIdx.x] = v[q];
      __syncthreads();
      for (int s = kRB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[((c * gridDim.x + blockIdx.x) * kTT + k) * 4 + q] = red[0];
      __syncthreads();
    }
  }
}

// structure-factor partial sums of one block: kKH x kKB reciprocal vectors
// against a chunk of particles.  Per-axis phase tables e^(2 pi i k x/L),
// k = 0..kHmax, of kKP particles sit in LDS, built by powers of the k = 1
// phase (negative k by conjugation).
template <typename M>
__global__ void __launch_bounds__(kKB) k_sfac(const double* __restrict__ pos, const M* __restrict__ mass,
                                              size_t n, const int* __restrict__ hv, size_t nh,
                                              double L, size_t chunk, double2* __restrict__ part) {
  __shared__ double2 tab[kKP][3][kHmax + 1];
  __shared__ double ms[kKP];
  int hx[kKH], hy[kKH], hz[kKH];
  double C[kKH], S[kKH];
#pragma unroll
  for (int q = 0; q < kKH; ++q) {
    const size_t hi = ((size_t)blockIdx.x * kKH + q) * kKB + threadIdx.x;
    const bool live = hi < nh;
    hx[q] = live ? hv[3 * hi] : 0;
    hy[q] = live ? hv[3 * hi + 1] : 0;
    hz[q] = live ? hv[3 * hi + 2] : 0;
    C[q] = S[q] = 0.0;
  }
  const size_t j0 = (size_t)blockIdx.y * chunk, j1 = (j0 + chunk < n) ? j0 + chunk : n;
  const double invL = 1.0 / L;
  for (size_t b = j0; b < j1; b += kKP) {
    __syncthreads();
    if (threadIdx.x < kKP * 3) {
      const int p = threadIdx.x / 3, ax = threadIdx.x % 3;
      const size_t j = b + p;
      double s1 = 0.0, c1 = 1.0;
      if (j < j1) sincospi(2.0 * (pos[(size_t)ax * n + j] * invL), &s1, &c1);
      double cr = 1.0, ci = 0.0;
      for (int k = 0; k <= kHmax; ++k) {
        tab[p][ax][k] = make_double2(cr, ci);
        const double nr = cr * c1 - ci * s1;
        ci = cr * s1 + ci * c1;
        cr = nr;
      }
    }
    if (threadIdx.x < kKP) ms[threadIdx.x] = (b + threadIdx.x < j1) ? mass_at(mass, b + threadIdx.x) : 0.0;
    __syncthreads();
    for (int p = 0; p < kKP; ++p) {
      const double m = ms[p];
#pragma unroll
      for (int q = 0; q < kKH; ++q) {
        const double2 X = tab[p][0][hx[q]];
        double2 Y = tab[p][1][hy[q] < 0 ? -hy[q] : hy[q]];
        double2 Z = tab[p][2][hz[q] < 0 ? -hz[q] : hz[q]];
        if (hy[q] < 0) Y.y = -Y.y;
        if (hz[q] < 0) Z.y = -Z.y;
        const double xr = X.x * Y.x - X.y * Y.y, xi = X.x * Y.y + X.y * Y.x;
        C[q] += m * (xr * Z.x - xi * Z.y);
        S[q] += m * (xr * Z.y + xi * Z.x);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kKH; ++q) {
    const size_t hi = ((size_t)blockIdx.x * kKH + q) * kKB + threadIdx.x;
    if (hi < nh) part[(size_t)blockIdx.y * nh + hi] = make_double2(C[q], S[q]);
  }
}

__global__ void k_sfac_sum(const double2* __restrict__ part, size_t nh, size_t nkc,
                           double2* __restrict__ sf) {
  const size_t h = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  double C = 0.0, S = 0.0;
  for (size_t c = 0; c < nkc; ++c) {
    const double2 v = part[c * nh + h];
    C += v.x;
    S += v.y;
  }
  sf[h] = make_double2(C, S);
}

// one block per target: reciprocal-space terms, the real-space partial sums,
// the self and background terms
template <typename M>
__global__ void __launch_bounds__(256) k_finish(const double* __restrict__ pos, const M* __restrict__ mass,
                                                size_t n, const int64_t* __restrict__ tg, size_t nt,
                                                const int* __restrict__ hv, const double* __restrict__ w,
                                                const double2* __restrict__ sf, size_t nh,
                                                const double* __restrict__ rpart, size_t nrc,
                                                double L, double G, double mtot,
                                                double* __restrict__ acc, double* __restrict__ pot) {
  const size_t t = blockIdx.x;
  const int64_t i = tg[t];
  const double x[3] = {pos[i], pos[n + i], pos[2 * n + i]};
  const double invL = 1.0 / L;
  double kx = 0.0, ky = 0.0, kz = 0.0, kp = 0.0;
  for (size_t h = threadIdx.x; h < nh; h += blockDim.x) {
    const int a = hv[3 * h], b = hv[3 * h + 1], c = hv[3 * h + 2];
    const double th = 2.0 * ((double)a * (x[0] * invL) + (double)b * (x[1] * invL) +
                             (double)c * (x[2] * invL));
    double s, co;
    sincospi(th, &s, &co);
    const double2 F = sf[h];
    const double sn = s * F.x - co * F.y;   // sum_j m_j sin(th_i - th_j)
    const double cs = co * F.x + s * F.y;   // sum_j m_j cos(th_i - th_j)
    kx += w[h] * a * sn;
    ky += w[h] * b * sn;
    kz += w[h] * c * sn;
    kp += w[h] * cs;
  }
  __shared__ double red[4][256];
  red[0][threadIdx.x] = kx;
  red[1][threadIdx.x] = ky;
  red[2][threadIdx.x] = kz;
  red[3][threadIdx.x] = kp;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  // real space: the chunks' partial sums in order
  const size_t tb = t / kTT, tk = t % kTT, ntt = (nt + kTT - 1) / kTT;
  double r[4] = {0, 0, 0, 0};
  for (size_t c = 0; c < nrc; ++c)
    for (int q = 0; q < 4; ++q) r[q] += rpart[((c * ntt + tb) * kTT + tk) * 4 + q];
  const double a = kAlphaL / L;
  const double mi = mass_at(mass, (size_t)i);
  // both halves of reciprocal space: force -(4/L^2) sum_half w h sin,
  // potential -(2/(pi L)) sum_half w cos
  const double fk = -4.0 * invL * invL;
  acc[t] = G * (r[0] + fk * red[0][0]);
  acc[nt + t] = G * (r[1] + fk * red[1][0]);
  acc[2 * nt + t] = G * (r[2] + fk * red[2][0]);
  if (pot) {
    // regular self term (the k-space sum includes j = i) and background
    const double self = 2.0 * a / sqrt(M_PI) * mi;
    const double bg = M_PI / (a * a * L * L * L) * mtot;
    pot[t] = G * (r[3] - 2.0 / (M_PI * L) * red[3][0] + self + bg);
  }
}

// total mass: per-block partial sums (grid-stride), then one block adds them
constexpr int kMassBlocks = 1024;

template <typename M>
__global__ void __launch_bounds__(256) k_mass_part(const M* __restrict__ mass, size_t n,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (size_t j = (size_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (size_t)kMassBlocks * 256)
    s += mass_at(mass, j);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_mass_total(double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < kMassBlocks; j += 256) s += part[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[0] = red[0];
}

template <typename M>
hotref_status run(size_t n, const double* pos, const M* mass, size_t nt, const int64_t* tg,
                  double box, double G, double eps, double* acc, double* pot, char* ws,
                  hipStream_t s) {
  const Sizes z = plan(n, nt);
  std::vector<double> w(z.nh);
  std::vector<int> h = half_space(w.data(), box);
  int* d_h = reinterpret_cast<int*>(ws + z.o_h);
  double* d_w = reinterpret_cast<double*>(ws + z.o_w);
  double2* d_sf = reinterpret_cast<double2*>(ws + z.o_sf);
  double2* d_kp = reinterpret_cast<double2*>(ws + z.o_kpart);
  double* d_rp = reinterpret_cast<double*>(ws + z.o_rpart);
  hipError_t e = hipMemcpyAsync(d_h, h.data(), 4 * h.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_w, w.data(), 8 * w.size(), hipMemcpyHostToDevice, s);
  // the total mass for the background term, summed in the structure-factor
  // partial-sum region before the structure factors are computed
  double mtot = 0.0;
  if (e == hipSuccess) {
    double* part = reinterpret_cast<double*>(d_kp);
    k_mass_part<M><<<kMassBlocks, 256, 0, s>>>(mass, n, part);
    k_mass_total<<<1, 256, 0, s>>>(part);
    e = hipMemcpyAsync(&mtot, part, 8, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host tables stay alive until here
  if (e != hipSuccess) {
    g_err = std::string("hotref setup: ") + hipGetErrorString(e);
    return HOTREF_EDEVICE;
  }
  const size_t ntt = (nt + kTT - 1) / kTT;
  k_real<M><<<dim3((unsigned)ntt, (unsigned)z.nrc), kRB, 0, s>>>(pos, mass, n, tg, nt, box, eps,
                                                                z.rchunk, d_rp);
  k_sfac<M><<<dim3((unsigned)((z.nh + kKB * kKH - 1) / (kKB * kKH)), (unsigned)z.nkc), kKB, 0, s>>>(
      pos, mass, n, d_h, z.nh, box, z.kchunk, d_kp);
  k_sfac_sum<<<(unsigned)((z.nh + 255) / 256), 256, 0, s>>>(d_kp, z.nh, z.nkc, d_sf);
  k_finish<M><<<(unsigned)nt, 256, 0, s>>>(pos, mass, n, tg, nt, d_h, d_w, d_sf, z.nh, d_rp,
                                           z.nrc, box, G, mtot, acc, pot);
  e = hipGetLastError();
  if (e != hipSuccess) {
    g_err = std::string("hotref launch: ") + hipGetErrorString(e);
    return HOTREF_EDEVICE;
  }
  return HOTREF_OK;
}

}  // namespace

extern "C" {

size_t hotref_scratch_size(size_t n, size_t ntargets) { return plan(n, ntargets).total; }

hotref_status hotref_ewald(size_t n, const double* pos, const void* mass, int mass_fp32,
                           size_t ntargets, const int64_t* targets, double box, double G,
                           double eps, double* acc, double* pot, void* scratch,
                           size_t scratch_bytes, void* stream) {
  if (ntargets == 0) return HOTREF_OK;
  if (n == 0 || !pos || !mass || !targets || !acc || !scratch || !(box > 0.0) ||
      !(eps >= 0.0) || !std::isfinite(G) || n >= (size_t(1) << 40)) {
    g_err = "bad argument";
    return HOTREF_EINVAL;
  }
  if (scratch_bytes < plan(n, ntargets).total) {
    g_err = "scratch smaller than hotref_scratch_size()";
    return HOTREF_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  char* ws = static_cast<char*>(scratch);
  return mass_fp32 ? run(n, pos, static_cast<const float*>(mass), ntargets, targets, box, G, eps,
                         acc, pot, ws, s)
                   : run(n, pos, static_cast<const double*>(mass), ntargets, targets, box, G,
                         eps, acc, pot, ws, s);
}

const char* hotref_last_error(void) { return g_err.c_str(); }

}  // extern "C"

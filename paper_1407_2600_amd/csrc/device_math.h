// Device helpers shared by the force and adjoint kernels: cell geometry,
// reciprocal square root, compensated accumulation, dual numbers and the
// multipole evaluation.
#pragma once

#include <type_traits>
#include <utility>

#include "hot_internal.h"

namespace hot {

using ::fma;  // the float/double overloads, next to the dual-number ones below

__device__ __forceinline__ void center_of(uint64_t key, int level, double L, double c[3]) {
  uint32_t ix = 0, iy = 0, iz = 0;
  for (int b = 0; b < level; ++b) {
    ix |= (uint32_t)((key >> (3 * b + 2)) & 1ull) << b;
    iy |= (uint32_t)((key >> (3 * b + 1)) & 1ull) << b;
    iz |= (uint32_t)((key >> (3 * b)) & 1ull) << b;
  }
  double s = ldexp(L, -level);
  c[0] = ((double)ix + 0.5) * s;
  c[1] = ((double)iy + 0.5) * s;
  c[2] = ((double)iz + 0.5) * s;
}

// ---------------------------------------------------------------- octants
// the far field is expanded about the centres of the 8 level-1 cells
__device__ __forceinline__ void octant_center(int o, double L, double c[3]) {
  const double h = 0.5 * L;
  c[0] = ((double)((o >> 2) & 1) + 0.5) * h;
  c[1] = ((double)((o >> 1) & 1) + 0.5) * h;
  c[2] = ((double)(o & 1) + 0.5) * h;
}

// first sorted index whose key's top octal digit is >= o (keys ascend, and
// bit 63 is the placeholder, so the top digit is non-decreasing)
__device__ __forceinline__ size_t digit_lb(const uint64_t* __restrict__ skey, size_t n,
                                           uint64_t o) {
  size_t lo = 0, hi = n;
  while (lo < hi) {
    const size_t mid = lo + ((hi - lo) >> 1);
    if (((skey[mid] >> 60) & 7ull) < o)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// [beg, end) of the sorted particles in octant o
__device__ __forceinline__ void octant_range(const uint64_t* __restrict__ skey, size_t n, int o,
                                             size_t* beg, size_t* end) {
  *beg = digit_lb(skey, n, (uint64_t)o);
  *end = (o == 7) ? n : digit_lb(skey, n, (uint64_t)(o + 1));
}

// wavefront-level LDS exchange: orders this wavefront's LDS writes before its later LDS reads by other lanes
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// ---------------------------------------------------------- far-field help
// Moment sums over particles split the (a, b) exponent pairs of x^a y^b z^c
// among kFarWaves wavefronts (pair q goes to wavefront q mod kFarWaves).
constexpr int kFarWaves = 4;

template <int PF>
struct FarPairs {
  static constexpr int N = (PF + 1) * (PF + 2) / 2;
  int a[N], b[N];
  constexpr FarPairs() : a(), b() {
    int k = 0;
    for (int x = 0; x <= PF; ++x)
      for (int y = 0; y <= PF - x; ++y) {
        a[k] = x;
        b[k] = y;
        ++k;
      }
  }
};

// number of moments wavefront W accumulates
template <int PF>
__host__ __device__ constexpr int far_wave_terms(int W) {
  constexpr FarPairs<PF> fp{};
  int t = 0;
  for (int q = W; q < FarPairs<PF>::N; q += kFarWaves) t += PF - fp.a[q] - fp.b[q] + 1;
  return t;
}

// binomial coefficients C(n, k), n <= 2 * 12, exact in FP64 (built at
// compile time from Pascal's rule)
struct BinomTable {
  double v[25][25];
  constexpr BinomTable() : v() {
    for (int i = 0; i < 25; ++i) {
      v[i][0] = 1.0;
      for (int k = 1; k <= i; ++k) v[i][k] = v[i - 1][k - 1] + (k < i ? v[i - 1][k] : 0.0);
    }
  }
};
__constant__ constexpr BinomTable kBinom{};

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// accumulator: plain in FP64, (hi, lo) TwoSum pairs (Knuth) in FP32
template <typename T, int K = 4>
struct Acc {
  T hi[K];
  T lo[K];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < K; ++k) hi[k] = lo[k] = (T)0;
  }
  __device__ __forceinline__ void fold1(int k, T x) {
    if constexpr (std::is_same<T, float>::value) {
      T s = hi[k] + x;
      T bb = s - hi[k];
      T err = (hi[k] - (s - bb)) + (x - bb);
      hi[k] = s;
      lo[k] += err;
    } else {
      hi[k] += x;
    }
  }
  __device__ __forceinline__ void fold(const T x[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) fold1(k, x[k]);
  }
  __device__ __forceinline__ double get(int k) const { return (double)hi[k] + (double)lo[k]; }
};

// ------------------------------------------------------------- dual numbers
// value + first-order directional derivative: evaluating the multipole field
// on duals gives its Jacobian applied to a direction in one pass
template <typename T>
struct Dual {
  T v, d;
  __device__ __forceinline__ Dual() : v(0), d(0) {}
  __device__ __forceinline__ Dual(T x) : v(x), d(0) {}
  __device__ __forceinline__ Dual(T x, T y) : v(x), d(y) {}
  __device__ __forceinline__ Dual& operator+=(const Dual& o) {
    v += o.v;
    d += o.d;
    return *this;
  }
  __device__ __forceinline__ Dual& operator+=(T o) {
    v += o;
    return *this;
  }
};
template <typename T>
__device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator+(Dual<T> a, T b) { return {a.v + b, a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) {
  return {a.v * b.v, fma(a.v, b.d, a.d * b.v)};
}
template <typename T>
__device__ __forceinline__ Dual<T> operator*(T a, Dual<T> b) { return {a * b.v, a * b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, T b) { return {a.v * b, a.d * b}; }
template <typename T>
__device__ __forceinline__ Dual<T> fma(Dual<T> a, Dual<T> b, Dual<T> c) {
  return {fma(a.v, b.v, c.v), fma(a.v, b.d, fma(a.d, b.v, c.d))};
}
template <typename T>
__device__ __forceinline__ Dual<T> fma(T a, Dual<T> b, Dual<T> c) {
  return {fma(a, b.v, c.v), fma(a, b.d, c.d)};
}
template <typename T>
__device__ __forceinline__ Dual<T> fma(Dual<T> a, T b, Dual<T> c) {
  return {fma(a.v, b, c.v), fma(a.d, b, c.d)};
}
template <typename T>
__device__ __forceinline__ Dual<T> rsqrt_t(Dual<T> x) {
  const T r = rsqrt_t(x.v);
  return {r, (T)(-0.5) * r * r * r * x.d};
}

// ------------------------------------------------------ coefficient sources
// compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (N > 0) static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// value and gradient of sum_q c_q h^q over |q| <= PF (multi-index order), by
// nested Horner schemes in z, then y, then x, each carrying the partial
// derivatives it needs; V = double or Dual<double>.  out = (grad, value).
template <int PF, typename V>
__device__ __forceinline__ void local_horner(const double* __restrict__ cq, V hx, V hy, V hz,
                                             V out[4]) {
  V X = V(0.0), Xx = V(0.0), Xy = V(0.0), Xz = V(0.0);
  static_for<PF + 1>([&](auto AA) {
    constexpr int a = PF - AA;
    V Y = V(0.0), Yy = V(0.0), Yz = V(0.0);
    static_for<PF - a + 1>([&](auto BB) {
      constexpr int b = PF - a - BB;
      V Z = V(cq[mi_index(a, b, PF - a - b)]), Zz = V(0.0);
      static_for<PF - a - b>([&](auto CC) {
        constexpr int c = PF - a - b - 1 - CC;
        Zz = fma(Zz, hz, Z);
        Z = fma(Z, hz, V(cq[mi_index(a, b, c)]));
      });
      Yy = fma(Yy, hy, Y);
      Yz = fma(Yz, hy, Zz);
      Y = fma(Y, hy, Z);
    });
    Xx = fma(Xx, hx, X);
    Xy = fma(Xy, hx, Yy);
    Xz = fma(Xz, hx, Yz);
    X = fma(X, hx, Y);
  });
  out[0] = Xx;
  out[1] = Xy;
  out[2] = Xz;
  out[3] = X;
}

// a coefficient block in memory
template <typename C>
struct PtrCoef {
  const C* __restrict__ p;
  template <int I>
  __device__ __forceinline__ C get() const {
    return p[I];
  }
};

// A coefficient block held by one 16-lane row: lane l of the row holds
// coefficients l, l + 16, l + 32, ...; coefficient I reaches every lane of the
// row by a DPP row broadcast from lane I % 16.
template <int NR>
struct RowCoef {
  float r[NR];
  template <int I>
  __device__ __forceinline__ float get() const {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, r[I >> 4]), 0x150 + (I & 15), 0xF,
                                        0xF, true));
  }
  // the block at p (n values), read by the calling row (rl = lane within it)
  __device__ __forceinline__ void load(const float* __restrict__ p, int n, int rl) {
#pragma unroll
    for (int j = 0; j < NR; ++j) r[j] = rl + 16 * j < n ? p[rl + 16 * j] : 0.0f;
  }
};

// A coefficient block read by w lanes into registers (lane l of them holds
// values l, l + w, ...; w = 16 unless given), on its way to an LDS slot.
template <typename T, int NR>
struct RowBlock {
  T r[NR];
  __device__ __forceinline__ void load(const T* __restrict__ p, int n, int rl, int w = 16) {
#pragma unroll
    for (int j = 0; j < NR; ++j) r[j] = rl + w * j < n ? p[rl + w * j] : (T)0;
  }
  __device__ __forceinline__ void store(T* __restrict__ slot, int n, int rl, int w = 16) const {
#pragma unroll
    for (int j = 0; j < NR; ++j)
      if (rl + w * j < n) slot[rl + w * j] = r[j];
  }
};

// a coefficient source from a pointer (or a RowCoef as it is)
template <typename C>
__device__ __forceinline__ PtrCoef<C> as_src(const C* p) {
  return PtrCoef<C>{p};
}
template <typename C, int NR>
__device__ __forceinline__ const RowCoef<NR>& as_src(const RowCoef<NR>& r) {
  return r;
}

// offset of part (m, j) in a coefficient block
__host__ __device__ constexpr int part_offset(int P, bool dip, int m0, int j0) {
  int o = 0;
  for (int m = 0; m <= P; ++m)
    for (int j = 0; j <= part_jmax(P, m); ++j) {
      if (m == m0 && j == j0) return o;
      if (part_stored(m, m - j, dip)) o += part_size(m - j);
    }
  return o;
}

// ---------------------------------------------------------------- multipole
// Phi = rinv sum_m rho^m P_m(R),
// grad Phi = rinv sum_m rho^m grad P_m - rinv rho R sum_m (2m+1) rho^m P_m,
// with the per-cell coefficient layout described in hot_internal.h.  V is the
// value type (T or Dual<T>), C the coefficient type, CF the coefficient
// source (PtrCoef or RowCoef).  out = (grad Phi, Phi).
// monomials R^k, |k| <= D, in multi-index order; entries below K0 are
// already filled in (a caller may pass lower-degree monomials it has)
template <int D, int K0 = 1, typename V>
__device__ __forceinline__ void monomials(V Rx, V Ry, V Rz, V* mono) {
  constexpr MI<D> mi{};
  if constexpr (K0 == 0) mono[0] = V(1);
#pragma unroll
  for (int k = K0 > 1 ? K0 : 1; k < nt(D); ++k) {
    const int a = mi.a[k], b = mi.b[k], c = mi.c[k];
    if (a > 0)
      mono[k] = (a + b + c == 1) ? Rx : mono[mi_index(a - 1, b, c)] * Rx;
    else if (b > 0)
      mono[k] = (b + c == 1) ? Ry : mono[mi_index(a, b - 1, c)] * Ry;
    else
      mono[k] = (c == 1) ? Rz : mono[mi_index(a, b, c - 1)] * Rz;
  }
}

// the evaluation given rinv, rho and the monomials of degree <= max(P-1, 0)
template <int P, bool DIP, typename V, typename C, typename CF>
__device__ __forceinline__ void m2p_eval_pre(V Rx, V Ry, V Rz, V rinv, V rho, const V* mono,
                                             const CF& cf, V out[4]) {
  // accumulators take their first contribution by assignment (which parts
  // exist is known at compile time), so no addition of zero is emitted
  V Pm[P + 1], Vx[P + 1], Vy[P + 1], Vz[P + 1];
  static_for<P + 1>([&](auto M) {
    constexpr int m = M;
    constexpr int J = part_jmax(P, m);
    static_for<J + 1>([&](auto JJ) {
      constexpr int j = JJ;
      constexpr int d = m - j;
      // does an earlier part of this m exist (then accumulate)?
      constexpr bool firstP = [] {
        for (int i = 0; i < j; ++i)
          if (part_stored(m, m - i, DIP)) return false;
        return true;
      }();
      constexpr bool firstV = [] {
        for (int i = 0; i < j; ++i)
          if (part_stored(m, m - i, DIP) && m - i > 0) return false;
        return true;
      }();
      if constexpr (part_stored(m, d, DIP)) {
        constexpr int o = part_offset(P, DIP, m, j);
        if constexpr (d == 0) {
          const C c0 = cf.template get<o>();
          if constexpr (firstP)
            Pm[m] = V(c0);
          else
            Pm[m] = Pm[m] + c0;
        } else {
          constexpr int nk = nte(d - 1);
          constexpr int base = nt(d - 2);
          V vx = cf.template get<o>() * mono[base], vy = cf.template get<o + nk>() * mono[base],
            vz = cf.template get<o + 2 * nk>() * mono[base];
          static_for<nk - 1>([&](auto KK) {
            constexpr int k = KK + 1;
            vx = fma(cf.template get<o + k>(), mono[base + k], vx);
            vy = fma(cf.template get<o + nk + k>(), mono[base + k], vy);
            vz = fma(cf.template get<o + 2 * nk + k>(), mono[base + k], vz);
          });
          if constexpr (firstV) {
            Vx[m] = vx;
            Vy[m] = vy;
            Vz[m] = vz;
          } else {
            Vx[m] += vx;
            Vy[m] += vy;
            Vz[m] += vz;
          }
          const V dot = fma(Rx, vx, fma(Ry, vy, Rz * vz));
          if constexpr (firstP)
            Pm[m] = dot * (C)(1.0 / d);
          else
            Pm[m] = fma(dot, (C)(1.0 / d), Pm[m]);
        }
      }
    });
    // parts that do not exist for this m leave zero accumulators
    constexpr bool anyP = [] {
      for (int i = 0; i <= J; ++i)
        if (part_stored(m, m - i, DIP)) return true;
      return false;
    }();
    constexpr bool anyV = [] {
      for (int i = 0; i <= J; ++i)
        if (part_stored(m, m - i, DIP) && m - i > 0) return true;
      return false;
    }();
    if constexpr (!anyP) Pm[m] = V((C)0);
    if constexpr (!anyV) Vx[m] = Vy[m] = Vz[m] = V((C)0);
  });
  V Pv = Pm[P], Q = (C)(2 * P + 1) * Pm[P], Gx = Vx[P], Gy = Vy[P], Gz = Vz[P];
#pragma unroll
  for (int m = P - 1; m >= 0; --m) {
    Pv = fma(Pv, rho, Pm[m]);
    Q = fma(Q, rho, (C)(2 * m + 1) * Pm[m]);
    Gx = fma(Gx, rho, Vx[m]);
    Gy = fma(Gy, rho, Vy[m]);
    Gz = fma(Gz, rho, Vz[m]);
  }
  const V rq = rho * Q;
  out[0] = rinv * fma(-rq, Rx, Gx);
  out[1] = rinv * fma(-rq, Ry, Gy);
  out[2] = rinv * fma(-rq, Rz, Gz);
  out[3] = rinv * Pv;
}

template <int P, bool DIP, typename V, typename C, typename CF>
__device__ __forceinline__ void m2p_eval_src(V Rx, V Ry, V Rz, C eps2, const CF& cf, V out[4]) {
  const V u = fma(Rx, Rx, fma(Ry, Ry, fma(Rz, Rz, V(eps2))));
  const V rinv = rsqrt_t(u);
  const V rho = rinv * rinv;
  constexpr int DM = P > 0 ? P - 1 : 0;
  V mono[nt(DM)];
  mono[0] = V((C)1);
  monomials<DM>(Rx, Ry, Rz, mono);
  m2p_eval_pre<P, DIP, V, C>(Rx, Ry, Rz, rinv, rho, mono, cf, out);
}

template <int P, bool DIP, typename V, typename C>
__device__ __forceinline__ void m2p_eval(V Rx, V Ry, V Rz, C eps2, const C* __restrict__ cf,
                                         V out[4]) {
  m2p_eval_src<P, DIP, V, C>(Rx, Ry, Rz, eps2, PtrCoef<C>{cf}, out);
}
template <int P, bool DIP, typename V, typename C, int NR>
__device__ __forceinline__ void m2p_eval(V Rx, V Ry, V Rz, C eps2, const RowCoef<NR>& cf,
                                         V out[4]) {
  m2p_eval_src<P, DIP, V, C>(Rx, Ry, Rz, eps2, cf, out);
}

// The two multipole evaluations of one adjoint (target, cell) term at the
// same R: the order-P mass expansion on dual numbers along g (field and its
// derivative along g) and the order-P+1 expansion with dipole parts of the
// effective charges (plain).  The plain one reuses the value parts of the
// dual distance and monomials, which are the same operations.
template <int P, typename T, typename CF, typename EF>
__device__ __forceinline__ void m2p_eval_adj(T Rx, T Ry, T Rz, T gx, T gy, T gz, T eps2,
                                             const CF& cf, const EF& ef, Dual<T> fm[4],
                                             T fe[4]) {
  const Dual<T> X(Rx, gx), Y(Ry, gy), Z(Rz, gz);
  const Dual<T> u = fma(X, X, fma(Y, Y, fma(Z, Z, Dual<T>(eps2))));
  const Dual<T> rinv = rsqrt_t(u);
  const Dual<T> rho = rinv * rinv;
  constexpr int DM = P > 0 ? P - 1 : 0;
  Dual<T> mono[nt(DM)];
  mono[0] = Dual<T>((T)1);
  monomials<DM>(X, Y, Z, mono);
  m2p_eval_pre<P, false, Dual<T>, T>(X, Y, Z, rinv, rho, mono, cf, fm);
  T m5[nt(P)];
#pragma unroll
  for (int k = 0; k < nt(DM); ++k) m5[k] = mono[k].v;
  monomials<P, (P > 0 ? nt(DM) : 1)>(Rx, Ry, Rz, m5);
  m2p_eval_pre<P + 1, true, T, T>(Rx, Ry, Rz, rinv.v, rho.v, m5, ef, fe);
}

// One multipole-list record (16 bytes): the (image << 27) | cell entry in w,
// and in x, y, z the offset of the cell's image-shifted centre of mass from
// the sink group's cell centre, evaluated in FP64 by the walk and rounded to
// FP32 once.  FP32 kernels use that offset; FP64 kernels evaluate it again in
// FP64 from the entry.
template <typename T>
__device__ __forceinline__ int m2p_record(const uint4 r, const double4* __restrict__ walk,
                                          double L, const double cA[3], T c[3]) {
  const int B = (int)(r.w & kCellMask);
  if constexpr (sizeof(T) == 4) {
    c[0] = __uint_as_float(r.x);
    c[1] = __uint_as_float(r.y);
    c[2] = __uint_as_float(r.z);
  } else {
    const int img = (int)(r.w >> 27);
    const double4 w = walk[B];
    c[0] = (T)(w.x + (double)(img / 9 - 1) * L - cA[0]);
    c[1] = (T)(w.y + (double)((img / 3) % 3 - 1) * L - cA[1]);
    c[2] = (T)(w.z + (double)(img % 3 - 1) * L - cA[2]);
  }
  return B;
}

// Coefficient block of a cell from its raw Cartesian moments M_k about the
// expansion centre (|k| <= P):
//   C_{m,k} = (2m-1)!! (-1)^j / (2^j k!) sum_{|i|=j} M_{k+2i} / i!,  |k| = m - j,
// so that P_m(R) = sum_k C_{m,k} R^k; parts of degree d >= 1 are stored as
// gradient coefficients (k'_a + 1) C_{m, k'+e_a}, |k'| = d - 1.  Every output
// is a fixed linear combination of moments, tabulated at compile time as
// (output, moment, weight) terms.
__host__ __device__ constexpr double cfact(int n) {
  double f = 1.0;
  for (int q = 2; q <= n; ++q) f *= (double)q;
  return f;
}

template <int P, bool DIP>
__host__ __device__ constexpr int coef_terms() {
  int n = 0;
  for (int m = 0; m <= P; ++m)
    for (int j = 0; j <= part_jmax(P, m); ++j) {
      const int d = m - j;
      if (part_stored(m, d, DIP)) n += part_size(d) * nte(j);
    }
  return n;
}

template <int P, bool DIP>
struct CoefTable {
  static constexpr int N = coef_terms<P, DIP>();
  int o[N], m[N];
  double w[N];
  constexpr CoefTable() : o(), m(), w() {
    int n = 0, out = 0;
    for (int mm = 0; mm <= P; ++mm) {
      double dfact = 1.0;  // (2m-1)!!
      for (int q = 1; q <= 2 * mm - 1; q += 2) dfact *= (double)q;
      for (int j = 0; j <= part_jmax(P, mm); ++j) {
        const int d = mm - j;
        if (!part_stored(mm, d, DIP)) continue;
        double pre = dfact * ((j & 1) ? -1.0 : 1.0);
        for (int q = 0; q < j; ++q) pre *= 0.5;
        // one output (ka, kb, kc) times a scale: terms over |i| = j
        auto emit = [&](int ka, int kb, int kc, double scale) {
          for (int ia = j; ia >= 0; --ia)
            for (int ib = j - ia; ib >= 0; --ib) {
              const int ic = j - ia - ib;
              o[n] = out;
              m[n] = mi_index(ka + 2 * ia, kb + 2 * ib, kc + 2 * ic);
              w[n] = scale * pre / (cfact(ia) * cfact(ib) * cfact(ic) * cfact(ka) * cfact(kb) *
                                    cfact(kc));
              ++n;
            }
          ++out;
        };
        if (d == 0) {
          emit(0, 0, 0, 1.0);
        } else {
          for (int a = 0; a < 3; ++a)
            for (int x = d - 1; x >= 0; --x)
              for (int y = d - 1 - x; y >= 0; --y) {
                const int z = d - 1 - x - y;
                const int ka1 = (a == 0 ? x : a == 1 ? y : z) + 1;
                emit(x + (a == 0), y + (a == 1), z + (a == 2), (double)ka1);
              }
        }
      }
    }
  }
};

// first table term of output k (terms are in output order)
template <int P, bool DIP>
__host__ __device__ constexpr int coef_term_start(int k) {
  constexpr CoefTable<P, DIP> t{};
  int n = 0;
  while (n < t.N && t.o[n] < k) ++n;
  return n;
}

// the coefficient block of moments M, each coefficient stored to out as soon
// as it is summed (the table's terms in order, from zero), then the padding
template <int P, bool DIP, typename T>
__device__ __forceinline__ void coef_store(const double* __restrict__ M, T* __restrict__ out) {
  constexpr CoefTable<P, DIP> tab{};
  constexpr int NCF = coef_count(P, DIP);
  constexpr int STR = coef_stride(P, DIP);
  static_for<NCF>([&](auto K) {
    constexpr int k = K;
    constexpr int a = coef_term_start<P, DIP>(k), b = coef_term_start<P, DIP>(k + 1);
    double v = 0.0;
    static_for<b - a>([&](auto I) {
      constexpr int t = a + I;
      v += tab.w[t] * M[tab.m[t]];
    });
    out[k] = (T)v;
  });
#pragma unroll
  for (int k = NCF; k < STR; ++k) out[k] = (T)0;
}


// Shift of raw moments to a centre displaced by -d (moments M_c about a
// daughter's centre, d = daughter centre - new centre):
//   M_k += sum_{j <= k} C(k, j) Mc_j d^(k - j),
// as compile-time (k, j, k - j, binomial) terms.
__host__ __device__ constexpr double cbinom(int n, int k) {
  double b = 1.0;
  for (int q = 0; q < k; ++q) b = b * (double)(n - q) / (double)(q + 1);
  return b;
}

template <int P>
__host__ __device__ constexpr int shift_terms() {
  MI<P> mi{};
  int n = 0;
  for (int k = 0; k < nt(P); ++k)
    for (int j = 0; j < nt(P); ++j)
      if (mi.a[j] <= mi.a[k] && mi.b[j] <= mi.b[k] && mi.c[j] <= mi.c[k]) ++n;
  return n;
}

template <int P>
struct ShiftTable {
  static constexpr int N = shift_terms<P>();
  int k[N], j[N], r[N];
  double w[N];
  constexpr ShiftTable() : k(), j(), r(), w() {
    MI<P> mi{};
    int n = 0;
    for (int kk = 0; kk < nt(P); ++kk)
      for (int jj = 0; jj < nt(P); ++jj) {
        if (mi.a[jj] > mi.a[kk] || mi.b[jj] > mi.b[kk] || mi.c[jj] > mi.c[kk]) continue;
        k[n] = kk;
        j[n] = jj;
        r[n] = mi_index(mi.a[kk] - mi.a[jj], mi.b[kk] - mi.b[jj], mi.c[kk] - mi.c[jj]);
        w[n] = cbinom(mi.a[kk], mi.a[jj]) * cbinom(mi.b[kk], mi.b[jj]) *
               cbinom(mi.c[kk], mi.c[jj]);
        ++n;
      }
  }
};

// monomials d^k, |k| <= P, in multi-index order
template <int P>
__device__ __forceinline__ void monomials(const double d[3], double* mono) {
  constexpr MI<P> mi{};
  mono[0] = 1.0;
#pragma unroll
  for (int k = 1; k < nt(P); ++k) {
    const int a = mi.a[k], b = mi.b[k], c = mi.c[k];
    if (a > 0)
      mono[k] = mono[mi_index(a - 1, b, c)] * d[0];
    else if (b > 0)
      mono[k] = mono[mi_index(a, b - 1, c)] * d[1];
    else
      mono[k] = mono[mi_index(a, b, c - 1)] * d[2];
  }
}

template <int P>
__device__ __forceinline__ void shift_add(const double* __restrict__ Mch, const double d[3],
                                          double* M) {
  constexpr ShiftTable<P> T{};
  double mono[nt(P)];
  monomials<P>(d, mono);
#pragma unroll
  for (int t = 0; t < T.N; ++t) M[T.k[t]] += T.w[t] * (Mch[T.j[t]] * mono[T.r[t]]);
}

}  // namespace hot

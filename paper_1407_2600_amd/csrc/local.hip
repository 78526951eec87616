// Group-level local expansions (paper Sec. 2.1: source cells that have
// interactions in common with the sinks of a sink group are bundled with
// them, the dual-tree m x n blocking).  The cells of a group's local list
// are re-expanded once about the group's centre c (the middle of its tight
// box) instead of being evaluated at every sink:
//     S_n = n! L_n = sum_k Mt_k D_(n+k)(c - z),   |n| <= Q, |k| <= P,
// with Mt_k = (-1)^|k| M_k / k! (raw moments about the cell's centre of mass
// z) and D_m = d^m g the derivatives of the Newtonian Green's function
// g = 1/|R| (the route's acceptance bound covers leaving out softening).
// The derivatives come from the recurrence
//     |R|^2 |m| D_m = -(2|m|-1) sum_i m_i R_i D_(m-e_i)
//                     - (|m|-1) sum_i m_i (m_i - 1) D_(m-2 e_i),
// obtained by writing (|R|^2 + 2 R.h + |h|^2) g(R+h)^2 = 1, applying h.grad
// and matching powers of h.  g is harmonic, so D_m and S_n are traceless:
// D_(a,b,c+2) = -D_(a+2,b,c) - D_(a,b+2,c), and likewise S.  The same
// relation folds every moment with two or more z indices into moments of
// the same degree with fewer (Mt_(a,b,c) D_(n+(a,b,c)) = -Mt_(a,b,c)
// D_(n+(a+2,b,c-2)) - Mt_(a,b,c) D_(n+(a,b+2,c-2))), once per cell: the
// contraction then runs over the 2d+1 folded moments of degree d with at
// most one z index, for the 2d+1 such S_n, and needs D_m with at most two
// z indices only.  The dependent S_n follow by the trace relation.
// Every sink then takes Phi += sum_n L_n (x - c)^n and its gradient.
//
// One wavefront per group: its lanes take the group's local-list entries
// one each (FP32 or FP64 arithmetic), the partial sums of S_n are added
// across the lanes in FP64 in a fixed order, and the lanes then evaluate the
// expansion at the group's sinks in FP64 and add it to their accumulators.
// The kernel runs between the direct and multipole kernels, when no other
// kernel writes the accumulators.
#include "device_math.h"

namespace hot {

constexpr int kLocalWaves = 4;

// (-1)^|k| / k! for |k| <= P, in multi-index order
template <int P>
struct LocalMomFac {
  double f[nt(P)];
  constexpr LocalMomFac() : f() {
    int n = 0;
    for (int d = 0; d <= P; ++d)
      for (int x = d; x >= 0; --x)
        for (int y = d - x; y >= 0; --y) {
          const int z = d - x - y;
          double v = 1.0;
          for (int i = 2; i <= x; ++i) v *= i;
          for (int i = 2; i <= y; ++i) v *= i;
          for (int i = 2; i <= z; ++i) v *= i;
          f[n++] = ((d % 2) ? -1.0 : 1.0) / v;
        }
  }
};

// 1 / n! for |n| <= Q, in multi-index order
template <int Q>
struct InvFactorial {
  double f[nt(Q)];
  constexpr InvFactorial() : f() {
    int n = 0;
    for (int d = 0; d <= Q; ++d)
      for (int x = d; x >= 0; --x)
        for (int y = d - x; y >= 0; --y) {
          const int z = d - x - y;
          double v = 1.0;
          for (int i = 2; i <= x; ++i) v *= i;
          for (int i = 2; i <= y; ++i) v *= i;
          for (int i = 2; i <= z; ++i) v *= i;
          f[n++] = 1.0 / v;
        }
  }
};

// components of multi-index number idx (multi-index order)
struct MIv {
  int a, b, c;
};
__host__ __device__ constexpr MIv mi_of(int idx) {
  int n = 0;
  for (int d = 0;; ++d)
    for (int x = d; x >= 0; --x)
      for (int y = d - x; y >= 0; --y) {
        if (n == idx) return MIv{x, y, d - x - y};
        ++n;
      }
}

// the folded moments kept per cell: at most one z index, no dipole (it
// vanishes about the centre of mass); fold_slot(k) is the place of moment k
// among them (multi-index order), -1 if it is not kept
__host__ __device__ constexpr bool fold_kept(int k) {
  const MIv v = mi_of(k);
  return v.c <= 1 && v.a + v.b + v.c != 1;
}
__host__ __device__ constexpr int fold_slot(int k) {
  if (!fold_kept(k)) return -1;
  int s = 0;
  for (int i = 0; i < k; ++i) s += fold_kept(i) ? 1 : 0;
  return s;
}
__host__ __device__ constexpr int fold_count(int P) {
  int s = 0;
  for (int i = 0; i < nt(P); ++i) s += fold_kept(i) ? 1 : 0;
  return s;
}

// the folded Mt of every cell (cell-major, fold_count(P) values of type T
// per cell), folded in FP64: in reverse multi-index order every component
// has received all that folds into it before it is itself folded away
template <int P, typename T>
__global__ void __launch_bounds__(256) k_local_moments(const double* __restrict__ mom,
                                                       uint32_t ncells, T* __restrict__ mt) {
  constexpr LocalMomFac<P> fac{};
  constexpr int NM = nt(P), NF = fold_count(P);
  const uint32_t c = blockIdx.x * 256 + threadIdx.x;
  if (c >= ncells) return;
  double v[NM];
  static_for<NM>([&](auto K) { v[K] = fac.f[K] * mom[(size_t)c * NM + K]; });
  static_for<NM>([&](auto KK) {
    constexpr int k = NM - 1 - KK;
    constexpr MIv kv = mi_of(k);
    if constexpr (kv.c >= 2) {
      v[mi_index(kv.a + 2, kv.b, kv.c - 2)] -= v[k];
      v[mi_index(kv.a, kv.b + 2, kv.c - 2)] -= v[k];
    }
  });
  static_for<NM>([&](auto K) {
    if constexpr (fold_kept(K)) {
      constexpr int slot = fold_slot(K);
      mt[(size_t)c * NF + slot] = (T)v[K];
    }
  });
}

// The lanes' re-expansion of one cell: D_m for |m| <= P+Q with at most two
// z indices, in multi-index order (the recurrence for at most one, the trace
// relation for two), each D_m added into the partial sums S_n of the
// independent n (c_n <= 1, n = m - k, k a folded moment) as soon as it
// exists, so that only the last degrees of D stay live.  Everything is
// unrolled at compile time.
template <int P, int Q, typename T>
__device__ __forceinline__ void m2l_entry(T Rx, T Ry, T Rz, const T* __restrict__ M, T* S) {
  constexpr int N = P + Q, ND = nt(N), NM = nt(P), NF = fold_count(P);
  T Mk[NF];
  static_for<NF>([&](auto I) { Mk[I] = M[I]; });
  const T s = Rx * Rx + Ry * Ry + Rz * Rz;
  const T d0 = rsqrt_t(s);
  const T is = d0 * d0;
  T mR[3][N + 1];
  static_for<N>([&](auto JJ) {
    constexpr int j = JJ + 1;
    mR[0][j] = (T)j * Rx;
    mR[1][j] = (T)j * Ry;
    mR[2][j] = (T)j * Rz;
  });
  T ad[N + 1], bd[N + 1];
  static_for<N>([&](auto DD) {
    constexpr int d = DD + 1;
    ad[d] = (T)(-(2.0 * d - 1.0) / d) * is;
    bd[d] = (T)(-(d - 1.0) / d) * is;
  });
  T D[ND];
  static_for<ND>([&](auto MM) {
    constexpr int m = MM;
    constexpr MIv mv = mi_of(m);
    constexpr int a = mv.a, b = mv.b, c = mv.c, d = a + b + c;
    if constexpr (c >= 3) {
      // not needed: m = n + k with c_n, c_k <= 1
    } else if constexpr (m == 0) {
      D[0] = d0;
    } else if constexpr (c == 2) {
      // traceless: (d/dz)^2 = -(d/dx)^2 - (d/dy)^2 on a harmonic function
      D[m] = -D[mi_index(a + 2, b, c - 2)] - D[mi_index(a, b + 2, c - 2)];
    } else {
      T u;
      if constexpr (a > 0) u = mR[0][a] * D[mi_index(a - 1, b, c)];
      if constexpr (b > 0) {
        if constexpr (a > 0)
          u = fma(mR[1][b], D[mi_index(a, b - 1, c)], u);
        else
          u = mR[1][b] * D[mi_index(a, b - 1, c)];
      }
      if constexpr (c > 0) {
        if constexpr (a > 0 || b > 0)
          u = fma(mR[2][c], D[mi_index(a, b, c - 1)], u);
        else
          u = mR[2][c] * D[mi_index(a, b, c - 1)];
      }
      if constexpr (a > 1 || b > 1) {
        T v;
        if constexpr (a > 1) v = (T)(a * (a - 1)) * D[mi_index(a - 2, b, c)];
        if constexpr (b > 1) {
          if constexpr (a > 1)
            v = fma((T)(b * (b - 1)), D[mi_index(a, b - 2, c)], v);
          else
            v = (T)(b * (b - 1)) * D[mi_index(a, b - 2, c)];
        }
        D[m] = fma(ad[d], u, bd[d] * v);
      } else {
        D[m] = ad[d] * u;
      }
    }
    // S_n += Mt_k D_m for every split m = n + k with n independent
    // (c_n <= 1), |n| <= Q, and k a folded moment
    static_for<NM>([&](auto KK) {
      constexpr int k = KK;
      constexpr MIv kv = mi_of(k);
      if constexpr (c <= 2 && fold_kept(k) && kv.a <= a && kv.b <= b && kv.c <= c &&
                    d - (kv.a + kv.b + kv.c) <= Q && c - kv.c <= 1) {
        constexpr int nidx = mi_index(a - kv.a, b - kv.b, c - kv.c);
        constexpr int slot = fold_slot(k);
        S[nidx] = fma(Mk[slot], D[m], S[nidx]);
      }
    });
  });
}

template <int P, int Q, typename T>
__global__ void __launch_bounds__(64 * kLocalWaves) k_m2l(Cells C, Groups G, uint32_t ngroups,
                                                          uint32_t gcap, double L,
                                                          const double* __restrict__ spos,
                                                          size_t n,
                                                          const uint32_t* __restrict__ list,
                                                          const T* __restrict__ mt,
                                                          double4* __restrict__ out) {
  constexpr int NF = fold_count(P), NQ = nt(Q);
  constexpr InvFactorial<Q> ifac{};
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t g = __builtin_amdgcn_readfirstlane(xcd_block() * kLocalWaves + wid);
  if (g >= ngroups) return;
  if (G.active && !G.active[g]) return;
  const uint32_t cnt = G.cnt_m2l[g];
  if (cnt == 0) return;
  // the group's local entries end where its accepted-cell region ends
  const uint32_t* __restrict__ ent = list + ((size_t)4 * G.off_m2l[g] - cnt);
  const double lo0 = G.lo[g], lo1 = G.lo[gcap + g], lo2 = G.lo[2 * (size_t)gcap + g];
  const double hi0 = G.hi[g], hi1 = G.hi[gcap + g], hi2 = G.hi[2 * (size_t)gcap + g];
  const double gc0 = 0.5 * (lo0 + hi0), gc1 = 0.5 * (lo1 + hi1), gc2 = 0.5 * (lo2 + hi2);

  // ---- the lanes' partial sums of n! L_n over their entries
  T S[NQ];  // only the entries with c_n <= 1 are used
  static_for<NQ>([&](auto I) { S[I] = (T)0; });
  for (uint32_t q = lane; q < cnt; q += 64) {
    // c - z from the cell's image-shifted centre of mass, in FP64 and then
    // rounded to the arithmetic type
    const uint32_t e = ent[q];
    const int B = (int)(e & kCellMask), img = (int)(e >> 27);
    const double4 w = C.walk[B];
    const T Rx = (T)(gc0 - (w.x + (double)(img / 9 - 1) * L));
    const T Ry = (T)(gc1 - (w.y + (double)((img / 3) % 3 - 1) * L));
    const T Rz = (T)(gc2 - (w.z + (double)(img % 3 - 1) * L));
    m2l_entry<P, Q, T>(Rx, Ry, Rz, mt + (size_t)B * NF, S);
  }
  // ---- sum over the lanes in FP64 (butterfly: every lane ends with the
  // sums), then the dependent S_n by the trace relation, and L_n = S_n / n!
  double Sd[NQ];
  static_for<NQ>([&](auto I) {
    constexpr MIv nv = mi_of(I);
    if constexpr (nv.c <= 1) {
      double v = (double)S[I];
#pragma unroll
      for (int w = 1; w < 64; w <<= 1) v += __shfl_xor(v, w, 64);
      Sd[I] = v;
    } else {
      Sd[I] = -Sd[mi_index(nv.a + 2, nv.b, nv.c - 2)] - Sd[mi_index(nv.a, nv.b + 2, nv.c - 2)];
    }
  });
  double Lc[NQ];
  static_for<NQ>([&](auto I) { Lc[I] = Sd[I] * ifac.f[I]; });
  // ---- evaluate at the group's sinks
  const int A = G.cell[g];
  const uint32_t first = C.first[A], count = C.count[A];
  for (uint32_t t = lane; t < count; t += 64) {
    const uint32_t s = first + t;
    double o4[4];
    local_horner<Q, double>(Lc, spos[s] - gc0, spos[n + s] - gc1, spos[2 * n + s] - gc2, o4);
    double4 o = out[s];
    o.x += o4[0];
    o.y += o4[1];
    o.z += o4[2];
    o.w += o4[3];
    out[s] = o;
  }
}

template <int P, int Q>
static hipError_t local_launch_pq(bool fp32, const Cells& C, const Groups& G, uint32_t ngroups,
                                  uint32_t gcap, double L, const double* spos, size_t n,
                                  const uint32_t* list, const void* mt, double4* out,
                                  hipStream_t s) {
  const unsigned nb = (ngroups + kLocalWaves - 1) / kLocalWaves;
  if (fp32)
    k_m2l<P, Q, float><<<nb, 64 * kLocalWaves, 0, s>>>(C, G, ngroups, gcap, L, spos, n, list,
                                                       (const float*)mt, out);
  else
    k_m2l<P, Q, double><<<nb, 64 * kLocalWaves, 0, s>>>(C, G, ngroups, gcap, L, spos, n, list,
                                                        (const double*)mt, out);
  return hipGetLastError();
}

template <int P>
static hipError_t local_launch_p(int q, bool fp32, const Cells& C, const Groups& G,
                                 uint32_t ngroups, uint32_t gcap, double L, const double* spos,
                                 size_t n, const uint32_t* list, const void* mt, double4* out,
                                 hipStream_t s) {
  switch (q) {
    case 2:
      return local_launch_pq<P, 2>(fp32, C, G, ngroups, gcap, L, spos, n, list, mt, out, s);
    case 4:
      return local_launch_pq<P, 4>(fp32, C, G, ngroups, gcap, L, spos, n, list, mt, out, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t local_moments_launch(bool fp32, int order, const double* mom, uint32_t ncells,
                                void* mt, hipStream_t s) {
  if (ncells == 0) return hipSuccess;
  const unsigned nb = (ncells + 255) / 256;
#define HOT_LM(P)                                                                        \
  case P:                                                                                \
    if (fp32)                                                                            \
      k_local_moments<P, float><<<nb, 256, 0, s>>>(mom, ncells, (float*)mt);             \
    else                                                                                 \
      k_local_moments<P, double><<<nb, 256, 0, s>>>(mom, ncells, (double*)mt);           \
    break;
  switch (order) {
    HOT_LM(0)
    HOT_LM(1)
    HOT_LM(2)
    HOT_LM(3)
    HOT_LM(4)
    default: return hipErrorInvalidValue;
  }
#undef HOT_LM
  return hipGetLastError();
}

hipError_t local_launch(bool fp32, int order, int q, const Cells& C, const Groups& G,
                        uint32_t ngroups, uint32_t gcap, double L, const double* spos, size_t n,
                        const uint32_t* list, const void* mt, double4* out, hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  switch (order) {
    case 0: return local_launch_p<0>(q, fp32, C, G, ngroups, gcap, L, spos, n, list, mt, out, s);
    case 1: return local_launch_p<1>(q, fp32, C, G, ngroups, gcap, L, spos, n, list, mt, out, s);
    case 2: return local_launch_p<2>(q, fp32, C, G, ngroups, gcap, L, spos, n, list, mt, out, s);
    case 3: return local_launch_p<3>(q, fp32, C, G, ngroups, gcap, L, spos, n, list, mt, out, s);
    case 4: return local_launch_p<4>(q, fp32, C, G, ngroups, gcap, L, spos, n, list, mt, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hot

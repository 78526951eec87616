// Host-side Taylor table of the periodic remainder (paper Sec. 2.1: a p=8
// local expansion accounts for the periodic images).  Built once per context
// in FP64.
//
// Psi(r) = psi_E(r) - sum_{|n|inf<=1} 1/|r + nL|, with the Ewald split
//   psi_E = sum_n erfc(a|r+nL|)/|r+nL|
//         + 1/(pi L) sum_{k!=0} exp(-pi^2 k^2/(a L)^2)/k^2 cos(2 pi k.r/L) - pi/(a^2 L^3),
// so Psi = sum_{|n|inf>=2} erfc/r  -  sum_{|n|inf<=1} erf/r  + reciprocal + const.
//
// For a radial term F(|c + h|) = G(s), s = |c+h|^2/2, the Taylor coefficients
// in h follow from the Faa di Bruno formula for a quadratic inner function:
//   d^t F / t! = sum_{2j <= t} c^(t-2j) / ((t-2j)! j! 2^|j|) G^(|t|-|j|)(|c|^2/2)
// (multi-index powers and factorials).  The s-derivatives of erfc(a r)/r are
// (-1)^m B_m(r) with Smith's recurrence
//   B_0 = erfc(a r)/r,  B_m = [(2m-1) B_{m-1} + (2a^2)^m/(a sqrt(pi)) e^{-a^2 r^2}] / r^2
// (W. Smith, "Point multipoles in the Ewald summation", 1982/1998), those of
// 1/r are (-1)^m (2m-1)!! r^-(2m+1), and at c = 0 the entire function
// erf(a r)/r has G^(m)(0) = (2a/sqrt(pi)) (-2a^2)^m / (2m+1).  The
// reciprocal terms are cos(a + w.h), a = w.r0, with coefficients
// c_{|t| mod 4} w^t / t!, c = (cos a, -sin a, -cos a, sin a).  Tables are
// built about an expansion point r0 (the offsets between octant centres).
#include <algorithm>
#include <cmath>
#include <vector>

#include "hot_internal.h"

namespace hot {

namespace {
struct Idx {
  std::vector<int> a, b, c;
  explicit Idx(int D) {
    for (int d = 0; d <= D; ++d)
      for (int x = d; x >= 0; --x)
        for (int y = d - x; y >= 0; --y) {
          a.push_back(x);
          b.push_back(y);
          c.push_back(d - x - y);
        }
  }
};

// add w * (Taylor coefficients of the radial term with s-derivatives Gm at
// the point c) to out; per axis W[t][j] = c^(t-2j) / ((t-2j)! j! 2^j)
void add_radial(const Idx& I, int D, const double c[3], const std::vector<double>& Gm, double w,
                const std::vector<double>& fact, double* out) {
  const int S = D + 1;
  std::vector<double> W(3 * S * S, 0.0);
  for (int a = 0; a < 3; ++a) {
    std::vector<double> pw(S, 1.0);
    for (int e = 1; e < S; ++e) pw[e] = pw[e - 1] * c[a];
    for (int t = 0; t < S; ++t)
      for (int j = 0; 2 * j <= t; ++j)
        W[(a * S + t) * S + j] = pw[t - 2 * j] / (fact[t - 2 * j] * fact[j] * std::ldexp(1.0, j));
  }
  const int N = (int)I.a.size();
  for (int q = 0; q < N; ++q) {
    const int ta = I.a[q], tb = I.b[q], tc = I.c[q];
    const int tdeg = ta + tb + tc;
    const double* Wx = &W[(0 * S + ta) * S];
    const double* Wy = &W[(1 * S + tb) * S];
    const double* Wz = &W[(2 * S + tc) * S];
    double acc = 0.0;
    for (int ja = 0; 2 * ja <= ta; ++ja) {
      if (Wx[ja] == 0.0) continue;
      for (int jb = 0; 2 * jb <= tb; ++jb) {
        const double xy = Wx[ja] * Wy[jb];
        if (xy == 0.0) continue;
        for (int jc = 0; 2 * jc <= tc; ++jc) acc += xy * Wz[jc] * Gm[tdeg - ja - jb - jc];
      }
    }
    out[q] += w * acc;
  }
}
}  // namespace

void psi_taylor_table(int D, double box, const double r0[3], double* out) {
  // first omitted real image is >= 4.5 L away: erfc(10.8) ~ 1e-52
  psi_taylor_table_split(D, box, r0, 2.4 / box, 4, 9, out);
}

void psi_taylor_table_split(int D, double box, const double r0[3], double alpha, int nreal,
                            int kmax, double* out) {
  const double L = box;
  Idx I(D);
  const int N = (int)I.a.size();
  for (int q = 0; q < N; ++q) out[q] = 0.0;
  std::vector<double> fact(D + 2, 1.0);
  for (int i = 1; i <= D + 1; ++i) fact[i] = fact[i - 1] * i;
  const double sqpi = std::sqrt(M_PI);
  std::vector<double> Gm(D + 1), B(D + 1);

  for (int nx = -nreal; nx <= nreal; ++nx)
    for (int ny = -nreal; ny <= nreal; ++ny)
      for (int nz = -nreal; nz <= nreal; ++nz) {
        const int ninf = std::max(std::abs(nx), std::max(std::abs(ny), std::abs(nz)));
        const double c[3] = {r0[0] + nx * L, r0[1] + ny * L, r0[2] + nz * L};
        const double r2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        if (r2 == 0.0) {
          // -erf(a r)/r about r = 0: only even multi-indices t = 2j
          for (int q = 0; q < N; ++q) {
            const int ta = I.a[q], tb = I.b[q], tc = I.c[q];
            if ((ta | tb | tc) & 1) continue;
            const int ja = ta / 2, jb = tb / 2, jc = tc / 2, jd = ja + jb + jc;
            const double g = 2.0 * alpha / sqpi * std::pow(-2.0 * alpha * alpha, jd) /
                             (2.0 * jd + 1.0);
            out[q] -= g / (fact[ja] * fact[jb] * fact[jc] * std::ldexp(1.0, jd));
          }
          continue;
        }
        if (ninf <= 1 && r2 < L * L) {
          // central image about an off-centre point: erfc/r - 1/r would cancel
          // many digits, so take the s-derivatives of the entire function
          // erf(a sqrt(2s))/sqrt(2s) = 2a/sqrt(pi) sum_k (-2a^2 s)^k/(k!(2k+1))
          // termwise: G^(m)(s0) = 2a/sqrt(pi) sum_{k>=m} (-2a^2)^k s0^(k-m)
          //                        / ((2k+1) (k-m)!)
          const double s0 = 0.5 * r2;
          for (int m = 0; m <= D; ++m) {
            double acc = 0.0;
            double term = std::pow(-2.0 * alpha * alpha, m);
            for (int k = m; k <= m + 80; ++k) {
              if (k > m) term *= -2.0 * alpha * alpha * s0 / (double)(k - m);
              acc += term / (2.0 * k + 1.0);
            }
            Gm[m] = -2.0 * alpha / sqpi * acc;
          }
          add_radial(I, D, c, Gm, 1.0, fact, out);
          continue;
        }
        const double r = std::sqrt(r2);
        const double ex = std::exp(-alpha * alpha * r2);
        B[0] = std::erfc(alpha * r) / r;
        double tw = 1.0;  // (2 a^2)^m
        for (int m = 1; m <= D; ++m) {
          tw *= 2.0 * alpha * alpha;
          B[m] = ((2.0 * m - 1.0) * B[m - 1] + tw / (alpha * sqpi) * ex) / r2;
        }
        if (ninf >= 2) {
          for (int m = 0; m <= D; ++m) Gm[m] = (m & 1 ? -1.0 : 1.0) * B[m];
        } else {
          // -erf/r = erfc/r - 1/r
          double inv = 1.0 / r;  // (2m-1)!! r^-(2m+1)
          for (int m = 0; m <= D; ++m) {
            if (m > 0) inv *= (2.0 * m - 1.0) / r2;
            Gm[m] = (m & 1 ? -1.0 : 1.0) * (B[m] - inv);
          }
        }
        add_radial(I, D, c, Gm, 1.0, fact, out);
      }

  // reciprocal space (k and -k give equal terms)
  const double pre = 1.0 / (M_PI * L);
  for (int kx = 0; kx <= kmax; ++kx)
    for (int ky = -kmax; ky <= kmax; ++ky)
      for (int kz = -kmax; kz <= kmax; ++kz) {
        if (kx == 0 && (ky < 0 || (ky == 0 && kz <= 0))) continue;
        const double k2 = (double)(kx * kx + ky * ky + kz * kz);
        const double A = 2.0 * pre * std::exp(-M_PI * M_PI * k2 / (alpha * alpha * L * L)) / k2;
        if (A < 1e-300) continue;
        const double w[3] = {2 * M_PI * kx / L, 2 * M_PI * ky / L, 2 * M_PI * kz / L};
        const double ph = w[0] * r0[0] + w[1] * r0[1] + w[2] * r0[2];
        const double cs[4] = {std::cos(ph), -std::sin(ph), -std::cos(ph), std::sin(ph)};
        double pw[3][64];
        for (int a = 0; a < 3; ++a) {
          pw[a][0] = 1.0;
          for (int e = 1; e <= D; ++e) pw[a][e] = pw[a][e - 1] * w[a];
        }
        for (int q = 0; q < N; ++q) {
          const int ta = I.a[q], tb = I.b[q], tc = I.c[q];
          const int td = ta + tb + tc;
          out[q] += A * cs[td & 3] * pw[0][ta] * pw[1][tb] * pw[2][tc] /
                    (fact[ta] * fact[tb] * fact[tc]);
        }
      }
  out[0] -= M_PI / (alpha * alpha * L * L * L);
}

}  // namespace hot

namespace hot {

// All 27 tables about the offsets (dx,dy,dz) L/2, dx,dy,dz in {-1,0,1}
// (table d = (dx+1)*9 + (dy+1)*3 + (dz+1)).  Psi has the symmetry of the cube
// (invariant under axis permutations and reflections), so only the centre,
// face, edge and corner offsets are computed; for r = R r_c with (R v)_{pi(i)}
// = s_i v_i,  T^r_t = prod_i s_i^(t_{pi(i)}) T^{r_c}_{(t_pi(0), t_pi(1), t_pi(2))}.
void psi_taylor_tables27(int D, double box, double* out) {
  const int N = nt(D);
  std::vector<double> canon(4 * (size_t)N);
  for (int k = 0; k < 4; ++k) {
    const double h = 0.5 * box;
    const double r0[3] = {k >= 1 ? h : 0.0, k >= 2 ? h : 0.0, k >= 3 ? h : 0.0};
    psi_taylor_table(D, box, r0, canon.data() + (size_t)k * N);
  }
  Idx I(D);
  for (int d = 0; d < 27; ++d) {
    const int r[3] = {d / 9 - 1, (d / 3) % 3 - 1, d % 3 - 1};
    int pi[3] = {0, 1, 2};
    // order axes by |r| descending (stable), so r_c = (1,..,1,0,..,0)
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j)
        if (std::abs(r[pi[j]]) > std::abs(r[pi[i]])) std::swap(pi[i], pi[j]);
    const int k = std::abs(r[0]) + std::abs(r[1]) + std::abs(r[2]);
    int sg[3];
    for (int i = 0; i < 3; ++i) sg[i] = r[pi[i]] < 0 ? -1 : 1;
    const double* src = canon.data() + (size_t)k * N;
    double* dst = out + (size_t)d * N;
    for (int q = 0; q < N; ++q) {
      const int t[3] = {I.a[q], I.b[q], I.c[q]};
      const int tp[3] = {t[pi[0]], t[pi[1]], t[pi[2]]};
      double sign = 1.0;
      for (int i = 0; i < 3; ++i)
        if (sg[i] < 0 && (tp[i] & 1)) sign = -sign;
      dst[q] = sign * src[mi_index(tp[0], tp[1], tp[2])];
    }
  }
}

}  // namespace hot

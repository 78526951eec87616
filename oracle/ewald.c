/* Ewald sums for the periodic box (oracle; test infrastructure only).
 *
 * The paper (Sec. 2.1) subtracts the uniform background density and treats
 * the periodic images beyond the nearest ones with a high-order (p=8) local
 * expansion, citing the periodic fast-multipole literature.  It gives no
 * formulas; the Ewald form used here is the textbook one for a unit point mass
 * in a cube of side L with a neutralising uniform background:
 *
 *   psi_E(r) = sum_n erfc(a|r+nL|)/|r+nL|
 *            + 1/(pi L) sum_{k!=0} exp(-pi^2 k^2/(a^2 L^2))/k^2 cos(2 pi k.r/L)
 *            - pi/(a^2 L^3)
 *
 * which is independent of the splitting parameter a (checked by the tests).
 * Psi(r) = psi_E(r) - sum_{|n|_inf<=1} 1/|r+nL| is the remainder that the
 * 27-image near field does not cover; its Taylor table at r=0 is computed by
 * 1-D series in u=|r|^2 composed with multivariate series in r.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define TWO_OVER_SQRTPI 1.1283791670955126

/* ---------------- direct Ewald potential ---------------- */

void or_ewald_psi(const double r[3], double L, double alpha, int nreal, int kmax,
                  double* psi, double grad[3]) {
  double p = 0.0, g[3] = {0, 0, 0};
  for (int nx = -nreal; nx <= nreal; ++nx)
    for (int ny = -nreal; ny <= nreal; ++ny)
      for (int nz = -nreal; nz <= nreal; ++nz) {
        double d[3] = {r[0] + nx * L, r[1] + ny * L, r[2] + nz * L};
        double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double e = erfc(alpha * rho) / rho;
        p += e;
        /* d/drho [erfc(a rho)/rho] */
        double dd = -(e + TWO_OVER_SQRTPI * alpha * exp(-alpha * alpha * rho * rho)) / rho;
        for (int a = 0; a < 3; ++a) g[a] += dd * d[a] / rho;
      }
  double pre = 1.0 / (M_PI * L);
  for (int kx = -kmax; kx <= kmax; ++kx)
    for (int ky = -kmax; ky <= kmax; ++ky)
      for (int kz = -kmax; kz <= kmax; ++kz) {
        if (!kx && !ky && !kz) continue;
        double k2 = (double)(kx * kx + ky * ky + kz * kz);
        double A = pre * exp(-M_PI * M_PI * k2 / (alpha * alpha * L * L)) / k2;
        double w[3] = {2 * M_PI * kx / L, 2 * M_PI * ky / L, 2 * M_PI * kz / L};
        double ph = w[0] * r[0] + w[1] * r[1] + w[2] * r[2];
        p += A * cos(ph);
        for (int a = 0; a < 3; ++a) g[a] -= A * w[a] * sin(ph);
      }
  p -= M_PI / (alpha * alpha * L * L * L);
  *psi = p;
  if (grad) { grad[0] = g[0]; grad[1] = g[1]; grad[2] = g[2]; }
}

double or_ewald_xi(double L, double alpha, int nreal, int kmax) {
  double p = 0.0;
  for (int nx = -nreal; nx <= nreal; ++nx)
    for (int ny = -nreal; ny <= nreal; ++ny)
      for (int nz = -nreal; nz <= nreal; ++nz) {
        if (!nx && !ny && !nz) continue;
        double rho = L * sqrt((double)(nx * nx + ny * ny + nz * nz));
        p += erfc(alpha * rho) / rho;
      }
  p -= TWO_OVER_SQRTPI * alpha; /* limit of -erf(a r)/r at r=0 */
  double pre = 1.0 / (M_PI * L);
  for (int kx = -kmax; kx <= kmax; ++kx)
    for (int ky = -kmax; ky <= kmax; ++ky)
      for (int kz = -kmax; kz <= kmax; ++kz) {
        if (!kx && !ky && !kz) continue;
        double k2 = (double)(kx * kx + ky * ky + kz * kz);
        p += pre * exp(-M_PI * M_PI * k2 / (alpha * alpha * L * L)) / k2;
      }
  p -= M_PI / (alpha * alpha * L * L * L);
  return p * L;
}

/* ---------------- Taylor table of the periodic remainder ---------------- */

/* 1-D Taylor coefficients (in delta = u-u0) of erfc(a sqrt(u))/sqrt(u) at
 * u0 > 0, orders 0..M.  erfc'(y) = -2/sqrt(pi) exp(-y^2) and y^2 = a^2 u, so
 * d/du erfc(a sqrt u) = -2/sqrt(pi) exp(-a^2 u) d(a sqrt u)/du; the series of
 * each factor is elementary. */
static void erfc_over_r_series(double u0, double a, int M, double* out) {
  double s[OR_DMAX + 3], is[OR_DMAX + 3], ex[OR_DMAX + 3], dy[OR_DMAX + 3];
  double er[OR_DMAX + 3], d[OR_DMAX + 3];
  double su = sqrt(u0);
  double c = 1.0, ci = 1.0;
  for (int m = 0; m <= M + 1; ++m) {
    /* binom(1/2,m) and binom(-1/2,m) */
    s[m] = su * c * pow(u0, -m);
    is[m] = ci / su * pow(u0, -m);
    c *= (0.5 - m) / (m + 1.0);
    ci *= (-0.5 - m) / (m + 1.0);
  }
  double e0 = exp(-a * a * u0);
  double f = 1.0;
  for (int m = 0; m <= M; ++m) {
    ex[m] = e0 * f; /* e0 (-a^2)^m / m! */
    f *= -a * a / (m + 1.0);
  }
  for (int m = 0; m <= M; ++m) dy[m] = a * (m + 1) * s[m + 1];
  for (int m = 0; m <= M; ++m) {
    double acc = 0.0;
    for (int i = 0; i <= m; ++i) acc += ex[i] * dy[m - i];
    d[m] = -TWO_OVER_SQRTPI * acc;
  }
  er[0] = erfc(a * su);
  for (int m = 1; m <= M; ++m) er[m] = d[m - 1] / m;
  for (int m = 0; m <= M; ++m) {
    double acc = 0.0;
    for (int i = 0; i <= m; ++i) acc += er[i] * is[m - i];
    out[m] = acc;
  }
}

static void inv_sqrt_series(double u0, int M, double* out) {
  double ci = 1.0;
  for (int m = 0; m <= M; ++m) {
    out[m] = ci / sqrt(u0) * pow(u0, -m);
    ci *= (-0.5 - m) / (m + 1.0);
  }
}

/* Multivariate series of F(|c+h|) where F(sqrt(u)) has 1-D coefficients phi
 * at u0=|c|^2: sum_m phi_m t^m with t = 2c.h + |h|^2; added (times w) to T. */
static void compose_radial(int D, const double c[3], const double* phi, int M, double w,
                           double* T) {
  int nt = or_nterms(D);
  double* t = calloc((size_t)nt, sizeof(double));
  double* P = calloc((size_t)nt, sizeof(double));
  double* Q = calloc((size_t)nt, sizeof(double));
  if (D >= 1) {
    t[or_mi(1, 0, 0)] = 2 * c[0];
    t[or_mi(0, 1, 0)] = 2 * c[1];
    t[or_mi(0, 0, 1)] = 2 * c[2];
  }
  if (D >= 2) {
    t[or_mi(2, 0, 0)] = 1;
    t[or_mi(0, 2, 0)] = 1;
    t[or_mi(0, 0, 2)] = 1;
  }
  P[0] = 1.0;
  T[0] += w * phi[0];
  for (int m = 1; m <= M; ++m) {
    or_ser_mul(D, t, P, Q);
    memcpy(P, Q, sizeof(double) * (size_t)nt);
    for (int i = 0; i < nt; ++i) T[i] += w * phi[m] * P[i];
  }
  free(t); free(P); free(Q);
}

/* Taylor coefficients of Psi about the point r0 (|r0|_inf <= L/2):
 * T_s = d^s Psi(r0) / s!.  Each real-space image term is a radial function
 * of |r0 + nL + h| expanded about c = r0 + nL; the reciprocal terms use
 * cos(a + w.h) = cos(a) cos(w.h) - sin(a) sin(w.h), a = w.r0. */
void or_psi_table_at(int D, double L, const double r0[3], double alpha, int nreal, int kmax,
                     double* T) {
  or_mi_init();
  int nt = or_nterms(D);
  memset(T, 0, sizeof(double) * (size_t)nt);
  double phi[OR_DMAX + 3], tmp[OR_DMAX + 3];
  for (int nx = -nreal; nx <= nreal; ++nx)
    for (int ny = -nreal; ny <= nreal; ++ny)
      for (int nz = -nreal; nz <= nreal; ++nz) {
        int ninf = abs(nx) > abs(ny) ? abs(nx) : abs(ny);
        if (abs(nz) > ninf) ninf = abs(nz);
        double c[3] = {r0[0] + nx * L, r0[1] + ny * L, r0[2] + nz * L};
        double u0 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        if (ninf >= 2) {
          erfc_over_r_series(u0, alpha, D, phi);
          compose_radial(D, c, phi, D, 1.0, T);
        } else if (u0 >= L * L) {
          /* -erf/r = erfc/r - 1/r */
          erfc_over_r_series(u0, alpha, D, phi);
          inv_sqrt_series(u0, D, tmp);
          for (int m = 0; m <= D; ++m) phi[m] -= tmp[m];
          compose_radial(D, c, phi, D, 1.0, T);
        } else if (u0 > 0.0) {
          /* close to the origin erfc/r - 1/r cancels many digits: expand the
           * entire function f(u) = erf(a sqrt u)/sqrt u
           *   = 2a/sqrt(pi) sum_k (-a^2 u)^k / (k! (2k+1))
           * about u0 directly: f^(m)(u0)/m! = 2a/sqrt(pi)
           *   sum_{k>=m} (-a^2)^k C(k,m) u0^(k-m) / (k! (2k+1)) */
          for (int m = 0; m <= D; ++m) {
            double acc = 0.0, term = 0.0;
            for (int k = m; k <= m + 80; ++k) {
              /* (-a^2)^k C(k,m) u0^(k-m) / k! = (-a^2)^k u0^(k-m) / (m! (k-m)!) */
              if (k == m) {
                term = pow(-alpha * alpha, m) / or_factorial(m);
              } else {
                term *= -alpha * alpha * u0 / (double)(k - m);
              }
              acc += term / (2.0 * k + 1.0);
            }
            phi[m] = -TWO_OVER_SQRTPI * alpha * acc;
          }
          compose_radial(D, c, phi, D, 1.0, T);
        } else {
          /* -erf(a sqrt u)/sqrt u at u0=0: entire series in u */
          double f = 1.0;
          for (int m = 0; m <= D; ++m) {
            phi[m] = -TWO_OVER_SQRTPI * alpha * f / (2.0 * m + 1.0);
            f *= -alpha * alpha / (m + 1.0);
          }
          compose_radial(D, c, phi, D / 2, 1.0, T);
        }
      }
  /* reciprocal space: cos(w.h) and sin(w.h) from the powers of w.h */
  double* lin = calloc((size_t)nt, sizeof(double));
  double* P = calloc((size_t)nt, sizeof(double));
  double* Q = calloc((size_t)nt, sizeof(double));
  double pre = 1.0 / (M_PI * L);
  for (int kx = -kmax; kx <= kmax; ++kx)
    for (int ky = -kmax; ky <= kmax; ++ky)
      for (int kz = -kmax; kz <= kmax; ++kz) {
        if (!kx && !ky && !kz) continue;
        double k2 = (double)(kx * kx + ky * ky + kz * kz);
        double A = pre * exp(-M_PI * M_PI * k2 / (alpha * alpha * L * L)) / k2;
        if (A == 0.0) continue;
        double w[3] = {2 * M_PI * kx / L, 2 * M_PI * ky / L, 2 * M_PI * kz / L};
        double a = w[0] * r0[0] + w[1] * r0[1] + w[2] * r0[2];
        double ca = cos(a), sa = sin(a);
        memset(lin, 0, sizeof(double) * (size_t)nt);
        if (D >= 1) {
          lin[or_mi(1, 0, 0)] = w[0];
          lin[or_mi(0, 1, 0)] = w[1];
          lin[or_mi(0, 0, 1)] = w[2];
        }
        memset(P, 0, sizeof(double) * (size_t)nt);
        P[0] = 1.0;
        T[0] += A * ca;
        double fact = 1.0;
        for (int m = 1; m <= D; ++m) {
          or_ser_mul(D, lin, P, Q);
          memcpy(P, Q, sizeof(double) * (size_t)nt);
          fact *= m;
          /* cos(a + x) = sum_m x^m/m! * {cos a, -sin a, -cos a, sin a}[m % 4] */
          double cm = (m % 4 == 0) ? ca : (m % 4 == 1) ? -sa : (m % 4 == 2) ? -ca : sa;
          double s = A * cm / fact;
          if (s == 0.0) continue;
          for (int i = 0; i < nt; ++i) T[i] += s * P[i];
        }
      }
  free(lin); free(P); free(Q);
  T[0] -= M_PI / (alpha * alpha * L * L * L);
}

void or_psi_table(int D, double L, double alpha, int nreal, int kmax, double* T) {
  const double r0[3] = {0.0, 0.0, 0.0};
  or_psi_table_at(D, L, r0, alpha, nreal, kmax, T);
}

/* ---------------- O1: direct periodic sum ---------------- */

static double wrapL(double x, double L) {
  if (x < 0.0) x += L;
  if (x >= L) x -= L;
  return x;
}

/* Exact periodic, softened, background-neutralised potential and
 * acceleration at the listed targets (original indices), by direct
 * summation over all sources:
 *   Phi_i = sum_{j!=i} m_j [psi_E(x_i-x_j) + sum_{|n|inf<=1} (g_eps-g_0)(x_i-x_j-nL)]
 *         + m_i [xi/L + sum_{n!=0,|n|inf<=1} (g_eps-g_0)(nL)]
 * with g_eps(r) = (|r|^2+eps^2)^(-1/2); pot = -G Phi, acc = G grad Phi.
 * The softening acts on the 27 nearest images of the wrapped positions (the
 * images the tree walks); all further images are unsoftened.  The reciprocal
 * part uses structure factors S(k) = sum_j m_j exp(2 pi i k.x_j / L). */
void or_direct_ewald(int64_t n, const double* pos, const double* mass, int64_t nt,
                     const int64_t* tgt, double L, double G, double eps, int kernel, double alpha,
                     int nreal, int kmax, double* acc, double* pot) {
  double* x[3];
  for (int a = 0; a < 3; ++a) {
    x[a] = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) x[a][i] = wrapL(pos[a * n + i], L);
  }
  double msum = 0.0;
  for (int64_t j = 0; j < n; ++j) msum += mass[j];
  /* half space of k vectors */
  int kw = 2 * kmax + 1;
  int nk = 0;
  int* kv = malloc(sizeof(int) * 3 * (size_t)kw * kw * kw);
  double* Ak = malloc(sizeof(double) * (size_t)kw * kw * kw);
  for (int kx = 0; kx <= kmax; ++kx)
    for (int ky = -kmax; ky <= kmax; ++ky)
      for (int kz = -kmax; kz <= kmax; ++kz) {
        if (kx == 0 && (ky < 0 || (ky == 0 && kz <= 0))) continue;
        double k2 = (double)(kx * kx + ky * ky + kz * kz);
        kv[3 * nk] = kx; kv[3 * nk + 1] = ky; kv[3 * nk + 2] = kz;
        Ak[nk] = 2.0 / (M_PI * L) * exp(-M_PI * M_PI * k2 / (alpha * alpha * L * L)) / k2;
        ++nk;
      }
  double* Sre = calloc((size_t)nk, sizeof(double));
  double* Sim = calloc((size_t)nk, sizeof(double));
#pragma omp parallel
  {
    double* lre = calloc((size_t)nk, sizeof(double));
    double* lim = calloc((size_t)nk, sizeof(double));
    double (*ec)[3] = malloc(sizeof(double[3]) * (size_t)kw);
    double (*es)[3] = malloc(sizeof(double[3]) * (size_t)kw);
#pragma omp for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
      for (int a = 0; a < 3; ++a)
        for (int k = -kmax; k <= kmax; ++k) {
          double ph = 2 * M_PI * k * x[a][j] / L;
          ec[k + kmax][a] = cos(ph);
          es[k + kmax][a] = sin(ph);
        }
      for (int q = 0; q < nk; ++q) {
        int i0 = kv[3 * q] + kmax, i1 = kv[3 * q + 1] + kmax, i2 = kv[3 * q + 2] + kmax;
        double cr = ec[i0][0] * ec[i1][1] - es[i0][0] * es[i1][1];
        double ci = ec[i0][0] * es[i1][1] + es[i0][0] * ec[i1][1];
        double dr = cr * ec[i2][2] - ci * es[i2][2];
        double di = cr * es[i2][2] + ci * ec[i2][2];
        lre[q] += mass[j] * dr;
        lim[q] += mass[j] * di;
      }
    }
#pragma omp critical
    for (int q = 0; q < nk; ++q) { Sre[q] += lre[q]; Sim[q] += lim[q]; }
    free(lre); free(lim); free(ec); free(es);
  }
  double xi = or_ewald_xi(L, alpha, nreal + 2, kmax);
  const int soft = eps > 0.0;
  /* self images of the softening correction */
  double self_soft = 0.0;
  for (int img = 0; img < 27; ++img) {
    if (img == 13) continue;
    double d[3] = {(img / 9 - 1) * L, ((img / 3) % 3 - 1) * L, (img % 3 - 1) * L};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double gs, fs;
    or_pair_kernel(kernel, r2, eps, &gs, &fs);
    self_soft += gs - 1.0 / sqrt(r2);
  }
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t t = 0; t < nt; ++t) {
    int64_t i = tgt[t];
    double xi_[3] = {x[0][i], x[1][i], x[2][i]};
    double phi = 0.0, g[3] = {0, 0, 0};
    /* reciprocal space */
    for (int q = 0; q < nk; ++q) {
      double w[3] = {2 * M_PI * kv[3 * q] / L, 2 * M_PI * kv[3 * q + 1] / L,
                     2 * M_PI * kv[3 * q + 2] / L};
      double ph = w[0] * xi_[0] + w[1] * xi_[1] + w[2] * xi_[2];
      double c = cos(ph), s = sin(ph);
      /* Re/Im of exp(i ph) * conj(S) */
      double re = c * Sre[q] + s * Sim[q];
      double im = s * Sre[q] - c * Sim[q];
      phi += Ak[q] * re;
      for (int a = 0; a < 3; ++a) g[a] -= Ak[q] * w[a] * im;
    }
    phi -= M_PI / (alpha * alpha * L * L * L) * msum;
    /* real space and near-image softening */
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r[3] = {xi_[0] - x[0][j], xi_[1] - x[1][j], xi_[2] - x[2][j]};
      double rm[3];
      for (int a = 0; a < 3; ++a) rm[a] = r[a] - L * nearbyint(r[a] / L);
      for (int nx = -nreal; nx <= nreal; ++nx)
        for (int ny = -nreal; ny <= nreal; ++ny)
          for (int nz = -nreal; nz <= nreal; ++nz) {
            double d[3] = {rm[0] + nx * L, rm[1] + ny * L, rm[2] + nz * L};
            double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double e = erfc(alpha * rho) / rho;
            double dd = -(e + TWO_OVER_SQRTPI * alpha * exp(-alpha * alpha * rho * rho)) / rho;
            phi += mass[j] * e;
            for (int a = 0; a < 3; ++a) g[a] += mass[j] * dd * d[a] / rho;
          }
      if (soft) {
        /* the softened kernel replaces the bare one on the 27 near images */
        for (int img = 0; img < 27; ++img) {
          double d[3] = {r[0] - (img / 9 - 1) * L, r[1] - ((img / 3) % 3 - 1) * L,
                         r[2] - (img % 3 - 1) * L};
          double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          double se, fe, s0 = 1.0 / sqrt(r2);
          or_pair_kernel(kernel, r2, eps, &se, &fe);
          phi += mass[j] * (se - s0);
          double f = -(fe - s0 * s0 * s0);
          for (int a = 0; a < 3; ++a) g[a] += mass[j] * f * d[a];
        }
      }
    }
    /* self term: real-space images of i itself, the -2a/sqrt(pi) limit,
     * and the softened near images; the reciprocal and background parts of
     * the self term are already in the structure-factor sum */
    double self_real = 0.0;
    for (int nx = -nreal - 2; nx <= nreal + 2; ++nx)
      for (int ny = -nreal - 2; ny <= nreal + 2; ++ny)
        for (int nz = -nreal - 2; nz <= nreal + 2; ++nz) {
          if (!nx && !ny && !nz) continue;
          double rho = L * sqrt((double)(nx * nx + ny * ny + nz * nz));
          self_real += erfc(alpha * rho) / rho;
        }
    phi += mass[i] * (self_real - TWO_OVER_SQRTPI * alpha + self_soft);
    (void)xi;
    for (int a = 0; a < 3; ++a) acc[a * nt + t] = G * g[a];
    if (pot) pot[t] = -G * phi;
  }
  free(kv); free(Ak); free(Sre); free(Sim);
  for (int a = 0; a < 3; ++a) free(x[a]);
}

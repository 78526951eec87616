/* Multi-indices and truncated multivariate power series (oracle; test
 * infrastructure only).
 *
 * The Taylor coefficients of the Green's function that the multipole
 * interactions need (paper Sec. 2.1: cells carry truncated multipole
 * expansions, quadrupole and hexadecapole at the leaves) are obtained here by
 * plain power-series algebra: g(R+h) = (u0 + 2R.h + |h|^2)^(-1/2) is expanded
 * with the binomial series in t = (2R.h + |h|^2)/u0.  No derivative recurrence
 * is used, so nothing here resembles the GPU library's contraction formulas.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

static int g_init = 0;
static int g_nt[OR_DMAX + 2];
static short g_a[4096], g_b[4096], g_c[4096], g_d[4096];
static int g_idx[OR_DMAX + 1][OR_DMAX + 1][OR_DMAX + 1];

void or_mi_init(void) {
  if (g_init) return;
  int n = 0;
  for (int d = 0; d <= OR_DMAX; ++d) {
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        int c = d - a - b;
        g_a[n] = (short)a; g_b[n] = (short)b; g_c[n] = (short)c; g_d[n] = (short)d;
        g_idx[a][b][c] = n;
        ++n;
      }
    g_nt[d] = n;
  }
  g_init = 1;
}

int or_nterms(int D) { or_mi_init(); return D < 0 ? 0 : g_nt[D]; }
int or_mi(int a, int b, int c) { or_mi_init(); return g_idx[a][b][c]; }
void or_mi_get(int idx, int* a, int* b, int* c) {
  or_mi_init(); *a = g_a[idx]; *b = g_b[idx]; *c = g_c[idx];
}
int or_mi_deg(int idx) { or_mi_init(); return g_d[idx]; }

double or_factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

void or_ser_mul(int D, const double* x, const double* y, double* out) {
  or_mi_init();
  int nt = g_nt[D];
  memset(out, 0, sizeof(double) * (size_t)nt);
  for (int i = 0; i < nt; ++i) {
    double xi = x[i];
    if (xi == 0.0) continue;
    int rem = D - g_d[i];
    int ntj = g_nt[rem];
    for (int j = 0; j < ntj; ++j) {
      int k = g_idx[g_a[i] + g_a[j]][g_b[i] + g_b[j]][g_c[i] + g_c[j]];
      out[k] += xi * y[j];
    }
  }
}

void or_green_taylor(int D, const double R[3], double eps2, double* T) {
  or_mi_init();
  int nt = g_nt[D];
  double u0 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2] + eps2;
  double t[4096], P[4096], Q[4096];
  memset(t, 0, sizeof(double) * (size_t)nt);
  if (D >= 1) {
    t[or_mi(1, 0, 0)] = 2.0 * R[0] / u0;
    t[or_mi(0, 1, 0)] = 2.0 * R[1] / u0;
    t[or_mi(0, 0, 1)] = 2.0 * R[2] / u0;
  }
  if (D >= 2) {
    t[or_mi(2, 0, 0)] = 1.0 / u0;
    t[or_mi(0, 2, 0)] = 1.0 / u0;
    t[or_mi(0, 0, 2)] = 1.0 / u0;
  }
  /* (1+t)^(-1/2) = sum_n binom(-1/2, n) t^n; t has no constant term, so the
   * powers beyond D vanish under truncation. */
  memset(P, 0, sizeof(double) * (size_t)nt);
  memset(T, 0, sizeof(double) * (size_t)nt);
  P[0] = 1.0;
  double cn = 1.0;
  T[0] = 1.0;
  for (int n = 1; n <= D; ++n) {
    cn *= (-0.5 - (double)(n - 1)) / (double)n;
    or_ser_mul(D, t, P, Q);
    memcpy(P, Q, sizeof(double) * (size_t)nt);
    for (int i = 0; i < nt; ++i) T[i] += cn * P[i];
  }
  double s = 1.0 / sqrt(u0);
  for (int i = 0; i < nt; ++i) T[i] *= s;
}

/* Oracle for the periodic tree-gravity force evaluation (test infrastructure).
 *
 * This is a plain, serial-per-target FP64 CPU implementation of what the GPU
 * library computes.  It exists to check the GPU library and is used only by
 * the tests, by the benchmark's CPU-baseline leg and by the smoke check; the
 * library never calls it, and the two share no code.
 *
 * Method (paper, Sec. 2.1 "2HOT"): particles get Morton keys, a hashed
 * oct-tree is built over the key-sorted list, cells carry truncated multipole
 * expansions, and each group of nearby sink particles walks the tree with a
 * multipole acceptance test, taking direct particle-particle interactions with
 * nearby leaves and multipole interactions with accepted cells.  Periodic
 * boundaries: the 27 nearest images are walked explicitly; all further images
 * enter through a high-order local expansion of the Ewald-summed remainder
 * (Sec. 2.1, the p=8 periodic local expansion).  The uniform background is
 * subtracted (Sec. 2.1) through the Ewald convention of a neutralising
 * background.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#define OR_DMAX 26 /* largest total degree of any power series */

typedef struct {
  double box, G, eps, theta;
  int order;      /* multipole order p of cells, 0..8 */
  int periodic;   /* 1: periodic box; 0: open boundaries (no images) */
  int leaf_max;   /* a cell with more particles than this is split */
  int group_max;  /* sink groups: largest cells with at most this many */
  int far_order;  /* order of the periodic local expansion */
  double err_tol; /* > 0: error-bound acceptance test (absolute acceleration
                     error allowed per accepted cell); 0: opening angle only */
  int kernel;     /* softening: 0 Plummer (eps), 1 Dehnen K1 of radius
                     (945/256) eps (Plummer-equivalent eps; kernel.c) */
  int local_order;  /* > 0: accepted cells far enough from a whole sink group
                       enter through a local expansion of this order about
                       the group's centre (tree.c); 0: none */
  double local_tol; /* absolute acceleration error allowed per cell for the
                       local expansion's truncation (> 0 to use it) */
} or_params;

/* ---- softening kernels (kernel.c) ---- */
/* pair functions g (potential) and f (force / r) at squared separation r2 */
void or_pair_kernel(int kernel, double r2, double eps, double* g, double* f);
/* support radius h of the K1 kernel for Plummer-equivalent softening eps */
double or_k1_radius(double eps);

/* ---- multi-indices and truncated power series (series.c) ---- */
void or_mi_init(void);
int or_nterms(int D);                /* number of multi-indices with |k| <= D */
int or_mi(int a, int b, int c);      /* index of (a,b,c) */
void or_mi_get(int idx, int* a, int* b, int* c);
int or_mi_deg(int idx);
double or_factorial(int n);
/* out = x*y truncated to total degree D (out must not alias x or y) */
void or_ser_mul(int D, const double* x, const double* y, double* out);
/* Taylor coefficients T_k(R) = d^k g(R) / k!, |k| <= D, of the softened
 * Green's function g(r) = (|r|^2 + eps^2)^(-1/2), by power-series algebra. */
void or_green_taylor(int D, const double R[3], double eps2, double* T);

/* ---- periodic remainder and Ewald sums (ewald.c) ---- */
/* Taylor table Tpsi_s = d^s Psi(0)/s!, |s| <= D, where Psi is the Ewald
 * potential minus the 27 nearest bare images. */
void or_psi_table(int D, double box, double alpha, int nreal, int kmax, double* T);
/* the same table about an expansion point r0 (|r0|_inf <= L/2) */
void or_psi_table_at(int D, double box, const double r0[3], double alpha, int nreal, int kmax,
                     double* T);
/* Ewald potential psi_E(r) of a unit mass with neutralising background
 * (value) and its gradient; r must not be a lattice vector. */
void or_ewald_psi(const double r[3], double box, double alpha, int nreal, int kmax,
                  double* psi, double grad[3]);
/* lim_{r->0} psi_E(r) - 1/r, times box (the Madelung-type constant xi). */
double or_ewald_xi(double box, double alpha, int nreal, int kmax);

#endif

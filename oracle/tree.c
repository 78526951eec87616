/* Same-acceptance-test FP64 tree code (oracle; test infrastructure only).
 *
 * Steps, in the order of the paper's Sec. 2.1:
 *  1. wrap positions into the box and assign each particle a 64-bit Morton
 *     key (the paper's Key; parent = key>>3, daughter = key<<3|octant);
 *  2. sort particles by key (ties by original index);
 *  3. build the oct-tree: a cell with more than leaf_max particles (and level
 *     below 21) is split into its non-empty daughters; cells are listed in
 *     pre-order, i.e. by (first particle, level);
 *  4. cell mass, centre of mass and raw Cartesian moments about the centre of
 *     mass, up to the multipole order (leaf quadrupole/hexadecapole);
 *  5. sink groups: the largest cells with at most group_max particles (or a
 *     leaf), sharing one interaction list per group (the m x n bundling);
 *  6. per group and per periodic image n in {-1,0,1}^3, a depth-first walk
 *     that accepts a cell for a multipole interaction when the acceptance
 *     test passes, takes a leaf that fails it as direct interactions, and
 *     opens other cells;
 *  7. forces: direct softened sums over the leaves, multipole interactions
 *     with the Taylor coefficients of the softened Green's function, and the
 *     periodic far field as local expansions about the 8 octant centres.
 *
 * Deterministic choices the paper leaves open are written out here so that an
 * independent implementation can reproduce keys, order, cells and lists bit
 * for bit: positions wrap by one add/subtract of L, quantise by
 * floor(x * (2^21/L)) clamped to 2^21-1, octant bits are (x,y,z) with x most
 * significant, the centre of mass is summed in key order at leaves and in
 * octant order over daughters (separate multiply and add, no fused
 * multiply-add), and the acceptance test is
 *     (s_B/theta + |com_B - centre_B|)^2 < d^2
 * with d the distance from com_B (shifted by the image) to the group's tight
 * bounding box, s_B the cell side.  This is the centre-of-mass opening
 * criterion with the offset correction of Barnes (1994) / Salmon & Warren
 * (1994), which keeps the expansion convergent for any theta < 1.
 *
 * With err_tol > 0 the opening radius is instead (or, with theta > 0 as
 * well, at least) the distance beyond which the Salmon & Warren (1994) bound
 * on the acceleration error of the order-p expansion,
 *     G B_(p+1) ((p+2) r - (p+1) b) / (r^(p+2) (r - b)^2),   r > b,
 * drops to err_tol (the paper sets its tolerance as an absolute acceleration
 * error, Sec. 2.1).  b is an upper bound on the distance of the cell's
 * particles from its centre of mass and B_(p+1) = sum m |x - com|^(p+1)
 * (order 0 is treated as order 1: the dipole about the centre of mass
 * vanishes).  Leaves sum B_k over their particles; above them B_2 follows
 * exactly by the parallel-axis identity, the other B_k and b are bounded
 * through the triangle inequality (binomially expanded powers), daughters in
 * octant order, and the radius is found by a fixed bisection in IEEE
 * operations only, so that any implementation reproduces it bit for bit.
 *
 * Group-level local expansions (local_order q > 0, local_tol > 0): the paper
 * bundles m source cells with the n sinks of a sink cell (Sec. 2.1, dual-tree
 * traversal).  A cell that passes the acceptance test and lies far from the
 * whole group is not evaluated at every sink; its order-p expansion is
 * instead re-expanded once about the group's centre c (the centre of its
 * tight box) to order q,
 *     L_n = sum_k (-1)^|k| C(n+k, k) M_k T_(n+k)(c - z),   |n| <= q,
 * with T_m(R) = d^m g(R)/m! the Taylor coefficients of the Newtonian Green's
 * function g = 1/|R| and z the cell's image-shifted centre of mass, and
 * every sink takes Phi += sum_n L_n (x - c)^n (and its gradient).  A sink
 * within a of c (a = half the diagonal of the tight box) sees every particle
 * of the cell at distance >= u = |c - z| - b.  For one point mass m the
 * acceleration error of the order-q truncation is at most
 *     G m t^q ((q+2) - (q+1) t) / (u^2 (1 - t)^2),   t = a/u < 1
 * (the Legendre expansion of 1/|x - s| about c, with |P_n| <= 1 and the
 * gradient of each solid harmonic of degree n bounded by (n+1) |y|^(n-1)),
 * and leaving out the Plummer softening changes its acceleration by at most
 * 1.5 G m eps^2 / (u - a)^4, u - a bounding the distance of any particle
 * from any sink (no change for the K1 kernel, whose accepted cells lie
 * beyond its radius).  The cell takes the local route when the sum of the
 * two with its mass is at most local_tol.  Written without divisions,
 *     A = G m a^q ((q+2) u - (q+1) a),   B = u^(q+1) (u - a)^2,
 *     C = 1.5 G m eps^2,                 D = (u - a)^4,
 * the test A D + C B <= local_tol B D is evaluated in this order of IEEE
 * operations (powers by repeated multiplication, a^q per group).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

#define MAXLEV 21
/* highest B_k carried up the tree: B_(p+1) at order p <= 4 */
#define OR_BK 5

typedef struct {
  uint64_t key;
  int level, is_leaf, nchild;
  int64_t first, count, parent;
  int64_t child[8];
  double m, mx[3], com[3], center[3], side, rcrit;
  double b2, bmax; /* sum m |x - com|^2 and a bound on max |x - com| */
  double bk[OR_BK + 1]; /* bounds on B_k = sum m |x - com|^k, k = 0..OR_BK
                           (B_0 = m, B_2 = b2 exactly) */
  double* M; /* raw moments about com, |k| <= order */
} cell_t;

typedef struct {
  int64_t n;
  int32_t* img;
  int64_t* cell;
  int64_t cap;
} list_t;

typedef struct {
  or_params p;
  int64_t n;
  double* x[3];    /* wrapped positions, original order */
  double* mass;    /* original order */
  uint64_t* key;   /* original order */
  int64_t* perm;   /* sorted -> original */
  double* sx[3];   /* sorted wrapped positions */
  double* sm;
  uint64_t* skey;
  cell_t* cells;
  int64_t ncells, ccap;
  int64_t* groups;
  int64_t ngroups;
  int64_t* group_of; /* sorted particle -> group number */
  double (*glo)[3];
  double (*ghi)[3];
  list_t* p2p;
  list_t* m2p;
  list_t* m2l; /* cells taken through the group's local expansion */
  int* gwalked;
  int walked;
  int nmom;          /* or_nterms(order) */
  /* periodic far field */
  int far_ok;
  double* Tpsi;  /* 27 tables (offsets between octant centres), |s| <= 2 far_order */
  double* Mroot; /* 8 octants x (|k| <= far_order) */
  double* Lam;   /* 8 octants x (|q| <= far_order) */
} tree_t;

/* ---------------- keys ---------------- */

static double wrap1(double x, double L) {
  if (x < 0.0) x += L;
  if (x >= L) x -= L;
  return x;
}

static uint64_t spread21(uint64_t v) {
  /* place bit b of v at bit 3b */
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ULL) << (3 * b);
  return r;
}

uint64_t or_key_of(double xw, double yw, double zw, double L) {
  double S = 2097152.0 / L;
  uint64_t q[3];
  double w[3] = {xw, yw, zw};
  for (int a = 0; a < 3; ++a) {
    double t = w[a] * S;
    uint64_t v = (uint64_t)(uint32_t)t;
    if (v > 2097151ULL) v = 2097151ULL;
    q[a] = v;
  }
  return (1ULL << 63) | (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
}

void or_keys(int64_t n, const double* pos, double L, uint64_t* keys, double* wrapped) {
  for (int64_t i = 0; i < n; ++i) {
    double w[3];
    for (int a = 0; a < 3; ++a) w[a] = wrap1(pos[a * n + i], L);
    keys[i] = or_key_of(w[0], w[1], w[2], L);
    if (wrapped)
      for (int a = 0; a < 3; ++a) wrapped[a * n + i] = w[a];
  }
}

typedef struct { uint64_t k; int64_t i; } kv_t;
static int kv_cmp(const void* A, const void* B) {
  const kv_t* a = A; const kv_t* b = B;
  if (a->k < b->k) return -1;
  if (a->k > b->k) return 1;
  return (a->i < b->i) ? -1 : (a->i > b->i);
}

void or_sort(int64_t n, const uint64_t* keys, int64_t* perm) {
  kv_t* kv = malloc(sizeof(kv_t) * (size_t)(n ? n : 1));
  for (int64_t i = 0; i < n; ++i) { kv[i].k = keys[i]; kv[i].i = i; }
  qsort(kv, (size_t)n, sizeof(kv_t), kv_cmp);
  for (int64_t i = 0; i < n; ++i) perm[i] = kv[i].i;
  free(kv);
}

/* ---------------- tree ---------------- */

static int64_t new_cell(tree_t* T) {
  if (T->ncells == T->ccap) {
    T->ccap = T->ccap ? 2 * T->ccap : 1024;
    T->cells = realloc(T->cells, sizeof(cell_t) * (size_t)T->ccap);
  }
  memset(&T->cells[T->ncells], 0, sizeof(cell_t));
  return T->ncells++;
}

static void cell_geometry(tree_t* T, cell_t* c) {
  /* integer cell coordinates from the key bits below the placeholder */
  uint64_t k = c->key;
  uint64_t ix = 0, iy = 0, iz = 0;
  for (int b = 0; b < c->level; ++b) {
    ix |= ((k >> (3 * b + 2)) & 1ULL) << b;
    iy |= ((k >> (3 * b + 1)) & 1ULL) << b;
    iz |= ((k >> (3 * b)) & 1ULL) << b;
  }
  c->side = ldexp(T->p.box, -c->level);
  c->center[0] = ((double)ix + 0.5) * c->side;
  c->center[1] = ((double)iy + 0.5) * c->side;
  c->center[2] = ((double)iz + 0.5) * c->side;
}

static int64_t build_rec(tree_t* T, int level, uint64_t key, int64_t first, int64_t count,
                         int64_t parent) {
  int64_t ci = new_cell(T);
  cell_t* c = &T->cells[ci];
  c->key = key; c->level = level; c->first = first; c->count = count; c->parent = parent;
  for (int o = 0; o < 8; ++o) c->child[o] = -1;
  cell_geometry(T, c);
  if (count > T->p.leaf_max && level < MAXLEV) {
    int shift = 3 * (MAXLEV - level - 1);
    int64_t s = first, end = first + count;
    for (int o = 0; o < 8; ++o) {
      int64_t b = s;
      while (s < end && (int)((T->skey[s] >> shift) & 7ULL) == o) ++s;
      if (s > b) {
        int64_t child = build_rec(T, level + 1, (key << 3) | (uint64_t)o, b, s - b, ci);
        c = &T->cells[ci]; /* realloc may move */
        c->child[o] = child;
        c->nchild++;
      }
    }
    c->is_leaf = 0;
  } else {
    c->is_leaf = 1;
  }
  return ci;
}

/* Salmon & Warren bound at distance r (see the header): separate IEEE
 * operations in a fixed order */
static double sw_bound(double gb, double b, int pe, double r) {
  double num = (double)(pe + 2) * r;
  num = num - (double)(pe + 1) * b;
  num = gb * num;
  double den = r;
  for (int i = 1; i < pe + 2; ++i) den = den * r;
  double rb = r - b;
  den = den * rb;
  den = den * rb;
  return num / den;
}

/* smallest radius (to bisection resolution) where the bound is <= tol;
 * bp = B_(pe+1), pe = max(p, 1) */
static double err_radius(double G, double bp, double b, int p, double tol) {
  int pe = p < 1 ? 1 : p;
  double gb = G * bp;
  if (!(gb > 0.0)) return b; /* a point mass: exact at any distance > b */
  double lo = b, hi = b + b;
  for (int i = 0; i < 4096 && sw_bound(gb, b, pe, hi) > tol; ++i) hi = hi + hi;
  for (int i = 0; i < 64; ++i) {
    double mid = 0.5 * (lo + hi);
    if (sw_bound(gb, b, pe, mid) <= tol)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

static void moments(tree_t* T) {
  int p = T->p.order;
  int nm = T->nmom;
  double theta = T->p.theta;
  /* children have larger indices than their parent: go backwards */
  for (int64_t ci = T->ncells - 1; ci >= 0; --ci) {
    cell_t* c = &T->cells[ci];
    double m = 0.0, mx[3] = {0.0, 0.0, 0.0};
    if (c->is_leaf) {
      for (int64_t s = c->first; s < c->first + c->count; ++s) {
        double ms = T->sm[s];
        m = m + ms;
        for (int a = 0; a < 3; ++a) {
          double t = ms * T->sx[a][s];
          mx[a] = mx[a] + t;
        }
      }
    } else {
      for (int o = 0; o < 8; ++o) {
        if (c->child[o] < 0) continue;
        cell_t* d = &T->cells[c->child[o]];
        m = m + d->m;
        for (int a = 0; a < 3; ++a) mx[a] = mx[a] + d->mx[a];
      }
    }
    c->m = m;
    for (int a = 0; a < 3; ++a) {
      c->mx[a] = mx[a];
      c->com[a] = (m != 0.0) ? mx[a] / m : c->center[a];
    }
    double dx = c->com[0] - c->center[0], dy = c->com[1] - c->center[1],
           dz = c->com[2] - c->center[2];
    double dd = dx * dx;
    dd = dd + dy * dy;
    dd = dd + dz * dz;
    double delta = sqrt(dd);
    /* second moment and extent about the centre of mass */
    /* B_k about the centre of mass: exact at leaves (sums over the
     * particles in key order); above them B_2 exactly by the parallel-axis
     * identity and the other B_k bounded through the triangle inequality,
     * |x - com| <= |x - com_d| + |com_d - com|, expanded binomially:
     *     B_k <= sum_d sum_j C(k, j) B_j(d) delta_d^(k-j),
     * daughters in octant order, j ascending */
    double b2 = 0.0, bmax = 0.0;
    double bk[OR_BK + 1];
    for (int k = 0; k <= OR_BK; ++k) bk[k] = 0.0;
    if (c->is_leaf) {
      double r2max = 0.0;
      for (int64_t s = c->first; s < c->first + c->count; ++s) {
        double ex = T->sx[0][s] - c->com[0], ey = T->sx[1][s] - c->com[1],
               ez = T->sx[2][s] - c->com[2];
        double r2 = ex * ex;
        r2 = r2 + ey * ey;
        r2 = r2 + ez * ez;
        double ms = T->sm[s];
        double t = ms * r2;
        b2 = b2 + t;
        if (r2 > r2max) r2max = r2;
        double r = sqrt(r2);
        double r3 = r2 * r, r4 = r2 * r2;
        double r5 = r4 * r;
        bk[1] = bk[1] + ms * r;
        bk[3] = bk[3] + ms * r3;
        bk[4] = bk[4] + ms * r4;
        bk[5] = bk[5] + ms * r5;
      }
      bmax = sqrt(r2max);
    } else {
      static const double binom[OR_BK + 1][OR_BK + 1] = {
          {1, 0, 0, 0, 0, 0}, {1, 1, 0, 0, 0, 0}, {1, 2, 1, 0, 0, 0},
          {1, 3, 3, 1, 0, 0}, {1, 4, 6, 4, 1, 0}, {1, 5, 10, 10, 5, 1}};
      for (int o = 0; o < 8; ++o) {
        if (c->child[o] < 0) continue;
        cell_t* d = &T->cells[c->child[o]];
        double ex = d->com[0] - c->com[0], ey = d->com[1] - c->com[1], ez = d->com[2] - c->com[2];
        double r2 = ex * ex;
        r2 = r2 + ey * ey;
        r2 = r2 + ez * ez;
        double t = d->m * r2;
        t = d->b2 + t;
        b2 = b2 + t;
        double dl = sqrt(r2);
        double e = d->bmax + dl;
        if (e > bmax) bmax = e;
        double dp[OR_BK + 1];
        dp[0] = 1.0;
        for (int k = 1; k <= OR_BK; ++k) dp[k] = dp[k - 1] * dl;
        for (int k = 1; k <= OR_BK; ++k) {
          if (k == 2) continue;
          double acc = 0.0;
          for (int j = 0; j <= k; ++j) {
            double u = binom[k][j] * d->bk[j];
            u = u * dp[k - j];
            acc = acc + u;
          }
          bk[k] = bk[k] + acc;
        }
      }
    }
    bk[0] = m;
    bk[2] = b2;
    for (int k = 0; k <= OR_BK; ++k) c->bk[k] = bk[k];
    c->b2 = b2;
    c->bmax = bmax;
    double rc = (theta > 0.0) ? c->side / theta + delta : 0.0;
    if (T->p.err_tol > 0.0) {
      int pe = p < 1 ? 1 : p;
      double re = err_radius(T->p.G, bk[pe + 1], bmax, p, T->p.err_tol);
      if (re > rc) rc = re;
    } else if (!(theta > 0.0)) {
      rc = INFINITY;
    }
    /* K1: accept only where every particle of the cell lies beyond the
     * kernel radius from every target, so that its Newtonian expansion is
     * the interaction it stands for */
    if (T->p.kernel == 1) {
      double rk = bmax + or_k1_radius(T->p.eps);
      if (rk > rc) rc = rk;
    }
    c->rcrit = rc;
    /* raw moments about the centre of mass, directly from the particles */
    c->M = calloc((size_t)nm, sizeof(double));
    for (int64_t s = c->first; s < c->first + c->count; ++s) {
      double d[3] = {T->sx[0][s] - c->com[0], T->sx[1][s] - c->com[1], T->sx[2][s] - c->com[2]};
      double pw[3][OR_DMAX + 1];
      for (int a = 0; a < 3; ++a) {
        pw[a][0] = 1.0;
        for (int e = 1; e <= p; ++e) pw[a][e] = pw[a][e - 1] * d[a];
      }
      for (int k = 0; k < nm; ++k) {
        int ka, kb, kc;
        or_mi_get(k, &ka, &kb, &kc);
        c->M[k] += T->sm[s] * pw[0][ka] * pw[1][kb] * pw[2][kc];
      }
    }
  }
}

static void groups_rec(tree_t* T, int64_t ci) {
  cell_t* c = &T->cells[ci];
  if (c->count <= T->p.group_max || c->is_leaf) {
    T->groups[T->ngroups++] = ci;
    return;
  }
  for (int o = 0; o < 8; ++o)
    if (c->child[o] >= 0) groups_rec(T, c->child[o]);
}

/* ---------------- far field ---------------- */

static double binom_mi(int qa, int qb, int qc, int ka, int kb, int kc) {
  /* C(q+k, q) per component */
  double r = 1.0;
  int q[3] = {qa, qb, qc}, k[3] = {ka, kb, kc};
  for (int a = 0; a < 3; ++a)
    r *= or_factorial(q[a] + k[a]) / (or_factorial(q[a]) * or_factorial(k[a]));
  return r;
}

/* octant (level-1 cell) of a wrapped position: the key's top octal digit */
static int octant_of(uint64_t key) { return (int)((key >> 60) & 7ULL); }

static void octant_center(const tree_t* T, int o, double c[3]) {
  double h = 0.5 * T->p.box;
  c[0] = ((double)((o >> 2) & 1) + 0.5) * h;
  c[1] = ((double)((o >> 1) & 1) + 0.5) * h;
  c[2] = ((double)(o & 1) + 0.5) * h;
}

/* Far field about the 8 octant centres c_o.  For a target in octant t and
 * the sources of octant s, Psi(x - y) is expanded about r0 = c_t - c_s (one
 * of 27 offsets of L/2 steps), with h = x - c_t and s_j = y_j - c_s:
 *   Lam^t_q = sum_s sum_k C(q+k, q) (-1)^|k| Tpsi^{c_t - c_s}_{q+k} M^s_k,
 *   M^s_k = sum_{j in s} m_j s_j^k,   Phi_far(x) = sum_q Lam^t_q h^q. */
static void far_setup(tree_t* T) {
  int pf = T->p.far_order;
  double L = T->p.box;
  int D = 2 * pf;
  int nT = or_nterms(D), nq = or_nterms(pf);
  T->Tpsi = calloc((size_t)27 * nT, sizeof(double));
  /* the tables depend only on (far_order, L): keep the last set */
  static double* cache = NULL;
  static int cache_D = -1;
  static double cache_L = 0.0;
#pragma omp critical(or_far_cache)
  {
    if (!(cache && cache_D == D && cache_L == L)) {
      free(cache);
      cache = calloc((size_t)27 * nT, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
      for (int d = 0; d < 27; ++d) {
        double r0[3] = {(d / 9 - 1) * 0.5 * L, ((d / 3) % 3 - 1) * 0.5 * L,
                        (d % 3 - 1) * 0.5 * L};
        /* alpha = 2/L; real images to |n|_inf = 4 (the first omitted image
         * is >= 4.5 L away: erfc(9) ~ 4e-37), reciprocal to |k|_inf = 6 */
        or_psi_table_at(D, L, r0, 2.0 / L, 4, 6, cache + (size_t)d * nT);
      }
      cache_D = D;
      cache_L = L;
    }
    memcpy(T->Tpsi, cache, sizeof(double) * 27 * (size_t)nT);
  }
  T->Mroot = calloc((size_t)8 * nq, sizeof(double));
  for (int64_t s = 0; s < T->n; ++s) {
    int o = octant_of(T->skey[s]);
    double c[3];
    octant_center(T, o, c);
    double d[3] = {T->sx[0][s] - c[0], T->sx[1][s] - c[1], T->sx[2][s] - c[2]};
    double pw[3][OR_DMAX + 1];
    for (int a = 0; a < 3; ++a) {
      pw[a][0] = 1.0;
      for (int e = 1; e <= pf; ++e) pw[a][e] = pw[a][e - 1] * d[a];
    }
    for (int k = 0; k < nq; ++k) {
      int ka, kb, kc;
      or_mi_get(k, &ka, &kb, &kc);
      T->Mroot[(size_t)o * nq + k] += T->sm[s] * pw[0][ka] * pw[1][kb] * pw[2][kc];
    }
  }
  T->Lam = calloc((size_t)8 * nq, sizeof(double));
  for (int t = 0; t < 8; ++t)
    for (int q = 0; q < nq; ++q) {
      int qa, qb, qc;
      or_mi_get(q, &qa, &qb, &qc);
      double acc = 0.0;
      for (int so = 0; so < 8; ++so) {
        int dx = ((t >> 2) & 1) - ((so >> 2) & 1), dy = ((t >> 1) & 1) - ((so >> 1) & 1),
            dz = (t & 1) - (so & 1);
        const double* Tp = T->Tpsi + (size_t)((dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)) * nT;
        const double* M = T->Mroot + (size_t)so * nq;
        for (int k = 0; k < nq; ++k) {
          int ka, kb, kc;
          or_mi_get(k, &ka, &kb, &kc);
          double sg = ((ka + kb + kc) % 2) ? -1.0 : 1.0;
          acc += binom_mi(qa, qb, qc, ka, kb, kc) * sg * Tp[or_mi(qa + ka, qb + kb, qc + kc)] * M[k];
        }
      }
      T->Lam[(size_t)t * nq + q] = acc;
    }
  T->far_ok = 1;
}

/* Phi_far(x) = sum_q Lam^t_q (x - c_t)^q and its gradient; t = octant of x */
static void far_eval(const tree_t* T, const double x[3], uint64_t key, double* phi, double g[3]) {
  int pf = T->p.far_order;
  int nq = or_nterms(pf);
  int t = octant_of(key);
  double c[3];
  octant_center(T, t, c);
  double h[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  double pw[3][OR_DMAX + 1];
  for (int a = 0; a < 3; ++a) {
    pw[a][0] = 1.0;
    for (int e = 1; e <= pf; ++e) pw[a][e] = pw[a][e - 1] * h[a];
  }
  const double* Lm = T->Lam + (size_t)t * nq;
  double P = 0.0, G[3] = {0, 0, 0};
  for (int q = 0; q < nq; ++q) {
    int qa, qb, qc;
    or_mi_get(q, &qa, &qb, &qc);
    double L = Lm[q];
    P += L * pw[0][qa] * pw[1][qb] * pw[2][qc];
    if (qa) G[0] += L * qa * pw[0][qa - 1] * pw[1][qb] * pw[2][qc];
    if (qb) G[1] += L * qb * pw[0][qa] * pw[1][qb - 1] * pw[2][qc];
    if (qc) G[2] += L * qc * pw[0][qa] * pw[1][qb] * pw[2][qc - 1];
  }
  *phi = P;
  for (int a = 0; a < 3; ++a) g[a] = G[a];
}

/* ---------------- public: build ---------------- */

void* or_tree_build(int64_t n, const double* pos, const double* mass, const or_params* prm) {
  or_mi_init();
  tree_t* T = calloc(1, sizeof(tree_t));
  T->p = *prm;
  T->n = n;
  double L = prm->box;
  for (int a = 0; a < 3; ++a) {
    T->x[a] = malloc(sizeof(double) * (size_t)(n ? n : 1));
    T->sx[a] = malloc(sizeof(double) * (size_t)(n ? n : 1));
  }
  T->mass = malloc(sizeof(double) * (size_t)(n ? n : 1));
  T->sm = malloc(sizeof(double) * (size_t)(n ? n : 1));
  T->key = malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
  T->skey = malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
  T->perm = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) T->x[a][i] = wrap1(pos[a * n + i], L);
    T->mass[i] = mass[i];
    T->key[i] = or_key_of(T->x[0][i], T->x[1][i], T->x[2][i], L);
  }
  or_sort(n, T->key, T->perm);
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = T->perm[s];
    for (int a = 0; a < 3; ++a) T->sx[a][s] = T->x[a][i];
    T->sm[s] = T->mass[i];
    T->skey[s] = T->key[i];
  }
  T->nmom = or_nterms(prm->order);
  if (n > 0) {
    build_rec(T, 0, 1ULL, 0, n, -1);
    moments(T);
    T->groups = malloc(sizeof(int64_t) * (size_t)T->ncells);
    groups_rec(T, 0);
    T->glo = malloc(sizeof(double[3]) * (size_t)T->ngroups);
    T->ghi = malloc(sizeof(double[3]) * (size_t)T->ngroups);
    T->group_of = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t g = 0; g < T->ngroups; ++g) {
      cell_t* c = &T->cells[T->groups[g]];
      for (int a = 0; a < 3; ++a) { T->glo[g][a] = INFINITY; T->ghi[g][a] = -INFINITY; }
      for (int64_t s = c->first; s < c->first + c->count; ++s) {
        T->group_of[s] = g;
        for (int a = 0; a < 3; ++a) {
          double v = T->sx[a][s];
          if (v < T->glo[g][a]) T->glo[g][a] = v;
          if (v > T->ghi[g][a]) T->ghi[g][a] = v;
        }
      }
    }
    if (prm->periodic) far_setup(T);
  }
  return T;
}

void or_tree_free(void* h) {
  tree_t* T = h;
  if (!T) return;
  for (int a = 0; a < 3; ++a) { free(T->x[a]); free(T->sx[a]); }
  free(T->mass); free(T->sm); free(T->key); free(T->skey); free(T->perm);
  for (int64_t c = 0; c < T->ncells; ++c) free(T->cells[c].M);
  free(T->cells); free(T->groups); free(T->glo); free(T->ghi); free(T->group_of);
  if (T->p2p) {
    for (int64_t g = 0; g < T->ngroups; ++g) {
      free(T->p2p[g].img); free(T->p2p[g].cell); free(T->m2p[g].img); free(T->m2p[g].cell);
      free(T->m2l[g].img); free(T->m2l[g].cell);
    }
    free(T->p2p); free(T->m2p); free(T->m2l); free(T->gwalked);
  }
  free(T->Tpsi); free(T->Mroot); free(T->Lam);
  free(T);
}

/* ---------------- walk ---------------- */

static void list_push(list_t* l, int img, int64_t cell) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 64;
    l->img = realloc(l->img, sizeof(int32_t) * (size_t)l->cap);
    l->cell = realloc(l->cell, sizeof(int64_t) * (size_t)l->cap);
  }
  l->img[l->n] = img;
  l->cell[l->n] = cell;
  l->n++;
}

static int is_ancestor_or_self(const cell_t* B, const cell_t* A) {
  if (B->level > A->level) return 0;
  return (A->key >> (3 * (A->level - B->level))) == B->key;
}

static int mac_accept(const tree_t* T, int64_t g, const cell_t* B, const int n[3]) {
  if (!(T->p.theta > 0.0) && !(T->p.err_tol > 0.0)) return 0;
  double L = T->p.box;
  double d[3];
  for (int a = 0; a < 3; ++a) {
    double c = B->com[a] + (double)n[a] * L;
    double lo = T->glo[g][a] - c, hi = c - T->ghi[g][a];
    double v = lo > hi ? lo : hi;
    d[a] = v > 0.0 ? v : 0.0;
  }
  double d2 = d[0] * d[0];
  d2 = d2 + d[1] * d[1];
  d2 = d2 + d[2] * d[2];
  double rc2 = B->rcrit * B->rcrit;
  return rc2 < d2;
}

/* centre c (middle of the tight box) and radius a (half its diagonal) of a
 * sink group, the expansion point of its local expansion */
static void group_centre(const tree_t* T, int64_t g, double c[3], double* a) {
  double e[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = 0.5 * (T->glo[g][k] + T->ghi[g][k]);
    e[k] = T->ghi[g][k] - c[k];
  }
  double a2 = e[0] * e[0];
  a2 = a2 + e[1] * e[1];
  a2 = a2 + e[2] * e[2];
  *a = sqrt(a2);
}

static double m2p_eps2(const tree_t* T);

/* an accepted cell takes the group's local expansion when the truncation
 * and softening bound of the header holds */
static int local_accept(const tree_t* T, int64_t g, const cell_t* B, const int n[3]) {
  const int q = T->p.local_order;
  if (q <= 0 || !(T->p.local_tol > 0.0)) return 0;
  double c[3], a;
  group_centre(T, g, c, &a);
  double L = T->p.box;
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = c[k] - (B->com[k] + (double)n[k] * L);
  double r2 = d[0] * d[0];
  r2 = r2 + d[1] * d[1];
  r2 = r2 + d[2] * d[2];
  double u = sqrt(r2) - B->bmax;
  if (!(u > a)) return 0;
  double aq = a;
  for (int i = 1; i < q; ++i) aq = aq * a;
  const double e2 = m2p_eps2(T);
  double gm = T->p.G * B->m;
  double A = gm * aq;
  A = A * ((double)(q + 2) * u - (double)(q + 1) * a);
  double uq = u;
  for (int i = 0; i < q; ++i) uq = uq * u; /* u^(q+1) */
  double w = u - a;
  double Bv = uq * w;
  Bv = Bv * w;
  double Cv = 1.5 * gm;
  Cv = Cv * e2;
  double w2 = w * w;
  double Dv = w2 * w2;
  double lhs = A * Dv;
  lhs = lhs + Cv * Bv;
  double rhs = Bv * Dv;
  rhs = T->p.local_tol * rhs;
  return lhs <= rhs;
}

static void walk_rec(tree_t* T, int64_t g, int img, const int n[3], int64_t bi) {
  const cell_t* A = &T->cells[T->groups[g]];
  const cell_t* B = &T->cells[bi];
  int zero = (n[0] == 0 && n[1] == 0 && n[2] == 0);
  if (zero && bi == T->groups[g]) return; /* own block: handled directly */
  if (!(zero && is_ancestor_or_self(B, A))) {
    if (mac_accept(T, g, B, n)) {
      if (local_accept(T, g, B, n))
        list_push(&T->m2l[g], img, bi);
      else
        list_push(&T->m2p[g], img, bi);
      return;
    }
    if (B->is_leaf) { list_push(&T->p2p[g], img, bi); return; }
  }
  for (int o = 0; o < 8; ++o)
    if (B->child[o] >= 0) walk_rec(T, g, img, n, B->child[o]);
}

static void ensure_lists(tree_t* T) {
  if (T->p2p) return;
  T->p2p = calloc((size_t)T->ngroups, sizeof(list_t));
  T->m2p = calloc((size_t)T->ngroups, sizeof(list_t));
  T->m2l = calloc((size_t)T->ngroups, sizeof(list_t));
  T->gwalked = calloc((size_t)T->ngroups, sizeof(int));
}

/* walk one sink group over all images (idempotent) */
static void walk_group(tree_t* T, int64_t g) {
  if (T->gwalked[g]) return;
  for (int img = 0; img < 27; ++img) {
    int n[3] = {img / 9 - 1, (img / 3) % 3 - 1, img % 3 - 1};
    if (!T->p.periodic && img != 13) continue;
    walk_rec(T, g, img, n, 0);
  }
  T->gwalked[g] = 1;
}

void or_tree_walk(void* h) {
  tree_t* T = h;
  if (T->walked || T->n == 0) return;
  ensure_lists(T);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t g = 0; g < T->ngroups; ++g) walk_group(T, g);
  T->walked = 1;
}

/* list of one group: returns its length; fills img/cell when non-NULL */
int64_t or_tree_group_list(void* h, int64_t g, int kind, int32_t* img, int64_t* cell) {
  tree_t* T = h;
  ensure_lists(T);
  walk_group(T, g);
  const list_t* l = kind == 2 ? &T->m2l[g] : kind ? &T->m2p[g] : &T->p2p[g];
  for (int64_t e = 0; e < l->n; ++e) {
    if (img) img[e] = l->img[e];
    if (cell) cell[e] = l->cell[e];
  }
  return l->n;
}

/* ---------------- forces ---------------- */

/* one source of mass m at (sx, sy, sz) acting on the target: Phi += m g,
 * grad Phi += m (source - target) f, with the softening kernel's g and f */
static void pair_add(double tx, double ty, double tz, double sx, double sy, double sz, double m,
                     int kernel, double eps, double* phi, double g[3]) {
  double d[3] = {sx - tx, sy - ty, sz - tz};
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double gv, fv;
  or_pair_kernel(kernel, r2, eps, &gv, &fv);
  *phi += m * gv;
  for (int a = 0; a < 3; ++a) g[a] += m * d[a] * fv;
}

/* multipole interactions expand the softened Green's function for Plummer
 * softening (so that a one-particle cell equals its direct interaction) and
 * the Newtonian one for the compact K1 kernel, whose cells are accepted only
 * when all their particles lie beyond its radius from every target */
static double m2p_eps2(const tree_t* T) {
  return T->p.kernel == 1 ? 0.0 : T->p.eps * T->p.eps;
}

static void m2p_add(const tree_t* T, const cell_t* B, const double R[3], double* phi,
                    double g[3]) {
  int p = T->p.order;
  double Tk[4096];
  or_green_taylor(p + 1, R, m2p_eps2(T), Tk);
  for (int k = 0; k < T->nmom; ++k) {
    int ka, kb, kc;
    or_mi_get(k, &ka, &kb, &kc);
    double sg = ((ka + kb + kc) % 2) ? -1.0 : 1.0;
    double Mk = sg * B->M[k];
    *phi += Mk * Tk[k];
    g[0] += Mk * (ka + 1) * Tk[or_mi(ka + 1, kb, kc)];
    g[1] += Mk * (kb + 1) * Tk[or_mi(ka, kb + 1, kc)];
    g[2] += Mk * (kc + 1) * Tk[or_mi(ka, kb, kc + 1)];
  }
}

/* adds the local expansion about c of one cell's order-p expansion (raw
 * moments M about its centre of mass z, R0 = c - z) to L_n, |n| <= q; the
 * tree passes eps2 = 0 (the route expands the Newtonian kernel) */
static void local_add(int p, int q, double eps2, const double* M, const double R0[3],
                      double* Lg) {
  const int nq = or_nterms(q), nm = or_nterms(p);
  double Tk[4096];
  or_green_taylor(p + q, R0, eps2, Tk);
  for (int ni = 0; ni < nq; ++ni) {
    int na, nb, nc;
    or_mi_get(ni, &na, &nb, &nc);
    double acc = 0.0;
    for (int k = 0; k < nm; ++k) {
      int ka, kb, kc;
      or_mi_get(k, &ka, &kb, &kc);
      double sg = ((ka + kb + kc) % 2) ? -1.0 : 1.0;
      acc += sg * binom_mi(na, nb, nc, ka, kb, kc) * M[k] * Tk[or_mi(na + ka, nb + kb, nc + kc)];
    }
    Lg[ni] += acc;
  }
}

/* Phi += sum_n L_n y^n and grad Phi += its gradient in y, |n| <= q */
static void local_poly(int q, const double* Lg, const double y[3], double* phi, double gr[3]) {
  double pw[3][OR_DMAX + 1];
  for (int k = 0; k < 3; ++k) {
    pw[k][0] = 1.0;
    for (int e = 1; e <= q; ++e) pw[k][e] = pw[k][e - 1] * y[k];
  }
  for (int ni = 0; ni < or_nterms(q); ++ni) {
    int na, nb, nc;
    or_mi_get(ni, &na, &nb, &nc);
    double Ln = Lg[ni];
    *phi += Ln * pw[0][na] * pw[1][nb] * pw[2][nc];
    if (na) gr[0] += Ln * na * pw[0][na - 1] * pw[1][nb] * pw[2][nc];
    if (nb) gr[1] += Ln * nb * pw[0][na] * pw[1][nb - 1] * pw[2][nc];
    if (nc) gr[2] += Ln * nc * pw[0][na] * pw[1][nb] * pw[2][nc - 1];
  }
}

/* local expansion of group g about its centre from the cells of its local
 * list, in list order */
static void group_local(const tree_t* T, int64_t g, double* Lg) {
  const int q = T->p.local_order;
  for (int i = 0; i < or_nterms(q); ++i) Lg[i] = 0.0;
  const list_t* ll = &T->m2l[g];
  double c[3], a;
  group_centre(T, g, c, &a);
  double L = T->p.box;
  for (int64_t e = 0; e < ll->n; ++e) {
    int img = ll->img[e];
    double sh[3] = {(img / 9 - 1) * L, ((img / 3) % 3 - 1) * L, (img % 3 - 1) * L};
    const cell_t* B = &T->cells[ll->cell[e]];
    double R[3] = {c[0] - (B->com[0] + sh[0]), c[1] - (B->com[1] + sh[1]),
                   c[2] - (B->com[2] + sh[2])};
    local_add(T->p.order, q, 0.0, B->M, R, Lg);
  }
}

static void local_eval(const tree_t* T, int64_t g, const double* Lg, const double x[3],
                       double* phi, double gr[3]) {
  double c[3], a;
  group_centre(T, g, c, &a);
  double y[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  local_poly(T->p.local_order, Lg, y, phi, gr);
}

/* accumulate Phi and grad Phi (grad w.r.t. the target position) at sorted
 * particle s of group g; Lg is the group's local expansion (NULL: none) */
static void target_eval(const tree_t* T, int64_t g, int64_t s, const double* Lg,
                        double* phi_out, double g_out[3]) {
  const cell_t* A = &T->cells[T->groups[g]];
  double L = T->p.box, eps = T->p.eps;
  int kern = T->p.kernel;
  double tx = T->sx[0][s], ty = T->sx[1][s], tz = T->sx[2][s];
  double phi = 0.0, gr[3] = {0, 0, 0};
  for (int64_t j = A->first; j < A->first + A->count; ++j) {
    if (j == s) continue;
    pair_add(tx, ty, tz, T->sx[0][j], T->sx[1][j], T->sx[2][j], T->sm[j], kern, eps, &phi, gr);
  }
  const list_t* lp = &T->p2p[g];
  for (int64_t e = 0; e < lp->n; ++e) {
    int img = lp->img[e];
    double sh[3] = {(img / 9 - 1) * L, ((img / 3) % 3 - 1) * L, (img % 3 - 1) * L};
    const cell_t* B = &T->cells[lp->cell[e]];
    for (int64_t j = B->first; j < B->first + B->count; ++j)
      pair_add(tx, ty, tz, T->sx[0][j] + sh[0], T->sx[1][j] + sh[1], T->sx[2][j] + sh[2],
               T->sm[j], kern, eps, &phi, gr);
  }
  const list_t* lm = &T->m2p[g];
  for (int64_t e = 0; e < lm->n; ++e) {
    int img = lm->img[e];
    double sh[3] = {(img / 9 - 1) * L, ((img / 3) % 3 - 1) * L, (img % 3 - 1) * L};
    const cell_t* B = &T->cells[lm->cell[e]];
    double R[3] = {tx - (B->com[0] + sh[0]), ty - (B->com[1] + sh[1]), tz - (B->com[2] + sh[2])};
    m2p_add(T, B, R, &phi, gr);
  }
  if (Lg) {
    double x[3] = {tx, ty, tz};
    local_eval(T, g, Lg, x, &phi, gr);
  }
  if (T->far_ok) {
    double pf, gf[3];
    double x[3] = {tx, ty, tz};
    far_eval(T, x, T->skey[s], &pf, gf);
    phi += pf;
    for (int a = 0; a < 3; ++a) gr[a] += gf[a];
  }
  *phi_out = phi;
  for (int a = 0; a < 3; ++a) g_out[a] = gr[a];
}

/* Forces for every particle (ngsel < 0) or for the particles of the listed
 * groups.  acc is 3 x n SoA in original order, pot is n (may be NULL);
 * entries of unselected particles are left untouched. */
void or_tree_forces(void* h, int64_t ngsel, const int64_t* gsel, double* acc, double* pot) {
  tree_t* T = h;
  if (T->n == 0) return;
  if (ngsel < 0) or_tree_walk(T);
  ensure_lists(T);
  int64_t ng = ngsel < 0 ? T->ngroups : ngsel;
  double G = T->p.G;
  int64_t n = T->n;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t gi = 0; gi < ng; ++gi) {
    int64_t g = ngsel < 0 ? gi : gsel[gi];
    walk_group(T, g);
    const cell_t* A = &T->cells[T->groups[g]];
    double Lg[4096];
    const int use_local = T->m2l[g].n > 0;
    if (use_local) group_local(T, g, Lg);
    for (int64_t s = A->first; s < A->first + A->count; ++s) {
      double phi, gr[3];
      target_eval(T, g, s, use_local ? Lg : NULL, &phi, gr);
      int64_t i = T->perm[s];
      for (int a = 0; a < 3; ++a) acc[a * n + i] = G * gr[a];
      if (pot) pot[i] = -G * phi;
    }
  }
}

/* 27-image softened direct sum plus the far-field expansion, for a set of
 * targets given by original index: the tree result at theta = 0. */
void or_direct_near_far(void* h, int64_t nt, const int64_t* tgt, double* acc, double* pot) {
  tree_t* T = h;
  double L = T->p.box, eps = T->p.eps, G = T->p.G;
  int kern = T->p.kernel;
  int64_t n = T->n;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nt; ++t) {
    int64_t i = tgt[t];
    double tx = T->x[0][i], ty = T->x[1][i], tz = T->x[2][i];
    double phi = 0.0, gr[3] = {0, 0, 0};
    for (int img = 0; img < 27; ++img) {
      if (!T->p.periodic && img != 13) continue;
      double sh[3] = {(img / 9 - 1) * L, ((img / 3) % 3 - 1) * L, (img % 3 - 1) * L};
      for (int64_t j = 0; j < n; ++j) {
        if (img == 13 && j == i) continue;
        pair_add(tx, ty, tz, T->x[0][j] + sh[0], T->x[1][j] + sh[1], T->x[2][j] + sh[2],
                 T->mass[j], kern, eps, &phi, gr);
      }
    }
    if (T->far_ok) {
      double pf, gf[3], x[3] = {tx, ty, tz};
      far_eval(T, x, T->key[i], &pf, gf);
      phi += pf;
      for (int a = 0; a < 3; ++a) gr[a] += gf[a];
    }
    for (int a = 0; a < 3; ++a) acc[a * nt + t] = G * gr[a];
    if (pot) pot[t] = -G * phi;
  }
}

/* ---------------- accessors ---------------- */

int64_t or_tree_ncells(void* h) { return ((tree_t*)h)->ncells; }
int64_t or_tree_ngroups(void* h) { return ((tree_t*)h)->ngroups; }

void or_tree_perm(void* h, int64_t* perm, uint64_t* skeys) {
  tree_t* T = h;
  for (int64_t s = 0; s < T->n; ++s) {
    if (perm) perm[s] = T->perm[s];
    if (skeys) skeys[s] = T->skey[s];
  }
}

void or_tree_cells(void* h, uint64_t* key, int32_t* level, int64_t* first, int64_t* count,
                   int32_t* is_leaf, double* mass, double* com, double* rcrit) {
  tree_t* T = h;
  int64_t nc = T->ncells;
  for (int64_t c = 0; c < nc; ++c) {
    const cell_t* C = &T->cells[c];
    if (key) key[c] = C->key;
    if (level) level[c] = C->level;
    if (first) first[c] = C->first;
    if (count) count[c] = C->count;
    if (is_leaf) is_leaf[c] = C->is_leaf;
    if (mass) mass[c] = C->m;
    if (com)
      for (int a = 0; a < 3; ++a) com[a * nc + c] = C->com[a];
    if (rcrit) rcrit[c] = C->rcrit;
  }
}

/* second moment about the centre of mass and extent bound of every cell */
void or_tree_cell_bounds(void* h, double* b2, double* bmax) {
  tree_t* T = h;
  for (int64_t c = 0; c < T->ncells; ++c) {
    b2[c] = T->cells[c].b2;
    bmax[c] = T->cells[c].bmax;
  }
}

/* the opening radius of the error-bound test for given B_2, b, order, tol */
void or_tree_cell_bk(void* h, int k, double* out) {
  tree_t* T = h;
  for (int64_t c = 0; c < T->ncells; ++c) out[c] = T->cells[c].bk[k];
}

double or_err_radius(double G, double bp, double b, int p, double tol) {
  return err_radius(G, bp, b, p, tol);
}

/* raw moments of cell c about its centre of mass (or_nterms(order) values) */
void or_tree_cell_moments(void* h, int64_t c, double* M) {
  tree_t* T = h;
  memcpy(M, T->cells[c].M, sizeof(double) * (size_t)T->nmom);
}

void or_tree_groups(void* h, int64_t* cell, double* lo, double* hi) {
  tree_t* T = h;
  int64_t ng = T->ngroups;
  for (int64_t g = 0; g < ng; ++g) {
    if (cell) cell[g] = T->groups[g];
    for (int a = 0; a < 3; ++a) {
      if (lo) lo[a * ng + g] = T->glo[g][a];
      if (hi) hi[a * ng + g] = T->ghi[g][a];
    }
  }
}

/* total list lengths (kind 0: direct, 1: multipole, 2: local expansion) */
int64_t or_tree_list_total(void* h, int kind) {
  tree_t* T = h;
  or_tree_walk(T);
  int64_t t = 0;
  for (int64_t g = 0; g < T->ngroups; ++g)
    t += (kind == 2 ? T->m2l[g].n : kind ? T->m2p[g].n : T->p2p[g].n);
  return t;
}

/* offsets (ngroups+1), image indices and cell indices of all lists of a kind,
 * groups in order, entries in walk order (image, then pre-order) */
void or_tree_lists(void* h, int kind, int64_t* off, int32_t* img, int64_t* cell) {
  tree_t* T = h;
  or_tree_walk(T);
  int64_t t = 0;
  for (int64_t g = 0; g < T->ngroups; ++g) {
    const list_t* l = kind == 2 ? &T->m2l[g] : kind ? &T->m2p[g] : &T->p2p[g];
    off[g] = t;
    for (int64_t e = 0; e < l->n; ++e) {
      img[t] = l->img[e];
      cell[t] = l->cell[e];
      ++t;
    }
  }
  off[T->ngroups] = t;
}

/* direct-interaction pair count (own blocks included) */
int64_t or_tree_pair_count(void* h) {
  tree_t* T = h;
  or_tree_walk(T);
  int64_t t = 0;
  for (int64_t g = 0; g < T->ngroups; ++g) {
    const cell_t* A = &T->cells[T->groups[g]];
    int64_t src = A->count - 1;
    for (int64_t e = 0; e < T->p2p[g].n; ++e) src += T->cells[T->p2p[g].cell[e]].count;
    t += A->count * src;
    (void)src;
  }
  return t;
}

void or_tree_far(void* h, double* Tpsi, double* Mroot, double* Lam) {
  tree_t* T = h;
  int pf = T->p.far_order;
  if (!T->far_ok) return;
  if (Tpsi) memcpy(Tpsi, T->Tpsi, sizeof(double) * 27 * (size_t)or_nterms(2 * pf));
  if (Mroot) memcpy(Mroot, T->Mroot, sizeof(double) * 8 * (size_t)or_nterms(pf));
  if (Lam) memcpy(Lam, T->Lam, sizeof(double) * 8 * (size_t)or_nterms(pf));
}

/* Multipole interaction of one cell built from the given particles (about
 * their centre of mass) at point x: value of Phi and grad Phi, order p. */
void or_multipole_eval(int64_t n, const double* pos, const double* mass, int order, double eps,
                       const double x[3], double* phi, double g[3]) {
  or_mi_init();
  double m = 0, mx[3] = {0, 0, 0};
  for (int64_t j = 0; j < n; ++j) {
    m += mass[j];
    for (int a = 0; a < 3; ++a) mx[a] += mass[j] * pos[a * n + j];
  }
  double com[3] = {mx[0] / m, mx[1] / m, mx[2] / m};
  int nm = or_nterms(order);
  double M[4096];
  memset(M, 0, sizeof(double) * (size_t)nm);
  for (int64_t j = 0; j < n; ++j) {
    for (int k = 0; k < nm; ++k) {
      int ka, kb, kc;
      or_mi_get(k, &ka, &kb, &kc);
      M[k] += mass[j] * pow(pos[j] - com[0], ka) * pow(pos[n + j] - com[1], kb) *
              pow(pos[2 * n + j] - com[2], kc);
    }
  }
  double R[3] = {x[0] - com[0], x[1] - com[1], x[2] - com[2]};
  double Tk[4096];
  or_green_taylor(order + 1, R, eps * eps, Tk);
  double P = 0, G3[3] = {0, 0, 0};
  for (int k = 0; k < nm; ++k) {
    int ka, kb, kc;
    or_mi_get(k, &ka, &kb, &kc);
    double Mk = (((ka + kb + kc) % 2) ? -1.0 : 1.0) * M[k];
    P += Mk * Tk[k];
    G3[0] += Mk * (ka + 1) * Tk[or_mi(ka + 1, kb, kc)];
    G3[1] += Mk * (kb + 1) * Tk[or_mi(ka, kb + 1, kc)];
    G3[2] += Mk * (kc + 1) * Tk[or_mi(ka, kb, kc + 1)];
  }
  *phi = P;
  for (int a = 0; a < 3; ++a) g[a] = G3[a];
}

/* The order-p expansion of one cell built from the given particles (about
 * their centre of mass), re-expanded to order q about c and evaluated at x:
 * Phi and grad Phi of the local expansion (the group-level route of the
 * tree, for pinning it against the multipole and direct sums). */
void or_local_eval(int64_t n, const double* pos, const double* mass, int order, int q,
                   double eps, const double c[3], const double x[3], double* phi, double g[3]) {
  or_mi_init();
  double m = 0, mx[3] = {0, 0, 0};
  for (int64_t j = 0; j < n; ++j) {
    m += mass[j];
    for (int a = 0; a < 3; ++a) mx[a] += mass[j] * pos[a * n + j];
  }
  double com[3] = {mx[0] / m, mx[1] / m, mx[2] / m};
  int nm = or_nterms(order);
  double M[4096];
  memset(M, 0, sizeof(double) * (size_t)nm);
  for (int64_t j = 0; j < n; ++j) {
    for (int k = 0; k < nm; ++k) {
      int ka, kb, kc;
      or_mi_get(k, &ka, &kb, &kc);
      M[k] += mass[j] * pow(pos[j] - com[0], ka) * pow(pos[n + j] - com[1], kb) *
              pow(pos[2 * n + j] - com[2], kc);
    }
  }
  double R0[3] = {c[0] - com[0], c[1] - com[1], c[2] - com[2]};
  double Lg[4096];
  memset(Lg, 0, sizeof(double) * (size_t)or_nterms(q));
  local_add(order, q, eps * eps, M, R0, Lg);
  double y[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  *phi = 0.0;
  g[0] = g[1] = g[2] = 0.0;
  local_poly(q, Lg, y, phi, g);
}

/* plain open-boundary direct sum (no images): the textbook softened sum */
void or_direct_open(int64_t n, const double* pos, const double* mass, double G, double eps,
                    int kernel, double* acc, double* pot) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double phi = 0, gr[3] = {0, 0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      pair_add(pos[i], pos[n + i], pos[2 * n + i], pos[j], pos[n + j], pos[2 * n + j], mass[j],
               kernel, eps, &phi, gr);
    }
    for (int a = 0; a < 3; ++a) acc[a * n + i] = G * gr[a];
    if (pot) pot[i] = -G * phi;
  }
}

/* ======================= adjoint (vector-Jacobian product) ===================
 * An extension beyond the paper.  For the loss L = sum_i gacc_i . a_i +
 * gpot_i phi_i, with a_i = G grad_i Phi_i and phi_i = -G Phi_i, the exact
 * derivatives of the direct sum, written as gathers over each particle's own
 * near pairs (r = x_k - x_j - nL, H = Hessian of g):
 *   xbar_k = G sum_j [ H(r) (m_j gacc_k - m_k gacc_j) - grad g(r) (m_j gpot_k + m_k gpot_j) ]
 *   mbar_k = -G sum_j [ gacc_j . grad g(r) + gpot_j g(r) ]
 * The tree version evaluates these sums with the forward lists: leaves and the
 * own group pair by pair, accepted cells through multipole expansions of the
 * three kinds of source (masses, vector charges gacc_j, scalar charges gpot_j)
 * about the cell's centre of mass, with Taylor coefficients to degree p+2.
 * The periodic far field is differentiated exactly: target side through the
 * local expansions, source side through adjoint local coefficients
 *   Lbar^t_q = G sum_{i in t} (gacc_i . grad h^q - gpot_i h^q)
 * carried back to the octant moments and on to each source particle.  At
 * theta = 0 this is the exact derivative of the 27-image + far-field sum. */

typedef struct {
  double* Qa;  /* per cell: 3 x nmom moments of the vector charges gacc */
  double* Qp;  /* per cell: nmom moments of the scalar charges gpot */
} adj_mom_t;

static void adj_moments(const tree_t* T, const double* sga, const double* sgp, adj_mom_t* A) {
  int p = T->p.order, nm = T->nmom;
  int64_t n = T->n;
  A->Qa = calloc((size_t)T->ncells * 3 * nm, sizeof(double));
  A->Qp = calloc((size_t)T->ncells * nm, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t ci = 0; ci < T->ncells; ++ci) {
    const cell_t* c = &T->cells[ci];
    double* qa = A->Qa + (size_t)ci * 3 * nm;
    double* qp = A->Qp + (size_t)ci * nm;
    for (int64_t s = c->first; s < c->first + c->count; ++s) {
      double d[3] = {T->sx[0][s] - c->com[0], T->sx[1][s] - c->com[1], T->sx[2][s] - c->com[2]};
      double pw[3][OR_DMAX + 1];
      for (int a = 0; a < 3; ++a) {
        pw[a][0] = 1.0;
        for (int e = 1; e <= p; ++e) pw[a][e] = pw[a][e - 1] * d[a];
      }
      for (int k = 0; k < nm; ++k) {
        int ka, kb, kc;
        or_mi_get(k, &ka, &kb, &kc);
        double mono = pw[0][ka] * pw[1][kb] * pw[2][kc];
        for (int a = 0; a < 3; ++a) qa[a * nm + k] += sga[a * n + s] * mono;
        qp[k] += sgp[s] * mono;
      }
    }
  }
}

/* exact pair adjoint: target k (tx, m_k, gacc_k, gpot_k), source j at (sx)
 * with m_j, gacc_j, gpot_j; r = x_k - x_j */
static void pair_adj(const double r[3], double eps2, double mk, const double gak[3], double gpk,
                     double mj, const double gaj[3], double gpj, double xb[3], double* mb) {
  double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
  double si = 1.0 / sqrt(r2);
  double si3 = si * si * si, si5 = si3 * si * si;
  double w[3], rw = 0.0, ra = 0.0;
  for (int a = 0; a < 3; ++a) {
    w[a] = mj * gak[a] - mk * gaj[a];
    rw += r[a] * w[a];
    ra += r[a] * gaj[a];
  }
  double cp = mj * gpk + mk * gpj;
  for (int a = 0; a < 3; ++a) {
    /* H w = -w/s^3 + 3 r (r.w)/s^5 ;  -grad g = r/s^3 */
    xb[a] += -w[a] * si3 + 3.0 * r[a] * rw * si5 + r[a] * si3 * cp;
  }
  /* -(gacc_j . grad g + gpot_j g) = (r . gacc_j)/s^3 - gpot_j/s */
  *mb += ra * si3 - gpj * si;
}

static int mi3(int a, int b, int c) { return or_mi(a, b, c); }

/* multipole adjoint of one accepted cell for one target */
static void m2p_adj(const tree_t* T, int64_t bi, const adj_mom_t* AM, const double R[3],
                    double mk, const double gak[3], double gpk, double xb[3], double* mb) {
  int p = T->p.order, nm = T->nmom;
  double Tk[4096];
  or_green_taylor(p + 2, R, T->p.eps * T->p.eps, Tk);
  const double* M = T->cells[bi].M;
  const double* Qa = AM->Qa + (size_t)bi * 3 * nm;
  const double* Qp = AM->Qp + (size_t)bi * nm;
  double Hm[3][3] = {{0}}, Gm[3] = {0}, Gp[3] = {0}, psiV = 0.0, Pp = 0.0, GV[3] = {0};
  for (int k = 0; k < nm; ++k) {
    int kk[3];
    or_mi_get(k, &kk[0], &kk[1], &kk[2]);
    double sg = ((kk[0] + kk[1] + kk[2]) % 2) ? -1.0 : 1.0;
    for (int a = 0; a < 3; ++a) {
      int e1[3] = {kk[0], kk[1], kk[2]};
      e1[a] += 1;
      double d1 = (double)e1[a] * Tk[mi3(e1[0], e1[1], e1[2])]; /* d_a T_k */
      Gm[a] += sg * M[k] * d1;
      Gp[a] += sg * Qp[k] * d1;
      psiV += sg * Qa[a * nm + k] * d1;
      for (int b = 0; b < 3; ++b) {
        int e2[3] = {e1[0], e1[1], e1[2]};
        e2[b] += 1;
        /* d_b d_a T_k = (k_a+1) (k+e_a)_b+1 ... T_{k+e_a+e_b} */
        double d2 = (double)e1[a] * (double)e2[b] * Tk[mi3(e2[0], e2[1], e2[2])];
        Hm[a][b] += sg * M[k] * d2;
        GV[b] += sg * Qa[a * nm + k] * d2;
      }
    }
    Pp += sg * Qp[k] * Tk[k];
  }
  for (int a = 0; a < 3; ++a) {
    double hv = Hm[a][0] * gak[0] + Hm[a][1] * gak[1] + Hm[a][2] * gak[2];
    xb[a] += hv - mk * GV[a] - gpk * Gm[a] - mk * Gp[a];
  }
  *mb += -(psiV + Pp);
}

/* far-field Hessian at x (target side): sum_q Lam_q d_a d_b h^q */
static void far_hess(const tree_t* T, const double x[3], uint64_t key, double Hf[3][3]) {
  int pf = T->p.far_order, nq = or_nterms(pf);
  int t = octant_of(key);
  double c[3];
  octant_center(T, t, c);
  double h[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  double pw[3][OR_DMAX + 1];
  for (int a = 0; a < 3; ++a) {
    pw[a][0] = 1.0;
    for (int e = 1; e <= pf; ++e) pw[a][e] = pw[a][e - 1] * h[a];
  }
  const double* Lm = T->Lam + (size_t)t * nq;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Hf[a][b] = 0.0;
  for (int q = 0; q < nq; ++q) {
    int e[3];
    or_mi_get(q, &e[0], &e[1], &e[2]);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        int f[3] = {e[0], e[1], e[2]};
        double coef = 1.0;
        coef *= f[a];
        if (f[a] == 0) continue;
        f[a] -= 1;
        coef *= f[b];
        if (f[b] == 0) continue;
        f[b] -= 1;
        Hf[a][b] += Lm[q] * coef * pw[0][f[0]] * pw[1][f[1]] * pw[2][f[2]];
      }
  }
}

/* Adjoint of or_tree_forces: gacc (3 x n SoA) and gpot (n or NULL) in
 * original order; writes xbar (3 x n) and mbar (n) in original order for every
 * particle (ngsel < 0) or for the particles of the listed groups. */
void or_tree_vjp(void* h, const double* gacc, const double* gpot, int64_t ngsel,
                 const int64_t* gsel, double* xbar, double* mbar) {
  tree_t* T = h;
  int64_t n = T->n;
  if (n == 0) return;
  double G = T->p.G, L = T->p.box, eps2 = T->p.eps * T->p.eps;
  /* cotangents in sorted order */
  double* sga = malloc(sizeof(double) * 3 * (size_t)n);
  double* sgp = calloc((size_t)n, sizeof(double));
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = T->perm[s];
    for (int a = 0; a < 3; ++a) sga[a * n + s] = gacc[a * n + i];
    if (gpot) sgp[s] = gpot[i];
  }
  adj_mom_t AM;
  adj_moments(T, sga, sgp, &AM);
  if (ngsel < 0) or_tree_walk(T);
  ensure_lists(T);
  int64_t ng = ngsel < 0 ? T->ngroups : ngsel;

  /* far field, source side: adjoint local coefficients over all targets */
  int pf = T->p.far_order, nq = or_nterms(pf), nT = or_nterms(2 * pf);
  double* Mbar = NULL;
  if (T->far_ok) {
    double* Lbar = calloc((size_t)8 * nq, sizeof(double));
    for (int64_t s = 0; s < n; ++s) {
      int t = octant_of(T->skey[s]);
      double c[3];
      octant_center(T, t, c);
      double hh[3] = {T->sx[0][s] - c[0], T->sx[1][s] - c[1], T->sx[2][s] - c[2]};
      double pw[3][OR_DMAX + 1];
      for (int a = 0; a < 3; ++a) {
        pw[a][0] = 1.0;
        for (int e = 1; e <= pf; ++e) pw[a][e] = pw[a][e - 1] * hh[a];
      }
      for (int q = 0; q < nq; ++q) {
        int e[3];
        or_mi_get(q, &e[0], &e[1], &e[2]);
        double v = -sgp[s] * pw[0][e[0]] * pw[1][e[1]] * pw[2][e[2]];
        if (e[0]) v += sga[s] * e[0] * pw[0][e[0] - 1] * pw[1][e[1]] * pw[2][e[2]];
        if (e[1]) v += sga[n + s] * e[1] * pw[0][e[0]] * pw[1][e[1] - 1] * pw[2][e[2]];
        if (e[2]) v += sga[2 * n + s] * e[2] * pw[0][e[0]] * pw[1][e[1]] * pw[2][e[2] - 1];
        Lbar[(size_t)t * nq + q] += G * v;
      }
    }
    Mbar = calloc((size_t)8 * nq, sizeof(double));
    for (int so = 0; so < 8; ++so)
      for (int k = 0; k < nq; ++k) {
        int ka, kb, kc;
        or_mi_get(k, &ka, &kb, &kc);
        double sg = ((ka + kb + kc) % 2) ? -1.0 : 1.0;
        double acc = 0.0;
        for (int t = 0; t < 8; ++t) {
          int dx = ((t >> 2) & 1) - ((so >> 2) & 1), dy = ((t >> 1) & 1) - ((so >> 1) & 1),
              dz = (t & 1) - (so & 1);
          const double* Tp = T->Tpsi + (size_t)((dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)) * nT;
          for (int q = 0; q < nq; ++q) {
            int qa, qb, qc;
            or_mi_get(q, &qa, &qb, &qc);
            acc += Lbar[(size_t)t * nq + q] * binom_mi(qa, qb, qc, ka, kb, kc) * sg *
                   Tp[or_mi(qa + ka, qb + kb, qc + kc)];
          }
        }
        Mbar[(size_t)so * nq + k] = acc;
      }
    free(Lbar);
  }

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t gi = 0; gi < ng; ++gi) {
    int64_t g = ngsel < 0 ? gi : gsel[gi];
    walk_group(T, g);
    const cell_t* A = &T->cells[T->groups[g]];
    for (int64_t s = A->first; s < A->first + A->count; ++s) {
      double xk[3] = {T->sx[0][s], T->sx[1][s], T->sx[2][s]};
      double mk = T->sm[s], gak[3] = {sga[s], sga[n + s], sga[2 * n + s]}, gpk = sgp[s];
      double xb[3] = {0, 0, 0}, mb = 0.0;
      for (int64_t j = A->first; j < A->first + A->count; ++j) {
        if (j == s) continue;
        double r[3] = {xk[0] - T->sx[0][j], xk[1] - T->sx[1][j], xk[2] - T->sx[2][j]};
        double gaj[3] = {sga[j], sga[n + j], sga[2 * n + j]};
        pair_adj(r, eps2, mk, gak, gpk, T->sm[j], gaj, sgp[j], xb, &mb);
      }
      const list_t* lp = &T->p2p[g];
      for (int64_t e = 0; e < lp->n; ++e) {
        int img = lp->img[e];
        double sh[3] = {(img / 9 - 1) * L, ((img / 3) % 3 - 1) * L, (img % 3 - 1) * L};
        const cell_t* B = &T->cells[lp->cell[e]];
        for (int64_t j = B->first; j < B->first + B->count; ++j) {
          double r[3] = {xk[0] - (T->sx[0][j] + sh[0]), xk[1] - (T->sx[1][j] + sh[1]),
                         xk[2] - (T->sx[2][j] + sh[2])};
          double gaj[3] = {sga[j], sga[n + j], sga[2 * n + j]};
          pair_adj(r, eps2, mk, gak, gpk, T->sm[j], gaj, sgp[j], xb, &mb);
        }
      }
      const list_t* lm = &T->m2p[g];
      for (int64_t e = 0; e < lm->n; ++e) {
        int img = lm->img[e];
        double sh[3] = {(img / 9 - 1) * L, ((img / 3) % 3 - 1) * L, (img % 3 - 1) * L};
        const cell_t* B = &T->cells[lm->cell[e]];
        double R[3] = {xk[0] - (B->com[0] + sh[0]), xk[1] - (B->com[1] + sh[1]),
                       xk[2] - (B->com[2] + sh[2])};
        m2p_adj(T, lm->cell[e], &AM, R, mk, gak, gpk, xb, &mb);
      }
      for (int a = 0; a < 3; ++a) xb[a] *= G;
      mb *= G;
      if (T->far_ok) {
        /* target side: G Hf gacc_k - G gpot_k grad Phi_far */
        double Hf[3][3], pf_, gf[3];
        far_hess(T, xk, T->skey[s], Hf);
        far_eval(T, xk, T->skey[s], &pf_, gf);
        for (int a = 0; a < 3; ++a)
          xb[a] += G * (Hf[a][0] * gak[0] + Hf[a][1] * gak[1] + Hf[a][2] * gak[2]) -
                   G * gpk * gf[a];
        /* source side: m_k sum_k Mbar_k grad s^k, sum_k Mbar_k s^k */
        int so = octant_of(T->skey[s]);
        double c[3];
        octant_center(T, so, c);
        double hh[3] = {xk[0] - c[0], xk[1] - c[1], xk[2] - c[2]};
        double pw[3][OR_DMAX + 1];
        for (int a = 0; a < 3; ++a) {
          pw[a][0] = 1.0;
          for (int e = 1; e <= pf; ++e) pw[a][e] = pw[a][e - 1] * hh[a];
        }
        const double* Mb = Mbar + (size_t)so * nq;
        for (int k = 0; k < nq; ++k) {
          int e[3];
          or_mi_get(k, &e[0], &e[1], &e[2]);
          mb += Mb[k] * pw[0][e[0]] * pw[1][e[1]] * pw[2][e[2]];
          if (e[0]) xb[0] += mk * Mb[k] * e[0] * pw[0][e[0] - 1] * pw[1][e[1]] * pw[2][e[2]];
          if (e[1]) xb[1] += mk * Mb[k] * e[1] * pw[0][e[0]] * pw[1][e[1] - 1] * pw[2][e[2]];
          if (e[2]) xb[2] += mk * Mb[k] * e[2] * pw[0][e[0]] * pw[1][e[1]] * pw[2][e[2] - 1];
        }
      }
      int64_t i = T->perm[s];
      for (int a = 0; a < 3; ++a) xbar[a * n + i] = xb[a];
      mbar[i] = mb;
    }
  }
  free(sga); free(sgp); free(AM.Qa); free(AM.Qp); free(Mbar);
}

// Oct-tree over the key-sorted particles (paper Sec. 2.1: the Morton keys
// implicitly define the tree topology; cells are the internal nodes and carry
// truncated multipole expansions; groups of nearby sinks share one list).
//
// Build: level by level from the root.  A cell with more than leaf_max
// particles below level 21 is split into its non-empty daughters, found by
// binary search for the octal digit boundaries inside its contiguous sorted
// range.  Cells are stored level-major; the daughters of a cell are
// contiguous and in octant order, so the octant-ordered sums below need no
// sorting.  A hash table from key to cell (the paper's hashed oct-tree) is
// filled once the cells are known.
//
// Moments, bottom-up: cell mass and sum m x in FP64 with separate multiply
// and add (leaves sum their particles in key order, internal cells their
// daughters in octant order), centre of mass = sum m x / m, the opening
// radius s/theta + |com - centre|, and raw Cartesian moments about the centre
// of mass (leaves directly, internal cells by shifting the daughters'
// moments).  From the raw moments each cell derives the coefficient block its
// multipole interactions use.
#include <algorithm>

#include "device_math.h"

namespace hot {

__device__ __forceinline__ void cell_center(uint64_t key, int level, double L, double c[3],
                                            double* side) {
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
  *side = s;
}

__global__ void k_root(Cells C, uint32_t n) {
  C.key[0] = 1ull;
  C.level[0] = 0;
  C.first[0] = 0;
  C.count[0] = n;
  C.child[0] = -1;
  C.nchild[0] = 0;
  C.parent[0] = -1;
}

// first sorted index in [lo, hi) whose octal digit (at `shift`) is >= o
__device__ __forceinline__ uint32_t digit_lower_bound(const uint64_t* __restrict__ skey,
                                                      uint32_t lo, uint32_t hi, int shift,
                                                      uint32_t o) {
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    uint32_t d = (uint32_t)((skey[mid] >> shift) & 7ull);
    if (d < o)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Eight lanes per cell, lane o finding where octant o starts in the cell's
// sorted range (the eight searches run side by side instead of one after the
// other, which shortens the dependent-load chain of the few large cells at
// the top levels); octant o ends where octant o + 1 starts, read from the
// next lane.  The eight lanes of a cell are consecutive lanes of one wave.
struct OctantSplit {
  uint32_t c, lo, e;
  bool split, nonempty;
  uint32_t mask;  // non-empty octants of the cell (bit o)
};

__device__ __forceinline__ OctantSplit octant_split(const Cells& C,
                                                    const uint64_t* __restrict__ skey,
                                                    uint64_t ci, uint32_t o, uint32_t beg,
                                                    uint32_t cnt, int level, int leaf_max) {
  OctantSplit r{0, 0, 0, false, false, 0};
  if (ci < cnt) {
    r.c = beg + (uint32_t)ci;
    const uint32_t first = C.first[r.c], count = C.count[r.c];
    r.split = (int)count > leaf_max && level < kMaxLevel;
    if (r.split) {
      const int shift = 3 * (kMaxLevel - level - 1);
      r.e = first + count;
      r.lo = o == 0 ? first : digit_lower_bound(skey, first, r.e, shift, o);
    }
  }
  // every lane takes part in the exchange and the vote
  const uint32_t next = __shfl_down(r.lo, 1, 8);
  if (o < 7) r.e = next;
  r.nonempty = r.split && r.e > r.lo;
  const unsigned long long votes = __ballot(r.nonempty);
  r.mask = (uint32_t)((votes >> (__lane_id() & ~7u)) & 0xffull);
  return r;
}

__global__ void __launch_bounds__(256) k_split_count(Cells C, const uint64_t* __restrict__ skey,
                                                     uint32_t beg, uint32_t cnt, int level,
                                                     int leaf_max, uint32_t* __restrict__ nch) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t ci = t >> 3;
  const uint32_t o = (uint32_t)(t & 7);
  const OctantSplit r = octant_split(C, skey, ci, o, beg, cnt, level, leaf_max);
  if (ci < cnt && o == 0) nch[ci] = (uint32_t)__popc(r.mask);
}

__global__ void __launch_bounds__(256) k_split_emit(Cells C, const uint64_t* __restrict__ skey,
                                                    uint32_t beg, uint32_t cnt, int level,
                                                    int leaf_max,
                                                    const uint32_t* __restrict__ choff,
                                                    uint32_t next, uint32_t cap) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t ci = t >> 3;
  const uint32_t o = (uint32_t)(t & 7);
  const OctantSplit r = octant_split(C, skey, ci, o, beg, cnt, level, leaf_max);
  if (ci >= cnt) return;
  const uint32_t c = r.c;
  if (!r.split) {
    if (o == 0) {
      C.child[c] = -1;
      C.nchild[c] = 0;
    }
    return;
  }
  const uint32_t out = next + choff[ci];
  if (r.nonempty) {
    const uint32_t d = out + (uint32_t)__popc(r.mask & ((1u << o) - 1u));
    if (d < cap) {  // over capacity: the host sees the total and fails the call
      C.key[d] = (C.key[c] << 3) | o;
      C.level[d] = level + 1;
      C.first[d] = r.lo;
      C.count[d] = r.e - r.lo;
      C.child[d] = -1;
      C.nchild[d] = 0;
      C.parent[d] = (int32_t)c;
    }
  }
  if (o == 0) {
    C.child[c] = (int32_t)out;
    C.nchild[c] = (int32_t)__popc(r.mask);
  }
}

// ----------------------------------------------------------- key -> cell hash
// The hashed oct-tree (paper Sec. 2.1): a table from a cell's key to its
// index, open addressing with linear probing over a power-of-two number of
// slots (at least twice the cells).  An empty slot holds key 0, which no cell
// has (every key carries the placeholder bit).  Insertion is one thread per
// cell with a compare-and-swap on the slot's key; slots are therefore filled
// in no fixed order, but every key maps to its one cell.
__device__ __forceinline__ uint64_t key_hash(uint64_t k) {
  // a 64-bit finaliser (xor-shift and odd-constant multiply rounds)
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__global__ void __launch_bounds__(256) k_hash_clear(uint64_t* __restrict__ hkey, size_t hcap) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < hcap;
       i += (size_t)gridDim.x * 256)
    hkey[i] = 0ull;
}

__global__ void __launch_bounds__(256) k_hash_insert(Cells C, uint32_t ncells,
                                                     unsigned long long* hkey,
                                                     uint32_t* __restrict__ hval, uint64_t mask) {
  const uint32_t c = blockIdx.x * 256 + threadIdx.x;
  if (c >= ncells) return;
  const unsigned long long k = C.key[c];
  uint64_t h = key_hash(k) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev = atomicCAS(hkey + h, 0ull, k);
    if (prev == 0ull || prev == k) {
      hval[h] = c;
      return;
    }
    h = (h + 1) & mask;
  }
}

__global__ void __launch_bounds__(256) k_hash_lookup(const uint64_t* __restrict__ hkey,
                                                     const uint32_t* __restrict__ hval,
                                                     uint64_t mask,
                                                     const uint64_t* __restrict__ q, size_t nq,
                                                     int32_t* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nq) return;
  const uint64_t k = q[i];
  int32_t r = -1;
  if (k != 0ull) {
    uint64_t h = key_hash(k) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
      const uint64_t s = hkey[h];
      if (s == k) {
        r = (int32_t)hval[h];
        break;
      }
      if (s == 0ull) break;
      h = (h + 1) & mask;
    }
  }
  out[i] = r;
}

// ------------------------------------------------------------------ moments
// Error-bound opening radius (Salmon & Warren 1994): the acceleration error
// of an order-p expansion of a cell with extent b about its centre of mass is
// at most G B_(p+1) ((p+2) r - (p+1) b) / (r^(p+2) (r - b)^2) at distance
// r > b, with B_(p+1) = sum m |x - com|^(p+1) (order 0 counts as order 1:
// the dipole about the centre of mass vanishes): summed over the particles
// at leaves, bounded above them (see k_moments).  The radius where
// the bound meets the tolerance is found by doubling, then 64 bisection
// steps, in separate IEEE operations only (contraction is off), so that every
// implementation of the same definition finds the same double.
__device__ double sw_bound(double gb, double b, int pe, double r) {
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

// bp = B_(pe+1), pe = max(p, 1)
__device__ double err_radius(double G, double bp, double b, int p, double tol) {
  const int pe = p < 1 ? 1 : p;
  const double gb = G * bp;
  if (!(gb > 0.0)) return b;
  double lo = b, hi = b + b;
  for (int i = 0; i < 4096 && sw_bound(gb, b, pe, hi) > tol; ++i) hi = hi + hi;
  for (int i = 0; i < 64; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (sw_bound(gb, b, pe, mid) <= tol)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

template <int P, typename T>
__global__ void __launch_bounds__(128) k_moments(Cells C, const double* __restrict__ spos,
                                                 const double* __restrict__ smass, size_t n,
                                                 uint32_t beg, uint32_t cnt, double L,
                                                 double theta, double G, double err_tol,
                                                 double k1h) {
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const uint32_t c = beg + t;
  constexpr int NM = nt(P);
  constexpr MI<P> mi{};
  double ctr[3], side;
  cell_center(C.key[c], C.level[c], L, ctr, &side);
  const int nc = C.nchild[c];
  const int c0 = C.child[c];
  const uint32_t f = C.first[c], e = f + C.count[c];
  double m = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
  if (nc == 0) {
    for (uint32_t s = f; s < e; ++s) {
      double ms = smass[s];
      m = m + ms;
      sx = sx + ms * spos[s];
      sy = sy + ms * spos[n + s];
      sz = sz + ms * spos[2 * n + s];
    }
  } else {
    for (int k = 0; k < nc; ++k) {
      double4 q = C.mmx[c0 + k];
      m = m + q.x;
      sx = sx + q.y;
      sy = sy + q.z;
      sz = sz + q.w;
    }
  }
  double com[3];
  if (m != 0.0) {
    com[0] = sx / m;
    com[1] = sy / m;
    com[2] = sz / m;
  } else {
    com[0] = ctr[0];
    com[1] = ctr[1];
    com[2] = ctr[2];
  }
  double dx = com[0] - ctr[0], dy = com[1] - ctr[1], dz = com[2] - ctr[2];
  double dd = dx * dx;
  dd = dd + dy * dy;
  dd = dd + dz * dz;
  // B_k = sum m |x - com|^k and the extent about the centre of mass: summed
  // over the particles at leaves (key order); above them B_2 by the
  // parallel-axis identity, the extent by the triangle inequality, and the
  // other B_k by the triangle inequality expanded binomially,
  //   B_k <= sum_d sum_j C(k, j) B_j(d) delta_d^(k-j)
  // (daughters in octant order, j ascending)
  double b2 = 0.0, bmax = 0.0;
  double bk[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // raw moments about the centre of mass (at a leaf summed in the same pass
  // over its particles as the B_k)
  double M[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) M[k] = 0.0;
  if (nc == 0) {
    double r2max = 0.0;
    for (uint32_t s = f; s < e; ++s) {
      const double ex = spos[s] - com[0], ey = spos[n + s] - com[1],
                   ez = spos[2 * n + s] - com[2];
      double r2 = ex * ex;
      r2 = r2 + ey * ey;
      r2 = r2 + ez * ez;
      const double ms = smass[s];
      const double t = ms * r2;
      b2 = b2 + t;
      if (r2 > r2max) r2max = r2;
      const double r = sqrt(r2);
      const double r3 = r2 * r, r4 = r2 * r2;
      const double r5 = r4 * r;
      bk[1] = bk[1] + ms * r;
      bk[3] = bk[3] + ms * r3;
      bk[4] = bk[4] + ms * r4;
      bk[5] = bk[5] + ms * r5;
      const double d[3] = {ex, ey, ez};
      double pw[3][P + 1];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pw[a][0] = 1.0;
#pragma unroll
        for (int q = 1; q <= P; ++q) pw[a][q] = pw[a][q - 1] * d[a];
      }
#pragma unroll
      for (int k = 0; k < NM; ++k) M[k] += ms * pw[0][mi.a[k]] * pw[1][mi.b[k]] * pw[2][mi.c[k]];
    }
    bmax = sqrt(r2max);
  } else {
    constexpr double binom[6][6] = {{1, 0, 0, 0, 0, 0}, {1, 1, 0, 0, 0, 0}, {1, 2, 1, 0, 0, 0},
                                    {1, 3, 3, 1, 0, 0}, {1, 4, 6, 4, 1, 0}, {1, 5, 10, 10, 5, 1}};
    for (int k = 0; k < nc; ++k) {
      const double4 wc = C.walk[c0 + k];
      const double2 bc = C.bnd[c0 + k];
      const double4 bq = C.bk[c0 + k];
      const double md = C.mmx[c0 + k].x;
      const double ex = wc.x - com[0], ey = wc.y - com[1], ez = wc.z - com[2];
      double r2 = ex * ex;
      r2 = r2 + ey * ey;
      r2 = r2 + ez * ez;
      double t = md * r2;
      t = bc.x + t;
      b2 = b2 + t;
      const double dl = sqrt(r2);
      const double eb = bc.y + dl;
      if (eb > bmax) bmax = eb;
      const double bd[6] = {md, bq.x, bc.x, bq.y, bq.z, bq.w};
      double dp[6];
      dp[0] = 1.0;
#pragma unroll
      for (int q = 1; q < 6; ++q) dp[q] = dp[q - 1] * dl;
#pragma unroll
      for (int q = 1; q < 6; ++q) {
        if (q == 2) continue;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j <= q; ++j) {
          double u = binom[q][j] * bd[j];
          u = u * dp[q - j];
          acc = acc + u;
        }
        bk[q] = bk[q] + acc;
      }
    }
  }
  C.bnd[c] = make_double2(b2, bmax);
  C.bk[c] = make_double4(bk[1], bk[3], bk[4], bk[5]);
  double rcrit = (theta > 0.0) ? side / theta + sqrt(dd) : 0.0;
  if (err_tol > 0.0) {
    constexpr int pe = P < 1 ? 1 : P;
    const double bp = pe + 1 == 2 ? b2 : pe + 1 == 3 ? bk[3] : pe + 1 == 4 ? bk[4] : bk[5];
    const double re = err_radius(G, bp, bmax, P, err_tol);
    if (re > rcrit) rcrit = re;
  } else if (!(theta > 0.0)) {
    rcrit = __builtin_inf();
  }
  // K1 softening: all of the cell's particles beyond the kernel radius
  if (k1h >= 0.0) {
    const double rk = bmax + k1h;
    if (rk > rcrit) rcrit = rk;
  }
  C.mmx[c] = make_double4(m, sx, sy, sz);
  C.walk[c] = make_double4(com[0], com[1], com[2], rcrit);

  // raw moments above the leaves: the daughters' shifted to this centre
  if (nc != 0) {
    for (int kc = 0; kc < nc; ++kc) {
      const int ch = c0 + kc;
      const double4 w = C.walk[ch];
      const double d[3] = {w.x - com[0], w.y - com[1], w.z - com[2]};
      const double* Mc = C.mom + (size_t)ch * NM;
      double Mch[NM];
#pragma unroll
      for (int k = 0; k < NM; ++k) Mch[k] = Mc[k];
      shift_add<P>(Mch, d, M);
    }
  }
  double* Mo = C.mom + (size_t)c * NM;
#pragma unroll
  for (int k = 0; k < NM; ++k) Mo[k] = M[k];
  coef_store<P, false, T>(M, (T*)C.coef + (size_t)c * coef_stride(P));
}

// ------------------------------------------------------------------- groups
__global__ void __launch_bounds__(256) k_group_flags(Cells C, uint32_t ncells, int gmax,
                                                     uint32_t* __restrict__ gflag,
                                                     int32_t* __restrict__ gcell_at) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const bool elig = ((int)C.count[c] <= gmax) || (C.nchild[c] == 0);
  bool isg = elig;
  if (c != 0) {
    const int p = C.parent[c];
    isg = elig && !((int)C.count[p] <= gmax);  // a parent is never a leaf
  }
  if (isg) {
    const uint32_t f = C.first[c];
    gflag[f] = 1u;
    gcell_at[f] = (int32_t)c;
  }
}

__global__ void __launch_bounds__(256) k_group_compact(const uint32_t* __restrict__ gflag,
                                                       const uint32_t* __restrict__ gid,
                                                       const int32_t* __restrict__ gcell_at,
                                                       size_t n, int32_t* __restrict__ gcell) {
  size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (gflag[s]) gcell[gid[s]] = gcell_at[s];
}

// one wavefront per sink group (grid-stride over the groups): the lanes read
// the group's particles together, then a butterfly min/max (exact, so the
// box does not depend on the order)
__global__ void __launch_bounds__(256) k_group_bbox(Cells C, Groups G, uint32_t ngroups,
                                                    uint32_t gcap, const double* __restrict__ spos,
                                                    size_t n) {
  const int lane = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * 4;
  for (uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6); g < ngroups; g += waves) {
    const int c = G.cell[g];
    const uint32_t f = C.first[c], cnt = C.count[c];
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    for (uint32_t t = lane; t < cnt; t += 64)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double v = spos[(size_t)a * n + f + t];
        lo[a] = v < lo[a] ? v : lo[a];
        hi[a] = v > hi[a] ? v : hi[a];
      }
#pragma unroll
    for (int w = 1; w < 64; w <<= 1)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double l = __shfl_xor(lo[a], w, 64), h = __shfl_xor(hi[a], w, 64);
        lo[a] = l < lo[a] ? l : lo[a];
        hi[a] = h > hi[a] ? h : hi[a];
      }
    if (lane < 3) {
      G.lo[(size_t)lane * gcap + g] = lane == 0 ? lo[0] : lane == 1 ? lo[1] : lo[2];
      G.hi[(size_t)lane * gcap + g] = lane == 0 ? hi[0] : lane == 1 ? hi[1] : hi[2];
    }
  }
}

// source records: FP32/FP64 offsets from the leaf centre and the mass; one
// sub-group of 2^wshift lanes per cell (the leaf size rounded up to a power
// of two, at most a wavefront; grid-stride over the cells), its lanes over
// the leaf's particles
template <typename T4, typename T>
__global__ void __launch_bounds__(256) k_srec(Cells C, uint32_t ncells,
                                              const double* __restrict__ spos,
                                              const double* __restrict__ smass, size_t n, double L,
                                              int wshift, T4* __restrict__ srec) {
  const int lane = threadIdx.x & 63;
  const uint32_t w = 1u << wshift, per_wave = 64u >> wshift;
  const uint32_t sub = (uint32_t)lane >> wshift, sl = (uint32_t)lane & (w - 1);
  const uint32_t step = gridDim.x * 4 * per_wave;
  for (uint32_t c = (blockIdx.x * 4 + (threadIdx.x >> 6)) * per_wave + sub; c < ncells;
       c += step) {
    if (C.nchild[c] != 0) continue;
    double ctr[3], side;
    cell_center(C.key[c], C.level[c], L, ctr, &side);
    const uint32_t f = C.first[c], cnt = C.count[c];
    for (uint32_t t = sl; t < cnt; t += w) {
      const uint32_t s = f + t;
      T4 r;
      r.x = (T)(spos[s] - ctr[0]);
      r.y = (T)(spos[n + s] - ctr[1]);
      r.z = (T)(spos[2 * n + s] - ctr[2]);
      r.w = (T)smass[s];
      srec[s] = r;
    }
  }
}

// ---------------------------------------------------------------- host side
hipError_t tree_root(const Cells& C, uint32_t n, hipStream_t s) {
  k_root<<<1, 1, 0, s>>>(C, n);
  return hipGetLastError();
}

hipError_t tree_split_level(const Cells& C, const uint64_t* skey, uint32_t beg, uint32_t cnt,
                            int level, int leaf_max, uint32_t* nch, uint32_t* total,
                            uint32_t* scan_tmp, hipStream_t s) {
  const unsigned g = (unsigned)((8 * (size_t)cnt + 255) / 256);  // eight lanes per cell
  k_split_count<<<g, 256, 0, s>>>(C, skey, beg, cnt, level, leaf_max, nch);
  return scan_u32(nch, nch, total, cnt, scan_tmp, s);
}

hipError_t tree_emit_level(const Cells& C, const uint64_t* skey, uint32_t beg, uint32_t cnt,
                           int level, int leaf_max, const uint32_t* choff, uint32_t next,
                           uint32_t cap, hipStream_t s) {
  const unsigned g = (unsigned)((8 * (size_t)cnt + 255) / 256);  // eight lanes per cell
  k_split_emit<<<g, 256, 0, s>>>(C, skey, beg, cnt, level, leaf_max, choff, next, cap);
  return hipGetLastError();
}

hipError_t tree_hash_build(const Cells& C, uint32_t ncells, uint64_t* hkey, uint32_t* hval,
                           size_t hcap, hipStream_t s) {
  const unsigned gc = (unsigned)std::min<size_t>((hcap + 255) / 256, 65536);
  k_hash_clear<<<gc, 256, 0, s>>>(hkey, hcap);
  if (ncells)
    k_hash_insert<<<(ncells + 255) / 256, 256, 0, s>>>(C, ncells, (unsigned long long*)hkey, hval,
                                                       (uint64_t)hcap - 1);
  return hipGetLastError();
}

hipError_t hash_lookup(const uint64_t* hkey, const uint32_t* hval, size_t hcap, const uint64_t* q,
                       size_t nq, int32_t* out, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  k_hash_lookup<<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(hkey, hval, (uint64_t)hcap - 1, q, nq,
                                                             out);
  return hipGetLastError();
}

template <int P, typename T>
static void moments_launch(const Cells& C, const double* spos, const double* smass, size_t n,
                           uint32_t beg, uint32_t cnt, double L, double theta, double G,
                           double err_tol, double k1h, hipStream_t s) {
  k_moments<P, T><<<(cnt + 127) / 128, 128, 0, s>>>(C, spos, smass, n, beg, cnt, L, theta, G,
                                                     err_tol, k1h);
}

hipError_t tree_moments_level(const Cells& C, const double* spos, const double* smass, size_t n,
                              uint32_t beg, uint32_t cnt, double L, double theta, double G,
                              double err_tol, double k1h, int order, bool fp32, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
#define HOT_MOM(P)                                                                          \
  case P:                                                                                   \
    if (fp32)                                                                               \
      moments_launch<P, float>(C, spos, smass, n, beg, cnt, L, theta, G, err_tol, k1h, s);  \
    else                                                                                    \
      moments_launch<P, double>(C, spos, smass, n, beg, cnt, L, theta, G, err_tol, k1h, s); \
    break;
  switch (order) {
    HOT_MOM(0)
    HOT_MOM(1)
    HOT_MOM(2)
    HOT_MOM(3)
    HOT_MOM(4)
    default:
      return hipErrorInvalidValue;
  }
#undef HOT_MOM
  return hipGetLastError();
}

hipError_t tree_groups(const Cells& C, uint32_t ncells, int gmax, size_t n, uint32_t* gflag,
                       uint32_t* gid, int32_t* gcell_at, const Groups& G, uint32_t* ngroups_dev,
                       uint32_t* scan_tmp, hipStream_t s) {
  hipError_t e = hipMemsetAsync(gflag, 0, n * sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  k_group_flags<<<(ncells + 255) / 256, 256, 0, s>>>(C, ncells, gmax, gflag, gcell_at);
  e = scan_u32(gflag, gid, ngroups_dev, n, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_group_compact<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(gflag, gid, gcell_at, n, G.cell);
  return hipGetLastError();
}

hipError_t tree_group_bbox(const Cells& C, const Groups& G, uint32_t ngroups, uint32_t gcap,
                           const double* spos, size_t n, hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  const unsigned g = std::min<uint32_t>((ngroups + 3) / 4, 1u << 16);  // four waves a block
  k_group_bbox<<<g, 256, 0, s>>>(C, G, ngroups, gcap, spos, n);
  return hipGetLastError();
}

hipError_t tree_srec(const Cells& C, uint32_t ncells, const double* spos, const double* smass,
                     size_t n, double L, int leaf_max, void* srec, bool fp32, hipStream_t s) {
  if (ncells == 0) return hipSuccess;
  int wshift = 0;
  while (wshift < 6 && (1 << wshift) < leaf_max) ++wshift;
  const uint32_t per_block = 4u * (64u >> wshift);  // four waves a block
  const unsigned g = std::min<uint32_t>((ncells + per_block - 1) / per_block, 1u << 16);
  if (fp32)
    k_srec<float4, float><<<g, 256, 0, s>>>(C, ncells, spos, smass, n, L, wshift, (float4*)srec);
  else
    k_srec<double4, double><<<g, 256, 0, s>>>(C, ncells, spos, smass, n, L, wshift,
                                               (double4*)srec);
  return hipGetLastError();
}

}  // namespace hot

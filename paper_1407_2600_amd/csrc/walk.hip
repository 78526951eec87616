// Tree walk that emits interaction lists (paper Sec. 2.1: the main stage, an
// independent traversal per sink group with the multipole acceptance test;
// sinks that are close together share one list, the m x n bundling).
//
// One 64-lane wavefront walks for one sink group.  The pending (image, cell)
// pairs live in an LDS stack; each step pops up to 64 of them, one per lane,
// and each lane decides for its pair:
//   - image 0 and the cell is the group itself: skip (the group's own
//     particles are handled directly by the force kernel);
//   - image 0 and the cell contains the group: open;
//   - acceptance test passes: the group's local list if the local-expansion
//     bound holds there (LocalPrm), else the multipole list (the count pass
//     counts both together; the emit pass decides, writing the 16-byte
//     multipole records from the front of the group's region and the local
//     entries, one 32-bit word each, from its back, and then the two counts
//     and the end of the region);
//   - a leaf: direct list;
//   - otherwise: open (push the daughters).
// Ballots and a wave prefix sum place the emitted entries and the pushed
// daughters without atomics, so the lists are deterministic.  The test is
//   (s_B/theta + |com_B - centre_B|)^2 < d^2,
// d the distance from com_B + n L to the group's tight bounding box, in FP64
// with separate multiply and add, so that every implementation of the same
// test takes the same decisions.  The first pass counts, the second writes at
// the scanned offsets.
#include "device_math.h"

namespace hot {

constexpr int kWalkWaves = 4;

template <bool EMIT, int STACK>
__global__ void __launch_bounds__(64 * kWalkWaves) k_walk(Cells C, Groups G, uint32_t ngroups,
                                                          uint32_t gcap, double L, int periodic,
                                                          LocalPrm lp,
                                                          uint32_t* __restrict__ p2p_list,
                                                          uint4* __restrict__ m2p_list,
                                                          uint32_t* __restrict__ status) {
  __shared__ uint32_t stack_all[kWalkWaves][STACK];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t g = __builtin_amdgcn_readfirstlane(xcd_block() * kWalkWaves + wid);
  if (g >= ngroups) return;  // whole wavefront leaves; no block barriers below
  if (G.active && !G.active[g]) {  // no target of this group is due: no lists
    if (!EMIT && lane == 0) {
      G.cnt_p2p[g] = 0;
      G.cnt_m2p[g] = 0;
      G.cnt_m2l[g] = 0;
    }
    return;
  }
  uint32_t* st = stack_all[wid];
  const int A = G.cell[g];
  const uint64_t keyA = C.key[A];
  const int levA = C.level[A];
  const double lo0 = G.lo[g], lo1 = G.lo[gcap + g], lo2 = G.lo[2 * (size_t)gcap + g];
  const double hi0 = G.hi[g], hi1 = G.hi[gcap + g], hi2 = G.hi[2 * (size_t)gcap + g];
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  double cA[3];
  center_of(keyA, levA, L, cA);
  // the group's local-expansion centre (middle of its tight box) and radius
  // (half the box diagonal)
  const bool local = lp.q > 0 && lp.tol > 0.0;
  const double gc0 = 0.5 * (lo0 + hi0), gc1 = 0.5 * (lo1 + hi1), gc2 = 0.5 * (lo2 + hi2);
  double ga, gaq;
  {
    const double e0 = hi0 - gc0, e1 = hi1 - gc1, e2 = hi2 - gc2;
    double a2 = e0 * e0;
    a2 = a2 + e1 * e1;
    a2 = a2 + e2 * e2;
    ga = sqrt(a2);
    gaq = ga;
    for (int i = 1; i < lp.q; ++i) gaq = gaq * ga;
  }

  uint32_t top;
  if (periodic) {
    if (lane < 27) st[lane] = ((uint32_t)lane << 27);
    top = 27;
  } else {
    if (lane == 0) st[0] = (13u << 27);
    top = 1;
  }
  uint32_t np = 0, nm = 0, nl = 0;
  uint32_t op = 0, om = 0, oe = 0;
  if (EMIT) {
    op = G.off_p2p[g];
    om = G.off_m2p[g];
    oe = om + G.cnt_m2p[g];  // end of the group's accepted region (count pass)
  }
  wave_sync();
  while (top > 0) {
    uint32_t room = (STACK - top) / 7;
    uint32_t k = top < 64 ? top : 64;
    k = k < room ? k : room;
    if (k == 0) {
      if (lane == 0) atomicOr(status, 4u);
      break;
    }
    top -= k;
    const bool active = (uint32_t)lane < k;
    const uint32_t e = active ? st[top + lane] : 0u;
    wave_sync();
    const int img = (int)(e >> 27);
    const int B = (int)(e & kCellMask);
    // 0 none, 1 open, 2 multipole, 3 direct, 4 local
    int action = 0;
    int nch = 0, ch0 = 0;
    double cc0 = 0.0, cc1 = 0.0, cc2 = 0.0;  // image-shifted centre of mass
    if (active) {
      const bool zero = (img == 13);
      if (!(zero && B == A)) {
        nch = C.nchild[B];
        ch0 = C.child[B];
        bool anc = false;
        if (zero) {
          const int levB = C.level[B];
          anc = (levB <= levA) && ((keyA >> (3 * (levA - levB))) == C.key[B]);
        }
        if (anc) {
          action = 1;
        } else {
          const double4 w = C.walk[B];
          const double n0 = (double)(img / 9 - 1), n1 = (double)((img / 3) % 3 - 1),
                       n2 = (double)(img % 3 - 1);
          const double c0 = w.x + n0 * L, c1 = w.y + n1 * L, c2 = w.z + n2 * L;
          cc0 = c0;
          cc1 = c1;
          cc2 = c2;
          double a0 = lo0 - c0, b0 = c0 - hi0;
          double a1 = lo1 - c1, b1 = c1 - hi1;
          double a2 = lo2 - c2, b2 = c2 - hi2;
          double v0 = a0 > b0 ? a0 : b0, v1 = a1 > b1 ? a1 : b1, v2 = a2 > b2 ? a2 : b2;
          double d0 = v0 > 0.0 ? v0 : 0.0, d1 = v1 > 0.0 ? v1 : 0.0, d2 = v2 > 0.0 ? v2 : 0.0;
          double dd = d0 * d0;
          dd = dd + d1 * d1;
          dd = dd + d2 * d2;
          const double rc2 = w.w * w.w;
          if (rc2 < dd) {
            action = 2;
            if (EMIT && local) {
              // truncation and softening bound of the group's local
              // expansion without divisions, A D + C B <= tol B D (IEEE
              // operations in a fixed order)
              const double m = C.mmx[B].x, b = C.bnd[B].y;
              const double r0 = gc0 - c0, r1 = gc1 - c1, r2 = gc2 - c2;
              double rr = r0 * r0;
              rr = rr + r1 * r1;
              rr = rr + r2 * r2;
              const double u = sqrt(rr) - b;
              if (u > ga) {
                const double gm = lp.G * m;
                double A = gm * gaq;
                A = A * ((double)(lp.q + 2) * u - (double)(lp.q + 1) * ga);
                double uq = u;
                for (int i = 0; i < lp.q; ++i) uq = uq * u;
                const double w = u - ga;
                double Bv = uq * w;
                Bv = Bv * w;
                double Cv = 1.5 * gm;
                Cv = Cv * lp.eps2;
                const double w2 = w * w;
                const double Dv = w2 * w2;
                double lhs = A * Dv;
                lhs = lhs + Cv * Bv;
                double rhs = Bv * Dv;
                rhs = lp.tol * rhs;
                if (lhs <= rhs) action = 4;
              }
            }
          } else if (nch == 0)
            action = 3;
          else
            action = 1;
        }
      }
    }
    const uint64_t bm = __ballot(action == 2);
    const uint64_t bp = __ballot(action == 3);
    const uint64_t bl = __ballot(action == 4);
    if (EMIT) {
      // local entries: the bare (image << 27 | cell) word, packed downwards
      // from the end of the group's accepted region
      if (action == 4)
        reinterpret_cast<uint32_t*>(m2p_list)[(size_t)4 * oe - 1 - nl -
                                              (uint32_t)__popcll(bl & below)] = e;
      if (action == 2)
        m2p_list[om + nm + (uint32_t)__popcll(bm & below)] =
            make_uint4(__float_as_uint((float)(cc0 - cA[0])), __float_as_uint((float)(cc1 - cA[1])),
                       __float_as_uint((float)(cc2 - cA[2])), e);
      if (action == 3) p2p_list[op + np + (uint32_t)__popcll(bp & below)] = e;
    }
    nm += (uint32_t)__popcll(bm);
    np += (uint32_t)__popcll(bp);
    nl += (uint32_t)__popcll(bl);
    // push the daughters of opened cells
    uint32_t cnt = (action == 1) ? (uint32_t)nch : 0u;
    uint32_t inc = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t t = __shfl_up(inc, d, 64);
      if (lane >= d) inc += t;
    }
    const uint32_t tot = __shfl(inc, 63, 64);
    const uint32_t pre = inc - cnt;
    for (uint32_t q = 0; q < cnt; ++q) st[top + pre + q] = ((uint32_t)img << 27) | (uint32_t)(ch0 + q);
    top += tot;
    wave_sync();
  }
  if (lane == 0) {
    if (!EMIT) {
      G.cnt_p2p[g] = np;
      G.cnt_m2p[g] = nm;  // multipole and local together
      G.cnt_m2l[g] = 0;
    } else {
      G.cnt_m2p[g] = nm;
      G.cnt_m2l[g] = nl;
      G.off_m2l[g] = oe;  // the local entries: words [4 oe - nl, 4 oe)
    }
  }
}

// 64-bit totals of the per-group list counts, and the largest group's list
// size in 4-byte words (a direct entry is one word, a multipole or local
// record four)
__global__ void __launch_bounds__(256) k_sum_counts(Groups G, uint32_t ngroups,
                                                    unsigned long long* __restrict__ sums,
                                                    uint32_t* __restrict__ maxw) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long p = 0, m = 0;
  uint32_t w = 0;
  if (g < ngroups) {
    p = G.cnt_p2p[g];
    m = G.cnt_m2p[g];
    w = (uint32_t)(p + 4 * m);
  }
  for (int d = 32; d > 0; d >>= 1) {
    p += __shfl_down(p, d, 64);
    m += __shfl_down(m, d, 64);
    const uint32_t o = __shfl_down(w, d, 64);
    w = o > w ? o : w;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&sums[0], p);
    atomicAdd(&sums[1], m);
    atomicMax(maxw, w);
  }
}

// after the count pass: the direct entries, the accepted cells (multipole and
// local together) and the largest group's list words
hipError_t sum_counts(const Groups& G, uint32_t ngroups, unsigned long long* sums, uint32_t* maxw,
                      hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  k_sum_counts<<<(ngroups + 255) / 256, 256, 0, s>>>(G, ngroups, sums, maxw);
  return hipGetLastError();
}

// per block of kCountBlock consecutive groups: the sums of their direct
// entries and accepted cells (64-bit), for planning list chunks
__global__ void __launch_bounds__(256) k_block_counts(Groups G, uint32_t ngroups,
                                                      unsigned long long* __restrict__ bp,
                                                      unsigned long long* __restrict__ bm) {
  __shared__ unsigned long long sp[4], sm[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long p = 0, m = 0;
  for (uint32_t i = 0; i < kCountBlock; i += 256) {
    const uint32_t g = blockIdx.x * kCountBlock + i + threadIdx.x;
    if (g < ngroups) {
      p += G.cnt_p2p[g];
      m += G.cnt_m2p[g];
    }
  }
  for (int d = 32; d > 0; d >>= 1) {
    p += __shfl_down(p, d, 64);
    m += __shfl_down(m, d, 64);
  }
  if (lane == 0) {
    sp[wid] = p;
    sm[wid] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bp[blockIdx.x] = sp[0] + sp[1] + sp[2] + sp[3];
    bm[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
  }
}

hipError_t block_counts(const Groups& G, uint32_t ngroups, unsigned long long* bp,
                        unsigned long long* bm, hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  k_block_counts<<<(ngroups + kCountBlock - 1) / kCountBlock, 256, 0, s>>>(G, ngroups, bp, bm);
  return hipGetLastError();
}

hipError_t walk_launch(bool emit, bool big, const Cells& C, const Groups& G, uint32_t ngroups,
                       uint32_t gcap, double L, int periodic, const LocalPrm& lp,
                       uint32_t* p2p_list, uint4* m2p_list, uint32_t* status, hipStream_t s) {
  if (ngroups == 0) return hipSuccess;
  const unsigned blocks = (ngroups + kWalkWaves - 1) / kWalkWaves;
  const unsigned th = 64 * kWalkWaves;
  if (emit && big)
    k_walk<true, kWalkStackBig><<<blocks, th, 0, s>>>(C, G, ngroups, gcap, L, periodic, lp,
                                                      p2p_list, m2p_list, status);
  else if (emit)
    k_walk<true, kWalkStack><<<blocks, th, 0, s>>>(C, G, ngroups, gcap, L, periodic, lp, p2p_list,
                                                   m2p_list, status);
  else if (big)
    k_walk<false, kWalkStackBig><<<blocks, th, 0, s>>>(C, G, ngroups, gcap, L, periodic, lp,
                                                       p2p_list, m2p_list, status);
  else
    k_walk<false, kWalkStack><<<blocks, th, 0, s>>>(C, G, ngroups, gcap, L, periodic, lp, p2p_list,
                                                    m2p_list, status);
  return hipGetLastError();
}

}  // namespace hot

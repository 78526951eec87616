// Interaction kernels (paper Sec. 2.1: the gravitational inner loops; direct
// interactions with the particles of nearby leaves and multipole interactions
// with accepted cells, m source cells x n sink particles per list).
//
// One 64-lane wavefront handles one sink group: each lane holds one target
// (tiles of 64 for larger groups) in registers, and the wavefront steps
// through the group's list together, so every source particle or cell record
// is wave-uniform and is read once per wavefront (source particles through an
// LDS stage, cell records through the scalar cache), feeding all 64 targets.
//
// Precision: coordinates are relative to the group's cell centre; positions,
// cell centres and centres of mass are FP64 and are differenced in FP64
// before rounding to the arithmetic type T.  In FP32, per-leaf (direct) and
// per-16-cell (multipole) partial sums are folded into a (hi, lo) pair with
// Knuth's TwoSum, so the long sums keep about twice FP32 precision.
#include "device_math.h"

namespace hot {

constexpr int kForceWaves = 4;

// ------------------------------------------------------------------- direct
// Direct interactions of one sink group per wavefront, targets in lanes, in
// passes of up to 64 targets: first the group's own particles (image 0,
// without the target itself), then every listed leaf with its image shift.
// Sources go through a per-wavefront LDS stage of kStage records {x, y, z, m}
// relative to the group's cell centre: the list is read 64 entries at a time,
// one entry per lane (leaf range and image-shifted leaf centre, in FP64, then
// rounded), a prefix sum over the lanes concatenates the entries' sources,
// and the lanes fill the stage from that concatenated stream before all
// targets read each staged source with a broadcast LDS load.
// TAIL selects the passes as in k_m2p: the main launch takes the passes over
// more than 32 targets; the tail launch takes a last pass of at most 32
// targets and splits the wave into 2, 4 or 8 sub-groups that share out the
// staged sources, adding their partial sums at the end.  Partial sums over
// one leaf image (at most 64 of its sources) are folded into the
// accumulators.  This kernel writes (not adds) the accumulators.
constexpr int kStage = 256;

// Softening of the direct kernel.  Plummer: g = (r^2 + e2)^(-1/2), f = g^3.
// Dehnen's compensating K1 (paper Sec. 2.1), compact density
// ~ (1 - x^2)^2 (1 - 11 x^2/5) of radius h, x = r/h: inside h
//   g = (945 - 2100 x^2 + 2646 x^4 - 1620 x^6 + 385 x^8) / (256 h),
//   f = (525 - 1323 x^2 + 1215 x^4 - 385 x^6) / (32 h^3),
// beyond it exactly Newtonian (g = 1/r, f = 1/r^3).  A source of mass m adds
// m g to the potential sum and m f (source - target) to the force sum.
template <typename T>
struct Soft {
  T e2;   // Plummer eps^2 (0 with K1)
  T h2;   // K1: h^2
  T ih2;  // K1: 1/h^2
  T cg;   // K1: 1/(256 h)
  T cf;   // K1: 1/(32 h^3)
};

template <typename T>
__device__ __forceinline__ void k1_gf(T r2, const Soft<T>& sf, T& g, T& f) {
  const bool in = r2 < sf.h2;
  const T x2 = r2 * sf.ih2;
  const T gp = fma(fma(fma(fma((T)385, x2, (T)-1620), x2, (T)2646), x2, (T)-2100), x2, (T)945) *
               sf.cg;
  const T fp = fma(fma(fma((T)-385, x2, (T)1215), x2, (T)-1323), x2, (T)525) * sf.cf;
  const T ri = rsqrt_t(in ? (T)1 : r2);
  g = in ? gp : ri;
  f = in ? fp : ri * (ri * ri);
}

// staged sources [a, b) against this lane's target; the partial sums are
// folded every 64 sources and at the end
template <typename T, typename T4, bool OWN, bool K1>
__device__ __forceinline__ void p2p_staged(const T4* __restrict__ st, int a, int b, uint32_t sub,
                                           uint32_t split, T tx, T ty, T tz, const Soft<T>& sf,
                                           uint32_t self_slot, Acc<T>& acc) {
  for (int b0 = a; b0 < b; b0 += 64) {
    const int b1 = b0 + 64 < b ? b0 + 64 : b;
    T part[4] = {0, 0, 0, 0};
#pragma unroll 4
    for (int j = b0 + (int)sub; j < b1; j += (int)split) {
      const T4 r = st[j];
      const T dx = r.x - tx, dy = r.y - ty, dz = r.z - tz;
      T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, sf.e2)));
      T mr, mr3;
      if constexpr (K1) {
        T g, f;
        k1_gf(r2, sf, g, f);
        mr = r.w * g;
        mr3 = r.w * f;
        if constexpr (OWN) {
          const bool self = (uint32_t)j == self_slot;
          mr = self ? (T)0 : mr;
          mr3 = self ? (T)0 : mr3;
        }
      } else if constexpr (OWN) {
        const bool self = (uint32_t)j == self_slot;
        r2 = self ? (T)1 : r2;
        const T ri = rsqrt_t(r2);
        mr = self ? (T)0 : r.w * ri;
        mr3 = mr * (ri * ri);
      } else {
        const T ri = rsqrt_t(r2);
        mr = r.w * ri;
        mr3 = mr * (ri * ri);
      }
      part[0] = fma(dx, mr3, part[0]);
      part[1] = fma(dy, mr3, part[1]);
      part[2] = fma(dz, mr3, part[2]);
      part[3] += mr;
    }
    acc.fold(part);
  }
}

// the per-wavefront LDS of the direct kernels
template <typename T, typename T4, int W, int S>
struct SourceStage {
  T4 st[W][S];
  uint32_t incl[W][64];
  uint32_t bf[W][64];
  T sh[W][3][64];
};

template <typename T, typename T4, bool TAIL, bool K1>
__device__ __forceinline__ void p2p_group(uint32_t g, SourceStage<T, T4, kForceWaves, kStage>& lds,
                                          Cells C, Groups G,
                                          double L, Soft<T> sf,
                                          const double* __restrict__ spos,
                                          const T4* __restrict__ srec, size_t n,
                                          const uint32_t* __restrict__ list,
                                          double4* __restrict__ out){
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T4* st = lds.st[wid];
  uint32_t* e_incl = lds.incl[wid];
  uint32_t* e_bf = lds.bf[wid];
  T(*e_sh)[64] = lds.sh[wid];
  const int A = __builtin_amdgcn_readfirstlane(G.cell[g]);
  const uint32_t first = __builtin_amdgcn_readfirstlane(C.first[A]);
  const uint32_t count = __builtin_amdgcn_readfirstlane(C.count[A]);
  const uint32_t tail0 = count - count % 64;
  const bool has_tail = count % 64 != 0 && count % 64 <= 32;
  if (TAIL && !has_tail) return;
  double cA[3];
  center_of(C.key[A], C.level[A], L, cA);
  const uint32_t off = G.off_p2p[g], cnt = G.cnt_p2p[g];
  for (uint32_t t0 = TAIL ? tail0 : 0; t0 < count; t0 += 64) {
    const uint32_t rem = count - t0;
    if (!TAIL && rem <= 32) break;
    const uint32_t split = !TAIL ? 1u : rem <= 8 ? 8u : rem <= 16 ? 4u : 2u;  // wave-uniform
    const int width = 64 / (int)split;
    const uint32_t sub = (uint32_t)(lane / width);
    const int tl = lane % width;
    const uint32_t s = first + t0 + tl;
    const bool act = (uint32_t)tl < rem;
    const uint32_t ss = act ? s : first;
    const T tx = (T)(spos[ss] - cA[0]), ty = (T)(spos[n + ss] - cA[1]),
            tz = (T)(spos[2 * n + ss] - cA[2]);
    Acc<T> acc;
    acc.zero();
    // own group (image 0), excluding the target itself
    for (uint32_t s0 = 0; s0 < count; s0 += kStage) {
      const int nb = (int)(count - s0 < (uint32_t)kStage ? count - s0 : (uint32_t)kStage);
      wave_sync();
      for (int k = lane; k < nb; k += 64) {
        const uint32_t j = first + s0 + (uint32_t)k;
        T4 r;
        r.x = (T)(spos[j] - cA[0]);
        r.y = (T)(spos[n + j] - cA[1]);
        r.z = (T)(spos[2 * n + j] - cA[2]);
        r.w = srec[j].w;
        st[k] = r;
      }
      wave_sync();
      p2p_staged<T, T4, true, K1>(st, 0, nb, sub, split, tx, ty, tz, sf, ss - first - s0, acc);
    }
    // listed leaves, 64 entries at a time
    for (uint32_t q0 = 0; q0 < cnt; q0 += 64) {
      const uint32_t ne = cnt - q0 < 64u ? cnt - q0 : 64u;
      uint32_t bc = 0, bf = 0;
      T sx = 0, sy = 0, sz = 0;
      if ((uint32_t)lane < ne) {
        const uint32_t e = list[off + q0 + (uint32_t)lane];
        const int img = (int)(e >> 27);
        const int B = (int)(e & kCellMask);
        double cB[3];
        center_of(C.key[B], C.level[B], L, cB);
        sx = (T)(cB[0] + (double)(img / 9 - 1) * L - cA[0]);
        sy = (T)(cB[1] + (double)((img / 3) % 3 - 1) * L - cA[1]);
        sz = (T)(cB[2] + (double)(img % 3 - 1) * L - cA[2]);
        bf = C.first[B];
        bc = C.count[B];
      }
      const uint32_t incl = wave_incl_scan(bc, lane);
      const uint32_t total = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
      wave_sync();
      e_incl[lane] = incl;
      e_bf[lane] = bf - (incl - bc);  // source index = e_bf + stream position
      e_sh[0][lane] = sx;
      e_sh[1][lane] = sy;
      e_sh[2][lane] = sz;
      uint32_t ecur = 0;  // first entry of the batch (wave-uniform)
      for (uint32_t s0 = 0; s0 < total; s0 += kStage) {
        const int nb = (int)(total - s0 < (uint32_t)kStage ? total - s0 : (uint32_t)kStage);
        wave_sync();
        for (int k = lane; k < nb; k += 64) {
          const uint32_t slot = s0 + (uint32_t)k;
          // the entry holding this stream position: the first with incl > slot
          int e = 0;
#pragma unroll
          for (int step = 32; step > 0; step >>= 1)
            if (e_incl[e + step - 1] <= slot) e += step;
          const T4 r = srec[e_bf[e] + slot];
          T4 v;
          v.x = e_sh[0][e] + r.x;
          v.y = e_sh[1][e] + r.y;
          v.z = e_sh[2][e] + r.z;
          v.w = r.w;
          st[k] = v;
        }
        wave_sync();
        // one leaf image at a time, so that each is folded on its own (the
        // images of one leaf can cancel to far below their size)
        const uint32_t s1 = s0 + (uint32_t)nb;
        uint32_t lo = ecur ? __builtin_amdgcn_readfirstlane(e_incl[ecur - 1]) : 0u;
        for (;;) {
          const uint32_t hi = __builtin_amdgcn_readfirstlane(e_incl[ecur]);
          const int a = (int)((lo > s0 ? lo : s0) - s0);
          const int b = (int)((hi < s1 ? hi : s1) - s0);
          p2p_staged<T, T4, false, K1>(st, a, b, sub, split, tx, ty, tz, sf, 0u, acc);
          if (hi > s1) break;  // the entry continues in the next batch
          lo = hi;
          ++ecur;
          if (hi == s1) break;
        }
      }
    }
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = acc.get(k);
    for (int w = width; w < 64; w <<= 1)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += __shfl_xor(v[k], w, 64);
    if (act && sub == 0) out[s] = make_double4(v[0], v[1], v[2], v[3]);
  }
}


// Multipole interactions of one sink group per wavefront, targets in lanes,
// in passes of up to 64 targets.  TAIL = false: the passes over more than 32
// targets, each walking the list once with every entry wave-uniform (scalar
// loads of the record and the cell's coefficients).  TAIL = true: the last
// pass when it has at most 32 targets (the remainder of a group of 65..96,
// or a small group), one group per block: the block's 4 wavefronts each
// split into 2, 4 or 8 sub-groups of 32, 16 or 8 lanes, the sub-groups take
// every 8th, 16th or 32nd list entry, and the partial sums are added across
// sub-groups and wavefronts at the end, so the lanes a short pass would leave
// idle do the work.  Separate launches keep the register budget (and
// occupancy) of the main pass independent of the tail's.
template <int P, typename T, bool TAIL>
__device__ __forceinline__ void m2p_group(uint32_t g, Cells C, Groups G,
                                          double L, T eps2,
                                          const double* __restrict__ spos,
                                          size_t n,
                                          const uint4* __restrict__ list,
                                          double4* __restrict__ out){
  constexpr int STR = coef_stride(P);
  // tail pass: one coefficient block per sub-group of each wavefront
  __shared__ __align__(16) T tail_cf[TAIL ? kForceWaves : 1][8][TAIL ? STR : 1];
  // tail pass: the block's wavefronts share out one group's list and add
  // their results through LDS in a fixed order
  __shared__ double tail_red[TAIL ? kForceWaves : 1][TAIL ? 32 : 1][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t nw = TAIL ? kForceWaves : 1, w0 = TAIL ? (uint32_t)wid : 0;
  const int A = __builtin_amdgcn_readfirstlane(G.cell[g]);
  const uint32_t first = __builtin_amdgcn_readfirstlane(C.first[A]);
  const uint32_t count = __builtin_amdgcn_readfirstlane(C.count[A]);
  double cA[3];
  center_of(C.key[A], C.level[A], L, cA);
  const uint32_t off = G.off_m2p[g], cnt = G.cnt_m2p[g];
  const T* __restrict__ coef = (const T*)C.coef;
  const uint32_t tail0 = count - count % 64;  // start of a pass of < 64 targets
  const bool has_tail = count % 64 != 0 && count % 64 <= 32;
  if (TAIL && !has_tail) return;
  for (uint32_t t0 = TAIL ? tail0 : 0; t0 < count; t0 += 64) {
    const uint32_t rem = count - t0;
    if (!TAIL && rem <= 32) break;
    const int split = !TAIL ? 1 : rem <= 8 ? 8 : rem <= 16 ? 4 : 2;  // wave-uniform
    const int width = 64 / split;
    const int sub = lane / width, tl = lane % width;
    const uint32_t s = first + t0 + tl;
    const bool act = (uint32_t)tl < rem;
    const uint32_t ss = act ? s : first;
    const T tx = (T)(spos[ss] - cA[0]), ty = (T)(spos[n + ss] - cA[1]),
            tz = (T)(spos[2 * n + ss] - cA[2]);
    Acc<T> acc;
    acc.zero();
    T part[4] = {0, 0, 0, 0};
    if (!TAIL) {
      for (uint32_t q = 0; q < cnt; ++q) {
        T c[3];
        const int B = m2p_record<T>(list[off + q], C.walk, L, cA, c);
        T r[4];
        m2p_eval<P, false, T, T>(tx - c[0], ty - c[1], tz - c[2], eps2, coef + (size_t)B * STR,
                                 r);
#pragma unroll
        for (int k = 0; k < 3; ++k) part[k] += r[k];
        // the potential sums many same-signed terms that the far field later
        // cancels almost entirely: fold every term
        acc.fold1(3, r[3]);
        if ((q & 15) == 15) {
          acc.fold(part);
#pragma unroll
          for (int k = 0; k < 3; ++k) part[k] = (T)0;
        }
      }
    } else {
      // each 16-lane row loads its sub-group's entry's coefficient block
      // spread over the row; the sub-group's first row puts it in the
      // sub-group's LDS slot, from which every lane reads it.  The next
      // entry is loaded while this one is evaluated.
      constexpr int NC = (STR + 7) / 8;  // values per loading lane (8 or 16 of them)
      const int wl = width < 16 ? width : 16;  // the sub-group's loading lanes
      const int rl = lane & (wl - 1);
      const uint32_t step = nw * split;
      T* cslot = &tail_cf[wid][sub][0];
      const bool writer = (lane & (width - 1)) < wl;
      RowBlock<T, NC> cf;
      T c[3] = {0, 0, 0};
      uint32_t q = w0 * split + (uint32_t)sub;
      if (q < cnt) {
        const int B = m2p_record<T>(list[off + q], C.walk, L, cA, c);
        cf.load(coef + (size_t)B * STR, STR, rl, wl);
      }
      uint32_t it = 0;
      while (q < cnt) {
        if (writer) cf.store(cslot, STR, rl, wl);
        wave_sync();
        const uint32_t qn = q + step;
        T c2[3] = {0, 0, 0};
        if (qn < cnt) {
          const int B = m2p_record<T>(list[off + qn], C.walk, L, cA, c2);
          cf.load(coef + (size_t)B * STR, STR, rl, wl);
        }
        T r[4];
        m2p_eval<P, false, T, T>(tx - c[0], ty - c[1], tz - c[2], eps2, (const T*)cslot, r);
#pragma unroll
        for (int k = 0; k < 3; ++k) part[k] += r[k];
        acc.fold1(3, r[3]);
        if ((++it & 15) == 0) {
          acc.fold(part);
#pragma unroll
          for (int k = 0; k < 3; ++k) part[k] = (T)0;
        }
        wave_sync();
        c[0] = c2[0];
        c[1] = c2[1];
        c[2] = c2[2];
        q = qn;
      }
    }
    acc.fold(part);
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = acc.get(k);
    for (int w = width; w < 64; w <<= 1)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += __shfl_xor(v[k], w, 64);
    if constexpr (TAIL) {
      if (sub == 0 && tl < 32)
#pragma unroll
        for (int k = 0; k < 4; ++k) tail_red[wid][tl][k] = v[k];
      __syncthreads();
      if (wid == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          v[k] = tail_red[0][tl < 32 ? tl : 0][k];
          for (int w = 1; w < kForceWaves; ++w) v[k] += tail_red[w][tl < 32 ? tl : 0][k];
        }
      }
    }
    if (act && sub == 0 && w0 == 0) {
      double4 o = out[s];
      o.x += v[0];
      o.y += v[1];
      o.z += v[2];
      o.w += v[3];
      out[s] = o;
    }
  }
}

// Main and tail passes are separate kernels (the tail pass needs more
// registers), launched tail first on the context's side stream so that its
// few long, lightly occupied wavefronts run beside the main passes.
template <typename T, typename T4, bool TAIL, bool K1>
__global__ void __launch_bounds__(64 * kForceWaves) k_p2p(Cells C, Groups G, uint32_t ngroups,
                                                          double L, Soft<T> sf,
                                                          const double* __restrict__ spos,
                                                          const T4* __restrict__ srec, size_t n,
                                                          const uint32_t* __restrict__ list,
                                                          double4* __restrict__ out) {
  __shared__ SourceStage<T, T4, kForceWaves, kStage> lds;
  const int wid = threadIdx.x >> 6;
  const uint32_t g = __builtin_amdgcn_readfirstlane(xcd_block() * kForceWaves + wid);
  if (g >= ngroups) return;
  if (G.active && !G.active[g]) return;  // no target due: nothing written
  p2p_group<T, T4, TAIL, K1>(g, lds, C, G, L, sf, spos, srec, n, list, out);
}

// main passes one group per wavefront; tail passes one group per block
template <int P, typename T, bool TAIL>
__global__ void __launch_bounds__(64 * kForceWaves) k_m2p(Cells C, Groups G, uint32_t ngroups,
                                                          double L, T eps2,
                                                          const double* __restrict__ spos,
                                                          size_t n,
                                                          const uint4* __restrict__ list,
                                                          double4* __restrict__ out) {
  const int wid = threadIdx.x >> 6;
  const uint32_t g =
      __builtin_amdgcn_readfirstlane(TAIL ? xcd_block() : xcd_block() * kForceWaves + wid);
  if (g >= ngroups) return;
  if (G.active && !G.active[g]) return;  // block- (tail) or wave-uniform (main)
  m2p_group<P, T, TAIL>(g, C, G, L, eps2, spos, n, list, out);
}

template <typename T, typename T4, bool K1>
static hipError_t p2p_launch_t(const Cells& C, const Groups& G, uint32_t ngroups, double L,
                               Soft<T> sf, const double* spos, const T4* srec, size_t n,
                               const uint32_t* list, double4* out, hipStream_t s,
                               const SideStream& side) {
  const unsigned nb = (ngroups + kForceWaves - 1) / kForceWaves;
  hipStream_t st;
  hipError_t e = side_fork(side, s, &st);
  if (e != hipSuccess) return e;
  k_p2p<T, T4, true, K1><<<nb, 64 * kForceWaves, 0, st>>>(C, G, ngroups, L, sf, spos, srec, n,
                                                          list, out);
  k_p2p<T, T4, false, K1><<<nb, 64 * kForceWaves, 0, s>>>(C, G, ngroups, L, sf, spos, srec, n,
                                                           list, out);
  e = hipGetLastError();
  return e != hipSuccess ? e : side_join(side, s);
}

template <typename T, typename T4>
static hipError_t p2p_launch_k(bool k1, const Cells& C, const Groups& G, uint32_t ngroups,
                               double L, double eps, const double* spos, const T4* srec, size_t n,
                               const uint32_t* list, double4* out, hipStream_t s,
                               const SideStream& side) {
  Soft<T> sf{};
  if (!k1) {
    sf.e2 = (T)(eps * eps);
    return p2p_launch_t<T, T4, false>(C, G, ngroups, L, sf, spos, srec, n, list, out, s, side);
  }
  const double h = k1_radius(eps);
  sf.h2 = (T)(h * h);
  sf.ih2 = (T)(1.0 / (h * h));
  sf.cg = (T)(1.0 / (256.0 * h));
  sf.cf = (T)(1.0 / (32.0 * h * h * h));
  return p2p_launch_t<T, T4, true>(C, G, ngroups, L, sf, spos, srec, n, list, out, s, side);
}

hipError_t p2p_launch(bool fp32, int kernel, const Cells& C, const Groups& G, uint32_t ngroups,
                      double L, double eps, const double* spos, const void* srec, size_t n,
                      const uint32_t* list, double4* out, hipStream_t s, const SideStream& side) {
  if (ngroups == 0) return hipSuccess;
  const bool k1 = kernel == HOT_KERNEL_K1;
  if (k1 && !(eps > 0.0)) return hipErrorInvalidValue;
  if (fp32)
    return p2p_launch_k<float, float4>(k1, C, G, ngroups, L, eps, spos, (const float4*)srec, n,
                                       list, out, s, side);
  return p2p_launch_k<double, double4>(k1, C, G, ngroups, L, eps, spos, (const double4*)srec, n,
                                       list, out, s, side);
}

template <int P, typename T>
static hipError_t m2p_launch_t(const Cells& C, const Groups& G, uint32_t ngroups, double L,
                               T eps2, const double* spos, size_t n, const uint4* list,
                               double4* out, hipStream_t s, const SideStream& side) {
  const unsigned nb = (ngroups + kForceWaves - 1) / kForceWaves;
  hipStream_t st;
  hipError_t e = side_fork(side, s, &st);
  if (e != hipSuccess) return e;
  k_m2p<P, T, true><<<ngroups, 64 * kForceWaves, 0, st>>>(C, G, ngroups, L, eps2, spos, n, list,
                                                           out);
  k_m2p<P, T, false><<<nb, 64 * kForceWaves, 0, s>>>(C, G, ngroups, L, eps2, spos, n, list, out);
  e = hipGetLastError();
  return e != hipSuccess ? e : side_join(side, s);
}

template <int P>
static hipError_t m2p_launch_p(bool fp32, const Cells& C, const Groups& G, uint32_t ngroups,
                               double L, double eps, const double* spos, size_t n,
                               const uint4* list, double4* out, hipStream_t s,
                               const SideStream& side) {
  if (fp32)
    return m2p_launch_t<P, float>(C, G, ngroups, L, (float)(eps * eps), spos, n, list, out, s,
                                  side);
  return m2p_launch_t<P, double>(C, G, ngroups, L, eps * eps, spos, n, list, out, s, side);
}

hipError_t m2p_launch(bool fp32, int order, const Cells& C, const Groups& G, uint32_t ngroups,
                      double L, double eps, const double* spos, size_t n, const uint4* list,
                      double4* out, hipStream_t s, const SideStream& side) {
  if (ngroups == 0) return hipSuccess;
  switch (order) {
    case 0: return m2p_launch_p<0>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s, side);
    case 1: return m2p_launch_p<1>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s, side);
    case 2: return m2p_launch_p<2>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s, side);
    case 3: return m2p_launch_p<3>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s, side);
    case 4: return m2p_launch_p<4>(fp32, C, G, ngroups, L, eps, spos, n, list, out, s, side);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hot

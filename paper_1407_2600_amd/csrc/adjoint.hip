// Adjoint of the force evaluation (vector-Jacobian product with respect to
// positions and masses; an extension beyond the paper).
//
// For the loss L = sum_i gacc_i . a_i + gpot_i phi_i the exact derivatives of
// the softened direct sum, as gathers over each particle's own interactions
// (r = x_k - x_j - nL, g the softened kernel, H its Hessian):
//   xbar_k = G sum_j [ H(r) (m_j gacc_k - m_k gacc_j) - grad g(r) (m_j gpot_k + m_k gpot_j) ]
//   mbar_k = -G sum_j [ gacc_j . grad g(r) + gpot_j g(r) ]
// They are evaluated with the forward pass's interaction lists:
//   - leaves and the own group pair by pair (k_p2p_adj);
//   - accepted cells (k_m2p_adj) through two expansions about the cell's
//     centre of mass: the mass expansion evaluated on dual numbers along
//     gacc_k, which yields grad Phi and H gacc_k in one pass, and one order
//     p+1 expansion of the effective charge distribution of the sources
//     (charges gpot_j plus dipoles gacc_j, both moment sets truncated at
//     order p like the mass moments, so
//       E_k = sum_j [gpot_j d^k [|k| <= p] - sum_a k_a gacc_j,a d^(k - e_a)]),
//     whose potential psi and gradient give mbar_k = -G psi and the
//     - G m_k grad psi part of xbar_k;
//   - the periodic far field differentiated exactly (far_adjoint below).
// At theta = 0 this is the exact derivative of the 27-image + far-field sum;
// for theta > 0 it is the tree approximation of that derivative.
#include "device_math.h"

namespace hot {

constexpr int kAdjWaves = 4;

// sorted cotangents: (gacc, gpot) per particle in the arithmetic type
template <typename T, typename T4>
__global__ void __launch_bounds__(256) k_adj_gather(const T* __restrict__ gacc,
                                                    const T* __restrict__ gpot, size_t n,
                                                    const uint32_t* __restrict__ idx,
                                                    T4* __restrict__ arec) {
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t i = idx[s];
  T4 r;
  r.x = gacc[i];
  r.y = gacc[n + i];
  r.z = gacc[2 * n + i];
  r.w = gpot ? gpot[i] : (T)0;
  arec[s] = r;
}

// Source-side cotangent moments about each cell's centre of mass, truncated
// like the mass moments: the charge part Q_k = sum_j gpot_j d^k for |k| <= P,
// and the dipole part A_k = -sum_j sum_a k_a gacc_j,a d^(k - e_a), which
// holds gacc moments up to order P and so reaches order P+1. Both are shifted
// exactly from the daughters (moments of a distribution shift without loss
// when every lower order is present), and only their sum
// E = Q + A, an order P+1 block, is turned into coefficients (dipole part
// kept). Shifting E itself would leak order P+1 charge terms into parents.
template <int P, typename T, typename T4>
__global__ void __launch_bounds__(128) k_adj_moments(Cells C, const double* __restrict__ spos,
                                                     const T4* __restrict__ arec, size_t n,
                                                     uint32_t beg, uint32_t cnt, double* emom,
                                                     T* __restrict__ ecoef) {
  constexpr int Q = P + 1;
  constexpr int NA = nt(Q), NQ = nt(P);
  constexpr MI<Q> mi{};
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const uint32_t c = beg + t;
  const double4 w = C.walk[c];
  const double com[3] = {w.x, w.y, w.z};
  const int nc = C.nchild[c];
  const int c0 = C.child[c];
  double A[NA], Qm[NQ];
#pragma unroll
  for (int k = 0; k < NA; ++k) A[k] = 0.0;
#pragma unroll
  for (int k = 0; k < NQ; ++k) Qm[k] = 0.0;
  if (nc == 0) {
    const uint32_t f = C.first[c], e = f + C.count[c];
    for (uint32_t s = f; s < e; ++s) {
      const T4 r = arec[s];
      const double q = (double)r.w;
      const double ga[3] = {(double)r.x, (double)r.y, (double)r.z};
      const double d[3] = {spos[s] - com[0], spos[n + s] - com[1], spos[2 * n + s] - com[2]};
      double pw[3][Q + 1];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pw[a][0] = 1.0;
#pragma unroll
        for (int e2 = 1; e2 <= Q; ++e2) pw[a][e2] = pw[a][e2 - 1] * d[a];
      }
#pragma unroll
      for (int k = 0; k < NA; ++k) {
        const int ka = mi.a[k], kb = mi.b[k], kc = mi.c[k];
        double v = 0.0;
        if (ka) v -= ka * ga[0] * pw[0][ka - 1] * pw[1][kb] * pw[2][kc];
        if (kb) v -= kb * ga[1] * pw[0][ka] * pw[1][kb - 1] * pw[2][kc];
        if (kc) v -= kc * ga[2] * pw[0][ka] * pw[1][kb] * pw[2][kc - 1];
        A[k] += v;
        if (k < NQ) Qm[k] += q * pw[0][ka] * pw[1][kb] * pw[2][kc];
      }
    }
  } else {
    for (int kc2 = 0; kc2 < nc; ++kc2) {
      const int ch = c0 + kc2;
      const double4 wc = C.walk[ch];
      const double d[3] = {wc.x - com[0], wc.y - com[1], wc.z - com[2]};
      const double* Mc = emom + (size_t)ch * (NA + NQ);
      double Mch[NA];
#pragma unroll
      for (int k = 0; k < NA; ++k) Mch[k] = Mc[k];
      shift_add<Q>(Mch, d, A);
      double Qch[NQ];
#pragma unroll
      for (int k = 0; k < NQ; ++k) Qch[k] = Mc[NA + k];
      shift_add<P>(Qch, d, Qm);
    }
  }
  double* Mo = emom + (size_t)c * (NA + NQ);
#pragma unroll
  for (int k = 0; k < NA; ++k) Mo[k] = A[k];
#pragma unroll
  for (int k = 0; k < NQ; ++k) Mo[NA + k] = Qm[k];
  // order-P+1 multi-indices come after all lower orders, so E = A + Q is a
  // prefix add
#pragma unroll
  for (int k = 0; k < NQ; ++k) A[k] += Qm[k];
  coef_store<Q, true, T>(A, ecoef + (size_t)c * coef_stride(Q, true));
}

// ---------------------------------------------------------------- direct
// per pair, with r = x_k - x_j:
//   xbar += -w/s^3 + r (3 (r.w)/s^5 + (m_j gpot_k + m_k gpot_j)/s^3),
//           w = m_j gacc_k - m_k gacc_j
//   mbar += (r . gacc_j)/s^3 - gpot_j/s
template <typename T>
__device__ __forceinline__ void pair_adj(T rx, T ry, T rz, T eps2, T mk, T gkx, T gky, T gkz,
                                         T gpk, T mj, T gjx, T gjy, T gjz, T gpj, T part[4]) {
  const T s2 = fma(rx, rx, fma(ry, ry, fma(rz, rz, eps2)));
  const T si = rsqrt_t(s2);
  const T si2 = si * si;
  const T si3 = si2 * si;
  const T si5 = si3 * si2;
  const T wx = fma(mj, gkx, -mk * gjx), wy = fma(mj, gky, -mk * gjy), wz = fma(mj, gkz, -mk * gjz);
  const T rw = fma(rx, wx, fma(ry, wy, rz * wz));
  const T cp = fma(mj, gpk, mk * gpj);
  const T al = fma((T)3 * rw, si5, si3 * cp);
  part[0] = fma(rx, al, fma(-wx, si3, part[0]));
  part[1] = fma(ry, al, fma(-wy, si3, part[1]));
  part[2] = fma(rz, al, fma(-wz, si3, part[2]));
  const T ra = fma(rx, gjx, fma(ry, gjy, rz * gjz));
  part[3] = fma(ra, si3, fma(-gpj, si, part[3]));
}

// Sources and their cotangents go through a per-wavefront LDS stage as in the
// forward direct kernel (list read 64 entries at a time, one per lane; the
// entries' sources concatenated by a prefix sum over the lanes); partial sums
// are folded per leaf image.
constexpr int kAdjStage = 128;

template <typename T, typename T4, bool OWN>
__device__ __forceinline__ void p2p_adj_staged(const T4* __restrict__ st,
                                               const T4* __restrict__ sa, int a, int b,
                                               uint32_t sub, uint32_t split, T tx, T ty, T tz,
                                               T eps2, T mk, const T4& ak, uint32_t self_slot,
                                               Acc<T>& acc) {
  for (int b0 = a; b0 < b; b0 += 64) {
    const int b1 = b0 + 64 < b ? b0 + 64 : b;
    T part[4] = {0, 0, 0, 0};
#pragma unroll 2
    for (int j = b0 + (int)sub; j < b1; j += (int)split) {
      const T4 r = st[j];
      const T4 aj = sa[j];
      if constexpr (OWN) {
        // the target itself: zero masses and cotangents and a unit distance
        // give no contribution
        const bool self = (uint32_t)j == self_slot;
        const T mj = self ? (T)0 : r.w;
        const T mkk = self ? (T)0 : mk;
        T rx = tx - r.x, ry = ty - r.y, rz = tz - r.z;
        rx = self ? (T)1 : rx;
        pair_adj<T>(rx, ry, rz, eps2, mkk, ak.x, ak.y, ak.z, ak.w, mj, self ? (T)0 : aj.x,
                    self ? (T)0 : aj.y, self ? (T)0 : aj.z, self ? (T)0 : aj.w, part);
      } else {
        pair_adj<T>(tx - r.x, ty - r.y, tz - r.z, eps2, mk, ak.x, ak.y, ak.z, ak.w, r.w, aj.x,
                    aj.y, aj.z, aj.w, part);
      }
    }
    acc.fold(part);
  }
}

// TAIL selects the passes as in the forward direct kernel: the main launch
// takes the passes over more than 32 targets, the tail launch a last pass of
// at most 32 targets with the wave split into 2 or 4 sub-groups that share
// out the staged sources.
template <typename T, typename T4, bool TAIL>
__global__ void __launch_bounds__(64 * kAdjWaves) k_p2p_adj(Cells C, Groups G, uint32_t ngroups,
                                                            double L, T eps2,
                                                            const double* __restrict__ spos,
                                                            const T4* __restrict__ srec,
                                                            const T4* __restrict__ arec, size_t n,
                                                            const uint32_t* __restrict__ list,
                                                            double4* __restrict__ out) {
  __shared__ T4 stage_all[kAdjWaves][kAdjStage];
  __shared__ T4 astage_all[kAdjWaves][kAdjStage];
  __shared__ uint32_t incl_all[kAdjWaves][64];
  __shared__ uint32_t bf_all[kAdjWaves][64];
  __shared__ T sh_all[kAdjWaves][3][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t g = __builtin_amdgcn_readfirstlane(xcd_block() * kAdjWaves + wid);
  if (g >= ngroups) return;
  T4* st = stage_all[wid];
  T4* sa = astage_all[wid];
  uint32_t* e_incl = incl_all[wid];
  uint32_t* e_bf = bf_all[wid];
  T(*e_sh)[64] = sh_all[wid];
  const int A = __builtin_amdgcn_readfirstlane(G.cell[g]);
  const uint32_t first = __builtin_amdgcn_readfirstlane(C.first[A]);
  const uint32_t count = __builtin_amdgcn_readfirstlane(C.count[A]);
  double cA[3];
  center_of(C.key[A], C.level[A], L, cA);
  const uint32_t off = G.off_p2p[g], cnt = G.cnt_p2p[g];
  const uint32_t tail0 = count - count % 64;
  const bool has_tail = count % 64 != 0 && count % 64 <= 32;
  if (TAIL && !has_tail) return;
  for (uint32_t t0 = TAIL ? tail0 : 0; t0 < count; t0 += 64) {
    const uint32_t rem = count - t0;
    if (!TAIL && rem <= 32) break;
    const uint32_t split = !TAIL ? 1u : rem <= 16 ? 4u : 2u;  // wave-uniform
    const int width = 64 / (int)split;
    const uint32_t sub = (uint32_t)(lane / width);
    const int tl = lane % width;
    const uint32_t s = first + t0 + tl;
    const bool act = (uint32_t)tl < rem;
    const uint32_t ss = act ? s : first;
    const T tx = (T)(spos[ss] - cA[0]), ty = (T)(spos[n + ss] - cA[1]),
            tz = (T)(spos[2 * n + ss] - cA[2]);
    const T mk = srec[ss].w;
    const T4 ak = arec[ss];
    Acc<T> acc;
    acc.zero();
    // own group (image 0)
    for (uint32_t s0 = 0; s0 < count; s0 += kAdjStage) {
      const int nb =
          (int)(count - s0 < (uint32_t)kAdjStage ? count - s0 : (uint32_t)kAdjStage);
      wave_sync();
      for (int k = lane; k < nb; k += 64) {
        const uint32_t j = first + s0 + (uint32_t)k;
        T4 r;
        r.x = (T)(spos[j] - cA[0]);
        r.y = (T)(spos[n + j] - cA[1]);
        r.z = (T)(spos[2 * n + j] - cA[2]);
        r.w = srec[j].w;
        st[k] = r;
        sa[k] = arec[j];
      }
      wave_sync();
      p2p_adj_staged<T, T4, true>(st, sa, 0, nb, sub, split, tx, ty, tz, eps2, mk, ak,
                                  ss - first - s0, acc);
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
      for (uint32_t s0 = 0; s0 < total; s0 += kAdjStage) {
        const int nb =
            (int)(total - s0 < (uint32_t)kAdjStage ? total - s0 : (uint32_t)kAdjStage);
        wave_sync();
        for (int k = lane; k < nb; k += 64) {
          const uint32_t slot = s0 + (uint32_t)k;
          int e = 0;  // the entry holding this stream position
#pragma unroll
          for (int step = 32; step > 0; step >>= 1)
            if (e_incl[e + step - 1] <= slot) e += step;
          const uint32_t j = e_bf[e] + slot;
          const T4 r = srec[j];
          T4 v;
          v.x = e_sh[0][e] + r.x;
          v.y = e_sh[1][e] + r.y;
          v.z = e_sh[2][e] + r.z;
          v.w = r.w;
          st[k] = v;
          sa[k] = arec[j];
        }
        wave_sync();
        const uint32_t s1 = s0 + (uint32_t)nb;
        uint32_t lo = ecur ? __builtin_amdgcn_readfirstlane(e_incl[ecur - 1]) : 0u;
        for (;;) {
          const uint32_t hi = __builtin_amdgcn_readfirstlane(e_incl[ecur]);
          const int a = (int)((lo > s0 ? lo : s0) - s0);
          const int b = (int)((hi < s1 ? hi : s1) - s0);
          p2p_adj_staged<T, T4, false>(st, sa, a, b, sub, split, tx, ty, tz, eps2, mk, ak, 0u,
                                       acc);
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

// --------------------------------------------------------------- multipole
// Passes of up to 64 targets as in the forward kernel: TAIL = false takes the
// passes over more than 32 targets with wave-uniform (scalar) loads; TAIL =
// true takes a last pass of at most 32 targets and splits the wave into 2 or
// 4 sub-groups that share out the list entries, each round staging the
// entries' mass and effective-charge coefficient blocks through LDS with
// coalesced loads, and adds the sub-groups' partial sums at the end.
template <int P, typename T, typename T4, bool TAIL>
__device__ __forceinline__ void m2p_adj_group(uint32_t g, Cells C, Groups G,
                                              double L, T eps2,
                                              const double* __restrict__ spos,
                                              const T4* __restrict__ srec,
                                              const T4* __restrict__ arec,
                                              const T* __restrict__ ecoef, size_t n,
                                              const uint4* __restrict__ list,
                                              double4* __restrict__ out){
  constexpr int STR = coef_stride(P);
  constexpr int ESTR = coef_stride(P + 1, true);
  // tail pass: per sub-group of each wavefront, the entry's blocks in LDS
  // (FP32: the effective-charge block; FP64: both)
  constexpr bool k64 = TAIL && sizeof(T) == 8, k32 = TAIL && sizeof(T) == 4;
  __shared__ __align__(16) T tl_cf64[k64 ? kAdjWaves : 1][4][k64 ? STR : 1];
  __shared__ __align__(16) T tl_ef64[k64 ? kAdjWaves : 1][4][k64 ? ESTR : 1];
  __shared__ __align__(16) T tl_ef32[k32 ? kAdjWaves : 1][4][k32 ? ESTR : 1];
  // tail pass: the block's wavefronts share out one group's list and add
  // their results through LDS in a fixed order
  __shared__ double tl_red[TAIL ? kAdjWaves : 1][TAIL ? 32 : 1][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t nw = TAIL ? kAdjWaves : 1, w0 = TAIL ? (uint32_t)wid : 0;
  const int A = __builtin_amdgcn_readfirstlane(G.cell[g]);
  const uint32_t first = __builtin_amdgcn_readfirstlane(C.first[A]);
  const uint32_t count = __builtin_amdgcn_readfirstlane(C.count[A]);
  const uint32_t tail0 = count - count % 64;
  const bool has_tail = count % 64 != 0 && count % 64 <= 32;
  if (TAIL && !has_tail) return;
  double cA[3];
  center_of(C.key[A], C.level[A], L, cA);
  const uint32_t off = G.off_m2p[g], cnt = G.cnt_m2p[g];
  const T* __restrict__ coef = (const T*)C.coef;
  for (uint32_t t0 = TAIL ? tail0 : 0; t0 < count; t0 += 64) {
    const uint32_t rem = count - t0;
    if (!TAIL && rem <= 32) break;
    const uint32_t split = !TAIL ? 1u : rem <= 16 ? 4u : 2u;  // wave-uniform
    const int width = 64 / (int)split;
    const uint32_t sub = (uint32_t)(lane / width);
    const int tl = lane % width;
    const uint32_t s = first + t0 + tl;
    const bool act = (uint32_t)tl < rem;
    const uint32_t ss = act ? s : first;
    const T tx = (T)(spos[ss] - cA[0]), ty = (T)(spos[n + ss] - cA[1]),
            tz = (T)(spos[2 * n + ss] - cA[2]);
    const T mk = srec[ss].w;
    const T4 ak = arec[ss];
    Acc<T> acc;
    acc.zero();
    T part[4] = {0, 0, 0, 0};
    // one (target, cell) term: the mass field and its derivative along gacc_k
    // (dual numbers), and the effective charges' potential and gradient
    auto term = [&](T Rx, T Ry, T Rz, const auto& cf, const auto& ef) {
      Dual<T> fm[4];
      T fe[4];
      m2p_eval_adj<P, T>(Rx, Ry, Rz, ak.x, ak.y, ak.z, eps2, as_src<T>(cf), as_src<T>(ef), fm, fe);
      part[0] += fm[0].d - ak.w * fm[0].v - mk * fe[0];
      part[1] += fm[1].d - ak.w * fm[1].v - mk * fe[1];
      part[2] += fm[2].d - ak.w * fm[2].v - mk * fe[2];
      part[3] -= fe[3];
    };
    if (!TAIL) {
      for (uint32_t q = 0; q < cnt; ++q) {
        T c[3];
        const int B = m2p_record<T>(list[off + q], C.walk, L, cA, c);
        term(tx - c[0], ty - c[1], tz - c[2], coef + (size_t)B * STR, ecoef + (size_t)B * ESTR);
        if ((q & 15) == 15) {
          acc.fold(part);
#pragma unroll
          for (int k = 0; k < 4; ++k) part[k] = (T)0;
        }
      }
    } else if constexpr (sizeof(T) == 4) {
      // FP32: each 16-lane row holds its sub-group's entry's mass-expansion
      // block spread over the row (row broadcasts feed it to its lanes); the
      // entry's effective-charge block goes to the sub-group's LDS slot and
      // is read from there.  The sub-group's next entry is loaded while this
      // one is evaluated.
      constexpr int NC = (STR + 15) / 16, NE = (ESTR + 15) / 16;
      const int rl = lane & 15;
      const uint32_t step = nw * split;
      T* eslot = &tl_ef32[wid][sub][0];
      const bool writer = (lane & (width - 1)) < 16;  // the sub-group's first row
      RowCoef<NC> cf;
      RowCoef<NE> ef;
      T c[3] = {0, 0, 0};
      uint32_t q = w0 * split + sub;
      if (q < cnt) {
        const int B = m2p_record<T>(list[off + q], C.walk, L, cA, c);
        cf.load(coef + (size_t)B * STR, STR, rl);
        ef.load(ecoef + (size_t)B * ESTR, ESTR, rl);
      }
      uint32_t it = 0;
      while (q < cnt) {
        if (writer)
#pragma unroll
          for (int j = 0; j < NE; ++j)
            if (rl + 16 * j < ESTR) eslot[rl + 16 * j] = ef.r[j];
        wave_sync();
        const uint32_t qn = q + step;
        RowCoef<NC> cf2;
        T c2[3] = {0, 0, 0};
        if (qn < cnt) {
          const int B = m2p_record<T>(list[off + qn], C.walk, L, cA, c2);
          cf2.load(coef + (size_t)B * STR, STR, rl);
          ef.load(ecoef + (size_t)B * ESTR, ESTR, rl);
        }
        term(tx - c[0], ty - c[1], tz - c[2], cf, (const T*)eslot);
        if ((++it & 15) == 0) {
          acc.fold(part);
#pragma unroll
          for (int k = 0; k < 4; ++k) part[k] = (T)0;
        }
        wave_sync();
        cf = cf2;
        c[0] = c2[0];
        c[1] = c2[1];
        c[2] = c2[2];
        q = qn;
      }
    } else {
      // FP64: both blocks through the sub-group's LDS slots (as the FP32
      // effective-charge block), the next entry loaded while this one is
      // evaluated
      constexpr int NC = (STR + 15) / 16, NE = (ESTR + 15) / 16;
      const int rl = lane & 15;
      const uint32_t step = nw * split;
      T* cslot = &tl_cf64[wid][sub][0];
      T* eslot = &tl_ef64[wid][sub][0];
      const bool writer = (lane & (width - 1)) < 16;
      RowBlock<T, NC> cf;
      RowBlock<T, NE> ef;
      T c[3] = {0, 0, 0};
      uint32_t q = w0 * split + sub;
      if (q < cnt) {
        const int B = m2p_record<T>(list[off + q], C.walk, L, cA, c);
        cf.load(coef + (size_t)B * STR, STR, rl);
        ef.load(ecoef + (size_t)B * ESTR, ESTR, rl);
      }
      uint32_t it = 0;
      while (q < cnt) {
        if (writer) {
          cf.store(cslot, STR, rl);
          ef.store(eslot, ESTR, rl);
        }
        wave_sync();
        const uint32_t qn = q + step;
        T c2[3] = {0, 0, 0};
        if (qn < cnt) {
          const int B = m2p_record<T>(list[off + qn], C.walk, L, cA, c2);
          cf.load(coef + (size_t)B * STR, STR, rl);
          ef.load(ecoef + (size_t)B * ESTR, ESTR, rl);
        }
        term(tx - c[0], ty - c[1], tz - c[2], (const T*)cslot, (const T*)eslot);
        if ((++it & 15) == 0) {
          acc.fold(part);
#pragma unroll
          for (int k = 0; k < 4; ++k) part[k] = (T)0;
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
        for (int k = 0; k < 4; ++k) tl_red[wid][tl][k] = v[k];
      __syncthreads();
      if (wid == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          v[k] = tl_red[0][tl < 32 ? tl : 0][k];
          for (int w = 1; w < kAdjWaves; ++w) v[k] += tl_red[w][tl < 32 ? tl : 0][k];
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

// ---------------------------------------------------------------- host side
hipError_t adj_gather_launch(bool fp32, const void* gacc, const void* gpot, size_t n,
                             const uint32_t* idx, void* arec, hipStream_t s) {
  unsigned g = (unsigned)((n + 255) / 256);
  if (fp32)
    k_adj_gather<float, float4><<<g, 256, 0, s>>>((const float*)gacc, (const float*)gpot, n, idx,
                                                  (float4*)arec);
  else
    k_adj_gather<double, double4><<<g, 256, 0, s>>>((const double*)gacc, (const double*)gpot, n,
                                                    idx, (double4*)arec);
  return hipGetLastError();
}

hipError_t adj_moments_level(bool fp32, int order, const Cells& C, const double* spos,
                             const void* arec, size_t n, uint32_t beg, uint32_t cnt, double* emom,
                             void* ecoef, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  unsigned g = (cnt + 127) / 128;
#define HOT_ADJM(P)                                                                          \
  case P:                                                                                    \
    if (fp32)                                                                                \
      k_adj_moments<P, float, float4><<<g, 128, 0, s>>>(C, spos, (const float4*)arec, n, beg, \
                                                        cnt, emom, (float*)ecoef);           \
    else                                                                                     \
      k_adj_moments<P, double, double4><<<g, 128, 0, s>>>(C, spos, (const double4*)arec, n,  \
                                                          beg, cnt, emom, (double*)ecoef);   \
    break;
  switch (order) {
    HOT_ADJM(0) HOT_ADJM(1) HOT_ADJM(2) HOT_ADJM(3) HOT_ADJM(4)
    default: return hipErrorInvalidValue;
  }
#undef HOT_ADJM
  return hipGetLastError();
}

template <typename T, typename T4>
static hipError_t p2p_adj_t(const Cells& C, const Groups& G, uint32_t ngroups, double L, T eps2,
                            const double* spos, const T4* srec, const T4* arec, size_t n,
                            const uint32_t* list, double4* out, hipStream_t s,
                            const SideStream& side) {
  const unsigned nb = (ngroups + kAdjWaves - 1) / kAdjWaves;
  hipStream_t st;
  hipError_t e = side_fork(side, s, &st);
  if (e != hipSuccess) return e;
  k_p2p_adj<T, T4, true><<<nb, 64 * kAdjWaves, 0, st>>>(C, G, ngroups, L, eps2, spos, srec, arec,
                                                        n, list, out);
  k_p2p_adj<T, T4, false><<<nb, 64 * kAdjWaves, 0, s>>>(C, G, ngroups, L, eps2, spos, srec, arec,
                                                         n, list, out);
  e = hipGetLastError();
  return e != hipSuccess ? e : side_join(side, s);
}

hipError_t p2p_adj_launch(bool fp32, const Cells& C, const Groups& G, uint32_t ngroups, double L,
                          double eps, const double* spos, const void* srec, const void* arec,
                          size_t n, const uint32_t* list, double4* out, hipStream_t s,
                          const SideStream& side) {
  if (ngroups == 0) return hipSuccess;
  if (fp32)
    return p2p_adj_t<float, float4>(C, G, ngroups, L, (float)(eps * eps), spos,
                                    (const float4*)srec, (const float4*)arec, n, list, out, s,
                                    side);
  return p2p_adj_t<double, double4>(C, G, ngroups, L, eps * eps, spos, (const double4*)srec,
                                    (const double4*)arec, n, list, out, s, side);
}

// Main passes one group per wavefront, tail passes one group per block; the
// tail pass goes on the side stream (as for the forward kernels).
template <int P, typename T, typename T4, bool TAIL>
__global__ void __launch_bounds__(64 * kAdjWaves) k_m2p_adj(Cells C, Groups G, uint32_t ngroups,
                                                            double L, T eps2,
                                                            const double* __restrict__ spos,
                                                            const T4* __restrict__ srec,
                                                            const T4* __restrict__ arec,
                                                            const T* __restrict__ ecoef, size_t n,
                                                            const uint4* __restrict__ list,
                                                            double4* __restrict__ out) {
  const int wid = threadIdx.x >> 6;
  const uint32_t g =
      __builtin_amdgcn_readfirstlane(TAIL ? xcd_block() : xcd_block() * kAdjWaves + wid);
  if (g >= ngroups) return;
  m2p_adj_group<P, T, T4, TAIL>(g, C, G, L, eps2, spos, srec, arec, ecoef, n, list, out);
}

template <int P, typename T, typename T4>
static hipError_t m2p_adj_t(const Cells& C, const Groups& G, uint32_t ngroups, double L, T eps2,
                            const double* spos, const T4* srec, const T4* arec, const T* ecoef,
                            size_t n, const uint4* list, double4* out, hipStream_t s,
                            const SideStream& side) {
  const unsigned nb = (ngroups + kAdjWaves - 1) / kAdjWaves;
  hipStream_t st;
  hipError_t e = side_fork(side, s, &st);
  if (e != hipSuccess) return e;
  k_m2p_adj<P, T, T4, true><<<ngroups, 64 * kAdjWaves, 0, st>>>(C, G, ngroups, L, eps2, spos,
                                                                 srec, arec, ecoef, n, list, out);
  k_m2p_adj<P, T, T4, false><<<nb, 64 * kAdjWaves, 0, s>>>(C, G, ngroups, L, eps2, spos, srec,
                                                            arec, ecoef, n, list, out);
  e = hipGetLastError();
  return e != hipSuccess ? e : side_join(side, s);
}

template <int P>
static hipError_t m2p_adj_p(bool fp32, const Cells& C, const Groups& G, uint32_t ngroups,
                            double L, double eps, const double* spos, const void* srec,
                            const void* arec, const void* ecoef, size_t n, const uint4* list,
                            double4* out, hipStream_t s, const SideStream& side) {
  if (fp32)
    return m2p_adj_t<P, float, float4>(C, G, ngroups, L, (float)(eps * eps), spos,
                                       (const float4*)srec, (const float4*)arec,
                                       (const float*)ecoef, n, list, out, s, side);
  return m2p_adj_t<P, double, double4>(C, G, ngroups, L, eps * eps, spos, (const double4*)srec,
                                       (const double4*)arec, (const double*)ecoef, n, list, out,
                                       s, side);
}

hipError_t m2p_adj_launch(bool fp32, int order, const Cells& C, const Groups& G, uint32_t ngroups,
                          double L, double eps, const double* spos, const void* srec,
                          const void* arec, const void* ecoef, size_t n, const uint4* list,
                          double4* out, hipStream_t s, const SideStream& side) {
  if (ngroups == 0) return hipSuccess;
  switch (order) {
#define HOT_MADJ(P) \
  case P:           \
    return m2p_adj_p<P>(fp32, C, G, ngroups, L, eps, spos, srec, arec, ecoef, n, list, out, s, side);
    HOT_MADJ(0) HOT_MADJ(1) HOT_MADJ(2) HOT_MADJ(3) HOT_MADJ(4)
#undef HOT_MADJ
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hot

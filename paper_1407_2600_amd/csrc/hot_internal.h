// Internal declarations of libhot (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/hot.h"

namespace hot {

constexpr int kMaxLevel = 21;        // 21 bits per axis in a 64-bit key
// support radius of the K1 softening kernel for the Plummer-equivalent
// softening eps (equal central potential: g(0) = 945/(256 h) = 1/eps)
inline double k1_radius(double eps) { return (945.0 / 256.0) * eps; }
constexpr int kMaxOrder = 4;         // cell multipole order built into the kernels
constexpr int kMaxRung = 16;         // block timesteps: steps down to dt / 2^16
constexpr int kMaxFarOrder = 12;     // far-field local expansion order
constexpr int kImgBits = 5;          // list entry = image << 27 | cell
constexpr uint32_t kCellMask = (1u << 27) - 1;
constexpr int kWalkStack = 2048;     // LDS walk stack entries per wave
constexpr int kWalkStackBig = 4096;  // fallback for groups with very many pending cells
constexpr int kSortBits = 9;
constexpr int kSortBins = 1 << kSortBits;
constexpr int kSortTile = 4096;      // keys per sort block
constexpr int kScanBlocks = 1024;    // blocks of the device-wide scan

// ---------------------------------------------------------------------------
// Compile-time multi-indices (a, b, c), ordered by total degree, then a
// descending, then b descending.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int nt(int D) { return D < 0 ? 0 : (D + 1) * (D + 2) * (D + 3) / 6; }
__host__ __device__ constexpr int nte(int d) { return d < 0 ? 0 : (d + 1) * (d + 2) / 2; }

__host__ __device__ constexpr int mi_index(int a, int b, int c) {
  int d = a + b + c;
  int off = 0;
  for (int x = d; x > a; --x) off += d - x + 1;
  off += (d - a) - b;
  return nt(d - 1) + off;
}

template <int D>
struct MI {
  static constexpr int N = nt(D);
  int a[N > 0 ? N : 1], b[N > 0 ? N : 1], c[N > 0 ? N : 1];
  constexpr MI() : a(), b(), c() {
    int n = 0;
    for (int d = 0; d <= D; ++d)
      for (int x = d; x >= 0; --x)
        for (int y = d - x; y >= 0; --y) {
          a[n] = x;
          b[n] = y;
          c[n] = d - x - y;
          ++n;
        }
  }
};

// Sizes of the per-cell multipole-interaction coefficient block for order P.
// The potential of a cell is written as Phi = rinv * sum_m rho^m P_m(R) with
// rinv = (R^2+eps^2)^(-1/2), rho = rinv^2 and P_m a polynomial whose
// homogeneous parts have degrees d = m - j, 0 <= j <= min(m, P - m).  Parts
// of degree d >= 1 are stored as their gradient coefficients (3 x nte(d-1)),
// parts of degree 0 as one constant.  For mass moments about the centre of
// mass the dipole part (m = 1, d = 1) vanishes and is not stored (DIP =
// false); the adjoint's effective charge distribution keeps it (DIP = true).
__host__ __device__ constexpr int part_jmax(int P, int m) { return m < P - m ? m : P - m; }
__host__ __device__ constexpr bool part_stored(int m, int d, bool dip = false) {
  return dip || !(m == 1 && d == 1);
}
__host__ __device__ constexpr int part_size(int d) { return d == 0 ? 1 : 3 * nte(d - 1); }
__host__ __device__ constexpr int coef_count(int P, bool dip = false) {
  int n = 0;
  for (int m = 0; m <= P; ++m)
    for (int j = 0; j <= part_jmax(P, m); ++j) {
      int d = m - j;
      if (part_stored(m, d, dip)) n += part_size(d);
    }
  return n;
}
// coefficient block padded to a multiple of 4 values (16-byte aligned rows)
__host__ __device__ constexpr int coef_stride(int P, bool dip = false) {
  return (coef_count(P, dip) + 3) / 4 * 4;
}

// Algorithmic flops of one multipole (cell, target) interaction in the
// formulation above, and of one direct pair (3 sub, 3 fma, rsqrt, 3 mul,
// 3 fma, 1 add; fma = 2, rsqrt = 1).
__host__ __device__ constexpr int m2p_flops(int P) {
  // R (3), u (3 fma = 6), rsqrt (1), rho (1)
  int f = 3 + 6 + 1 + 1;
  // monomials of degree 2..P-1 (one multiply each)
  for (int d = 2; d <= P - 1; ++d) f += nte(d);
  for (int m = 0; m <= P; ++m)
    for (int j = 0; j <= part_jmax(P, m); ++j) {
      int d = m - j;
      if (!part_stored(m, d) || d == 0) continue;
      f += 2 * 3 * nte(d - 1);  // gradient polynomial (fma)
      f += 2 * 3 + 1;           // R . V (3 fma) and the 1/d scale
      f += 3 + 1;               // add to V_m and to P_m
    }
  // Horner over m for Pv, Q (2 fma each) and Gv (3 fma), then combine
  f += P * (2 + 2 + 6) + 2 * P;
  f += 1 + 1 + 1 + 3 * 2 + 3;  // Phi, rho*Q, grad (3 fma), scale by rinv
  f += 4;                       // accumulate
  return f;
}
constexpr int kP2PFlops = 20;

// Algorithmic flops of the group-level local route (fma = 2), as the
// kernel formulates it: per local-list entry, the derivatives D_m,
// |m| <= P+Q, of the Newtonian kernel with at most two z indices (setup:
// |R|^2, its reciprocal square root and square, the scaled R_i and the
// per-degree factors; at most one z index by the recurrence, one
// multiply-add per nonzero m_i and per m_i >= 2 plus the combination; two z
// indices by the trace relation, one add) and the contraction
// S_n += Mt'_k D_(n+k) for the independent n (at most one z index),
// |n| <= Q, and the folded moments k (at most one z index, |k| <= P, no
// dipole); per sink, the value and gradient of the order-Q polynomial
// (4 fma per term) after the offset.  The folding itself is per cell.
__host__ __device__ constexpr int m2l_flops(int P, int Q) {
  const int N = P + Q;
  int f = 5 + 1 + 1 + 3 * N + 2 * N;
  for (int d = 1; d <= N; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        const int c = d - a - b;
        if (c >= 3) continue;
        if (c == 2) {
          f += 1;
          continue;
        }
        const int nz = (a > 0) + (b > 0) + (c > 0), n2 = (a > 1) + (b > 1);
        f += 2 * nz - 1;
        f += n2 > 0 ? 2 * n2 - 1 + 3 : 1;
      }
  int pairs = 0;
  for (int dn = 0; dn <= Q; ++dn)
    for (int dk = 0; dk <= P; ++dk) {
      if (dk == 1) continue;
      pairs += (2 * dn + 1) * (2 * dk + 1);
    }
  return f + 2 * pairs;
}
__host__ __device__ constexpr int l2p_flops(int Q) { return 3 + 8 * nt(Q); }

// Workgroups are dispatched round-robin over the chip's 8 XCDs, each with its
// own L2.  Kernels that give each wave one sink group renumber their blocks
// so that every XCD receives one contiguous range of block indices:
// neighbouring groups, which share most of their interaction lists, then
// read the same cells through the same L2.  A bijection on [0, gridDim.x).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_index(uint32_t b, uint32_t nb) {
  const uint32_t x = b % kXcds, i = b / kXcds;
  const uint32_t q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + i;
}
__device__ __forceinline__ uint32_t xcd_block() { return xcd_index(blockIdx.x, gridDim.x); }

// ---------------------------------------------------------------------------
// Device data of one force evaluation (pointers into the caller's workspace).
// ---------------------------------------------------------------------------
struct Cells {
  uint64_t* key;     // Morton key with placeholder bit
  int32_t* level;
  uint32_t* first;
  uint32_t* count;
  int32_t* child;    // index of the first child (children are contiguous)
  int32_t* nchild;   // 0 for a leaf
  int32_t* parent;
  double4* mmx;      // (m, sum m x, sum m y, sum m z), FP64
  double4* walk;     // (com.x, com.y, com.z, rcrit)
  double2* bnd;      // (sum m |x - com|^2, bound on max |x - com|)
  double4* bk;       // bounds on B_k = sum m |x - com|^k for k = 1, 3, 4, 5
  double* mom;       // raw moments about the com, nt(order) x cap (cell-major)
  void* coef;        // multipole coefficients, coef_stride x cap (cell-major), T
};

struct Groups {
  int32_t* cell;
  const uint8_t* active;  // nullptr: every group; else only groups with active[g] != 0
                          // get lists and forces (block timesteps: the groups holding a
                          // particle whose step ends now)
  double* lo;        // 3 x cap
  double* hi;        // 3 x cap
  uint32_t* cnt_p2p;
  uint32_t* cnt_m2p;
  uint32_t* off_p2p;
  uint32_t* off_m2p;
  uint32_t* cnt_m2l;  // cells taken through the group's local expansion
  uint32_t* off_m2l;  // end of the group's accepted-cell region (16-byte records):
                      // its local entries are the cnt_m2l words before it
};

// Group-level local expansions (Newtonian kernel): an accepted cell goes to
// the group's local list when the truncation bound of the order-q local
// expansion about the group's centre, G m t^q ((q+2) - (q+1) t) /
// (u^2 (1-t)^2) with u = |c - z| - b and t = a/u, plus the softening change
// 1.5 G m eps2 / (u - a)^4, is at most tol (q = 0: never).
struct LocalPrm {
  int q;
  double tol;
  double G;
  double eps2;  // Plummer softening squared (0 for the K1 kernel)
};

// A dispatch holds fewer than 2^32 work-items, so kernels that give each sink
// group a wavefront (or a block) run on at most kGroupBatch groups per launch
// (the group arrays taken from the batch's first group on; the box arrays
// keep their stride).
constexpr uint32_t kGroupBatch = 1u << 22;
// groups per block of the list-chunk planning sums (a multiple of 256)
constexpr uint32_t kCountBlock = 1024;

inline Groups groups_from(const Groups& G, uint32_t g0) {
  Groups B = G;
  B.cell += g0;
  B.lo += g0;
  B.hi += g0;
  B.cnt_p2p += g0;
  B.cnt_m2p += g0;
  B.off_p2p += g0;
  B.off_m2p += g0;
  B.cnt_m2l += g0;
  B.off_m2l += g0;
  if (B.active) B.active += g0;
  return B;
}

// f(groups of the batch, their number) for consecutive batches of at most
// batch groups
template <typename F>
inline hipError_t for_group_batches(const Groups& G, uint32_t ng, uint32_t batch, F&& f) {
  for (uint32_t g0 = 0; g0 < ng; g0 += batch) {
    const uint32_t nb = ng - g0 < batch ? ng - g0 : batch;
    const hipError_t e = f(groups_from(G, g0), nb);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// list chunks whose stages are timed one by one (beyond, only the chunk
// loop as a whole is timed)
constexpr int kChunkEvents = 64;

struct Plan {
  size_t n;
  size_t cap_cells;
  size_t cap_groups;
  size_t cap_list;   // list region in 4-byte words
  size_t total;      // preferred bytes: every region, lists at their hinted size
  size_t min_total;  // smallest workspace for the call the plan was made for
  // offsets of every buffer (bytes from the workspace start)
  size_t o_key[2], o_idx[2], o_spos, o_smass, o_srec, o_acc, o_tmp;
  size_t o_scan, o_hist, o_ctr;
  size_t o_c_key, o_c_level, o_c_first, o_c_count, o_c_child, o_c_nchild, o_c_parent;
  size_t o_c_mmx, o_c_walk, o_c_bnd, o_c_bk, o_c_mom, o_c_coef, o_c_mloc;
  size_t hcap, o_h_key, o_h_val;  // key -> cell hash (slots, key and value arrays)
  size_t o_g_cell, o_g_lo, o_g_hi, o_g_cp, o_g_cm, o_g_op, o_g_om, o_g_cl, o_g_ol, o_g_act;
  size_t o_far_part, o_far_mom, o_far_lam;
  size_t o_arec, o_adj, o_c_emom, o_c_ecoef, o_far_mbar;
  size_t o_kv_g, o_kv_x, o_kv_m;  // reverse leapfrog sweep: gacc, xbar and mbar of one step
  size_t o_kv_sx, o_kv_sv;        // snapshots of the in/out arrays of hot_kdk and hot_kdk_vjp
  size_t o_list;
};

}  // namespace hot

// the context (opaque to callers)
namespace hot {
// A second stream of the context on which the force kernels' tail passes run
// beside their main passes (forked from and joined back to the caller's
// stream with two events).  Absent (null stream) if it could not be created;
// then the passes run one after the other on the caller's stream.
struct SideStream {
  hipStream_t st;
  hipEvent_t fork, join;
};

// the stream the tail pass goes on: the side stream, after it has waited for
// the work already queued on s (or s itself without a side stream)
inline hipError_t side_fork(const SideStream& side, hipStream_t s, hipStream_t* out) {
  *out = s;
  if (!side.st) return hipSuccess;
  hipError_t e = hipEventRecord(side.fork, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(side.st, side.fork, 0);
  if (e == hipSuccess) *out = side.st;
  return e;
}

// s waits for the tail pass queued on the side stream
inline hipError_t side_join(const SideStream& side, hipStream_t s) {
  if (!side.st) return hipSuccess;
  hipError_t e = hipEventRecord(side.join, side.st);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, side.join, 0);
  return e;
}
}  // namespace hot

struct hot_ctx {
  hot_params p;
  int device;
  double S;            // 2^21 / L (key quantisation)
  double* d_tpsi;      // 27 Ewald tables (octant-centre offsets), nt(2 far_order) each
  int n_tpsi;
  // learned capacities (grow after an overflow)
  double cells_per_particle;
  double list_per_particle;
  // last call
  hot_stats stats;
  size_t last_n;
  int have_last;
  hipStream_t last_stream;
  hot::Plan last_plan;
  void* last_ws;
  uint32_t last_ncells;
  uint32_t last_ngroups;
  size_t last_accepted;  // accepted cells of the last evaluation (multipole + local)
  uint32_t* host_buf;  // pinned host memory for counter read-backs
  int last_chunks;     // list chunks of the last evaluation
  int last_cev;        // chunks timed one by one in the last evaluation (0: none)
  // the tree and lists the workspace holds (hot_vjp_after_forces)
  struct TreeRecord {
    int valid;
    const double* pos;
    const void* mass;
    size_t n, ws_bytes, words, o_list, cap_cells;
    void* ws;
    hipStream_t stream;
    uint32_t lvl[hot::kMaxLevel + 3];
    int nlev;
    uint32_t ncells, ngroups;
    size_t tp, tm;
  } tree;
  hipEvent_t ev[8];
  int events_ok;
  // sink groups per launch of the per-group kernels (kGroupBatch; smaller
  // only when the environment variable HOT_GROUP_BATCH asks for it, which
  // the tests use to check that batched launches give identical results)
  uint32_t group_batch;
  // per-chunk timing events when the lists are processed in chunks: chunk k
  // records cev[4k] before its walk emit pass, cev[4k+1] before its direct
  // kernel, cev[4k+2] before its local expansions, cev[4k+3] before its
  // multipole kernel and cev[4k+4] after it
  hipEvent_t cev[4 * hot::kChunkEvents + 1];
  int cev_ok;
  hot::SideStream side;
};

namespace hot {
// host-side Ewald remainder table (ewald_table.cpp)
void psi_taylor_table(int D, double box, const double r0[3], double* out);
// the 27 tables about the offsets between octant centres (cubic symmetry)
void psi_taylor_tables27(int D, double box, double* out);
// the same with an explicit Ewald split (alpha, real images |n|_inf <= nreal,
// reciprocal |k|_inf <= kmax)
void psi_taylor_table_split(int D, double box, const double r0[3], double alpha, int nreal,
                            int kmax, double* out);

void set_error(const std::string& msg);
hot_status device_error(hipError_t e, const char* what);

// device-wide exclusive scan of n uint32 values (n may live on the device);
// out[i] = sum_{k<i} in[i]; *total = sum.  in and out may alias.
hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint32_t* total, size_t n,
                    uint32_t* block_sums, hipStream_t s);
}  // namespace hot

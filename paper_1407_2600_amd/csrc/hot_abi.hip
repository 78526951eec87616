// C ABI of libhot: parameter checks, workspace plan, and the sequence of
// stages of one force evaluation (keys, sort, tree, moments, groups, walk,
// interactions, far field).  See include/hot.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hot_internal.h"

namespace hot {
// stage launchers (other translation units)
hipError_t launch_keys(const double* pos, size_t n, double L, double S, uint64_t* key,
                       uint32_t* idx, uint32_t* bad, hipStream_t s);
hipError_t radix_sort(uint64_t* key_in, uint32_t* idx_in, uint64_t* key_out, uint32_t* idx_out,
                      size_t n, uint32_t* hist, uint32_t* scan_tmp, hipStream_t s);
hipError_t launch_gather(const double* pos, const void* mass, bool fp32, size_t n, double L,
                         const uint32_t* idx, double* spos, double* smass, uint32_t* bad,
                         hipStream_t s);
hipError_t tree_root(const Cells& C, uint32_t n, hipStream_t s);
hipError_t tree_split_level(const Cells& C, const uint64_t* skey, uint32_t beg, uint32_t cnt,
                            int level, int leaf_max, uint32_t* nch, uint32_t* total,
                            uint32_t* scan_tmp, hipStream_t s);
hipError_t tree_emit_level(const Cells& C, const uint64_t* skey, uint32_t beg, uint32_t cnt,
                           int level, int leaf_max, const uint32_t* choff, uint32_t next,
                           uint32_t cap, hipStream_t s);
hipError_t tree_hash_build(const Cells& C, uint32_t ncells, uint64_t* hkey, uint32_t* hval,
                           size_t hcap, hipStream_t s);
hipError_t hash_lookup(const uint64_t* hkey, const uint32_t* hval, size_t hcap, const uint64_t* q,
                       size_t nq, int32_t* out, hipStream_t s);
hipError_t tree_moments_level(const Cells& C, const double* spos, const double* smass, size_t n,
                              uint32_t beg, uint32_t cnt, double L, double theta, double G,
                              double err_tol, double k1h, int order,
                              bool fp32, hipStream_t s);
hipError_t tree_groups(const Cells& C, uint32_t ncells, int gmax, size_t n, uint32_t* gflag,
                       uint32_t* gid, int32_t* gcell_at, const Groups& G, uint32_t* ngroups_dev,
                       uint32_t* scan_tmp, hipStream_t s);
hipError_t tree_group_bbox(const Cells& C, const Groups& G, uint32_t ngroups, uint32_t gcap,
                           const double* spos, size_t n, hipStream_t s);
hipError_t tree_srec(const Cells& C, uint32_t ncells, const double* spos, const double* smass,
                     size_t n, double L, int leaf_max, void* srec, bool fp32, hipStream_t s);
hipError_t walk_launch(bool emit, bool big, const Cells& C, const Groups& G, uint32_t ngroups,
                       uint32_t gcap, double L, int periodic, const LocalPrm& lp,
                       uint32_t* p2p_list, uint4* m2p_list, uint32_t* status, hipStream_t s);
hipError_t local_moments_launch(bool fp32, int order, const double* mom, uint32_t ncells,
                                void* mt, hipStream_t s);
hipError_t local_launch(bool fp32, int order, int q, const Cells& C, const Groups& G,
                        uint32_t ngroups, uint32_t gcap, double L, const double* spos, size_t n,
                        const uint32_t* list, const void* mt, double4* out, hipStream_t s);
hipError_t sum_counts(const Groups& G, uint32_t ngroups, unsigned long long* sums, uint32_t* maxw,
                      hipStream_t s);
hipError_t block_counts(const Groups& G, uint32_t ngroups, unsigned long long* bp,
                        unsigned long long* bm, hipStream_t s);
hipError_t count_pairs(const Cells& C, const Groups& G, uint32_t ngroups, bool local,
                       const uint32_t* p2p_list, unsigned long long* out,
                       unsigned long long* slots, hipStream_t s);
hipError_t p2p_launch(bool fp32, int kernel, const Cells& C, const Groups& G, uint32_t ngroups,
                      double L, double eps, const double* spos, const void* srec, size_t n,
                      const uint32_t* list, double4* out, hipStream_t s, const SideStream& side);
hipError_t m2p_launch(bool fp32, int order, const Cells& C, const Groups& G, uint32_t ngroups,
                      double L, double eps, const double* spos, size_t n, const uint4* list,
                      double4* out, hipStream_t s, const SideStream& side);
hipError_t far_launch(int far_order, const double* spos, const double* smass,
                      const uint64_t* skey, const double4* near, size_t n, const uint32_t* idx,
                      double box, double G, const double* tpsi, double* part, int nblk_max,
                      double* mroot, double* lam, int periodic, const uint8_t* rung, int rmin,
                      bool fp32, void* acc, void* pot, hipStream_t s);
hipError_t kick_rung_launch(bool fp32, void* vel, const void* acc, const uint8_t* rung, size_t n,
                            int rmin, double dt, hipStream_t s);
hipError_t rung_assign_launch(bool fp32, const void* acc, uint8_t* rung, size_t n, int rmin,
                              double dt, int max_rung, double eta, double eps, hipStream_t s);
hipError_t group_active_launch(const Cells& C, const Groups& G, uint32_t ngroups,
                               const uint32_t* idx, const uint8_t* rung, int rmin, uint8_t* act,
                               hipStream_t s);
hipError_t rung_max_launch(const uint8_t* rung, size_t n, uint32_t* out, hipStream_t s);
hipError_t far_prepare_launch(int far_order, const double* spos, const double* smass,
                              const uint64_t* skey, size_t n, double box, const double* tpsi,
                              double* part, int nblk_max, double* mom, double* lam,
                              hipStream_t s);
hipError_t adj_gather_launch(bool fp32, const void* gacc, const void* gpot, size_t n,
                             const uint32_t* idx, void* arec, hipStream_t s);
hipError_t adj_moments_level(bool fp32, int order, const Cells& C, const double* spos,
                             const void* arec, size_t n, uint32_t beg, uint32_t cnt, double* emom,
                             void* ecoef, hipStream_t s);
hipError_t p2p_adj_launch(bool fp32, const Cells& C, const Groups& G, uint32_t ngroups, double L,
                          double eps, const double* spos, const void* srec, const void* arec,
                          size_t n, const uint32_t* list, double4* out, hipStream_t s,
                          const SideStream& side);
hipError_t m2p_adj_launch(bool fp32, int order, const Cells& C, const Groups& G, uint32_t ngroups,
                          double L, double eps, const double* spos, const void* srec,
                          const void* arec, const void* ecoef, size_t n, const uint4* list,
                          double4* out, hipStream_t s, const SideStream& side);
hipError_t far_adj_launch(int far_order, const double* spos, const double* smass,
                          const uint64_t* skey, const void* arec, const double4* near, size_t n,
                          const uint32_t* idx, double box, double G, const double* tpsi,
                          double* part, int nblk_max, const double* lam, double* lb, double* mbar,
                          int periodic, bool fp32, double* xbar, void* mbar_out, hipStream_t s);
hipError_t kick_launch(bool fp32, void* vel, const void* acc, size_t n, double h, hipStream_t s);
hipError_t kdk_adj_drift_launch(bool fp32, void* vbar, const double* xbar, void* gacc, size_t n,
                                double dt, double c, bool drift, hipStream_t s);
hipError_t kdk_adj_accum_launch(bool fp32, double* xbar, const double* tx, void* mbar,
                                const void* tm, size_t n, bool first, hipStream_t s);
hipError_t zero_launch(void* p, size_t bytes, hipStream_t s);
hipError_t drift_launch(bool fp32, double* pos, const void* vel, size_t n, double dt, double L,
                        hipStream_t s);

// Device scratch of hot_forces_noalloc: one array per GPU the library runs on
// (allocated when the code object is loaded there, held until the process
// ends).  Host code uses it only through the device address that
// hipGetSymbolAddress returns for the current device (scratch_ptr below).
constexpr size_t kNoAllocBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
thread_local std::string g_err;

// per-device address of `scratch`, resolved once per device at context
// creation (with that device current)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
bool g_scratch_done[kMaxDevices];

void resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_done[dev]) return;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[dev] = e;
  g_scratch_ptr[dev] = (e == hipSuccess) ? p : nullptr;
  g_scratch_done[dev] = true;
  if (e != hipSuccess) (void)hipGetLastError();
}
constexpr int kFarBlocks = 64;  // far-moment blocks per octant
constexpr size_t kAlign = 256;

size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// words of the context's pinned host buffer (kHostWords uint32) that receive
// the pair counters (two u64) and the multipole lane-step and local-route
// counters (six u64) at the end of every evaluation
constexpr int kHostPairs = 56;
constexpr int kHostSlots = 64;
constexpr int kHostWords = 128;
// counters in the workspace (uint32 unless noted)
enum { CTR_BAD = 0, CTR_TOTAL = 1, CTR_NGROUPS = 2, CTR_TP = 3, CTR_TM = 4, CTR_STATUS = 5,
       CTR_PAIRS = 8 /* two u64 at 8..11 */, CTR_SUMS = 12 /* two u64 at 12..15 */,
       CTR_MAXW = 18, CTR_READ = 20, CTR_SLOTS = 24 /* six u64 at 24..35 */,
       CTR_RMAX = 60 /* block timesteps: largest rung */,
       CTR_N = 64 };
// largest list region requested for one evaluation (4-byte words); larger
// list sets are processed in chunks of consecutive groups
constexpr size_t kListMaxWords = size_t(1) << 30;
// smallest list region accepted (bytes)
constexpr size_t kListMinBytes = size_t(1) << 20;
// workspace regions a call needs beyond the forward ones
constexpr unsigned kNeedAdjoint = 1, kNeedSnapshot = 2, kNeedReverse = 4;

// the group-level local route is in use
bool local_on(const hot_params& p) { return p.local_order > 0 && p.local_tol > 0.0; }

bool valid_params(const hot_params* p, std::string* why) {
  if (!(p->box > 0.0) || !std::isfinite(p->box)) return *why = "box must be finite and > 0", false;
  if (!std::isfinite(p->G)) return *why = "G must be finite", false;
  if (!(p->eps >= 0.0) || !std::isfinite(p->eps)) return *why = "eps must be >= 0", false;
  if (!(p->theta >= 0.0 && p->theta < 1.0)) return *why = "theta must be in [0, 1)", false;
  if (!(p->err_tol >= 0.0 && std::isfinite(p->err_tol)))
    return *why = "err_tol must be finite and >= 0", false;
  if (p->order < 0 || p->order > kMaxOrder) return *why = "order must be in 0..4", false;
  if (p->periodic != 0 && p->periodic != 1) return *why = "periodic must be 0 or 1", false;
  if (p->leaf_max < 1 || p->leaf_max > 255) return *why = "leaf_max must be in 1..255", false;
  if (p->group_max < 1 || p->group_max > 4096) return *why = "group_max must be in 1..4096", false;
  if (p->far_order < 0 || p->far_order > kMaxFarOrder)
    return *why = "far_order must be in 0..12", false;
  if (p->precision != HOT_FP64 && p->precision != HOT_FP32)
    return *why = "precision must be HOT_FP64 or HOT_FP32", false;
  if (p->kernel != HOT_KERNEL_PLUMMER && p->kernel != HOT_KERNEL_K1)
    return *why = "kernel must be HOT_KERNEL_PLUMMER or HOT_KERNEL_K1", false;
  if (p->kernel == HOT_KERNEL_K1 && !(p->eps > 0.0))
    return *why = "the K1 kernel needs eps > 0", false;
  if (p->local_order != 0 && p->local_order != 2 && p->local_order != 4)
    return *why = "local_order must be 0, 2 or 4", false;
  if (!(p->local_tol >= 0.0 && std::isfinite(p->local_tol)))
    return *why = "local_tol must be finite and >= 0", false;
  return true;
}

Plan make_plan(const hot_ctx* c, size_t n, size_t ws_bytes, unsigned need) {
  Plan P{};
  P.n = n;
  const bool fp32 = c->p.precision == HOT_FP32;
  const size_t tsz = fp32 ? 4 : 8;
  P.cap_cells = (size_t)std::ceil(c->cells_per_particle * (double)n) + 1024;
  P.cap_groups = std::min(P.cap_cells, n + 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += up(bytes);
    return r;
  };
  P.o_key[0] = take(8 * n);
  P.o_key[1] = take(8 * n);
  P.o_idx[0] = take(4 * n);
  P.o_idx[1] = take(4 * n);
  P.o_spos = take(24 * n);
  P.o_smass = take(8 * n);
  P.o_srec = take(4 * tsz * n);
  P.o_acc = take(32 * n);
  P.o_tmp = take(4 * std::max(n, P.cap_cells));  // split-level counts / group ids
  P.o_scan = take(4 * (kScanBlocks + 64));
  const size_t nblk_sort = (n + kSortTile - 1) / kSortTile;
  P.o_hist = take(4 * kSortBins * std::max<size_t>(nblk_sort, 1));
  P.o_ctr = take(4 * CTR_N);
  const size_t C = P.cap_cells;
  const int NM = nt(c->p.order);
  const int STR = coef_stride(c->p.order);
  P.o_c_key = take(8 * C);
  P.o_c_level = take(4 * C);
  P.o_c_first = take(4 * C);
  P.o_c_count = take(4 * C);
  P.o_c_child = take(4 * C);
  P.o_c_nchild = take(4 * C);
  P.o_c_parent = take(4 * C);
  P.o_c_mmx = take(32 * C);
  P.o_c_walk = take(32 * C);
  P.o_c_bnd = take(16 * C);
  P.o_c_bk = take(32 * C);
  P.o_c_mom = take(8 * (size_t)NM * C);
  P.o_c_coef = take(tsz * (size_t)STR * C);
  // key -> cell hash: a power of two of slots, at least twice the cells
  P.hcap = 1024;
  while (P.hcap < 2 * C) P.hcap <<= 1;
  P.o_h_key = take(8 * P.hcap);
  P.o_h_val = take(4 * P.hcap);
  const size_t Gc = P.cap_groups;
  P.o_g_cell = take(4 * Gc);
  P.o_g_lo = take(24 * Gc);
  P.o_g_hi = take(24 * Gc);
  P.o_g_cp = take(4 * Gc);
  P.o_g_cm = take(4 * Gc);
  P.o_g_op = take(4 * Gc);
  P.o_g_om = take(4 * Gc);
  P.o_g_cl = take(4 * Gc);
  P.o_g_ol = take(4 * Gc);
  P.o_g_act = take(Gc);
  // local route: the cells' moments scaled for it
  P.o_c_mloc = local_on(c->p) ? take(tsz * (size_t)NM * C) : 0;
  const int NQ = nt(c->p.far_order);
  P.o_far_part = take(8 * 8 * (size_t)NQ * kFarBlocks);
  P.o_far_mom = take(8 * 8 * (size_t)NQ);
  P.o_far_lam = take(8 * 8 * (size_t)NQ);
  // ---- list region, then the regions only some calls use, carved from the
  // top of the workspace so that a forward-only caller need not provide them
  P.o_list = o;
  const size_t want_list =
      std::max(std::min((size_t)std::ceil(c->list_per_particle * (double)n) + 65536, kListMaxWords),
               kListMinBytes / 4);
  const size_t C2 = P.cap_cells;
  // adjoint: sorted cotangents, per-particle results, cotangent moments
  // (charges order p, gacc-derived order p+1) and coefficients, far-field
  // adjoint moments
  const size_t sz_arec = up(4 * tsz * n), sz_adj = up(32 * n);
  const size_t sz_emom = up(8 * (size_t)(nt(c->p.order + 1) + nt(c->p.order)) * C2);
  const size_t sz_ecoef = up(tsz * (size_t)coef_stride(c->p.order + 1, true) * C2);
  const size_t sz_fmbar = up(8 * 8 * (size_t)NQ);
  const size_t bytes_a = sz_arec + sz_adj + sz_emom + sz_ecoef + sz_fmbar;
  // leapfrog: the in/out snapshots, and the reverse sweep's scratch
  const size_t sz_sx = up(24 * n), sz_sv = up(3 * tsz * n);
  const size_t sz_g = up(3 * tsz * n), sz_x = up(24 * n), sz_m = up(tsz * n);
  const size_t bytes_s = sz_sx + sz_sv, bytes_r = sz_g + sz_x + sz_m;
  P.total = o + up(4 * want_list) + bytes_a + bytes_s + bytes_r;
  const size_t top = ((need & kNeedAdjoint) ? bytes_a : 0) +
                     ((need & kNeedSnapshot) ? bytes_s : 0) +
                     ((need & kNeedReverse) ? bytes_r : 0);
  P.min_total = o + kListMinBytes + top;
  size_t t = ws_bytes == 0 ? P.total : (ws_bytes & ~size_t(255));
  if (t < o + top) t = o + top;  // (the caller's size is checked against min_total)
  if (need & kNeedSnapshot) {
    P.o_kv_sv = (t -= sz_sv);
    P.o_kv_sx = (t -= sz_sx);
  }
  if (need & kNeedReverse) {
    P.o_kv_m = (t -= sz_m);
    P.o_kv_x = (t -= sz_x);
    P.o_kv_g = (t -= sz_g);
  }
  if (need & kNeedAdjoint) {
    P.o_far_mbar = (t -= sz_fmbar);
    P.o_c_ecoef = (t -= sz_ecoef);
    P.o_c_emom = (t -= sz_emom);
    P.o_adj = (t -= sz_adj);
    P.o_arec = (t -= sz_arec);
  }
  P.cap_list = ws_bytes == 0 ? want_list : (t - o) / 4;
  return P;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

Cells cells_of(void* ws, const Plan& P) {
  Cells C;
  C.key = at<uint64_t>(ws, P.o_c_key);
  C.level = at<int32_t>(ws, P.o_c_level);
  C.first = at<uint32_t>(ws, P.o_c_first);
  C.count = at<uint32_t>(ws, P.o_c_count);
  C.child = at<int32_t>(ws, P.o_c_child);
  C.nchild = at<int32_t>(ws, P.o_c_nchild);
  C.parent = at<int32_t>(ws, P.o_c_parent);
  C.mmx = at<double4>(ws, P.o_c_mmx);
  C.walk = at<double4>(ws, P.o_c_walk);
  C.bnd = at<double2>(ws, P.o_c_bnd);
  C.bk = at<double4>(ws, P.o_c_bk);
  C.mom = at<double>(ws, P.o_c_mom);
  C.coef = at<void>(ws, P.o_c_coef);
  return C;
}

Groups groups_of(void* ws, const Plan& P) {
  Groups G;
  G.cell = at<int32_t>(ws, P.o_g_cell);
  G.lo = at<double>(ws, P.o_g_lo);
  G.hi = at<double>(ws, P.o_g_hi);
  G.cnt_p2p = at<uint32_t>(ws, P.o_g_cp);
  G.cnt_m2p = at<uint32_t>(ws, P.o_g_cm);
  G.off_p2p = at<uint32_t>(ws, P.o_g_op);
  G.off_m2p = at<uint32_t>(ws, P.o_g_om);
  G.cnt_m2l = at<uint32_t>(ws, P.o_g_cl);
  G.off_m2l = at<uint32_t>(ws, P.o_g_ol);
  G.active = nullptr;
  return G;
}

#define HOT_CHECK(call, what)                           \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return device_error(e_, what); \
  } while (0)

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

hot_status device_error(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return HOT_EDEVICE;
}

// read back a few counters (synchronises the stream)
static hipError_t readback(hipStream_t s, const uint32_t* dev, uint32_t* host, int count) {
  hipError_t e = hipMemcpyAsync(host, dev, sizeof(uint32_t) * count, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// adjoint inputs/outputs (hot_vjp); NULL for a force evaluation
struct VjpArgs {
  const void* gacc;
  const void* gpot;
  double* xbar;
  void* mbar;
};

// need: the optional workspace regions of the calling entry point (the
// layout must be the same for every evaluation within one call)
// after_forces: an adjoint may use the tree and lists the workspace holds
// from the context's last evaluation (hot_vjp_after_forces)
// rung, rmin: block timesteps, forces only for the particles with
// rung[i] >= rmin (their groups get lists; the others' acc and pot are left
// as they are); nullptr: every particle
static hot_status forces_impl(hot_ctx* c, size_t n, const double* pos, const void* mass, void* acc,
                              void* pot, void* ws, size_t ws_bytes, hipStream_t s, unsigned need,
                              const VjpArgs* vjp = nullptr, bool after_forces = false,
                              const uint8_t* rung = nullptr, int rmin = 0) {
  const hot_params& p = c->p;
  const bool fp32 = p.precision == HOT_FP32;
  Plan P = make_plan(c, n, ws_bytes, need);
  if (ws_bytes < P.min_total) {
    g_err = "workspace too small: need at least " + std::to_string(P.min_total) +
            " bytes (" + std::to_string(P.total) + " preferred), got " + std::to_string(ws_bytes);
    c->stats.ws_bytes_needed = P.total;
    return HOT_ENOMEM;
  }
  if (P.cap_cells >= (size_t)kCellMask) {
    g_err = "too many cells for 27-bit list entries";
    return HOT_EUNSUPPORTED;
  }
  uint32_t* ctr = at<uint32_t>(ws, P.o_ctr);
  uint32_t* scan_tmp = at<uint32_t>(ws, P.o_scan);
  uint64_t* key0 = at<uint64_t>(ws, P.o_key[0]);
  uint64_t* key1 = at<uint64_t>(ws, P.o_key[1]);
  uint32_t* idx0 = at<uint32_t>(ws, P.o_idx[0]);
  uint32_t* idx1 = at<uint32_t>(ws, P.o_idx[1]);
  double* spos = at<double>(ws, P.o_spos);
  double* smass = at<double>(ws, P.o_smass);
  void* srec = at<void>(ws, P.o_srec);
  double4* near = at<double4>(ws, P.o_acc);
  uint32_t* tmp = at<uint32_t>(ws, P.o_tmp);
  Cells C = cells_of(ws, P);
  Groups G = groups_of(ws, P);
  uint32_t* host = c->host_buf;

  const hot_ctx::TreeRecord& R = c->tree;
  const bool use_tree = after_forces && vjp && R.valid && R.pos == pos && R.mass == mass &&
                        R.n == n && R.ws == ws && R.ws_bytes == ws_bytes && R.stream == s &&
                        R.o_list == P.o_list && R.cap_cells == P.cap_cells &&
                        R.words <= P.cap_list;
  c->tree.valid = 0;  // this call writes the workspace; recorded again at the end
  std::vector<uint32_t> lvl(kMaxLevel + 3, 0);
  int nlev = 1;
  uint32_t ncells = 0, ngroups = 0;
  bool big = false;
  // tm counts the accepted cells, multipole and local entries together (the
  // walk's count pass does not split them; its emit pass does), with room for
  // a 16-byte record each
  size_t tp = 0, tm = 0;
  struct Chunk {
    uint32_t g0, g1;
    size_t tp, tm;
  };
  const bool local = local_on(p);
  const LocalPrm lp{local ? p.local_order : 0, local ? p.local_tol : 0.0, p.G,
                    p.kernel == HOT_KERNEL_K1 ? 0.0 : p.eps * p.eps};
  std::vector<Chunk> chunks;

  if (c->events_ok) HOT_CHECK(hipEventRecord(c->ev[0], s), "event");
  if (use_tree) {
    // keys, order, cells, groups and lists as the recorded evaluation left them
    std::copy(R.lvl, R.lvl + kMaxLevel + 3, lvl.begin());
    nlev = R.nlev;
    ncells = R.ncells;
    ngroups = R.ngroups;
    tp = R.tp;
    tm = R.tm;
    chunks.push_back({0, ngroups, tp, tm});
    if (c->events_ok) HOT_CHECK(hipEventRecord(c->ev[1], s), "event");
    if (c->events_ok) HOT_CHECK(hipEventRecord(c->ev[2], s), "event");
  } else {
  HOT_CHECK(zero_launch(ctr, 4 * CTR_N, s), "clear counters");
  // keys into the second buffer pair; the sort leaves them in the first
  HOT_CHECK(launch_keys(pos, n, p.box, c->S, key1, idx1, ctr + CTR_BAD, s), "keys");
  HOT_CHECK(radix_sort(key1, idx1, key0, idx0, n, at<uint32_t>(ws, P.o_hist), scan_tmp, s),
            "sort");
  HOT_CHECK(launch_gather(pos, mass, fp32, n, p.box, idx0, spos, smass, ctr + CTR_BAD, s),
            "gather");
  if (c->events_ok) HOT_CHECK(hipEventRecord(c->ev[1], s), "event");

  // ---- tree, level by level
  HOT_CHECK(tree_root(C, (uint32_t)n, s), "tree root");
  lvl[0] = 0;
  lvl[1] = 1;
  for (int l = 0; l < kMaxLevel; ++l) {
    const uint32_t cnt = lvl[l + 1] - lvl[l];
    HOT_CHECK(tree_split_level(C, key0, lvl[l], cnt, l, p.leaf_max, tmp, ctr + CTR_TOTAL,
                               scan_tmp, s),
              "tree split");
    // the emit pass goes ahead of the read-back (it writes nothing beyond the
    // cell capacity; an overflow fails the call below)
    HOT_CHECK(tree_emit_level(C, key0, lvl[l], cnt, l, p.leaf_max, tmp, lvl[l + 1],
                              (uint32_t)std::min(P.cap_cells, (size_t)UINT32_MAX), s),
              "tree emit");
    HOT_CHECK(readback(s, ctr, host, 2), "readback");
    if (l == 0 && host[CTR_BAD]) {
      g_err = (host[CTR_BAD] & 1u) ? "positions must be finite and inside (-L, 2L)"
                                   : "masses must be finite and >= 0";
      return HOT_EINVAL;
    }
    const uint32_t tot = host[CTR_TOTAL];
    if (tot == 0) break;
    if ((size_t)lvl[l + 1] + tot > P.cap_cells) {
      c->cells_per_particle = std::min(2.0 * c->cells_per_particle,
                                       (double)(kCellMask - 4096) / (double)n);
      c->stats.ws_bytes_needed = make_plan(c, n, 0, need).total;
      g_err = "cell capacity exceeded; call hot_workspace_size again and retry";
      return HOT_EOVERFLOW;
    }
    lvl[l + 2] = lvl[l + 1] + tot;
    nlev = l + 2;
  }
  ncells = lvl[nlev];
  HOT_CHECK(tree_hash_build(C, ncells, at<uint64_t>(ws, P.o_h_key), at<uint32_t>(ws, P.o_h_val),
                            P.hcap, s),
            "key hash");
  // K1: cells are accepted only beyond their extent plus the kernel radius
  const double k1h = p.kernel == HOT_KERNEL_K1 ? k1_radius(p.eps) : -1.0;
  for (int l = nlev - 1; l >= 0; --l)
    HOT_CHECK(tree_moments_level(C, spos, smass, n, lvl[l], lvl[l + 1] - lvl[l], p.box, p.theta,
                                 p.G, p.err_tol, k1h, p.order, fp32, s),
              "moments");
  if (local)
    HOT_CHECK(local_moments_launch(fp32, p.order, C.mom, ncells, at<void>(ws, P.o_c_mloc), s),
              "local-route moments");
  uint32_t* gflag = tmp;
  uint32_t* gid = reinterpret_cast<uint32_t*>(key1);
  int32_t* gcell_at = reinterpret_cast<int32_t*>(idx1);
  HOT_CHECK(tree_groups(C, ncells, p.group_max, n, gflag, gid, gcell_at, G, ctr + CTR_NGROUPS,
                        scan_tmp, s),
            "groups");
  HOT_CHECK(tree_srec(C, ncells, spos, smass, n, p.box, p.leaf_max, srec, fp32, s),
            "source records");
  HOT_CHECK(readback(s, ctr, host, 8), "readback");
  ngroups = host[CTR_NGROUPS];
  if (ngroups > P.cap_groups) {
    g_err = "internal: group capacity exceeded";
    return HOT_EDEVICE;
  }
  HOT_CHECK(tree_group_bbox(C, G, ngroups, (uint32_t)P.cap_groups, spos, n, s), "bbox");
  if (rung) {
    uint8_t* act = at<uint8_t>(ws, P.o_g_act);
    HOT_CHECK(group_active_launch(C, G, ngroups, idx0, rung, rmin, act, s), "due groups");
    G.active = act;
  }
  if (c->events_ok) HOT_CHECK(hipEventRecord(c->ev[2], s), "event");

  // ---- walk: count pass over all groups (again with the larger stack if
  // some group's pending cells overflowed the default one)
  for (;;) {
    HOT_CHECK(for_group_batches(G, ngroups, c->group_batch,
                                [&](const Groups& B, uint32_t nb) {
                                  return walk_launch(false, big, C, B, nb,
                                                     (uint32_t)P.cap_groups, p.box, p.periodic,
                                                     lp, nullptr, nullptr, ctr + CTR_STATUS, s);
                                }),
              "walk count");
    HOT_CHECK(sum_counts(G, ngroups, reinterpret_cast<unsigned long long*>(ctr + CTR_SUMS),
                         ctr + CTR_MAXW, s),
              "list totals");
    HOT_CHECK(readback(s, ctr, host, CTR_READ), "readback");
    if (!(host[CTR_STATUS] & 4u)) break;
    if (big) {
      g_err = "tree-walk stack overflow: a sink group has more pending cells than the walk "
              "stack holds (reduce group_max or the opening radius)";
      return HOT_EUNSUPPORTED;
    }
    big = true;
    HOT_CHECK(zero_launch(ctr + CTR_STATUS, 4, s), "clear status");
    HOT_CHECK(zero_launch(ctr + CTR_SUMS, 4 * (CTR_READ - CTR_SUMS), s), "clear totals");
  }
  unsigned long long sums[2];
  std::memcpy(sums, host + CTR_SUMS, sizeof(sums));
  tp = sums[0];
  tm = sums[1];
  const size_t maxw = host[CTR_MAXW];
  // list words: direct entries 1, accepted cells 4 (room for a multipole
  // record; a local entry takes 1 of them), plus 16-byte alignment
  const size_t words = tp + 4 * tm + 4;
  c->list_per_particle = std::max(c->list_per_particle, 1.25 * (double)words / (double)n);
  if (maxw + 4 > P.cap_list) {
    c->stats.ws_bytes_needed = make_plan(c, n, 0, need).total;
    g_err = "interaction-list capacity below one group's lists; call hot_workspace_size again";
    return HOT_EOVERFLOW;
  }
  // chunks of consecutive groups whose lists fit the list region together;
  // a chunk's offsets are 32-bit: words for its direct entries, 16-byte
  // records for its accepted cells
  const size_t cap = P.cap_list, off_max = (size_t)UINT32_MAX - 64;
  auto fits = [&](size_t wp, size_t wm) {
    return wp + 4 * wm + 4 <= cap && wp <= off_max && wm <= off_max;
  };
  if (fits(tp, tm)) {
    chunks.push_back({0, ngroups, tp, tm});
  } else {
    // greedy over groups in order (a new chunk when the next group would
    // overflow), taken a block of kCountBlock groups at a time where the whole
    // block fits: only the blocks where a chunk ends are read group by group.
    // The block sums go to the second key buffer (free after the groups).
    const uint32_t nb = (ngroups + kCountBlock - 1) / kCountBlock;
    unsigned long long* bp = reinterpret_cast<unsigned long long*>(key1);
    unsigned long long* bm = bp + nb;
    HOT_CHECK(block_counts(G, ngroups, bp, bm, s), "list totals");
    std::vector<unsigned long long> hp(nb), hm(nb);
    HOT_CHECK(hipMemcpyAsync(hp.data(), bp, 8 * (size_t)nb, hipMemcpyDeviceToHost, s), "readback");
    HOT_CHECK(hipMemcpyAsync(hm.data(), bm, 8 * (size_t)nb, hipMemcpyDeviceToHost, s), "readback");
    HOT_CHECK(hipStreamSynchronize(s), "readback");
    std::vector<uint32_t> cp(kCountBlock), cm(kCountBlock);
    Chunk ch{0, 0, 0, 0};
    for (uint32_t b = 0; b < nb; ++b) {
      const uint32_t g0 = b * kCountBlock, g1 = std::min(ngroups, g0 + kCountBlock);
      if (fits(ch.tp + hp[b], ch.tm + hm[b])) {
        ch.g1 = g1;
        ch.tp += hp[b];
        ch.tm += hm[b];
        continue;
      }
      HOT_CHECK(hipMemcpyAsync(cp.data(), G.cnt_p2p + g0, 4 * (size_t)(g1 - g0),
                               hipMemcpyDeviceToHost, s),
                "readback");
      HOT_CHECK(hipMemcpyAsync(cm.data(), G.cnt_m2p + g0, 4 * (size_t)(g1 - g0),
                               hipMemcpyDeviceToHost, s),
                "readback");
      HOT_CHECK(hipStreamSynchronize(s), "readback");
      for (uint32_t g = g0; g < g1; ++g) {
        const size_t gp = cp[g - g0], gm = cm[g - g0];
        if (ch.g1 > ch.g0 && !fits(ch.tp + gp, ch.tm + gm)) {
          chunks.push_back(ch);
          ch = Chunk{g, g, 0, 0};
        }
        ch.g1 = g + 1;
        ch.tp += gp;
        ch.tm += gm;
      }
    }
    chunks.push_back(ch);
  }
  }  // !use_tree

  void* arec = nullptr;
  double4* adj = nullptr;
  void* ecoef = nullptr;
  if (vjp) {
    // adjoint: sorted cotangents and the cotangent moments of every cell
    arec = at<void>(ws, P.o_arec);
    adj = at<double4>(ws, P.o_adj);
    double* emom = at<double>(ws, P.o_c_emom);
    ecoef = at<void>(ws, P.o_c_ecoef);
    HOT_CHECK(adj_gather_launch(fp32, vjp->gacc, vjp->gpot, n, idx0, arec, s), "adjoint gather");
    for (int l = nlev - 1; l >= 0; --l)
      HOT_CHECK(adj_moments_level(fp32, p.order, C, spos, arec, n, lvl[l], lvl[l + 1] - lvl[l],
                                  emom, ecoef, s),
                "adjoint moments");
  }
  const bool single = chunks.size() == 1;
  // chunked lists: each chunk's emit pass, direct and multipole kernels are
  // timed with the context's chunk events (up to kChunkEvents chunks)
  const bool cev = !single && c->events_ok && c->cev_ok && chunks.size() <= (size_t)kChunkEvents;
  if (!single && c->events_ok) HOT_CHECK(hipEventRecord(c->ev[3], s), "event");
  uint32_t* p2p_list = at<uint32_t>(ws, P.o_list);
  size_t ck = 0;
  for (const Chunk& k : chunks) {
    if (cev) HOT_CHECK(hipEventRecord(c->cev[4 * ck], s), "event");
    const uint32_t ng = k.g1 - k.g0;
    Groups Gk = G;  // the chunk's groups (the box arrays keep their stride)
    Gk.cell += k.g0;
    Gk.lo += k.g0;
    Gk.hi += k.g0;
    Gk.cnt_p2p += k.g0;
    Gk.cnt_m2p += k.g0;
    Gk.off_p2p += k.g0;
    Gk.off_m2p += k.g0;
    Gk.cnt_m2l += k.g0;
    Gk.off_m2l += k.g0;
    if (Gk.active) Gk.active += k.g0;
    // a group's accepted cells: its multipole records from off_m2p on, its
    // local entries (32-bit words) at the end of the same region (the emit
    // pass sets off_m2l, a word index, and both counts)
    uint4* m2p_list = reinterpret_cast<uint4*>(p2p_list + ((k.tp + 3) & ~size_t(3)));
    if (!use_tree) {
      HOT_CHECK(scan_u32(Gk.cnt_p2p, Gk.off_p2p, ctr + CTR_TP, ng, scan_tmp, s), "scan");
      HOT_CHECK(scan_u32(Gk.cnt_m2p, Gk.off_m2p, ctr + CTR_TM, ng, scan_tmp, s), "scan");
      HOT_CHECK(for_group_batches(Gk, ng, c->group_batch,
                                  [&](const Groups& B, uint32_t nb) {
                                    return walk_launch(true, big, C, B, nb,
                                                       (uint32_t)P.cap_groups, p.box, p.periodic,
                                                       lp, p2p_list, m2p_list,
                                                       ctr + CTR_STATUS, s);
                                  }),
                "walk emit");
      HOT_CHECK(count_pairs(C, Gk, ng, local, p2p_list,
                            reinterpret_cast<unsigned long long*>(ctr + CTR_PAIRS),
                            reinterpret_cast<unsigned long long*>(ctr + CTR_SLOTS), s),
                "pair count");
    }
    if (single && c->events_ok) HOT_CHECK(hipEventRecord(c->ev[3], s), "event");
    if (cev) HOT_CHECK(hipEventRecord(c->cev[4 * ck + 1], s), "event");
    if (!vjp) {
      HOT_CHECK(for_group_batches(Gk, ng, c->group_batch,
                                  [&](const Groups& B, uint32_t nb) {
                                    return p2p_launch(fp32, p.kernel, C, B, nb, p.box, p.eps,
                                                      spos, srec, n, p2p_list, near, s, c->side);
                                  }),
                "direct kernel");
      if (single && c->events_ok) HOT_CHECK(hipEventRecord(c->ev[4], s), "event");
      if (cev) HOT_CHECK(hipEventRecord(c->cev[4 * ck + 2], s), "event");
      // group-level local expansions, between the direct and multipole
      // kernels (no other kernel writes the accumulators meanwhile)
      if (local)
        HOT_CHECK(for_group_batches(Gk, ng, c->group_batch,
                                    [&](const Groups& B, uint32_t nb) {
                                      return local_launch(fp32, p.order, p.local_order, C, B, nb,
                                                          (uint32_t)P.cap_groups, p.box, spos, n,
                                                          reinterpret_cast<const uint32_t*>(
                                                              m2p_list),
                                                          at<void>(ws, P.o_c_mloc),
                                                          near, s);
                                    }),
                  "local expansions");
      if (single && c->events_ok) HOT_CHECK(hipEventRecord(c->ev[7], s), "event");
      if (cev) HOT_CHECK(hipEventRecord(c->cev[4 * ck + 3], s), "event");
      // multipoles expand the softened kernel for Plummer, the Newtonian one
      // for K1 (accepted cells lie beyond its radius)
      HOT_CHECK(for_group_batches(Gk, ng, c->group_batch,
                                  [&](const Groups& B, uint32_t nb) {
                                    return m2p_launch(fp32, p.order, C, B, nb, p.box,
                                                      p.kernel == HOT_KERNEL_K1 ? 0.0 : p.eps,
                                                      spos, n, m2p_list, near, s, c->side);
                                  }),
                "multipole kernel");
    } else {
      HOT_CHECK(for_group_batches(Gk, ng, c->group_batch,
                                  [&](const Groups& B, uint32_t nb) {
                                    return p2p_adj_launch(fp32, C, B, nb, p.box, p.eps, spos,
                                                          srec, arec, n, p2p_list, adj, s,
                                                          c->side);
                                  }),
                "adjoint direct kernel");
      if (single && c->events_ok) HOT_CHECK(hipEventRecord(c->ev[4], s), "event");
      if (single && c->events_ok) HOT_CHECK(hipEventRecord(c->ev[7], s), "event");
      if (cev) HOT_CHECK(hipEventRecord(c->cev[4 * ck + 2], s), "event");
      if (cev) HOT_CHECK(hipEventRecord(c->cev[4 * ck + 3], s), "event");
      HOT_CHECK(for_group_batches(Gk, ng, c->group_batch,
                                  [&](const Groups& B, uint32_t nb) {
                                    return m2p_adj_launch(fp32, p.order, C, B, nb, p.box, p.eps,
                                                          spos, srec, arec, ecoef, n, m2p_list,
                                                          adj, s, c->side);
                                  }),
                "adjoint multipole kernel");
    }
    ++ck;
    if (cev) HOT_CHECK(hipEventRecord(c->cev[4 * ck], s), "event");
  }
  if (!single && c->events_ok) HOT_CHECK(hipEventRecord(c->ev[4], s), "event");
  if (!single && c->events_ok) HOT_CHECK(hipEventRecord(c->ev[7], s), "event");
  if (c->events_ok) HOT_CHECK(hipEventRecord(c->ev[5], s), "event");

  if (!vjp) {
    HOT_CHECK(far_launch(p.far_order, spos, smass, key0, near, n, idx0, p.box, p.G, c->d_tpsi,
                         at<double>(ws, P.o_far_part), kFarBlocks, at<double>(ws, P.o_far_mom),
                         at<double>(ws, P.o_far_lam), p.periodic, rung, rmin, fp32, acc, pot, s),
              "far field");
  } else {
    if (p.periodic)
      HOT_CHECK(far_prepare_launch(p.far_order, spos, smass, key0, n, p.box, c->d_tpsi,
                                   at<double>(ws, P.o_far_part), kFarBlocks,
                                   at<double>(ws, P.o_far_mom), at<double>(ws, P.o_far_lam), s),
                "far field");
    HOT_CHECK(far_adj_launch(p.far_order, spos, smass, key0, arec, adj, n, idx0, p.box, p.G,
                             c->d_tpsi, at<double>(ws, P.o_far_part), kFarBlocks,
                             at<double>(ws, P.o_far_lam), at<double>(ws, P.o_far_mom),
                             at<double>(ws, P.o_far_mbar),
                             p.periodic, fp32, vjp->xbar, vjp->mbar, s),
              "far-field adjoint");
  }
  // the pair counters go to the context's pinned host buffer, so that
  // hot_get_stats reads no device memory (the workspace may be gone by then)
  HOT_CHECK(hipMemcpyAsync(c->host_buf + kHostPairs, ctr + CTR_PAIRS, 16, hipMemcpyDeviceToHost,
                           s),
            "pair counters");
  HOT_CHECK(hipMemcpyAsync(c->host_buf + kHostSlots, ctr + CTR_SLOTS, 48, hipMemcpyDeviceToHost,
                           s),
            "lane-step counters");
  if (c->events_ok) HOT_CHECK(hipEventRecord(c->ev[6], s), "event");
  c->last_chunks = (int)chunks.size();
  c->last_cev = cev ? (int)chunks.size() : 0;

  hot_stats& st = c->stats;
  std::memset(&st, 0, sizeof(st));
  st.n = (int64_t)n;
  st.ncells = ncells;
  st.ngroups = ngroups;
  st.nlevels = nlev;
  st.p2p_entries = (int64_t)tp;
  // split into multipole and local entries once the lane-step counters are
  // on the host (settle_entries)
  st.m2p_entries = (int64_t)tm;
  st.m2l_entries = 0;
  c->last_accepted = tm;
  st.list_chunks = (int64_t)chunks.size();
  st.ws_bytes_needed = P.total;
  c->have_last = 1;
  c->last_n = n;
  c->last_stream = s;
  c->last_plan = P;
  c->last_ws = ws;
  c->last_ncells = ncells;
  c->last_ngroups = ngroups;
  if (chunks.size() == 1 && !rung) {
    hot_ctx::TreeRecord& T = c->tree;
    T.pos = pos;
    T.mass = mass;
    T.n = n;
    T.ws = ws;
    T.ws_bytes = ws_bytes;
    T.stream = s;
    T.words = tp + 4 * tm + 4;
    T.o_list = P.o_list;
    T.cap_cells = P.cap_cells;
    std::copy(lvl.begin(), lvl.end(), T.lvl);
    T.nlev = nlev;
    T.ncells = ncells;
    T.ngroups = ngroups;
    T.tp = tp;
    T.tm = tm;
    T.valid = 1;
  }
  return HOT_OK;
}

}  // namespace hot

using namespace hot;

// ---- comoving kick and drift factors: K = int da / (a^2 H), D = int da /
// (a^3 H) over [a1, a2], integrated in u = ln a (da = a du, a smooth
// integrand), composite Gauss-Legendre with 16 nodes per panel and panels at
// most 0.05 wide in u
namespace {
struct GaussLegendre16 {
  double x[16], w[16];
  GaussLegendre16() {
    // roots of P_16 by Newton's method from the usual cosine guesses
    const int m = 16;
    for (int i = 0; i < m; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (m + 0.5)), dp = 0.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = 0.0;
        for (int j = 1; j <= m; ++j) {
          const double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
        }
        dp = m * (z * p0 - p1) / (z * z - 1.0);
        const double z1 = z;
        z = z1 - p0 / dp;
        if (std::fabs(z - z1) < 1e-16) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};
const GaussLegendre16& gauss16() {
  static const GaussLegendre16 g;
  return g;
}
// H(a)^2 / h0^2
double hubble2(double a, double om, double ol) {
  return om / (a * a * a) + (1.0 - om - ol) / (a * a) + ol;
}
}  // namespace

static bool comoving_factors(double a1, double a2, double om, double ol, double h0, double* K,
                             double* D) {
  if (!(a1 > 0.0) || !(a2 > 0.0) || !std::isfinite(a1) || !std::isfinite(a2) ||
      !(h0 > 0.0) || !std::isfinite(h0) || !std::isfinite(om) || !std::isfinite(ol))
    return false;
  const double u1 = std::log(a1), u2 = std::log(a2);
  const int panels = std::max(1, (int)std::ceil(std::fabs(u2 - u1) / 0.05));
  const double hw = 0.5 * (u2 - u1) / panels;
  const GaussLegendre16& g = gauss16();
  double k = 0.0, d = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double mid = u1 + (2 * p + 1) * hw;
    for (int i = 0; i < 16; ++i) {
      const double a = std::exp(mid + hw * g.x[i]);
      const double h2 = hubble2(a, om, ol);
      if (!(h2 > 0.0)) return false;
      const double e = g.w[i] / std::sqrt(h2);  // da / H = a du / H
      k += e / a;                               // a du / (a^2 H)
      d += e / (a * a);                         // a du / (a^3 H)
    }
  }
  *K = k * hw / h0;
  *D = d * hw / h0;
  return true;
}

extern "C" {

const char* hot_version(void) { return "libhot 0.1 (gfx950)"; }

hot_status hot_far_table(int far_order, double box, int offset, double* out, size_t count) {
  if (far_order < 0 || far_order > kMaxFarOrder || !(box > 0.0) || !out || offset < 0 ||
      offset > 26 || count < (size_t)nt(2 * far_order)) {
    g_err = "bad argument";
    return HOT_EINVAL;
  }
  const double r0[3] = {(offset / 9 - 1) * 0.5 * box, ((offset / 3) % 3 - 1) * 0.5 * box,
                        (offset % 3 - 1) * 0.5 * box};
  psi_taylor_table(2 * far_order, box, r0, out);
  return HOT_OK;
}

const char* hot_last_error(void) { return g_err.c_str(); }

hot_status hot_create(const hot_params* params, hot_ctx** out) {
  if (!out) {
    g_err = "out is NULL";
    return HOT_EINVAL;
  }
  *out = nullptr;
  if (!params) {
    g_err = "params is NULL";
    return HOT_EINVAL;
  }
  std::string why;
  if (!valid_params(params, &why)) {
    g_err = why;
    return HOT_EINVAL;
  }
  hot_ctx* c = new hot_ctx();
  std::memset(c, 0, sizeof(*c));
  c->p = *params;
  c->S = 2097152.0 / params->box;
  c->cells_per_particle = 4.0 / params->leaf_max + 0.02;  // grows on overflow
  c->group_batch = kGroupBatch;
  if (const char* gb = std::getenv("HOT_GROUP_BATCH")) {
    const long v = std::strtol(gb, nullptr, 10);
    if (v > 0 && (unsigned long)v < kGroupBatch) c->group_batch = (uint32_t)v;
  }
  c->list_per_particle = 96.0;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return device_error(e, "hipGetDevice");
  }
  resolve_scratch(c->device);
  const int D = 2 * params->far_order;
  c->n_tpsi = nt(D);
  std::vector<double> tab((size_t)27 * c->n_tpsi);
  if (params->periodic) psi_taylor_tables27(D, params->box, tab.data());
  e = hipMalloc(&c->d_tpsi, sizeof(double) * tab.size());
  if (e == hipSuccess)
    e = hipMemcpy(c->d_tpsi, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->host_buf, 4 * kHostWords, hipHostMallocDefault);
  if (e != hipSuccess) {
    hot_destroy(c);
    return device_error(e, "context allocation");
  }
  c->events_ok = 1;
  for (int i = 0; i < 8; ++i)
    if (hipEventCreate(&c->ev[i]) != hipSuccess) c->events_ok = 0;
  c->cev_ok = 1;
  for (int i = 0; i < 4 * kChunkEvents + 1; ++i)
    if (hipEventCreate(&c->cev[i]) != hipSuccess) c->cev_ok = 0;
  (void)hipGetLastError();
  if (hipStreamCreateWithFlags(&c->side.st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->side.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->side.join, hipEventDisableTiming) != hipSuccess) {
    if (c->side.st) (void)hipStreamDestroy(c->side.st);
    if (c->side.fork) (void)hipEventDestroy(c->side.fork);
    c->side = hot::SideStream{};
    (void)hipGetLastError();
  }
  *out = c;
  return HOT_OK;
}

void hot_destroy(hot_ctx* c) {
  if (!c) return;
  if (c->d_tpsi) (void)hipFree(c->d_tpsi);
  if (c->host_buf) (void)hipHostFree(c->host_buf);
  for (int i = 0; i < 8; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  for (int i = 0; i < 4 * kChunkEvents + 1; ++i)
    if (c->cev[i]) (void)hipEventDestroy(c->cev[i]);
  if (c->side.st) (void)hipStreamDestroy(c->side.st);
  if (c->side.fork) (void)hipEventDestroy(c->side.fork);
  if (c->side.join) (void)hipEventDestroy(c->side.join);
  delete c;
}

size_t hot_workspace_size(const hot_ctx* c, size_t n) {
  if (!c) return 0;
  return make_plan(c, n, 0, kNeedAdjoint | kNeedSnapshot | kNeedReverse).total;
}

size_t hot_workspace_size_min(const hot_ctx* c, size_t n, unsigned calls) {
  if (!c) return 0;
  unsigned need = 0;
  if (calls & (HOT_CALL_VJP | HOT_CALL_KDK_VJP)) need |= kNeedAdjoint;
  if (calls & (HOT_CALL_KDK | HOT_CALL_KDK_VJP)) need |= kNeedSnapshot;
  if (calls & HOT_CALL_KDK_VJP) need |= kNeedReverse;
  return make_plan(c, n, 0, need).min_total;
}

hot_status hot_forces(hot_ctx* c, size_t n, const double* pos, const void* mass, void* acc,
                      void* pot, void* ws, size_t ws_bytes, void* stream) {
  if (!c) {
    g_err = "ctx is NULL";
    return HOT_EINVAL;
  }
  if (n == 0) return HOT_OK;
  if (!pos || !mass || !acc || !ws) {
    g_err = "NULL pointer argument";
    return HOT_EINVAL;
  }
  if (n >= (size_t)0xffffffffu) {
    g_err = "n must be < 2^32";
    return HOT_EINVAL;
  }
  return forces_impl(c, n, pos, mass, acc, pot, ws, ws_bytes, (hipStream_t)stream, 0);
}

hot_status hot_forces_noalloc(hot_ctx* c, size_t n, const double* pos, const void* mass,
                              void* acc, void* pot, void* stream) {
  if (!c) {
    g_err = "ctx is NULL";
    return HOT_EINVAL;
  }
  if (n == 0) return HOT_OK;
  if (!pos || !mass || !acc) {
    g_err = "NULL pointer argument";
    return HOT_EINVAL;
  }
  if (n >= (size_t)0xffffffffu) {
    g_err = "n must be < 2^32";
    return HOT_EINVAL;
  }
  int dev = -1;
  HOT_CHECK(hipGetDevice(&dev), "hipGetDevice");
  if (dev != c->device) {
    g_err = "the current device is not the context's device";
    return HOT_EINVAL;
  }
  if (dev >= kMaxDevices || !g_scratch_done[dev] || !g_scratch_ptr[dev]) {
    g_err = std::string("no-allocation scratch unavailable on this device: ") +
            ((dev < kMaxDevices && g_scratch_done[dev]) ? hipGetErrorString(g_scratch_err[dev])
                                                        : "not resolved");
    return HOT_EDEVICE;
  }
  void* ws = g_scratch_ptr[dev];
  // the structures must fit the fixed array; the interaction lists take what
  // is left and are processed in chunks of sink groups when they do not fit
  for (int attempt = 0; attempt < 4; ++attempt) {
    const Plan P = make_plan(c, n, kNoAllocBytes, 0);
    if (P.min_total > kNoAllocBytes) {
      g_err = "n = " + std::to_string(n) + " needs " + std::to_string(P.min_total) +
              " bytes of scratch; hot_forces_noalloc has " + std::to_string(kNoAllocBytes) +
              " (use hot_forces with a workspace)";
      return HOT_ENOMEM;
    }
    const hot_status st =
        forces_impl(c, n, pos, mass, acc, pot, ws, kNoAllocBytes, (hipStream_t)stream, 0);
    if (st != HOT_EOVERFLOW) return st;
    // a learned capacity grew (cells, or one group's lists): retry if the
    // structures still fit
  }
  return HOT_EOVERFLOW;
}

hot_status hot_kdk(hot_ctx* c, size_t n, double* pos, void* vel, const void* mass, void* acc,
                   void* pot, double dt, int nsteps, unsigned flags, void* ws, size_t ws_bytes,
                   void* stream) {
  if (!c) {
    g_err = "ctx is NULL";
    return HOT_EINVAL;
  }
  if (n == 0) return HOT_OK;
  if (!pos || !vel || !mass || !acc || !ws || nsteps < 0 || !std::isfinite(dt)) {
    g_err = "bad argument";
    return HOT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool fp32 = c->p.precision == HOT_FP32;
  const size_t tsz = fp32 ? 4 : 8;
  c->stats.kdk_steps_done = 0;
  const bool snap = !(flags & HOT_KDK_NO_SNAPSHOT);
  const unsigned need = snap ? kNeedSnapshot : 0;
  const Plan P = make_plan(c, n, ws_bytes, need);
  if (ws_bytes < P.min_total) {
    g_err = "workspace smaller than hot_workspace_size_min(HOT_CALL_KDK)";
    return HOT_ENOMEM;
  }
  hot_status st;
  if (!(flags & HOT_ACC_VALID)) {
    st = forces_impl(c, n, pos, mass, acc, pot, ws, ws_bytes, s, need);
    if (st != HOT_OK) return st;
  }
  double* sx = snap ? at<double>(ws, P.o_kv_sx) : nullptr;
  void* sv = snap ? at<void>(ws, P.o_kv_sv) : nullptr;
  for (int k = 0; k < nsteps; ++k) {
    // snapshot of the step's start, restored if its force evaluation fails
    if (snap) {
      HOT_CHECK(hipMemcpyAsync(sx, pos, 24 * n, hipMemcpyDeviceToDevice, s), "snapshot");
      HOT_CHECK(hipMemcpyAsync(sv, vel, 3 * tsz * n, hipMemcpyDeviceToDevice, s), "snapshot");
    }
    HOT_CHECK(kick_launch(fp32, vel, acc, n, 0.5 * dt, s), "kick");
    HOT_CHECK(drift_launch(fp32, pos, vel, n, dt, c->p.box, s), "drift");
    st = forces_impl(c, n, pos, mass, acc, pot, ws, ws_bytes, s, need);
    if (st != HOT_OK) {
      // acc is written only by a successful evaluation
      if (snap) {
        HOT_CHECK(hipMemcpyAsync(pos, sx, 24 * n, hipMemcpyDeviceToDevice, s), "restore");
        HOT_CHECK(hipMemcpyAsync(vel, sv, 3 * tsz * n, hipMemcpyDeviceToDevice, s), "restore");
        HOT_CHECK(hipStreamSynchronize(s), "restore");
      }
      return st;
    }
    HOT_CHECK(kick_launch(fp32, vel, acc, n, 0.5 * dt, s), "kick");
    c->stats.kdk_steps_done = k + 1;
  }
  return HOT_OK;
}

hot_status hot_comoving_factors(double a1, double a2, double omega_m, double omega_l, double h0,
                                double* out) {
  if (!out || !comoving_factors(a1, a2, omega_m, omega_l, h0, &out[0], &out[1])) {
    g_err = "bad argument (a1, a2, h0 > 0 and finite, H^2 > 0 on [a1, a2], out not NULL)";
    return HOT_EINVAL;
  }
  return HOT_OK;
}

hot_status hot_kdk_comoving(hot_ctx* c, size_t n, double* pos, void* vel, const void* mass,
                            void* acc, void* pot, double a0, double da, int nsteps,
                            double omega_m, double omega_l, double h0, unsigned flags, void* ws,
                            size_t ws_bytes, void* stream) {
  if (!c) {
    g_err = "ctx is NULL";
    return HOT_EINVAL;
  }
  if (n == 0) return HOT_OK;
  if (!pos || !vel || !mass || !acc || !ws || nsteps < 0 || !std::isfinite(da)) {
    g_err = "bad argument";
    return HOT_EINVAL;
  }
  // the whole path first (a_k is monotone in k, so its ends bound it), so
  // that a bad background fails before any particle moves
  {
    double k_unused, d_unused;
    if (!comoving_factors(a0, a0 + nsteps * da, omega_m, omega_l, h0, &k_unused, &d_unused)) {
      g_err = "bad background (a0 > 0, every a_k > 0, h0 > 0, H^2 > 0 on the path)";
      return HOT_EINVAL;
    }
  }
  // one step's factors: opening kick, drift, closing kick
  auto factors = [&](int k, double* f) {
    const double ak = a0 + k * da, ah = ak + 0.5 * da, a1 = a0 + (k + 1) * da;
    double u;
    return comoving_factors(ak, ah, omega_m, omega_l, h0, &f[0], &u) &&
           comoving_factors(ak, a1, omega_m, omega_l, h0, &u, &f[1]) &&
           comoving_factors(ah, a1, omega_m, omega_l, h0, &f[2], &u);
  };
  hipStream_t s = (hipStream_t)stream;
  const bool fp32 = c->p.precision == HOT_FP32;
  const size_t tsz = fp32 ? 4 : 8;
  c->stats.kdk_steps_done = 0;
  const bool snap = !(flags & HOT_KDK_NO_SNAPSHOT);
  const unsigned need = snap ? kNeedSnapshot : 0;
  const Plan P = make_plan(c, n, ws_bytes, need);
  if (ws_bytes < P.min_total) {
    g_err = "workspace smaller than hot_workspace_size_min(HOT_CALL_KDK)";
    return HOT_ENOMEM;
  }
  hot_status st;
  if (!(flags & HOT_ACC_VALID)) {
    st = forces_impl(c, n, pos, mass, acc, pot, ws, ws_bytes, s, need);
    if (st != HOT_OK) return st;
  }
  double* sx = snap ? at<double>(ws, P.o_kv_sx) : nullptr;
  void* sv = snap ? at<void>(ws, P.o_kv_sv) : nullptr;
  for (int k = 0; k < nsteps; ++k) {
    double f[3];
    if (!factors(k, f)) {
      g_err = "bad background on a step (H^2 <= 0 at a quadrature node)";
      return HOT_EINVAL;
    }
    if (snap) {
      HOT_CHECK(hipMemcpyAsync(sx, pos, 24 * n, hipMemcpyDeviceToDevice, s), "snapshot");
      HOT_CHECK(hipMemcpyAsync(sv, vel, 3 * tsz * n, hipMemcpyDeviceToDevice, s), "snapshot");
    }
    HOT_CHECK(kick_launch(fp32, vel, acc, n, f[0], s), "kick");
    HOT_CHECK(drift_launch(fp32, pos, vel, n, f[1], c->p.box, s), "drift");
    st = forces_impl(c, n, pos, mass, acc, pot, ws, ws_bytes, s, need);
    if (st != HOT_OK) {
      if (snap) {
        HOT_CHECK(hipMemcpyAsync(pos, sx, 24 * n, hipMemcpyDeviceToDevice, s), "restore");
        HOT_CHECK(hipMemcpyAsync(vel, sv, 3 * tsz * n, hipMemcpyDeviceToDevice, s), "restore");
        HOT_CHECK(hipStreamSynchronize(s), "restore");
      }
      return st;
    }
    HOT_CHECK(kick_launch(fp32, vel, acc, n, f[2], s), "kick");
    c->stats.kdk_steps_done = k + 1;
  }
  return HOT_OK;
}

hot_status hot_kdk_block(hot_ctx* c, size_t n, double* pos, void* vel, const void* mass,
                         void* acc, void* pot, uint8_t* rung, double dt, int max_rung, double eta,
                         int nsteps, unsigned flags, void* ws, size_t ws_bytes, void* stream) {
  if (!c) {
    g_err = "ctx is NULL";
    return HOT_EINVAL;
  }
  if (n == 0) return HOT_OK;
  if (!pos || !vel || !mass || !acc || !rung || !ws || nsteps < 0 || !std::isfinite(dt) ||
      max_rung < 0 || max_rung > kMaxRung || !(eta > 0.0) || !std::isfinite(eta)) {
    g_err = "bad argument (max_rung must be in 0..16, eta > 0)";
    return HOT_EINVAL;
  }
  if (n >= (size_t)0xffffffffu) {
    g_err = "n must be < 2^32";
    return HOT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool fp32 = c->p.precision == HOT_FP32;
  c->stats.kdk_steps_done = 0;
  const Plan P = make_plan(c, n, ws_bytes, 0);
  if (ws_bytes < P.min_total) {
    g_err = "workspace smaller than hot_workspace_size_min(HOT_CALL_FORCES)";
    return HOT_ENOMEM;
  }
  hot_status st;
  if (!(flags & HOT_ACC_VALID)) {
    st = forces_impl(c, n, pos, mass, acc, pot, ws, ws_bytes, s, 0);
    if (st != HOT_OK) return st;
  }
  const double eps = c->p.eps;
  if (!(flags & HOT_RUNG_VALID))
    HOT_CHECK(rung_assign_launch(fp32, acc, rung, n, 0, dt, max_rung, eta, eps, s), "rungs");
  // the largest rung in use: a substep boundary where no particle is due
  // only drifts
  uint32_t* ctr = at<uint32_t>(ws, P.o_ctr);
  uint32_t* host = c->host_buf;
  auto largest_rung = [&](int* out) -> hipError_t {
    hipError_t e = rung_max_launch(rung, n, ctr + CTR_RMAX, s);
    if (e == hipSuccess) e = readback(s, ctr + CTR_RMAX, host, 1);
    *out = (int)host[0];
    return e;
  };
  int rmax = 0;
  HOT_CHECK(largest_rung(&rmax), "rungs");
  if (rmax > max_rung) {
    g_err = "a rung on entry exceeds max_rung";
    return HOT_EINVAL;
  }
  const uint32_t S = 1u << max_rung;
  const double sub = ldexp(dt, -max_rung);
  for (int k = 0; k < nsteps; ++k) {
    for (uint32_t q = 0; q < S; ++q) {
      // the particles whose step starts at substep q: every rung at q = 0,
      // else rung >= max_rung - (trailing zeros of q)
      const int rstart = q == 0 ? 0 : max_rung - __builtin_ctz(q);
      if (rstart <= rmax) HOT_CHECK(kick_rung_launch(fp32, vel, acc, rung, n, rstart, dt, s), "kick");
      HOT_CHECK(drift_launch(fp32, pos, vel, n, sub, c->p.box, s), "drift");
      // those whose step ends at the next boundary
      const int rend = q + 1 == S ? 0 : max_rung - __builtin_ctz(q + 1);
      if (rend > rmax) continue;
      st = forces_impl(c, n, pos, mass, acc, pot, ws, ws_bytes, s, 0, nullptr, false, rung, rend);
      if (st != HOT_OK) return st;  // pos, vel, acc and rung are then undefined
      HOT_CHECK(kick_rung_launch(fp32, vel, acc, rung, n, rend, dt, s), "kick");
      if (!(flags & HOT_RUNG_FIXED)) {
        HOT_CHECK(rung_assign_launch(fp32, acc, rung, n, rend, dt, max_rung, eta, eps, s),
                  "rungs");
        HOT_CHECK(largest_rung(&rmax), "rungs");
      }
    }
    c->stats.kdk_steps_done = k + 1;
  }
  return HOT_OK;
}

hot_status hot_vjp(hot_ctx* c, size_t n, const double* pos, const void* mass, const void* gacc,
                   const void* gpot, double* xbar, void* mbar, void* ws, size_t ws_bytes,
                   void* stream) {
  if (!c) {
    g_err = "ctx is NULL";
    return HOT_EINVAL;
  }
  if (c->p.kernel != HOT_KERNEL_PLUMMER) {
    g_err = "the adjoint is built for Plummer softening only";
    return HOT_EUNSUPPORTED;
  }
  if (local_on(c->p)) {
    g_err = "the adjoint is built without group-level local expansions";
    return HOT_EUNSUPPORTED;
  }
  if (n == 0) return HOT_OK;
  if (!pos || !mass || !gacc || !xbar || !mbar || !ws) {
    g_err = "NULL pointer argument";
    return HOT_EINVAL;
  }
  if (n >= (size_t)0xffffffffu) {
    g_err = "n must be < 2^32";
    return HOT_EINVAL;
  }
  VjpArgs a{gacc, gpot, xbar, mbar};
  return forces_impl(c, n, pos, mass, nullptr, nullptr, ws, ws_bytes, (hipStream_t)stream,
                     kNeedAdjoint, &a);
}

hot_status hot_vjp_after_forces(hot_ctx* c, size_t n, const double* pos, const void* mass,
                                const void* gacc, const void* gpot, double* xbar, void* mbar,
                                void* ws, size_t ws_bytes, void* stream) {
  if (!c) {
    g_err = "ctx is NULL";
    return HOT_EINVAL;
  }
  if (c->p.kernel != HOT_KERNEL_PLUMMER) {
    g_err = "the adjoint is built for Plummer softening only";
    return HOT_EUNSUPPORTED;
  }
  if (local_on(c->p)) {
    g_err = "the adjoint is built without group-level local expansions";
    return HOT_EUNSUPPORTED;
  }
  if (n == 0) return HOT_OK;
  if (!pos || !mass || !gacc || !xbar || !mbar || !ws) {
    g_err = "NULL pointer argument";
    return HOT_EINVAL;
  }
  if (n >= (size_t)0xffffffffu) {
    g_err = "n must be < 2^32";
    return HOT_EINVAL;
  }
  VjpArgs a{gacc, gpot, xbar, mbar};
  return forces_impl(c, n, pos, mass, nullptr, nullptr, ws, ws_bytes, (hipStream_t)stream,
                     kNeedAdjoint, &a, true);
}

hot_status hot_kdk_vjp(hot_ctx* c, size_t n, int nsteps, const double* pos_ckpt, const void* mass,
                       double dt, double* xbar, void* vbar, void* mbar, void* ws, size_t ws_bytes,
                       void* stream) {
  if (!c) {
    g_err = "ctx is NULL";
    return HOT_EINVAL;
  }
  if (c->p.kernel != HOT_KERNEL_PLUMMER) {
    g_err = "the adjoint is built for Plummer softening only";
    return HOT_EUNSUPPORTED;
  }
  if (local_on(c->p)) {
    g_err = "the adjoint is built without group-level local expansions";
    return HOT_EUNSUPPORTED;
  }
  if (n == 0) return HOT_OK;
  if (!pos_ckpt || !mass || !xbar || !vbar || !ws || nsteps < 0 || !std::isfinite(dt)) {
    g_err = "bad argument";
    return HOT_EINVAL;
  }
  if (n >= (size_t)0xffffffffu) {
    g_err = "n must be < 2^32";
    return HOT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool fp32 = c->p.precision == HOT_FP32;
  const size_t tsz = fp32 ? 4 : 8;
  if (nsteps == 0) {
    if (mbar) HOT_CHECK(zero_launch(mbar, tsz * n, s), "clear mbar");
    return HOT_OK;
  }
  // the scratch of the sweep sits in the workspace regions reserved for it,
  // which the force derivative itself does not touch
  Plan P = make_plan(c, n, ws_bytes, kNeedAdjoint | kNeedSnapshot | kNeedReverse);
  if (ws_bytes < P.min_total) {
    g_err = "workspace smaller than hot_workspace_size_min(HOT_CALL_KDK_VJP)";
    return HOT_ENOMEM;
  }
  void* gacc = at<void>(ws, P.o_kv_g);
  double* tx = at<double>(ws, P.o_kv_x);
  void* tm = at<void>(ws, P.o_kv_m);
  double* sx = at<double>(ws, P.o_kv_sx);
  void* sv = at<void>(ws, P.o_kv_sv);
  HOT_CHECK(hipMemcpyAsync(sx, xbar, 24 * n, hipMemcpyDeviceToDevice, s), "snapshot");
  HOT_CHECK(hipMemcpyAsync(sv, vbar, 3 * tsz * n, hipMemcpyDeviceToDevice, s), "snapshot");
  const size_t stride = 3 * n;
  for (int k = nsteps; k >= 0; --k) {
    // k == nsteps: closing kick of the last step only (no drift yet)
    const double cf = (k == nsteps || k == 0) ? 0.5 * dt : dt;
    HOT_CHECK(kdk_adj_drift_launch(fp32, vbar, xbar, gacc, n, dt, cf, k != nsteps, s),
              "adjoint drift");
    VjpArgs a{gacc, nullptr, tx, tm};
    hot_status st = forces_impl(c, n, pos_ckpt + (size_t)k * stride, mass, nullptr, nullptr, ws,
                                ws_bytes, s,
                                kNeedAdjoint | kNeedSnapshot | kNeedReverse, &a);
    if (st != HOT_OK) {
      HOT_CHECK(hipMemcpyAsync(xbar, sx, 24 * n, hipMemcpyDeviceToDevice, s), "restore");
      HOT_CHECK(hipMemcpyAsync(vbar, sv, 3 * tsz * n, hipMemcpyDeviceToDevice, s), "restore");
      HOT_CHECK(hipStreamSynchronize(s), "restore");
      return st;
    }
    HOT_CHECK(kdk_adj_accum_launch(fp32, xbar, tx, mbar, tm, n, k == nsteps, s), "adjoint sum");
  }
  return HOT_OK;
}

// the walk's count pass counts accepted cells without deciding between the
// multipole and the local route; the pair-count kernel after the emit pass
// counts the local entries.  Once its counters are on the host (the last
// call's work has finished), split the total.
static void settle_entries(hot_ctx* m) {
  unsigned long long sl[6];
  std::memcpy(sl, m->host_buf + kHostSlots, sizeof(sl));
  const size_t tl = local_on(m->p) ? (size_t)sl[3] : 0;
  m->stats.m2l_entries = (int64_t)tl;
  m->stats.m2p_entries = (int64_t)(m->last_accepted - tl);
}

// per-group offsets of one list kind in the list region (32-bit words for the
// direct and local lists from their bases, 16-byte records for the multipole
// list) and the packed CSR offsets of the same entries; the multipole records
// and local entries of a group share its accepted-cell region
static hipError_t list_layout(hot_ctx* c, void* ws, int kind, std::vector<size_t>& raw,
                              std::vector<int64_t>& packed) {
  const Plan& P = c->last_plan;
  const size_t ng = c->last_ngroups;
  std::vector<uint32_t> cnt(ng);
  raw.assign(ng, 0);
  packed.assign(ng + 1, 0);
  if (ng == 0) return hipSuccess;
  const size_t o_cnt = kind == 2 ? P.o_g_cl : kind ? P.o_g_cm : P.o_g_cp;
  const size_t o_off = kind == 2 ? P.o_g_ol : kind ? P.o_g_om : P.o_g_op;
  std::vector<uint32_t> off(ng);
  hipError_t e = hipMemcpy(cnt.data(), at<char>(ws, o_cnt), 4 * ng, hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(off.data(), at<char>(ws, o_off), 4 * ng, hipMemcpyDeviceToHost);
  for (size_t g = 0; g < ng; ++g) {
    packed[g + 1] = packed[g] + cnt[g];
    // local entries: the words before the end of the group's region
    raw[g] = kind == 2 ? (cnt[g] ? 4 * (size_t)off[g] - cnt[g] : 0) : off[g];
  }
  return e;
}

hot_status hot_get_stats(const hot_ctx* c, hot_stats* out) {
  if (!c || !out) {
    g_err = "NULL argument";
    return HOT_EINVAL;
  }
  hot_ctx* m = const_cast<hot_ctx*>(c);
  if (m->have_last) {
    // wait for the last call's work: its final event (or its stream)
    const hipError_t w = m->events_ok ? hipEventSynchronize(m->ev[6])
                                      : hipStreamSynchronize(m->last_stream);
    if (w == hipSuccess && m->events_ok) {
      // stages: ev0 sort ev1 build ev2 walk ev3 direct ev4 local ev7
      // multipole ev5 far ev6
      float t[7] = {0}, tl = 0;
      for (int i = 1; i <= 4; ++i) (void)hipEventElapsedTime(&t[i], m->ev[i - 1], m->ev[i]);
      (void)hipEventElapsedTime(&tl, m->ev[4], m->ev[7]);
      (void)hipEventElapsedTime(&t[5], m->ev[7], m->ev[5]);
      (void)hipEventElapsedTime(&t[6], m->ev[5], m->ev[6]);
      float tot = 0;
      (void)hipEventElapsedTime(&tot, m->ev[0], m->ev[6]);
      if (m->last_cev > 0) {
        // chunked lists: the emit passes count as walk, the direct, local
        // and multipole kernels are summed over the chunks
        float w = 0, d = 0, l = 0, q = 0;
        for (int k = 0; k < m->last_cev; ++k) {
          float a = 0, b = 0, e = 0, f = 0;
          (void)hipEventElapsedTime(&a, m->cev[4 * k], m->cev[4 * k + 1]);
          (void)hipEventElapsedTime(&b, m->cev[4 * k + 1], m->cev[4 * k + 2]);
          (void)hipEventElapsedTime(&e, m->cev[4 * k + 2], m->cev[4 * k + 3]);
          (void)hipEventElapsedTime(&f, m->cev[4 * k + 3], m->cev[4 * k + 4]);
          w += a;
          d += b;
          l += e;
          q += f;
        }
        t[3] += w;
        t[4] = d;
        tl = l;
        t[5] = q;
      }
      m->stats.ms_m2l = tl;
      m->stats.ms_sort = t[1];
      m->stats.ms_build = t[2];
      m->stats.ms_walk = t[3];
      m->stats.ms_p2p = t[4];
      m->stats.ms_m2p = t[5];
      m->stats.ms_far = t[6];
      m->stats.ms_total = tot;
    }
    unsigned long long pr[2] = {0, 0};
    if (w == hipSuccess) {
      std::memcpy(pr, m->host_buf + kHostPairs, sizeof(pr));
      m->stats.p2p_pairs = (int64_t)pr[0];
      m->stats.m2p_pairs = (int64_t)pr[1];
      m->stats.flops_p2p = (double)pr[0] * kP2PFlops;
      m->stats.flops_m2p = (double)pr[1] * m2p_flops(m->p.order);
      unsigned long long sl[6];
      std::memcpy(sl, m->host_buf + kHostSlots, sizeof(sl));
      m->stats.m2p_lanes_main = (int64_t)sl[0];
      m->stats.m2p_lanes_tail = (int64_t)sl[1];
      m->stats.m2p_pairs_tail = (int64_t)sl[2];
      m->stats.m2l_pairs = (int64_t)sl[4];
      settle_entries(m);
      m->stats.flops_m2l = (double)sl[3] * m2l_flops(m->p.order, m->p.local_order) +
                           (double)sl[5] * l2p_flops(m->p.local_order);
    }
  }
  *out = m->stats;
  return HOT_OK;
}

hot_status hot_debug_sizes(const hot_ctx* c, int64_t* n, int64_t* ncells, int64_t* ngroups,
                           int64_t* p2p_entries, int64_t* m2p_entries) {
  if (!c || !c->have_last) {
    g_err = "no previous hot_forces call";
    return HOT_EINVAL;
  }
  hot_ctx* m = const_cast<hot_ctx*>(c);
  HOT_CHECK(hipStreamSynchronize(m->last_stream), "sync");
  settle_entries(m);
  if (n) *n = (int64_t)c->last_n;
  if (ncells) *ncells = c->last_ncells;
  if (ngroups) *ngroups = c->last_ngroups;
  if (p2p_entries) *p2p_entries = c->stats.p2p_entries;
  if (m2p_entries) *m2p_entries = c->stats.m2p_entries;
  return HOT_OK;
}

hot_status hot_debug_export(hot_ctx* c, void* ws, hot_debug* o) {
  if (!c || !c->have_last || !o || !ws) {
    g_err = "no previous hot_forces call or NULL argument";
    return HOT_EINVAL;
  }
  if (c->last_chunks != 1 && (o->p2p_offset || o->p2p_entry || o->m2p_offset || o->m2p_entry ||
                              o->m2l_offset || o->m2l_entry)) {
    g_err = "the last evaluation processed its lists in chunks; they are not all in memory";
    return HOT_EINVAL;
  }
  const Plan& P = c->last_plan;
  hipStream_t s = c->last_stream;
  HOT_CHECK(hipStreamSynchronize(s), "sync");
  const size_t n = c->last_n, nc = c->last_ncells, ng = c->last_ngroups;
  auto cp = [&](void* dst, size_t off, size_t bytes) -> hipError_t {
    if (!dst || bytes == 0) return hipSuccess;
    return hipMemcpy(dst, at<char>(ws, off), bytes, hipMemcpyDeviceToHost);
  };
  HOT_CHECK(cp(o->sorted_keys, P.o_key[0], 8 * n), "export");
  HOT_CHECK(cp(o->perm, P.o_idx[0], 4 * n), "export");
  HOT_CHECK(cp(o->cell_key, P.o_c_key, 8 * nc), "export");
  HOT_CHECK(cp(o->cell_level, P.o_c_level, 4 * nc), "export");
  HOT_CHECK(cp(o->cell_first, P.o_c_first, 4 * nc), "export");
  HOT_CHECK(cp(o->cell_count, P.o_c_count, 4 * nc), "export");
  if (o->cell_com || o->cell_mass) {
    std::vector<double> w(4 * nc), mm(4 * nc);
    HOT_CHECK(cp(w.data(), P.o_c_walk, 32 * nc), "export");
    HOT_CHECK(cp(mm.data(), P.o_c_mmx, 32 * nc), "export");
    for (size_t i = 0; i < nc; ++i) {
      if (o->cell_com)
        for (int a = 0; a < 3; ++a) o->cell_com[a * nc + i] = w[4 * i + a];
      if (o->cell_mass) o->cell_mass[i] = mm[4 * i];
    }
  }
  HOT_CHECK(cp(o->group_cell, P.o_g_cell, 4 * ng), "export");
  settle_entries(c);
  const size_t tp = c->stats.p2p_entries;
  const bool local = local_on(c->p);
  std::vector<size_t> raw;
  std::vector<int64_t> packed;
  for (int kind = 0; kind < 3; ++kind) {
    int64_t* ooff = kind == 2 ? o->m2l_offset : kind ? o->m2p_offset : o->p2p_offset;
    uint32_t* oent = kind == 2 ? o->m2l_entry : kind ? o->m2p_entry : o->p2p_entry;
    if (!ooff && !oent) continue;
    if (kind == 2 && !local) {
      if (ooff)
        for (size_t g = 0; g <= ng; ++g) ooff[g] = 0;
      continue;
    }
    HOT_CHECK(list_layout(c, ws, kind, raw, packed), "export");
    if (ooff) std::copy(packed.begin(), packed.end(), ooff);
    if (!oent || packed[ng] == 0) continue;
    if (kind == 0) {
      HOT_CHECK(cp(oent, P.o_list, 4 * tp), "export");
      continue;
    }
    // the accepted-cell region: a multipole entry is the last word of its
    // 16-byte record, a local entry a word of its own; packed in group order
    const size_t acc = c->last_accepted;
    std::vector<uint32_t> rec(4 * acc);
    HOT_CHECK(cp(rec.data(), P.o_list + 4 * ((tp + 3) & ~size_t(3)), 16 * acc), "export");
    for (size_t g = 0; g < ng; ++g)
      for (int64_t i = 0; i < packed[g + 1] - packed[g]; ++i)
        oent[packed[g] + i] =
            kind == 2 ? rec[raw[g] + (size_t)i] : rec[4 * (raw[g] + (size_t)i) + 3];
  }
  return HOT_OK;
}

hot_status hot_cell_lookup(hot_ctx* c, void* ws, size_t nq, const uint64_t* keys, int32_t* cells,
                           void* stream) {
  if (!c || !c->have_last || !ws) {
    g_err = "no previous force evaluation or NULL workspace";
    return HOT_EINVAL;
  }
  if (nq == 0) return HOT_OK;
  if (!keys || !cells) {
    g_err = "NULL pointer argument";
    return HOT_EINVAL;
  }
  if (ws != c->last_ws) {
    g_err = "the workspace is not that of the last evaluation";
    return HOT_EINVAL;
  }
  const Plan& P = c->last_plan;
  HOT_CHECK(hash_lookup(at<uint64_t>(ws, P.o_h_key), at<uint32_t>(ws, P.o_h_val), P.hcap, keys, nq,
                        cells, (hipStream_t)stream),
            "key lookup");
  return HOT_OK;
}

hot_status hot_debug_list_range(hot_ctx* c, void* ws, int kind, int64_t first, int64_t count,
                                uint32_t* out) {
  if (!c || !c->have_last || !ws || (count > 0 && !out) || kind < 0 || kind > 2 ||
      first < 0 || count < 0) {
    g_err = "no previous hot_forces call or bad argument";
    return HOT_EINVAL;
  }
  if (c->last_chunks != 1) {
    g_err = "the last evaluation processed its lists in chunks; they are not all in memory";
    return HOT_EINVAL;
  }
  const Plan& P = c->last_plan;
  HOT_CHECK(hipStreamSynchronize(c->last_stream), "sync");
  settle_entries(c);
  const int64_t total = kind == 2 ? c->stats.m2l_entries
                      : kind     ? c->stats.m2p_entries
                                 : c->stats.p2p_entries;
  if (first + count > total) {
    g_err = "entry range beyond the list";
    return HOT_EINVAL;
  }
  if (count == 0) return HOT_OK;
  if (kind == 0) {
    HOT_CHECK(hipMemcpy(out, at<uint32_t>(ws, P.o_list) + first, 4 * (size_t)count,
                        hipMemcpyDeviceToHost),
              "export");
    return HOT_OK;
  }
  // a multipole entry is the last word of its 16-byte record, a local entry a
  // word of its own; copy group by group from the packed index range
  std::vector<size_t> raw;
  std::vector<int64_t> packed;
  HOT_CHECK(list_layout(c, ws, kind, raw, packed), "export");
  const size_t tp = (size_t)c->stats.p2p_entries;
  const uint32_t* reg = at<uint32_t>(ws, P.o_list) + ((tp + 3) & ~size_t(3));
  const size_t stride = kind == 2 ? 1 : 4, last = kind == 2 ? 0 : 3;
  size_t g = (size_t)(std::upper_bound(packed.begin(), packed.end(), first) - packed.begin()) - 1;
  for (int64_t i = first; i < first + count; ++g) {
    const int64_t take = std::min(packed[g + 1], first + count) - i;
    if (take <= 0) continue;
    HOT_CHECK(hipMemcpy2D(out + (i - first), 4,
                          reg + stride * (raw[g] + (size_t)(i - packed[g])) + last,
                          4 * stride, 4, (size_t)take, hipMemcpyDeviceToHost),
              "export");
    i += take;
  }
  return HOT_OK;
}

}  // extern "C"

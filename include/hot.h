/* libhot -- periodic tree-gravity force evaluation on one AMD Instinct MI355X
 * (gfx950), behind a plain C ABI.
 *
 * The method is the pure tree code of the paper's Sec. 2.1 ("2HOT"):
 * particles get 64-bit Morton keys, are sorted by key, a hashed oct-tree is
 * built over the sorted list, cells carry truncated Cartesian multipole
 * expansions, and groups of nearby sink particles share one interaction list
 * produced by a tree walk with a multipole acceptance test (the m x n
 * bundling of sinks and sources).  Periodic boundaries: the 27 nearest images
 * of the box are walked explicitly; every further image enters through
 * high-order local expansions of the Ewald-summed remainder about the centres
 * of the box's 8 octants (Sec. 2.1, the p=8 periodic local expansion), which
 * also subtracts the uniform background density.  A kick-drift-kick step wraps the force
 * evaluation, with fixed steps or with power-of-two block timesteps (Sec. 2.1:
 * the adaptive symplectic integrator).
 *
 * Conventions for every call
 * --------------------------
 *  - Arrays are device pointers (HIP global memory) owned by the caller,
 *    structure-of-arrays: positions are 3 x n FP64 (x[0..n), y[0..n),
 *    z[0..n)); accelerations 3 x n; masses and potentials n.  The element type
 *    of mass, acc, pot and vel is FP64 when hot_params.precision == HOT_FP64
 *    and FP32 when it is HOT_FP32; positions are always FP64.
 *  - Positions may lie anywhere in (-L, 2L) per axis; they are wrapped into
 *    [0, L) internally.  Values outside that range, NaN or Inf give
 *    HOT_EINVAL.  Masses must be >= 0.
 *  - Units: potential phi_i = -G sum_j m_j g(x_i - x_j) and acceleration
 *    a_i = -grad phi_i, with the softened kernel g (Plummer,
 *    g(r) = (|r|^2+eps^2)^(-1/2), or K1; see hot_params.kernel) on the 27
 *    nearest images and the unsoftened Ewald kernel (neutralising
 *    background) on all others; a particle's own periodic images contribute.
 *  - Scratch memory comes from the caller: every compute call takes a device
 *    workspace of at least hot_workspace_size_min(ctx, n) bytes (preferably
 *    hot_workspace_size(ctx, n)), aligned to 256
 *    bytes.  The library never allocates device memory in a compute call; it
 *    owns only the context (parameters, the Ewald table, a few device
 *    constants, a second HIP stream with two events, timing events and a
 *    small pinned host buffer), created by hot_create and released by
 *    hot_destroy.
 *  - Calls are enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*; NULL = the default stream).  A compute call synchronises that
 *    stream to size its launches: once per tree level (the next level's
 *    cell count), after the sink groups and after the walk's count pass
 *    (group and list totals); it returns after the last kernel is enqueued; outputs are ready once the
 *    stream is synchronised.  The force kernels' tail passes (the last <= 32
 *    targets of a sink group) run on the context's second stream, which
 *    waits for the caller's stream through an event before them, and the
 *    caller's stream waits for them through another event before anything
 *    that reads their results: all ordering stays on the device and follows
 *    the caller's stream.
 *  - Errors are status codes; nothing throws across the ABI.  A message for
 *    the last failure on the calling thread is in hot_last_error().  Inputs
 *    are never modified, except the in/out arrays of hot_kdk.
 *  - HOT_EOVERFLOW means a data-dependent capacity (cells, or the lists of a
 *    single sink group) did not fit in the workspace.  The context records what was
 *    needed; call hot_workspace_size again (it now returns a larger size),
 *    allocate that much and repeat the call.  Nothing was written to outputs.
 *  - One context may be used by one host thread at a time.
 */
#ifndef HOT_H
#define HOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HOT_OK = 0,
  HOT_EINVAL = 1,       /* bad argument or input value */
  HOT_ENOMEM = 2,       /* workspace smaller than hot_workspace_size() */
  HOT_EOVERFLOW = 3,    /* data-dependent capacity exceeded; resize, retry */
  HOT_EDEVICE = 4,      /* a HIP runtime call failed; see hot_last_error() */
  HOT_EUNSUPPORTED = 5  /* parameter combination not built into the library */
} hot_status;

typedef enum { HOT_FP64 = 0, HOT_FP32 = 1 } hot_precision;

/* Parameters of one simulation (paper Sec. 2.1; the opening angle and the
 * multipole order stand in for the paper's error-tolerance parameter). */
typedef struct {
  double box;      /* side L of the periodic cube, > 0 */
  double G;        /* gravitational constant */
  double eps;      /* Plummer softening length, >= 0 */
  double theta;    /* opening angle, 0 <= theta < 1; with err_tol == 0,
                      0 = exact direct sum */
  int order;       /* multipole order p of cells, 0..4 (2 = quadrupole,
                      4 = hexadecapole: the leaf-level expansions of Sec. 2.1) */
  int periodic;    /* 1 = periodic box, 0 = open boundaries (no images) */
  int leaf_max;    /* a cell with more particles is split (1..255) */
  int group_max;   /* sink groups: largest cells with at most this many
                      particles share an interaction list (1..4096) */
  int far_order;   /* order of the periodic far-field local expansion,
                      0..12 (the paper uses 8) */
  int precision;   /* hot_precision: FP64 throughout, or FP32 interaction
                      arithmetic on cell-relative coordinates with
                      compensated accumulation and FP64 positions, cell
                      centres of mass, moments and far field */
  double err_tol;  /* > 0: error-bound acceptance test (the paper's absolute
                      error tolerance, Sec. 2.1): a cell is accepted only
                      beyond the distance at which the Salmon & Warren bound
                      on its expansion's acceleration error, computed from
                      the cell's B_(p+1) = sum m |x - com|^(p+1) (exact at
                      leaves, bounded from the daughters above them) and its
                      extent, falls to err_tol (acceleration units); with
                      theta > 0 as well,
                      the larger of the two opening radii applies.
                      0 = opening angle only.  Finite, >= 0.  A
                      fixed fraction (about 0.1) of the rms acceleration
                      of the previous step keeps the rms force error near
                      1e-3 of the rms acceleration. */
  int kernel;      /* softening kernel (paper Sec. 2.1): HOT_KERNEL_PLUMMER,
                      or HOT_KERNEL_K1, Dehnen's compensating kernel, read as
                      the compact density ~ (1 - x^2)^2 (1 - 11 x^2/5),
                      x = r/h < 1, of radius h = (945/256) eps, so that eps
                      is its Plummer-equivalent softening (equal central
                      potential); exactly Newtonian beyond h.  With K1,
                      multipole interactions use the Newtonian expansion and
                      a cell is accepted only if all its particles lie
                      farther than h from every target of the group; eps
                      must be > 0.  The adjoints (hot_vjp, hot_kdk_vjp) are
                      built for Plummer softening only. */
  int local_order; /* 0, 2 or 4.  > 0 (with local_tol > 0): group-level
                      local expansions (the dual-tree blocking of source
                      cells with the sinks of a sink group, Sec. 2.1).  An
                      accepted cell whose order-p expansion, re-expanded to
                      this order about the group's centre c (the middle of
                      its tight box), keeps the truncation's acceleration
                      error bound
                        G m t^q ((q+2) - (q+1) t) / (u^2 (1-t)^2) <= local_tol,
                      u = |c - z| - b, t = a/u < 1 (m, z, b: the cell's
                      mass, image-shifted centre of mass and extent bound;
                      a: half the diagonal of the group's tight box), is
                      evaluated once per group instead of once per sink;
                      each sink then evaluates the local polynomial.  0 =
                      every accepted cell is evaluated at every sink.  The
                      adjoints do not support it (HOT_EUNSUPPORTED). */
  double local_tol; /* acceleration units, finite, >= 0; 0 = no local
                      expansions */
} hot_params;

#define HOT_KERNEL_PLUMMER 0
#define HOT_KERNEL_K1 1

/* Per-call statistics of the last compute call on a context. */
typedef struct {
  int64_t n;              /* particles */
  int64_t ncells;         /* tree cells */
  int64_t ngroups;        /* sink groups */
  int64_t nlevels;        /* deepest level + 1 */
  int64_t p2p_entries;    /* direct-interaction list entries (leaf x image) */
  int64_t m2p_entries;    /* multipole list entries (cell x image) */
  int64_t p2p_pairs;      /* particle-particle interactions evaluated */
  int64_t m2p_pairs;      /* particle-cell interactions evaluated */
  double flops_p2p;       /* algorithmic flops of the direct kernel */
  double flops_m2p;       /* algorithmic flops of the multipole kernel */
  double ms_total;        /* stream time of the whole call (ms) */
  double ms_sort;         /* keys + sort + gather */
  double ms_build;        /* tree levels, moments, groups */
  double ms_walk;         /* both walk passes */
  double ms_p2p;          /* direct kernel */
  double ms_m2p;          /* multipole kernel (walk emit, direct and
                             multipole times are summed over the list chunks
                             when there are at most 64 of them; beyond that
                             ms_p2p holds the whole chunk loop and ms_m2p 0) */
  double ms_far;          /* far field + unpermute */
  size_t ws_bytes_needed; /* workspace that would have sufficed */
  int64_t kdk_steps_done; /* steps hot_kdk completed in its last call */
  int64_t list_chunks;    /* group ranges the interaction lists were processed
                             in (1 unless they exceeded the list region) */
  int64_t m2p_lanes_main; /* lane-steps of the multipole kernel's main pass
                             (64 per pass of more than 32 targets per list
                             entry); m2p_pairs / (this + m2p_lanes_tail) is
                             its lane use */
  int64_t m2p_lanes_tail; /* lane-steps of its tail pass (the last pass of at
                             most 32 targets: 8, 16 or 32 lanes per entry) */
  int64_t m2p_pairs_tail; /* particle-cell interactions of the tail pass */
  int64_t m2l_entries;    /* local-list entries (cell x image) */
  int64_t m2l_pairs;      /* particle-cell interactions they stand for (the
                             entries times the sinks of their groups) */
  double flops_m2l;       /* algorithmic flops of the local expansions
                             (re-expansions and their evaluation at sinks) */
  double ms_m2l;          /* local-expansion kernel (summed over the list
                             chunks like ms_m2p) */
} hot_stats;

/* Host copies of the internal structures of the last hot_forces call, for
 * checking against an independent implementation.  The caller passes host
 * buffers of the sizes given by hot_debug_sizes (any may be NULL to skip).
 * Cells are in the library's internal order; lists are grouped per sink
 * group in the internal group order.  List entries encode (image << 27) |
 * cell, image = (nx+1)*9 + (ny+1)*3 + (nz+1). */
typedef struct {
  uint64_t* sorted_keys;  /* n */
  uint32_t* perm;         /* n: sorted position -> original index */
  uint64_t* cell_key;     /* ncells: Morton key with placeholder bit */
  int32_t* cell_level;    /* ncells */
  int32_t* cell_first;    /* ncells: first sorted particle */
  int32_t* cell_count;    /* ncells */
  double* cell_com;       /* 3 x ncells SoA */
  double* cell_mass;      /* ncells */
  int32_t* group_cell;    /* ngroups: cell index of each sink group */
  int64_t* p2p_offset;    /* ngroups + 1 */
  uint32_t* p2p_entry;    /* p2p_entries */
  int64_t* m2p_offset;    /* ngroups + 1 */
  uint32_t* m2p_entry;    /* m2p_entries */
  int64_t* m2l_offset;    /* ngroups + 1: local lists (local_order > 0) */
  uint32_t* m2l_entry;    /* hot_stats.m2l_entries */
} hot_debug;

typedef struct hot_ctx hot_ctx;

/* Create a context.  Validates the parameters (HOT_EINVAL), builds the
 * far-field Ewald table on the host in FP64 and uploads it (HOT_EDEVICE on
 * a HIP failure), and creates the context's second stream (default
 * priority) and its two events on the current HIP device; if those cannot
 * be created the tail passes run on the caller's stream after the main
 * passes instead.  *out is NULL on failure. */
hot_status hot_create(const hot_params* params, hot_ctx** out);

/* Release a context (NULL is allowed). */
void hot_destroy(hot_ctx* ctx);

/* Preferred bytes of device workspace for any compute call on n particles:
 * every structure, and room for all interaction lists at once (up to 4 GiB
 * of lists).  Grows
 * after a call that needed more, so the next call fits.  0 if ctx is NULL. */
size_t hot_workspace_size(const hot_ctx* ctx, size_t n);

/* Smallest workspace the given calls accept for n particles (calls: a
 * bitwise OR of HOT_CALL_*): the structures those calls use plus 1 MiB of
 * list space.  hot_forces needs only the forward structures; hot_kdk adds
 * state snapshots; hot_vjp adds the adjoint's cotangent structures;
 * hot_kdk_vjp needs both.  Between this and hot_workspace_size the
 * interaction lists are built and consumed in chunks of consecutive sink
 * groups (paper Sec. 2.1: groups are independent), which gives the same
 * results.  0 if ctx is NULL. */
#define HOT_CALL_FORCES 1u
#define HOT_CALL_KDK 2u
#define HOT_CALL_VJP 4u
#define HOT_CALL_KDK_VJP 8u
size_t hot_workspace_size_min(const hot_ctx* ctx, size_t n, unsigned calls);

/* Accelerations and potentials of n particles (paper Sec. 2.1: the force
 * evaluation of one timestep).
 *   pos   device, 3 x n FP64 SoA, read only
 *   mass  device, n, FP64 or FP32 (precision), read only
 *   acc   device, 3 x n (precision), written
 *   pot   device, n (precision), written; may be NULL
 *   workspace, ws_bytes  device scratch (>= hot_workspace_size)
 *   stream  hipStream_t or NULL
 * Returns HOT_OK, HOT_EINVAL (n == 0 is allowed and does nothing; NULL
 * pointers with n > 0, non-finite or out-of-range positions), HOT_ENOMEM,
 * HOT_EOVERFLOW or HOT_EDEVICE. */
hot_status hot_forces(hot_ctx* ctx, size_t n, const double* pos, const void* mass, void* acc,
                      void* pot, void* workspace, size_t ws_bytes, void* stream);

/* hot_forces without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as hot_forces,
 * bit-identical results; the scratch is a fixed 256 MiB array in device
 * memory that the library holds on every GPU it has run on (allocated when
 * the library's code object is loaded there, released at process exit).
 * Nothing is allocated: no hipMalloc, hipFree or allocating library call.
 * The forward structures for n particles must fit the array (FP32 mode,
 * order 4, leaf 16: about 750,000 particles; less in FP64 mode or with
 * smaller leaves); larger n gives HOT_ENOMEM with the size it would need.
 * The interaction lists take the rest and are built and consumed in chunks
 * of sink groups when they do not fit (same results).  The call runs on the
 * context's device, which must be current (HOT_EINVAL otherwise).  Every
 * call on one GPU, from any context or thread, shares that GPU's array and
 * leaves its contents behind: calls that overlap in time on one GPU (other
 * host threads, or streams that are not ordered after each other) race and
 * give undefined results; calls ordered on one stream are safe.  A later
 * hot_vjp_after_forces does not reuse this call's tree. */
hot_status hot_forces_noalloc(hot_ctx* ctx, size_t n, const double* pos, const void* mass,
                              void* acc, void* pot, void* stream);

/* nsteps fixed-step kick-drift-kick leapfrog steps of length dt:
 * v += a dt/2; x = wrap(x + v dt); a = forces(x); v += a dt/2.
 *   pos   device, 3 x n FP64, in/out (wrapped into [0, L) on return)
 *   vel   device, 3 x n (precision), in/out
 *   mass  device, n (precision), read only
 *   acc   device, 3 x n (precision), in/out: on entry the accelerations at
 *         pos if (flags & HOT_ACC_VALID), otherwise they are computed first;
 *         on return the accelerations at the final positions
 *   pot   device, n (precision) or NULL: potentials at the final positions
 * Same errors as hot_forces.  A failing force evaluation leaves pos, vel and
 * acc at the end of the last completed step (restored from a snapshot in the
 * workspace); hot_get_stats reports that step count as kdk_steps_done, and
 * acc is valid there whenever kdk_steps_done > 0 or HOT_ACC_VALID was given,
 * so after HOT_EOVERFLOW the caller resizes the workspace and repeats the
 * call for the remaining steps.  With HOT_KDK_NO_SNAPSHOT no snapshot is
 * kept (the workspace needs only hot_workspace_size_min(HOT_CALL_FORCES),
 * 36 bytes per particle less), and after a failure pos and vel are
 * undefined. */
#define HOT_ACC_VALID 1u
#define HOT_KDK_NO_SNAPSHOT 2u
hot_status hot_kdk(hot_ctx* ctx, size_t n, double* pos, void* vel, const void* mass, void* acc,
                   void* pot, double dt, int nsteps, unsigned flags, void* workspace,
                   size_t ws_bytes, void* stream);

/* The kick-drift-kick steps of hot_kdk in comoving coordinates of an
 * expanding background (paper Sec. 2.1: the symplectic integrator; Sec. 3:
 * comoving cosmological volumes in a flat background with omega_m 0.295 and
 * omega_lambda 0.705).  pos are comoving
 * positions in the periodic box, vel the canonical momenta per unit mass
 * p = a^2 dx/dt, and the force evaluation is the peculiar one the tree
 * computes from comoving positions and masses (its periodic sum subtracts
 * the mean density).  The equations of motion dx/dt = p / a^2 and
 * dp/dt = acc / a give, over a step from a_k to a_k+1 = a_k + da in the
 * scale factor, with a_h = a_k + da/2:
 *   p += acc K(a_k, a_h); x = wrap(x + p D(a_k, a_k+1)); acc = forces(x);
 *   p += acc K(a_h, a_k+1),
 * K(a1, a2) = int da / (a^2 H(a)) and D(a1, a2) = int da / (a^3 H(a))
 * (hot_comoving_factors), H(a) = h0 sqrt(omega_m a^-3 + omega_k a^-2 +
 * omega_l), omega_k = 1 - omega_m - omega_l.  Time is in units of the
 * context's G: h0 is the Hubble constant in those units (with G = 1 and the
 * mean comoving density rho, 4 pi rho / 3 = omega_m h0^2 / 2 holds for a
 * consistent background; the library does not impose it).
 *   a0 > 0   the scale factor at the start; da the step in it (any sign;
 *            every a_k must stay > 0 and H^2 > 0 on the path)
 *   omega_m, omega_l, h0 > 0  the background
 * Other arguments, flags, errors and the failure behaviour as hot_kdk
 * (kdk_steps_done counts the completed steps). */
hot_status hot_kdk_comoving(hot_ctx* ctx, size_t n, double* pos, void* vel, const void* mass,
                            void* acc, void* pot, double a0, double da, int nsteps,
                            double omega_m, double omega_l, double h0, unsigned flags,
                            void* workspace, size_t ws_bytes, void* stream);

/* The kick and drift factors of hot_kdk_comoving over [a1, a2] (a1, a2 > 0):
 * out[0] = K = int_a1^a2 da / (a^2 H(a)), out[1] = D = int_a1^a2 da /
 * (a^3 H(a)), by Gauss-Legendre quadrature in ln a (16 nodes per panel,
 * panels at most 0.05 wide in ln a).  Host-only; touches no GPU.  HOT_EINVAL
 * on non-positive or non-finite a1, a2, h0, a non-finite omega, or
 * H^2 <= 0 somewhere in [a1, a2]. */
hot_status hot_comoving_factors(double a1, double a2, double omega_m, double omega_l, double h0,
                                double* out);

/* Block (multiple) timesteps: nsteps steps of length dt of the paper's
 * adaptive symplectic integrator (Sec. 2.1), read as hierarchical
 * kick-drift-kick on power-of-two rungs.  Particle i advances in steps of
 * dt / 2^rung[i], rung 0..max_rung; time moves in substeps of
 * dt / 2^max_rung, through which every particle drifts.  At each substep
 * boundary the particles whose step ends there get new accelerations (one
 * force evaluation whose lists and kernels cover only the sink groups that
 * hold such a particle; the tree is built from all particles at the current
 * positions), a closing half kick, and, unless HOT_RUNG_FIXED, a new rung:
 * the largest step dt / 2^r not above eta sqrt(eps / |a|), but no larger
 * than the steps that can start at this boundary.  Particles starting a
 * step get an opening half kick with their current acceleration.  A
 * boundary where no particle is due only drifts (the largest rung is read
 * back after every rung update, one stream synchronisation).  With fixed
 * rungs the scheme is time-reversible; max_rung = 0 is hot_kdk's leapfrog.
 *   pos, vel, mass, acc, pot  as hot_kdk (acc/pot of a particle are those of
 *         its last force evaluation)
 *   rung  device, n uint8, in/out: on entry the rungs if (flags &
 *         HOT_RUNG_VALID), otherwise computed from acc first; on return the
 *         rungs for the next step
 *   dt    the step of rung 0; max_rung 0..16; eta > 0 the step parameter
 * flags: HOT_ACC_VALID, HOT_RUNG_VALID, HOT_RUNG_FIXED.  The workspace must
 * hold hot_workspace_size_min(ctx, n, HOT_CALL_FORCES).  Errors as
 * hot_forces; after a failure pos, vel, acc and rung are undefined (no
 * snapshot is kept; size the workspace with a hot_forces call on the same
 * particles first).  hot_get_stats reports the last substep's force
 * evaluation and the completed steps. */
#define HOT_RUNG_VALID 4u
#define HOT_RUNG_FIXED 8u
hot_status hot_kdk_block(hot_ctx* ctx, size_t n, double* pos, void* vel, const void* mass,
                         void* acc, void* pot, uint8_t* rung, double dt, int max_rung, double eta,
                         int nsteps, unsigned flags, void* workspace, size_t ws_bytes,
                         void* stream);

/* Vector-Jacobian product of hot_forces (an extension beyond the paper):
 * given cotangents gacc (3 x n) and gpot (n, or NULL for zero) of the
 * outputs, returns
 *   xbar = (d acc/d pos)^T gacc + (d pot/d pos)^T gpot   (3 x n FP64)
 *   mbar = (d acc/d mass)^T gacc + (d pot/d mass)^T gpot (n, precision)
 * for the tree approximation of the forces at the same parameters (the
 * exact derivative of the direct sum when theta == 0).  gacc, gpot and mbar
 * use the precision type; xbar is FP64.  Same errors as hot_forces;
 * HOT_EUNSUPPORTED if the build lacks the adjoint for the order, with the
 * K1 softening kernel, or with group-level local expansions. */
hot_status hot_vjp(hot_ctx* ctx, size_t n, const double* pos, const void* mass, const void* gacc,
                   const void* gpot, double* xbar, void* mbar, void* workspace, size_t ws_bytes,
                   void* stream);

/* hot_vjp for a backward pass that follows its forward evaluation (an
 * extension beyond the paper).  When the last evaluation that completed on
 * this context (by any entry point: a force evaluation of hot_forces or
 * hot_kdk, or an adjoint) ran with the same pos, mass, n, workspace (pointer
 * and size) and stream, processed its interaction lists in one pass, and
 * those lists lie below the adjoint's workspace regions, the keys, tree,
 * groups and lists it left in the workspace are used as they are: the
 * adjoint runs on the same lists, so the result is bit-identical to
 * hot_vjp's.  Otherwise it is hot_vjp.  The caller guarantees that pos and
 * mass still hold the values of that evaluation and that nothing else wrote
 * the workspace in between (no other context shares it); the library
 * compares only pointers and sizes.  Arguments, results and errors as
 * hot_vjp. */
hot_status hot_vjp_after_forces(hot_ctx* ctx, size_t n, const double* pos, const void* mass,
                                const void* gacc, const void* gpot, double* xbar, void* mbar,
                                void* workspace, size_t ws_bytes, void* stream);

/* Reverse-mode derivative of nsteps hot_kdk steps (an extension beyond the
 * paper), for differentiating a trajectory with per-step checkpoints: only
 * the positions are stored, and the tree of every step is rebuilt here.
 *   pos_ckpt  device, (nsteps + 1) x 3 x n FP64, read only: the positions at
 *             the start of each step and after the last one, as hot_kdk
 *             produced them
 *   mass      device, n (precision), read only
 *   xbar      device, 3 x n FP64, in/out: on entry the cotangent of the final
 *             positions, on return that of the initial positions
 *   vbar      device, 3 x n (precision), in/out: likewise for velocities
 *   mbar      device, n (precision) or NULL: written with the cotangent of
 *             the masses
 * The force derivatives are those of hot_vjp (exact for theta == 0), taken
 * once per stored position: the closing kick of one step and the opening
 * kick of the next share it.  nsteps == 0 leaves xbar, vbar unchanged and
 * zeroes mbar.  Same errors as hot_forces; on any failure xbar and vbar are
 * restored to their values on entry, so the call can be repeated. */
hot_status hot_kdk_vjp(hot_ctx* ctx, size_t n, int nsteps, const double* pos_ckpt,
                       const void* mass, double dt, double* xbar, void* vbar, void* mbar,
                       void* workspace, size_t ws_bytes, void* stream);

/* Statistics of the last compute call on ctx.  Waits on the host until that
 * call's device work has finished (it synchronises on the call's final
 * event, or on its stream if the context has no events), then reports the
 * stage times of the context's HIP events and the pair counters the call
 * copied to the context's pinned host memory.  It reads no workspace memory,
 * so the workspace of that call may already be released. */
hot_status hot_get_stats(const hot_ctx* ctx, hot_stats* out);

/* Sizes for hot_debug_export after the last hot_forces call.  Synchronises
 * that call's stream (the split of accepted cells into multipole and local
 * entries is known once its work has finished). */
hot_status hot_debug_sizes(const hot_ctx* ctx, int64_t* n, int64_t* ncells, int64_t* ngroups,
                           int64_t* p2p_entries, int64_t* m2p_entries);

/* Copy the internal structures of the last hot_forces call to host buffers
 * (synchronises the stream of that call).  The workspace of that call must
 * still hold its contents.  HOT_EINVAL if no hot_forces call preceded, or if
 * list buffers are requested after a call that processed its lists in chunks
 * (hot_stats.list_chunks > 1). */
hot_status hot_debug_export(hot_ctx* ctx, void* workspace, hot_debug* out);

/* Look up cells by key in the hashed oct-tree of the last force evaluation
 * (paper Sec. 2.1: a key is translated into its cell's storage through a
 * hash table).  Every evaluation builds the table from its cells: open
 * addressing, linear probing, at least twice as many slots as cells.
 *   workspace  the workspace of that evaluation, still holding its contents
 *   keys       device, nq uint64 cell keys (Morton key with placeholder bit:
 *              root 1, daughter = parent << 3 | octant)
 *   cells      device, nq int32, written: the cell's index in the library's
 *              cell order (the order of hot_debug's cell arrays), or -1 if
 *              the tree has no such cell
 * Enqueued on stream; results are ready once it is synchronised.
 * HOT_EINVAL if no evaluation preceded, on NULL pointers with nq > 0, or if
 * workspace is not the last evaluation's. */
hot_status hot_cell_lookup(hot_ctx* ctx, void* workspace, size_t nq, const uint64_t* keys,
                           int32_t* cells, void* stream);

/* Copy count interaction-list entries of the last hot_forces call, starting
 * at entry first of the whole list of the given kind (0 = direct, 1 =
 * multipole, 2 = local; the per-group ranges are the offsets
 * hot_debug_export gives),
 * to the host buffer out (count uint32 values, encoded as in hot_debug).
 * For checking selected sink groups' lists of a large evaluation without
 * copying all of them.  Synchronises the stream of that call.  HOT_EINVAL
 * if no hot_forces call preceded, if its lists were processed in chunks, or
 * if the range lies beyond the list. */
hot_status hot_debug_list_range(hot_ctx* ctx, void* workspace, int kind, int64_t first,
                                int64_t count, uint32_t* out);

/* A Taylor table of the periodic far field, as built by hot_create:
 * Tpsi_s = d^s Psi(r0) / s!, |s| <= 2 far_order, of the periodic remainder
 * Psi = Ewald potential minus the 27 nearest bare images (paper Sec. 2.1:
 * the periodic local expansion), about the point r0 = (dx, dy, dz) L/2 with
 * offset = (dx+1)*9 + (dy+1)*3 + (dz+1), dx, dy, dz in {-1, 0, 1}: the
 * offsets between the centres of the 8 octants about which the far field is
 * expanded.  Multi-indices (a,b,c) are ordered by total degree, then a
 * descending, then b descending.  out: host array of count >=
 * (D+1)(D+2)(D+3)/6 doubles, D = 2 far_order.  Host-only; touches no GPU.
 * HOT_EINVAL on bad arguments. */
hot_status hot_far_table(int far_order, double box, int offset, double* out, size_t count);

/* Message describing the last failure on the calling thread ("" if none). */
const char* hot_last_error(void);

/* Library version string. */
const char* hot_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HOT_H */

/* libhotref -- exact periodic accelerations and potentials of selected
 * target particles by direct Ewald summation, FP64, on one AMD Instinct
 * MI355X (gfx950).
 *
 * A measurement instrument beside libhot (include/hot.h), not part of its
 * force path: it gives the rms force error of a tree evaluation (the paper's
 * accuracy measure, Sec. 2.1: absolute force errors against the rms
 * acceleration) at sizes no CPU reference reaches, such as one GPU's share of
 * the paper's 10240^3 run (Sec. 3).  It shares no code with libhot.
 *
 * What it computes, for each target i (an index into the particle arrays):
 *   phi_i = -G sum_j m_j psi(x_i - x_j)   (j = i: its periodic images only)
 *   a_i   = -grad_i phi_i
 * where psi is the periodic Green's function of the unit-L cube with a
 * neutralising uniform background (Ewald summation, split 8/L), softened
 * Plummer-wise, 1/|R| -> (|R|^2 + eps^2)^(-1/2), on every image closer than
 * 0.7 L to the target.  Images beyond that stay unsoftened; the difference
 * is below 3 eps^2/L^2 of each such term.  Positions may lie anywhere
 * (separations are reduced to the nearest image); distinct particles must
 * not coincide.  The series are truncated at about 1e-14 of the result.
 *
 * Conventions as libhot: device pointers owned by the caller, SoA, calls
 * enqueued on the caller's HIP stream (NULL = default stream), status codes,
 * a thread-local message in hotref_last_error().  hotref_ewald synchronises
 * its stream once (after uploading its small reciprocal-vector table and
 * reading back the total mass), then returns with the rest enqueued.
 */
#ifndef HOTREF_H
#define HOTREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HOTREF_OK = 0,
  HOTREF_EINVAL = 1,  /* bad argument, or scratch too small */
  HOTREF_EDEVICE = 2  /* a HIP runtime call failed */
} hotref_status;

/* Bytes of device scratch hotref_ewald needs for n particles and ntargets
 * targets (a few tens of MB at n = 2^30, ntargets = 10^3). */
size_t hotref_scratch_size(size_t n, size_t ntargets);

/* Accelerations and potentials of ntargets targets.
 *   pos      device, 3 x n FP64 SoA, read only
 *   mass     device, n, FP32 (mass_fp32 != 0) or FP64, read only
 *   targets  device, ntargets int64 indices in [0, n), read only
 *   box, G, eps  side L > 0, gravitational constant, softening >= 0
 *   acc      device, 3 x ntargets FP64 SoA, written
 *   pot      device, ntargets FP64, written; may be NULL
 *   scratch  device, >= hotref_scratch_size(n, ntargets) bytes
 * HOTREF_EINVAL on NULL pointers, n == 0, bad box/eps/G or small scratch;
 * ntargets == 0 does nothing.  Target indices are not checked. */
hotref_status hotref_ewald(size_t n, const double* pos, const void* mass, int mass_fp32,
                           size_t ntargets, const int64_t* targets, double box, double G,
                           double eps, double* acc, double* pot, void* scratch,
                           size_t scratch_bytes, void* stream);

/* Vector-ALU throughput probe: runs one kind of wavefront-wide independent
 * arithmetic chains on the default stream (kind 0: FP32 fma, 1: FP32 mul,
 * 2: FP32 add, 3: FP32 fma/mul/add in turn, 4: FP32 fma with one reciprocal
 * square root per 16 operations, 5: FP64 fma, 6: FP32 fma accumulating
 * into the chain), repeats times after one
 * 20 warm-up launches, and reports the mean ms per launch and the wave instructions of
 * one launch.  scratch: device, >= hotref_valu_probe_scratch() bytes
 * (written).  Synchronises the default stream.  It measures the issue
 * ceiling the force kernels' unpacked FP32 arithmetic runs against. */
size_t hotref_valu_probe_scratch(void);
hotref_status hotref_valu_probe(int kind, void* scratch, size_t scratch_bytes, int repeats,
                                double* ms, double* wave_instructions);

/* Message describing the last failure on the calling thread ("" if none). */
const char* hotref_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HOTREF_H */

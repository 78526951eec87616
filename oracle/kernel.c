/* Softening kernels of the pair interaction (oracle; test infrastructure).
 *
 * A pair at separation r contributes m g(r) to Phi and m (y - x) f(r) to
 * grad Phi, where a point mass has the potential -G m g(r) and the
 * acceleration -G m r f(r) toward it.
 *
 * Plummer (kernel 0): g = (r^2 + eps^2)^(-1/2), f = g^3.
 *
 * Dehnen's compensating kernel K1 (kernel 1; paper Sec. 2.1 uses it for
 * small-scale force softening and cites Dehnen 2001, without giving its
 * form).  Read here as the compact-support density
 *     rho(r) = C (1 - x^2)^2 (1 - 11 x^2 / 5),   x = r/h < 1,   0 beyond,
 * the (1 - x^2)^2 kernel with the term that makes its second moment vanish
 * (int rho r^2 dV = 0: "compensating"), normalised to unit mass.  The force
 * follows from the enclosed mass M(x) = int_0^r 4 pi r'^2 rho dr', worked out
 * by hand from that density:
 *     M(x) = (525 x^3 - 1323 x^5 + 1215 x^7 - 385 x^9) / 32,   M(1) = 1,
 *     f(r) = M(x) / r^3 = (525 - 1323 x^2 + 1215 x^4 - 385 x^6) / (32 h^3),
 * and the potential from g(r) = 1/h + int_r^h r' f(r') dr':
 *     g(r) = (945 - 2100 x^2 + 2646 x^4 - 1620 x^6 + 385 x^8) / (256 h).
 * Beyond h both are exactly Newtonian (g = 1/r, f = 1/r^3).  The paper
 * quotes softening as a "Plummer equivalent" length eps; here h is set so
 * that the central potential equals Plummer's, g(0) = 945/(256 h) = 1/eps,
 * i.e. h = (945/256) eps.
 */
#include <math.h>

#include "oracle.h"

double or_k1_radius(double eps) { return (945.0 / 256.0) * eps; }

void or_pair_kernel(int kernel, double r2, double eps, double* g, double* f) {
  if (kernel == 1) {
    const double h = or_k1_radius(eps);
    if (r2 < h * h) {
      const double x2 = r2 / (h * h);
      *g = (945.0 - 2100.0 * x2 + 2646.0 * x2 * x2 - 1620.0 * x2 * x2 * x2 +
            385.0 * x2 * x2 * x2 * x2) / (256.0 * h);
      *f = (525.0 - 1323.0 * x2 + 1215.0 * x2 * x2 - 385.0 * x2 * x2 * x2) / (32.0 * h * h * h);
      return;
    }
    const double ri = 1.0 / sqrt(r2);
    *g = ri;
    *f = ri * ri * ri;
    return;
  }
  const double si = 1.0 / sqrt(r2 + eps * eps);
  *g = si;
  *f = si * si * si;
}

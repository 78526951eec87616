"""Write nfw256_ref.npz: oracle reference accelerations and potentials
for sampled targets of the 256^3 clustered workload (70% of the particles in
NFW halos, 30% uniform background).

Calls only the oracle (and the seeded workload generator):
  * ``near_far``  -- the theta=0 tree result (27-image softened direct sum plus
    the order-8 far-field expansion) on 4096 evenly spaced targets: the
    reference for the rms force error of the tree at a given opening angle;
  * ``ewald``     -- the exact periodic direct sum (Ewald split) on the first
    16 of them: measures the far-field truncation floor at this size.

Usage: python tests/golden/make_nfw256_ref.py  (about 40 minutes on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

NT = 4096   # near_far targets
NE = 16     # Ewald targets


def main():
    pos, mass, prm = workloads.make("nfw256")
    n = pos.shape[1]
    targets = np.arange(0, n, n // NT, dtype=np.int64)[:NT]
    T = oracle.Tree(pos, mass, dict(prm, theta=0.0))
    acc_nf, pot_nf = T.direct_near_far(targets)
    t_ew = targets[:NE]
    acc_ew, pot_ew = oracle.direct_ewald(pos, mass, prm, targets=t_ew)
    out = os.path.join(HERE, "nfw256_ref.npz")
    np.savez(out, targets=targets, acc_near_far=acc_nf, pot_near_far=pot_nf,
             targets_ewald=t_ew, acc_ewald=acc_ew, pot_ewald=pot_ew,
             far_order=prm["far_order"], eps=prm["eps"])
    e = oracle.rms_rel_error(acc_nf[:, :NE], acc_ew)
    print(f"wrote {out}; far-field floor (near_far vs Ewald, {NE} targets): {e:.3e}")


if __name__ == "__main__":
    main()

"""Write zeldovich128_heldout.npz: exact periodic accelerations and potentials
(the oracle's direct Ewald sum, the plain definition) of the 128^3 Zel'dovich
workload on 1024 held-out targets.

The targets are drawn with a fixed seed from the particles that are NOT in the
10^4 evenly spaced targets of zeldovich128_ref.npz, on which the operating
point of the error-bound acceptance test is chosen: the rms force error at
that operating point is then reported on targets that played no part in
choosing it.  They also serve as the exact reference for the library's FP64
direct-summation mode at this size.

Calls only the oracle and the seeded workload generator.

Usage: python tests/golden/make_zeldovich128_heldout.py  (a few minutes on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

NH = 1024     # held-out targets
NT = 10000    # the selection targets of zeldovich128_ref.npz (multiples of n // NT)
SEED = 2024


def main():
    pos, mass, prm = workloads.make("zeldovich128")
    n = pos.shape[1]
    selection = np.arange(0, n, n // NT, dtype=np.int64)[:NT]
    pool = np.setdiff1d(np.arange(n, dtype=np.int64), selection)
    rng = np.random.default_rng(SEED)
    targets = np.sort(rng.choice(pool, size=NH, replace=False)).astype(np.int64)
    acc, pot = oracle.direct_ewald(pos, mass, prm, targets=targets)
    out = os.path.join(HERE, "zeldovich128_heldout.npz")
    np.savez(out, targets=targets, acc_ewald=acc, pot_ewald=pot, eps=prm["eps"], seed=SEED)
    print(f"wrote {out}: {NH} targets, rms |a| = {np.sqrt(np.mean(np.sum(acc ** 2, 0))):.4e}")


if __name__ == "__main__":
    main()

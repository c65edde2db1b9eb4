"""Write the density-matrix reference for the trajectory-mean test: <Z_q> of
the FP64 oracle's exact density-matrix evolution (Sec. 2.4 channels applied
as rho -> sum_b K_b rho K_b^dagger after each gate) for the 10-qubit (2 x 5
grid) depth-24 random circuit with depolarizing p = 1e-3 after one-qubit
gates, 1e-2 (two-qubit Kronecker form) after CZ and amplitude damping
gamma = 5e-4 per qubit per layer, generator seed 4010.

Run from the repository root: python tests/golden/make_dm_reference.py
It calls only the oracle and the seeded circuit generator.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2008_07140_amd import circuits as cg  # noqa: E402

N, DEPTH, SEED = 10, 24, 4010
RATES = (1e-3, 1e-2, 5e-4)
OUT = os.path.join(HERE, "dm_n10_d24_workload_rates.txt")


def main():
    ops = cg.random_circuit(2, 5, DEPTH, seed=SEED, dep1=RATES[0], dep2=RATES[1], damping=RATES[2])
    z = oracle.dm_expect_z(oracle.dm_run(N, ops))
    with open(OUT, "w") as f:
        f.write("# <Z_q>, q = 0..%d, exact density matrix (FP64 oracle): 2x5 grid, depth %d, seed %d,\n"
                % (N - 1, DEPTH, SEED))
        f.write("# depolarizing %g (1q) / %g (CZ, Kronecker form), amplitude damping %g per layer\n" % RATES)
        f.write("# written by tests/golden/make_dm_reference.py\n")
        for v in z:
            f.write("%.17g\n" % v)
    print("wrote", OUT, np.round(z, 6))


if __name__ == "__main__":
    main()

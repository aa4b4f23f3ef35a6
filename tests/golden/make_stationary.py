"""Writes the oracle's stationary state of the two-mode model at depth 2 (28
ADOs of 25 x 25) used by the Krylov equilibration test in
tests/test_gpu_parity.py (calls only oracle/ and the seeded inputs of
workloads/; run from the repository root: python tests/golden/make_stationary.py).

rho_eq solves L rho = 0 with tr rho_0 = 1 (sparse direct solve; Sec. II.C:
the long-time limit of the propagation from |0><0|).
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from oracle import heom as oh  # noqa: E402
from oracle import model as om  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    params, _ = w.cfg2()
    params["depth"] = 2
    o = om.build(params)
    rho = oh.stationary_state(o)
    np.savez_compressed(os.path.join(HERE, "cfg2_depth2_rho_eq.npz"), rho=rho, depth=2,
                        residual=oh.residual(o, rho))
    print("cfg2_depth2_rho_eq.npz", rho.shape, "residual", oh.residual(o, rho), flush=True)


if __name__ == "__main__":
    main()

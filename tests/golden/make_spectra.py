"""Writes the oracle's 2D responses and correlation spectra used by
tests/test_gpu_spectra.py (calls only oracle/ and the seeded inputs of
workloads/; run from the repository root: python tests/golden/make_spectra.py).

* cfg1_spectrum.npz: the single-mode model at its full configuration (35 ADOs,
  32 x 32 grid every 100 RK4 steps, t2 = 0).
* cfg2_depth2_spectra.npz: the two-mode model reduced to depth 2 (28 ADOs) on a
  32 x 32 grid every 10 steps, at both of its t2 values (0 and 100 fs = 654
  steps).
rho_eq is the stationary state L rho = 0, tr rho_0 = 1 (sparse direct solve,
Sec. II.C: the long-time limit of the propagation from |0><0|); R follows the
paper's pathway recipe (Eqs. echo, virtual-echo) and S_C Eq.
correlation-spectrum.
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


def write(name, params, grid):
    o = om.build(params)
    rho = oh.stationary_state(o)
    R = oh.response_2d(o, rho, grid)
    dt_s = grid["steps_per_sample"] * params["dt"]
    S = np.stack([oh.correlation_spectrum(R[q, 0], R[q, 1], dt_s) for q in range(R.shape[0])])
    np.savez(os.path.join(HERE, name), R=R, S_C=S, n1=grid["n1"], n3=grid["n3"],
             steps_per_sample=grid["steps_per_sample"], t2_steps=np.asarray(grid["t2_steps"]),
             depth=params["depth"], residual=oh.residual(o, rho))
    print(name, R.shape, "max|S_C|", float(np.max(np.abs(S))), flush=True)


if __name__ == "__main__":
    p1, g1 = w.cfg1()
    write("cfg1_spectrum.npz", p1, g1)
    p2, g2 = w.cfg2()
    p2["depth"] = 2
    write("cfg2_depth2_spectra.npz", p2, {"n1": 32, "n3": 32, "steps_per_sample": 10,
                                          "t2_steps": list(g2["t2_steps"])})

"""2D correlation spectra at the benchmark configurations (Sec. II.C, Eqs.
echo, virtual-echo, correlation-spectrum), through the C ABI:

* against the oracle's responses and spectra stored in tests/golden (written
  by tests/golden/make_spectra.py, which calls only oracle/): the single-mode
  model at its full configuration and the two-mode model at depth 2 with both
  t2 values; rho_eq from the library's GMRES stationary solve;
* the FP32 path against the FP64 path over the full lengths of the
  three-mode model (depth 3, full 128 x 128 grid, t2 = 200 fs: 1307 + 1270
  FP32 RK4 steps per trajectory with the batched t2 and t3 propagations).

Tolerances: FP64 1e-9 of the peak (rho_eq is solved to a residual of 1e-12;
the oracle's is exact), FP32 1e-4 of the peak (the FP32 path's target).
"""

import os

import numpy as np
import pytest

import workloads as w

P = pytest.importorskip("paper_2601_20550_amd")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _peak_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _golden(name):
    with np.load(os.path.join(GOLDEN, name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


@pytest.mark.parametrize("name,which,depth,spa", [("cfg1_spectrum.npz", "cfg1", None, 5000),
                                                  ("cfg2_depth2_spectra.npz", "cfg2", 2, 500)])
def test_spectra_match_oracle(name, which, depth, spa):
    ref = _golden(name)
    params = getattr(w, which)()[0]
    if depth is not None:
        params["depth"] = depth
    assert int(ref["depth"]) == params["depth"]
    grid = {"n1": int(ref["n1"]), "n3": int(ref["n3"]), "steps_per_sample": int(ref["steps_per_sample"]),
            "t2_steps": [int(x) for x in ref["t2_steps"]]}
    m = P.heom_model_build(params)
    # GMRES applications of spa RK4 steps (about 50 time units each)
    rho, _, res = P.heom_equilibrate_krylov(m, tol=1e-12, steps_per_apply=spa, max_applies=400)
    assert res <= 1e-12
    dt_s = grid["steps_per_sample"] * params["dt"]
    for prec, method, tol in (("fp64", "adjoint", 1e-9), ("fp64", "direct", 1e-9), ("fp32", "adjoint", 1e-4),
                              ("fp32", "direct", 1e-4)):
        R = P.heom_response_2d(m, rho, grid, prec, method)
        assert _peak_err(R, ref["R"]) < tol, (prec, method)
        for q in range(R.shape[0]):
            S = P.heom_spectrum_2d(R[q, 0], R[q, 1], dt_s)
            assert _peak_err(S, ref["S_C"][q]) < tol, (prec, method, q)


def test_fp32_full_grid_t2_200fs_matches_fp64():
    params, grid = w.cfg3(depth=3)
    g = dict(grid)
    g["t2_steps"] = [grid["t2_steps"][-1]]  # 200 fs
    assert g["n1"] == 128 and g["n3"] == 128 and g["t2_steps"][0] == 1307
    m = P.heom_model_build(params)
    rho, _, res = P.heom_equilibrate_krylov(m, tol=1e-10, max_applies=400)
    assert res <= 1e-10
    R64 = P.heom_response_2d(m, rho, g, "fp64", "adjoint")
    R32 = P.heom_response_2d(m, rho, g, "fp32", "direct")
    dt_s = g["steps_per_sample"] * params["dt"]
    S64 = P.heom_spectrum_2d(R64[0, 0], R64[0, 1], dt_s)
    S32 = P.heom_spectrum_2d(R32[0, 0], R32[0, 1], dt_s)
    assert _peak_err(R32, R64) < 1e-4
    assert _peak_err(S32, S64) < 1e-4

"""GPU parity of the paper's water models (Tables I-III; reading of the tables
in workloads.water_two_mode / water_three_mode) at reduced hierarchy depth,
against the CPU FP64 oracle: the linear response R1 and its line shape
(Eq. R1 and the 1D spectrum, Sec. II.C) for both models at three and four
levels per mode, and a small
2D response of the two-mode model.  The input state is 200 oracle RK4 steps
from the ground state (parity holds for any input; the oracle's dense
stationary solve is too slow at these sizes).

Tolerances: FP64 1e-10 of the peak (a few hundred RK4 steps, summation
order), FP32 1e-4 of the peak (the FP32 path's target).
"""

import numpy as np
import pytest

import workloads as w
from oracle import heom as oh
from oracle import model as om

P = pytest.importorskip("paper_2601_20550_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _relerr(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


MODELS = {"two": w.water_two_mode, "three": w.water_three_mode}


@pytest.mark.parametrize("which,levels,depth", [("two", 4, 2), ("two", 3, 2), ("three", 3, 1), ("three", 4, 1)])
def test_water_linear_response_parity(which, levels, depth):
    p = MODELS[which](n_levels=levels, depth=depth)
    o = om.build(p)
    rho = oh.propagate(o, oh.ground_state_hierarchy(o), 200)
    n, sps = 48, 8
    ref = oh.linear_response(o, rho, n, sps)
    m = P.heom_model_build(p)
    r = P.State(m, 1, "fp64")
    r.upload(rho[None])
    dt_s = sps * p["dt"]
    ref_I = oh.linear_spectrum(ref, dt_s)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        got = P.heom_linear_response(m, r, n, sps, prec)
        assert _relerr(got, ref) < tol, prec
        assert _relerr(P.heom_spectrum_1d(got, dt_s), ref_I) < tol, prec


def test_water_two_mode_2d_response_parity():
    p = w.water_two_mode(n_levels=3, depth=2)
    o = om.build(p)
    rho = oh.propagate(o, oh.ground_state_hierarchy(o), 200)
    grid = {"n1": 4, "n3": 4, "steps_per_sample": 4, "t2_steps": [0, 6]}
    ref = oh.response_2d(o, rho, grid)
    m = P.heom_model_build(p)
    r = P.State(m, 1, "fp64")
    r.upload(rho[None])
    for method in ("direct", "adjoint"):
        assert _relerr(P.heom_response_2d(m, r, grid, "fp64", method), ref) < 1e-10, method
        assert _relerr(P.heom_response_2d(m, r, grid, "fp32", method), ref) < 1e-4, method

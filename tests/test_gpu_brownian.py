"""GPU parity for Brownian (underdamped-oscillator) bath spectral densities.

These baths give each mode a complex-conjugate pair of exponential rates: the
ADO damping sum_j n_j nu_j is complex and the bra-side coupling coefficients
are the partner term's conjugated coefficient rather than conj(c_j).  Every
right-hand-side kernel (generic VALU, matrix-core with compile-time and
runtime mode shapes, the multi-instance launch) is compared against the CPU
FP64 oracle with the tolerances of the Drude parity tests: relative 1e-12
(FP64) and 2e-6 (FP32) per right-hand side, 1e-10 / 1e-4 for responses.
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


def _params(which, depth=None):
    if which == "cfg3b":
        return w.cfg3_brownian(depth=depth)[0]
    p = getattr(w, which)()[0]
    if depth is not None:
        p["depth"] = depth
    p["decomp"] = "pade"
    wb = {"cfg1": [1.5], "cfg2": [1.5, 0.3]}[which]
    return w.with_brownian_baths(p, wb)


CASES = [("cfg1", 3), ("cfg2", 2), ("cfg3b", 2)]


@pytest.mark.parametrize("which,depth", CASES)
@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kernel", ["generic", "mfma", "mfma_dyn", "kron", "mfma_gh"])
def test_rhs_parity_brownian(which, depth, adjoint, prec, kernel):
    params = _params(which, depth)
    o = om.build(params)
    assert np.any(np.imag(o.nu) != 0)
    m = P.heom_model_build(params)
    if kernel in ("kron", "mfma_gh") and (prec != "fp32" or which != "cfg3b"):
        # both need FP32 and the three-mode (4, 4, 5) shape (d = 80)
        with pytest.raises(P.heom2dvs.HeomError):
            P.heom_model_set_kernel(m, prec, kernel)
        return
    P.heom_model_set_kernel(m, prec, kernel)
    x = w.random_hierarchy(3, len(o.hier), o.d, seed=17, scale_by_depth=0.3 ** o.hier.n.sum(1))
    xin = P.State(m, 3, prec)
    xout = P.State(m, 3, prec)
    xin.upload(x)
    P.heom_rhs(m, xin, xout, adjoint)
    ref = oh.rhs(o, x, adjoint=adjoint)
    assert _relerr(xout.download(), ref) < (1e-12 if prec == "fp64" else 2e-6)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_rk4_steps_parity_brownian(prec, tol):
    params = _params("cfg2", 3)
    o = om.build(params)
    m = P.heom_model_build(params)
    x = w.random_hierarchy(2, len(o.hier), o.d, seed=5, hermitian=True, scale_by_depth=0.3 ** o.hier.n.sum(1))
    s = P.State(m, 2, prec)
    for adjoint in (False, True):
        s.upload(x)
        P.heom_propagate(m, s, 6, adjoint=adjoint)
        assert _relerr(s.download(), oh.propagate(o, x, 6, adjoint=adjoint)) < tol


def test_harmonic_linear_response_brownian_bath():
    # the GPU path against the oracle and against the Langevin closed form of
    # a harmonic mode in a Brownian bath (the oracle pin's configuration)
    params = w.harmonic_pin(depth=4, K=2, dt=0.02, n_keep=6, gamma=0.5, omega_b=2.0)
    o = om.build(params)
    m = P.heom_model_build(params)
    rho = P.State(m, 1, "fp64")
    rho.set_ground()
    ref = oh.linear_response(o, oh.ground_state_hierarchy(o), 16, 50)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        got = P.heom_linear_response(m, rho, 16, 50, prec)
        assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref)), prec
    num = np.array([1.0, 0.5, 4.0])
    den = np.polyadd(np.polymul([1.0, 0.0, 1.0], num), 0.1 * 0.5 * np.array([1.0, 0.5, 0.0]))
    poles = np.roots(den)
    t = np.arange(16.0)
    chi = np.zeros(16)
    for i, s in enumerate(poles):
        dd = np.prod([s - q for k, q in enumerate(poles) if k != i])
        chi = chi + np.real(np.polyval(num, s) / dd * np.exp(s * t))
    got = P.heom_linear_response(m, rho, 16, 50, "fp64")
    assert np.max(np.abs(got.real - chi)) < 1e-5


@pytest.mark.parametrize("which,depth,n,sps,t2", [("cfg2", 2, 5, 5, [0, 10]), ("cfg3b", 1, 3, 4, [0, 6])])
@pytest.mark.parametrize("method", ["direct", "adjoint"])
def test_response_2d_parity_brownian(which, depth, n, sps, t2, method):
    params = _params(which, depth)
    o = om.build(params)
    m = P.heom_model_build(params)
    rho_ref = oh.propagate(o, oh.ground_state_hierarchy(o), 40)
    rho = P.State(m, 1, "fp64")
    rho.upload(rho_ref[None])
    grid = {"n1": n, "n3": n, "steps_per_sample": sps, "t2_steps": t2}
    ref = oh.response_2d(o, rho_ref, grid)
    assert _relerr(P.heom_response_2d(m, rho, grid, "fp64", method), ref) < 1e-10
    assert _relerr(P.heom_response_2d(m, rho, grid, "fp32", method), ref) < 1e-4


def test_krylov_stationary_state_brownian():
    params = _params("cfg1", 3)
    params["dt"] = 0.05
    o = om.build(params)
    ref = oh.stationary_state(o)
    m = P.heom_model_build(params)
    rho, applies, res = P.heom_equilibrate_krylov(m, tol=1e-11)
    assert res <= 1e-11 and applies > 0
    assert np.max(np.abs(rho.download()[0] - ref)) < 1e-8 * np.max(np.abs(ref))


def test_multi_instance_batch_with_brownian_and_drude_instances():
    # one launch per size class over instances with complex and real rates
    insts = [_params("cfg2", 2), w.cfg2()[0], _params("cfg1", 3)]
    insts[1]["depth"] = 2
    for p in insts:
        p["dt"] = 0.05  # a batch shares one time step
    models = [P.heom_model_build(p) for p in insts]
    oracles = [om.build(p) for p in insts]
    states, refs = [], []
    for i, (m, o) in enumerate(zip(models, oracles)):
        x = w.random_hierarchy(2, len(o.hier), o.d, seed=30 + i, hermitian=True,
                               scale_by_depth=0.3 ** o.hier.n.sum(1))
        s = P.State(m, 2, "fp32")
        s.upload(x)
        states.append(s)
        refs.append(oh.propagate(o, x, 4))
    b = P.heom_batch_create(models)
    P.heom_batch_propagate(b, states, 4)
    for s, ref in zip(states, refs):
        assert _relerr(s.download(), ref) < 1e-5


def test_gradient_rejects_complex_rates():
    params = _params("cfg2", 1)
    m = P.heom_model_build(params)
    r = P.State(m, 1, "fp64")
    r.set_ground()
    grid = {"n1": 2, "n3": 2, "steps_per_sample": 1, "t2_steps": [0]}
    W = np.ones((1, 2, 2, 2), dtype=complex)
    with pytest.raises(P.heom2dvs.HeomError) as e:
        P.heom_response_2d_vjp(m, r, grid, W)
    assert e.value.code == P.heom2dvs.HEOM_ERR_PARAM

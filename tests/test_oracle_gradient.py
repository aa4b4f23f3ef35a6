"""Pins of the oracle's gradient machinery (CPU only).

The forward pieces (model build, stationary state, responses, spectrum) are
pinned in test_oracle_pins.py.  Here: the spectrum adjoint against the
forward spectrum map (dot-product identity), the completeness of the
operator-level decomposition (theta-level differences of the loss equal the
operator-level differences chained with the build's operator directions),
the least-squares property at the target, and step-size consistency.
"""

import numpy as np
import pytest

import workloads as w
from oracle import gradient as og
from oracle import heom as oh


def test_spectrum_vjp_dot_product():
    rng = np.random.default_rng(3)
    for n1, n3, dt_s in ((6, 6, 0.4), (5, 7, 1.0)):
        RI = rng.standard_normal((n1, n3)) + 1j * rng.standard_normal((n1, n3))
        RII = rng.standard_normal((n1, n3)) + 1j * rng.standard_normal((n1, n3))
        G = rng.standard_normal((2 * n3, 2 * n1))
        lhs = np.sum(G * oh.correlation_spectrum(RI, RII, dt_s))
        W = og.spectrum_vjp(G, n1, n3, dt_s)
        rhs = np.real(np.sum(W[0] * RI) + np.sum(W[1] * RII))
        assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.fixture(scope="module")
def fit_case():
    params, grid, theta_t = w.cfg5_small()
    _, _, _, S_t = og.spectra(w.apply_theta(params, theta_t), grid)
    return params, grid, S_t


@pytest.fixture(scope="module")
def fit_gradient(fit_case):
    params, grid, S_t = fit_case
    return og.loss_gradient_fd(params, grid, S_t, w.apply_theta, w.theta_size(params))


def test_gradient_zero_at_target(fit_case, fit_gradient):
    # J(theta* + h e_i) = O(h^2): the central difference at the minimum is O(h^2)
    params, grid, _ = fit_case
    _, _, _, S0 = og.spectra(params, grid)
    n = w.theta_size(params)
    g = og.loss_gradient_fd(params, grid, S0, w.apply_theta, n)
    assert og.loss(params, grid, S0) == 0.0
    assert np.max(np.abs(g)) < 1e-6 * np.max(np.abs(fit_gradient))


def test_theta_gradient_equals_operator_chain(fit_case, fit_gradient):
    params, grid, S_t = fit_case
    n = w.theta_size(params)
    g_fd = fit_gradient
    m, rho, R, S = og.spectra(params, grid)
    dt_s = grid["steps_per_sample"] * params["dt"]
    W = np.stack([og.spectrum_vjp(2.0 * (S[q] - S_t[q]), grid["n1"], grid["n3"], dt_s)
                  for q in range(len(S))])
    g_op = og.operator_gradient_fd(m, rho, grid, W, stationary=True)
    dirs = w.theta_directions(params)
    g_chain = np.array([og.contract(g_op, og.operator_directions_fd(params, dirs[i]))
                        for i in range(n)])
    assert np.max(np.abs(g_fd)) > 1e-3
    assert np.max(np.abs(g_chain - g_fd)) < 1e-6 * np.max(np.abs(g_fd))


def test_step_size_consistency(fit_case, fit_gradient):
    params, grid, S_t = fit_case
    n = w.theta_size(params)
    a = fit_gradient
    b = og.loss_gradient_fd(params, grid, S_t, w.apply_theta, n, rel_step=1e-4)
    assert np.max(np.abs(a - b)) < 1e-6 * np.max(np.abs(a))

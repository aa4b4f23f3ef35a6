"""Gradients of a least-squares spectrum fit (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Objective.  For parameters p(theta) (multiplicative factors theta on g3, g4,
the coupling constants, V1, V2, zeta and gamma), the fit minimises

  J(theta) = sum_q sum_{W3, W1} ( S_C,q(W3, W1; theta) - S*_q(W3, W1) )^2

where S_C,q is the correlation spectrum (Eq. correlation-spectrum) of the
third-order responses (Eqs. RFTIRI, echo, virtual-echo) at the q-th waiting
time t2, computed from the stationary state rho_eq of the HEOM (L rho_eq = 0,
tr rho_eq,0 = 1; Sec. II.C) with the classic RK4 propagator.

Everything here is a plain restatement by central finite differences of the
forward oracle: theta-level derivatives of J, operator-level derivatives of a
linear functional Re sum W R of the responses (H, the single-mode couplings
v_s, mu, the bath coefficients c_j and rates nu_j), and the operator
directions d(operators)/d theta_i of the model build.  The adjoint of the
spectrum map (spectrum_vjp) is written out from the DFT definition.
"""

from __future__ import annotations

from dataclasses import replace

import numpy as np

from . import heom as oh
from . import model as om


# ------------------------------------------------------------ forward -------

def spectra(params, grid, rho_eq=None):
    """(model, rho_eq, R, [S_C for every t2]) of a parameter dictionary."""
    m = om.build(params)
    rho = oh.stationary_state(m) if rho_eq is None else rho_eq
    R = oh.response_2d(m, rho, grid)
    dt_s = grid["steps_per_sample"] * m.dt
    S = [oh.correlation_spectrum(R[q, 0], R[q, 1], dt_s) for q in range(R.shape[0])]
    return m, rho, R, S


def loss(params, grid, S_target):
    """J = sum_q sum (S_C,q - S*_q)^2."""
    _, _, _, S = spectra(params, grid)
    return float(sum(np.sum((a - b) ** 2) for a, b in zip(S, S_target)))


def loss_gradient_fd(params, grid, S_target, theta_apply, n_theta, rel_step=1e-5):
    """dJ/dtheta at theta = 1 by central differences with step rel_step.

    theta_apply(params, theta) returns the scaled parameters."""
    g = np.zeros(n_theta)
    for i in range(n_theta):
        tp = np.ones(n_theta)
        tm = np.ones(n_theta)
        tp[i] += rel_step
        tm[i] -= rel_step
        g[i] = (loss(theta_apply(params, tp), grid, S_target)
                - loss(theta_apply(params, tm), grid, S_target)) / (2.0 * rel_step)
    return g


# ------------------------------------------------- spectrum adjoint ---------

def spectrum_vjp(G, n1, n3, dt_s):
    """Weights W[P][j][k] with sum <G, S_C(R_I, R_II)> = Re sum_P,j,k W[P] R[P].

    S_C = sigma (S_I(W3, -W1) + S_II(W3, W1)) and
    S_P = Im(dt_s^2 E3 R_P^T E1^T) with E(W, t) = w_t exp(i W t); Im(z) = Re(-i z),
    so W_P[j][k] = -i sigma dt_s^2 sum_{W3,W1} G[W3][W1] E3[W3][k] E1_P[W1][j].
    G has shape (2 n3, 2 n1)."""
    w1 = oh.frequency_grid(n1, dt_s)
    w3 = oh.frequency_grid(n3, dt_s)
    t1 = dt_s * np.arange(n1)
    t3 = dt_s * np.arange(n3)
    wt1 = np.ones(n1)
    wt1[0] = 0.5
    wt3 = np.ones(n3)
    wt3[0] = 0.5
    E3 = wt3[None, :] * np.exp(1j * np.outer(w3, t3))
    out = []
    for flip in (True, False):
        E1 = wt1[None, :] * np.exp(1j * np.outer(-w1 if flip else w1, t1))
        W = -1j * oh.SIGMA * dt_s * dt_s * (E1.T @ G.T @ E3)      # (n1, n3)
        out.append(W)
    return np.stack(out)


# ------------------------------------------- operator-level gradients -------

def objective(model, rho_eq, grid, W):
    """Re sum_{q,P,j,k} W[q,P,j,k] R[q,P,j,k]."""
    R = oh.response_2d(model, rho_eq, grid)
    return float(np.real(np.sum(W * R)))


def _with_mu(model, mu):
    N = om.quanta(model.dims)
    mp = np.where(N[:, None] > N[None, :], mu, 0.0)
    return replace(model, mu=mu, mu_plus=mp, mu_minus=mp.T.copy())


def operator_gradient_fd(model, rho_eq, grid, W, step=1e-6, stationary=False):
    """Central differences of objective() with respect to every entry of H,
    of each single-mode v_s (embedded as v_s on mode s), of mu (with mu+ and
    mu- re-derived), to Re c_j, Im c_j and nu_j.  With stationary=True rho_eq is
    recomputed as the stationary state of every perturbed model; otherwise it
    is held fixed."""
    def f(m):
        r = oh.stationary_state(m) if stationary else rho_eq
        return objective(m, r, grid, W)

    def cd(make):
        return (f(make(step)) - f(make(-step))) / (2.0 * step)

    d = model.d
    gH = np.zeros((d, d))
    gmu = np.zeros((d, d))
    for a in range(d):
        for b in range(d):
            E = np.zeros((d, d))
            E[a, b] = 1.0
            gH[a, b] = cd(lambda e: replace(model, H=model.H + e * E))
            gmu[a, b] = cd(lambda e: _with_mu(model, model.mu + e * E))
    gv = []
    for s, ds in enumerate(model.dims):
        g = np.zeros((ds, ds))
        for a in range(ds):
            for b in range(ds):
                E = np.zeros((ds, ds))
                E[a, b] = 1.0
                dV = om.embed({s: E}, model.dims)

                def mk(e, s=s, dV=dV):
                    V = list(model.V)
                    V[s] = V[s] + e * dV
                    return replace(model, V=V)
                g[a, b] = cd(mk)
        gv.append(g)
    M = len(model.nu)
    gc = np.zeros((M, 2))
    gnu = np.zeros(M)
    for j in range(M):
        for part, z in ((0, 1.0), (1, 1j)):
            def mk(e, j=j, z=z):
                c = model.c.copy()
                c[j] += e * z
                return replace(model, c=c)
            gc[j, part] = cd(mk)

        def mkn(e, j=j):
            nu = model.nu.copy()
            nu[j] += e
            return replace(model, nu=nu)
        gnu[j] = cd(mkn)
    return {"H": gH, "v": gv, "mu": gmu, "c": gc, "nu": gnu}


def operator_directions_fd(params, direction, step=1e-6):
    """d(operators)/d(params) along a parameter direction (a dictionary of
    the same layout holding the derivative of every number), by central
    differences of the model build: dict with H, v (list), mu, c (M x 2), nu."""
    def shifted(e):
        import copy
        p = copy.deepcopy(params)
        for m, dm in zip(p["modes"], direction["modes"]):
            for key in ("omega", "g3", "g4", "V1", "V2", "zeta", "gamma", "mu1", "mu2"):
                m[key] += e * dm[key]
        for c, dc in zip(p.get("couplings", []), direction.get("couplings", [])):
            for key in ("g_st", "g_s2t", "g_st2", "mu_st"):
                c[key] += e * dc[key]
        p["beta"] += e * direction["beta"]
        m = om.build(p)
        return {"H": m.H, "v": [mo.v for mo in m.modes], "mu": m.mu,
                "c": np.stack([m.c.real, m.c.imag], axis=1), "nu": m.nu}

    a, b = shifted(step), shifted(-step)
    out = {}
    for key in ("H", "mu", "c", "nu"):
        out[key] = (a[key] - b[key]) / (2.0 * step)
    out["v"] = [(x - y) / (2.0 * step) for x, y in zip(a["v"], b["v"])]
    return out


def contract(g, dop):
    """sum over all operator entries of gradient x direction."""
    tot = np.sum(g["H"] * dop["H"]) + np.sum(g["mu"] * dop["mu"])
    tot += np.sum(g["c"] * dop["c"]) + np.sum(g["nu"] * dop["nu"])
    tot += sum(np.sum(x * y) for x, y in zip(g["v"], dop["v"]))
    return float(tot)

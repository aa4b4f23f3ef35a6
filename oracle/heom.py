"""HEOM propagation, response functions and 2D spectra (oracle).

Hierarchy states are complex arrays of shape (..., N_ado, d, d); leading axes
are independent trajectories.  Everything is double precision.

Right-hand side (Eq. HEOM_DB with Theta_j from Eqs. Pade1/Pade2 written as
Theta_j X = c_j V X - cb_j X V, see oracle.bath):

  d rho_n/dt = -i (H rho_n - rho_n H) - (sum_j n_j nu_j) rho_n
               - i sum_j n_j (c_j V_s(j) rho_{n-e_j} - cb_j rho_{n-e_j} V_s(j))
               - i sum_j (V_s(j) rho_{n+e_j} - rho_{n+e_j} V_s(j)),

where cb_j = conj(c_j) for the real rates of a Drude bath and, for the
complex-conjugate pair of rates of a Brownian bath, the conjugated
coefficient of the partner term (bath.bra_coefficients).

with ADOs outside the index set treated as zero.  Time stepping is the classic
four-stage Runge-Kutta method with a fixed step (Sec. III).

Response functions (Sec. II.C):
  R1(t)        = i tr{ mu G(t) mu^x rho_eq }                    (Eq. R1)
  R3_P(t3,t2,t1) = i^3 tr{ mu G(t3) D3^x G(t2) D2^x G(t1) D1^x rho_eq }
                                                     (Eqs. RFTIRI, echo,
                                                      virtual-echo)
with (D1, D2, D3) = (mu_minus, mu_plus, mu_plus) for the rephasing pathway I
(k3 + k2 - k1) and (mu_plus, mu_minus, mu_plus) for the non-rephasing pathway
II (k3 - k2 + k1), and (mu, mu, mu) for the full response.  The trace acts on
the system density operator, i.e. the ADO with n = 0.  Following the four-step
recipe of the linear-response paragraph and the pathway recipe of Sec. II.C,
the t1 trajectory is propagated once with snapshots, every snapshot receives
D2, is propagated over t2, receives D3 and is propagated over t3 while the
trace is sampled.

Spectra (Eqs. 2D-rephasing, 2D-nonrephasing, correlation-spectrum), with the
time integrals discretised by the trapezoid rule on the sample grid (weight
1/2 at t = 0), zero-padding to 2N points and Omega_m = 2 pi m / (2 N dt_s),
m = -N..N-1:

  S_P(W3, W1) = Im sum_j sum_k w_j w_k dt_s^2 exp(i W3 t3_k + i W1 t1_j) R_P[j, k]
  S_C(W3, W1) = sigma [ S_I(W3, -W1) + S_II(W3, W1) ],  sigma = -1,

sigma being fixed so that the 0 -> 1 -> 0 diagonal peak is positive and the
0 -> 1 -> 2 peak negative, as the paper describes its figures.
"""

from __future__ import annotations

import numpy as np

from .model import Model


# ----------------------------------------------------------------- RHS ------

def rhs(model: Model, rho, adjoint: bool = False):
    """L rho (adjoint=False) or L^T rho (adjoint=True).

    L^T is the transpose with respect to the bilinear pairing
    <A, X> = sum_n sum_ab A_n[a, b] X_n[a, b]; with H and V_s real symmetric
    it moves the n_j c_j factor from the lower to the upper neighbour:
      (L^T A)_m = -i H^x A_m - gamma_m A_m - i sum_j V^x A_{m-e_j}
                  - i sum_j (m_j + 1)(c_j V A_{m+e_j} - cb_j A_{m+e_j} V).
    """
    H = model.H
    hier = model.hier
    out = -1j * (H @ rho - rho @ H) - model.gamma_sum[:, None, None] * rho
    cb = model.c_bra
    for j in range(hier.n_terms):
        V = model.V[model.term_mode[j]]
        cj = model.c[j]
        up = hier.up[:, j]
        dn = hier.down[:, j]
        mu_ = up >= 0
        md_ = dn >= 0
        if not adjoint:
            X = rho[..., up[mu_], :, :]
            out[..., mu_, :, :] += -1j * (V @ X - X @ V)
            Y = rho[..., dn[md_], :, :]
            nj = hier.n[md_, j][:, None, None]
            out[..., md_, :, :] += -1j * nj * (cj * (V @ Y) - cb[j] * (Y @ V))
        else:
            Y = rho[..., dn[md_], :, :]
            out[..., md_, :, :] += -1j * (V @ Y - Y @ V)
            X = rho[..., up[mu_], :, :]
            nj = (hier.n[mu_, j] + 1)[:, None, None]
            out[..., mu_, :, :] += -1j * nj * (cj * (V @ X) - cb[j] * (X @ V))
    return out


def rk4_step(model: Model, rho, h=None, adjoint: bool = False):
    """One classic RK4 step of size h (default model.dt)."""
    h = model.dt if h is None else h
    k1 = rhs(model, rho, adjoint)
    k2 = rhs(model, rho + 0.5 * h * k1, adjoint)
    k3 = rhs(model, rho + 0.5 * h * k2, adjoint)
    k4 = rhs(model, rho + h * k3, adjoint)
    return rho + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def propagate(model: Model, rho, n_steps: int, adjoint: bool = False):
    for _ in range(int(n_steps)):
        rho = rk4_step(model, rho, adjoint=adjoint)
    return rho


# ------------------------------------------------- assembled Liouvillian ----

def liouvillian_matrix(model: Model, adjoint: bool = False):
    """Sparse matrix of L acting on the row-major flattening of (N_ado, d, d).

    Built block by block from the operator forms: for row-major vec,
    vec(A X B) = (A kron B^T) vec(X), so A^x -> kron(A, I) - kron(I, A^T).
    This is an assembly independent of rhs(), used as its brute-force check
    and for the stationary state.
    """
    import scipy.sparse as sp
    d = model.d
    I = sp.identity(d, format="csr")
    hier = model.hier
    N = len(hier)
    Hc = sp.kron(sp.csr_matrix(model.H), I) - sp.kron(I, sp.csr_matrix(model.H.T))
    VL = [sp.kron(sp.csr_matrix(V), I) for V in model.V]
    VR = [sp.kron(I, sp.csr_matrix(V.T)) for V in model.V]
    blocks = [[None] * N for _ in range(N)]
    cb = model.c_bra
    for i in range(N):
        blocks[i][i] = -1j * Hc - model.gamma_sum[i] * sp.identity(d * d)
        for j in range(hier.n_terms):
            s = model.term_mode[j]
            up, dn = hier.up[i, j], hier.down[i, j]
            cj = model.c[j]
            if up >= 0:
                blk = -1j * (VL[s] - VR[s])
                blocks[i][up] = blk if blocks[i][up] is None else blocks[i][up] + blk
            if dn >= 0:
                blk = -1j * hier.n[i, j] * (cj * VL[s] - cb[j] * VR[s])
                blocks[i][dn] = blk if blocks[i][dn] is None else blocks[i][dn] + blk
    Lm = sp.bmat(blocks, format="csr")
    return Lm.T.tocsr() if adjoint else Lm


def stationary_state(model: Model):
    """Solution of L rho = 0 normalised by tr rho_0 = 1 (sparse direct solve).

    The equation for element (n=0, a=0, b=0) is replaced by the normalisation;
    for a unique stationary state the system is then non-singular.
    """
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    d = model.d
    Lm = liouvillian_matrix(model).tolil()
    row = np.zeros(Lm.shape[1], dtype=complex)
    row[[a * d + a for a in range(d)]] = 1.0
    Lm[0, :] = row
    b = np.zeros(Lm.shape[0], dtype=complex)
    b[0] = 1.0
    x = spla.spsolve(sp.csc_matrix(Lm), b)
    return x.reshape(len(model.hier), d, d)


# ------------------------------------------------------- equilibration ------

def ground_state_hierarchy(model: Model):
    """rho_{n=0} = |0><0| and all other ADOs zero (first step of Sec. II.C recipe)."""
    rho = np.zeros((len(model.hier), model.d, model.d), dtype=complex)
    rho[0, 0, 0] = 1.0
    return rho


def residual(model: Model, rho):
    """max over ADOs and elements of |(L rho)_n[a, b]|."""
    return float(np.max(np.abs(rhs(model, rho))))


def equilibrate(model: Model, tol: float, check_every: int, min_steps: int,
                max_steps: int, rho0=None):
    """Propagate from the factorised state until the residual is below tol.

    The residual is evaluated after every check_every steps once at least
    min_steps steps have been taken; propagation stops at the first check
    that passes or at max_steps.  Returns (rho_eq, steps, residual).
    """
    rho = ground_state_hierarchy(model) if rho0 is None else rho0.copy()
    steps = 0
    res = None
    while steps < max_steps:
        k = min(check_every, max_steps - steps)
        rho = propagate(model, rho, k)
        steps += k
        res = None
        if steps >= min_steps:
            res = residual(model, rho)
            if res <= tol:
                break
    if res is None:
        res = residual(model, rho)
    return rho, steps, res


# ------------------------------------------------------------ dipoles -------

def commutator(D, rho):
    """D^x rho = D rho - rho D on every ADO."""
    return D @ rho - rho @ D


def trace_n0(A, rho):
    """tr(A rho_0) on the n = 0 ADO, for every leading trajectory index."""
    r0 = rho[..., 0, :, :]
    return np.einsum("ba,...ab->...", A, r0)


def pathway_dipoles(model: Model, pathway):
    """(D1, D2, D3) of a named pathway; an explicit triple passes through."""
    if not isinstance(pathway, str):
        return tuple(pathway)
    if pathway == "I":
        return model.mu_minus, model.mu_plus, model.mu_plus
    if pathway == "II":
        return model.mu_plus, model.mu_minus, model.mu_plus
    if pathway == "full":
        return model.mu, model.mu, model.mu
    raise ValueError(pathway)


def linear_response(model: Model, rho_eq, n: int, steps_per_sample: int):
    """R1(t_k) = i tr{mu rho'_0(t_k)}, rho'(0) = mu^x rho_eq, t_k = k * dt_s."""
    X = commutator(model.mu, rho_eq)
    out = np.zeros(n, dtype=complex)
    for k in range(n):
        if k:
            X = propagate(model, X, steps_per_sample)
        out[k] = 1j * trace_n0(model.mu, X)
    return out


def response_2d(model: Model, rho_eq, grid, pathways=("I", "II")):
    """R[t2 index][pathway][j (t1)][k (t3)] as a complex array."""
    n1, n3 = int(grid["n1"]), int(grid["n3"])
    sps = int(grid["steps_per_sample"])
    t2_steps = [int(s) for s in grid["t2_steps"]]
    if any(b < a for a, b in zip(t2_steps, t2_steps[1:])):
        raise ValueError("t2 steps must be non-decreasing")
    R = np.zeros((len(t2_steps), len(pathways), n1, n3), dtype=complex)
    for p, pw in enumerate(pathways):
        D1, D2, D3 = pathway_dipoles(model, pw)
        X = commutator(D1, rho_eq)
        snaps = []
        for j in range(n1):
            if j:
                X = propagate(model, X, sps)
            snaps.append(X)
        Y = commutator(D2, np.stack(snaps))          # (n1, N_ado, d, d)
        done = 0
        for i, t2 in enumerate(t2_steps):
            Y = propagate(model, Y, t2 - done)
            done = t2
            Z = commutator(D3, Y)
            for k in range(n3):
                if k:
                    Z = propagate(model, Z, sps)
                R[i, p, :, k] = (1j) ** 3 * trace_n0(model.mu, Z)
    return R


# ------------------------------------------------------------ spectra -------

SIGMA = -1.0


def frequency_grid(n: int, dt_s: float):
    """Omega_m = 2 pi m / (2 n dt_s), m = -n..n-1."""
    m = np.arange(-n, n)
    return 2.0 * np.pi * m / (2 * n * dt_s)


def pathway_spectrum(R, dt_s: float, flip_w1: bool = False):
    """S_P(W3, W1) on the (2 n3) x (2 n1) grid, rows W3, columns W1."""
    n1, n3 = R.shape
    w1 = frequency_grid(n1, dt_s)
    w3 = frequency_grid(n3, dt_s)
    if flip_w1:
        w1 = -w1
    t1 = dt_s * np.arange(n1)
    t3 = dt_s * np.arange(n3)
    wt1 = np.ones(n1)
    wt1[0] = 0.5
    wt3 = np.ones(n3)
    wt3[0] = 0.5
    E1 = wt1[None, :] * np.exp(1j * np.outer(w1, t1))     # (2 n1, n1)
    E3 = wt3[None, :] * np.exp(1j * np.outer(w3, t3))     # (2 n3, n3)
    S = np.imag(dt_s * dt_s * (E3 @ R.T @ E1.T))
    return S


def correlation_spectrum(R_I, R_II, dt_s: float):
    """S_C(W3, W1) = sigma [S_I(W3, -W1) + S_II(W3, W1)]."""
    return SIGMA * (pathway_spectrum(R_I, dt_s, flip_w1=True) + pathway_spectrum(R_II, dt_s))


def linear_spectrum(R1, dt_s: float):
    """I(W) = sum_k w_k dt_s exp(i W t_k) R1(t_k) on the 2n grid (complex)."""
    n = len(R1)
    w = frequency_grid(n, dt_s)
    t = dt_s * np.arange(n)
    wt = np.ones(n)
    wt[0] = 0.5
    return np.array([dt_s * np.sum(wt * np.exp(1j * W * t) * R1) for W in w])

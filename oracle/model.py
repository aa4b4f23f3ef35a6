"""System operators of the MAB model in the product eigenbasis (oracle).

Paper, Sec. II.A.  Units hbar = 1, dimensionless coordinates, m_s = 1 in the
bath formulas.  For every mode s:

  * H_A = omega (p^2 + q^2)/2 + g3 q^3/3! + g4 q^4/4!   (Eqs. System
    Hamiltonian and Potentials; the quartic term is optional),
  * V_s(q) = V1 q + V2 q^2/2                              (Eq. h_int),
  * counter term H_C = Lambda V_s(q)^2 with Lambda = zeta gamma / 2
    (Eqs. counter Hamiltonian, counterterm, counter2).

Operators q^k, p^2 and V(q)^2 are built from harmonic-oscillator ladder
operators in an (N_b + 4)-level basis and then restricted to N_b levels, which
gives exact matrix elements for powers up to four.  H_A is diagonalised in the
N_b levels and the n_keep lowest eigenvectors U are kept (largest-magnitude
component made positive).  In that basis

  Q1 = U^T q U,  Q2 = U^T q^2 U,  v_s = V1 Q1 + V2 Q2 / 2,
  delta_s = Lambda U^T V(q)^2 U      (Eq. counter2),

and the product basis (mode 0 slowest, Sec. II.A) carries

  H_S' = sum_s [diag(E_s) + delta_s]_s
         + sum_{s<t} g_st Q1_s Q1_t + (g_s2t Q2_s Q1_t + g_st2 Q1_s Q2_t)/6
                                                   (Eqs. Potential ss',
                                                    total_hamiltonian),
  mu   = sum_s mu1_s Q1_s + 1/2 sum_s mu2_s Q2_s + sum_{s<t} mu_st Q1_s Q1_t
                                                   (Eq. NLdip),
  V_s  = v_s acting on mode s (identity on the others)  (Eq. sys_interaction).

Rotating-wave split of the dipole used for the rephasing / non-rephasing
pathways: with N(a) the total number of kept quanta of product state a,
mu_plus[a, b] = mu[a, b] if N(a) > N(b) else 0, and mu_minus = mu_plus^T.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import bath
from .hierarchy import Hierarchy


def ladder(n: int):
    """Annihilation operator a in an n-level harmonic-oscillator basis."""
    a = np.zeros((n, n))
    for k in range(1, n):
        a[k - 1, k] = np.sqrt(k)
    return a


@dataclass
class ModeOps:
    E: np.ndarray        # kept eigenvalues of H_A, ascending
    U: np.ndarray        # N_b x n_keep eigenvectors
    Q1: np.ndarray       # U^T q U
    Q2: np.ndarray       # U^T q^2 U
    v: np.ndarray        # V1 Q1 + V2 Q2 / 2
    delta: np.ndarray    # Lambda U^T V(q)^2 U
    Lam: float


def single_mode(mode) -> ModeOps:
    nb = int(mode["n_basis"])
    big = nb + 4
    a = ladder(big)
    q = (a + a.T) / np.sqrt(2.0)
    d = a - a.T
    p2 = -(d @ d) / 2.0
    q2 = q @ q
    q3 = q2 @ q
    q4 = q3 @ q
    Vq = mode["V1"] * q + mode["V2"] * q2 / 2.0
    V2op = Vq @ Vq
    HA = mode["omega"] * (p2 + q2) / 2.0 + mode["g3"] * q3 / 6.0 + mode["g4"] * q4 / 24.0
    HA = HA[:nb, :nb]
    w, U = np.linalg.eigh(HA)
    keep = int(mode["n_keep"])
    w, U = w[:keep], U[:, :keep].copy()
    for i in range(keep):
        k = int(np.argmax(np.abs(U[:, i])))
        if U[k, i] < 0:
            U[:, i] = -U[:, i]
    Q1 = U.T @ q[:nb, :nb] @ U
    Q2 = U.T @ q2[:nb, :nb] @ U
    v = mode["V1"] * Q1 + mode["V2"] * Q2 / 2.0
    Lam = mode["zeta"] * mode["gamma"] / 2.0
    delta = Lam * (U.T @ V2op[:nb, :nb] @ U)
    return ModeOps(E=w, U=U, Q1=Q1, Q2=Q2, v=v, delta=delta, Lam=Lam)


def embed(ops_by_mode, dims):
    """Kronecker product over modes; ops_by_mode maps mode -> matrix, others identity."""
    out = np.ones((1, 1))
    for s, ds in enumerate(dims):
        out = np.kron(out, ops_by_mode.get(s, np.eye(ds)))
    return out


def quanta(dims):
    """N(a) = total number of kept quanta of each product state (mode 0 slowest)."""
    N = np.zeros(1, dtype=np.int64)
    for ds in dims:
        N = (N[:, None] + np.arange(ds)[None, :]).reshape(-1)
    return N


@dataclass
class Model:
    """Everything the HEOM needs: operators, bath terms and the hierarchy."""
    H: np.ndarray                 # d x d real symmetric H_S'
    V: list                       # per mode: full d x d V_s
    mu: np.ndarray                # d x d dipole
    mu_plus: np.ndarray
    mu_minus: np.ndarray
    term_mode: np.ndarray         # mode of each exponential term j
    nu: np.ndarray                # nu_j (real, or complex for a Brownian bath)
    c: np.ndarray                 # c_j (complex)
    hier: Hierarchy
    dt: float = 0.01
    dims: tuple = ()
    modes: list = field(default_factory=list)
    cb: np.ndarray = None         # bra-side coefficients; None means conj(c)

    @property
    def d(self):
        return self.H.shape[0]

    @property
    def gamma_sum(self):
        """sum_j n_j nu_j for every ADO."""
        return self.hier.n @ self.nu

    @property
    def c_bra(self):
        """Coefficients of the bra-side coupling (conj(c) for real rates)."""
        return np.conj(self.c) if self.cb is None else self.cb


def make_model(H, V, mu, term_mode, nu, c, depth, dt=0.01, dims=None, modes=None, cb=None, rate_cut=0.0):
    """Assemble a Model from explicit operators (used by engine-level checks).

    Complex rates nu_j (Brownian baths) need the bra-side coefficients cb;
    by default they are derived from (nu, c) by bath.bra_coefficients.
    """
    d = H.shape[0]
    dims = tuple(dims) if dims is not None else (d,)
    if int(np.prod(dims)) != d:
        raise ValueError("mode dimensions do not multiply to d")
    N = quanta(dims)
    mu = np.asarray(mu, dtype=float)
    mu_plus = np.where(N[:, None] > N[None, :], mu, 0.0)
    hier = Hierarchy(len(nu), depth, np.real(np.asarray(nu, dtype=complex)), rate_cut)
    nu = np.asarray(nu, dtype=complex)
    c = np.asarray(c, dtype=complex)
    if np.all(nu.imag == 0):
        nu = nu.real.copy()
        cb = None if cb is None else np.asarray(cb, dtype=complex)
    elif cb is None:
        # each bath's correlation is conjugated on its own terms
        tm = np.asarray(term_mode)
        cb = np.empty_like(c)
        for s in np.unique(tm):
            sel = tm == s
            cb[sel] = bath.bra_coefficients(nu[sel], c[sel])
    return Model(H=np.asarray(H, dtype=float), V=[np.asarray(v, dtype=float) for v in V],
                 mu=mu, mu_plus=mu_plus, mu_minus=mu_plus.T.copy(),
                 term_mode=np.asarray(term_mode, dtype=np.int64),
                 nu=nu, c=c, hier=hier, dt=dt, dims=dims, modes=list(modes or []), cb=cb)


def flip_sign(m: ModeOps, i: int) -> ModeOps:
    """Same mode with eigenvector i negated (physical results must not change)."""
    S = np.ones(len(m.E))
    S[i] = -1.0
    return ModeOps(E=m.E, U=m.U * S[None, :], Q1=S[:, None] * m.Q1 * S[None, :],
                   Q2=S[:, None] * m.Q2 * S[None, :], v=S[:, None] * m.v * S[None, :],
                   delta=S[:, None] * m.delta * S[None, :], Lam=m.Lam)


def build(params) -> Model:
    """Model from a parameter dictionary (layout documented in workloads.configs)."""
    return build_from_modes(params, [single_mode(m) for m in params["modes"]])


def build_from_modes(params, modes) -> Model:
    """Product-basis model from already diagonalised single modes."""
    dims = tuple(len(m.E) for m in modes)
    H = np.zeros((int(np.prod(dims)),) * 2)
    for s, m in enumerate(modes):
        H += embed({s: np.diag(m.E) + m.delta}, dims)
    mu = np.zeros_like(H)
    for s, (m, p) in enumerate(zip(modes, params["modes"])):
        mu += p["mu1"] * embed({s: m.Q1}, dims) + 0.5 * p["mu2"] * embed({s: m.Q2}, dims)
    for cp in params.get("couplings", []):
        s, t = int(cp["s"]), int(cp["t"])
        if s == t:
            raise ValueError("coupling needs two different modes")
        if s > t:
            raise ValueError("couplings are given with s < t")
        ms, mt = modes[s], modes[t]
        H += cp["g_st"] * embed({s: ms.Q1, t: mt.Q1}, dims)
        H += cp["g_s2t"] / 6.0 * embed({s: ms.Q2, t: mt.Q1}, dims)
        H += cp["g_st2"] / 6.0 * embed({s: ms.Q1, t: mt.Q2}, dims)
        mu += cp["mu_st"] * embed({s: ms.Q1, t: mt.Q1}, dims)
    V = [embed({s: m.v}, dims) for s, m in enumerate(modes)]
    term_mode, nus, cs = [], [], []
    for s, p in enumerate(params["modes"]):
        if p.get("omega_b", 0.0) > 0.0:
            nu, c = bath.brownian_terms(p["zeta"], p["gamma"], p["omega_b"], params["beta"],
                                        int(p["K"]), params.get("decomp", "pade"))
        else:
            nu, c = bath.drude_terms(p["zeta"], p["gamma"], params["beta"], int(p["K"]),
                                     params.get("decomp", "pade"))
        term_mode += [s] * len(nu)
        nus += list(nu)
        cs += list(c)
    return make_model(H, V, mu, term_mode, nus, cs, int(params["depth"]),
                      dt=float(params["dt"]), dims=dims, modes=modes,
                      rate_cut=float(params.get("rate_cut", 0.0)))

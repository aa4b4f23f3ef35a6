"""Seeded parameter sets for the multi-mode anharmonic Brownian (MAB) model.

Every function returns a plain JSON-serialisable dictionary.  Units: hbar = 1,
energies in units of omega0 (the harmonic frequency of the first mode), time in
1/omega0, temperature given as beta*hbar*omega0.  Coordinates are dimensionless
and the bath formulas take m_s = 1.

Parameter dictionary layout (both the oracle and the C-ABI binding read it):

    {"modes": [{"omega", "g3", "g4", "V1", "V2", "zeta", "gamma",
                "mu1", "mu2", "n_basis", "n_keep", "K"}, ...],
     "couplings": [{"s", "t", "g_st", "g_s2t", "g_st2", "mu_st"}, ...],
     "beta", "depth", "decomp" ("pade" | "matsubara"), "dt",
     optional "rate_cut" (hierarchy filter; modes may add "omega_b")}

Mode keys follow the model of Sec. II.A: the potential
omega*q^2/2 + g3 q^3/3! + g4 q^4/4! (Eq. Potentials plus an optional quartic
term), the system-bath coupling V(q) = V1 q + V2 q^2/2 (Eq. h_int, LL and SL
parts), the Drude bath (zeta, gamma) of Eq. drude with K low-temperature terms,
and the dipole mu1 q + mu2 q^2/2 (Eq. NLdip, diagonal part).  Coupling keys
are the coefficients of Eq. Potential ss' (g_st q_s q_t, g_s2t q_s^2 q_t / 6,
g_st2 q_s q_t^2 / 6) and the cross dipole mu_st q_s q_t.

The workloads stand in for the paper's water models (Tables I-III), which are
not a public benchmark: they keep the structure (two stretches plus a bend,
cubic/quartic anharmonicity, bilinear and Fermi couplings, Drude baths, a
handful of levels per mode) with seeded draws.
"""

from __future__ import annotations

import math

import numpy as np

# 1/omega0 in femtoseconds for omega0 = 3470 cm^-1 (the symmetric stretch).
FS_PER_TIME_UNIT = 1.0e15 / (2.0 * math.pi * 2.99792458e10 * 3470.0)


def fs_to_steps(t_fs: float, dt: float) -> int:
    """Number of RK4 steps of size dt closest to t_fs femtoseconds."""
    return int(round(t_fs / FS_PER_TIME_UNIT / dt))


def _mode(rng, omega, n_keep, K, zeta=0.1, gamma=0.2, mu1=1.0, mu2=0.2,
          n_basis=12):
    g3 = float(rng.uniform(-0.3, -0.1))
    g4 = float(rng.uniform(0.01, 0.05))
    V1 = float(rng.uniform(0.5, 1.0))
    V2 = float(rng.uniform(0.0, 0.2))
    return {"omega": float(omega), "g3": g3, "g4": g4, "V1": V1, "V2": V2,
            "zeta": float(zeta), "gamma": float(gamma), "mu1": float(mu1),
            "mu2": float(mu2), "n_basis": int(n_basis), "n_keep": int(n_keep),
            "K": int(K)}


def _coupling(s, t, g_st=0.0, g_s2t=0.0, g_st2=0.0, mu_st=0.0):
    return {"s": int(s), "t": int(t), "g_st": float(g_st),
            "g_s2t": float(g_s2t), "g_st2": float(g_st2),
            "mu_st": float(mu_st)}


def response_grid(n, steps_per_sample, t2_steps):
    """t1/t3 grid of n samples spaced steps_per_sample RK4 steps apart."""
    return {"n1": int(n), "n3": int(n), "steps_per_sample": int(steps_per_sample),
            "t2_steps": [int(s) for s in t2_steps]}


def cfg1(seed: int = 0):
    """One anharmonic mode, 6 kept levels, K=2 Matsubara terms, depth 4.

    35 ADOs of 6x6; dt = 0.01; 32x32 grid at t2 = 0.
    """
    rng = np.random.default_rng(seed)
    m = _mode(rng, 1.0, n_keep=6, K=2, mu1=1.0, mu2=0.2)
    params = {"modes": [m], "couplings": [], "beta": 10.0, "depth": 4,
              "decomp": "matsubara", "dt": 0.01}
    return params, response_grid(32, 100, [0])


def cfg2(seed: int = 0):
    """Two coupled modes (omega 1.0 : 0.45), 5x5 states, K=2 Pade, depth 5.

    462 ADOs of 25x25; dt = 0.1; 64x64 grid at t2 in {0, 100 fs}.
    """
    rng = np.random.default_rng(seed)
    modes = [_mode(rng, 1.0, n_keep=5, K=2), _mode(rng, 0.45, n_keep=5, K=2)]
    g12 = float(rng.uniform(0.0, 0.05))
    g122 = float(rng.uniform(0.0, 0.05))
    couplings = [_coupling(0, 1, g_st=g12, g_st2=g122, mu_st=0.02)]
    params = {"modes": modes, "couplings": couplings, "beta": 10.0,
              "depth": 5, "decomp": "pade", "dt": 0.1}
    return params, response_grid(64, 10, [0, fs_to_steps(100.0, 0.1)])


def cfg3(seed: int = 0, depth: int = 6):
    """Water-like three-mode model: sym/asym stretch and bend (1 : 1.03 : 0.44).

    4x4x5 = 80 states, K=2 Pade per mode (9 exponential terms), depth 6
    (5005 ADOs of 80x80); dt = 0.1; 128x128 grid at t2 = 0, 50, 100, 200 fs.
    """
    rng = np.random.default_rng(seed)
    modes = [_mode(rng, 1.0, n_keep=4, K=2), _mode(rng, 1.03, n_keep=4, K=2),
             _mode(rng, 0.44, n_keep=5, K=2)]
    g01, g02, g12 = (float(x) for x in rng.uniform(0.0, 0.05, size=3))
    f02, f12 = (float(x) for x in rng.uniform(0.0, 0.05, size=2))
    couplings = [_coupling(0, 1, g_st=g01, mu_st=0.02),
                 _coupling(0, 2, g_st=g02, g_st2=f02, mu_st=0.02),
                 _coupling(1, 2, g_st=g12, g_st2=f12, mu_st=0.02)]
    params = {"modes": modes, "couplings": couplings, "beta": 10.0,
              "depth": int(depth), "decomp": "pade", "dt": 0.1}
    t2 = [0] + [fs_to_steps(t, 0.1) for t in (50.0, 100.0, 200.0)]
    return params, response_grid(128, 10, t2)


def _hierarchy_size(n_terms: int, depth: int) -> int:
    # size of the triangular index set {n in N^M : |n| <= L}; used only for
    # the redraw rule of the mixed-instance workload below
    return math.comb(n_terms + depth, depth)


def cfg4_instances(n_instances: int = 64, seed: int = 0):
    """Uneven batch: 1-3 modes (6, 25 or 80 states), K in {1,2}, depth 3..6.

    Draws whose hierarchy has fewer than 35 ADOs are redrawn.  Each instance
    has a 64x64 grid at t2 = 0 with dt = 0.1.
    """
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n_instances:
        n_modes = int(rng.integers(1, 4))
        Ks = [int(k) for k in rng.integers(1, 3, size=n_modes)]
        depth = int(rng.integers(3, 7))
        if _hierarchy_size(sum(k + 1 for k in Ks), depth) < 35:
            continue
        keep = {1: [6], 2: [5, 5], 3: [4, 4, 5]}[n_modes]
        omegas = {1: [1.0], 2: [1.0, 0.45], 3: [1.0, 1.03, 0.44]}[n_modes]
        modes = [_mode(rng, w, n_keep=k, K=K) for w, k, K in zip(omegas, keep, Ks)]
        couplings = []
        for s in range(n_modes):
            for t in range(s + 1, n_modes):
                couplings.append(_coupling(s, t, g_st=float(rng.uniform(0, 0.05)),
                                           g_st2=float(rng.uniform(0, 0.05)),
                                           mu_st=0.02))
        out.append(({"modes": modes, "couplings": couplings, "beta": 10.0,
                     "depth": depth, "decomp": "pade", "dt": 0.1},
                    response_grid(64, 10, [0])))
    return out


def cfg5(seed: int = 0):
    """Gradient workload: the three-mode depth-6 model, 64x64 grid, t2 in {0, 100 fs}.

    Returns (params, grid, theta_scale) where theta_scale holds the +-5%
    perturbation factors of the 12 fitted parameters (g3 x3, g4 x3, bilinear
    scale, Fermi scale, V1, V2, zeta, gamma) used to make the target spectrum.
    """
    params, _ = cfg3(seed)
    rng = np.random.default_rng(seed + 1000)
    r = rng.choice([-1.0, 1.0], size=12)
    grid = response_grid(64, 10, [0, fs_to_steps(100.0, 0.1)])
    return params, grid, [float(1.0 + 0.05 * x) for x in r]


def harmonic_pin(omega=1.0, zeta=0.1, gamma=0.2, V1=1.0, beta=10.0, K=2,
                 depth=4, n_keep=6, decomp="pade", dt=0.01, omega_b=0.0):
    """Harmonic mode with linear (LL) coupling and a linear dipole (Drude
    bath, or a Brownian bath of frequency omega_b when omega_b > 0)."""
    m = {"omega": omega, "g3": 0.0, "g4": 0.0, "V1": V1, "V2": 0.0,
         "zeta": zeta, "gamma": gamma, "mu1": 1.0, "mu2": 0.0,
         "n_basis": 12, "n_keep": n_keep, "K": K}
    if omega_b > 0.0:
        m["omega_b"] = float(omega_b)
    return {"modes": [m], "couplings": [], "beta": beta, "depth": depth,
            "decomp": decomp, "dt": dt}


def with_brownian_baths(params, omega_b=0.25, gamma=None):
    """Copy of params whose baths are Brownian (underdamped-oscillator)
    spectral densities of frequency omega_b (one value or one per mode)
    instead of Drude ones; zeta, K and the decomposition are kept, gamma
    optionally replaced.  Each mode then has K + 2 exponential terms."""
    import copy
    p = copy.deepcopy(params)
    wb = list(omega_b) if isinstance(omega_b, (list, tuple)) else [omega_b] * len(p["modes"])
    for m, x in zip(p["modes"], wb):
        m["omega_b"] = float(x)
        if gamma is not None:
            m["gamma"] = float(gamma)
    return p


def cfg3_brownian(seed: int = 0, depth: int = 5):
    """cfg3's three modes with Brownian baths (omega_b = 0.25, gamma = 0.2,
    K = 2 Pade): 12 exponential terms, 6188 ADOs of 80 x 80 at depth 5."""
    params, grid = cfg3(seed, depth=depth)
    return with_brownian_baths(params, 0.25), grid


def theta_size(params) -> int:
    """Number of fitted factors: g3 and g4 per mode, then bilinear and Fermi
    coupling scales, then common V1, V2, zeta and gamma scales."""
    return 2 * len(params["modes"]) + 6


def apply_theta(params, theta):
    """Parameters with the multiplicative factors theta applied (theta = 1: unchanged)."""
    import copy
    n = len(params["modes"])
    theta = [float(x) for x in theta]
    if len(theta) != theta_size(params):
        raise ValueError("theta has the wrong length")
    p = copy.deepcopy(params)
    for s, m in enumerate(p["modes"]):
        m["g3"] *= theta[s]
        m["g4"] *= theta[n + s]
        m["V1"] *= theta[2 * n + 2]
        m["V2"] *= theta[2 * n + 3]
        m["zeta"] *= theta[2 * n + 4]
        m["gamma"] *= theta[2 * n + 5]
    for c in p.get("couplings", []):
        c["g_st"] *= theta[2 * n]
        c["g_s2t"] *= theta[2 * n + 1]
        c["g_st2"] *= theta[2 * n + 1]
    return p


def theta_directions(params):
    """d params / d theta_i for every factor (params are linear in theta): one
    dictionary per factor with the same layout, every number set to the
    derivative of that field (zero where theta_i does not enter)."""
    import copy
    out = []
    for i in range(theta_size(params)):
        e = [0.0] * theta_size(params)
        e[i] = 1.0
        p = copy.deepcopy(params)
        n = len(p["modes"])
        for s, (m, m0) in enumerate(zip(p["modes"], params["modes"])):
            for key in ("omega", "g3", "g4", "V1", "V2", "zeta", "gamma", "mu1", "mu2"):
                m[key] = 0.0
            m["g3"] = m0["g3"] * e[s]
            m["g4"] = m0["g4"] * e[n + s]
            m["V1"] = m0["V1"] * e[2 * n + 2]
            m["V2"] = m0["V2"] * e[2 * n + 3]
            m["zeta"] = m0["zeta"] * e[2 * n + 4]
            m["gamma"] = m0["gamma"] * e[2 * n + 5]
        for c, c0 in zip(p.get("couplings", []), params.get("couplings", [])):
            c["g_st"] = c0["g_st"] * e[2 * n]
            c["g_s2t"] = c0["g_s2t"] * e[2 * n + 1]
            c["g_st2"] = c0["g_st2"] * e[2 * n + 1]
            c["mu_st"] = 0.0
        p["beta"] = 0.0
        out.append(p)
    return out


# ---------------------------------------------------------------------------
# The paper's water models (Sec. IV, Tables I-III).  Their energy unit is
# omega0 = 4000 cm^-1, so these dictionaries use it (not the 3470 cm^-1 of
# the seeded workloads): time unit 1/omega0 = 1.3271 fs.

WATER_OMEGA0_CM = 4000.0
FS_PER_TIME_UNIT_WATER = 1.0e15 / (2.0 * math.pi * 2.99792458e10 * WATER_OMEGA0_CM)
_CM_PER_KELVIN = 0.69503476   # k_B / (h c) in cm^-1 per K

# Table rows: (nu_s [cm^-1], gamma_s/omega0, zeta~, V_LL~, V_SL~, g_{s^3}~, mu_s~, mu_ss~)
_WATER_STRETCH_2 = (3520.0, 5.0e-3, 9.0, 0.0, 1.0, -0.5, 3.3, 1.2e-2)
_WATER_BEND = (1710.0, 2.0e-2, 0.8, 0.0, 1.0, -0.7, 1.8, 0.0)
_WATER_ASYM = (3570.0, 5.0e-3, 9.0, 0.0, 1.0, -0.5, 3.3, 1.2e-2)
_WATER_SYM = (3470.0, 5.0e-3, 9.0, 0.0, 1.0, -0.5, 3.3, 1.2e-2)
# Table III: (s, t, g_st~, g_s2t~, g_st2~, mu_st~) for 1-1', 1-2, 1'-2
# (the garbled "-2,6 x 10^-2" read as -2.6e-2)
_WATER_3_COUPLINGS = ((0, 1, -5.0e-3, 0.32, -4.2e-3, 0.0),
                      (0, 2, 1.0e-7, -2.6e-2, 4.0e-4, 2.0e-3),
                      (1, 2, -8.0e-4, 1.2e-1, -1.2e-2, 2.0e-3))


def _water_mode(row, n_keep, K, n_basis):
    """One mode from a table row.  Reading of the caption's normalisations:
    each relation x~ = f x is applied as x = f x~ (the literal direction,
    x = x~ / f, gives the bend a cubic barrier far below its zero-point
    energy), with mu_0 and nu_0 read as omega0:
    zeta = (omega0/omega_s)^2 zeta~, V_LL = (omega_s/omega0) V_LL~,
    V_SL = V_SL~, g3 = (omega_s/omega0)^3 g~, mu_s = (omega0/omega_s) mu~,
    mu_ss = (omega0/omega_s)^2 mu_ss~.  No quartic term (the tables give
    none)."""
    nu, gam, zeta_t, vll_t, vsl_t, g3_t, mu_t, muss_t = row
    r = nu / WATER_OMEGA0_CM
    return {"omega": r, "g3": g3_t * r ** 3, "g4": 0.0, "V1": vll_t * r, "V2": vsl_t,
            "zeta": zeta_t / r ** 2, "gamma": gam, "mu1": mu_t / r, "mu2": muss_t / r ** 2,
            "n_basis": int(n_basis), "n_keep": int(n_keep), "K": int(K)}


def water_beta(temperature_k: float = 300.0) -> float:
    """beta hbar omega0 at the given temperature (the paper states none; 300 K
    is assumed)."""
    return WATER_OMEGA0_CM / (_CM_PER_KELVIN * float(temperature_k))


def water_two_mode(n_levels: int = 4, K: int = 4, depth: int = 4, dt_fs: float = 0.25,
                   temperature_k: float = 300.0, n_basis: int = 16):
    """Table I: OH stretch (3520 cm^-1) and bend (1710 cm^-1), n_levels kept
    eigenstates each, K Pade terms per mode, Fermi coupling g_{11'^2}~ = 0.2
    and cross dipole 2e-3 (the caption's 1' labels read as the bend; no
    bilinear or g_{1^2 1'} term).  Depth 4 at the paper's dt = 0.25 fs (depth 5
    leaves the RK4 stability region for the fastest Pade rate; use
    dt_fs = 0.2 there)."""
    modes = [_water_mode(_WATER_STRETCH_2, n_levels, K, n_basis),
             _water_mode(_WATER_BEND, n_levels, K, n_basis)]
    couplings = [_coupling(0, 1, g_st=0.0, g_s2t=0.0, g_st2=0.2, mu_st=2.0e-3)]
    return {"modes": modes, "couplings": couplings, "beta": water_beta(temperature_k),
            "depth": int(depth), "decomp": "pade", "dt": float(dt_fs) / FS_PER_TIME_UNIT_WATER}


def water_three_mode(n_levels: int = 4, K: int = 4, depth: int = 4, dt_fs: float = 0.25,
                     temperature_k: float = 300.0, n_basis: int = 16):
    """Tables II-III: asymmetric (3570) and symmetric (3470 cm^-1) stretches
    and the bend (1710 cm^-1), n_levels kept eigenstates each (d = 64 at
    four), K Pade terms per mode (M = 3 (K + 1) = 15 at K = 4), the
    strong-coupling intermode terms of Table III.  Depth 4 (3876 ADOs) at
    dt = 0.25 fs, as for the two-mode model."""
    modes = [_water_mode(_WATER_ASYM, n_levels, K, n_basis),
             _water_mode(_WATER_SYM, n_levels, K, n_basis),
             _water_mode(_WATER_BEND, n_levels, K, n_basis)]
    couplings = [_coupling(s, t, g_st=a, g_s2t=b, g_st2=c, mu_st=m)
                 for s, t, a, b, c, m in _WATER_3_COUPLINGS]
    return {"modes": modes, "couplings": couplings, "beta": water_beta(temperature_k),
            "depth": int(depth), "decomp": "pade", "dt": float(dt_fs) / FS_PER_TIME_UNIT_WATER}


def cfg5_small(seed: int = 0):
    """Reduced gradient workload (same layout as cfg5): two anharmonic modes
    kept at 3 and 2 levels (d = 6) with bilinear and Fermi couplings, K = 1 Pade
    term per mode, depth 2 (15 ADOs), dt = 0.1, a 6 x 6 grid every 4 steps and
    t2 in {0, 8 steps}.  Returns (params, grid, theta_target)."""
    rng = np.random.default_rng(seed + 77)
    modes = [_mode(rng, 1.0, n_keep=3, K=1), _mode(rng, 0.45, n_keep=2, K=1)]
    modes[0]["n_basis"] = 8
    modes[1]["n_basis"] = 8
    couplings = [_coupling(0, 1, g_st=float(rng.uniform(0.02, 0.05)),
                           g_s2t=float(rng.uniform(0.02, 0.05)),
                           g_st2=float(rng.uniform(0.02, 0.05)), mu_st=0.02)]
    params = {"modes": modes, "couplings": couplings, "beta": 10.0, "depth": 2,
              "decomp": "pade", "dt": 0.1}
    r = rng.choice([-1.0, 1.0], size=theta_size(params))
    return params, response_grid(6, 4, [0, 8]), [float(1.0 + 0.05 * x) for x in r]


def paper_scale(seed: int = 0, depth: int = 5, temperature_k: float = 300.0):
    """The hierarchy scale of the paper's own water runs: three modes (sym,
    asym stretch, bend; 1 : 1.03 : 0.44) kept at 4 levels each (d = 64), K = 4
    Pade terms per mode (15 exponential terms), depth 5 (15,504 ADOs); the
    temperature is an assumption (300 K: beta hbar omega0 = 3470 / 208.5);
    other parameters drawn as in cfg3; dt = 0.1, 64 x 64 grid at t2 = 0."""
    rng = np.random.default_rng(seed + 500)
    modes = [_mode(rng, 1.0, n_keep=4, K=4), _mode(rng, 1.03, n_keep=4, K=4),
             _mode(rng, 0.44, n_keep=4, K=4)]
    g01, g02, g12 = (float(x) for x in rng.uniform(0.0, 0.05, size=3))
    f02, f12 = (float(x) for x in rng.uniform(0.0, 0.05, size=2))
    couplings = [_coupling(0, 1, g_st=g01, mu_st=0.02),
                 _coupling(0, 2, g_st=g02, g_st2=f02, mu_st=0.02),
                 _coupling(1, 2, g_st=g12, g_st2=f12, mu_st=0.02)]
    beta = 3470.0 / (0.69503476 * float(temperature_k))
    params = {"modes": modes, "couplings": couplings, "beta": beta,
              "depth": int(depth), "decomp": "pade", "dt": 0.1}
    return params, response_grid(64, 10, [0])

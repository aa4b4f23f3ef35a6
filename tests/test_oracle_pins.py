"""Pins of the CPU oracle against what the theory fixes (no GPU).

Each test ties one part of the oracle to a closed form, an exact invariant, a
textbook special case or a brute-force computation that does not reuse the
piece under test.
"""

import itertools
import math

import mpmath
import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sla

import workloads as w
from oracle import bath, heom, hierarchy
from oracle import model as om


# ---------------------------------------------------------------- bath ------

def test_pade_k1_by_hand():
    # [0/1] Pade of F(z) = 1/6 - z/360 + ...: (1/6)/(1 + z/60) = 10/(z + 60),
    # so 4 eta = 10 and xi^2 = 60.
    xi, eta = bath.pade_poles(1)
    assert xi[0] == pytest.approx(math.sqrt(60.0), rel=1e-14)
    assert eta[0] == pytest.approx(2.5, rel=1e-14)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_pade_order_of_contact(K):
    # coth(x/2) - approx = O(x^(4K+1)) as x -> 0 because the Pade approximant
    # matches 2K Taylor coefficients of F(z), z = x^2.  Measured against
    # high-precision coth, halving x must shrink the error by 2^(4K+1).
    xi, eta = bath.pade_poles(K, high_precision=True)
    mpmath.mp.dps = 60

    def err(x):
        x = mpmath.mpf(x)
        approx = 2 / x + sum(4 * e * x / (x * x + s ** 2) for s, e in zip(xi, eta))
        return abs(mpmath.coth(x / 2) - approx)

    ratio = float(err(0.4) / err(0.2))
    assert ratio == pytest.approx(2.0 ** (4 * K + 1), rel=0.05)


def test_pade_accuracy_and_matsubara_limit():
    x = np.linspace(0.05, 10.0, 400)
    exact = 1.0 / np.tanh(x / 2)
    e2 = np.max(np.abs(bath.coth_approx(x, *bath.pade_poles(2)) - exact))
    e4 = np.max(np.abs(bath.coth_approx(x, *bath.pade_poles(4)) - exact))
    assert 1e-3 < e2 < 1e-2
    assert e4 < 1e-6
    # many Pade poles: the lowest ones approach the Matsubara frequencies 2 pi k
    xi, eta = bath.pade_poles(16)
    np.testing.assert_allclose(xi[:3], 2 * np.pi * np.arange(1, 4), rtol=1e-9)
    np.testing.assert_allclose(eta[:3], 1.0, rtol=1e-9)
    # Matsubara sum converges to coth slowly (error ~ 1/K)
    xm, em = bath.matsubara_poles(4000)
    assert abs(bath.coth_approx(np.array([3.0]), xm, em)[0] - 1 / np.tanh(1.5)) < 1e-3


def test_bath_correlation_matches_fdt_integral():
    # C(t) = int_0^inf J(w) [coth(beta w / 2) cos(wt) - i sin(wt)] dw with the
    # Drude density J = (zeta/pi) gamma^2 w/(w^2 + gamma^2), the normalisation
    # for which int J/w dw = zeta gamma / 2 = Lambda (Eqs. SDF, counter4,
    # counterterm).  The exponential terms must reproduce it for t > 0; the
    # [K-1/K] decomposition drops only a part concentrated at short times.
    zeta, gamma, beta = 0.1, 0.2, 10.0

    def J(x):
        return zeta / np.pi * gamma ** 2 * x / (x * x + gamma ** 2)

    def J_coth(x):
        g = 2.0 / beta if x == 0 else x / np.tanh(beta * x / 2)
        return zeta / np.pi * gamma ** 2 / (x * x + gamma ** 2) * g

    lam = si.quad(lambda x: zeta / np.pi * gamma ** 2 / (x * x + gamma ** 2), 0, np.inf)[0]
    assert lam == pytest.approx(zeta * gamma / 2, rel=1e-10)

    def err(K, t):
        nu, c = bath.drude_terms(zeta, gamma, beta, K, "pade")
        re = si.quad(J_coth, 0, np.inf, weight="cos", wvar=t, limlst=200)[0]
        # -int J sin(wt) dw has the closed form -(zeta gamma^2/2) exp(-gamma t)
        im = -si.quad(J, 0, np.inf, weight="sin", wvar=t, limlst=200)[0]
        C = np.sum(c * np.exp(-nu * t))
        assert abs(im + zeta * gamma ** 2 / 2 * np.exp(-gamma * t)) < 1e-7 * abs(c[0])
        assert abs(C.imag + zeta * gamma ** 2 / 2 * np.exp(-gamma * t)) < 1e-15
        return abs(C.real - re) / abs(c[0])

    for t in (1.0, 2.0, 5.0, 9.0):
        assert err(12, t) < 1e-7
    assert err(2, 5.0) < 1e-4 and err(2, 9.0) < 1e-4
    assert err(2, 2.0) > err(4, 2.0) > err(12, 2.0)


def test_brownian_density_normalisation_and_overdamped_limit():
    # int J/w dw = zeta gamma / 2 (the Drude Lambda, so the counter term is
    # shared); for gamma >> omega_b the density is the Drude one of cutoff
    # omega_b^2/gamma with the same Lambda.
    zeta, gamma, wb = 0.1, 0.5, 2.0
    lam = si.quad(lambda x: bath.brownian_density(x, zeta, gamma, wb) / x, 0, np.inf, limit=400)[0]
    assert lam == pytest.approx(zeta * gamma / 2, rel=1e-9)
    g, wb2 = 400.0, 2.0
    G = wb2 ** 2 / g
    zd = zeta * g / G
    x = np.array([0.01, 0.1, 0.3, 1.0])
    drude = zd / np.pi * G ** 2 * x / (x * x + G ** 2)
    np.testing.assert_allclose(bath.brownian_density(x, zeta, g, wb2), drude, rtol=1e-3)


@pytest.mark.parametrize("gamma,wb", [(0.2, 1.0), (0.5, 2.0), (3.0, 1.0)])
def test_brownian_correlation_matches_fdt_integral(gamma, wb):
    # C(t) = int_0^inf J(w) [coth(beta w/2) cos wt - i sin wt] dw for the
    # Brownian density, by quadrature: (i) with coth replaced by the very
    # decomposition the terms use, the residue sum is exact for t > 0;
    # (ii) with the exact coth, K = 12 Pade terms converge to it; (iii) the
    # imaginary part has the closed form -(zeta gamma wb^2/(2 r)) e^{-gamma t/2}
    # sin(r t), r = sqrt(wb^2 - gamma^2/4) (a sinh for the overdamped case).
    zeta, beta = 0.1, 10.0

    def J(x):
        return bath.brownian_density(x, zeta, gamma, wb)

    def re_part(t, coth):
        def f(x):
            return 2.0 / beta * J(1e-300) / 1e-300 if x == 0 else J(x) * coth(x)
        return si.quad(f, 0, np.inf, weight="cos", wvar=t, limlst=400, limit=400)[0]

    r = np.sqrt(complex(wb ** 2 - gamma ** 2 / 4))
    xi2, eta2 = bath.pade_poles(2)
    nu2, c2 = bath.brownian_terms(zeta, gamma, wb, beta, 2, "pade")
    nu12, c12 = bath.brownian_terms(zeta, gamma, wb, beta, 12, "pade")
    scale = np.max(np.abs(c12))
    for t in (1.0, 3.0, 7.0):
        im_closed = np.real(-(zeta * gamma * wb ** 2 / (2 * r)) * np.exp(-gamma * t / 2) * np.sin(r * t))
        im_quad = -si.quad(J, 0, np.inf, weight="sin", wvar=t, limlst=400, limit=400)[0]
        assert abs(im_quad - im_closed) < 1e-7 * scale
        for nu, c in ((nu2, c2), (nu12, c12)):
            C = np.sum(c * np.exp(-nu * t))
            assert abs(C.imag - im_closed) < 1e-13 * scale
        # coth_approx(beta w) is the decomposed coth(beta w / 2)
        dec = re_part(t, lambda x: bath.coth_approx(np.array([beta * x]), xi2, eta2)[0])
        assert abs(np.sum(c2 * np.exp(-nu2 * t)).real - dec) < 1e-8 * scale
        exact = re_part(t, lambda x: 1.0 / np.tanh(beta * x / 2))
        assert abs(np.sum(c12 * np.exp(-nu12 * t)).real - exact) < 1e-6 * scale
    # C(0) is real: the imaginary parts of the pair cancel
    assert abs(np.sum(c12).imag) < 1e-15 * scale


@pytest.mark.parametrize("decomp", ["pade", "matsubara"])
@pytest.mark.parametrize("K", [1, 2, 4])
def test_zero_frequency_sum_rule(decomp, K):
    # int_0^inf Re C(t) dt = (pi/beta) J'(0) for any coth decomposition with
    # the exact 2/x pole: sum_j Re(c_j/nu_j) must reproduce zeta/beta (Drude)
    # and zeta gamma^2/(beta wb^2) (Brownian); the imaginary parts integrate
    # to -int J(w)/w dw = -Lambda.
    z, g, b, wb = 0.1, 0.2, 10.0, 0.7
    nu, c = bath.drude_terms(z, g, b, K, decomp)
    assert np.sum(c / nu).real == pytest.approx(z / b, rel=1e-12)
    assert np.sum(c / nu).imag == pytest.approx(-z * g / 2, rel=1e-12)
    nu, c = bath.brownian_terms(z, g, wb, b, K, decomp)
    assert np.sum(c / nu).real == pytest.approx(z * g * g / (b * wb * wb), rel=1e-12)
    assert np.sum(c / nu).imag == pytest.approx(-z * g / 2, rel=1e-12)


def test_bra_coefficients_pairing():
    nu, c = bath.brownian_terms(0.1, 0.2, 1.0, 10.0, 2)
    cb = bath.bra_coefficients(nu, c)
    assert abs(nu[0] - np.conj(nu[1])) < 1e-15
    assert cb[0] == np.conj(c[1]) and cb[1] == np.conj(c[0])
    np.testing.assert_array_equal(cb[2:], np.conj(c[2:]))
    np.testing.assert_array_equal(bath.bra_coefficients(nu, cb), c)
    nd, cd = bath.drude_terms(0.1, 0.2, 10.0, 3)
    np.testing.assert_array_equal(bath.bra_coefficients(nd, cd), np.conj(cd))
    # C(t)* = sum_j cb_j exp(-nu_j t)
    for t in (0.5, 2.0):
        assert abs(np.conj(np.sum(c * np.exp(-nu * t))) - np.sum(cb * np.exp(-nu * t))) < 1e-16


def test_bath_singular_gamma_rejected():
    xi, _ = bath.pade_poles(2)
    with pytest.raises(ValueError):
        bath.drude_terms(0.1, xi[0] / 10.0, 10.0, 2, "pade")


# ----------------------------------------------------------- hierarchy ------

@pytest.mark.parametrize("M,L,N,NL", [(3, 4, 35, 15), (6, 5, 462, 252), (9, 6, 5005, 3003)])
def test_hierarchy_counts(M, L, N, NL):
    h = hierarchy.Hierarchy(M, L)
    assert len(h) == N == math.comb(M + L, L)
    assert int(np.sum(h.n.sum(1) == L)) == NL
    # neighbour maps are mutually inverse
    for j in range(M):
        has = h.down[:, j] >= 0
        assert np.all(h.up[h.down[has, j], j] == np.nonzero(has)[0])
    # ordered by depth, unique
    assert np.all(np.diff(h.n.sum(1)) >= 0)
    assert len(set(map(tuple, h.n))) == N


def test_hierarchy_brute_force_small():
    h = hierarchy.Hierarchy(3, 3)
    brute = {n for n in np.ndindex(4, 4, 4) if sum(n) <= 3}
    assert set(map(tuple, h.n.tolist())) == brute


# -------------------------------------------------------- single mode -------

def test_rate_filtered_hierarchy_brute_force_and_closure():
    rates = np.array([0.2, 0.63, 1.95, 0.1])
    for cut in (0.5, 1.3, 2.0, 100.0):
        h = hierarchy.Hierarchy(4, 4, rates, cut)
        brute = [n for n in itertools.product(range(5), repeat=4)
                 if sum(n) <= 4 and float(np.dot(n, rates)) <= cut * (1 + 1e-9)]
        assert sorted(h.ados, key=lambda n: (sum(n), n)) == h.ados
        assert set(h.ados) == set(brute)
        for i, n in enumerate(h.ados):  # closed under n -> n - e_j
            for j in range(4):
                if n[j] > 0:
                    assert h.down[i, j] >= 0
    assert hierarchy.Hierarchy(4, 4, rates, 100.0).ados == hierarchy.Hierarchy(4, 4).ados


def test_rate_filtered_rhs_is_restricted_full_rhs():
    # truncating the index set means the removed ADOs are zero: the filtered
    # generator equals P L P^T with P the restriction to the kept ADOs
    p, _ = w.cfg2()
    p["depth"] = 3
    full = om.build(p)
    p["rate_cut"] = 0.9
    filt = om.build(p)
    assert 0 < len(filt.hier) < len(full.hier)
    keep = np.array([full.hier.index[n] for n in filt.hier.ados])
    x = w.random_hierarchy(1, len(filt.hier), filt.d, seed=4)[0]
    X = np.zeros((len(full.hier), full.d, full.d), dtype=complex)
    X[keep] = x
    np.testing.assert_allclose(heom.rhs(filt, x), heom.rhs(full, X)[keep], atol=1e-14)
    np.testing.assert_allclose(heom.rhs(filt, x, adjoint=True), heom.rhs(full, X, adjoint=True)[keep],
                               atol=1e-14)


def test_harmonic_mode_ladder():
    mode = dict(omega=1.3, g3=0.0, g4=0.0, V1=1.0, V2=0.0, zeta=0.0, gamma=0.2,
                mu1=1.0, mu2=0.0, n_basis=12, n_keep=6, K=1)
    m = om.single_mode(mode)
    np.testing.assert_allclose(m.E, 1.3 * (np.arange(6) + 0.5), atol=1e-12)
    Q1 = np.diag(np.sqrt(np.arange(1, 6) / 2.0), 1)
    np.testing.assert_allclose(np.abs(m.Q1), np.abs(Q1 + Q1.T), atol=1e-12)
    # q^2 is built before truncation: <5|q^2|5> = 5.5, not (Q1 Q1)[5,5] = 2.5
    assert m.Q2[5, 5] == pytest.approx(5.5, abs=1e-12)


def test_anharmonic_levels_perturbation_theory():
    # E_n = (n+1/2) + (g4/32)(2n^2+2n+1) - (g3^2/288)(30n^2+30n+11) + O(g^3)
    g3, g4 = -0.02, 0.01
    mode = dict(omega=1.0, g3=g3, g4=g4, V1=1.0, V2=0.0, zeta=0.0, gamma=0.2,
                mu1=1.0, mu2=0.0, n_basis=40, n_keep=6, K=1)
    m = om.single_mode(mode)
    n = np.arange(6)
    pt = (n + 0.5) + g4 / 32 * (2 * n * n + 2 * n + 1) - g3 * g3 / 288 * (30 * n * n + 30 * n + 11)
    assert np.max(np.abs(m.E - pt)) < 1e-4


def test_operators_symmetric_and_counter_term():
    p, _ = w.cfg3(depth=1)
    m = om.build(p)
    for A in [m.H, m.mu] + m.V:
        np.testing.assert_allclose(A, A.T, atol=1e-13)
    np.testing.assert_allclose(m.mu_plus + m.mu_minus + np.where(
        om.quanta(m.dims)[:, None] == om.quanta(m.dims)[None, :], m.mu, 0.0), m.mu, atol=0)
    # harmonic mode with V = q: H_S' = H_A + Lambda q^2 exactly in the kept basis
    mode = dict(omega=1.0, g3=0.0, g4=0.0, V1=1.0, V2=0.0, zeta=0.1, gamma=0.2,
                mu1=1.0, mu2=0.0, n_basis=12, n_keep=5, K=1)
    mm = om.build({"modes": [mode], "couplings": [], "beta": 10.0, "depth": 1,
                   "decomp": "pade", "dt": 0.1})
    k = np.arange(5)
    q2 = np.diag(k + 0.5) + np.diag(np.sqrt((k[:-2] + 1) * (k[:-2] + 2)) / 2, 2)
    q2 = q2 + np.triu(q2, 1).T
    np.testing.assert_allclose(mm.H, np.diag(k + 0.5) + 0.01 * q2, atol=1e-13)


def _harmonic_mode(omega, keep, nb=None, **kw):
    mode = dict(omega=omega, g3=0.0, g4=0.0, V1=1.0, V2=0.0, zeta=0.0, gamma=0.2,
                mu1=0.0, mu2=0.0, n_basis=nb or keep, n_keep=keep, K=1)
    mode.update(kw)
    return mode


def _coupled(modes, couplings):
    return om.build({"modes": modes, "couplings": couplings, "beta": 10.0, "depth": 0,
                     "decomp": "pade", "dt": 0.1})


def _cpl(s, t, g_st=0.0, g_s2t=0.0, g_st2=0.0, mu_st=0.0):
    return dict(s=s, t=t, g_st=g_st, g_s2t=g_s2t, g_st2=g_st2, mu_st=mu_st)


def test_bilinear_coupling_gives_normal_mode_ladder():
    # Two harmonic modes H = sum_s w_s (p_s^2 + q_s^2)/2 + g q_1 q_2 (Eq.
    # Potential ss' with only the bilinear term): with x_s = q_s / sqrt(w_s)
    # this is a pair of oscillators of unit mass with the potential matrix
    # [[w1^2, g sqrt(w1 w2)], [g sqrt(w1 w2), w2^2]], so the exact spectrum is
    # sum_k Omega_k (n_k + 1/2) with Omega_k^2 its eigenvalues.  A factor of 2
    # in the coupling, or the coupling on the wrong operator, moves the levels.
    w1, w2, g = 1.0, 0.45, 0.05
    m = _coupled([_harmonic_mode(w1, 24), _harmonic_mode(w2, 24)], [_cpl(0, 1, g_st=g)])
    Om = np.sqrt(np.linalg.eigvalsh(np.array([[w1 * w1, g * np.sqrt(w1 * w2)],
                                              [g * np.sqrt(w1 * w2), w2 * w2]])))
    ladder = np.sort([Om[0] * (a + 0.5) + Om[1] * (b + 0.5) for a in range(8) for b in range(8)])[:8]
    E = np.linalg.eigvalsh(m.H)[:8]
    np.testing.assert_allclose(E, ladder, atol=1e-9)
    # sanity: the uncoupled ladder differs at this accuracy
    assert np.max(np.abs(np.sort([w1 * (a + .5) + w2 * (b + .5) for a in range(8) for b in range(8)])[:8]
                         - ladder)) > 1e-4


def test_mode_coupling_and_dipole_matrix_elements_by_hand():
    # Harmonic modes, so the kept basis is the number basis and
    # <1|q|0> = 1/sqrt(2), <0|q^2|2> = 1/sqrt(2).  Index of |n_0, n_1> with
    # mode 0 slowest: n_0 * d_1 + n_1.
    d1 = 4
    idx = lambda n0, n1: n0 * d1 + n1  # noqa: E731
    for key, pair, expect in [
        ("g_s2t", ((0, 1), (2, 0)), 1 / 12),   # (g_s2t/6) <0|q^2|2> <1|q|0>
        ("g_st2", ((1, 0), (0, 2)), 1 / 12),   # (g_st2/6) <1|q|0> <0|q^2|2>
        ("g_st", ((1, 1), (0, 0)), 1 / 2),     # g_st <1|q|0> <1|q|0>
    ]:
        g = 0.07
        m = _coupled([_harmonic_mode(1.0, 4, nb=12), _harmonic_mode(0.45, d1, nb=12)], [_cpl(0, 1, **{key: g})])
        (a0, a1), (b0, b1) = pair
        assert m.H[idx(a0, a1), idx(b0, b1)] == pytest.approx(g * expect, rel=1e-12), key
        # the mirrored placement (the term on the other mode) is absent
        if key != "g_st":
            assert abs(m.H[idx(a1, a0), idx(b1, b0)]) < 1e-14, key
    # dipole: (mu2/2) <0|q^2|2> = mu2 / (2 sqrt 2); mu_st <1|q|0>^2 = mu_st / 2
    mu2, mu_st = 0.3, 0.04
    m = _coupled([_harmonic_mode(1.0, 4, nb=12, mu2=mu2), _harmonic_mode(0.45, d1, nb=12)],
                 [_cpl(0, 1, mu_st=mu_st)])
    assert m.mu[idx(0, 0), idx(2, 0)] == pytest.approx(mu2 / (2 * np.sqrt(2)), rel=1e-12)
    assert m.mu[idx(0, 0), idx(0, 2)] == pytest.approx(0.0, abs=1e-15)
    assert m.mu[idx(1, 1), idx(0, 0)] == pytest.approx(mu_st / 2, rel=1e-12)
    assert m.mu[idx(1, 0), idx(0, 0)] == pytest.approx(0.0, abs=1e-15)   # mu1 = 0


def test_three_mode_index_order_and_quanta_from_digits():
    # (4, 4, 5) product basis, mode 0 slowest: a = 20 n_0 + 5 n_1 + n_2.
    dims = (4, 4, 5)
    modes = [_harmonic_mode(1.0, 4, nb=12, mu1=1.0), _harmonic_mode(1.03, 4, nb=12, mu1=1.0),
             _harmonic_mode(0.44, 5, nb=12, mu1=1.0, mu2=0.2)]
    g = 0.05
    m = _coupled(modes, [_cpl(1, 2, g_s2t=g), _cpl(0, 2, g_st=g)])
    digits = [(a // 20, (a // 5) % 4, a % 5) for a in range(80)]
    a, b = digits.index((0, 0, 1)), digits.index((0, 2, 0))
    assert (a, b) == (1, 10)
    assert m.H[a, b] == pytest.approx(g / 12, rel=1e-12)            # <0_1 1_2|(g/6) q_1^2 q_2|2_1 0_2>
    assert m.H[digits.index((1, 0, 1)), 0] == pytest.approx(g / 2, rel=1e-12)  # g <1|q|0>_0 <1|q|0>_2
    # diagonal: the harmonic levels of the three modes
    for a, (n0, n1, n2) in enumerate(digits):
        assert m.H[a, a] == pytest.approx(1.0 * (n0 + .5) + 1.03 * (n1 + .5) + 0.44 * (n2 + .5), abs=1e-12)
    # V_s acts on its own digit only
    for s in range(3):
        nz = np.argwhere(np.abs(m.V[s]) > 0)
        for a, b in nz:
            da, db = digits[a], digits[b]
            assert all(da[t] == db[t] for t in range(3) if t != s)
    # mu_plus keeps exactly the elements that raise the number of quanta
    N = np.array([sum(dg) for dg in digits])
    np.testing.assert_array_equal(om.quanta(dims), N)
    for a in range(80):
        for b in range(80):
            want = m.mu[a, b] if N[a] > N[b] else 0.0
            assert m.mu_plus[a, b] == want
    np.testing.assert_array_equal(m.mu_minus, m.mu_plus.T)
    assert m.mu_plus[digits.index((0, 0, 1)), 0] == pytest.approx(1 / np.sqrt(2), rel=1e-12)
    assert m.mu_plus[0, digits.index((0, 0, 1))] == 0.0


# ------------------------------------------------------ RHS and RK4 ---------

def _small_model():
    p, _ = w.cfg1()
    return om.build(p)


def _brownian_model(depth=3):
    p, _ = w.cfg1()
    p["modes"][0]["omega_b"] = 1.5
    p["modes"][0]["gamma"] = 0.4
    p["depth"] = depth
    p["decomp"] = "pade"
    return om.build(p)


@pytest.mark.parametrize("bath_kind", ["drude", "brownian"])
def test_rhs_matches_assembled_liouvillian(bath_kind):
    m = _small_model() if bath_kind == "drude" else _brownian_model()
    x = w.random_hierarchy(1, len(m.hier), m.d, seed=3)[0]
    Lm = heom.liouvillian_matrix(m)
    np.testing.assert_allclose(Lm @ x.reshape(-1), heom.rhs(m, x).reshape(-1), atol=1e-13)


@pytest.mark.parametrize("cfg", ["cfg1", "cfg2small", "brownian"])
def test_adjoint_dot_product(cfg):
    if cfg == "cfg1":
        m = _small_model()
    elif cfg == "brownian":
        m = _brownian_model()
    else:
        p, _ = w.cfg2()
        p["depth"] = 2
        m = om.build(p)
    x = w.random_hierarchy(1, len(m.hier), m.d, seed=5)[0]
    y = w.random_hierarchy(1, len(m.hier), m.d, seed=6)[0]
    lhs = np.sum(y * heom.rhs(m, x))
    rhs_ = np.sum(heom.rhs(m, y, adjoint=True) * x)
    assert abs(lhs - rhs_) < 1e-12 * abs(lhs)


def test_rk4_is_fourth_order_taylor_polynomial():
    # For a linear, time-independent L one classic RK4 step is exactly
    # sum_{k<=4} (hL)^k / k! applied to the state.
    m = _small_model()
    x = w.random_hierarchy(1, len(m.hier), m.d, seed=7)[0].reshape(-1)
    Lm = heom.liouvillian_matrix(m)
    h = 0.3
    acc, term = x.copy(), x.copy()
    for k in range(1, 5):
        term = h * (Lm @ term) / k
        acc = acc + term
    got = heom.rk4_step(m, x.reshape(len(m.hier), m.d, m.d), h=h).reshape(-1)
    np.testing.assert_allclose(got, acc, atol=1e-12)


def test_rk4_against_matrix_exponential():
    m = _small_model()
    rho = heom.ground_state_hierarchy(m)
    t = 2.0
    exact = sla.expm(heom.liouvillian_matrix(m).toarray() * t) @ rho.reshape(-1)
    errs = []
    for h in (0.1, 0.05):
        steps = int(round(t / h))
        y = rho
        for _ in range(steps):
            y = heom.rk4_step(m, y, h=h)
        errs.append(np.max(np.abs(y.reshape(-1) - exact)))
    assert errs[1] < 1e-8
    assert errs[0] / errs[1] == pytest.approx(16.0, rel=0.15)


def test_liouvillian_spectrum_stable_with_single_stationary_state():
    m = _small_model()
    ev = np.linalg.eigvals(heom.liouvillian_matrix(m).toarray())
    assert np.max(ev.real) < 1e-12
    assert int(np.sum(np.abs(ev) < 1e-9)) == 1
    st = heom.stationary_state(m)
    assert np.trace(st[0]).real == pytest.approx(1.0, abs=1e-13)
    assert np.max(np.abs(heom.rhs(m, st))) < 1e-13


# --------------------------------------------------------- invariants -------

def test_trace_and_hermiticity_preserved():
    m = _small_model()
    rho = heom.ground_state_hierarchy(m)
    rho = heom.propagate(m, rho, 200)
    assert np.trace(rho[0]).real == pytest.approx(1.0, abs=1e-13)
    assert abs(np.trace(rho[0]).imag) < 1e-14
    herm = np.max(np.abs(rho - np.conj(np.swapaxes(rho, -1, -2))))
    assert herm < 1e-14
    X = heom.commutator(m.mu, rho)
    assert abs(np.trace(X[0])) < 1e-14
    X = heom.propagate(m, X, 50)
    assert abs(np.trace(X[0])) < 1e-14


def test_equilibrate_reaches_stationary_state_from_it():
    # Starting at the stationary solution the residual check passes at once.
    m = _small_model()
    st = heom.stationary_state(m)
    rho, steps, res = heom.equilibrate(m, 1e-12, 10, 0, 100, rho0=st)
    assert steps == 10 and res < 1e-12
    np.testing.assert_allclose(rho, st, atol=1e-12)


def test_weak_coupling_equilibrium_is_gibbs():
    # zeta -> 0 with Pade K=4: rho_0 of the stationary state -> exp(-beta H_S)/Z
    # (Gibbs state of the bare system Hamiltonian; the counter-term makes the
    # O(zeta) shift vanish at leading order in the populations).
    mode = dict(omega=1.0, g3=-0.2, g4=0.02, V1=1.0, V2=0.0, zeta=0.002, gamma=0.5,
                mu1=1.0, mu2=0.0, n_basis=12, n_keep=4, K=4)
    p = {"modes": [mode], "couplings": [], "beta": 2.0, "depth": 2,
         "decomp": "pade", "dt": 0.05}
    m = om.build(p)
    st = heom.stationary_state(m)
    E = om.single_mode(mode).E
    g = np.exp(-2.0 * (E - E[0]))
    g /= g.sum()
    pops = np.real(np.diag(st[0]))
    assert np.max(np.abs(pops - g)) < 5e-3
    assert abs(pops[1] - g[1]) / g[1] < 0.03


# ------------------------------------------------------ closed forms --------

def _unitary_response(H, D1, D2, D3, mu, rho0, t1, t2, t3):
    E, U = np.linalg.eigh(H)

    def G(X, t):
        P = U @ np.diag(np.exp(-1j * E * t)) @ U.T
        return P @ X @ P.conj().T

    def cx(D, X):
        return D @ X - X @ D

    X = G(cx(D1, rho0), t1)
    Y = G(cx(D2, X), t2)
    Z = G(cx(D3, Y), t3)
    return (1j) ** 3 * np.trace(mu @ Z)


def test_no_bath_response_is_sum_over_states():
    # zeta = 0: no ADO is ever populated and rho_0 evolves unitarily; R_P is
    # the textbook closed form built from the eigenstates of H_S'.
    p, _ = w.cfg2()
    for mode in p["modes"]:
        mode["zeta"] = 0.0
        mode["n_keep"] = 3
    p["depth"] = 1
    p["dt"] = 0.05
    m = om.build(p)
    rho = heom.ground_state_hierarchy(m)
    grid = {"n1": 4, "n3": 5, "steps_per_sample": 10, "t2_steps": [0, 7]}
    R = heom.response_2d(m, rho, grid, pathways=("I", "II", "full"))
    for i, t2s in enumerate(grid["t2_steps"]):
        for pidx, pw in enumerate(("I", "II", "full")):
            D1, D2, D3 = heom.pathway_dipoles(m, pw)
            for j in range(4):
                for k in range(5):
                    ex = _unitary_response(m.H, D1, D2, D3, m.mu, rho[0],
                                           0.5 * j, 0.05 * t2s, 0.5 * k)
                    assert abs(R[i, pidx, j, k] - ex) < 1e-6 * (1 + abs(ex))


@pytest.mark.parametrize("bath_kind", ["drude", "brownian"])
def test_pure_dephasing_cumulant(bath_kind):
    # Diagonal H and V: rho_ab(t) = rho_ab(0) exp(-i w_ab t)
    #   * exp[-(v_a - v_b)(v_a g(t) - v_b conj(g(t)))],
    # g(t) = sum_j c_j (exp(-nu_j t) + nu_j t - 1)/nu_j^2 (second-order
    # cumulant, exact for a Gaussian bath); the hierarchy converges to it.
    # The Brownian bath has a complex-conjugate pair of rates, whose bra-side
    # couplings carry the partner's conjugated coefficient.
    eps = np.array([0.0, 1.0, 1.9])
    v = np.array([0.0, 0.6, 1.3])
    if bath_kind == "drude":
        nu, c = bath.drude_terms(0.1, 0.5, 2.0, 3, "pade")
    else:
        nu, c = bath.brownian_terms(0.1, 0.5, 1.2, 2.0, 2, "pade")
    errs = []
    for L in (4, 8):
        m = om.make_model(np.diag(eps), [np.diag(v)], np.zeros((3, 3)),
                          [0] * len(nu), nu, c, L, dt=0.01)
        rho = np.zeros((len(m.hier), 3, 3), dtype=complex)
        rho[0] = 1.0 / 3.0
        t = 3.0
        rho = heom.propagate(m, rho, 300)
        g = np.sum(c * (np.exp(-nu * t) + nu * t - 1) / nu ** 2)
        ex = np.empty((3, 3), dtype=complex)
        for a in range(3):
            for b in range(3):
                ex[a, b] = (1 / 3) * np.exp(-1j * (eps[a] - eps[b]) * t) * np.exp(
                    -(v[a] - v[b]) * (v[a] * g - v[b] * np.conj(g)))
        errs.append(np.max(np.abs(rho[0] - ex)))
    assert errs[1] < 1e-7
    assert errs[1] < errs[0]


def _chi_brownian(t, omega0, gamma, zeta, V1):
    # chi(s) = (s + gamma)/((s^2 + w0^2)(s + gamma) + V1^2 zeta gamma s)
    poles = np.roots([1.0, gamma, omega0 ** 2 + V1 * V1 * zeta * gamma, omega0 ** 2 * gamma])
    tot = 0.0
    for i, s in enumerate(poles):
        den = np.prod([s - q for k, q in enumerate(poles) if k != i])
        tot = tot + (s + gamma) / den * np.exp(s * t)
    return np.real(tot)


def test_brownian_closed_form_worked_values():
    assert _chi_brownian(1.0, 1, 0.2, 0.1, 1.0) == pytest.approx(0.8386119, abs=1e-7)
    assert _chi_brownian(5.0, 1, 0.2, 0.1, 1.0) == pytest.approx(-0.9269534, abs=1e-7)
    assert _chi_brownian(20.0, 1, 0.2, 0.1, 1.0) == pytest.approx(0.9288736, abs=1e-7)


@pytest.mark.parametrize("beta,K,decomp", [(10.0, 2, "pade"), (10.0, 2, "matsubara"),
                                           (3.0, 1, "pade")])
def test_harmonic_linear_response_is_brownian_oscillator(beta, K, decomp):
    # Harmonic mode, LL coupling, linear dipole: R1(t) = mu1^2 chi(t), the
    # classical Brownian-oscillator response, independent of beta and K.
    p = w.harmonic_pin(depth=4, K=K, dt=0.02, n_keep=6, beta=beta, decomp=decomp)
    m = om.build(p)
    R1 = heom.linear_response(m, heom.ground_state_hierarchy(m), 16, 50)
    ex = np.array([_chi_brownian(t, 1.0, 0.2, 0.1, 1.0) for t in np.arange(16.0)])
    assert np.max(np.abs(R1.imag)) < 1e-12
    assert np.max(np.abs(R1.real - ex)) < 2e-5


def _chi_brownian_bath(t, omega0, gamma, zeta, V1, wb):
    # friction kernel of the Brownian density: xi(s) = zeta gamma (s + gamma)/(s^2 + gamma s + wb^2);
    # chi(s) = 1/(s^2 + w0^2 + V1^2 s xi(s)), inverted over the four poles
    num = np.array([1.0, gamma, wb * wb])
    den = np.polyadd(np.polymul([1.0, 0.0, omega0 ** 2], num),
                     V1 * V1 * zeta * gamma * np.array([1.0, gamma, 0.0]))
    poles = np.roots(den)
    tot = 0.0
    for i, s in enumerate(poles):
        dd = np.prod([s - q for k, q in enumerate(poles) if k != i])
        tot = tot + np.polyval(num, s) / dd * np.exp(s * t)
    return np.real(tot)


def test_brownian_bath_closed_form_against_langevin_ode():
    # the same chi(t) as the impulse response of the Langevin equation
    # x'' + w0^2 x + V1^2 int xi(t - u) x'(u) du = 0, x(0) = 0, x'(0) = 1, with
    # the kernel realised by an auxiliary damped oscillator g'' + gamma g' +
    # wb^2 g = x', friction force zeta gamma (g' + gamma g)
    w0, gamma, zeta, V1, wb = 1.0, 0.5, 0.1, 1.0, 2.0

    def f(t, u):
        x, y, g, h = u
        return [y, -w0 ** 2 * x - V1 ** 2 * zeta * gamma * (h + gamma * g), h, y - gamma * h - wb ** 2 * g]

    ts = np.arange(16.0)
    sol = si.solve_ivp(f, (0, 15.0), [0.0, 1.0, 0.0, 0.0], t_eval=ts, rtol=1e-12, atol=1e-14,
                       method="DOP853")
    ex = np.array([_chi_brownian_bath(t, w0, gamma, zeta, V1, wb) for t in ts])
    assert np.max(np.abs(sol.y[0] - ex)) < 1e-10


@pytest.mark.parametrize("beta,K,decomp", [(10.0, 2, "pade"), (10.0, 2, "matsubara"),
                                           (3.0, 1, "pade")])
def test_harmonic_linear_response_brownian_bath(beta, K, decomp):
    # Harmonic mode coupled to an underdamped Brownian bath (complex rates):
    # R1(t) = chi(t) of the Langevin equation with the Brownian friction
    # kernel, independent of beta and K; R1 stays real.
    p = w.harmonic_pin(depth=4, K=K, dt=0.02, n_keep=6, beta=beta, decomp=decomp,
                       gamma=0.5, omega_b=2.0)
    m = om.build(p)
    assert np.any(np.abs(np.imag(m.nu)) > 0)
    R1 = heom.linear_response(m, heom.ground_state_hierarchy(m), 16, 50)
    ex = np.array([_chi_brownian_bath(t, 1.0, 0.5, 0.1, 1.0, 2.0) for t in np.arange(16.0)])
    assert np.max(np.abs(R1.imag)) < 1e-12
    assert np.max(np.abs(R1.real - ex)) < 1e-5


def test_harmonic_third_order_response_vanishes():
    p = w.harmonic_pin(depth=3, K=2, dt=0.05, n_keep=6)
    m = om.build(p)
    grid = {"n1": 4, "n3": 4, "steps_per_sample": 20, "t2_steps": [0]}
    R = heom.response_2d(m, heom.ground_state_hierarchy(m), grid, pathways=("I", "II", "full"))
    R1 = heom.linear_response(m, heom.ground_state_hierarchy(m), 4, 20)
    assert np.max(np.abs(R)) < 1e-6 * np.max(np.abs(R1))


def test_full_response_is_real_and_sum_of_27_pathways():
    p, _ = w.cfg1()
    p["dt"] = 0.05
    m = om.build(p)
    rho = heom.propagate(m, heom.ground_state_hierarchy(m), 100)
    grid = {"n1": 3, "n3": 3, "steps_per_sample": 10, "t2_steps": [4]}
    R = heom.response_2d(m, rho, grid, pathways=("full",))[0, 0]
    assert np.max(np.abs(R.imag)) < 1e-12 * np.max(np.abs(R))
    mu0 = m.mu - m.mu_plus - m.mu_minus
    parts = (m.mu_plus, m.mu_minus, mu0)
    triples = [(a, b, c) for a in parts for b in parts for c in parts]
    R27 = heom.response_2d(m, rho, grid, pathways=triples)[0]
    np.testing.assert_allclose(R27.sum(0), R, atol=1e-13 * np.max(np.abs(R)))


def test_response_invariant_under_eigenvector_signs():
    p, _ = w.cfg2()
    p["depth"] = 1
    for mode in p["modes"]:
        mode["n_keep"] = 3
    p["dt"] = 0.1
    modes = [om.single_mode(mm) for mm in p["modes"]]
    m1 = om.build_from_modes(p, modes)
    m2 = om.build_from_modes(p, [om.flip_sign(modes[0], 1), om.flip_sign(modes[1], 2)])
    grid = {"n1": 3, "n3": 3, "steps_per_sample": 5, "t2_steps": [3]}
    R1 = heom.response_2d(m1, heom.ground_state_hierarchy(m1), grid)
    R2 = heom.response_2d(m2, heom.ground_state_hierarchy(m2), grid)
    assert not np.allclose(m1.mu, m2.mu)
    np.testing.assert_allclose(R1, R2, atol=1e-14)


def test_depth_convergence():
    p, _ = w.cfg1()
    p["dt"] = 0.05
    grid = {"n1": 6, "n3": 6, "steps_per_sample": 20, "t2_steps": [0]}
    Rs = []
    for L in (1, 2, 3, 4):
        p["depth"] = L
        m = om.build(p)
        Rs.append(heom.response_2d(m, heom.ground_state_hierarchy(m), grid))
    d = [np.max(np.abs(Rs[i + 1] - Rs[i])) for i in range(3)]
    assert d[0] > d[1] > d[2]


# ------------------------------------------------------------ spectra -------

def test_spectrum_geometric_series():
    # R[j, k] = exp(-i a t1_j - i b t3_k): each trapezoid-weighted sum is a
    # finite geometric series, sum_{j<n} r^j - 1/2 = (1 - r^n)/(1 - r) - 1/2.
    n1, n3, dts = 8, 6, 0.7
    a, b = 1.1, -0.6
    t1 = dts * np.arange(n1)
    t3 = dts * np.arange(n3)
    R = np.exp(-1j * a * t1)[:, None] * np.exp(-1j * b * t3)[None, :]
    S = heom.pathway_spectrum(R, dts)
    w1 = heom.frequency_grid(n1, dts)
    w3 = heom.frequency_grid(n3, dts)

    def geo(W, x, n):
        r = np.exp(1j * (W - x) * dts)
        return (1 - r ** n) / (1 - r) - 0.5

    ex = np.imag(dts * dts * geo(w3[:, None], b, n3) * geo(w1[None, :], a, n1))
    np.testing.assert_allclose(S, ex, atol=1e-12)
    assert S.shape == (2 * n3, 2 * n1)


def test_linear_spectrum_geometric_series():
    # R1(t_k) = exp(-(c + i a) t_k): the trapezoid-weighted sum is
    # dt ((1 - r^n)/(1 - r) - 1/2) with r = exp((i (W - a) - c) dt)
    n, dts, a, c = 11, 0.6, 0.9, 0.05
    t = dts * np.arange(n)
    R1 = np.exp(-(c + 1j * a) * t)
    W = heom.frequency_grid(n, dts)
    r = np.exp((1j * (W - a) - c) * dts)
    ex = dts * ((1 - r ** n) / (1 - r) - 0.5)
    got = heom.linear_spectrum(R1, dts)
    np.testing.assert_allclose(got, ex, atol=1e-12)
    assert got.shape == (2 * n,)


@pytest.mark.slow
def test_correlation_spectrum_sign_convention():
    # Strongly anharmonic oscillator: the 0->1->0 diagonal peak (near w10, w10)
    # is positive and the 0->1->2 peak (near w21 on the W3 axis) negative.
    mode = dict(omega=1.0, g3=-0.6, g4=0.0, V1=0.5, V2=0.0, zeta=0.3, gamma=0.5,
                mu1=1.0, mu2=0.0, n_basis=12, n_keep=4, K=2)
    p = {"modes": [mode], "couplings": [], "beta": 10.0, "depth": 2,
         "decomp": "pade", "dt": 0.05}
    m = om.build(p)
    grid = {"n1": 48, "n3": 48, "steps_per_sample": 20, "t2_steps": [0]}
    R = heom.response_2d(m, heom.ground_state_hierarchy(m), grid)
    S = heom.correlation_spectrum(R[0, 0], R[0, 1], 1.0)
    wg = heom.frequency_grid(48, 1.0)
    E = np.linalg.eigvalsh(m.H)
    w10, w21 = E[1] - E[0], E[2] - E[1]
    assert w10 - w21 > 0.15
    imax = np.unravel_index(np.argmax(S), S.shape)
    imin = np.unravel_index(np.argmin(S), S.shape)
    step = wg[1] - wg[0]
    assert S[imax] > 0 and S[imin] < 0
    assert abs(wg[imax[0]] - w10) <= step and abs(wg[imax[1]] - w10) <= step
    assert abs(wg[imin[0]] - w21) <= 1.5 * step and abs(wg[imin[1]] - w10) <= step

"""Bath correlations as sums of exponentials (oracle; test infrastructure).

Drude baths follow the paper directly; underdamped Brownian baths (the HEOM
admits other spectral densities, Sec. II.B) use the same residue construction
and are defined in brownian_terms below.

Paper, Sec. II.B: for the Drude spectral density the bath correlation is a sum
of decaying exponentials.  The fluctuation part needs the expansion of
coth(beta*omega/2); the paper uses the [K-1/K] Pade approximant of that
function (Eqs. Pade1, Pade2) and the Matsubara expansion appears in Eq. L2.

Both decompositions are written here in the common form

    coth(x/2) ~= 2/x + sum_k 4 eta_k x / (x^2 + xi_k^2),

with Matsubara xi_k = 2 pi k, eta_k = 1, and the Pade poles/weights obtained
by constructing the Pade approximant of

    F(z) = (coth(x/2) - 2/x)/x,  z = x^2,

from its Taylor series (Bernoulli numbers) in exact rational arithmetic and
finding the roots of its denominator.  (This is a different route from the
tridiagonal-eigenvalue construction of Hu, Xu and Yan cited by the paper; the
Pade approximant is unique, so both give the same poles.)

The exponential terms of mode s are then (Eqs. Pade1, Pade2 with m_s = 1,
hbar = 1 and the counter-term constant Lambda = zeta*gamma/2):

    nu_0 = gamma,
    c_0  = (zeta*gamma/beta) (1 + sum_k 2 eta_k gamma^2/(gamma^2 - nu_k^2))
           - i zeta gamma^2 / 2,
    nu_k = xi_k / beta,
    c_k  = -(zeta gamma^2/beta) 2 eta_k nu_k / (gamma^2 - nu_k^2),   k >= 1,

so that Theta_k X = Re(c_k) V^x X + i Im(c_k) V^o X = c_k V X - conj(c_k) X V.
"""

from __future__ import annotations

from fractions import Fraction
from math import factorial, pi

import mpmath
import numpy as np


def bernoulli_numbers(n_max: int):
    """Exact Bernoulli numbers B_0..B_n_max (B_1 = -1/2) by the standard recurrence.

    sum_{k=0}^{m} C(m+1, k) B_k = 0 for m >= 1, B_0 = 1.
    """
    from math import comb
    B = [Fraction(1)]
    for m in range(1, n_max + 1):
        s = sum(Fraction(comb(m + 1, k)) * B[k] for k in range(m))
        B.append(-s / (m + 1))
    return B


def coth_taylor_F(n_coef: int):
    """Taylor coefficients f_0..f_{n_coef-1} of F(z) = (coth(x/2) - 2/x)/x in z = x^2.

    From x/2 coth(x/2) = sum_n B_{2n} x^{2n}/(2n)!:  f_m = 2 B_{2m+2}/(2m+2)!.
    """
    B = bernoulli_numbers(2 * n_coef + 2)
    return [2 * B[2 * m + 2] / factorial(2 * m + 2) for m in range(n_coef)]


def _solve_fraction(A, b):
    """Gaussian elimination in exact rationals."""
    n = len(b)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def pade_poles(K: int, high_precision: bool = False):
    """[K-1/K] Pade decomposition of coth: returns (xi[K], eta[K]) ascending in xi.

    high_precision=True returns lists of mpmath numbers (60 digits) instead of
    float arrays.
    """
    if K == 0:
        return np.zeros(0), np.zeros(0)
    f = coth_taylor_F(2 * K)
    # denominator Q(z) = 1 + q_1 z + ... + q_K z^K; numerator P of degree K-1;
    # Q F - P = O(z^{2K})  ->  sum_{i=0}^{K} q_i f_{m-i} = 0 for m = K..2K-1.
    A = [[f[m - i] for i in range(1, K + 1)] for m in range(K, 2 * K)]
    b = [-f[m] for m in range(K, 2 * K)]
    q = [Fraction(1)] + _solve_fraction(A, b)
    p = [sum(q[i] * f[m - i] for i in range(m + 1)) for m in range(K)]
    mpmath.mp.dps = 60
    qc = [mpmath.mpf(x.numerator) / x.denominator for x in q]
    pc = [mpmath.mpf(x.numerator) / x.denominator for x in p]
    roots = mpmath.polyroots(list(reversed(qc)), maxsteps=400, extraprec=400)
    xi, eta = [], []
    for z in roots:
        z = mpmath.re(z)
        Pz = sum(pc[m] * z ** m for m in range(K))
        dQ = sum(i * qc[i] * z ** (i - 1) for i in range(1, K + 1))
        xi.append(mpmath.sqrt(-z))
        eta.append(Pz / dQ / 4)
    order = sorted(range(K), key=lambda i: xi[i])
    if high_precision:
        return [xi[i] for i in order], [eta[i] for i in order]
    return (np.array([float(xi[i]) for i in order]),
            np.array([float(eta[i]) for i in order]))


def matsubara_poles(K: int):
    """Matsubara expansion: xi_k = 2 pi k, eta_k = 1 (k = 1..K)."""
    return np.array([2 * pi * k for k in range(1, K + 1)], dtype=float), np.ones(K)


def coth_approx(x, xi, eta):
    """The decomposed coth(x/2) = 2/x + sum_k 4 eta_k x/(x^2 + xi_k^2)."""
    x = np.asarray(x, dtype=float)
    return 2.0 / x + sum(4 * e * x / (x * x + s * s) for s, e in zip(xi, eta))


def drude_terms(zeta, gamma, beta, K, decomp="pade"):
    """Exponential terms (nu_j, c_j), j = 0..K, of one Drude bath.

    C(t) = sum_j c_j exp(-nu_j t) is the bath correlation whose HEOM couplings
    are Theta_j (Eqs. Pade1, Pade2).  Raises ValueError when gamma coincides
    with a pole (the coefficients of Eq. Pade1 are then singular).
    """
    xi, eta = (pade_poles(K) if decomp == "pade" else matsubara_poles(K))
    nu_k = xi / beta
    if np.any(np.abs(gamma ** 2 - nu_k ** 2) < 1e-12):
        raise ValueError("gamma coincides with a low-temperature pole")
    nus = [float(gamma)]
    s = 1.0 + sum(2 * e * gamma ** 2 / (gamma ** 2 - n ** 2) for e, n in zip(eta, nu_k))
    cs = [complex(zeta * gamma / beta * s, -zeta * gamma ** 2 / 2)]
    for e, n in zip(eta, nu_k):
        nus.append(float(n))
        cs.append(complex(-(zeta * gamma ** 2 / beta) * 2 * e * n / (gamma ** 2 - n ** 2), 0.0))
    return np.array(nus), np.array(cs)


def bra_coefficients(nu, c):
    """Coefficients of the conjugate correlation on the same exponentials.

    C(t)* = sum_j conj(c_j) exp(-conj(nu_j) t); written over the terms
    exp(-nu_j t) of C(t) it reads sum_j cb_j exp(-nu_j t) with
    cb_j = conj(c_j') where nu_j' = conj(nu_j).  The hierarchy's bra-side
    coupling uses cb_j (Theta_j X = c_j V X - cb_j X V); for real rates
    cb_j = conj(c_j) (Eqs. Pade1, Pade2), for a complex-conjugate pair of rates
    the two terms swap their conjugated coefficients.
    """
    nu = np.asarray(nu, dtype=complex)
    c = np.asarray(c, dtype=complex)
    cb = np.empty_like(c)
    for j in range(len(nu)):
        partner = [i for i in range(len(nu)) if abs(nu[i] - np.conj(nu[j])) <= 1e-12 * (1 + abs(nu[j]))]
        if len(partner) != 1:
            raise ValueError("exponential rates must be distinct and closed under conjugation")
        cb[j] = np.conj(c[partner[0]])
    return cb


def brownian_density(w, zeta, gamma, omega_b):
    """Underdamped Brownian spectral density in the normalisation of the Drude one:

    J(w) = (zeta/pi) gamma^2 omega_b^2 w / ((omega_b^2 - w^2)^2 + gamma^2 w^2),

    whose int_0^inf J(w)/w dw = zeta gamma / 2 equals the Drude Lambda (so the
    counter term is unchanged), and which becomes the Drude density of cutoff
    omega_b^2/gamma and the same Lambda when gamma >> omega_b.
    """
    return zeta / np.pi * gamma ** 2 * omega_b ** 2 * w / ((omega_b ** 2 - w * w) ** 2 + gamma ** 2 * w * w)


def brownian_terms(zeta, gamma, omega_b, beta, K, decomp="pade"):
    """Exponential terms (nu_j, c_j), j = 0..K+1, of one Brownian bath.

    C(t) = int_0^inf J(w) [coth(beta w/2) cos wt - i sin wt] dw with coth
    replaced by its decomposition (Pade [K-1/K] or K Matsubara terms) is, for
    t > 0, the sum of the residues of J(w) (1 + coth(beta w/2))/2 exp(-i w t)
    in the lower half plane (the same construction that gives Eqs. Pade1 and
    Pade2 for the Drude density):

      * the two poles w_p of J, rate nu_p = i w_p (a complex-conjugate pair
        gamma/2 +- i sqrt(omega_b^2 - gamma^2/4) when underdamped),
        c_p = -2 pi i Res_{w_p} J (1 + coth(beta w_p/2))/2;
      * the poles w = -i xi_k/beta of the coth decomposition, rate
        nu_k = xi_k/beta, c_k = -2 pi i (eta_k/beta) J(-i nu_k).

    Returns complex arrays (nu, c).  Raises ValueError at critical damping
    (omega_b = gamma/2, a double pole) or when a rate coincides with a pole.
    """
    xi, eta = (pade_poles(K) if decomp == "pade" else matsubara_poles(K))
    if abs(omega_b ** 2 - gamma ** 2 / 4) < 1e-12:
        raise ValueError("critically damped Brownian density (double pole)")
    A = zeta / np.pi * gamma ** 2 * omega_b ** 2
    # J(w) = A w / prod_i (w - w_i), w_i the roots of w^4 + (gamma^2 - 2 omega_b^2) w^2 + omega_b^4
    roots = np.roots([1.0, 0.0, gamma ** 2 - 2 * omega_b ** 2, 0.0, omega_b ** 4]).astype(complex)

    def coth_dec(x):
        return 2.0 / x + sum(4 * e * x / (x * x + s * s) for s, e in zip(xi, eta))

    nus, cs = [], []
    for p, wp in enumerate(roots):
        if wp.imag >= 0:
            continue
        res = A * wp / np.prod([wp - wi for i, wi in enumerate(roots) if i != p])
        nus.append(1j * wp)
        cs.append(-2j * np.pi * res * 0.5 * (1.0 + coth_dec(beta * wp)))
    if len(nus) != 2:
        raise ValueError("Brownian density needs omega_b > 0, gamma > 0")
    # the pair in the order (+Im, -Im); two real (overdamped) rates ascending
    order = sorted(range(2), key=lambda i: (-nus[i].imag, nus[i].real))
    nus = [nus[i] for i in order]
    cs = [cs[i] for i in order]
    for s, e in zip(xi, eta):
        nk = s / beta
        den = (omega_b ** 2 + nk * nk) ** 2 - gamma ** 2 * nk * nk
        if abs(den) < 1e-12 or any(abs(nk - n) < 1e-12 for n in nus):
            raise ValueError("a Brownian rate coincides with a low-temperature pole")
        Jk = A * (-1j * nk) / den
        nus.append(complex(nk))
        cs.append(-2j * np.pi * (e / beta) * Jk)
    return np.array(nus, dtype=complex), np.array(cs, dtype=complex)

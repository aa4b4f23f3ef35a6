// Host construction of the MAB-model operators, Drude-bath terms and HEOM
// hierarchy tables (FP64).  Everything here runs once per parameter set.
//
// Model (Sec. II.A): for each mode, H_A = omega (p^2 + q^2)/2 + g3 q^3/3! +
// g4 q^4/4! in a harmonic basis of n_basis levels (operator powers are formed
// with four extra levels so every kept matrix element is exact), diagonalised;
// the n_keep lowest eigenvectors U span the kept basis.  In that basis:
//   Q1 = U^T q U, Q2 = U^T q^2 U, v_s = V1 Q1 + V2 Q2/2          (Eq. h_int)
//   delta_s = Lambda U^T V(q)^2 U, Lambda = zeta gamma / 2       (Eqs. counter2, counterterm)
// Product basis (mode 0 slowest):
//   H_S' = sum_s (diag E_s + delta_s) + sum_{s<t} g_st Q1 Q1 + (g_s2t Q2 Q1 + g_st2 Q1 Q2)/6
//   mu   = sum_s mu1 Q1 + mu2 Q2/2 + sum_{s<t} mu_st Q1 Q1                (Eq. NLdip)
// Bath (Sec. II.B, Eqs. Pade1/Pade2 with m_s = 1, hbar = 1): exponential
// terms nu_0 = gamma, c_0 = (zeta gamma/beta)(1 + sum_k 2 eta_k gamma^2/
// (gamma^2 - nu_k^2)) - i zeta gamma^2/2; nu_k = xi_k/beta,
// c_k = -(zeta gamma^2/beta) 2 eta_k nu_k/(gamma^2 - nu_k^2), so that
// Theta_k X = c_k V X - conj(c_k) X V.
// Hierarchy (text after Eq. HEOM_DB): |n| <= depth, depth-then-lexicographic order.
#include "model.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>

namespace heom {

namespace {

using Mat = std::vector<double>;

Mat matmul(const Mat& A, const Mat& B, int n) {
  Mat C(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double a = A[i * n + k];
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
    }
  return C;
}

// U^T A U restricted: A is nb x nb (leading block of an n x n matrix), U is nb x keep.
Mat project(const Mat& A, int n, int nb, const Mat& U, int keep) {
  Mat T(static_cast<size_t>(nb) * keep, 0.0);  // A U
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < keep; ++j) {
      double s = 0.0;
      for (int k = 0; k < nb; ++k) s += A[i * n + k] * U[k * keep + j];
      T[i * keep + j] = s;
    }
  Mat R(static_cast<size_t>(keep) * keep, 0.0);
  for (int i = 0; i < keep; ++i)
    for (int j = 0; j < keep; ++j) {
      double s = 0.0;
      for (int k = 0; k < nb; ++k) s += U[k * keep + i] * T[k * keep + j];
      R[i * keep + j] = s;
    }
  return R;
}

struct ModeBasis {
  std::vector<double> E;
  Mat Q1, Q2, v, delta;
};

ModeBasis diagonalise_mode(const heom_mode& m) {
  const int nb = m.n_basis, keep = m.n_keep, n = nb + 4;
  Mat q(static_cast<size_t>(n) * n, 0.0), dm(static_cast<size_t>(n) * n, 0.0);
  for (int k = 1; k < n; ++k) {
    double s = std::sqrt(static_cast<double>(k));
    // a[k-1][k] = sqrt(k);  q = (a + a^T)/sqrt2,  a - a^T
    q[(k - 1) * n + k] += s / std::sqrt(2.0);
    q[k * n + (k - 1)] += s / std::sqrt(2.0);
    dm[(k - 1) * n + k] += s;
    dm[k * n + (k - 1)] -= s;
  }
  Mat p2 = matmul(dm, dm, n);
  for (auto& x : p2) x *= -0.5;
  Mat q2 = matmul(q, q, n), q3 = matmul(q2, q, n), q4 = matmul(q3, q, n);
  Mat Vq(q.size());
  for (size_t i = 0; i < q.size(); ++i) Vq[i] = m.V1 * q[i] + 0.5 * m.V2 * q2[i];
  Mat V2op = matmul(Vq, Vq, n);
  Mat HA(static_cast<size_t>(nb) * nb);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {
      size_t k = static_cast<size_t>(i) * n + j;
      HA[i * nb + j] = 0.5 * m.omega * (p2[k] + q2[k]) + m.g3 * q3[k] / 6.0 + m.g4 * q4[k] / 24.0;
    }
  std::vector<double> w, Vecs;
  jacobi_eigen(HA, nb, w, Vecs);
  Mat U(static_cast<size_t>(nb) * keep);
  for (int j = 0; j < keep; ++j) {
    int imax = 0;
    for (int i = 1; i < nb; ++i)
      if (std::fabs(Vecs[i * nb + j]) > std::fabs(Vecs[imax * nb + j])) imax = i;
    double sgn = Vecs[imax * nb + j] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < nb; ++i) U[i * keep + j] = sgn * Vecs[i * nb + j];
  }
  ModeBasis b;
  b.E.assign(w.begin(), w.begin() + keep);
  b.Q1 = project(q, n, nb, U, keep);
  b.Q2 = project(q2, n, nb, U, keep);
  b.v.resize(b.Q1.size());
  for (size_t i = 0; i < b.v.size(); ++i) b.v[i] = m.V1 * b.Q1[i] + 0.5 * m.V2 * b.Q2[i];
  const double Lam = 0.5 * m.zeta * m.gamma;
  b.delta = project(V2op, n, nb, U, keep);
  for (auto& x : b.delta) x *= Lam;
  return b;
}

// Adds coef * (A_s (x) B_t) (identity on other modes) to the d x d matrix M.
// t < 0 means a single-mode operator A_s.
void add_embedded(Mat& M, const HostModel& hm, double coef, int s, const Mat& A, int t,
                  const Mat* B) {
  const int d = hm.d;
  for (int a = 0; a < d; ++a)
    for (int c = 0; c < d; ++c) {
      bool same = true;
      int as = 0, cs = 0, at = 0, ct = 0;
      for (int r = 0; r < hm.n_modes; ++r) {
        int da = (a / hm.strides[r]) % hm.dims[r], dc = (c / hm.strides[r]) % hm.dims[r];
        if (r == s) {
          as = da;
          cs = dc;
        } else if (r == t) {
          at = da;
          ct = dc;
        } else if (da != dc) {
          same = false;
          break;
        }
      }
      if (!same) continue;
      double val = A[as * hm.dims[s] + cs];
      if (t >= 0) val *= (*B)[at * hm.dims[t] + ct];
      M[static_cast<size_t>(a) * d + c] += coef * val;
    }
}

std::string key_of(const std::vector<int>& n) {
  return std::string(n.begin(), n.end());
}

void enumerate_level(int M, int level, std::vector<int>& cur, int pos,
                     std::vector<std::vector<int>>& out) {
  if (pos == M - 1) {
    cur[pos] = level;
    out.push_back(cur);
    return;
  }
  for (int x = 0; x <= level; ++x) {
    cur[pos] = x;
    enumerate_level(M, level - x, cur, pos + 1, out);
  }
}

}  // namespace

void jacobi_eigen(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V) {
  V.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = cs * akp - sn * akq;
          A[k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = cs * apk - sn * aqk;
          A[q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = cs * vkp - sn * vkq;
          V[k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return A[x * n + x] < A[y * n + y]; });
  w.resize(n);
  std::vector<double> Vs(static_cast<size_t>(n) * n);
  for (int j = 0; j < n; ++j) {
    w[j] = A[order[j] * n + order[j]];
    for (int i = 0; i < n; ++i) Vs[i * n + j] = V[i * n + order[j]];
  }
  V.swap(Vs);
}

void pade_poles(int K, std::vector<double>& xi, std::vector<double>& eta) {
  xi.clear();
  eta.clear();
  if (K <= 0) return;
  // poles: positive eigenvalues lambda of the 2K x 2K tridiagonal matrix with
  // off-diagonal 1/sqrt((2m+1)(2m+3)), xi = 2/lambda
  auto tri_poles = [](int n, int shift) {
    std::vector<double> A(static_cast<size_t>(n) * n, 0.0), w, V;
    for (int m = 1; m < n; ++m) {
      double b = 1.0 / std::sqrt(static_cast<double>((2 * m + 1 + shift) * (2 * m + 3 + shift)));
      A[(m - 1) * n + m] = b;
      A[m * n + (m - 1)] = b;
    }
    jacobi_eigen(A, n, w, V);
    std::vector<double> out;
    for (double x : w)
      if (x > 1e-12) out.push_back(2.0 / x);
    std::sort(out.begin(), out.end());
    return out;
  };
  xi = tri_poles(2 * K, 0);
  std::vector<double> zt = K > 1 ? tri_poles(2 * K - 1, 2) : std::vector<double>{};
  for (int j = 0; j < K; ++j) {
    double num = 1.0, den = 1.0;
    for (double z : zt) num *= z * z - xi[j] * xi[j];
    for (int k = 0; k < K; ++k)
      if (k != j) den *= xi[k] * xi[k] - xi[j] * xi[j];
    eta.push_back(0.5 * K * (2 * K + 3) * num / den);
  }
}

HostModel build_host_model(const heom_params& p) {
  if (p.n_modes < 1 || p.n_modes > 4 || !p.modes)
    throw std::invalid_argument("n_modes must be 1..4");
  if (p.depth < 0 || p.depth > 40) throw std::invalid_argument("depth must be 0..40");
  if (!(p.dt > 0.0)) throw std::invalid_argument("dt must be positive");
  if (!(p.beta > 0.0)) throw std::invalid_argument("beta must be positive");
  if (p.decomp != HEOM_PADE && p.decomp != HEOM_MATSUBARA)
    throw std::invalid_argument("unknown decomposition");
  HostModel hm;
  hm.n_modes = p.n_modes;
  hm.dt = p.dt;
  hm.depth = p.depth;
  std::vector<ModeBasis> mb;
  for (int s = 0; s < p.n_modes; ++s) {
    const heom_mode& m = p.modes[s];
    if (m.n_basis < 1 || m.n_basis > 64 || m.n_keep < 1 || m.n_keep > m.n_basis)
      throw std::invalid_argument("mode " + std::to_string(s) + ": need 1 <= n_keep <= n_basis <= 64");
    if (m.K < 0 || m.K > 16) throw std::invalid_argument("K must be 0..16");
    if (!(m.gamma > 0.0) || m.zeta < 0.0) throw std::invalid_argument("need gamma > 0, zeta >= 0");
    if (m.omega_b < 0.0 || !std::isfinite(m.omega_b))
      throw std::invalid_argument("mode " + std::to_string(s) + ": omega_b must be >= 0 (0 = Drude bath)");
    mb.push_back(diagonalise_mode(m));
    hm.dims[s] = m.n_keep;
  }
  hm.d = 1;
  for (int s = p.n_modes - 1; s >= 0; --s) {
    hm.strides[s] = hm.d;
    hm.d *= hm.dims[s];
  }
  if (hm.d > 128) throw std::invalid_argument("product dimension above 128");
  const int d = hm.d;
  hm.H.assign(static_cast<size_t>(d) * d, 0.0);
  hm.mu.assign(static_cast<size_t>(d) * d, 0.0);
  for (int s = 0; s < p.n_modes; ++s) {
    const int ds = hm.dims[s];
    Mat h = mb[s].delta;
    for (int i = 0; i < ds; ++i) h[i * ds + i] += mb[s].E[i];
    add_embedded(hm.H, hm, 1.0, s, h, -1, nullptr);
    add_embedded(hm.mu, hm, p.modes[s].mu1, s, mb[s].Q1, -1, nullptr);
    add_embedded(hm.mu, hm, 0.5 * p.modes[s].mu2, s, mb[s].Q2, -1, nullptr);
    hm.v.push_back(mb[s].v);
  }
  for (int i = 0; i < p.n_couplings; ++i) {
    const heom_coupling& cp = p.couplings[i];
    if (cp.s < 0 || cp.t >= p.n_modes || cp.s >= cp.t)
      throw std::invalid_argument("coupling " + std::to_string(i) + ": need 0 <= s < t < n_modes");
    add_embedded(hm.H, hm, cp.g_st, cp.s, mb[cp.s].Q1, cp.t, &mb[cp.t].Q1);
    add_embedded(hm.H, hm, cp.g_s2t / 6.0, cp.s, mb[cp.s].Q2, cp.t, &mb[cp.t].Q1);
    add_embedded(hm.H, hm, cp.g_st2 / 6.0, cp.s, mb[cp.s].Q1, cp.t, &mb[cp.t].Q2);
    add_embedded(hm.mu, hm, cp.mu_st, cp.s, mb[cp.s].Q1, cp.t, &mb[cp.t].Q1);
  }
  // rotating-wave split by total kept quanta
  hm.quanta.assign(d, 0);
  for (int a = 0; a < d; ++a)
    for (int s = 0; s < p.n_modes; ++s) hm.quanta[a] += (a / hm.strides[s]) % hm.dims[s];
  hm.mu_plus.assign(static_cast<size_t>(d) * d, 0.0);
  hm.mu_minus.assign(static_cast<size_t>(d) * d, 0.0);
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      if (hm.quanta[a] > hm.quanta[b]) {
        hm.mu_plus[a * d + b] = hm.mu[a * d + b];
        hm.mu_minus[b * d + a] = hm.mu[a * d + b];
      }
  // bath terms
  for (int s = 0; s < p.n_modes; ++s) {
    const heom_mode& m = p.modes[s];
    std::vector<double> xi, eta;
    if (p.decomp == HEOM_PADE) {
      pade_poles(m.K, xi, eta);
    } else {
      for (int k = 1; k <= m.K; ++k) {
        xi.push_back(2.0 * M_PI * k);
        eta.push_back(1.0);
      }
    }
    const double g = m.gamma, z = m.zeta, beta = p.beta;
    auto add_term = [&](cplx nu, cplx c, cplx cb) {
      hm.term_mode.push_back(s);
      hm.nu.push_back(nu.real());
      hm.nu_im.push_back(nu.imag());
      hm.c.push_back(c);
      hm.cb.push_back(cb);
    };
    if (m.omega_b > 0.0) {
      // Brownian density J(w) = (zeta/pi) gamma^2 wb^2 w / ((wb^2 - w^2)^2 + gamma^2 w^2):
      // the two lower-half-plane poles w = +-r - i gamma/2 of J give the rates
      // nu = gamma/2 +- i r with r = sqrt(wb^2 - gamma^2/4) (imaginary when
      // overdamped) and c = +-(zeta gamma wb^2 / (4 r)) (coth(beta w/2) + 1), the
      // coth taken in its decomposed form; the decomposition's poles give real
      // rates xi_k/beta with c_k = -(2 zeta gamma^2 wb^2/beta) eta_k nu_k /
      // ((wb^2 + nu_k^2)^2 - gamma^2 nu_k^2).
      const double wb = m.omega_b;
      const cplx r = std::sqrt(cplx(wb * wb - 0.25 * g * g, 0.0));
      if (std::abs(r) < 1e-6) throw std::invalid_argument("mode " + std::to_string(s) + ": critically damped Brownian bath");
      auto coth_dec = [&](cplx x) {
        cplx v = 2.0 / x;
        for (size_t k = 0; k < xi.size(); ++k) v += 4.0 * eta[k] * x / (x * x + xi[k] * xi[k]);
        return v;
      };
      const cplx pref = z * g * wb * wb / (4.0 * r);
      const cplx w1 = r - cplx(0.0, 0.5 * g), w2 = -r - cplx(0.0, 0.5 * g);
      const cplx nu1 = cplx(0.0, 1.0) * w1, nu2 = cplx(0.0, 1.0) * w2;
      const cplx c1 = pref * (coth_dec(beta * w1) + 1.0);
      const cplx c2 = -pref * (coth_dec(beta * w2) + 1.0);
      // bra side: C(t)* puts conj(c1) on exp(-conj(nu1) t); for a conjugate
      // pair that is the partner's rate, for two real rates its own
      const bool pair = std::fabs(nu1.imag()) > 0.0;
      add_term(nu1, c1, pair ? std::conj(c2) : std::conj(c1));
      add_term(nu2, c2, pair ? std::conj(c1) : std::conj(c2));
      for (size_t k = 0; k < xi.size(); ++k) {
        const double nk = xi[k] / beta;
        const double den = (wb * wb + nk * nk) * (wb * wb + nk * nk) - g * g * nk * nk;
        if (std::fabs(den) < 1e-12 || std::abs(nu1 - nk) < 1e-12 || std::abs(nu2 - nk) < 1e-12)
          throw std::invalid_argument("mode " + std::to_string(s) + ": a Brownian rate coincides with a low-temperature pole");
        const double ck = -(2.0 * z * g * g * wb * wb / beta) * eta[k] * nk / den;
        add_term(nk, ck, ck);
      }
      continue;
    }
    double sum = 1.0;
    for (int k = 0; k < m.K; ++k) {
      double nk = xi[k] / beta;
      if (std::fabs(g * g - nk * nk) < 1e-12)
        throw std::invalid_argument("mode " + std::to_string(s) + ": gamma coincides with a low-temperature pole");
      sum += 2.0 * eta[k] * g * g / (g * g - nk * nk);
    }
    const cplx c0(z * g / beta * sum, -0.5 * z * g * g);
    add_term(g, c0, std::conj(c0));
    for (int k = 0; k < m.K; ++k) {
      double nk = xi[k] / beta;
      const cplx ck(-(z * g * g / beta) * 2.0 * eta[k] * nk / (g * g - nk * nk), 0.0);
      add_term(nk, ck, std::conj(ck));
    }
  }
  for (double x : hm.nu_im) hm.complex_rates = hm.complex_rates || x != 0.0;
  hm.n_terms = static_cast<int>(hm.nu.size());
  const int M = hm.n_terms;
  // hierarchy
  std::vector<std::vector<int>> ados;
  {
    std::vector<int> cur(M, 0);
    for (int level = 0; level <= p.depth; ++level) {
      if (M == 0) {
        if (level == 0) ados.push_back({});
        continue;
      }
      enumerate_level(M, level, cur, 0, ados);
    }
  }
  if (p.rate_cut < 0.0 || !std::isfinite(p.rate_cut)) throw std::invalid_argument("rate_cut must be >= 0");
  if (p.rate_cut > 0.0) {
    // rate filter: sum_j n_j Re nu_j <= rate_cut (closed under n -> n - e_j)
    std::vector<std::vector<int>> kept;
    for (auto& n : ados) {
      double r = 0.0;
      for (int j = 0; j < M; ++j) r += n[j] * hm.nu[j];
      if (r <= p.rate_cut * (1.0 + 1e-9)) kept.push_back(std::move(n));
    }
    ados.swap(kept);
  }
  if (ados.size() > 2000000) throw std::invalid_argument("hierarchy larger than 2e6 ADOs");
  hm.n_ado = static_cast<int>(ados.size());
  std::map<std::string, int> index;
  for (int i = 0; i < hm.n_ado; ++i) index[key_of(ados[i])] = i;
  hm.ado_n.resize(static_cast<size_t>(hm.n_ado) * M);
  hm.ado_depth.resize(hm.n_ado);
  hm.gamma_sum.resize(hm.n_ado);
  hm.gamma_sum_im.resize(hm.n_ado);
  for (int i = 0; i < hm.n_ado; ++i) {
    int dep = 0;
    double gs = 0.0, gi = 0.0;
    for (int j = 0; j < M; ++j) {
      hm.ado_n[static_cast<size_t>(i) * M + j] = ados[i][j];
      dep += ados[i][j];
      gs += ados[i][j] * hm.nu[j];
      gi += ados[i][j] * hm.nu_im[j];
    }
    hm.ado_depth[i] = dep;
    hm.gamma_sum[i] = gs;
    hm.gamma_sum_im[i] = gi;
  }
  // neighbour lists, grouped by mode
  auto build_nb = [&](Neighbours& nb, bool adjoint) {
    nb.ptr.assign(static_cast<size_t>(hm.n_ado) * hm.n_modes + 1, 0);
    for (int i = 0; i < hm.n_ado; ++i) {
      for (int s = 0; s < hm.n_modes; ++s) {
        nb.ptr[static_cast<size_t>(i) * hm.n_modes + s] = static_cast<int>(nb.idx.size());
        for (int j = 0; j < M; ++j) {
          if (hm.term_mode[j] != s) continue;
          std::vector<int> n = ados[i];
          const int nj = n[j];
          // upper neighbour n + e_j
          n[j] = nj + 1;
          auto it = index.find(key_of(n));
          if (it != index.end()) {
            nb.idx.push_back(it->second);
            nb.tj.push_back(j);
            nb.tj.push_back(0);
            if (!adjoint) {
              nb.aL.push_back(1.0);
              nb.aR.push_back(1.0);
            } else {
              nb.aL.push_back(static_cast<double>(nj + 1) * hm.c[j]);
              nb.aR.push_back(static_cast<double>(nj + 1) * hm.cb[j]);
            }
          }
          // lower neighbour n - e_j
          if (nj > 0) {
            n[j] = nj - 1;
            nb.idx.push_back(index.at(key_of(n)));
            nb.tj.push_back(j);
            nb.tj.push_back(nj);
            if (!adjoint) {
              nb.aL.push_back(static_cast<double>(nj) * hm.c[j]);
              nb.aR.push_back(static_cast<double>(nj) * hm.cb[j]);
            } else {
              nb.aL.push_back(1.0);
              nb.aR.push_back(1.0);
            }
          }
        }
      }
    }
    nb.ptr[static_cast<size_t>(hm.n_ado) * hm.n_modes] = static_cast<int>(nb.idx.size());
  };
  build_nb(hm.fwd, false);
  build_nb(hm.adj, true);
  return hm;
}

}  // namespace heom

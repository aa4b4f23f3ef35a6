// Host-side model of the MAB oscillator HEOM (FP64): operators in the product
// eigenbasis, bath exponential terms and hierarchy tables.  Built once per
// parameter set; the device copy lives in heom_model (capi.hip).
#pragma once

#include <complex>
#include <string>
#include <vector>

#include "heom2dvs.h"

namespace heom {

using cplx = std::complex<double>;

struct Neighbours {
  // CSR over (ado, mode): entries ptr[ado*n_modes + s] .. ptr[ado*n_modes + s + 1]
  // list the hierarchy neighbours m whose contribution to ADO `ado` goes
  // through mode s's coupling operator V_s as  -i (aL V_s rho_m - aR rho_m V_s).
  std::vector<int> ptr, idx;
  std::vector<cplx> aL, aR;
  // per entry: (term j, n_j of ADO `ado`) for a lower neighbour n - e_j, (j, 0)
  // for an upper neighbour n + e_j
  std::vector<int> tj;
};

struct HostModel {
  int n_modes = 0;
  int dims[4] = {1, 1, 1, 1};
  int strides[4] = {1, 1, 1, 1};
  int d = 0;
  double dt = 0.0;
  int depth = 0;
  std::vector<double> H, mu, mu_plus, mu_minus;   // d*d row-major
  std::vector<std::vector<double>> v;            // per mode dims[s]^2
  std::vector<int> quanta;                       // per product state
  int n_terms = 0;
  std::vector<int> term_mode;
  std::vector<double> nu;                        // Re nu_j
  std::vector<double> nu_im;                     // Im nu_j (Brownian pairs)
  std::vector<cplx> c;
  std::vector<cplx> cb;                          // bra-side coefficients
  bool complex_rates = false;                    // some Im nu_j != 0
  int n_ado = 0;
  std::vector<int> ado_n;                        // n_ado * n_terms
  std::vector<int> ado_depth;
  std::vector<double> gamma_sum;                 // Re sum_j n_j nu_j
  std::vector<double> gamma_sum_im;              // Im sum_j n_j nu_j
  Neighbours fwd, adj;
};

// Throws std::invalid_argument with a message for bad parameters.
HostModel build_host_model(const heom_params& p);

// Symmetric eigen-decomposition by cyclic Jacobi rotations: A (n x n,
// row-major) is overwritten; eigenvalues ascending, eigenvectors as columns of
// V (row-major n x n).
void jacobi_eigen(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V);

// [K-1/K] Pade decomposition of coth(x/2) = 2/x + sum_k 4 eta_k x/(x^2 + xi_k^2)
// from the tridiagonal-matrix eigenvalue construction of Hu, Xu and Yan.
void pade_poles(int K, std::vector<double>& xi, std::vector<double>& eta);

}  // namespace heom

// Launch wrappers of the adjoint-gradient kernels (grad.hip), FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace heom {

// Forward-generator tables of a model for the gradient kernels.
struct GradOps {
  const double* v;      // per mode dims[s]^2, packed at v_off[s]
  const int* nb_ptr;    // forward neighbour CSR over (ado, mode)
  const int* nb_idx;
  const double* nb_a;   // (aL.re, aL.im, aR.re, aR.im) per entry
  const int* nb_tj;     // (term j, count n_j) per entry; count 0 for an upper neighbour
  const int* ado_n;     // n_ado x n_terms
  int v_off[4];
  int dims[4];
  int strides[4];
  int n_modes;
  int d;
  int n_ado;
  int n_terms;
};

// Whether the gradient kernels support a model: d <= 80, every mode dimension
// d_s <= 8 with d_s * d <= 512, and at most 4 exponential terms per mode.
bool grad_supported(int d, const int* dims, int n_modes, int max_terms_per_mode);
int grad_max_parts();

// out[0] + i out[1] = sum conj(x) y over n_mats complex d x d matrices (FP64);
// partial must hold 2 hdot_parts() doubles.
int hdot_parts();
void launch_hdot(const double* x, const double* y, long long n_mats, int d, double* partial, double* out,
                 hipStream_t stream);

// y += a x (complex a) over n_mats complex d x d matrices (FP64).
void launch_axpy(double a_re, double a_im, const double* x, double* y, long long n_mats, int d,
                 hipStream_t stream);

// out[r] = (accumulate ? out[r] : 0) + sum_s coef[r][s] in[s]; hierarchies of
// n_mats complex d x d matrices ([mat][re|im][d][d]) at strides in_stride /
// out_stride doubles; coef_dev: device [n_out][n_in] complex.
void launch_combine(const double* in, long long in_stride, int n_in, double* out, long long out_stride, int n_out,
                    const double* coef_dev, int accumulate, long long n_mats, int d, hipStream_t stream);

// partial[w][d*d] += Re(f sum_items (u z^T - z^T u)) for workgroup w (< grad_max_parts()).
void launch_gemm_grad(const double* u, const double* z, long long n_items, int d, double f_re, double f_im,
                      double* partial, hipStream_t stream);

// out[i] += sum_p partial[p][i], i < len.
void launch_reduce_parts(const double* partial, int n_parts, long long len, double* out, hipStream_t stream);

// Mode-s coupling, bath-coefficient and (s == 0) rate gradients of <u, L z>
// over n_items = n_traj x n_ado items: gv_s (ds x ds), gc ([n_terms][2]) and
// gnu ([n_terms]) accumulated with atomics.
void launch_nb_grad(const GradOps& g, int s, const double* u, const double* z, long long n_items, double* gv_s,
                    double* gc, double* gnu, hipStream_t stream);

}  // namespace heom

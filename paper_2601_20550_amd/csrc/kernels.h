// Device-side data of one model and the launch wrappers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace heom {

// Operators and hierarchy tables of a model on the device, in precision T.
// The neighbour coefficients are stored as 4 values per entry:
// (aL.re, aL.im, aR.re, aR.im).
template <typename T>
struct DevOps {
  const T* H;          // d x d
  const T* v;          // per mode dims[s]^2, packed
  const T* gamma;      // per ADO: Re sum_j n_j nu_j
  const T* gamma_im;   // per ADO: Im sum_j n_j nu_j, or null when every rate is real
  const int* nb_ptr;   // n_ado * n_modes + 1
  const int* nb_idx;
  const T* nb_a;
  int v_off[4];
  int dims[4];
  int strides[4];
  int n_modes;
  int d;
  int n_ado;
};

// out = L(in)                      (y == nullptr)
// out = y + coef * L(in)           (y != nullptr; out may alias y)
// for n_traj trajectories stored back to back ([traj][ado][re|im][d][d]).
template <typename T>
void launch_rhs(const DevOps<T>& op, const T* in, const T* y, T* out, double coef, int n_traj,
                hipStream_t stream);

// True when the matrix-core kernel can run a model of product dimension d and
// n_modes modes of dims[s] kept levels: the LDS planes fit 160 KB and every
// single-mode operator fits its 8 x 8 LDS slot.
template <typename T>
bool mfma_supported(int d, int n_modes, const int* dims);

// Same operation on the matrix cores: persistent workgroups of ceil(d/16)
// waves, one matrix at a time.  Hp: H zero-padded to DP x DP, DP =
// 16 ceil(d/16).  variant 1 forces the runtime mode-shape kernel; otherwise a
// compile-time shape is used when one matches the model.
template <typename T>
void launch_rhs_mfma(const DevOps<T>& op, const T* Hp, const T* in, const T* y, T* out, double coef,
                     int n_traj, int variant, hipStream_t stream);
// The matrix-core kernel with H read from its padded global copy instead of
// LDS (three workgroups per CU): FP32, d in 65..80, packed v_s of at most
// 128 values.  Hp as for launch_rhs_mfma.
template <typename T>
bool mfma_gh_supported(int d, int n_modes, const int* dims);
template <typename T>
void launch_rhs_mfma_gh(const DevOps<T>& op, const T* Hp, const T* in, const T* y, T* out, double coef, int n_traj,
                        hipStream_t stream);
// True when launch_rhs_mfma has a compile-time mode shape for this model
// (otherwise variants 0 and 1 run the same kernel).
template <typename T>
bool mfma_static_shape(const DevOps<T>& op);

// Compute units of the current device (cached).
int cu_count();

// Arguments of the matrix-core kernel for three-mode models in the (S; 4, 4)
// device basis a = 16 a_S + 4 a_M + a_F (FP32): H in that basis, the tables of
// DevOps, the table index of the modes in the roles S, M, F and their
// single-mode operators (row-major; vS is NB x NB with NB = d / 16).
struct KronArgs {
  const float* H;
  const float* gamma;
  const float* gamma_im;
  const int* nb_ptr;
  const int* nb_idx;
  const float* nb_a;
  int n_modes;
  int n_ado;
  int mode_S, mode_M, mode_F;
  float vS[64];
  float vM[16];
  float vF[16];
};

// Roles (S, M, F) of the modes when the model has the (S; 4, 4) structure
// the kernel needs (three modes, d = 64 or 80, two modes of 4 levels and the
// slow one of d / 16 levels); false otherwise.
bool kron_roles(int d, int n_modes, const int* dims, int* roles);
bool kron_supported(int d, int n_modes, const int* dims);
// out = y + coef L(in) (or L(in) when y is null) over n_traj trajectories in
// the device basis; one wave per real plane of an output matrix.
void launch_rhs_kron(const KronArgs& a, int d, const float* in, const float* y, float* out, double coef, int n_traj,
                     hipStream_t stream);

// One model instance inside a multi-instance launch (see
// launch_rhs_mfma_multi): its tables, its padded H, the input, base (y, may be
// null) and output hierarchies of its n_traj trajectories, and its first item
// in the launch (items of an instance: n_traj x n_ado).
template <typename T>
struct InstDesc {
  DevOps<T> op;
  const T* Hp;
  const T* in;
  const T* y;
  T* out;
  long long item_begin;
};

// Matrix-core RHS / RK4 stage over several instances of one size class
// (nb = ceil(d/16) equal for all) in one persistent launch.  desc: device
// array of n_inst descriptors sorted by item_begin; vw = 16 / sizeof(T) if
// every instance has d divisible by it, else 1.
// Launch shape of one class (0 / -1: the defaults): resident workgroups per
// CU (at most what LDS and registers allow) and the neighbour-sum form
// (1: X_s accumulated in LDS, 0: in registers; only where both exist).
struct MultiShape {
  int wg_per_cu = 0;
  int xl = -1;
};
template <typename T>
void launch_rhs_mfma_multi(const InstDesc<T>* desc, int n_inst, int nb, int vw, double coef, long long n_items,
                           hipStream_t stream, MultiShape shape = MultiShape());
// Workgroups that launch uses for one class.
template <typename T>
long long rhs_mfma_multi_grid(int nb, int vw, long long n_items, MultiShape shape = MultiShape());
// Whether both neighbour-sum forms exist for this class.
template <typename T>
bool multi_has_alt_xl(int nb);

// One size class of a single-launch multi-class stage: its instances are
// desc[inst_first, inst_first + n_inst) (items numbered from 0 within the
// class), served by workgroups [wg_begin, wg_end).
struct FusedClass {
  int nb;          // ceil(d / 16)
  int vw;          // vector width (16 / sizeof(T) if every d is divisible by it, else 1)
  int inst_first;
  int n_inst;
  long long n_items;
  int wg_begin;
  int wg_end;
};
constexpr int kFusedMaxNb = 5;   // classes up to d = 80

// Workgroup width (waves) of the single-launch kernel for these classes, 0 if
// some class is beyond kFusedMaxNb.
template <typename T>
int fused_block_waves(const int* nbs, int n);
// LDS bytes a class of ceil(d/16) = nb needs (the launch takes the largest).
template <typename T>
size_t fused_lds_bytes(int nb);
// Resident workgroups per CU of the single-launch kernel at this width and LDS.
template <typename T>
int fused_workgroups_per_cu(int waves, size_t lds);
// One RK4 stage (out = y + coef L(in) per instance descriptor) over every
// class in cls (device array, ordered by wg_begin; the last wg_end = grid).
template <typename T>
void launch_rhs_mfma_fused(const FusedClass* cls, int n_cls, const InstDesc<T>* desc, int waves, size_t lds,
                           int grid, double coef, hipStream_t stream);

// dst = D^x src (or (D^T)^x src) on every ADO, FP64 arithmetic.
template <typename T>
void launch_commutator(const double* D, int transpose, const T* src, T* dst, int d,
                       long long n_mats, hipStream_t stream);

// out[b * out_stride] = tr(A rho_{b, n=0}) (complex, FP64; out_stride in
// complex units), rho_b at stride traj_stride elements.
template <typename T>
void launch_trace(const double* A, const T* state, int d, long long traj_stride, int n_traj,
                  double* out, long long out_stride, hipStream_t stream);

// Largest |z| over n_mats complex d x d matrices (NaN counts as +inf).
// partial must hold n_mats doubles; result written to *result (device).
template <typename T>
void launch_absmax(const T* x, int d, long long n_mats, double* partial, double* result,
                   hipStream_t stream);

// dst (precision D) <- src (precision S), n elements.
template <typename S, typename D>
void launch_convert(const S* src, D* dst, long long n, hipStream_t stream);

// x <- 0 then x[traj][ado 0][re][0][0] = 1.
template <typename T>
void launch_set_ground(T* x, long long traj_stride, int n_traj, long long n_total,
                       hipStream_t stream);

// Bilinear pairings R[j][k] = factor * sum_e P_k[e] Y_j[e] (complex, FP64
// accumulation) between n1 hierarchies Y and n3 hierarchies P, each of
// n_ado complex d x d matrices in planar layout.  out: [n1][n3] complex
// (interleaved doubles, device).  work must hold
// pair_work_doubles(n1, n3, n_ado, d) doubles.
size_t pair_work_doubles(int n1, int n3, int n_ado, int d);
template <typename T>
void launch_pairing(const T* Y, int n1, const T* P, int n3, int n_ado, int d, double fac_re,
                    double fac_im, double* work, double* out, hipStream_t stream);

// 2D correlation spectrum from R_I, R_II ([n1][n3] complex, device) into
// S ([2 n3][2 n1], device).  work must hold 2 * 2 * n3 * n1 * 2 doubles.
void launch_spectrum(const double* RI, const double* RII, int n1, int n3, double dt_s,
                     double* work, double* S, hipStream_t stream);

}  // namespace heom

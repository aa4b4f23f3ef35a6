// HIP kernels of the HEOM-2DVS hot path (gfx950).
//
// State layout: a hierarchy of one trajectory is n_ado complex d x d matrices
// stored planar, [ado][re|im][d][d]; trajectories are stored back to back.
// Work unit of the right-hand-side kernels: one (trajectory, ADO) matrix.
#include <hip/hip_runtime.h>

#include <cmath>
#include <stdexcept>
#include <string>

#include "kernels.h"

namespace heom {

namespace {

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Generic fused RHS / RK4-stage kernel (any d <= 128, FP32 or FP64).
//
//   L(rho)_n = -i (H rho_n - rho_n H) - gamma_n rho_n
//              - i sum_s (V_s X_s - Y_s V_s),
//   gamma_n = sum_j n_j nu_j (complex when a bath has complex rates),
//   X_s = sum_{m in nb(n,s)} aL_m rho_m,  Y_s = sum_{m in nb(n,s)} aR_m rho_m,
//
// where the neighbour lists and coefficients (from the host tables) encode the
// down-coupling n_j Theta_j rho_{n-e_j} and the up-coupling V^x rho_{n+e_j} of
// the HEOM (or their transposes for the adjoint).  V_s acts on mode s only:
// (V_s X)[a][c] = sum_k v_s[a_s][k] X[a with digit s = k][c].
//
// Real/imaginary split: Re L = H Im - Im H + ..., Im L = -(H Re - Re H) + ...,
// so the commutator is done on one staged component at a time (LDS holds a
// single real d x d matrix).
// ---------------------------------------------------------------------------
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void rhs_generic_kernel(DevOps<T> op, const T* __restrict__ in,
                                                         const T* y, T* out, T coef) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int d = op.d;
  const int dd = d * d;
  const long long item = blockIdx.x;
  const int n = static_cast<int>(item % op.n_ado);
  const long long traj_base = (item - n) * 2LL * dd;  // first ADO of this trajectory
  const long long base = item * 2LL * dd;
  const T* rin = in + base;
  const T* H = op.H;

  T accR[EPT], accI[EPT];

  // commutator with H, real part of L: H Im - Im H
  for (int e = threadIdx.x; e < dd; e += NT) sm[e] = rin[dd + e];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    accR[i] = T(0);
    if (e < dd) {
      const int a = e / d, c = e - (e / d) * d;
      T s = T(0);
      for (int k = 0; k < d; ++k) s += H[a * d + k] * sm[k * d + c] - sm[a * d + k] * H[k * d + c];
      accR[i] = s;
    }
  }
  __syncthreads();
  // imaginary part of L: -(H Re - Re H)
  for (int e = threadIdx.x; e < dd; e += NT) sm[e] = rin[e];
  __syncthreads();
  const T g = op.gamma[n];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    accI[i] = T(0);
    if (e < dd) {
      const int a = e / d, c = e - (e / d) * d;
      T s = T(0);
      for (int k = 0; k < d; ++k) s += H[a * d + k] * sm[k * d + c] - sm[a * d + k] * H[k * d + c];
      accI[i] = -s - g * rin[dd + e];
      accR[i] -= g * sm[e];
      if (op.gamma_im) {  // complex rates: -(g + i gi) rho
        const T gi = op.gamma_im[n];
        accR[i] += gi * rin[dd + e];
        accI[i] -= gi * sm[e];
      }
    }
  }
  // couplings to the hierarchy neighbours through V_s
  for (int s = 0; s < op.n_modes; ++s) {
    const int p0 = op.nb_ptr[n * op.n_modes + s];
    const int p1 = op.nb_ptr[n * op.n_modes + s + 1];
    if (p0 == p1) continue;
    const int ds = op.dims[s], st = op.strides[s];
    const T* vs = op.v + op.v_off[s];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e >= dd) continue;
      const int a = e / d, c = e - (e / d) * d;
      const int as = (a / st) % ds, cs = (c / st) % ds;
      T lR = T(0), lI = T(0), rR = T(0), rI = T(0);
      for (int q = p0; q < p1; ++q) {
        const T* rm = in + traj_base + static_cast<long long>(op.nb_idx[q]) * 2 * dd;
        const T aLr = op.nb_a[4 * q], aLi = op.nb_a[4 * q + 1];
        const T aRr = op.nb_a[4 * q + 2], aRi = op.nb_a[4 * q + 3];
        T xR = T(0), xI = T(0), yR = T(0), yI = T(0);
        for (int k = 0; k < ds; ++k) {
          const T vl = vs[as * ds + k];
          const int row = a + (k - as) * st;
          xR += vl * rm[row * d + c];
          xI += vl * rm[dd + row * d + c];
          const T vr = vs[k * ds + cs];
          const int col = c + (k - cs) * st;
          yR += vr * rm[a * d + col];
          yI += vr * rm[dd + a * d + col];
        }
        lR += aLr * xR - aLi * xI;
        lI += aLr * xI + aLi * xR;
        rR += aRr * yR - aRi * yI;
        rI += aRr * yI + aRi * yR;
      }
      // -i (l - r)
      accR[i] += lI - rI;
      accI[i] -= lR - rR;
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e >= dd) continue;
    if (y) {
      const T yr = y[base + e], yi = y[base + dd + e];
      out[base + e] = yr + coef * accR[i];
      out[base + dd + e] = yi + coef * accI[i];
    } else {
      out[base + e] = accR[i];
      out[base + dd + e] = accI[i];
    }
  }
}

template <typename T, int NT, int EPT>
void rhs_generic_launch(const DevOps<T>& op, const T* in, const T* y, T* out, T coef,
                        long long n_items, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((rhs_generic_kernel<T, NT, EPT>), dim3(static_cast<unsigned>(n_items)),
                     dim3(NT), lds, stream, op, in, y, out, coef);
}

// ---------------------------------------------------------------------------
// Commutator with a real FP64 operator: dst = D src - src D (or with D^T).
// One block per matrix; FP64 arithmetic regardless of the storage type.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void commutator_kernel(const double* __restrict__ D, int transpose,
                                                         const T* __restrict__ src, T* dst, int d) {
  const int dd = d * d;
  const long long base = static_cast<long long>(blockIdx.x) * 2 * dd;
  const T* x = src + base;
  for (int e = threadIdx.x; e < dd; e += blockDim.x) {
    const int a = e / d, c = e - (e / d) * d;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < d; ++k) {
      const double dak = transpose ? D[k * d + a] : D[a * d + k];
      const double dkc = transpose ? D[c * d + k] : D[k * d + c];
      sr += dak * static_cast<double>(x[k * d + c]) - static_cast<double>(x[a * d + k]) * dkc;
      si += dak * static_cast<double>(x[dd + k * d + c]) - static_cast<double>(x[dd + a * d + k]) * dkc;
    }
    dst[base + e] = static_cast<T>(sr);
    dst[base + dd + e] = static_cast<T>(si);
  }
}

// Same operation with D and the matrix staged in LDS and 4 x 4 output blocks
// per thread (FP64 arithmetic, the matrix kept in its storage type in LDS):
// one block of ceil(d/4)^2 threads (rounded up to whole waves) per matrix.
// Summation over k in the same order as commutator_kernel.
template <typename T>
__global__ __launch_bounds__(512) void commutator_tiled_kernel(const double* __restrict__ D, int transpose,
                                                                const T* __restrict__ src, T* dst, int d) {
  extern __shared__ unsigned char smem_raw[];
  const int ld = d + 1;
  double* sD = reinterpret_cast<double*>(smem_raw);
  T* sXr = reinterpret_cast<T*>(sD + d * ld);
  T* sXi = sXr + d * ld;
  const int dd = d * d;
  const long long base = static_cast<long long>(blockIdx.x) * 2 * dd;
  for (int e = threadIdx.x; e < dd; e += blockDim.x) {
    const int a = e / d, c = e - (e / d) * d;
    sD[a * ld + c] = transpose ? D[c * d + a] : D[e];
    sXr[a * ld + c] = src[base + e];
    sXi[a * ld + c] = src[base + dd + e];
  }
  __syncthreads();
  const int nt = (d + 3) / 4;
  const int t = threadIdx.x;
  if (t >= nt * nt) return;
  const int a0 = 4 * (t / nt), c0 = 4 * (t - (t / nt) * nt);
  double accR[4][4], accI[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      accR[i][j] = 0.0;
      accI[i][j] = 0.0;
    }
  for (int k = 0; k < d; ++k) {
    double dA[4], dB[4], xr[4], xi[4], yr[4], yi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool ok = a0 + i < d;
      dA[i] = ok ? sD[(a0 + i) * ld + k] : 0.0;                                // D[a][k]
      yr[i] = ok ? static_cast<double>(sXr[(a0 + i) * ld + k]) : 0.0;          // X[a][k]
      yi[i] = ok ? static_cast<double>(sXi[(a0 + i) * ld + k]) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool ok = c0 + j < d;
      dB[j] = ok ? sD[k * ld + c0 + j] : 0.0;                                  // D[k][c]
      xr[j] = ok ? static_cast<double>(sXr[k * ld + c0 + j]) : 0.0;            // X[k][c]
      xi[j] = ok ? static_cast<double>(sXi[k * ld + c0 + j]) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        accR[i][j] += dA[i] * xr[j] - yr[i] * dB[j];
        accI[i][j] += dA[i] * xi[j] - yi[i] * dB[j];
      }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (a0 + i < d && c0 + j < d) {
        const int e = (a0 + i) * d + c0 + j;
        dst[base + e] = static_cast<T>(accR[i][j]);
        dst[base + dd + e] = static_cast<T>(accI[i][j]);
      }
}

// ---------------------------------------------------------------------------
// tr(A rho_0) per trajectory, FP64.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void trace_kernel(const double* __restrict__ A, const T* __restrict__ x,
                                                    int d, long long traj_stride, double* out,
                                                    long long out_stride) {
  __shared__ double red[2][256];
  const int dd = d * d;
  const T* r = x + static_cast<long long>(blockIdx.x) * traj_stride;
  double sr = 0.0, si = 0.0;
  for (int e = threadIdx.x; e < dd; e += 256) {
    const int a = e / d, c = e - (e / d) * d;
    const double w = A[c * d + a];
    sr += w * static_cast<double>(r[e]);
    si += w * static_cast<double>(r[dd + e]);
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = si;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x * out_stride] = red[0][0];
    out[2 * blockIdx.x * out_stride + 1] = red[1][0];
  }
}

// ---------------------------------------------------------------------------
// max |z| per matrix, then over matrices.
// ---------------------------------------------------------------------------
__device__ inline double nanmax(double a, double b) {
  if (a != a || b != b) return INFINITY;
  return a > b ? a : b;
}

template <typename T>
__global__ __launch_bounds__(256) void absmax_kernel(const T* __restrict__ x, int d, double* partial) {
  __shared__ double red[256];
  const int dd = d * d;
  const T* r = x + static_cast<long long>(blockIdx.x) * 2 * dd;
  double m = 0.0;
  for (int e = threadIdx.x; e < dd; e += 256) {
    const double re = static_cast<double>(r[e]), im = static_cast<double>(r[dd + e]);
    m = nanmax(m, sqrt(re * re + im * im));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = nanmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void max_reduce_kernel(const double* __restrict__ partial, long long n,
                                                         double* result) {
  __shared__ double red[256];
  double m = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) m = nanmax(m, partial[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = nanmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *result = red[0];
}

template <typename S, typename D>
__global__ __launch_bounds__(256) void convert_kernel(const S* __restrict__ src, D* __restrict__ dst,
                                                      long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    dst[i] = static_cast<D>(src[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void fill_zero_kernel(T* x, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) x[i] = T(0);
}

template <typename T>
__global__ void set_one_kernel(T* x, long long traj_stride, int n_traj) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_traj) x[b * traj_stride] = T(1);
}

// ---------------------------------------------------------------------------
// Pairing R[j][k] = fac * sum_e P_k[e] Y_j[e] (complex bilinear, FP64).
// Split-K tiled product: block (chunk, jt, kt) computes a 16x16 tile of
// partial sums over a contiguous range of the element index; a second kernel
// sums the chunks in a fixed order (deterministic).
// ---------------------------------------------------------------------------
constexpr int PT = 16;         // tile edge
constexpr int PCHUNK = 65536;  // complex elements per split-K chunk

template <typename T>
__global__ __launch_bounds__(PT* PT) void pairing_kernel(const T* __restrict__ Y, int n1,
                                                         const T* __restrict__ P, int n3, int n_ado,
                                                         int d, long long n_elem, double* work) {
  __shared__ double sYr[PT][PT + 1], sYi[PT][PT + 1], sPr[PT][PT + 1], sPi[PT][PT + 1];
  const int tx = threadIdx.x % PT, ty = threadIdx.x / PT;
  const int j0 = blockIdx.y * PT, k0 = blockIdx.z * PT;
  const long long e0 = static_cast<long long>(blockIdx.x) * PCHUNK;
  const long long e1 = min(e0 + PCHUNK, n_elem);
  const long long dd = static_cast<long long>(d) * d;
  const long long traj_stride = static_cast<long long>(n_ado) * 2 * dd;
  double accR = 0.0, accI = 0.0;
  for (long long e = e0; e < e1; e += PT) {
    // load a PT x PT slab: rows = trajectories, cols = elements e..e+PT
    {
      const long long ee = e + tx;
      double yr = 0, yi = 0, pr = 0, pi = 0;
      if (ee < e1) {
        const long long m = ee / dd, r = ee - m * dd;
        const long long off = m * 2 * dd + r;
        if (j0 + ty < n1) {
          const T* y = Y + static_cast<long long>(j0 + ty) * traj_stride;
          yr = static_cast<double>(y[off]);
          yi = static_cast<double>(y[off + dd]);
        }
        if (k0 + ty < n3) {
          const T* p = P + static_cast<long long>(k0 + ty) * traj_stride;
          pr = static_cast<double>(p[off]);
          pi = static_cast<double>(p[off + dd]);
        }
      }
      sYr[ty][tx] = yr;
      sYi[ty][tx] = yi;
      sPr[ty][tx] = pr;
      sPi[ty][tx] = pi;
    }
    __syncthreads();
    // thread (ty, tx) owns pair (j0 + ty, k0 + tx)
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const double a = sYr[ty][q], b = sYi[ty][q], c = sPr[tx][q], dq = sPi[tx][q];
      accR += a * c - b * dq;
      accI += a * dq + b * c;
    }
    __syncthreads();
  }
  const int j = j0 + ty, k = k0 + tx;
  if (j < n1 && k < n3) {
    double* w = work + (static_cast<long long>(blockIdx.x) * n1 * n3 + static_cast<long long>(j) * n3 + k) * 2;
    w[0] = accR;
    w[1] = accI;
  }
}

__global__ __launch_bounds__(256) void pairing_reduce_kernel(const double* __restrict__ work, int n_chunk,
                                                             int n_pairs, double fr, double fi,
                                                             double* out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n_pairs) return;
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < n_chunk; ++c) {
    sr += work[(static_cast<long long>(c) * n_pairs + p) * 2];
    si += work[(static_cast<long long>(c) * n_pairs + p) * 2 + 1];
  }
  out[2 * p] = fr * sr - fi * si;
  out[2 * p + 1] = fr * si + fi * sr;
}

// ---------------------------------------------------------------------------
// 2D spectrum.  Stage 1: T_P[m3][j] = sum_k w_k exp(i W3_m3 t3_k) R_P[j][k].
// Stage 2: S[m3][m1] = -Im dt^2 (sum_j w_j exp(-i W1 t1_j) T_I[m3][j]
//                                 + sum_j w_j exp(+i W1 t1_j) T_II[m3][j]).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void spectrum_stage1(const double* __restrict__ RI,
                                                       const double* __restrict__ RII, int n1, int n3,
                                                       double dt, double* T) {
  const long long id = blockIdx.x * 256LL + threadIdx.x;
  const long long total = 2LL * 2 * n3 * n1;
  if (id >= total) return;
  const int j = static_cast<int>(id % n1);
  const int m3 = static_cast<int>((id / n1) % (2 * n3));
  const int P = static_cast<int>(id / (static_cast<long long>(n1) * 2 * n3));
  const double* R = P == 0 ? RI : RII;
  const double W3 = 2.0 * M_PI * (m3 - n3) / (2.0 * n3 * dt);
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < n3; ++k) {
    const double w = k == 0 ? 0.5 : 1.0;
    double sn, cs;
    sincos(W3 * dt * k, &sn, &cs);
    const double rr = R[2 * (static_cast<long long>(j) * n3 + k)];
    const double ri = R[2 * (static_cast<long long>(j) * n3 + k) + 1];
    sr += w * (cs * rr - sn * ri);
    si += w * (cs * ri + sn * rr);
  }
  T[2 * id] = sr;
  T[2 * id + 1] = si;
}

__global__ __launch_bounds__(256) void spectrum_stage2(const double* __restrict__ T, int n1, int n3,
                                                       double dt, double* S) {
  const long long id = blockIdx.x * 256LL + threadIdx.x;
  if (id >= 4LL * n3 * n1) return;
  const int m1 = static_cast<int>(id % (2 * n1));
  const int m3 = static_cast<int>(id / (2 * n1));
  const double W1 = 2.0 * M_PI * (m1 - n1) / (2.0 * n1 * dt);
  double acc = 0.0;  // imaginary part of the sum
  for (int P = 0; P < 2; ++P) {
    const double sgn = P == 0 ? -1.0 : 1.0;
    const double* Tp = T + 2 * (static_cast<long long>(P) * 2 * n3 * n1 + static_cast<long long>(m3) * n1);
    for (int j = 0; j < n1; ++j) {
      const double w = j == 0 ? 0.5 : 1.0;
      double sn, cs;
      sincos(sgn * W1 * dt * j, &sn, &cs);
      acc += w * (cs * Tp[2 * j + 1] + sn * Tp[2 * j]);
    }
  }
  S[id] = -dt * dt * acc;
}

template <int NT>
constexpr int ept_for(int dd) {
  return (dd + NT - 1) / NT;
}

}  // namespace

// ---------------------------------------------------------------- wrappers --

template <typename T>
void launch_rhs(const DevOps<T>& op, const T* in, const T* y, T* out, double coef, int n_traj,
                hipStream_t stream) {
  const long long n_items = static_cast<long long>(n_traj) * op.n_ado;
  if (n_items == 0) return;
  const int dd = op.d * op.d;
  const size_t lds = static_cast<size_t>(dd) * sizeof(T);
  const T c = static_cast<T>(coef);
  if (dd <= 64) {
    rhs_generic_launch<T, 64, 1>(op, in, y, out, c, n_items, lds, stream);
  } else {
    const int need = (dd + 255) / 256;
    if (need <= 1) rhs_generic_launch<T, 256, 1>(op, in, y, out, c, n_items, lds, stream);
    else if (need <= 2) rhs_generic_launch<T, 256, 2>(op, in, y, out, c, n_items, lds, stream);
    else if (need <= 4) rhs_generic_launch<T, 256, 4>(op, in, y, out, c, n_items, lds, stream);
    else if (need <= 8) rhs_generic_launch<T, 256, 8>(op, in, y, out, c, n_items, lds, stream);
    else if (need <= 16) rhs_generic_launch<T, 256, 16>(op, in, y, out, c, n_items, lds, stream);
    else if (need <= 25) rhs_generic_launch<T, 256, 25>(op, in, y, out, c, n_items, lds, stream);
    else if (need <= 40) rhs_generic_launch<T, 256, 40>(op, in, y, out, c, n_items, lds, stream);
    else rhs_generic_launch<T, 256, 64>(op, in, y, out, c, n_items, lds, stream);
  }
  check_launch("rhs kernel");
}

template <typename T>
void launch_commutator(const double* D, int transpose, const T* src, T* dst, int d, long long n_mats,
                       hipStream_t stream) {
  if (n_mats == 0) return;
  // LDS-staged kernel when D (double) and the matrix (T) fit in 160 KB;
  // src and dst must not overlap (every caller writes another buffer)
  const size_t lds = static_cast<size_t>(d) * (d + 1) * (sizeof(double) + 2 * sizeof(T));
  const int nt = (d + 3) / 4;
  const int threads = ((nt * nt + 63) / 64) * 64;
  if (lds <= 160 * 1024 && threads <= 512) {
    static bool configured = false;
    if (!configured) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&commutator_tiled_kernel<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      configured = true;
    }
    hipLaunchKernelGGL((commutator_tiled_kernel<T>), dim3(static_cast<unsigned>(n_mats)), dim3(threads), lds,
                       stream, D, transpose, src, dst, d);
  } else {
    hipLaunchKernelGGL((commutator_kernel<T>), dim3(static_cast<unsigned>(n_mats)), dim3(256), 0, stream,
                       D, transpose, src, dst, d);
  }
  check_launch("commutator kernel");
}

template <typename T>
void launch_trace(const double* A, const T* state, int d, long long traj_stride, int n_traj, double* out,
                  long long out_stride, hipStream_t stream) {
  if (n_traj == 0) return;
  hipLaunchKernelGGL((trace_kernel<T>), dim3(n_traj), dim3(256), 0, stream, A, state, d, traj_stride, out,
                     out_stride);
  check_launch("trace kernel");
}

template <typename T>
void launch_absmax(const T* x, int d, long long n_mats, double* partial, double* result, hipStream_t stream) {
  hipLaunchKernelGGL((absmax_kernel<T>), dim3(static_cast<unsigned>(n_mats)), dim3(256), 0, stream, x, d,
                     partial);
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, stream, partial, n_mats, result);
  check_launch("absmax kernel");
}

template <typename S, typename D>
void launch_convert(const S* src, D* dst, long long n, hipStream_t stream) {
  if (n == 0) return;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((convert_kernel<S, D>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, src,
                     dst, n);
  check_launch("convert kernel");
}

template <typename T>
void launch_set_ground(T* x, long long traj_stride, int n_traj, long long n_total, hipStream_t stream) {
  long long blocks = (n_total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks > 0)
    hipLaunchKernelGGL((fill_zero_kernel<T>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, x,
                       n_total);
  if (n_traj > 0)
    hipLaunchKernelGGL((set_one_kernel<T>), dim3((n_traj + 63) / 64), dim3(64), 0, stream, x, traj_stride,
                       n_traj);
  check_launch("set ground");
}

size_t pair_work_doubles(int n1, int n3, int n_ado, int d) {
  const long long n_elem = static_cast<long long>(n_ado) * d * d;
  const long long n_chunk = (n_elem + PCHUNK - 1) / PCHUNK;
  return static_cast<size_t>(n_chunk) * n1 * n3 * 2;
}

template <typename T>
void launch_pairing(const T* Y, int n1, const T* P, int n3, int n_ado, int d, double fr, double fi,
                    double* work, double* out, hipStream_t stream) {
  const long long n_elem = static_cast<long long>(n_ado) * d * d;
  const int n_chunk = static_cast<int>((n_elem + PCHUNK - 1) / PCHUNK);
  dim3 grid(n_chunk, (n1 + PT - 1) / PT, (n3 + PT - 1) / PT);
  hipLaunchKernelGGL((pairing_kernel<T>), grid, dim3(PT * PT), 0, stream, Y, n1, P, n3, n_ado, d, n_elem,
                     work);
  const int n_pairs = n1 * n3;
  hipLaunchKernelGGL(pairing_reduce_kernel, dim3((n_pairs + 255) / 256), dim3(256), 0, stream, work, n_chunk,
                     n_pairs, fr, fi, out);
  check_launch("pairing kernel");
}

void launch_spectrum(const double* RI, const double* RII, int n1, int n3, double dt_s, double* work,
                     double* S, hipStream_t stream) {
  const long long t1 = 4LL * n3 * n1;
  hipLaunchKernelGGL(spectrum_stage1, dim3(static_cast<unsigned>((t1 + 255) / 256)), dim3(256), 0, stream, RI,
                     RII, n1, n3, dt_s, work);
  hipLaunchKernelGGL(spectrum_stage2, dim3(static_cast<unsigned>((t1 + 255) / 256)), dim3(256), 0, stream,
                     work, n1, n3, dt_s, S);
  check_launch("spectrum kernels");
}

// explicit instantiations
template void launch_rhs<double>(const DevOps<double>&, const double*, const double*, double*, double, int,
                                 hipStream_t);
template void launch_rhs<float>(const DevOps<float>&, const float*, const float*, float*, double, int,
                                hipStream_t);
template void launch_commutator<double>(const double*, int, const double*, double*, int, long long,
                                        hipStream_t);
template void launch_commutator<float>(const double*, int, const float*, float*, int, long long, hipStream_t);
template void launch_trace<double>(const double*, const double*, int, long long, int, double*, long long,
                                   hipStream_t);
template void launch_trace<float>(const double*, const float*, int, long long, int, double*, long long,
                                  hipStream_t);
template void launch_absmax<double>(const double*, int, long long, double*, double*, hipStream_t);
template void launch_absmax<float>(const float*, int, long long, double*, double*, hipStream_t);
template void launch_convert<double, float>(const double*, float*, long long, hipStream_t);
template void launch_convert<float, double>(const float*, double*, long long, hipStream_t);
template void launch_convert<double, double>(const double*, double*, long long, hipStream_t);
template void launch_convert<float, float>(const float*, float*, long long, hipStream_t);
template void launch_set_ground<double>(double*, long long, int, long long, hipStream_t);
template void launch_set_ground<float>(float*, long long, int, long long, hipStream_t);
template void launch_pairing<double>(const double*, int, const double*, int, int, int, double, double, double*,
                                     double*, hipStream_t);
template void launch_pairing<float>(const float*, int, const float*, int, int, int, double, double, double*,
                                    double*, hipStream_t);

}  // namespace heom

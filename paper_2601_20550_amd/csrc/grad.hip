// Kernels of the adjoint (reverse-mode) gradient of the responses, FP64.
//
// The HEOM generator L (Sec. II.B, Eq. HEOM_DB) is linear in the system
// Hamiltonian H, in the single-mode coupling operators v_s (entering as
// V_s = v_s on mode s), in the bath coefficients c_j and in the rates nu_j.
// For an adjoint hierarchy u and a forward hierarchy z, the derivative of the
// bilinear pairing <u, L z> (sum over all ADOs and matrix elements, no
// conjugation) with respect to those operators is a sum over ADOs n of
//
//   dH   : Re(-i (u_n z_n^T - z_n^T u_n))
//   dv_s : Im(TL) - Im(TR),  TL[a][a'] = sum_{r,y} u_n[(a,r)][y] zL_s[(a',r)][y],
//                            TR[a][a'] = sum_{x,r} zR_s[x][(a,r)] u_n[x][(a',r)],
//          zL_s = sum_{up j in s} z_{n+e_j} + sum_{down j in s} n_j c_j z_{n-e_j},
//          zR_s = the same with conj(c_j),   ((a,r): mode-s digit a, other digits r)
//   dRe c_j : n_j Im(<V_s u_n, z_{n-e_j}> - <u_n V_s, z_{n-e_j}>)
//   dIm c_j : n_j Re(<V_s u_n, z_{n-e_j}> + <u_n V_s, z_{n-e_j}>)
//   dnu_j   : -n_j Re <u_n, z_n>
//
// The same pairing with a dipole commutator D^x in place of L gives
// dD = Re(u z^T - z^T u) (factor f = 1 in gemm_grad instead of -i).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <string>

#include "grad.h"

namespace heom {

namespace {

constexpr int GT = 256;           // threads per workgroup
constexpr int MAXDS = 8;          // largest single-mode dimension supported
constexpr int MAXQ = 8;           // neighbour entries per (ADO, mode)
constexpr int MAXDOWN = 4;        // lower neighbours per (ADO, mode)

void check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

int g_cus = 0;
int cus() {
  if (!g_cus) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
      g_cus = p.multiProcessorCount;
    if (g_cus <= 0) g_cus = 256;
  }
  return g_cus;
}

// ------------------------------------------------------------ combine ------
// out[r] = (acc ? out[r] : 0) + sum_s coef[r][s] in[s]   (complex coefficients)
__global__ __launch_bounds__(GT) void combine_kernel(const double* __restrict__ in, long long in_stride, int n_in,
                                                     double* __restrict__ out, long long out_stride, int n_out,
                                                     const double* __restrict__ coef, int coef_ld, int acc,
                                                     long long n_c, long long dd) {
  for (long long c = blockIdx.x * static_cast<long long>(GT) + threadIdx.x; c < n_c;
       c += static_cast<long long>(gridDim.x) * GT) {
    const long long mat = c / dd, e = c - mat * dd;
    const long long off = mat * 2 * dd + e;
    double xr[16], xi[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      if (s < n_in) {
        xr[s] = in[s * in_stride + off];
        xi[s] = in[s * in_stride + off + dd];
      } else {
        xr[s] = 0.0;
        xi[s] = 0.0;
      }
    }
    for (int r = 0; r < n_out; ++r) {
      double ar = 0.0, ai = 0.0;
      if (acc) {
        ar = out[r * out_stride + off];
        ai = out[r * out_stride + off + dd];
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if (s < n_in) {
          const double cr = coef[2 * (r * coef_ld + s)], ci = coef[2 * (r * coef_ld + s) + 1];
          ar += cr * xr[s] - ci * xi[s];
          ai += cr * xi[s] + ci * xr[s];
        }
      }
      out[r * out_stride + off] = ar;
      out[r * out_stride + off + dd] = ai;
    }
  }
}

// ---------------------------------------------------------- gemm_grad ------
// partial[blockIdx.x][i][j] += Re(f * sum_items (u z^T - z^T u)[i][j]) on the
// FP64 matrix cores (v_mfma_f64_16x16x4: A[i][k] at lane i + 16 k, B[k][j] at
// lane j + 16 k, accumulator element r at row lq + 4 r, column lr).  NB waves
// (d <= 16 NB): the item's z is staged in LDS (zero padded to DP x DP);
// wave w accumulates the tiles (w, tj) of Re(f u z^T), A = f u from global
// memory (rows 16 w ..), B = z^T from LDS, and the tiles (ti, w) of
// Re(z^T f u), A = z^T from LDS, B = f u from global memory (columns 16 w ..).
// The two sums meet in LDS once per launch.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int NB>
__global__ __launch_bounds__(NB * 64) void gemm_grad_kernel(const double* __restrict__ u, const double* __restrict__ z,
                                                            long long n_items, int d, double f_re, double f_im,
                                                            double* __restrict__ partial) {
  constexpr int DP = 16 * NB;
  constexpr int LDZ = DP + 1;
  constexpr int NT = NB * 64;
  HIP_DYNAMIC_SHARED(double, lds);
  double* zr = lds;
  double* zi = lds + DP * LDZ;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const long long dd = static_cast<long long>(d) * d;
  f64x4 acc1[NB], acc2[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    acc1[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    acc2[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  for (int e = tid; e < 2 * DP * LDZ; e += NT) lds[e] = 0.0;
  const int ia = 16 * w + lr;  // row of f u in the first sum, column in the second
  for (long long it = blockIdx.x; it < n_items; it += gridDim.x) {
    const double* U = u + it * 2 * dd;
    const double* Z = z + it * 2 * dd;
    __syncthreads();  // previous item's LDS reads are complete
    // z in groups of SG elements per thread, every load of a group issued
    // before its LDS stores (a load-then-store loop pays one memory round
    // trip per element row)
    constexpr int SG = (NB >= 3 && NB <= 5) ? 4 * NB : 2 * NB;
    for (int e0 = tid; e0 < d * d; e0 += SG * NT) {
      double vr[SG], vi[SG];
#pragma unroll
      for (int g = 0; g < SG; ++g) {
        const int e = e0 + g * NT;
        const int ec = e < d * d ? e : e0;
        vr[g] = Z[ec];
        vi[g] = Z[ec + dd];
      }
#pragma unroll
      for (int g = 0; g < SG; ++g) {
        const int e = e0 + g * NT;
        if (e < d * d) {
          const int x = e / d, y = e - x * d;
          zr[x * LDZ + y] = vr[g];
          zi[x * LDZ + y] = vi[g];
        }
      }
    }
    __syncthreads();
    // Re(f u z^T): sum over columns c of u and z.  The u loads are
    // unconditional (clamped address, zero selected outside the matrix) so
    // that they can be issued ahead of the matrix-core chain.
#pragma unroll NB
    for (int c0 = 0; c0 < DP; c0 += 4) {
      const int c = c0 + lk;
      const bool in = ia < d && c < d;
      const int off = in ? ia * d + c : 0;
      const double ur0 = U[off], ui0 = U[off + dd];
      const double ur = in ? ur0 : 0.0, ui = in ? ui0 : 0.0;
      const double ar = f_re * ur - f_im * ui, ai = -(f_re * ui + f_im * ur);
#pragma unroll
      for (int tj = 0; tj < NB; ++tj) {
        const int j = 16 * tj + lr;
        acc1[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, zr[j * LDZ + c], acc1[tj], 0, 0, 0);
        acc1[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, zi[j * LDZ + c], acc1[tj], 0, 0, 0);
      }
    }
    // Re(z^T f u): sum over rows x of z and u
#pragma unroll NB
    for (int x0 = 0; x0 < DP; x0 += 4) {
      const int x = x0 + lk;
      const bool in = x < d && ia < d;
      const int off = in ? x * d + ia : 0;
      const double ur0 = U[off], ui0 = U[off + dd];
      const double ur = in ? ur0 : 0.0, ui = in ? ui0 : 0.0;
      const double br = f_re * ur - f_im * ui, bi = -(f_re * ui + f_im * ur);
#pragma unroll
      for (int ti = 0; ti < NB; ++ti) {
        const int i = 16 * ti + lr;
        acc2[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(zr[x * LDZ + i], br, acc2[ti], 0, 0, 0);
        acc2[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(zi[x * LDZ + i], bi, acc2[ti], 0, 0, 0);
      }
    }
  }
  // G = sum1 - sum2 in LDS: wave w owns tile row w of the first sum and tile
  // column w of the second
  __syncthreads();
  double* G = lds;  // DP x LDZ
#pragma unroll
  for (int tj = 0; tj < NB; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) G[(16 * w + lk + 4 * r) * LDZ + 16 * tj + lr] = acc1[tj][r];
  __syncthreads();
#pragma unroll
  for (int ti = 0; ti < NB; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) G[(16 * ti + lk + 4 * r) * LDZ + 16 * w + lr] -= acc2[ti][r];
  __syncthreads();
  double* P = partial + static_cast<long long>(blockIdx.x) * dd;
  for (int e = tid; e < d * d; e += NT) {
    const int i = e / d, j = e - i * d;
    P[e] += G[i * LDZ + j];
  }
}

template <int NB>
size_t gemm_grad_lds() {
  constexpr int DP = 16 * NB;
  return sizeof(double) * 2 * DP * (DP + 1);
}

__global__ void reduce_parts_kernel(const double* __restrict__ partial, int n_parts, long long len,
                                    double* __restrict__ out) {
  const long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
  if (i >= len) return;
  double s = 0.0;
  for (int p = 0; p < n_parts; ++p) s += partial[p * len + i];
  out[i] += s;
}

// ------------------------------------------------------------ nb_grad ------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline int digit_row(int a, int r, int ds, int S) {
  // product index with mode-s digit a and remaining digits r = hi * S + lo
  const int hi = r / S, lo = r - hi * S;
  return (hi * ds + a) * S + lo;
}

// One launch per mode s (DS = its dimension), NT = 512 threads.  Thread
// t < DS * d owns the row digit ap = t / d and the column y = t % d, whose
// mode-s digit dc is then fixed too; it loops over the rest r of the row
// index (x = (ap, r)), so every accumulator index is a compile-time constant:
//   TL[a][ap]  += Im(u[(a,r)][y] zL[x][y])          (a < DS)
//   TR[dc][a'] += Im(zR[x][y] u[x][(a',r_y)])       (a' < DS)
// Each neighbour element is loaded once, coalesced along y.  Lower-neighbour
// pairings and <u_n, z_n> are reduced per item; TL and TR once per
// workgroup at the end.
constexpr int NBT = 512;

template <int DS>
__global__ __launch_bounds__(NBT) void nb_grad_kernel(GradOps g, int s, const double* __restrict__ u,
                                                      const double* __restrict__ z, long long n_items,
                                                      double* __restrict__ gv, double* __restrict__ gc,
                                                      double* __restrict__ gnu) {
  HIP_DYNAMIC_SHARED(double, lds);
  constexpr int NV = 4 * MAXDOWN + 2;
  constexpr int NW = NBT / 64;
  const int d = g.d, S = g.strides[s], LD = d + 1;
  const long long dd = static_cast<long long>(d) * d;
  double* sur = lds;
  double* sui = sur + d * LD;
  double* sv = sui + d * LD;                                   // DS * DS (<= MAXDS^2)
  double* red = sv + MAXDS * MAXDS;                            // NW x NV
  int* qi = reinterpret_cast<int*>(red + NW * NV);             // per item: idx, term, count
  double* qa = reinterpret_cast<double*>(qi + 4 * MAXQ);       // aL re, aL im
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const bool active = tid < DS * d;
  const int ap = active ? tid / d : 0, y = active ? tid % d : 0;
  const int R = d / DS;
  const int hy = y / (DS * S), dc = (y / S) % DS, ly = y % S;
  const int ry0 = hy * DS * S + ly;  // column index of y with mode-s digit 0
  for (int e = tid; e < DS * DS; e += NBT) sv[e] = g.v[g.v_off[s] + e];
  double TL[DS], TR[DS];
#pragma unroll
  for (int a = 0; a < DS; ++a) TL[a] = TR[a] = 0.0;
  for (long long it = blockIdx.x; it < n_items; it += gridDim.x) {
    const long long traj = it / g.n_ado;
    const int n = static_cast<int>(it - traj * g.n_ado);
    const double* U = u + it * 2 * dd;
    const double* Zt = z + traj * g.n_ado * 2 * dd;
    __syncthreads();
    // u in groups of 8 elements per thread, loads before LDS stores (as in
    // gemm_grad_kernel)
    for (int e0 = tid; e0 < d * d; e0 += 8 * NBT) {
      double vr[8], vi[8];
#pragma unroll
      for (int g8 = 0; g8 < 8; ++g8) {
        const int e = e0 + g8 * NBT;
        const int ec = e < d * d ? e : e0;
        vr[g8] = U[ec];
        vi[g8] = U[ec + dd];
      }
#pragma unroll
      for (int g8 = 0; g8 < 8; ++g8) {
        const int e = e0 + g8 * NBT;
        if (e < d * d) {
          const int x = e / d, yy = e - x * d;
          sur[x * LD + yy] = vr[g8];
          sui[x * LD + yy] = vi[g8];
        }
      }
    }
    const int q0 = g.nb_ptr[n * g.n_modes + s];
    const int nq = min(g.nb_ptr[n * g.n_modes + s + 1] - q0, MAXQ);
    if (tid < nq) {
      qi[4 * tid] = g.nb_idx[q0 + tid];
      qi[4 * tid + 1] = g.nb_tj[2 * (q0 + tid)];
      qi[4 * tid + 2] = g.nb_tj[2 * (q0 + tid) + 1];
      qa[2 * tid] = g.nb_a[4 * (q0 + tid)];
      qa[2 * tid + 1] = g.nb_a[4 * (q0 + tid) + 1];
    }
    __syncthreads();
    double pLr[MAXDOWN], pLi[MAXDOWN], pRr[MAXDOWN], pRi[MAXDOWN];
#pragma unroll
    for (int k = 0; k < MAXDOWN; ++k) pLr[k] = pLi[k] = pRr[k] = pRi[k] = 0.0;
    double Pr = 0.0, Pi = 0.0;
    if (active) {
      for (int r = 0; r < R; ++r) {
        const int hr = r / S, lr = r - hr * S;
        const int xr0 = hr * DS * S + lr;  // row index with mode-s digit 0
        const int x = xr0 + ap * S;
        double vur = 0.0, vui = 0.0, uvr = 0.0, uvi = 0.0;
        double uar[DS], uai[DS], ubr[DS], ubi[DS];
#pragma unroll
        for (int a = 0; a < DS; ++a) {
          uar[a] = sur[(xr0 + a * S) * LD + y];
          uai[a] = sui[(xr0 + a * S) * LD + y];
          const double va = sv[ap * DS + a];
          vur += va * uar[a];          // (V u)[x][y]
          vui += va * uai[a];
          ubr[a] = sur[x * LD + ry0 + a * S];
          ubi[a] = sui[x * LD + ry0 + a * S];
          const double vb = sv[a * DS + dc];
          uvr += ubr[a] * vb;          // (u V)[x][y]
          uvi += ubi[a] * vb;
        }
        // every neighbour element of this row is requested before any is
        // used: one memory latency per row instead of one per neighbour
        double zrq[MAXQ], ziq[MAXQ];
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
          zrq[q] = 0.0;
          ziq[q] = 0.0;
          if (q < nq) {
            const double* Zm = Zt + static_cast<long long>(qi[4 * q]) * 2 * dd;
            zrq[q] = Zm[x * d + y];
            ziq[q] = Zm[x * d + y + dd];
          }
        }
        double zLr = 0.0, zLi = 0.0, zRr = 0.0, zRi = 0.0;
        int kd = 0;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
          if (q >= nq) break;
          const double zr_ = zrq[q], zi_ = ziq[q];
          const double cr = qa[2 * q], ci = qa[2 * q + 1];
          zLr += cr * zr_ - ci * zi_;
          zLi += cr * zi_ + ci * zr_;
          zRr += cr * zr_ + ci * zi_;
          zRi += cr * zi_ - ci * zr_;
          if (qi[4 * q + 2] > 0) {
#pragma unroll
            for (int k = 0; k < MAXDOWN; ++k)
              if (k == kd) {
                pLr[k] += vur * zr_ - vui * zi_;
                pLi[k] += vur * zi_ + vui * zr_;
                pRr[k] += uvr * zr_ - uvi * zi_;
                pRi[k] += uvr * zi_ + uvi * zr_;
              }
            ++kd;
          }
        }
#pragma unroll
        for (int a = 0; a < DS; ++a) {
          TL[a] += uar[a] * zLi + uai[a] * zLr;
          TR[a] += zRr * ubi[a] + zRi * ubr[a];
        }
        if (s == 0) {
          const double* Zn = Zt + static_cast<long long>(n) * 2 * dd;
          const double zr_ = Zn[x * d + y], zi_ = Zn[x * d + y + dd];
          const double ur_ = sur[x * LD + y], ui_ = sui[x * LD + y];
          Pr += ur_ * zr_ - ui_ * zi_;
          Pi += ur_ * zi_ + ui_ * zr_;
        }
      }
    }
    // per-item reduction of the lower-neighbour pairings and <u_n, z_n>
    double vals[NV];
#pragma unroll
    for (int k = 0; k < MAXDOWN; ++k) {
      vals[4 * k] = pLr[k];
      vals[4 * k + 1] = pLi[k];
      vals[4 * k + 2] = pRr[k];
      vals[4 * k + 3] = pRi[k];
    }
    vals[NV - 2] = Pr;
    vals[NV - 1] = Pi;
#pragma unroll
    for (int k = 0; k < NV; ++k) vals[k] = wave_sum(vals[k]);
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < NV; ++k) red[wave * NV + k] = vals[k];
    __syncthreads();
    if (tid == 0) {
      double tot[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        tot[k] = 0.0;
        for (int w = 0; w < NW; ++w) tot[k] += red[w * NV + k];
      }
      int kd = 0;
      for (int q = 0; q < nq && kd < MAXDOWN; ++q) {
        const int cnt = qi[4 * q + 2];
        if (cnt > 0) {
          const int j = qi[4 * q + 1];
          const double lr_ = tot[4 * kd], li = tot[4 * kd + 1], rr = tot[4 * kd + 2], ri = tot[4 * kd + 3];
          atomicAdd(&gc[2 * j], cnt * (li - ri));
          atomicAdd(&gc[2 * j + 1], cnt * (lr_ + rr));
          ++kd;
        }
      }
      if (s == 0) {
        for (int j = 0; j < g.n_terms; ++j) {
          const int cnt = g.ado_n[static_cast<long long>(n) * g.n_terms + j];
          if (cnt > 0) atomicAdd(&gnu[j], -cnt * tot[NV - 2]);
        }
      }
    }
  }
  // workgroup reduction: gv[a][ap] += TL[a], gv[dc][a'] -= TR[a']
  __syncthreads();
  double* sacc = sur;  // the u planes are free now
  for (int e = tid; e < DS * DS; e += NBT) sacc[e] = 0.0;
  __syncthreads();
  if (active) {
#pragma unroll
    for (int a = 0; a < DS; ++a) {
      atomicAdd(&sacc[a * DS + ap], TL[a]);
      atomicAdd(&sacc[dc * DS + a], -TR[a]);
    }
  }
  __syncthreads();
  for (int e = tid; e < DS * DS; e += NBT) atomicAdd(&gv[e], sacc[e]);
}

size_t nb_grad_lds(int d) {
  return sizeof(double) * (2 * static_cast<size_t>(d) * (d + 1) + MAXDS * MAXDS + (NBT / 64) * (4 * MAXDOWN + 2)) +
         sizeof(int) * 4 * MAXQ + sizeof(double) * 2 * MAXQ + 64;
}

template <int DS>
void nb_grad_ds(const GradOps& g, int s, const double* u, const double* z, long long n_items, double* gv_s,
                double* gc, double* gnu, hipStream_t stream) {
  const size_t lds = nb_grad_lds(g.d);
  static size_t attr = 0;
  if (lds > attr) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&nb_grad_kernel<DS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
      throw std::runtime_error("nb_grad: LDS attribute");
    attr = lds;
  }
  const long long per_cu = std::max<long long>(1, (160 * 1024) / static_cast<long long>(lds));
  const long long grid = std::min<long long>(n_items, cus() * per_cu);
  if (grid <= 0) return;
  hipLaunchKernelGGL((nb_grad_kernel<DS>), dim3(static_cast<unsigned>(grid)), dim3(NBT), lds, stream, g, s, u, z,
                     n_items, gv_s, gc, gnu);
  check("nb_grad kernel");
}

// ---------------------------------------------------------------- hdot -----
// partial[b] = sum over this block's complex elements of conj(x) y
__global__ __launch_bounds__(GT) void hdot_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                  long long n_c, long long dd, double* __restrict__ partial) {
  __shared__ double sr[GT / 64], si[GT / 64];
  double ar = 0.0, ai = 0.0;
  for (long long c = blockIdx.x * static_cast<long long>(GT) + threadIdx.x; c < n_c;
       c += static_cast<long long>(gridDim.x) * GT) {
    const long long mat = c / dd, e = c - mat * dd;
    const long long off = mat * 2 * dd + e;
    const double xr = x[off], xi = x[off + dd], yr = y[off], yi = y[off + dd];
    ar += xr * yr + xi * yi;
    ai += xr * yi - xi * yr;
  }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  if (lane == 0) {
    sr[wave] = ar;
    si[wave] = ai;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0, ti = 0.0;
    for (int w = 0; w < GT / 64; ++w) {
      tr += sr[w];
      ti += si[w];
    }
    partial[2 * blockIdx.x] = tr;
    partial[2 * blockIdx.x + 1] = ti;
  }
}

__global__ void hdot_final_kernel(const double* __restrict__ partial, int n, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double tr = 0.0, ti = 0.0;
  for (int b = 0; b < n; ++b) {
    tr += partial[2 * b];
    ti += partial[2 * b + 1];
  }
  out[0] = tr;
  out[1] = ti;
}

// y += a x (complex a) over n_c complex elements
__global__ __launch_bounds__(GT) void axpy_kernel(double ar, double ai, const double* __restrict__ x,
                                                  double* __restrict__ y, long long n_c, long long dd) {
  for (long long c = blockIdx.x * static_cast<long long>(GT) + threadIdx.x; c < n_c;
       c += static_cast<long long>(gridDim.x) * GT) {
    const long long mat = c / dd, e = c - mat * dd;
    const long long off = mat * 2 * dd + e;
    const double xr = x[off], xi = x[off + dd];
    y[off] += ar * xr - ai * xi;
    y[off + dd] += ar * xi + ai * xr;
  }
}

}  // namespace

int grad_max_parts() { return 1024; }

bool grad_supported(int d, const int* dims, int n_modes, int max_terms_per_mode) {
  if (d > 80) return false;
  for (int s = 0; s < n_modes; ++s)
    if (dims[s] > MAXDS || dims[s] * d > NBT) return false;
  return 2 * max_terms_per_mode <= MAXQ && max_terms_per_mode <= MAXDOWN;
}

int hdot_parts() { return 1024; }

void launch_hdot(const double* x, const double* y, long long n_mats, int d, double* partial, double* out,
                 hipStream_t stream) {
  const long long dd = static_cast<long long>(d) * d;
  const long long n_c = n_mats * dd;
  const int blocks = static_cast<int>(std::max<long long>(1, std::min<long long>((n_c + GT - 1) / GT, hdot_parts())));
  hipLaunchKernelGGL(hdot_kernel, dim3(blocks), dim3(GT), 0, stream, x, y, n_c, dd, partial);
  hipLaunchKernelGGL(hdot_final_kernel, dim3(1), dim3(64), 0, stream, partial, blocks, out);
  check("hdot kernel");
}

void launch_axpy(double a_re, double a_im, const double* x, double* y, long long n_mats, int d,
                 hipStream_t stream) {
  const long long dd = static_cast<long long>(d) * d;
  const long long n_c = n_mats * dd;
  const int blocks = static_cast<int>(std::max<long long>(1, std::min<long long>((n_c + GT - 1) / GT, 65536)));
  hipLaunchKernelGGL(axpy_kernel, dim3(blocks), dim3(GT), 0, stream, a_re, a_im, x, y, n_c, dd);
  check("axpy kernel");
}

void launch_combine(const double* in, long long in_stride, int n_in, double* out, long long out_stride, int n_out,
                    const double* coef_dev, int accumulate, long long n_mats, int d, hipStream_t stream) {
  const long long dd = static_cast<long long>(d) * d;
  const long long n_c = n_mats * dd;
  const int blocks = static_cast<int>(std::min<long long>((n_c + GT - 1) / GT, 65536));
  for (int s0 = 0; s0 < n_in; s0 += 16) {
    const int k = std::min(16, n_in - s0);
    hipLaunchKernelGGL(combine_kernel, dim3(blocks), dim3(GT), 0, stream, in + s0 * in_stride, in_stride, k, out,
                       out_stride, n_out, coef_dev + 2 * s0, n_in, (s0 > 0 || accumulate) ? 1 : 0, n_c, dd);
  }
  check("combine kernel");
}

template <int NB>
void gemm_grad_nb(const double* u, const double* z, long long n_items, int d, double fr, double fi,
                  double* partial, hipStream_t stream) {
  const size_t lds = gemm_grad_lds<NB>();
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_grad_kernel<NB>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
      throw std::runtime_error("gemm_grad: LDS attribute");
    attr = true;
  }
  const long long per_cu = std::max<long long>(1, (160 * 1024) / static_cast<long long>(lds));
  const long long grid = std::min<long long>({n_items, cus() * per_cu, grad_max_parts()});
  if (grid <= 0) return;
  hipLaunchKernelGGL((gemm_grad_kernel<NB>), dim3(static_cast<unsigned>(grid)), dim3(NB * 64), lds, stream, u, z,
                     n_items, d, fr, fi, partial);
  check("gemm_grad kernel");
}

void launch_gemm_grad(const double* u, const double* z, long long n_items, int d, double f_re, double f_im,
                      double* partial, hipStream_t stream) {
  switch ((d + 15) / 16) {
    case 1: gemm_grad_nb<1>(u, z, n_items, d, f_re, f_im, partial, stream); break;
    case 2: gemm_grad_nb<2>(u, z, n_items, d, f_re, f_im, partial, stream); break;
    case 3: gemm_grad_nb<3>(u, z, n_items, d, f_re, f_im, partial, stream); break;
    case 4: gemm_grad_nb<4>(u, z, n_items, d, f_re, f_im, partial, stream); break;
    case 5: gemm_grad_nb<5>(u, z, n_items, d, f_re, f_im, partial, stream); break;
    default: throw std::runtime_error("gemm_grad: d > 80");
  }
}

void launch_reduce_parts(const double* partial, int n_parts, long long len, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(static_cast<unsigned>((len + 255) / 256)), dim3(256), 0, stream,
                     partial, n_parts, len, out);
  check("reduce kernel");
}

void launch_nb_grad(const GradOps& g, int s, const double* u, const double* z, long long n_items, double* gv_s,
                    double* gc, double* gnu, hipStream_t stream) {
  switch (g.dims[s]) {
    case 1: nb_grad_ds<1>(g, s, u, z, n_items, gv_s, gc, gnu, stream); break;
    case 2: nb_grad_ds<2>(g, s, u, z, n_items, gv_s, gc, gnu, stream); break;
    case 3: nb_grad_ds<3>(g, s, u, z, n_items, gv_s, gc, gnu, stream); break;
    case 4: nb_grad_ds<4>(g, s, u, z, n_items, gv_s, gc, gnu, stream); break;
    case 5: nb_grad_ds<5>(g, s, u, z, n_items, gv_s, gc, gnu, stream); break;
    case 6: nb_grad_ds<6>(g, s, u, z, n_items, gv_s, gc, gnu, stream); break;
    case 7: nb_grad_ds<7>(g, s, u, z, n_items, gv_s, gc, gnu, stream); break;
    case 8: nb_grad_ds<8>(g, s, u, z, n_items, gv_s, gc, gnu, stream); break;
    default: throw std::runtime_error("nb_grad: mode dimension > 8");
  }
}

}  // namespace heom

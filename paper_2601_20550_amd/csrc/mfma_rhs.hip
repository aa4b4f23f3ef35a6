// Fused HEOM right-hand side + RK4 stage on the matrix cores (gfx950 MFMA).
//
// A persistent workgroup of NB = ceil(d/16) row blocks (one or two waves per
// block) loops over (trajectory, ADO) matrices and computes
// out = y + coef * L(in)  for each.  Each wave owns a row block (16 rows) of
// the zero-padded DP x DP output (DP = 16 NB), or half of its column tiles,
// and computes every term of those outputs:
//
//   L rho = -i (H rho - rho H) - gamma_n rho + sum_s [ -i V_s X_s + i Y_s V_s ],
//   X_s = sum_q aL_q rho_{m_q},   Y_s = sum_q aR_q rho_{m_q}
//       = X_s + sum_q (aR_q - aL_q) rho_{m_q},
//
// with H real symmetric, V_s = v_s acting on mode s only, and the neighbour
// lists (m_q, aL_q, aR_q) of the host tables; aR = conj(aL) for Drude baths,
// so only the entries with complex coefficients enter the second sum, and
// gamma_n = sum_j n_j nu_j is complex only for complex rates (Brownian baths).
//
//   * H rho and rho H run on v_mfma 16x16x4 (FP32 or FP64) with H and rho
//     (two real planes) staged in LDS, rows padded to 16-byte alignment.
//   * The neighbour sums are formed from coalesced row-block loads (each
//     neighbour matrix is read once per workgroup), staged in the rho planes
//     of LDS, and contracted with v_s on the VALU.  The mode structure
//     (kept levels and strides of every mode) is a compile-time Shape for the
//     common cases, so the digit arithmetic of the Kronecker contractions is
//     constant-folded; DynShape handles any other shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <string>

#include "kernels.h"

namespace heom {

int cu_count() {
  static int count = 0;
  if (count == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      count = prop.multiProcessorCount;
    if (count <= 0) count = 256;
  }
  return count;
}

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Operand layouts (lane = 16 lq + lr): A[i][k] at lane i + 16 k, B[k][j] at
// lane j + 16 k.  Accumulator element r of a lane holds row crow(lq, r) and
// column lr: rows 4 lq .. 4 lq + 3 for the FP32 instruction, rows lq, lq + 4,
// lq + 8, lq + 12 for the FP64 one.
template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
  using acc = f32x4;
  __device__ static inline acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int crow(int lq, int r) { return 4 * lq + r; }
};

template <>
struct Mfma<double> {
  using acc = f64x4;
  __device__ static inline acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int crow(int lq, int r) { return lq + 4 * r; }
};

// Mode structure known at compile time.
template <int NM, int D0, int D1 = 1, int D2 = 1, int D3 = 1>
struct StaticShape {
  __device__ StaticShape(const int*, const int*, int, int) {}
  __device__ static constexpr int nm() { return NM; }
  __device__ static constexpr int dim(int s) { return s == 0 ? D0 : s == 1 ? D1 : s == 2 ? D2 : D3; }
  __host__ __device__ static constexpr int stride(int s) {
    return s == 0 ? D1 * D2 * D3 : s == 1 ? D2 * D3 : s == 2 ? D3 : 1;
  }
  __device__ static constexpr int d() { return D0 * D1 * D2 * D3; }
  static bool matches(int nm_, const int* dims, const int* strides) {
    if (nm_ != NM) return false;
    const int D[4] = {D0, D1, D2, D3};
    for (int s = 0; s < NM; ++s)
      if (dims[s] != D[s] || strides[s] != stride(s)) return false;
    return true;
  }
};

// Mode structure read from the kernel arguments.
struct DynShape {
  int nm_, d_, dims_[4], strides_[4];
  __device__ DynShape(const int* dims, const int* strides, int nm, int d) : nm_(nm), d_(d) {
    for (int s = 0; s < 4; ++s) {
      dims_[s] = dims[s];
      strides_[s] = strides[s];
    }
  }
  __device__ int nm() const { return nm_; }
  __device__ int dim(int s) const { return dims_[s]; }
  __device__ int stride(int s) const { return strides_[s]; }
  __device__ int d() const { return d_; }
};

// Row padding of the LDS planes: 16 bytes (4 FP32 or 2 FP64 elements) keep
// every row 16-byte aligned, so that the slab phases (staging, neighbour sums,
// the Y pass, epilogue) use 16-byte LDS accesses: FP32 at NB = 5 measured 6%
// faster per launch with half the bank-conflict cycles (two workgroups still
// fit), FP64 at NB = 5 2% faster; the largest layouts (FP32 NB = 7, FP64
// NB = 5) still fit 160 KB.
constexpr int lds_pad(size_t elem, int) { return elem == 4 ? 4 : 2; }

// LDS layout (elements of T): rho planes Re, Im and H, each DP x LD with
// LD = DP + lds_pad, then v_s (4 x 64 values).
// With HG (H read from its zero-padded global copy instead of LDS) the H plane
// is dropped and the single-mode operators are packed as in DevOps::v (at
// most kPackedV values): 54.3 KB instead of 81.6 KB at d = 80 in FP32, so
// three workgroups share a CU instead of two.
constexpr int kPackedV = 128;

template <typename T, int NB, bool HG = false>
struct Lds {
  static constexpr int DP = 16 * NB;
  static constexpr int LD = DP + lds_pad(sizeof(T), NB);
  static constexpr int PLANE = DP * LD;
  static constexpr int HOFF = 2 * PLANE;
  static constexpr int VOFF = HG ? HOFF : HOFF + PLANE;
  static constexpr size_t bytes = (VOFF + (HG ? kPackedV : 4 * 64)) * sizeof(T);
};

// Vector of VW elements of T (one 16-byte global access per lane when
// VW * sizeof(T) = 16).
template <typename T, int VW>
struct Vec {
  typedef T type __attribute__((ext_vector_type(VW)));
};
template <typename T>
struct Vec<T, 1> {
  typedef T type;
};

template <typename T, int VW>
__device__ inline T vget(const typename Vec<T, VW>::type& v, int i) {
  if constexpr (VW == 1) {
    return v;
  } else {
    return v[i];
  }
}

template <typename T, int VW>
__device__ inline void vset(typename Vec<T, VW>::type& v, int i, T x) {
  if constexpr (VW == 1) {
    v = x;
  } else {
    v[i] = x;
  }
}

// Launch shape per size class (measured on MI355X):
//  * FP32, NB = 5 (d = 65..80): one wave per row block with the neighbour
//    sums X_s accumulated in LDS, at most 128 VGPRs: two 5-wave workgroups
//    (2 x 79 KB of LDS) share a CU and overlap their phases.
//  * otherwise two waves per row block for 4 <= NB <= 6 (accumulators and
//    neighbour registers of a wave fit three waves per SIMD, so a 2 NB-wave
//    workgroup spreads over the four SIMDs), one below.
//  * FP64 always accumulates X_s in LDS (its register form spills).
template <typename T, int NB>
constexpr int wpr_of() {
  if (sizeof(T) == 4 && NB == 5) return 1;
  return (NB >= 4 && NB <= 6) ? 2 : 1;
}
template <typename T, int NB>
constexpr bool x_in_lds() {
  return sizeof(T) == 8 || NB == 5;
}
// minimum waves per SIMD requested from the register allocator
template <typename T, int NB, bool XL = x_in_lds<T, NB>()>
constexpr int minw_of() {
  if (wpr_of<T, NB>() == 2) return 3;
  if (sizeof(T) == 4) return XL ? 4 : 2;
  return 1;
}

// Vectors of a neighbour slab whose loads are issued together before they
// are used (FP32 keeps three in flight within its 128-VGPR budget; FP64,
// with more registers, the whole slab); 0: slabs of more than five vectors
// (d > 96) keep the per-vector loop, their kernels already spill.
template <typename T, int RV>
constexpr int gather_group() {
  if (RV > 5) return 0;
  return sizeof(T) == 4 ? (RV < 3 ? RV : 3) : RV;
}

// Stages H (zero padded to DP x DP), the single-mode operators v_s and zero
// padding of the rho planes into LDS.
template <typename T, int NB, typename Shape, bool HG = false>
__device__ inline void stage_operators(const DevOps<T>& op, const Shape& sh, const T* __restrict__ Hp, T* sRe,
                                       T* sH, T* sV) {
  using L = Lds<T, NB, HG>;
  constexpr int DP = L::DP, LD = L::LD, NT = NB * 64 * wpr_of<T, NB>();
  if constexpr (!HG) {
    for (int e = threadIdx.x; e < DP * DP; e += NT) {
      const int r = e / DP, c = e - (e / DP) * DP;
      sH[r * LD + c] = Hp[e];
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (s >= sh.nm()) break;
    const int ds2 = sh.dim(s) * sh.dim(s);
    for (int e = threadIdx.x; e < ds2; e += NT) sV[(HG ? op.v_off[s] : s * 64) + e] = op.v[op.v_off[s] + e];
  }
  // only the d x d block of the rho planes is rewritten per matrix
  for (int e = threadIdx.x; e < 2 * L::PLANE; e += NT) sRe[e] = T(0);
}

// out = y + coef * L(in) (y may be null: out = L(in)) for matrix `item` of a
// hierarchy batch whose trajectories start at `in`, `y`, `out`; H and v_s are
// already in LDS.  The workgroup has NB * WPR waves: for the matrix-core and
// contraction work wave w owns row block w / WPR and the column tiles
// [ (w % WPR) JT, ... ) (JT = ceil(NB / WPR)); for the memory phases
// (neighbour sums, epilogue) it owns the slab of 16 / WPR rows starting at
// row (16 / WPR) w.
template <typename T, int NB, typename Shape, int VW, int WPR, bool XL = x_in_lds<T, NB>(), bool HG = false>
__device__ __forceinline__ void rhs_item(const DevOps<T>& op, const Shape& sh, const T* __restrict__ in,
                                         const T* y, T* out, T coef, long long item, T* sRe, T* sIm,
                                         const T* sH, const T* sV) {
  using L = Lds<T, NB>;
  using M = Mfma<T>;
  using acc_t = typename M::acc;
  using vec_t = typename Vec<T, VW>::type;
  constexpr int DP = L::DP, LD = L::LD;
  // row stride of H: the LDS plane, or the zero-padded DP x DP global copy
  constexpr int HLD = HG ? DP : LD;
  constexpr int NT = NB * 64 * WPR;
  constexpr int JT = (NB + WPR - 1) / WPR;   // column tiles per wave
  constexpr int SR = 16 / WPR;               // slab rows per wave
  // vectors per lane covering a slab of SR rows of DP columns
  constexpr int RV = (SR * DP + VW * 64 - 1) / (VW * 64);
  // 16-byte LDS accesses in the slab phases when the rows are 16-byte aligned
  // (VW elements at a column multiple of VW)
  constexpr bool VL = VW * sizeof(T) == 16 && (LD * sizeof(T)) % 16 == 0;
  const int d = sh.d();
  const long long dd = static_cast<long long>(d) * d;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int rows0 = 16 * (wave / WPR);       // row block (matrix-core phases)
  const int j0 = (wave % WPR) * JT;          // first column tile
  const int srow0 = SR * wave;               // slab (memory phases)
  const int sb_rows = srow0 < d ? (d - srow0 < SR ? d - srow0 : SR) : 0;
  const int sb_elems = sb_rows * d;
  (void)DP;
  // Per-lane index arithmetic is redone for every item: an opaque copy of
  // the lane id keeps the compiler from hoisting hundreds of LDS addresses
  // of the unrolled loops out of the item loop (register pressure).
  int lane_v = lane;
  asm volatile("" : "+v"(lane_v));
  const int lr = lane_v & 15;
  const int lq = lane_v >> 4;
  const int n = static_cast<int>(item % op.n_ado);
  const long long base = item * 2 * dd;
  const long long traj_base = (item - n) * 2 * dd;
  const T* rin = in + base;

  __syncthreads();  // previous item's LDS reads are complete
  // ---- stage rho_n: 16-byte loads, d x d block of the LDS planes -------
  for (int v = threadIdx.x; v * VW < dd; v += NT) {
    const vec_t xr = *reinterpret_cast<const vec_t*>(rin + static_cast<long long>(v) * VW);
    const vec_t xi = *reinterpret_cast<const vec_t*>(rin + dd + static_cast<long long>(v) * VW);
    const int e = v * VW, r = e / d, c = e - (e / d) * d;
    if constexpr (VL) {
      *reinterpret_cast<vec_t*>(&sRe[r * LD + c]) = xr;
      *reinterpret_cast<vec_t*>(&sIm[r * LD + c]) = xi;
    } else {
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        sRe[r * LD + c + i] = vget<T, VW>(xr, i);
        sIm[r * LD + c + i] = vget<T, VW>(xi, i);
      }
    }
  }
  __syncthreads();

  // ---- H commutator of row block / column tiles -------------------------
  //   Re L += H Im - Im H,   Im L += Re H - H Re
  acc_t Rre[JT], Rim[JT];
#pragma unroll
  for (int jj = 0; jj < JT; ++jj) {
    Rre[jj] = acc_t{0, 0, 0, 0};
    Rim[jj] = acc_t{0, 0, 0, 0};
  }
  if constexpr (sizeof(T) == 4 && WPR == 2 && (LD % 4) == 0) {
    // k = 16 blk + 4 lq + t: each lane's four k of a block are contiguous, so
    // the A operands (rows of H, Re, Im) and H[k][col] = H[col][k] (H is
    // symmetric) come from 16-byte LDS reads (FP32 with two waves per row
    // block: d = 64 measured 140.0 -> 134.4 ms per launch; the one-wave
    // shape of d = 80 gained nothing and keeps the loop below)
    using v4 = typename Vec<T, 4>::type;
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
      const int kb = 16 * blk + 4 * lq;
      const v4 hA4 = *reinterpret_cast<const v4*>(&sH[(rows0 + lr) * HLD + kb]);
      const v4 aRe4 = *reinterpret_cast<const v4*>(&sRe[(rows0 + lr) * LD + kb]);
      const v4 aIm4 = *reinterpret_cast<const v4*>(&sIm[(rows0 + lr) * LD + kb]);
      v4 hB4[JT];
#pragma unroll
      for (int jj = 0; jj < JT; ++jj)
        if (j0 + jj < NB) hB4[jj] = *reinterpret_cast<const v4*>(&sH[(16 * (j0 + jj) + lr) * HLD + kb]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = kb + t;
        const T hA = hA4[t], nhA = -hA4[t], aRe = aRe4[t], naIm = -aIm4[t];
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
          if (j0 + jj < NB) {
            const int j = j0 + jj;
            const T hB = hB4[jj][t];
            Rre[jj] = M::mma(hA, sIm[k * LD + 16 * j + lr], Rre[jj]);
            Rre[jj] = M::mma(naIm, hB, Rre[jj]);
            Rim[jj] = M::mma(nhA, sRe[k * LD + 16 * j + lr], Rim[jj]);
            Rim[jj] = M::mma(aRe, hB, Rim[jj]);
          }
        }
      }
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < 4 * NB; ++kk) {
      const int k = 4 * kk + lq;
      const T hA = sH[(rows0 + lr) * HLD + k];
      const T nhA = -hA;
      const T aRe = sRe[(rows0 + lr) * LD + k];
      const T naIm = -sIm[(rows0 + lr) * LD + k];
#pragma unroll
      for (int jj = 0; jj < JT; ++jj) {
        if (j0 + jj < NB) {
          const int j = j0 + jj;
          const T hB = sH[k * HLD + 16 * j + lr];
          Rre[jj] = M::mma(hA, sIm[k * LD + 16 * j + lr], Rre[jj]);
          Rre[jj] = M::mma(naIm, hB, Rre[jj]);
          Rim[jj] = M::mma(nhA, sRe[k * LD + 16 * j + lr], Rim[jj]);
          Rim[jj] = M::mma(aRe, hB, Rim[jj]);
        }
      }
    }
  }
  // damping -(g + i gi) rho; gi != 0 only for complex rates (Brownian baths)
  const T g = op.gamma[n];
  const T gi = op.gamma_im ? op.gamma_im[n] : T(0);
#pragma unroll
  for (int jj = 0; jj < JT; ++jj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = rows0 + M::crow(lq, r), c = 16 * (j0 + jj) + lr;
      if (j0 + jj < NB) {
        Rre[jj][r] -= g * sRe[a * LD + c];
        Rim[jj][r] -= g * sIm[a * LD + c];
        if (gi != T(0)) {
          Rre[jj][r] += gi * sIm[a * LD + c];
          Rim[jj][r] -= gi * sRe[a * LD + c];
        }
      }
    }

  // The neighbour phase (global loads, LDS accumulation, v_s contractions)
  // runs at raised wave priority so that it is issued ahead of the other
  // workgroup's matrix-core phase on the same CU (measured: 1.5-4% per
  // launch); the epilogue drops back to the default.
  __builtin_amdgcn_s_setprio(1);
  // ---- couplings to the hierarchy neighbours ----------------------------
  // Each wave forms X_s (and Y_s) for its slab rows from 16-byte neighbour
  // loads: in registers, staged once per mode in the LDS planes, or
  // accumulated directly in the LDS planes (x_in_lds: FP64, whose register
  // form spills, and the FP32 shape that runs two workgroups per CU).
#pragma unroll 1
  for (int s = 0; s < 4; ++s) {
    if (s >= sh.nm()) break;
    const int p0 = op.nb_ptr[n * op.n_modes + s];
    const int p1 = op.nb_ptr[n * op.n_modes + s + 1];
    if (p0 == p1) continue;  // uniform across the workgroup
    const int ds = sh.dim(s), st = sh.stride(s);
    const T* vs = sV + (HG ? op.v_off[s] : s * 64);
    bool have_w = false;
    if constexpr (XL) {
      __syncthreads();  // every wave is done with the previous LDS content
      for (int q = p0; q < p1; ++q) {
        const T* rm = in + traj_base + static_cast<long long>(op.nb_idx[q]) * 2 * dd + srow0 * d;
        const T ar = op.nb_a[4 * q], ai = op.nb_a[4 * q + 1];
        have_w = have_w || op.nb_a[4 * q + 2] != ar || op.nb_a[4 * q + 3] != ai;
        const bool first = q == p0;
        constexpr int G = gather_group<T, RV>();
        if (G > 0 && sb_elems == RV * 64 * VW) {
          // The slab lies wholly inside the matrix (uniform over the wave):
          // the loads of a group of vectors are issued before their LDS
          // updates, so the memory latency is paid once per group.  (With the
          // per-vector bounds test below each load stays next to its use and
          // every vector costs a full round trip: d = 80 measured 93.4 ->
          // 86.8 ms per launch in FP32, 42.2 -> 39.0 ms in FP64.)
          constexpr int GS = G > 0 ? G : 1;
#pragma unroll
          for (int k0 = 0; k0 < RV; k0 += GS) {
            vec_t gr[GS], gi[GS];
#pragma unroll
            for (int k = k0; k < k0 + GS && k < RV; ++k) {
              const int e = (lane + 64 * k) * VW;
              gr[k - k0] = *reinterpret_cast<const vec_t*>(rm + e);
              gi[k - k0] = *reinterpret_cast<const vec_t*>(rm + dd + e);
            }
#pragma unroll
            for (int k = k0; k < k0 + GS && k < RV; ++k) {
              const int e = (lane + 64 * k) * VW;
              const int r = srow0 + e / d, c = e - (e / d) * d;
              const vec_t br = gr[k - k0], bi = gi[k - k0];
              const vec_t xr_ = ar * br - ai * bi;
              const vec_t xi_ = ar * bi + ai * br;
              if constexpr (VL) {
                vec_t* pr = reinterpret_cast<vec_t*>(&sRe[r * LD + c]);
                vec_t* pi = reinterpret_cast<vec_t*>(&sIm[r * LD + c]);
                if (first) {
                  *pr = xr_;
                  *pi = xi_;
                } else {
                  *pr += xr_;
                  *pi += xi_;
                }
              } else {
#pragma unroll
                for (int i = 0; i < VW; ++i) {
                  if (first) {
                    sRe[r * LD + c + i] = vget<T, VW>(xr_, i);
                    sIm[r * LD + c + i] = vget<T, VW>(xi_, i);
                  } else {
                    sRe[r * LD + c + i] += vget<T, VW>(xr_, i);
                    sIm[r * LD + c + i] += vget<T, VW>(xi_, i);
                  }
                }
              }
            }
          }
          continue;
        }
#pragma unroll
        for (int k = 0; k < RV; ++k) {
          const int e = (lane + 64 * k) * VW;
          if (e < sb_elems) {
            const vec_t br = *reinterpret_cast<const vec_t*>(rm + e);
            const vec_t bi = *reinterpret_cast<const vec_t*>(rm + dd + e);
            const int r = srow0 + e / d, c = e - (e / d) * d;
            if constexpr (VL) {
              vec_t* pr = reinterpret_cast<vec_t*>(&sRe[r * LD + c]);
              vec_t* pi = reinterpret_cast<vec_t*>(&sIm[r * LD + c]);
              const vec_t xr_ = ar * br - ai * bi;
              const vec_t xi_ = ar * bi + ai * br;
              if (first) {
                *pr = xr_;
                *pi = xi_;
              } else {
                *pr += xr_;
                *pi += xi_;
              }
            } else {
#pragma unroll
              for (int i = 0; i < VW; ++i) {
                const T xr_ = ar * vget<T, VW>(br, i) - ai * vget<T, VW>(bi, i);
                const T xi_ = ar * vget<T, VW>(bi, i) + ai * vget<T, VW>(br, i);
                if (first) {
                  sRe[r * LD + c + i] = xr_;
                  sIm[r * LD + c + i] = xi_;
                } else {
                  sRe[r * LD + c + i] += xr_;
                  sIm[r * LD + c + i] += xi_;
                }
              }
            }
          }
        }
      }
      __syncthreads();
    } else {
      vec_t xr[RV], xi[RV], wr[RV], wi[RV];
#pragma unroll
      for (int k = 0; k < RV; ++k) {
#pragma unroll
        for (int i = 0; i < VW; ++i) {
          vset<T, VW>(xr[k], i, T(0));
          vset<T, VW>(xi[k], i, T(0));
          vset<T, VW>(wr[k], i, T(0));
          vset<T, VW>(wi[k], i, T(0));
        }
      }
      for (int q = p0; q < p1; ++q) {
        const T* rm = in + traj_base + static_cast<long long>(op.nb_idx[q]) * 2 * dd + srow0 * d;
        const T ar = op.nb_a[4 * q], ai = op.nb_a[4 * q + 1];
        // W accumulates Y_s - X_s = sum_q (aR_q - aL_q) rho_q
        const T dr = op.nb_a[4 * q + 2] - ar, di = op.nb_a[4 * q + 3] - ai;
        const bool cplx = dr != T(0) || di != T(0);
        have_w = have_w || cplx;
        if (gather_group<T, RV>() > 0 && sb_elems == RV * 64 * VW) {
          // whole slab inside the matrix: its loads first (as above)
          vec_t gr[RV], gi[RV];
#pragma unroll
          for (int k = 0; k < RV; ++k) {
            const int e = (lane + 64 * k) * VW;
            gr[k] = *reinterpret_cast<const vec_t*>(rm + e);
            gi[k] = *reinterpret_cast<const vec_t*>(rm + dd + e);
          }
#pragma unroll
          for (int k = 0; k < RV; ++k) {
            xr[k] += ar * gr[k] - ai * gi[k];
            xi[k] += ar * gi[k] + ai * gr[k];
            if (cplx) {
              wr[k] += dr * gr[k] - di * gi[k];
              wi[k] += dr * gi[k] + di * gr[k];
            }
          }
          continue;
        }
#pragma unroll
        for (int k = 0; k < RV; ++k) {
          const int e = (lane + 64 * k) * VW;
          if (e < sb_elems) {
            const vec_t br = *reinterpret_cast<const vec_t*>(rm + e);
            const vec_t bi = *reinterpret_cast<const vec_t*>(rm + dd + e);
            xr[k] += ar * br - ai * bi;
            xi[k] += ar * bi + ai * br;
            if (cplx) {
              wr[k] += dr * br - di * bi;
              wi[k] += dr * bi + di * br;
            }
          }
        }
      }
      __syncthreads();  // every wave is done with the previous LDS content
#pragma unroll
      for (int k = 0; k < RV; ++k) {
        const int e = (lane + 64 * k) * VW;
        if (e < sb_elems) {
          const int r = srow0 + e / d, c = e - (e / d) * d;
          if constexpr (VL) {
            *reinterpret_cast<vec_t*>(&sRe[r * LD + c]) = xr[k];
            *reinterpret_cast<vec_t*>(&sIm[r * LD + c]) = xi[k];
          } else {
#pragma unroll
            for (int i = 0; i < VW; ++i) {
              sRe[r * LD + c + i] = vget<T, VW>(xr[k], i);
              sIm[r * LD + c + i] = vget<T, VW>(xi[k], i);
            }
          }
        }
      }
      __syncthreads();
      // left product below; Y_s = X_s - 2i W afterwards from the registers
      {
        int as[4], r0[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = rows0 + M::crow(lq, r);
          as[r] = (a / st) % ds;
          r0[r] = a - as[r] * st;
        }
        for (int k = 0; k < ds; ++k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const T v = vs[as[r] * ds + k];
            const int rowoff = (r0[r] + k * st) * LD + lr;
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
              if (j0 + jj < NB) {
                Rre[jj][r] += v * sIm[rowoff + 16 * (j0 + jj)];
                Rim[jj][r] -= v * sRe[rowoff + 16 * (j0 + jj)];
              }
            }
          }
        }
      }
      __syncthreads();  // left products read other waves' rows
      if (have_w) {
#pragma unroll
        for (int k = 0; k < RV; ++k) {
          const int e = (lane + 64 * k) * VW;
          if (e < sb_elems) {
            const int r = srow0 + e / d, c = e - (e / d) * d;
            if constexpr (VL) {
              *reinterpret_cast<vec_t*>(&sRe[r * LD + c]) = xr[k] + wr[k];
              *reinterpret_cast<vec_t*>(&sIm[r * LD + c]) = xi[k] + wi[k];
            } else {
#pragma unroll
              for (int i = 0; i < VW; ++i) {
                sRe[r * LD + c + i] = vget<T, VW>(xr[k], i) + vget<T, VW>(wr[k], i);
                sIm[r * LD + c + i] = vget<T, VW>(xi[k], i) + vget<T, VW>(wi[k], i);
              }
            }
          }
        }
      }
      __syncthreads();
    }
    if constexpr (XL) {
      // left product: (V_s X_s)[a][c] = sum_k v_s[a_s][k] X_s[a + (k - a_s) st][c];  L += -i V X
      {
        int as[4], r0[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = rows0 + M::crow(lq, r);
          as[r] = (a / st) % ds;
          r0[r] = a - as[r] * st;
        }
        for (int k = 0; k < ds; ++k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const T v = vs[as[r] * ds + k];
            const int rowoff = (r0[r] + k * st) * LD + lr;
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
              if (j0 + jj < NB) {
                Rre[jj][r] += v * sIm[rowoff + 16 * (j0 + jj)];
                Rim[jj][r] -= v * sRe[rowoff + 16 * (j0 + jj)];
              }
            }
          }
        }
      }
      // Y_s = X_s + sum_q (aR_q - aL_q) rho_q on the slab rows: a second
      // pass over the neighbours whose bra coefficient differs
      if (have_w) {
        __syncthreads();  // left products read other waves' rows
        for (int q = p0; q < p1; ++q) {
          const T dr = op.nb_a[4 * q + 2] - op.nb_a[4 * q], di = op.nb_a[4 * q + 3] - op.nb_a[4 * q + 1];
          if (dr == T(0) && di == T(0)) continue;
          const T* rm = in + traj_base + static_cast<long long>(op.nb_idx[q]) * 2 * dd + srow0 * d;
#pragma unroll
          for (int k = 0; k < RV; ++k) {
            const int e = (lane + 64 * k) * VW;
            if (e < sb_elems) {
              const vec_t br = *reinterpret_cast<const vec_t*>(rm + e);
              const vec_t bi = *reinterpret_cast<const vec_t*>(rm + dd + e);
              const int r = srow0 + e / d, c = e - (e / d) * d;
              if constexpr (VL) {
                *reinterpret_cast<vec_t*>(&sRe[r * LD + c]) += dr * br - di * bi;
                *reinterpret_cast<vec_t*>(&sIm[r * LD + c]) += dr * bi + di * br;
              } else {
#pragma unroll
                for (int i = 0; i < VW; ++i) {
                  sRe[r * LD + c + i] += dr * vget<T, VW>(br, i) - di * vget<T, VW>(bi, i);
                  sIm[r * LD + c + i] += dr * vget<T, VW>(bi, i) + di * vget<T, VW>(br, i);
                }
              }
            }
          }
        }
      }
      __syncthreads();
    }
    // right product: (Y_s V_s)[a][c] = sum_k Y_s[a][c + (k - c_s) st] v_s[k][c_s];  L += i Y V
    {
      int cs[JT], c0[JT];
#pragma unroll
      for (int jj = 0; jj < JT; ++jj) {
        const int c = 16 * (j0 + jj) + lr;
        cs[jj] = (c / st) % ds;
        c0[jj] = c - cs[jj] * st;
      }
      for (int k = 0; k < ds; ++k) {
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
          if (j0 + jj < NB) {
            const T v = vs[k * ds + cs[jj]];
            const int coloff = c0[jj] + k * st;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int a = rows0 + M::crow(lq, r);
              Rre[jj][r] -= v * sIm[a * LD + coloff];
              Rim[jj][r] += v * sRe[a * LD + coloff];
            }
          }
        }
      }
    }
  }

  __builtin_amdgcn_s_setprio(0);
  // ---- epilogue: out = y + coef * L ---------------------------------------
  // transpose the accumulators through LDS so that y and out move in
  // 16-byte vectors (slab rows).  Only the d x d block is written: the
  // padding rows and columns of the planes must stay zero (the matrix-core
  // products multiply them by the zero padding of H, and the accumulators
  // there hold contraction and damping terms of padding entries that would
  // otherwise feed back and grow from one matrix to the next).
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < JT; ++jj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = rows0 + M::crow(lq, r), c = 16 * (j0 + jj) + lr;
      if (j0 + jj < NB && a < d && c < d) {
        sRe[a * LD + c] = Rre[jj][r];
        sIm[a * LD + c] = Rim[jj][r];
      }
    }
  __syncthreads();
  {
    const long long ob = base + srow0 * d;
    vec_t yr[RV], yi[RV];
    if (y) {
#pragma unroll
      for (int k = 0; k < RV; ++k) {
        const int e = (lane + 64 * k) * VW;
        if (e < sb_elems) {
          // y and out are streamed (read and written once per launch, 33 GB at
          // the benchmark size): non-temporal accesses leave the caches to the
          // neighbour matrices, which are read up to 2M times
          yr[k] = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(y + ob + e));
          yi[k] = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(y + ob + dd + e));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < RV; ++k) {
      const int e = (lane + 64 * k) * VW;
      if (e < sb_elems) {
        const int r = srow0 + e / d, c = e - (e / d) * d;
        vec_t orr, oi;
        if constexpr (VL) {
          orr = *reinterpret_cast<const vec_t*>(&sRe[r * LD + c]);
          oi = *reinterpret_cast<const vec_t*>(&sIm[r * LD + c]);
          if (y) {
            orr = yr[k] + coef * orr;
            oi = yi[k] + coef * oi;
          }
        } else {
#pragma unroll
          for (int i = 0; i < VW; ++i) {
            T lre = sRe[r * LD + c + i], lim = sIm[r * LD + c + i];
            if (y) {
              lre = vget<T, VW>(yr[k], i) + coef * lre;
              lim = vget<T, VW>(yi[k], i) + coef * lim;
            }
            vset<T, VW>(orr, i, lre);
            vset<T, VW>(oi, i, lim);
          }
        }
        __builtin_nontemporal_store(orr, reinterpret_cast<vec_t*>(out + ob + e));
        __builtin_nontemporal_store(oi, reinterpret_cast<vec_t*>(out + ob + dd + e));
      }
    }
  }
}

template <typename T, int NB, typename Shape, int MINW, int VW>
__global__ __launch_bounds__((NB * 64 * wpr_of<T, NB>()), MINW) void rhs_mfma_kernel(DevOps<T> op, const T* __restrict__ Hp,
                                                                 const T* __restrict__ in, const T* y, T* out,
                                                                 T coef, long long n_items) {
  using L = Lds<T, NB>;
  extern __shared__ unsigned char smem_raw[];
  T* sRe = reinterpret_cast<T*>(smem_raw);
  T* sIm = sRe + L::PLANE;
  T* sH = sRe + L::HOFF;
  T* sV = sRe + L::VOFF;
  const Shape sh(op.dims, op.strides, op.n_modes, op.d);
  stage_operators<T, NB, Shape>(op, sh, Hp, sRe, sH, sV);
  for (long long item = blockIdx.x; item < n_items; item += gridDim.x)
    rhs_item<T, NB, Shape, VW, wpr_of<T, NB>()>(op, sh, in, y, out, coef, item, sRe, sIm, sH, sV);
}

// rhs_mfma_kernel with H read from its zero-padded global copy (L1 / L2
// resident, 25.6 KB at d = 80 in FP32) and the v_s packed, for the LDS of
// three workgroups per CU.
template <typename T, int NB, typename Shape, int MINW, int VW>
__global__ __launch_bounds__((NB * 64 * wpr_of<T, NB>()), MINW) void rhs_mfma_gh_kernel(DevOps<T> op,
                                                                                       const T* __restrict__ Hp,
                                                                                       const T* __restrict__ in,
                                                                                       const T* y, T* out, T coef,
                                                                                       long long n_items) {
  using L = Lds<T, NB, true>;
  extern __shared__ unsigned char smem_raw[];
  T* sRe = reinterpret_cast<T*>(smem_raw);
  T* sIm = sRe + L::PLANE;
  T* sV = sRe + L::VOFF;
  const Shape sh(op.dims, op.strides, op.n_modes, op.d);
  stage_operators<T, NB, Shape, true>(op, sh, Hp, sRe, nullptr, sV);
  for (long long item = blockIdx.x; item < n_items; item += gridDim.x)
    rhs_item<T, NB, Shape, VW, wpr_of<T, NB>(), x_in_lds<T, NB>(), true>(op, sh, in, y, out, coef, item, sRe, sIm,
                                                                         Hp, sV);
}

// Several model instances of one size class (same ceil(d/16)) in one
// persistent launch.  Instance i owns items [desc[i].item_begin,
// desc[i+1].item_begin).  A workgroup re-stages H and v_s whenever the
// instance of its next item differs from the previous one.
template <typename T, int NB, int MINW, int VW, bool XL>
__global__ __launch_bounds__((NB * 64 * wpr_of<T, NB>()), MINW) void rhs_mfma_multi_kernel(const InstDesc<T>* __restrict__ desc,
                                                                       int n_inst, T coef, long long n_items) {
  using L = Lds<T, NB>;
  extern __shared__ unsigned char smem_raw[];
  T* sRe = reinterpret_cast<T*>(smem_raw);
  T* sIm = sRe + L::PLANE;
  T* sH = sRe + L::HOFF;
  T* sV = sRe + L::VOFF;
  int cur = -1;
  for (long long item = blockIdx.x; item < n_items; item += gridDim.x) {
    int lo = 0, hi = n_inst - 1;  // last instance with item_begin <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (desc[mid].item_begin <= item) lo = mid;
      else hi = mid - 1;
    }
    const InstDesc<T>& di = desc[lo];
    const DynShape sh(di.op.dims, di.op.strides, di.op.n_modes, di.op.d);
    if (lo != cur) {
      __syncthreads();  // previous instance's LDS reads are complete
      stage_operators<T, NB, DynShape>(di.op, sh, di.Hp, sRe, sH, sV);
      cur = lo;
    }
    rhs_item<T, NB, DynShape, VW, wpr_of<T, NB>(), XL>(di.op, sh, di.in, di.y, di.out, coef, item - di.item_begin,
                                                      sRe, sIm, sH, sV);
  }
}

// ------------------------------------------------ one launch, all classes --
// Several size classes in one persistent launch.  Workgroups
// [cls[c].wg_begin, cls[c].wg_end) serve class c; a workgroup has W waves,
// the widest class's count, and the waves a narrower class does not use end
// at entry (a workgroup barrier waits only for the waves still running).
// Each class runs the item code of its own NB, with the neighbour sums X_s in
// LDS (fewer registers: one register budget serves every class).
template <typename T>
__host__ __device__ constexpr int class_waves(int nb) {
  return nb * ((sizeof(T) == 4 && nb == 5) ? 1 : (nb >= 4 && nb <= 6) ? 2 : 1);
}

template <typename T, int NB, int VW>
__device__ __forceinline__ void fused_items(const FusedClass& fc, const InstDesc<T>* __restrict__ desc, T coef,
                                            unsigned char* smem) {
  using L = Lds<T, NB>;
  T* sRe = reinterpret_cast<T*>(smem);
  T* sIm = sRe + L::PLANE;
  T* sH = sRe + L::HOFF;
  T* sV = sRe + L::VOFF;
  const InstDesc<T>* dc = desc + fc.inst_first;
  const long long step = fc.wg_end - fc.wg_begin;
  int cur = -1;
  for (long long item = static_cast<long long>(blockIdx.x) - fc.wg_begin; item < fc.n_items; item += step) {
    int lo = 0, hi = fc.n_inst - 1;  // last instance of the class with item_begin <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (dc[mid].item_begin <= item) lo = mid;
      else hi = mid - 1;
    }
    const InstDesc<T>& di = dc[lo];
    const DynShape sh(di.op.dims, di.op.strides, di.op.n_modes, di.op.d);
    if (lo != cur) {
      __syncthreads();  // previous instance's LDS reads are complete
      stage_operators<T, NB, DynShape>(di.op, sh, di.Hp, sRe, sH, sV);
      cur = lo;
    }
    rhs_item<T, NB, DynShape, VW, wpr_of<T, NB>(), true>(di.op, sh, di.in, di.y, di.out, coef,
                                                        item - di.item_begin, sRe, sIm, sH, sV);
  }
}

template <typename T, int W, int NB>
__device__ __forceinline__ void fused_dispatch(const FusedClass& fc, const InstDesc<T>* desc, T coef,
                                               unsigned char* smem) {
  if constexpr (NB <= kFusedMaxNb) {
    if (fc.nb == NB) {
      if constexpr (class_waves<T>(NB) <= W) {
        constexpr int VF = 16 / sizeof(T);
        if (fc.vw == VF) fused_items<T, NB, VF>(fc, desc, coef, smem);
        else fused_items<T, NB, 1>(fc, desc, coef, smem);
      }
      return;
    }
    fused_dispatch<T, W, NB + 1>(fc, desc, coef, smem);
  }
}

// at most 128 VGPRs in FP32 (two workgroups of up to 8 waves per CU), 168 in
// FP64 (one 10-wave workgroup per CU)
template <typename T>
constexpr int fused_minw() {
  return sizeof(T) == 4 ? 4 : 3;
}

template <typename T, int W>
__global__ __launch_bounds__(W * 64, fused_minw<T>()) void rhs_mfma_fused_kernel(const FusedClass* __restrict__ cls,
                                                                                int n_cls,
                                                                                const InstDesc<T>* __restrict__ desc,
                                                                                T coef) {
  extern __shared__ unsigned char smem_raw[];
  const int b = static_cast<int>(blockIdx.x);
  int c = 0;
  while (c + 1 < n_cls && b >= cls[c].wg_end) ++c;
  const FusedClass fc = cls[c];
  if (b < fc.wg_begin || b >= fc.wg_end) return;
  if (static_cast<int>(threadIdx.x >> 6) >= class_waves<T>(fc.nb)) return;
  fused_dispatch<T, W, 1>(fc, desc, coef, smem_raw);
}

template <typename T, int NB, typename Shape, int VW>
void launch_shape_vw(const DevOps<T>& op, const T* Hp, const T* in, const T* y, T* out, T coef, long long n_items,
                     int wg_per_cu, hipStream_t stream) {
  const size_t lds = Lds<T, NB>::bytes;
  constexpr int MINW = minw_of<T, NB>();
  auto kern = &rhs_mfma_kernel<T, NB, Shape, MINW, VW>;
  static bool configured = false;
  if (!configured) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
    configured = true;
  }
  int fit = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void*>(kern),
                                                   NB * 64 * wpr_of<T, NB>(), lds) == hipSuccess &&
      fit > 0 && fit < wg_per_cu)
    wg_per_cu = fit;
  long long grid = static_cast<long long>(cu_count()) * wg_per_cu;
  if (grid > n_items) grid = n_items;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(NB * 64 * wpr_of<T, NB>()), lds, stream, op, Hp,
                     in, y, out, coef,
                     n_items);
}

// 16-byte vectors when every row starts on a 16-byte boundary
template <typename T, int NB, typename Shape>
void launch_shape(const DevOps<T>& op, const T* Hp, const T* in, const T* y, T* out, T coef, long long n_items,
                  int wg_per_cu, hipStream_t stream) {
  constexpr int VW = 16 / sizeof(T);
  if (op.d % VW == 0)
    launch_shape_vw<T, NB, Shape, VW>(op, Hp, in, y, out, coef, n_items, wg_per_cu, stream);
  else
    launch_shape_vw<T, NB, Shape, 1>(op, Hp, in, y, out, coef, n_items, wg_per_cu, stream);
}

template <typename T, int NB>
void launch_dyn(const DevOps<T>& op, const T* Hp, const T* in, const T* y, T* out, T coef, long long n_items,
                int wg_per_cu, hipStream_t stream) {
  launch_shape<T, NB, DynShape>(op, Hp, in, y, out, coef, n_items, wg_per_cu, stream);
}

}  // namespace

namespace {

template <typename T, int VW>
void launch_gh_vw(const DevOps<T>& op, const T* Hp, const T* in, const T* y, T* out, T coef, long long n_items,
                  hipStream_t stream) {
  constexpr int NB = 5;
  const size_t lds = Lds<T, NB, true>::bytes;
  auto kern = &rhs_mfma_gh_kernel<T, NB, DynShape, minw_of<T, NB>(), VW>;
  static bool configured = false;
  if (!configured) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
    configured = true;
  }
  int wg = static_cast<int>((160 * 1024) / lds);
  int fit = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void*>(kern),
                                                   NB * 64 * wpr_of<T, NB>(), lds) == hipSuccess &&
      fit > 0 && fit < wg)
    wg = fit;
  if (wg < 1) wg = 1;
  long long grid = static_cast<long long>(cu_count()) * wg;
  if (grid > n_items) grid = n_items;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(NB * 64 * wpr_of<T, NB>()), lds, stream, op, Hp,
                     in, y, out, coef, n_items);
}

}  // namespace

template <typename T>
bool mfma_gh_supported(int d, int n_modes, const int* dims) {
  if (sizeof(T) != 4 || (d + 15) / 16 != 5 || !mfma_supported<T>(d, n_modes, dims)) return false;
  int nv = 0;
  for (int s = 0; s < n_modes; ++s) nv += dims[s] * dims[s];
  return nv <= kPackedV;
}

template <typename T>
void launch_rhs_mfma_gh(const DevOps<T>& op, const T* Hp, const T* in, const T* y, T* out, double coef, int n_traj,
                        hipStream_t stream) {
  const long long n_items = static_cast<long long>(n_traj) * op.n_ado;
  if (n_items == 0) return;
  if (!mfma_gh_supported<T>(op.d, op.n_modes, op.dims))
    throw std::runtime_error("the H-from-global matrix-core kernel needs FP32, d in 65..80 and packed v_s <= 128");
  if constexpr (sizeof(T) == 4) {
    const T c = static_cast<T>(coef);
    if (op.d % 4 == 0) launch_gh_vw<T, 4>(op, Hp, in, y, out, c, n_items, stream);
    else launch_gh_vw<T, 1>(op, Hp, in, y, out, c, n_items, stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("mfma gh kernel: ") + hipGetErrorString(e));
}

template <typename T>
bool mfma_supported(int d, int n_modes, const int* dims) {
  if (d < 1 || d > 128) return false;
  // v_s is staged in a fixed slot of 64 values per mode (Lds::VOFF): at most
  // four modes of at most 8 kept levels each
  if (n_modes < 1 || n_modes > 4) return false;
  for (int s = 0; s < n_modes; ++s)
    if (dims[s] < 1 || dims[s] > 8) return false;
  const int NB = (d + 15) / 16;
  const size_t DP = 16 * NB;
  const size_t lds = (3 * DP * (DP + lds_pad(sizeof(T), NB)) + 4 * 64) * sizeof(T);
  return lds <= 160 * 1024;
}

template <typename T>
bool mfma_static_shape(const DevOps<T>& op) {
  return (sizeof(T) == 8 && StaticShape<3, 4, 4, 5>::matches(op.n_modes, op.dims, op.strides)) ||
         StaticShape<1, 6>::matches(op.n_modes, op.dims, op.strides);
}

template <typename T>
void launch_rhs_mfma(const DevOps<T>& op, const T* Hp, const T* in, const T* y, T* out, double coef, int n_traj,
                     int variant, hipStream_t stream) {
  const long long n_items = static_cast<long long>(n_traj) * op.n_ado;
  if (n_items == 0) return;
  const T c = static_cast<T>(coef);
  // persistent grid: as many workgroups per CU as fit in LDS (160 KB)
  const size_t DP = 16 * ((op.d + 15) / 16);
  const size_t lds = (3 * DP * (DP + lds_pad(sizeof(T), (op.d + 15) / 16)) + 4 * 64) * sizeof(T);
  int wg = static_cast<int>((160 * 1024) / lds);
  if (wg < 1) wg = 1;
  if (wg > 8) wg = 8;
  const bool specialised = variant != 1;
  // compile-time shapes where they measured faster than the runtime shape
  // (MI355X): (4,4,5) in FP64 and (6).  The runtime shape keeps fewer
  // registers live and won for (4,4,5) in FP32 (101.0 vs 103.8 ms per launch
  // at 128 trajectories) and for (5,5) in both precisions (FP32 15.0 vs
  // 22.7 ms at 2048 trajectories, FP64 7.5 vs 12.6 ms at 512).
  if (specialised && sizeof(T) == 8 && StaticShape<3, 4, 4, 5>::matches(op.n_modes, op.dims, op.strides)) {
    launch_shape<T, 5, StaticShape<3, 4, 4, 5>>(op, Hp, in, y, out, c, n_items, wg, stream);
  } else if (specialised && StaticShape<1, 6>::matches(op.n_modes, op.dims, op.strides)) {
    launch_shape<T, 1, StaticShape<1, 6>>(op, Hp, in, y, out, c, n_items, wg, stream);
  } else {
    switch ((op.d + 15) / 16) {
      case 1: launch_dyn<T, 1>(op, Hp, in, y, out, c, n_items, wg, stream); break;
      case 2: launch_dyn<T, 2>(op, Hp, in, y, out, c, n_items, wg, stream); break;
      case 3: launch_dyn<T, 3>(op, Hp, in, y, out, c, n_items, wg, stream); break;
      case 4: launch_dyn<T, 4>(op, Hp, in, y, out, c, n_items, wg, stream); break;
      case 5: launch_dyn<T, 5>(op, Hp, in, y, out, c, n_items, wg, stream); break;
      case 6: launch_dyn<T, 6>(op, Hp, in, y, out, c, n_items, wg, stream); break;
      case 7: launch_dyn<T, 7>(op, Hp, in, y, out, c, n_items, wg, stream); break;
      case 8: launch_dyn<T, 8>(op, Hp, in, y, out, c, n_items, wg, stream); break;
      default: throw std::runtime_error("MFMA RHS kernel supports d <= 128");
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("mfma rhs kernel: ") + hipGetErrorString(e));
}

namespace {

// persistent grid of the per-class launch: the CU count times the
// workgroups per CU that LDS and registers allow (at most 8), or fewer when
// the shape asks for it
template <typename T, int NB, int VW, bool XL>
long long multi_grid_nb(long long n_items, int wg_per_cu) {
  const size_t lds = Lds<T, NB>::bytes;
  auto kern = &rhs_mfma_multi_kernel<T, NB, minw_of<T, NB, XL>(), VW, XL>;
  static bool configured = false;
  if (!configured) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
    configured = true;
  }
  int wg = static_cast<int>((160 * 1024) / lds);
  if (wg < 1) wg = 1;
  if (wg > 8) wg = 8;
  int fit = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void*>(kern),
                                                   NB * 64 * wpr_of<T, NB>(), lds) == hipSuccess &&
      fit > 0 && fit < wg)
    wg = fit;
  if (wg_per_cu > 0 && wg_per_cu < wg) wg = wg_per_cu;
  long long grid = static_cast<long long>(cu_count()) * wg;
  if (grid > n_items) grid = n_items;
  return grid;
}

template <typename T, int NB, int VW, bool XL>
void launch_multi_nb(const InstDesc<T>* desc, int n_inst, T coef, long long n_items, int wg_per_cu,
                     hipStream_t stream) {
  const size_t lds = Lds<T, NB>::bytes;
  auto kern = &rhs_mfma_multi_kernel<T, NB, minw_of<T, NB, XL>(), VW, XL>;
  const long long grid = multi_grid_nb<T, NB, VW, XL>(n_items, wg_per_cu);
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(NB * 64 * wpr_of<T, NB>()), lds, stream, desc,
                     n_inst, coef, n_items);
}

// the alternative neighbour-sum form exists for the FP32 classes whose
// default keeps X_s in registers and whose LDS form the single-launch kernel
// also runs (ceil(d/16) <= 4)
template <typename T, int NB>
constexpr bool has_alt_xl() {
  return sizeof(T) == 4 && NB <= 4;
}

template <typename T, int NB>
bool use_xl(int xl) {
  if constexpr (has_alt_xl<T, NB>()) {
    return xl < 0 ? x_in_lds<T, NB>() : xl != 0;
  } else {
    return x_in_lds<T, NB>();
  }
}

template <typename T, int NB>
void launch_multi_vw(const InstDesc<T>* desc, int n_inst, int vw, T coef, long long n_items, MultiShape shape,
                     hipStream_t stream) {
  constexpr int VF = 16 / sizeof(T);
  constexpr bool DEF = x_in_lds<T, NB>();
  if (has_alt_xl<T, NB>() && use_xl<T, NB>(shape.xl) != DEF) {
    if constexpr (has_alt_xl<T, NB>()) {
      if (vw == VF) launch_multi_nb<T, NB, VF, !DEF>(desc, n_inst, coef, n_items, shape.wg_per_cu, stream);
      else launch_multi_nb<T, NB, 1, !DEF>(desc, n_inst, coef, n_items, shape.wg_per_cu, stream);
    }
    return;
  }
  if (vw == VF) launch_multi_nb<T, NB, VF, DEF>(desc, n_inst, coef, n_items, shape.wg_per_cu, stream);
  else launch_multi_nb<T, NB, 1, DEF>(desc, n_inst, coef, n_items, shape.wg_per_cu, stream);
}

template <typename T, int NB>
long long multi_grid_vw(int vw, long long n_items, MultiShape shape) {
  constexpr int VF = 16 / sizeof(T);
  constexpr bool DEF = x_in_lds<T, NB>();
  if (has_alt_xl<T, NB>() && use_xl<T, NB>(shape.xl) != DEF) {
    if constexpr (has_alt_xl<T, NB>()) {
      return vw == VF ? multi_grid_nb<T, NB, VF, !DEF>(n_items, shape.wg_per_cu)
                      : multi_grid_nb<T, NB, 1, !DEF>(n_items, shape.wg_per_cu);
    }
  }
  return vw == VF ? multi_grid_nb<T, NB, VF, DEF>(n_items, shape.wg_per_cu)
                  : multi_grid_nb<T, NB, 1, DEF>(n_items, shape.wg_per_cu);
}

}  // namespace

template <typename T>
bool multi_has_alt_xl(int nb) {
  switch (nb) {
    case 1: return has_alt_xl<T, 1>();
    case 2: return has_alt_xl<T, 2>();
    case 3: return has_alt_xl<T, 3>();
    case 4: return has_alt_xl<T, 4>();
    default: return false;
  }
}

template <typename T>
long long rhs_mfma_multi_grid(int nb, int vw, long long n_items, MultiShape shape) {
  switch (nb) {
    case 1: return multi_grid_vw<T, 1>(vw, n_items, shape);
    case 2: return multi_grid_vw<T, 2>(vw, n_items, shape);
    case 3: return multi_grid_vw<T, 3>(vw, n_items, shape);
    case 4: return multi_grid_vw<T, 4>(vw, n_items, shape);
    case 5: return multi_grid_vw<T, 5>(vw, n_items, shape);
    case 6: return multi_grid_vw<T, 6>(vw, n_items, shape);
    case 7: return multi_grid_vw<T, 7>(vw, n_items, shape);
    default: throw std::runtime_error("multi-instance MFMA kernel supports ceil(d/16) <= 7");
  }
}

template <typename T>
void launch_rhs_mfma_multi(const InstDesc<T>* desc, int n_inst, int nb, int vw, double coef, long long n_items,
                           hipStream_t stream, MultiShape shape) {
  if (n_items == 0 || n_inst == 0) return;
  const T c = static_cast<T>(coef);
  switch (nb) {
    case 1: launch_multi_vw<T, 1>(desc, n_inst, vw, c, n_items, shape, stream); break;
    case 2: launch_multi_vw<T, 2>(desc, n_inst, vw, c, n_items, shape, stream); break;
    case 3: launch_multi_vw<T, 3>(desc, n_inst, vw, c, n_items, shape, stream); break;
    case 4: launch_multi_vw<T, 4>(desc, n_inst, vw, c, n_items, shape, stream); break;
    case 5: launch_multi_vw<T, 5>(desc, n_inst, vw, c, n_items, shape, stream); break;
    case 6: launch_multi_vw<T, 6>(desc, n_inst, vw, c, n_items, shape, stream); break;
    case 7: launch_multi_vw<T, 7>(desc, n_inst, vw, c, n_items, shape, stream); break;
    default: throw std::runtime_error("multi-instance MFMA kernel supports ceil(d/16) <= 7");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("mfma multi kernel: ") + hipGetErrorString(e));
}

template <typename T>
size_t fused_lds_bytes(int nb) {
  const size_t DP = 16 * static_cast<size_t>(nb);
  return (3 * DP * (DP + lds_pad(sizeof(T), nb)) + 4 * 64) * sizeof(T);
}

namespace {

template <typename T, int W>
void fused_attr_w(size_t lds) {
  static size_t configured = 0;
  if (lds > configured) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&rhs_mfma_fused_kernel<T, W>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
      throw std::runtime_error("fused kernel: LDS attribute");
    configured = lds;
  }
}

template <typename T, int W>
int fused_fit_w(size_t lds) {
  auto kern = &rhs_mfma_fused_kernel<T, W>;
  fused_attr_w<T, W>(lds);
  int fit = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void*>(kern), W * 64, lds) !=
          hipSuccess ||
      fit < 1)
    fit = 1;
  return fit;
}

template <typename T, int W>
void fused_launch_w(const FusedClass* cls, int n_cls, const InstDesc<T>* desc, size_t lds, int grid, T coef,
                    hipStream_t stream) {
  fused_attr_w<T, W>(lds);
  hipLaunchKernelGGL((rhs_mfma_fused_kernel<T, W>), dim3(static_cast<unsigned>(grid)), dim3(W * 64), lds, stream,
                     cls, n_cls, desc, coef);
}

}  // namespace

template <typename T>
int fused_block_waves(const int* nbs, int n) {
  int need = 0;
  for (int i = 0; i < n; ++i) {
    if (nbs[i] < 1 || nbs[i] > kFusedMaxNb) return 0;
    need = std::max(need, class_waves<T>(nbs[i]));
  }
  if (need == 0) return 0;
  if (sizeof(T) == 4) return need <= 5 ? 5 : 8;
  return 10;
}

template <typename T>
int fused_workgroups_per_cu(int waves, size_t lds) {
  if constexpr (sizeof(T) == 4) {
    if (waves == 5) return fused_fit_w<T, 5>(lds);
    if (waves == 8) return fused_fit_w<T, 8>(lds);
  } else {
    if (waves == 10) return fused_fit_w<T, 10>(lds);
  }
  throw std::runtime_error("fused kernel: unsupported block width");
}

template <typename T>
void launch_rhs_mfma_fused(const FusedClass* cls, int n_cls, const InstDesc<T>* desc, int waves, size_t lds,
                           int grid, double coef, hipStream_t stream) {
  if (grid <= 0 || n_cls <= 0) return;
  const T c = static_cast<T>(coef);
  if constexpr (sizeof(T) == 4) {
    if (waves == 5) fused_launch_w<T, 5>(cls, n_cls, desc, lds, grid, c, stream);
    else if (waves == 8) fused_launch_w<T, 8>(cls, n_cls, desc, lds, grid, c, stream);
    else throw std::runtime_error("fused kernel: unsupported block width");
  } else {
    if (waves == 10) fused_launch_w<T, 10>(cls, n_cls, desc, lds, grid, c, stream);
    else throw std::runtime_error("fused kernel: unsupported block width");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("mfma fused kernel: ") + hipGetErrorString(e));
}

template size_t fused_lds_bytes<float>(int);
template size_t fused_lds_bytes<double>(int);
template int fused_block_waves<float>(const int*, int);
template int fused_block_waves<double>(const int*, int);
template int fused_workgroups_per_cu<float>(int, size_t);
template int fused_workgroups_per_cu<double>(int, size_t);
template void launch_rhs_mfma_fused<float>(const FusedClass*, int, const InstDesc<float>*, int, size_t, int, double,
                                           hipStream_t);
template void launch_rhs_mfma_fused<double>(const FusedClass*, int, const InstDesc<double>*, int, size_t, int,
                                            double, hipStream_t);

template bool multi_has_alt_xl<float>(int);
template bool multi_has_alt_xl<double>(int);
template long long rhs_mfma_multi_grid<float>(int, int, long long, MultiShape);
template long long rhs_mfma_multi_grid<double>(int, int, long long, MultiShape);
template void launch_rhs_mfma_multi<float>(const InstDesc<float>*, int, int, int, double, long long, hipStream_t,
                                           MultiShape);
template void launch_rhs_mfma_multi<double>(const InstDesc<double>*, int, int, int, double, long long, hipStream_t,
                                            MultiShape);

template bool mfma_gh_supported<float>(int, int, const int*);
template bool mfma_gh_supported<double>(int, int, const int*);
template void launch_rhs_mfma_gh<float>(const DevOps<float>&, const float*, const float*, const float*, float*,
                                        double, int, hipStream_t);
template bool mfma_static_shape<float>(const DevOps<float>&);
template bool mfma_static_shape<double>(const DevOps<double>&);
template bool mfma_supported<float>(int, int, const int*);
template bool mfma_supported<double>(int, int, const int*);
template void launch_rhs_mfma<float>(const DevOps<float>&, const float*, const float*, const float*, float*,
                                     double, int, int, hipStream_t);
template void launch_rhs_mfma<double>(const DevOps<double>&, const double*, const double*, const double*,
                                      double*, double, int, int, hipStream_t);

}  // namespace heom

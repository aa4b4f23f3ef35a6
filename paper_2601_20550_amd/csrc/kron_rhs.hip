// Fused HEOM right-hand side + RK4 stage for three-mode models whose product
// basis factorises as (S; 4, 4): one slow mode of NB levels and two fast modes
// of 4 levels, in the device basis a = 16 a_S + 4 a_M + a_F (the builder
// reorders the basis so; states are permuted at the host boundary).  Eq.
// HEOM_DB (Sec. II.B) per ADO n:
//
//   L rho = -i (H rho - rho H) - gamma_n rho + sum_s ( [V_s, X_s] - W_s V_s ) (-i),
//   X_s = sum_q aL_q rho_{m_q},   W_s = sum_q (aR_q - aL_q) rho_{m_q},
//
// with V_s = v_s acting on mode s only and the neighbour lists (m_q, aL_q,
// aR_q) of the host tables.
//
// One wave computes one real plane (Re or Im) of one output matrix; the two
// planes of a matrix are independent work items.  The wave owns the whole
// d x d plane as NB x NB matrix-core tiles of the transposed output, so that
//
//   * -i [H, rho] is two real products on v_mfma_f32_16x16x4 per plane,
//     (Re L)^T = Im^T H - H Im^T and (Im L)^T = -(Re^T H - H Re^T), with H
//     (symmetric) in LDS and the rho operands loaded from global memory
//     (k permuted within blocks of 16 so that one operand is a 16-byte load);
//   * every coupling operator contracts registers it already holds: in the
//     accumulator, lane (lq, lr) and register r of tile (I, J) hold
//     L[16 J + lr][16 I + 4 lq + r], so the row digits are (J, lr / 4, lr % 4)
//     and the column digits (I, lq, r).  V_F on rows is a quad broadcast
//     (DPP), V_M on rows a rotation within 16 lanes (DPP), V_S on rows and
//     columns a sum over the wave's own tiles, V_F on columns a sum over the
//     wave's own registers, and V_M on columns a fetch from the other three
//     16-lane rows (ds_bpermute);
//   * neighbour tiles, damping and the RK4 update use 16-byte accesses in the
//     same layout.
//
// No LDS is used for the hierarchy matrices, so a CU holds eight waves (two
// workgroups of four) and the matrix-core phase of one wave overlaps the
// neighbour loads and VALU contractions of the others.
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "kernels.h"

namespace heom {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KRON_WAVES = 4;          // waves per workgroup
constexpr int KRON_WG_PER_CU = 2;

// Loads from a wave-uniform base plus a 32-bit per-lane element offset (the
// base stays in scalar registers; one vector register per address).
__device__ __forceinline__ f32x4 ld16(const float* base, unsigned off) {
  return *reinterpret_cast<const f32x4*>(base + off);
}
__device__ __forceinline__ float ld4(const float* base, unsigned off) { return base[off]; }
__device__ __forceinline__ f32x4 ld16_nt(const float* base, unsigned off) {
  return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(base + off));
}

// value of lane 4 (lane / 4) + k (quad broadcast)
template <int K>
__device__ __forceinline__ float quad_bcast(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), K * 0x55, 0xf, 0xf, true));
}

// value of lane 16 (lane / 16) + (lane - 4 M) mod 16 (rotation within a row of 16)
template <int M>
__device__ __forceinline__ float row_ror4(float x) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x120 + 4 * M, 0xf, 0xf, true));
}

// x of the lane with the same lane % 16 in the row of 16 lanes M rows further
// on (cyclically): lane 16 ((lane / 16 + M) mod 4) + lane % 16.  Through the
// LDS crossbar (ds_bpermute, no LDS memory); byte_addr is that lane times 4.
__device__ __forceinline__ float row_fetch(float x, int byte_addr) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(byte_addr, __builtin_bit_cast(int, x)));
}

// Keeps the accumulator updates of a strip (or of all tiles) where they are
// written: without it the compiler sinks the contraction arithmetic towards
// the epilogue, keeping every strip's neighbour sums live (register spills).
template <int NB>
__device__ __forceinline__ void pin_strip(f32x4 (&acc)[NB][NB], int J) {
#pragma unroll
  for (int I = 0; I < NB; ++I) asm volatile("" : "+v"(acc[I][J]));
}
template <int NB>
__device__ __forceinline__ void pin_all(f32x4 (&acc)[NB][NB]) {
#pragma unroll
  for (int J = 0; J < NB; ++J) pin_strip<NB>(acc, J);
}

// Per-lane contraction coefficients of the fast modes.
struct LaneCoef {
  float fl[4];  // V_F on rows:  v_F[a_F][k]                 (a_F = lr % 4)
  float ml[4];  // V_M on rows:  v_M[a_M][(a_M - m) mod 4]   (a_M = lr / 4, rotation by 4 m)
  float mr[4];  // V_M on columns: v_M[(c_M + m) mod 4][c_M] (c_M = lq, row of 16 lanes m further on)
  int ra[4];    // byte address of the lane 16 m rows further on (m = 1..3 used)
};

// The coupling terms of one mode of role R (0: slow mode S, 1: M, 2: F) for
// ADO n: for every row strip J, X_s and W_s of the strip's tiles are summed
// from the neighbour tiles and contracted into the accumulators.  sg = +1 for
// the real plane, -1 for the imaginary plane; P is the plane of the neighbours
// that enters with the real part of the coefficients (the imaginary plane for
// the real output), Q the other one.
template <int NB, int R>
__device__ __forceinline__ void coupling_terms(const KronArgs& a, int s, int n, const float* trajP, const float* trajQ,
                                               float sg, const LaneCoef& lc, unsigned lane_off,
                                               f32x4 (&acc)[NB][NB]) {
  constexpr int D = 16 * NB;
  constexpr long long DD2 = 2LL * D * D;
  const int p0 = a.nb_ptr[n * a.n_modes + s];
  const int p1 = a.nb_ptr[n * a.n_modes + s + 1];
  if (p0 == p1) return;  // uniform across the wave
  bool need_w = false;
  for (int q = p0; q < p1; ++q)
    need_w = need_w || a.nb_a[4 * q + 2] != a.nb_a[4 * q] || a.nb_a[4 * q + 3] != a.nb_a[4 * q + 1];
  const float* v = R == 0 ? a.vS : R == 1 ? a.vM : a.vF;  // single-mode operator (kernel arguments: scalar)
  // Unrolled (the strip index selects accumulator registers), with a
  // scheduling barrier per strip so that the next strip's loads are not
  // hoisted above this strip's contractions (register pressure).
#pragma unroll
  for (int J = 0; J < NB; ++J) {
    f32x4 X[NB], W[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      X[I] = f32x4{0, 0, 0, 0};
      W[I] = f32x4{0, 0, 0, 0};
    }
    const unsigned toff = lane_off + 16u * J * D;
#pragma unroll 1
    for (int q = p0; q < p1; ++q) {
      const long long mo = static_cast<long long>(a.nb_idx[q]) * DD2;
      const float* bP = trajP + mo;
      const float* bQ = trajQ + mo;
      const float aLr = a.nb_a[4 * q], aLi = a.nb_a[4 * q + 1];
      const float aRr = a.nb_a[4 * q + 2], aRi = a.nb_a[4 * q + 3];
      const float cP = sg * aLr, dP = sg * (aRr - aLr), dQ = aRi - aLi;
      f32x4 p[NB];
#pragma unroll
      for (int I = 0; I < NB; ++I) p[I] = ld16(bP, toff + 16 * I);
      if (aLi != 0.0f || dQ != 0.0f) {
        f32x4 o[NB];
#pragma unroll
        for (int I = 0; I < NB; ++I) o[I] = ld16(bQ, toff + 16 * I);
#pragma unroll
        for (int I = 0; I < NB; ++I) {
          X[I] += aLi * o[I];
          W[I] += dQ * o[I];
        }
      }
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        X[I] += cP * p[I];
        if (need_w) W[I] += dP * p[I];
      }
    }
    // Y = X + W enters the right product
#pragma unroll
    for (int I = 0; I < NB; ++I) W[I] += X[I];
    if constexpr (R == 0) {
      // rows: a_S = J; columns: c_S = I
#pragma unroll
      for (int I = 0; I < NB; ++I) {
#pragma unroll
        for (int Jp = 0; Jp < NB; ++Jp) acc[I][Jp] += v[Jp * NB + J] * X[I];
#pragma unroll
        for (int Ip = 0; Ip < NB; ++Ip) acc[Ip][J] -= v[I * NB + Ip] * W[I];
      }
      pin_all<NB>(acc);
    } else if constexpr (R == 1) {
#pragma unroll
      for (int I = 0; I < NB; ++I) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x = X[I][r];
          float t = lc.ml[0] * x;
          t += lc.ml[1] * row_ror4<1>(x);
          t += lc.ml[2] * row_ror4<2>(x);
          t += lc.ml[3] * row_ror4<3>(x);
          const float y = W[I][r];
          t -= lc.mr[0] * y;
          t -= lc.mr[1] * row_fetch(y, lc.ra[1]);
          t -= lc.mr[2] * row_fetch(y, lc.ra[2]);
          t -= lc.mr[3] * row_fetch(y, lc.ra[3]);
          acc[I][J][r] += t;
        }
      }
      pin_strip<NB>(acc, J);
    } else {
#pragma unroll
      for (int I = 0; I < NB; ++I) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x = X[I][r];
          float t = lc.fl[0] * quad_bcast<0>(x);
          t += lc.fl[1] * quad_bcast<1>(x);
          t += lc.fl[2] * quad_bcast<2>(x);
          t += lc.fl[3] * quad_bcast<3>(x);
#pragma unroll
          for (int k = 0; k < 4; ++k) t -= v[k * 4 + r] * W[I][k];
          acc[I][J][r] += t;
        }
      }
      pin_strip<NB>(acc, J);
    }
  }
}

template <int NB>
__global__ __launch_bounds__(64 * KRON_WAVES, KRON_WG_PER_CU) void rhs_kron_kernel(
    KronArgs a, const float* __restrict__ in, const float* y, float* out, float coef, long long n_mats) {
  constexpr int D = 16 * NB;
  constexpr int LD = D + 4;  // 16-byte row padding (16-byte LDS reads of H rows)
  constexpr long long DD = static_cast<long long>(D) * D;
  __shared__ float sH[D * LD];
  for (int e = threadIdx.x; e < D * D; e += 64 * KRON_WAVES) sH[(e / D) * LD + e % D] = a.H[e];
  __syncthreads();

  // wave-uniform (readfirstlane tells the compiler so: the item, its ADO and
  // every table entry are then scalar values and the branches uniform)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lq = lane >> 4;
  LaneCoef lc;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    lc.fl[k] = a.vF[(lr & 3) * 4 + k];
    lc.ml[k] = a.vM[(lr >> 2) * 4 + (((lr >> 2) - k) & 3)];
    lc.mr[k] = a.vM[((lq + k) & 3) * 4 + lq];
    lc.ra[k] = 4 * (16 * ((lq + k) & 3) + lr);
  }
  // Wave index: the waves of one XCD (workgroups are dealt to the eight XCDs
  // round-robin) take consecutive work items, so that the ADOs processed
  // together on an XCD are hierarchy neighbours of one another more often and
  // meet in its L2.
  const long long G = gridDim.x;
  long long wid;
  if (G % 8 == 0)
    wid = ((blockIdx.x % 8) * (G / 8) + blockIdx.x / 8) * KRON_WAVES + wave;
  else
    wid = static_cast<long long>(blockIdx.x) * KRON_WAVES + wave;
  const long long n_work = 2 * n_mats;
  const long long stride = G * KRON_WAVES;
  // element offset of this lane's 16-byte slot in tile (0, 0) of a plane:
  // row lr, columns 4 lq .. 4 lq + 3
  const unsigned lane_off = lr * D + 4 * lq;
  for (long long p = wid; p < n_work; p += stride) {
    const long long mat = p >> 1;
    const int plane = static_cast<int>(p & 1);  // 0: Re L, 1: Im L
    const int n = static_cast<int>(mat % a.n_ado);
    const float sg = plane == 0 ? 1.0f : -1.0f;
    const float* rho = in + mat * 2 * DD;
    const float* Xp = rho + (plane == 0 ? DD : 0);  // plane entering the commutator with H
    const float* Op = rho + (plane == 0 ? 0 : DD);  // the other plane

    f32x4 acc[NB][NB];
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J) acc[I][J] = f32x4{0, 0, 0, 0};

    // ---- -i [H, rho] : acc(I,J) = sg sum_k (X[k][16I+i] H[k][16J+j] - H[16I+i][k] X[16J+j][k])
    // with k = 16 blk + 4 lq + t for the t-th product of block blk
#pragma unroll 1
    for (int blk = 0; blk < NB; ++blk) {
      float xa[NB][4];
      f32x4 xb[NB], hb[NB];
      const unsigned oa = (16u * blk + 4 * lq) * D + lr;   // X[16 blk + 4 lq + t][16 I + lr]
      const unsigned ob = lr * D + 16u * blk + 4 * lq;     // X[16 J + lr][16 blk + 4 lq ..]
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int t = 0; t < 4; ++t) xa[I][t] = sg * ld4(Xp, oa + t * D + 16 * I);
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        xb[J] = -sg * ld16(Xp, ob + 16 * J * D);
        hb[J] = *reinterpret_cast<const f32x4*>(&sH[(16 * J + lr) * LD + 16 * blk + 4 * lq]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
          for (int J = 0; J < NB; ++J) {
            acc[I][J] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[I][t], hb[J][t], acc[I][J], 0, 0, 0);
            acc[I][J] = __builtin_amdgcn_mfma_f32_16x16x4f32(hb[I][t], xb[J][t], acc[I][J], 0, 0, 0);
          }
    }

    pin_all<NB>(acc);

    // ---- damping: Re L -= g Re rho - gi Im rho;  Im L -= g Im rho + gi Re rho
    {
      const float g = a.gamma[n];
      const float gi = a.gamma_im ? a.gamma_im[n] : 0.0f;
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        // one strip at a time (scheduling barrier: the loads of the other
        // strips are not hoisted here, which would exceed the register budget)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int I = 0; I < NB; ++I) acc[I][J] -= g * ld16(Op, lane_off + 16 * J * D + 16 * I);
        pin_strip<NB>(acc, J);
      }
      if (gi != 0.0f) {
#pragma unroll
        for (int J = 0; J < NB; ++J) {
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int I = 0; I < NB; ++I) acc[I][J] += (sg * gi) * ld16(Xp, lane_off + 16 * J * D + 16 * I);
          pin_strip<NB>(acc, J);
        }
      }
    }

    // ---- couplings to the hierarchy neighbours, mode by mode
    {
      const float* traj = in + (mat - n) * 2 * DD;
      const float* trajP = traj + (plane == 0 ? DD : 0);
      const float* trajQ = traj + (plane == 0 ? 0 : DD);
      coupling_terms<NB, 0>(a, a.mode_S, n, trajP, trajQ, sg, lc, lane_off, acc);
      coupling_terms<NB, 1>(a, a.mode_M, n, trajP, trajQ, sg, lc, lane_off, acc);
      coupling_terms<NB, 2>(a, a.mode_F, n, trajP, trajQ, sg, lc, lane_off, acc);
    }

    // ---- epilogue: out = y + coef L (y may alias out; y and out are streamed)
    {
      const long long pb = mat * 2 * DD + (plane == 0 ? 0 : DD);
      const float* yb = y ? y + pb : nullptr;
      float* obase = out + pb;
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int I = 0; I < NB; ++I) {
          const unsigned e = lane_off + 16 * J * D + 16 * I;
          f32x4 v = acc[I][J];
          if (yb) v = ld16_nt(yb, e) + coef * v;
          __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(obase + e));
        }
      }
    }
  }
}

template <int NB>
void launch_kron_nb(const KronArgs& a, const float* in, const float* y, float* out, float coef, long long n_mats,
                    hipStream_t stream) {
  auto kern = &rhs_kron_kernel<NB>;
  int per_cu = KRON_WG_PER_CU;
  int fit = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void*>(kern), 64 * KRON_WAVES, 0) ==
          hipSuccess &&
      fit > 0 && fit < per_cu)
    per_cu = fit;
  long long grid = static_cast<long long>(cu_count()) * per_cu;
  const long long waves_needed = (2 * n_mats + KRON_WAVES - 1) / KRON_WAVES;
  if (grid > waves_needed) grid = waves_needed;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(64 * KRON_WAVES), 0, stream, a, in, y, out, coef,
                     n_mats);
}

}  // namespace

bool kron_supported(int d, int n_modes, const int* dims) {
  int roles[3];
  return kron_roles(d, n_modes, dims, roles);
}

bool kron_roles(int d, int n_modes, const int* dims, int* roles) {
  // three modes, two of them with 4 levels and the third with 4 or 5: the
  // slow mode S is the one with 5 levels (the first one if all have 4), M and
  // F the others in their order
  if (n_modes != 3 || (d != 64 && d != 80)) return false;
  int s = -1;
  for (int i = 0; i < 3; ++i)
    if (dims[i] == d / 16) {
      s = i;
      break;
    }
  if (s < 0) return false;
  int k = 0, rest[2];
  for (int i = 0; i < 3; ++i)
    if (i != s) rest[k++] = i;
  if (dims[rest[0]] != 4 || dims[rest[1]] != 4) return false;
  roles[0] = s;
  roles[1] = rest[0];
  roles[2] = rest[1];
  return true;
}

void launch_rhs_kron(const KronArgs& a, int d, const float* in, const float* y, float* out, double coef, int n_traj,
                     hipStream_t stream) {
  const long long n_mats = static_cast<long long>(n_traj) * a.n_ado;
  if (n_mats == 0) return;
  const float c = static_cast<float>(coef);
  if (d == 80)
    launch_kron_nb<5>(a, in, y, out, c, n_mats, stream);
  else if (d == 64)
    launch_kron_nb<4>(a, in, y, out, c, n_mats, stream);
  else
    throw std::runtime_error("kron RHS kernel: d must be 64 or 80");
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("kron rhs kernel: ") + hipGetErrorString(e));
}

}  // namespace heom

// Fused HEOM right-hand side + RK4 stage for three-mode models whose product
// basis factorises as (S; 4, 4): one slow mode of NB levels and two fast modes
// of 4 levels, in the device basis a = 16 a_S + 4 a_M + a_F (the builder
// reorders the basis so; states are permuted at the host boundary).  Eq.
// HEOM_DB (Sec. II.B) per ADO n:
//
//   L rho = -i [H, rho] - gamma_n rho - i sum_s ( V_s X_s - Y_s V_s ),
//   X_s = sum_q aL_q rho_{m_q},   Y_s = sum_q aR_q rho_{m_q},
//
// with V_s = v_s acting on mode s only and the neighbour lists (m_q, aL_q,
// aR_q) of the host tables.
//
// A workgroup of NB waves computes one real plane (Re or Im) of one output
// matrix at a time (the two planes of a matrix are independent work items).
// Wave w owns the 16 columns 16 w .. 16 w + 15 of the plane, as NB
// matrix-core tiles of the transposed output: lane (lq, lr) and register r of
// tile J hold L[16 J + lr][16 w + 4 lq + r].  The row digits of the device
// basis are (J, lr / 4, lr % 4) and the column digits (w, lq, r), so
//
//   * -i [H, rho] is two real products on v_mfma_f32_16x16x4 per plane,
//     (Re L)^T = Im^T H - H Im^T and (Im L)^T = -(Re^T H - H Re^T), with H
//     (symmetric) in LDS and the rho operands loaded from global memory
//     (k permuted within blocks of 16 so that one operand is a 16-byte load);
//   * V_F on rows is a quad broadcast (DPP), V_M on rows a rotation within 16
//     lanes (DPP), V_S on rows a sum over the wave's own tiles, V_F on
//     columns a sum over the wave's own registers, V_M on columns a fetch
//     from the other three 16-lane rows (ds_bpermute), and V_S on columns a
//     sum over the other waves' column strips, exchanged through LDS;
//   * neighbour tiles, damping and the RK4 update use 16-byte accesses in the
//     same layout.
//
// With 20 accumulator registers per wave a CU holds three workgroups (15
// waves), so memory latency of one wave is covered by the others.
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "kernels.h"

namespace heom {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KRON_WG_PER_CU = 3;

// Loads from a wave-uniform base plus a 32-bit per-lane element offset, taken
// as a 32-bit byte offset so that the base stays in scalar registers (the
// global_load form with a scalar base and a 32-bit vector offset).
__device__ __forceinline__ const char* byte_at(const float* base, unsigned off) {
  return reinterpret_cast<const char*>(base) + (off << 2);
}
__device__ __forceinline__ f32x4 ld16(const float* base, unsigned off) {
  return *reinterpret_cast<const f32x4*>(byte_at(base, off));
}
__device__ __forceinline__ float ld4(const float* base, unsigned off) {
  return *reinterpret_cast<const float*>(byte_at(base, off));
}
__device__ __forceinline__ f32x4 ld16_nt(const float* base, unsigned off) {
  return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(byte_at(base, off)));
}
__device__ __forceinline__ void st16_nt(float* base, unsigned off, f32x4 v) {
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(reinterpret_cast<char*>(base) + (off << 2)));
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

// x of the lane whose byte address is byte_addr (4 x lane), through the LDS
// crossbar (ds_bpermute, no LDS memory)
__device__ __forceinline__ float lane_fetch(float x, int byte_addr) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(byte_addr, __builtin_bit_cast(int, x)));
}

// Keeps accumulator updates where they are written: without it the compiler
// sinks contraction arithmetic towards the epilogue, keeping neighbour sums
// live (register spills).
template <int NB>
__device__ __forceinline__ void pin(f32x4 (&acc)[NB]) {
#pragma unroll
  for (int J = 0; J < NB; ++J) asm volatile("" : "+v"(acc[J]));
}

// Per-lane contraction coefficients of the fast modes.
struct LaneCoef {
  float fl[4];  // V_F on rows:  v_F[a_F][k]                 (a_F = lr % 4)
  float ml[4];  // V_M on rows:  v_M[a_M][(a_M - m) mod 4]   (a_M = lr / 4, rotation by 4 m)
  float mr[4];  // V_M on columns: v_M[(c_M + m) mod 4][c_M] (c_M = lq, row of 16 lanes m further on)
  int ra[4];    // byte address of the lane 16 m rows further on (m = 1..3 used)
};

// Sums X = sum_q aL_q rho_q and Y = sum_q aR_q rho_q over the neighbours of
// one mode for the wave's NB tiles (column strip), as one real plane with the
// sign convention of the output plane: for the real plane (sg = +1) X and Y
// are Im X_s and Im Y_s; for the imaginary plane (sg = -1) they are -Re X_s
// and -Re Y_s.  P is the plane of the neighbours entering with the real part
// of the coefficients, Q the other one.  Returns false if the mode has no
// neighbours (X = Y = 0).
template <int NB>
__device__ __forceinline__ bool neighbour_sums(const KronArgs& a, int s, int n, const float* trajP,
                                               const float* trajQ, float sg, unsigned soff, f32x4 (&X)[NB],
                                               f32x4 (&Y)[NB]) {
  constexpr int D = 16 * NB;
  constexpr long long DD2 = 2LL * D * D;
  const int p0 = a.nb_ptr[n * a.n_modes + s];
  const int p1 = a.nb_ptr[n * a.n_modes + s + 1];
  if (p0 == p1) return false;  // uniform across the wave
#pragma unroll
  for (int J = 0; J < NB; ++J) {
    X[J] = f32x4{0, 0, 0, 0};
    Y[J] = f32x4{0, 0, 0, 0};
  }
#pragma unroll 1
  for (int q = p0; q < p1; ++q) {
    const long long mo = static_cast<long long>(a.nb_idx[q]) * DD2;
    const float aLr = a.nb_a[4 * q], aLi = a.nb_a[4 * q + 1];
    const float aRr = a.nb_a[4 * q + 2], aRi = a.nb_a[4 * q + 3];
    const float cX = sg * aLr, cY = sg * aRr;
    {
      f32x4 p[NB];
#pragma unroll
      for (int J = 0; J < NB; ++J) p[J] = ld16(trajP + mo + 16 * J * D, soff);
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        X[J] += cX * p[J];
        Y[J] += cY * p[J];
      }
    }
    // the other plane only for complex coefficients (after the first one's
    // registers are free: one load set live at a time)
    if (aLi != 0.0f || aRi != 0.0f) {
      f32x4 o[NB];
#pragma unroll
      for (int J = 0; J < NB; ++J) o[J] = ld16(trajQ + mo + 16 * J * D, soff);
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        X[J] += aLi * o[J];
        Y[J] += aRi * o[J];
      }
    }
  }
  return true;
}

template <int NB>
__global__ __launch_bounds__(64 * NB) __attribute__((amdgpu_waves_per_eu(4, 4))) void rhs_kron_kernel(
    KronArgs a, const float* __restrict__ in, const float* y, float* out, float coef, long long n_mats) {
  constexpr int D = 16 * NB;
  constexpr int LD = D + 4;  // 16-byte row padding (16-byte LDS reads of H rows)
  constexpr long long DD = static_cast<long long>(D) * D;
  __shared__ float sH[D * LD];
  __shared__ f32x4 sY[NB][NB][64];  // Y_S tiles of every wave: [strip][J][lane]
  __shared__ float sv[NB * NB + 16];  // v_S, v_F (read as uniform LDS values where used)
  for (int e = threadIdx.x; e < D * D; e += 64 * NB) sH[(e / D) * LD + e % D] = a.H[e];
  if (threadIdx.x < NB * NB) sv[threadIdx.x] = a.vS[threadIdx.x];
  else if (threadIdx.x < NB * NB + 16) sv[threadIdx.x] = a.vF[threadIdx.x - NB * NB];
  __syncthreads();
  const float* vS = sv;
  const float* vF = sv + NB * NB;

  // wave-uniform (readfirstlane tells the compiler so: the item, its ADO and
  // every table entry are then scalar values and the branches uniform)
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // column strip
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
  // Work item of this workgroup: the workgroups of one XCD (dealt to the
  // eight XCDs round-robin) take consecutive items, so that the ADOs
  // processed together on an XCD are hierarchy neighbours of one another more
  // often and meet in its L2.
  const long long G = gridDim.x;
  const long long first = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  // element offset of this lane's 16-byte slot in tile J = 0 of the strip:
  // row lr, columns 16 w + 4 lq .. + 3
  const unsigned soff = lr * D + 16 * w + 4 * lq;
  const unsigned oa = 4 * lq * D + lr;   // X[16 blk + 4 lq + t][16 w + lr] from the block base
  const unsigned ob = lr * D + 4 * lq;   // X[16 J + lr][16 blk + 4 lq ..] from the block base
  for (long long p = first; p < 2 * n_mats; p += G) {
    const long long mat = p >> 1;
    const int plane = static_cast<int>(p & 1);  // 0: Re L, 1: Im L
    const int n = static_cast<int>(mat % a.n_ado);
    const float sg = plane == 0 ? 1.0f : -1.0f;
    const float* rho = in + mat * 2 * DD;
    const float* Xp = rho + (plane == 0 ? DD : 0);  // plane entering the commutator with H
    const float* Op = rho + (plane == 0 ? 0 : DD);  // the other plane

    f32x4 acc[NB];
#pragma unroll
    for (int J = 0; J < NB; ++J) acc[J] = f32x4{0, 0, 0, 0};

    // ---- -i [H, rho]: acc(J) = sg sum_k (X[k][16w+i] H[k][16J+j] - H[16w+i][k] X[16J+j][k]),
    // k = 16 blk + 4 lq + t for the t-th product of block blk.  Operands:
    // xa = X[16 blk + 4 lq + t][16 w + lr] (A of X^T H), xb = X[16 J + lr][16 blk
    // + 4 lq + t] (B of H X^T), hb = H[16 J + lr][16 blk + 4 lq + t] (B of X^T
    // H) and hw = H[16 w + lr][..] (A of H X^T; H is symmetric)
#pragma unroll 1
    for (int blk = 0; blk < NB; ++blk) {
      float xa[4];
      f32x4 xb[NB], hb[NB];
      // uniform block bases (scalar registers) plus loop-invariant lane offsets
      const float* pa = Xp + 16 * blk * D + 16 * w;
      const float* pb = Xp + 16 * blk;
#pragma unroll
      for (int t = 0; t < 4; ++t) xa[t] = sg * ld4(pa, oa + t * D);
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        xb[J] = -sg * ld16(pb + 16 * J * D, ob);
        hb[J] = *reinterpret_cast<const f32x4*>(&sH[(16 * J + lr) * LD + 16 * blk + 4 * lq]);
      }
      const f32x4 hw = *reinterpret_cast<const f32x4*>(&sH[(16 * w + lr) * LD + 16 * blk + 4 * lq]);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int J = 0; J < NB; ++J) {
          acc[J] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[t], hb[J][t], acc[J], 0, 0, 0);
          acc[J] = __builtin_amdgcn_mfma_f32_16x16x4f32(hw[t], xb[J][t], acc[J], 0, 0, 0);
        }
    }

    // ---- damping: Re L -= g Re rho - gi Im rho;  Im L -= g Im rho + gi Re rho
    {
      const float g = a.gamma[n];
      const float gi = a.gamma_im ? a.gamma_im[n] : 0.0f;
#pragma unroll
      for (int J = 0; J < NB; ++J) acc[J] -= g * ld16(Op + 16 * J * D, soff);
      if (gi != 0.0f) {
#pragma unroll
        for (int J = 0; J < NB; ++J) acc[J] += (sg * gi) * ld16(Xp + 16 * J * D, soff);
      }
    }
    pin<NB>(acc);

    const float* traj = in + (mat - n) * 2 * DD;
    const float* trajP = traj + (plane == 0 ? DD : 0);
    const float* trajQ = traj + (plane == 0 ? 0 : DD);
    f32x4 X[NB], Y[NB];
    // ---- slow mode S: rows a_S = J (own tiles); columns c_S = w (the other
    // waves' strips, through LDS after the barrier below)
    const bool has_s = neighbour_sums<NB>(a, a.mode_S, n, trajP, trajQ, sg, soff, X, Y);
    __syncthreads();  // every wave is done reading sY of the previous item
    if (has_s) {
#pragma unroll
      for (int J = 0; J < NB; ++J) {
#pragma unroll
        for (int Jp = 0; Jp < NB; ++Jp) acc[Jp] += vS[Jp * NB + J] * X[J];
        sY[w][J][lane] = Y[J];
      }
    }
    pin<NB>(acc);
    // ---- mode M: rows a_M = lr / 4 (rotation), columns c_M = lq (lane fetch)
    if (neighbour_sums<NB>(a, a.mode_M, n, trajP, trajQ, sg, soff, X, Y)) {
#pragma unroll
      for (int J = 0; J < NB; ++J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x = X[J][r], yv = Y[J][r];
          float t = lc.ml[0] * x;
          t += lc.ml[1] * row_ror4<1>(x);
          t += lc.ml[2] * row_ror4<2>(x);
          t += lc.ml[3] * row_ror4<3>(x);
          t -= lc.mr[0] * yv;
          t -= lc.mr[1] * lane_fetch(yv, lc.ra[1]);
          t -= lc.mr[2] * lane_fetch(yv, lc.ra[2]);
          t -= lc.mr[3] * lane_fetch(yv, lc.ra[3]);
          acc[J][r] += t;
        }
      }
    }
    pin<NB>(acc);
    // ---- mode F: rows a_F = lr % 4 (quad broadcast), columns c_F = r (own registers)
    if (neighbour_sums<NB>(a, a.mode_F, n, trajP, trajQ, sg, soff, X, Y)) {
#pragma unroll
      for (int J = 0; J < NB; ++J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x = X[J][r];
          float t = lc.fl[0] * quad_bcast<0>(x);
          t += lc.fl[1] * quad_bcast<1>(x);
          t += lc.fl[2] * quad_bcast<2>(x);
          t += lc.fl[3] * quad_bcast<3>(x);
#pragma unroll
          for (int k = 0; k < 4; ++k) t -= vF[k * 4 + r] * Y[J][k];
          acc[J][r] += t;
        }
      }
    }
    pin<NB>(acc);
    __syncthreads();  // sY of every wave written
    if (has_s) {
      // (Y V_S)[a][c] = sum_k Y[a][c_S = k] v_S[k][c_S]: this strip's c_S = w
#pragma unroll
      for (int Ip = 0; Ip < NB; ++Ip) {
        const float v = vS[Ip * NB + w];
#pragma unroll
        for (int J = 0; J < NB; ++J) acc[J] -= v * sY[Ip][J][lane];
      }
    }

    // ---- epilogue: out = y + coef L (y may alias out; y and out are streamed)
    {
      const long long pb = mat * 2 * DD + (plane == 0 ? 0 : DD);
      const float* yb = y ? y + pb : nullptr;
      float* obase = out + pb;
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        f32x4 v = acc[J];
        if (yb) v = ld16_nt(yb + 16 * J * D, soff) + coef * v;
        st16_nt(obase + 16 * J * D, soff, v);
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
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void*>(kern), 64 * NB, 0) ==
          hipSuccess &&
      fit > 0 && fit < per_cu)
    per_cu = fit;
  long long grid = static_cast<long long>(cu_count()) * per_cu;
  if (grid > 2 * n_mats) grid = 2 * n_mats;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(64 * NB), 0, stream, a, in, y, out, coef, n_mats);
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

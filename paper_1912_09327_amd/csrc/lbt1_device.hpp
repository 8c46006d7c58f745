// Device-side arithmetic of the LBMTau1 D2Q9 step for gfx950.
//
// Method (arXiv:1912.09327): with tau = 1 the populations leaving a node are
// its equilibria (Eq. LBMTau1), so the new density and momentum of a fluid
// node x are the sums, over the nine directions q, of the equilibrium
// f^eq_q of the upwind node x - e_q (Eq. rhotau1, Eq. utau1, Algorithm 1).
// A link whose upwind node is a wall contributes w_q rho(x) (Eq. feqnoslip,
// the paper's rule) or, under half-way bounce-back, the equilibrium x sent
// toward the wall.
//
// Arithmetic form used by every kernel (so that all kernels agree bit for
// bit): the density is carried as the deviation d = rho - 1, and
// Eq. maxwellboltzmann is expanded in the momentum J = j + F (the force
// shift of Algorithm 1) and the tensor P = J J / rho:
//     f^eq_q - w_q = w_q [ d + 3 e_q.J + 4.5 (e_q.J)^2 / rho - 1.5 |J|^2 / rho ].
// The constant parts w_q of the nine terms arriving at any node sum to one,
// so the new deviation is the sum of the bracketed parts alone; the rounding
// of reduced-precision arithmetic then scales with |d|, not with rho ~ 1.
// One reciprocal per source node replaces the per-link divisions of the
// paper's listing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbt1 {

enum : int { P_F64 = 0, P_F32 = 1, P_F16S = 2, P_BF16S = 3 };
enum : uint8_t { NODE_FLUID = 0, NODE_SOLID = 1, NODE_FIXED = 2 };
enum : int { WALL_PAPER = 0, WALL_HALFWAY = 1 };

// ----------------------------------------------------------------- storage codecs
template <int P> struct Traits;
template <> struct Traits<P_F64> {
  using S = double;  // stored value
  using C = double;  // arithmetic
  static constexpr bool kScaled = false;
  __device__ static inline C dec(S s) { return s; }
  __device__ static inline S enc(C c) { return c; }
};
template <> struct Traits<P_F32> {
  using S = float;
  using C = float;
  static constexpr bool kScaled = false;
  __device__ static inline C dec(S s) { return s; }
  __device__ static inline S enc(C c) { return c; }
};
template <> struct Traits<P_F16S> {
  using S = uint16_t;  // IEEE binary16 bits
  using C = float;
  static constexpr bool kScaled = true;
  __device__ static inline C dec(S s) { return (float)__builtin_bit_cast(_Float16, s); }
  // v_cvt_f16_f32: round to nearest even under the default mode
  __device__ static inline S enc(C c) { return __builtin_bit_cast(uint16_t, (_Float16)c); }
};
template <> struct Traits<P_BF16S> {
  using S = uint16_t;  // bfloat16 bits
  using C = float;
  static constexpr bool kScaled = true;
  __device__ static inline C dec(S s) { return __builtin_bit_cast(float, (uint32_t)s << 16); }
  // gfx950 v_cvt_pk_bf16_f32: round to nearest even
  __device__ static inline S enc(C c) { return __builtin_bit_cast(uint16_t, (__bf16)c); }
};

template <typename C> __device__ inline C recip(C x);
template <> __device__ inline float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double recip<double>(double x) { return 1.0 / x; }

template <typename C> __device__ inline C fmaC(C a, C b, C c);
template <> __device__ inline float fmaC<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ inline double fmaC<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// D2Q9 velocities in the paper's order (section 2) and their inverses.
__device__ constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kInv[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// ----------------------------------------------------------------- emission
// The nine equilibrium deviations a source node with deviation d and
// momentum (jx, jy) sends out, f[q] travelling along e_q.
template <typename C>
__device__ __forceinline__ void emit(C d, C jx, C jy, C Fx, C Fy, C f[9]) {
  const C Jx = jx + Fx;
  const C Jy = jy + Fy;
  const C inv = recip<C>(C(1) + d);
  const C ux = Jx * inv;
  const C uy = Jy * inv;
  const C pxx = Jx * ux;
  const C pyy = Jy * uy;
  const C pxy = Jx * uy;
  const C t = pxx + pyy;
  // every bracket holds base = d - 1.5 tr P: the rest link's is base itself
  const C base = fmaC<C>(C(-1.5), t, d);
  f[0] = C(4.0 / 9.0) * base;
  const C b9 = C(1.0 / 9.0) * base;
  // axes: w = 1/9, bracket base + 4.5 P_aa +- 3 J_a
  const C bx = fmaC<C>(C(0.5), pxx, b9);
  const C by = fmaC<C>(C(0.5), pyy, b9);
  f[1] = fmaC<C>(C(1.0 / 3.0), Jx, bx);
  f[3] = fmaC<C>(C(-1.0 / 3.0), Jx, bx);
  f[2] = fmaC<C>(C(1.0 / 3.0), Jy, by);
  f[4] = fmaC<C>(C(-1.0 / 3.0), Jy, by);
  // diagonals: w = 1/36, bracket base + 4.5 tr P +- 9 P_xy + 3 e.J (base / 36 is
  // b9 / 4, exact)
  const C bd = fmaC<C>(C(0.125), t, C(0.25) * b9);
  const C bp = fmaC<C>(C(0.25), pxy, bd);
  const C bm = fmaC<C>(C(-0.25), pxy, bd);
  const C sp = Jx + Jy;
  const C sm = Jx - Jy;
  f[5] = fmaC<C>(C(1.0 / 12.0), sp, bp);
  f[7] = fmaC<C>(C(-1.0 / 12.0), sp, bp);
  f[8] = fmaC<C>(C(1.0 / 12.0), sm, bm);
  f[6] = fmaC<C>(C(-1.0 / 12.0), sm, bm);
}

// Deviation part of Eq. feqnoslip, w_q d(x), for an axis (1/9) or diagonal (1/36) link.
template <typename C> __device__ __forceinline__ C wall_axis(C d) { return C(1.0 / 9.0) * d; }
template <typename C> __device__ __forceinline__ C wall_diag(C d) { return C(1.0 / 36.0) * d; }

// ----------------------------------------------------------------- multiphase
// Shan-Chen pseudopotential psi(rho) = rho0 (1 - exp(-rho / rho0)).
template <typename C> __device__ inline C sc_exp(C x);
template <> __device__ inline float sc_exp<float>(float x) { return expf(x); }
template <> __device__ inline double sc_exp<double>(double x) { return exp(x); }
template <typename C>
__device__ __forceinline__ C sc_psi(C rho, C rho0, C inv_rho0) {
  return rho0 * (C(1) - sc_exp<C>(-rho * inv_rho0));
}
// Interaction force of a node (the paper's Eq. f_sc with alpha_k = w_k and
// G(e_k) = -G e_k): F = -G psi_0 sum_k w_k psi_k e_k, psi_0 the node's own
// pseudopotential and psi_k that of its neighbour along e_k.
template <typename C>
__device__ __forceinline__ void sc_force(const C (&psi)[9], C G, C &fx, C &fy) {
  const C sx = C(1.0 / 9.0) * (psi[1] - psi[3]) + C(1.0 / 36.0) * ((psi[5] - psi[6]) + (psi[8] - psi[7]));
  const C sy = C(1.0 / 9.0) * (psi[2] - psi[4]) + C(1.0 / 36.0) * ((psi[5] - psi[7]) + (psi[6] - psi[8]));
  const C a = -G * psi[0];
  fx = a * sx;
  fy = a * sy;
}

// ----------------------------------------------------------------- target sums
// Arrivals g[q] at a node (g[q] travelled along e_q, from x - e_q).  Grouped
// by the source row: y-1 (q = 5, 2, 6), y (1, 0, 3), y+1 (8, 4, 7).  This
// order is part of the contract between kernels: all of them use it.
// ----------------------------------------------------------------- lane exchange
// Neighbour values along the wavefront: lane_left(x) is lane l - 1's x,
// lane_right(x) lane l + 1's.  Lanes 0 and 63 hold halo columns whose values are
// never stored, so what they receive at the open end does not matter.
// FP32 and FP64 kernels are bound by latency: they use the whole-wavefront DPP
// shifts of this chip family (a VALU move, often folded into the add or
// subtract that consumes it; the lane without a source reads zero).  16-bit
// storage kernels are bound by VALU issue: their exchange stays on the LDS
// permute path, which issues outside the VALU.
constexpr int kDppWaveShl1 = 0x130;  // lane l reads lane l + 1
constexpr int kDppWaveShr1 = 0x138;  // lane l reads lane l - 1
template <int CTRL> __device__ __forceinline__ int dpp_shift(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xf, 0xf, true);
}
template <int CTRL> __device__ __forceinline__ float dpp_shift(float x) {
  return __int_as_float(dpp_shift<CTRL>(__float_as_int(x)));
}
template <int CTRL> __device__ __forceinline__ double dpp_shift(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_shift<CTRL>((int)(b & 0xffffffffLL)), hi = dpp_shift<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int P, typename X> __device__ __forceinline__ X lane_left(X x) {
  if constexpr (sizeof(typename Traits<P>::S) == 2) return __shfl_up(x, 1);
  else return dpp_shift<kDppWaveShr1>(x);
}
template <int P, typename X> __device__ __forceinline__ X lane_right(X x) {
  if constexpr (sizeof(typename Traits<P>::S) == 2) return __shfl_down(x, 1);
  else return dpp_shift<kDppWaveShl1>(x);
}

template <typename C> __device__ __forceinline__ C row_sum(C a, C b, C c) { return (a + b) + c; }
template <typename C> __device__ __forceinline__ C row_dif(C a, C c) { return a - c; }
template <typename C>
__device__ __forceinline__ void finish(C sm, C xm, C s0, C x0, C sp, C xp, C &d, C &jx, C &jy) {
  d = (sm + s0) + sp;
  jx = (xm + x0) + xp;
  jy = sm - sp;
}

// ----------------------------------------------------------------- kernel arguments
// Bytes of the trash area per moment field.  Lane l of a wavefront redirects a
// store of VEC values to element l * VEC of a field's region, so every kernel
// asserts 64 * VEC * sizeof(stored value) <= kTrashRegion.
constexpr long kTrashRegion = 1024;

struct StepArgs {
  const void *src[3];  // d, jx, jy planes of the current parity
  void *dst[3];        // planes of the next parity
  const uint8_t *flags;
  int nx, ny;
  int pitch;           // flag row stride in values (nx rounded up to 64)
  int rs;              // moment row stride in values (pitch, or 3 * pitch when the
                       // three moment rows of a lattice row are adjacent)
  uint32_t periodic;   // bit 0 x, bit 1 y
  double fx, fy;       // body force
  double sc_d, sc_j;   // decode scales (stored * sc = value)
  double is_d, is_j;   // encode scales (value * is = stored)
  void *trash;         // 3 KiB of device scratch, one kTrashRegion per moment field:
                       // target of the stores of lanes and rows outside the grid, so
                       // that stores need no branch
  double sc_G, sc_rho0;  // multiphase kernels: Shan-Chen coupling and psi scale
};

// Source coordinate along one axis: wrapped when periodic (any distance, so
// strips taller than a small periodic grid stay in bounds), -1 when outside.
__device__ __forceinline__ int wrap_axis(int c, int n, bool periodic) {
  if (c >= 0 && c < n) return c;
  if (!periodic) return -1;
  c %= n;
  return c < 0 ? c + n : c;
}

template <int P>
__device__ __forceinline__ void load_node(const StepArgs &a, long idx, typename Traits<P>::C &d,
                                          typename Traits<P>::C &jx, typename Traits<P>::C &jy) {
  using T = Traits<P>;
  using S = typename T::S;
  using C = typename T::C;
  d = T::dec(static_cast<const S *>(a.src[0])[idx]);
  jx = T::dec(static_cast<const S *>(a.src[1])[idx]);
  jy = T::dec(static_cast<const S *>(a.src[2])[idx]);
  if (T::kScaled) {
    d *= C(a.sc_d);
    jx *= C(a.sc_j);
    jy *= C(a.sc_j);
  }
}

}  // namespace lbt1

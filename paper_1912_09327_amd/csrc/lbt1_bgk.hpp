// Stored-population D2Q9 BGK step (Eq. lbm) for gfx950: the standard method
// the paper starts from, kept for the memory and speed comparison of
// section 4 (2 Q + N_f values per node against 2 N_f) and for tau != 1.
//
// Every node keeps its nine populations as deviations g_q = f_q - w_q in the
// storage format of the grid.  One step, one thread per node (push form):
// load the node's own nine populations, form rho - 1 and j, relax toward the
// equilibrium of (rho, (j + tau F) / rho) with rate 1 / tau, and send each
// relaxed population to the neighbour it points at.  A population that would
// enter a wall comes back to the sender reversed: the zero-velocity
// equilibrium w_q rho(x) of the sender (Eq. feqnoslip) or, under half-way
// bounce-back, the relaxed population itself.  FIXED nodes hold the
// equilibrium of their moments (with the force shift) in both parities and
// send it unchanged; nothing is sent into them.
#pragma once
#include "lbt1_args.hpp"
#include "lbt1_device.hpp"

namespace lbt1 {

// Blocks of 64 x 4 nodes.  Consecutive blocks of the launch go to different
// XCDs, each with its own L2; the tiles are dealt out so that one XCD works
// on a contiguous run of tiles along the rows, and the stores that spill one
// node past a tile edge meet the neighbouring tile's stores in the same L2.
// rho - 1 of a node from its nine deviations (the order every kernel uses)
template <typename C>
__device__ __forceinline__ C pop_density(const C (&g)[9]) {
  return (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) + g[8];
}

// Multiphase: the pseudopotential of every node (SOLID nodes hold the
// zero-velocity equilibrium of their given density, so theirs is that of the
// given density).
template <int P>
__global__ void __launch_bounds__(256) k_bgk_psi(BgkArgs a) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  const int t = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
  if (t >= a.tiles) return;
  const int by = t / a.tiles_x;
  const int x = (t - by * a.tiles_x) * 64 + (threadIdx.x & 63);
  const int y = by * 4 + (threadIdx.x >> 6);
  if (x >= a.nx || y >= a.ny) return;
  const long i = (long)y * a.rs + x;
  C g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    g[q] = T::dec(static_cast<const S *>(a.src[q])[i]);
    if (T::kScaled) g[q] *= C(a.sc);
  }
  static_cast<C *>(a.psi)[(long)y * a.pitch + x] =
      sc_psi<C>(C(1) + pop_density<C>(g), C(a.sc_rho0), C(1.0 / a.sc_rho0));
}

template <int P, bool HASWALL, int WALL, bool SC>
__global__ void __launch_bounds__(256) k_bgk_step(BgkArgs a) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  const int t = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
  if (t >= a.tiles) return;
  const int by = t / a.tiles_x;
  const int x = (t - by * a.tiles_x) * 64 + (threadIdx.x & 63);
  const int y = by * 4 + (threadIdx.x >> 6);
  if (x >= a.nx || y >= a.ny) return;
  const long i = (long)y * a.rs + x;
  uint8_t fl = NODE_FLUID;
  if (HASWALL) {
    fl = a.flags[(long)y * a.pitch + x];
    if (fl == NODE_SOLID) return;
  }
  const C sc = C(a.sc), is = C(a.is);
  C g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    g[q] = T::dec(static_cast<const S *>(a.src[q])[i]);
    if (T::kScaled) g[q] *= sc;
  }
  // moments of the deviations: rho - 1 = sum g, j = sum e g (sum w e = 0)
  const C d = pop_density<C>(g);
  const C jx = ((g[1] - g[3]) + (g[5] - g[6])) + (g[8] - g[7]);
  const C jy = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
  C post[9];
  if (!HASWALL || fl == NODE_FLUID) {
    C Fx = C(a.fx), Fy = C(a.fy);
    if (SC) {
      const C *ps = static_cast<const C *>(a.psi);
      C psi[9];
      psi[0] = ps[(long)y * a.pitch + x];
#pragma unroll
      for (int k = 1; k < 9; ++k) {
        const int tx = wrap_axis(x + kEx[k], a.nx, a.periodic & 1u);
        const int ty = wrap_axis(y + kEy[k], a.ny, a.periodic & 2u);
        psi[k] = (tx < 0 || ty < 0) ? psi[0] : ps[(long)ty * a.pitch + tx];
      }
      C gx, gy;
      sc_force<C>(psi, C(a.sc_G), gx, gy);
      Fx = C(a.tau) * (C(a.bfx) + gx);
      Fy = C(a.tau) * (C(a.bfy) + gy);
    }
    C geq[9];
    emit<C>(d, jx, jy, Fx, Fy, geq);
    const C om = C(a.omega);
#pragma unroll
    for (int q = 0; q < 9; ++q) post[q] = fmaC<C>(om, geq[q] - g[q], g[q]);
  } else {
#pragma unroll
    for (int q = 0; q < 9; ++q) post[q] = g[q];  // FIXED: its stored equilibrium
  }
  const bool px = a.periodic & 1u, py = a.periodic & 2u;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    int tx = x + kEx[q], ty = y + kEy[q];
    bool wall = false;
    if (tx < 0 || tx >= a.nx) {
      if (px) tx = tx < 0 ? tx + a.nx : tx - a.nx;
      else wall = true;
    }
    if (ty < 0 || ty >= a.ny) {
      if (py) ty = ty < 0 ? ty + a.ny : ty - a.ny;
      else wall = true;
    }
    uint8_t tf = NODE_FLUID;
    if (HASWALL && !wall) tf = a.flags[(long)ty * a.pitch + tx];
    C v = post[q];
    long dst = (long)ty * a.rs + tx;
    int dq = q;
    if (HASWALL) {
      if (wall || tf == NODE_SOLID) {
        if (fl != NODE_FLUID) continue;
        dq = kInv[q];
        dst = i;
        if (WALL == WALL_PAPER) v = (q <= 4) ? wall_axis<C>(d) : wall_diag<C>(d);
      } else if (tf == NODE_FIXED) {
        continue;
      }
    }
    if (T::kScaled) v *= is;
    static_cast<S *>(a.dst[dq])[dst] = T::enc(v);
  }
}

// out slots as k_reduce_partial: 0 sum (rho - 1), 1 sum jx, 2 sum jy,
// 3 max residual, 4 non-finite count, 5 FLUID count.
template <int P>
__global__ void __launch_bounds__(256) k_bgk_reduce_partial(BgkReduceArgs a) {
  using T = Traits<P>;
  using S = typename T::S;
  const bool want_res = a.what & 4u;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const long n = (long)a.nx * a.ny;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int y = (int)(k / a.nx);
    const int x = (int)(k - (long)y * a.nx);
    const long i = (long)y * a.rs + x;
    if (a.flags && a.flags[(long)y * a.pitch + x] != NODE_FLUID) continue;
    double g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = (double)T::dec(static_cast<const S *>(a.cur[q])[i]) * a.sc;
    const double d = (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) + g[8];
    const double jx = ((g[1] - g[3]) + (g[5] - g[6])) + (g[8] - g[7]);
    const double jy = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
    acc[0] += d;
    acc[1] += jx;
    acc[2] += jy;
    acc[4] += (__builtin_isfinite(d) && __builtin_isfinite(jx) && __builtin_isfinite(jy)) ? 0.0 : 1.0;
    acc[5] += 1.0;
    if (want_res) {
      S *s0 = static_cast<S *>(a.snap[0]);
      S *s1 = static_cast<S *>(a.snap[1]);
      S *s2 = static_cast<S *>(a.snap[2]);
      const long si = (long)y * a.snap_rs + x;
      const double sr = 1.0 + (double)T::dec(s0[si]) * a.sc_d;
      const double su = (double)T::dec(s1[si]) * a.sc_j / sr;
      const double sv = (double)T::dec(s2[si]) * a.sc_j / sr;
      const double rho = 1.0 + d;
      acc[3] = __builtin_fmax(acc[3], __builtin_fmax(__builtin_fabs(jx / rho - su), __builtin_fabs(jy / rho - sv)));
      s0[si] = T::enc((typename T::C)(d * a.is_d));
      s1[si] = T::enc((typename T::C)(jx * a.is_j));
      s2[si] = T::enc((typename T::C)(jy * a.is_j));
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double o = __shfl_xor(acc[q], off);
      acc[q] = q == 3 ? __builtin_fmax(acc[q], o) : acc[q] + o;
    }
  }
  __shared__ double part[4][6];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 6; ++q) part[wave][q] = acc[q];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int q = threadIdx.x;
    double v = part[0][q];
    for (int w = 1; w < 4; ++w) v = q == 3 ? __builtin_fmax(v, part[w][q]) : v + part[w][q];
    a.partials[blockIdx.x * 6 + q] = v;
  }
}

}  // namespace lbt1

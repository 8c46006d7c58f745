// Multiphase LBMTau1 (the paper's section on the moments-only MRT form and
// its Shan-Chen example): with tau = 1 a node sends the equilibria of its
// moments and of its interaction force F (Eq. f_sc), which enters exactly
// like the body force (equilibrium velocity (j + F_body + F) / rho).  F of a
// node needs the pseudopotential psi of its eight neighbours, so the update
// of a node depends on its 5 x 5 neighbourhood.
//
//  * gather: one thread per node; the force of each of the nine sources is
//    formed from the densities around it.  Any geometry.  A SOLID neighbour
//    contributes the psi of its stored density, a neighbour outside a
//    non-periodic axis that of the node itself.
//  * strip: periodic grids without wall nodes.  No psi field is stored: the
//    wavefront computes psi once per loaded row and lane, takes the
//    neighbouring lanes' edge values through shuffles, and emits a source row
//    once the row after it has been loaded; a strip loads NY + 4 rows.  As in
//    the fused kernel, lanes 0 and 63 are wrong in their outer column, so
//    lanes 1..62 are exact for VEC >= 2.
// Both compute psi, the force sum and the emission in the same order, so they
// agree bit for bit.
#pragma once
#include "lbt1_fused.hpp"
#include "lbt1_step.hpp"

namespace lbt1 {

template <int P>
__device__ __forceinline__ typename Traits<P>::C node_psi(const StepArgs &a, long idx) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  C d = T::dec(static_cast<const S *>(a.src[0])[idx]);
  if (T::kScaled) d *= C(a.sc_d);
  return sc_psi<C>(C(1) + d, C(a.sc_rho0), C(1.0 / a.sc_rho0));
}

// Total force (body + interaction) of source node (sx, sy), in range and not SOLID.
template <int P>
__device__ __forceinline__ void source_force(const StepArgs &a, int sx, int sy, typename Traits<P>::C &fx,
                                             typename Traits<P>::C &fy) {
  using C = typename Traits<P>::C;
  C psi[9];
  psi[0] = node_psi<P>(a, (long)sy * a.rs + sx);
#pragma unroll
  for (int k = 1; k < 9; ++k) {
    const int tx = wrap_axis(sx + kEx[k], a.nx, a.periodic & 1u);
    const int ty = wrap_axis(sy + kEy[k], a.ny, a.periodic & 2u);
    psi[k] = (tx < 0 || ty < 0) ? psi[0] : node_psi<P>(a, (long)ty * a.rs + tx);
  }
  C gx, gy;
  sc_force<C>(psi, C(a.sc_G), gx, gy);
  fx = C(a.fx) + gx;
  fy = C(a.fy) + gy;
}

template <int P, bool HASWALL, int WALL>
__global__ void __launch_bounds__(256) k_step_sc_gather(StepArgs a) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const long i = (long)y * a.rs + x;
  if (HASWALL && a.flags[(long)y * a.pitch + x] != NODE_FLUID) return;  // held in both parities
  C d0, jx0, jy0;
  load_node<P>(a, i, d0, jx0, jy0);
  C own[9];
  if (HASWALL && WALL == WALL_HALFWAY) {
    C fx, fy;
    source_force<P>(a, x, y, fx, fy);
    emit<C>(d0, jx0, jy0, fx, fy, own);
  }
  C g[9];
  {
    C fx, fy;
    source_force<P>(a, x, y, fx, fy);
    C f[9];
    emit<C>(d0, jx0, jy0, fx, fy, f);
    g[0] = f[0];
  }
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    const int sx = wrap_axis(x - kEx[q], a.nx, a.periodic & 1u);
    const int sy = wrap_axis(y - kEy[q], a.ny, a.periodic & 2u);
    bool solid = (sx < 0) || (sy < 0);
    if (HASWALL && !solid) solid = a.flags[(long)sy * a.pitch + sx] == NODE_SOLID;
    if (!solid) {
      C d, jx, jy, fx, fy;
      load_node<P>(a, (long)sy * a.rs + sx, d, jx, jy);
      source_force<P>(a, sx, sy, fx, fy);
      C f[9];
      emit<C>(d, jx, jy, fx, fy, f);
      g[q] = f[q];
    } else if (WALL == WALL_PAPER) {
      g[q] = (q <= 4) ? wall_axis<C>(d0) : wall_diag<C>(d0);
    } else {
      g[q] = own[kInv[q]];
    }
  }
  C dn, jxn, jyn;
  finish<C>(row_sum(g[5], g[2], g[6]), row_dif(g[5], g[6]), row_sum(g[1], g[0], g[3]), row_dif(g[1], g[3]),
            row_sum(g[8], g[4], g[7]), row_dif(g[8], g[7]), dn, jxn, jyn);
  if (T::kScaled) {
    dn *= C(a.is_d);
    jxn *= C(a.is_j);
    jyn *= C(a.is_j);
  }
  static_cast<S *>(a.dst[0])[i] = T::enc(dn);
  static_cast<S *>(a.dst[1])[i] = T::enc(jxn);
  static_cast<S *>(a.dst[2])[i] = T::enc(jyn);
}

template <int P, int VEC, int NY>
__device__ __forceinline__ void sc_strip_body(const StepArgs &a, const int chunk0, const int y0, const int lane) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  using SP = Pack<S, VEC>;
  static_assert(VEC >= 2, "lanes 1..62 are exact only with two or more columns per lane");
  const int ny = a.ny;
  const long rs = a.rs;
  const C sd = C(a.sc_d), sj = C(a.sc_j), ed = C(a.is_d), ej = C(a.is_j);
  const C G = C(a.sc_G), rho0 = C(a.sc_rho0), irho0 = C(1.0 / a.sc_rho0);
  const C bfx = C(a.fx), bfy = C(a.fy);
  const S *__restrict__ s0 = static_cast<const S *>(a.src[0]);
  const S *__restrict__ s1 = static_cast<const S *>(a.src[1]);
  const S *__restrict__ s2 = static_cast<const S *>(a.src[2]);
  S *__restrict__ d0p = static_cast<S *>(a.dst[0]);
  S *__restrict__ d1p = static_cast<S *>(a.dst[1]);
  S *__restrict__ d2p = static_cast<S *>(a.dst[2]);
  const int nch = a.nx / VEC;
  const int ch = chunk0 - 1 + lane;
  const int chw = (ch >= 0 && ch < nch) ? ch : ((ch % nch) + nch) % nch;  // periodic in x
  const int xc = chw * VEC;
  const bool lane_out = lane >= 1 && lane <= 62 && ch < nch;

  struct Row {
    SP raw[3];
  };
  // a decoded row and its pseudopotential, with the edge values of the lanes
  // on either side
  struct Dec {
    C d[VEC], jx[VEC], jy[VEC], psi[VEC];
    C psiL, psiR;  // psi of the column left of this chunk / right of it
  };
  auto load_row = [&](const int i, Row &dst) __attribute__((always_inline)) {
    const long row = wrap_axis(y0 - 2 + i, ny, true);
    const long idx = row * rs + xc;
    dst.raw[0] = *reinterpret_cast<const SP *>(s0 + idx);
    dst.raw[1] = *reinterpret_cast<const SP *>(s1 + idx);
    dst.raw[2] = *reinterpret_cast<const SP *>(s2 + idx);
  };
  auto decode = [&](const Row &r, Dec &o) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      C d = T::dec(r.raw[0].v[v]), jx = T::dec(r.raw[1].v[v]), jy = T::dec(r.raw[2].v[v]);
      if (T::kScaled) {
        d *= sd;
        jx *= sj;
        jy *= sj;
      }
      o.d[v] = d;
      o.jx[v] = jx;
      o.jy[v] = jy;
      o.psi[v] = sc_psi<C>(C(1) + d, rho0, irho0);
    }
    o.psiL = lane_left<P>(o.psi[VEC - 1]);
    o.psiR = lane_right<P>(o.psi[0]);
  };
  auto left = [](const Dec &r, int v) -> C { return v > 0 ? r.psi[v - 1] : r.psiL; };
  auto right = [](const Dec &r, int v) -> C { return v < VEC - 1 ? r.psi[v + 1] : r.psiR; };

  FusedStage<P, VEC> st = {};
  Dec dec[3];
  constexpr int PF = kPrefetch;
  constexpr int NR = NY + 4;
  Row ring[PF + 1];
#pragma unroll
  for (int i = 0; i < PF; ++i) load_row(i, ring[i]);
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    if (i + PF < NR) load_row(i + PF, ring[(i + PF) % (PF + 1)]);
    __builtin_amdgcn_sched_barrier(0);
    decode(ring[i % (PF + 1)], dec[i % 3]);
    if (i < 2) continue;
    // source row i - 1 (lattice row y0 - 3 + i), between rows i - 2 and i
    const Dec &lo = dec[(i + 1) % 3], &mid = dec[(i + 2) % 3], &hi = dec[i % 3];
    C Fx[VEC], Fy[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      C psi[9];
      psi[0] = mid.psi[v];
      psi[1] = right(mid, v);
      psi[2] = hi.psi[v];
      psi[3] = left(mid, v);
      psi[4] = lo.psi[v];
      psi[5] = right(hi, v);
      psi[6] = left(hi, v);
      psi[7] = left(lo, v);
      psi[8] = right(lo, v);
      C gx, gy;
      sc_force<C>(psi, G, gx, gy);
      Fx[v] = bfx + gx;
      Fy[v] = bfy + gy;
    }
    const int j = i - 2;  // index of the source row entering the emission stage
    C dn[VEC], jxn[VEC], jyn[VEC];
    fused_feed<P, VEC>(st, j >= 2, mid.d, mid.jx, mid.jy, Fx, Fy, dn, jxn, jyn);
    if (j < 2) continue;
    SP out[3];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      C x0 = dn[v], x1 = jxn[v], x2 = jyn[v];
      if (T::kScaled) {
        x0 *= ed;
        x1 *= ej;
        x2 *= ej;
      }
      out[0].v[v] = T::enc(x0);
      out[1].v[v] = T::enc(x1);
      out[2].v[v] = T::enc(x2);
    }
    const int t = y0 + i - 4;  // target row completed now
    const bool ok = t < ny && lane_out;
    const long idx = (long)t * rs + xc;
    S *trash = static_cast<S *>(a.trash) + lane * VEC;
    const long tq = kTrashRegion / sizeof(S);
    static_assert(64 * VEC * sizeof(S) <= kTrashRegion, "a wavefront's redirected stores fit one trash region");
    *reinterpret_cast<SP *>(ok ? d0p + idx : trash) = out[0];
    *reinterpret_cast<SP *>(ok ? d1p + idx : trash + tq) = out[1];
    *reinterpret_cast<SP *>(ok ? d2p + idx : trash + 2 * tq) = out[2];
  }
}

// Two multiphase steps per pass (periodic grids without walls).  Each step
// widens the set of wrong halo columns by two (the force needs the neighbours'
// psi, the emission the neighbours' emissions), so lanes 1..62 stay exact for
// two steps only at 4 or more columns per lane.  The wavefront walks NY + 8
// source rows (lattice rows y0 - 4 ...): stage 0 completes rows of step t+1 as
// the single-step body does; each passes through the storage codec as a store
// and reload would, and stage 1 forms its psi, force and emissions from them
// and completes rows of step t+2.  Same arithmetic and order as single steps.
template <int P, int VEC, int NY>
__device__ __forceinline__ void sc_fused_body(const StepArgs &a, const int chunk0, const int y0, const int lane) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  using SP = Pack<S, VEC>;
  static_assert(VEC >= 4, "lanes 1..62 stay exact for two multiphase steps at four or more columns per lane");
  const int ny = a.ny;
  const long rs = a.rs;
  const C sd = C(a.sc_d), sj = C(a.sc_j), ed = C(a.is_d), ej = C(a.is_j);
  const C G = C(a.sc_G), rho0 = C(a.sc_rho0), irho0 = C(1.0 / a.sc_rho0);
  const C bfx = C(a.fx), bfy = C(a.fy);
  const S *__restrict__ s0 = static_cast<const S *>(a.src[0]);
  const S *__restrict__ s1 = static_cast<const S *>(a.src[1]);
  const S *__restrict__ s2 = static_cast<const S *>(a.src[2]);
  S *__restrict__ d0p = static_cast<S *>(a.dst[0]);
  S *__restrict__ d1p = static_cast<S *>(a.dst[1]);
  S *__restrict__ d2p = static_cast<S *>(a.dst[2]);
  const int nch = a.nx / VEC;
  const int ch = chunk0 - 1 + lane;
  const int chw = (ch >= 0 && ch < nch) ? ch : ((ch % nch) + nch) % nch;  // periodic in x
  const int xc = chw * VEC;
  const bool lane_out = lane >= 1 && lane <= 62 && ch < nch;

  struct Row {
    SP raw[3];
  };
  struct Dec {
    C d[VEC], jx[VEC], jy[VEC], psi[VEC];
    C psiL, psiR;
  };
  auto load_row = [&](const int i, Row &dst) __attribute__((always_inline)) {
    const long row = wrap_axis(y0 - 4 + i, ny, true);
    const long idx = row * rs + xc;
    dst.raw[0] = *reinterpret_cast<const SP *>(s0 + idx);
    dst.raw[1] = *reinterpret_cast<const SP *>(s1 + idx);
    dst.raw[2] = *reinterpret_cast<const SP *>(s2 + idx);
  };
  auto decode = [&](const SP (&raw)[3], Dec &o) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      C d = T::dec(raw[0].v[v]), jx = T::dec(raw[1].v[v]), jy = T::dec(raw[2].v[v]);
      if (T::kScaled) {
        d *= sd;
        jx *= sj;
        jy *= sj;
      }
      o.d[v] = d;
      o.jx[v] = jx;
      o.jy[v] = jy;
      o.psi[v] = sc_psi<C>(C(1) + d, rho0, irho0);
    }
    o.psiL = lane_left<P>(o.psi[VEC - 1]);
    o.psiR = lane_right<P>(o.psi[0]);
  };
  auto left = [](const Dec &r, int v) -> C { return v > 0 ? r.psi[v - 1] : r.psiL; };
  auto right = [](const Dec &r, int v) -> C { return v < VEC - 1 ? r.psi[v + 1] : r.psiR; };
  // force on the middle row of three decoded rows, then that row into a stage;
  // when the stage completes a row, it is returned in storage form
  auto stage_row = [&](FusedStage<P, VEC> &st, const Dec &lo, const Dec &mid, const Dec &hi, const int j,
                       SP (&out)[3]) __attribute__((always_inline)) {
    C Fx[VEC], Fy[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      C psi[9];
      psi[0] = mid.psi[v];
      psi[1] = right(mid, v);
      psi[2] = hi.psi[v];
      psi[3] = left(mid, v);
      psi[4] = lo.psi[v];
      psi[5] = right(hi, v);
      psi[6] = left(hi, v);
      psi[7] = left(lo, v);
      psi[8] = right(lo, v);
      C gx, gy;
      sc_force<C>(psi, G, gx, gy);
      Fx[v] = bfx + gx;
      Fy[v] = bfy + gy;
    }
    C dn[VEC], jxn[VEC], jyn[VEC];
    fused_feed<P, VEC>(st, j >= 2, mid.d, mid.jx, mid.jy, Fx, Fy, dn, jxn, jyn);
    if (j < 2) return;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      C x0 = dn[v], x1 = jxn[v], x2 = jyn[v];
      if (T::kScaled) {
        x0 *= ed;
        x1 *= ej;
        x2 *= ej;
      }
      out[0].v[v] = T::enc(x0);
      out[1].v[v] = T::enc(x1);
      out[2].v[v] = T::enc(x2);
    }
  };

  FusedStage<P, VEC> st0 = {}, st1 = {};
  Dec dec0[3], dec1[3];
  constexpr int PF = kPrefetch;
  constexpr int NR = NY + 8;
  Row ring[PF + 1];
#pragma unroll
  for (int i = 0; i < PF; ++i) load_row(i, ring[i]);
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    if (i + PF < NR) load_row(i + PF, ring[(i + PF) % (PF + 1)]);
    __builtin_amdgcn_sched_barrier(0);
    decode(ring[i % (PF + 1)].raw, dec0[i % 3]);
    if (i < 2) continue;
    // stage 0: source row i - 1 between rows i - 2 and i
    SP mid[3];
    stage_row(st0, dec0[(i + 1) % 3], dec0[(i + 2) % 3], dec0[i % 3], i - 2, mid);
    if (i < 4) continue;
    // stage 1 receives row k = i - 4 of step t+1 (lattice row y0 - 2 + k)
    const int k = i - 4;
    decode(mid, dec1[k % 3]);
    if (k < 2) continue;
    SP out[3];
    stage_row(st1, dec1[(k + 1) % 3], dec1[(k + 2) % 3], dec1[k % 3], k - 2, out);
    if (k < 4) continue;
    const int t = y0 + k - 4;  // lattice row of step t+2 completed now
    const bool ok = t < ny && lane_out;
    const long idx = (long)t * rs + xc;
    S *trash = static_cast<S *>(a.trash) + lane * VEC;
    const long tq = kTrashRegion / sizeof(S);
    static_assert(64 * VEC * sizeof(S) <= kTrashRegion, "a wavefront's redirected stores fit one trash region");
    *reinterpret_cast<SP *>(ok ? d0p + idx : trash) = out[0];
    *reinterpret_cast<SP *>(ok ? d1p + idx : trash + tq) = out[1];
    *reinterpret_cast<SP *>(ok ? d2p + idx : trash + 2 * tq) = out[2];
  }
}

template <int P, int VEC, int NY>
__global__ void __launch_bounds__(256) k_step_sc_fused(StepArgs a, StripMap m) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int xcd = blockIdx.x & 7;
  const int local = blockIdx.x >> 3;
  const int begin = xcd * m.per_xcd;
  const int end = min(m.units, begin + m.per_xcd);
  const int stride = m.persistent ? (int)(gridDim.x >> 3) : m.units;
  for (int u = begin + local; u < end; u += stride) {
    const int s = u * 4 + wave;
    const int sy = s / m.strips_x;
    const int sx = s - sy * m.strips_x;
    if (sy < m.strips_y) sc_fused_body<P, VEC, NY>(a, sx * 62, sy * NY, lane);
  }
}

template <int P, int VEC, int NY>
__global__ void __launch_bounds__(256) k_step_sc_strip(StepArgs a, StripMap m) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int xcd = blockIdx.x & 7;
  const int local = blockIdx.x >> 3;
  const int begin = xcd * m.per_xcd;
  const int end = min(m.units, begin + m.per_xcd);
  const int stride = m.persistent ? (int)(gridDim.x >> 3) : m.units;
  for (int u = begin + local; u < end; u += stride) {
    const int s = u * 4 + wave;
    const int sy = s / m.strips_x;
    const int sx = s - sy * m.strips_x;
    if (sy < m.strips_y) sc_strip_body<P, VEC, NY>(a, sx * 62, sy * NY, lane);
  }
}

}  // namespace lbt1

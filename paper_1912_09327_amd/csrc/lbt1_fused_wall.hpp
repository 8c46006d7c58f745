// Two LBMTau1 steps per pass over memory on grids with walls, fixed nodes and
// non-periodic axes (the wall-aware counterpart of lbt1_fused.hpp).
//
// A wavefront walks NY + 4 source rows of its strip.  Stage 0 completes a row
// of step t+1 (the wall rule of Eq. feqnoslip or half-way bounce-back, fixed
// nodes emitting their constant equilibrium) one source row after its last
// source arrived, and feeds it straight into stage 1, which completes rows of
// step t+2 the same way.  An intermediate row passes through the storage codec
// exactly as a store and reload would, and carries its SOLID and FLUID bits
// with it; a non-FLUID node's output is its raw stored value, which never
// changes.  Rows outside a non-periodic axis arrive flagged SOLID, rows of a
// periodic axis wrap, so the intermediate rows above and below the strip are
// exact where the single-step kernel would read them.  Lanes 1..62 stay exact
// for two stages at two or more columns per lane (see lbt1_fused.hpp).
//
// Loads, stores and the store redirection of lanes and rows outside the grid
// are those of the single-step strip kernel; the arithmetic and its order are
// those of strip_body, so two fused steps give the bits of two single steps.
#pragma once
#include "lbt1_fused.hpp"
#include "lbt1_step.hpp"

namespace lbt1 {

template <int P, int WALL, int VEC>
struct WallStage {
  using C = typename Traits<P>::C;
  using SP = Pack<typename Traits<P>::S, VEC>;
  ArrW<C, VEC> upA, upB, lev;
  C own_d[VEC];                                     // pending target row: decoded d
  C own_f[WALL == WALL_HALFWAY ? 9 : 1][VEC];       // and its emissions (half-way rule)
  SP own_raw[3];                                    // and its storage form
  uint32_t own_fluid;                               // and its FLUID bits
};

// One source row into a stage: decoded and scaled values d, jx, jy, storage
// form raw, SOLID and FLUID bits per column.  When emit_row, the pending target
// row (the row before this one) is completed into out (storage form) with its
// SOLID and FLUID bits.
template <int P, int WALL, int VEC, bool UNIT>
__device__ __forceinline__ void wall_feed(WallStage<P, WALL, VEC> &st, const bool odd, const bool emit_row,
                                          const typename Traits<P>::C (&d)[VEC],
                                          const typename Traits<P>::C (&jx)[VEC],
                                          const typename Traits<P>::C (&jy)[VEC],
                                          const Pack<typename Traits<P>::S, VEC> (&raw)[3], const uint32_t sbits,
                                          const uint32_t fbits, const typename Traits<P>::C Fx,
                                          const typename Traits<P>::C Fy, const typename Traits<P>::C ed,
                                          const typename Traits<P>::C ej, Pack<typename Traits<P>::S, VEC> (&out)[3],
                                          uint32_t &out_solid, uint32_t &out_fluid) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  C f[VEC][9];
#pragma unroll
  for (int v = 0; v < VEC; ++v) emit<C>(d[v], jx[v], jy[v], Fx, Fy, f[v]);
  const C L1 = lane_left<P>(f[VEC - 1][1]);
  const C L5 = lane_left<P>(f[VEC - 1][5]);
  const C L8 = lane_left<P>(f[VEC - 1][8]);
  const C R3 = lane_right<P>(f[0][3]);
  const C R6 = lane_right<P>(f[0][6]);
  const C R7 = lane_right<P>(f[0][7]);
  const int Ls = lane_left<P>((int)((sbits >> (VEC - 1)) & 1u));
  const int Rs = lane_right<P>((int)(sbits & 1u));
  auto bit_l = [&](int v) -> uint32_t { return v > 0 ? (sbits >> (v - 1)) & 1u : (uint32_t)Ls; };
  auto bit_r = [&](int v) -> uint32_t { return v < VEC - 1 ? (sbits >> (v + 1)) & 1u : (uint32_t)Rs; };
  ArrW<C, VEC> &up_old = odd ? st.upB : st.upA;

  if (emit_row) {
    uint32_t os = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const C a8 = v > 0 ? f[v - 1][8] : L8;
      const C a4 = f[v][4];
      const C a7 = v < VEC - 1 ? f[v + 1][7] : R7;
      const uint32_t ub = up_old.sb >> (3 * v), lb = st.lev.sb >> (3 * v);
      C w5, w2, w6, w1, w3, w8, w4, w7;
      if constexpr (WALL == WALL_PAPER) {
        w2 = w1 = w3 = w4 = wall_axis<C>(st.own_d[v]);
        w5 = w6 = w8 = w7 = wall_diag<C>(st.own_d[v]);
      } else {
        w5 = st.own_f[7][v];
        w2 = st.own_f[4][v];
        w6 = st.own_f[8][v];
        w1 = st.own_f[3][v];
        w3 = st.own_f[1][v];
        w8 = st.own_f[6][v];
        w4 = st.own_f[2][v];
        w7 = st.own_f[5][v];
      }
      const C g5 = (ub & 1u) ? w5 : up_old.a[0][v];
      const C g2 = (ub & 2u) ? w2 : up_old.a[1][v];
      const C g6 = (ub & 4u) ? w6 : up_old.a[2][v];
      const C g1 = (lb & 1u) ? w1 : st.lev.a[0][v];
      const C g0 = st.lev.a[1][v];
      const C g3 = (lb & 4u) ? w3 : st.lev.a[2][v];
      const C g8 = bit_l(v) ? w8 : a8;
      const C g4 = ((sbits >> v) & 1u) ? w4 : a4;
      const C g7 = bit_r(v) ? w7 : a7;
      C dn, jxn, jyn;
      finish<C>(row_sum(g5, g2, g6), row_dif(g5, g6), row_sum(g1, g0, g3), row_dif(g1, g3), row_sum(g8, g4, g7),
                row_dif(g8, g7), dn, jxn, jyn);
      if (T::kScaled && !UNIT) {
        dn *= ed;
        jxn *= ej;
        jyn *= ej;
      }
      S e0 = T::enc(dn), e1 = T::enc(jxn), e2 = T::enc(jyn);
      if (!((st.own_fluid >> v) & 1u)) {
        e0 = st.own_raw[0].v[v];
        e1 = st.own_raw[1].v[v];
        e2 = st.own_raw[2].v[v];
      }
      out[0].v[v] = e0;
      out[1].v[v] = e1;
      out[2].v[v] = e2;
      os |= ((lb >> 1) & 1u) << v;  // the pending row's own SOLID bit
    }
    out_solid = os;
    out_fluid = st.own_fluid;
  }

  // arrivals of this row for the targets in the next row (up) and this row (level)
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    up_old.a[0][v] = v > 0 ? f[v - 1][5] : L5;
    up_old.a[1][v] = f[v][2];
    up_old.a[2][v] = v < VEC - 1 ? f[v + 1][6] : R6;
    st.lev.a[0][v] = v > 0 ? f[v - 1][1] : L1;
    st.lev.a[1][v] = f[v][0];
    st.lev.a[2][v] = v < VEC - 1 ? f[v + 1][3] : R3;
  }
  uint32_t sb = 0;
#pragma unroll
  for (int v = 0; v < VEC; ++v) sb |= (bit_l(v) | (((sbits >> v) & 1u) << 1) | (bit_r(v) << 2)) << (3 * v);
  up_old.sb = sb;
  st.lev.sb = sb;
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    st.own_d[v] = d[v];
    if constexpr (WALL == WALL_HALFWAY) {
#pragma unroll
      for (int q = 1; q < 9; ++q) st.own_f[q][v] = f[v][q];
    }
  }
  st.own_fluid = fbits;
  st.own_raw[0] = raw[0];
  st.own_raw[1] = raw[1];
  st.own_raw[2] = raw[2];
}

// UNIT: both storage scales are 1 (the default), so the codec's scaling
// multiplications are exact no-ops and are left out.  PF: source rows whose loads
// are in flight ahead of the row being fed.
template <int P, int WALL, int VEC, int NY, bool UNIT, int PF = kPrefetch>
__device__ __forceinline__ void fused_wall_body(const StepArgs &a, const int chunk0, const int y0, const int lane) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  using SP = Pack<S, VEC>;
  using FP = Pack<uint8_t, VEC>;
  static_assert(VEC >= 2, "lanes 1..62 stay exact for two stages at two or more columns per lane");
  static_assert(NY + 4 <= 40, "strip height");

  const int ny = a.ny;
  const long pitch = a.pitch, rs = a.rs;
  const bool px = a.periodic & 1u, py = a.periodic & 2u;
  const C Fx = C(a.fx), Fy = C(a.fy);
  const C sd = C(a.sc_d), sj = C(a.sc_j), ed = C(a.is_d), ej = C(a.is_j);
  const S *__restrict__ s0 = static_cast<const S *>(a.src[0]);
  const S *__restrict__ s1 = static_cast<const S *>(a.src[1]);
  const S *__restrict__ s2 = static_cast<const S *>(a.src[2]);
  S *__restrict__ d0p = static_cast<S *>(a.dst[0]);
  S *__restrict__ d1p = static_cast<S *>(a.dst[1]);
  S *__restrict__ d2p = static_cast<S *>(a.dst[2]);
  // columns as in strip_body: a partial last chunk only where x is not periodic
  const int nch = (a.nx + VEC - 1) / VEC;
  const int ch = chunk0 - 1 + lane;
  bool col_ok = true;
  int chw = ch;
  if (ch < 0 || ch >= nch) {
    if (px)
      chw = ((ch % nch) + nch) % nch;
    else
      col_ok = false;
  }
  const int xc = col_ok ? chw * VEC : 0;
  const bool lane_out = lane >= 1 && lane <= 62 && ch < nch;

  struct Row {
    SP raw[3];
    FP fl;
  };
  // source row i is lattice row y0 - 2 + i; unconditional loads as in strip_body
  auto load_row = [&](const int i, Row &dst) __attribute__((always_inline)) {
    const int rr = wrap_axis(y0 - 2 + i, ny, py);
    const bool row_ok = rr >= 0;
    const long row = row_ok ? rr : 0;
    const long idx = row * rs + xc;
    dst.raw[0] = *reinterpret_cast<const SP *>(s0 + idx);
    dst.raw[1] = *reinterpret_cast<const SP *>(s1 + idx);
    dst.raw[2] = *reinterpret_cast<const SP *>(s2 + idx);
    const FP f = *reinterpret_cast<const FP *>(a.flags + row * pitch + xc);
#pragma unroll
    for (int v = 0; v < VEC; ++v) dst.fl.v[v] = (row_ok && col_ok) ? f.v[v] : (uint8_t)NODE_SOLID;
  };
  auto decode = [&](const SP (&raw)[3], C (&d)[VEC], C (&jx)[VEC], C (&jy)[VEC]) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      d[v] = T::dec(raw[0].v[v]);
      jx[v] = T::dec(raw[1].v[v]);
      jy[v] = T::dec(raw[2].v[v]);
      if (T::kScaled && !UNIT) {
        d[v] *= sd;
        jx[v] *= sj;
        jy[v] *= sj;
      }
    }
  };

  WallStage<P, WALL, VEC> stage[2] = {};
  constexpr int NR = NY + 4;
  Row ring[PF + 1];
#pragma unroll
  for (int i = 0; i < PF; ++i) load_row(i, ring[i]);
#pragma clang loop unroll(full)
  for (int i = 0; i < NR; ++i) {
    if (i + PF < NR) load_row(i + PF, ring[(i + PF) % (PF + 1)]);
    __builtin_amdgcn_sched_barrier(0);
    const Row &cur = ring[i % (PF + 1)];
    uint32_t sbits = 0, fbits = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      sbits |= (uint32_t)(cur.fl.v[v] == NODE_SOLID) << v;
      fbits |= (uint32_t)(cur.fl.v[v] == NODE_FLUID) << v;
    }
    C d[VEC], jx[VEC], jy[VEC];
    decode(cur.raw, d, jx, jy);
    SP mid[3];
    uint32_t ms = 0, mf = 0;
    wall_feed<P, WALL, VEC, UNIT>(stage[0], (i & 1) != 0, i >= 2, d, jx, jy, cur.raw, sbits, fbits, Fx, Fy, ed, ej, mid,
                            ms, mf);
    if (i < 2) continue;
    // stage 1 receives row j = i - 2 (lattice row y0 - 1 + j), a row of step t+1
    const int j = i - 2;
    decode(mid, d, jx, jy);
    SP out[3];
    uint32_t os = 0, of = 0;
    wall_feed<P, WALL, VEC, UNIT>(stage[1], (j & 1) != 0, j >= 2, d, jx, jy, mid, ms, mf, Fx, Fy, ed, ej, out, os, of);
    if (j < 2) continue;
    // rows past ny and lanes past nx write to the trash area (no branch)
    const int t = y0 + j - 2;  // lattice row of step t+2 leaving stage 1
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

template <int P, int WALL, int VEC, int NY>
__global__ void __launch_bounds__(256) k_step_fused_wall(StepArgs a, StripMap m) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int xcd = blockIdx.x & 7;
  const int local = blockIdx.x >> 3;
  const int begin = xcd * m.per_xcd;
  const int end = min(m.units, begin + m.per_xcd);
  const int stride = m.persistent ? (int)(gridDim.x >> 3) : m.units;
  for (int u = begin + local; u < end; u += stride) {
    const int s = u * 4 + wave;  // same strip order as the single-step kernel
    const int sy = s / m.strips_x;
    const int sx = s - sy * m.strips_x;
    if (sy >= m.strips_y) continue;
    // a strip no wall, fixed node or grid edge reaches within two steps takes the
    // wall-free two-step body (same bits; most strips of a large cavity).  Not in
    // FP64, where the two bodies together would spill scalar registers.
    const bool interior = P != P_F64 && strip_interior<VEC>(a, sx * 62, sy * NY, NY, 2);
    const bool unit = !Traits<P>::kScaled || (a.sc_d == 1.0 && a.sc_j == 1.0 && a.is_d == 1.0 && a.is_j == 1.0);
    if constexpr (P != P_F64) {
      if (interior) {
        if (unit)  // wave-uniform
          fused_body<P, VEC, NY, 2, true>(a, sx * 62, sy * NY, lane);
        else
          fused_body<P, VEC, NY, 2, false>(a, sx * 62, sy * NY, lane);
        continue;
      }
    }
    if (unit) {
      fused_wall_body<P, WALL, VEC, NY, true>(a, sx * 62, sy * NY, lane);
    } else {
      fused_wall_body<P, WALL, VEC, NY, false>(a, sx * 62, sy * NY, lane);
    }
  }
}

}  // namespace lbt1

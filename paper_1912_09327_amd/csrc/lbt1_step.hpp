// LBMTau1 step kernels for gfx950 (templates; instantiated in lbt1_kernels.hip).
//
// Two kernel families compute the same update with the same operation order
// (the per-source emission of lbt1_device.hpp and the per-target sums in
// `finish`), so their results are bitwise identical:
//
//  * gather: one thread per node reads its nine upwind neighbours.  Simple,
//    any size; the nine reads per node are served by the caches.
//  * strip: one wavefront walks a strip of NY rows and 62 chunks of VEC
//    columns; each lane owns one chunk.  Every source node's moments are read
//    once per strip and its nine emissions computed once; the emissions that
//    cross to the neighbouring chunk go through a one-lane shuffle.  A strip
//    reads its NY rows plus one halo row above and below, and one halo chunk
//    on each side.
#pragma once
#include <type_traits>

#include "lbt1_args.hpp"
#include "lbt1_device.hpp"

namespace lbt1 {

template <typename S, int VEC>
struct alignas(sizeof(S) * VEC) Pack {
  S v[VEC];
};


// ================================================================ gather kernel
template <int P, bool HASWALL, int WALL>
__device__ __forceinline__ void gather_node(const StepArgs &a, int x, int y) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  const long i = (long)y * a.rs + x;
  if (HASWALL && a.flags[(long)y * a.pitch + x] != NODE_FLUID) return;  // held in both parities
  const C Fx = C(a.fx), Fy = C(a.fy);
  C d0, jx0, jy0;
  load_node<P>(a, i, d0, jx0, jy0);
  C own[9];
  emit<C>(d0, jx0, jy0, Fx, Fy, own);
  C g[9];
  g[0] = own[0];
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    const int sx = wrap_axis(x - kEx[q], a.nx, a.periodic & 1u);
    const int sy = wrap_axis(y - kEy[q], a.ny, a.periodic & 2u);
    bool solid = (sx < 0) || (sy < 0);
    const long s = solid ? 0 : (long)sy * a.rs + sx;
    if (HASWALL && !solid) solid = a.flags[(long)sy * a.pitch + sx] == NODE_SOLID;
    if (!solid) {
      C d, jx, jy;
      load_node<P>(a, s, d, jx, jy);
      C f[9];
      emit<C>(d, jx, jy, Fx, Fy, f);
      g[q] = f[q];
    } else if (WALL == WALL_PAPER) {
      g[q] = (q <= 4) ? wall_axis<C>(d0) : wall_diag<C>(d0);
    } else {
      g[q] = own[kInv[q]];
    }
  }
  C dn, jxn, jyn;
  finish<C>(row_sum(g[5], g[2], g[6]), row_dif(g[5], g[6]), row_sum(g[1], g[0], g[3]),
            row_dif(g[1], g[3]), row_sum(g[8], g[4], g[7]), row_dif(g[8], g[7]), dn, jxn, jyn);
  if (T::kScaled) {
    dn *= C(a.is_d);
    jxn *= C(a.is_j);
    jyn *= C(a.is_j);
  }
  static_cast<S *>(a.dst[0])[i] = T::enc(dn);
  static_cast<S *>(a.dst[1])[i] = T::enc(jxn);
  static_cast<S *>(a.dst[2])[i] = T::enc(jyn);
}

// blockDim (64, 4); grid (ceil(nx/64), ceil(ny/4))
template <int P, bool HASWALL, int WALL>
__global__ void __launch_bounds__(256) k_step_gather(StepArgs a) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  gather_node<P, HASWALL, WALL>(a, x, y);
}

// ================================================================ strip kernel
template <typename C, int VEC>
struct ArrW {  // arrivals from one source row, three per target column, with wall bits
  C a[3][VEC];
  uint32_t sb;  // bit 3*v + k: the source of a[k][v] is a wall
};
template <typename C, int VEC>
struct ArrS {  // the same arrivals already reduced (no walls): row sum and x difference
  C s[VEC];
  C x[VEC];
};


// Rows whose loads are issued ahead of the row being computed.
constexpr int kPrefetch = 2;

// A strip is 62 * VEC output columns by NY output rows.  Lane l of the
// wavefront owns the VEC-column chunk (chunk0 - 1 + l): lanes 1..62 are the
// strip's own chunks, lane 0 and lane 63 load the neighbouring strips' edge
// chunks, so every emission that crosses a chunk boundary comes from the lane
// next door through one shuffle and no separate halo pass is needed.  The halo
// chunks are aligned vector loads of cache lines the neighbouring strips read
// at the same time.
// UNIT: both storage scales are 1 (the default), so the codec's scaling
// multiplications are exact no-ops and are left out.
// COLF (with HASWALL): the caller has checked that every column of the strip's
// footprint carries the same flags in all of its rows (walls that run down whole
// columns, as a grid's sides do away from its top and bottom rows).  The flags are
// then read from one row; whether the columns to the left and right of a column are
// walls, and whether the column is FLUID, is known once for the whole strip; and the
// arrivals from the node's own column (straight up and down) are never from a wall
// when the node is FLUID, so only the six arrivals from the neighbouring columns go
// through a select.  Same values summed in the same order: same bits.
// PF: rows whose loads are in flight ahead of the row being computed.
template <int P, bool HASWALL, int WALL, int VEC, int NY, bool UNIT = false, bool COLF = false, int PF = kPrefetch>
__device__ __forceinline__ void strip_body(const StepArgs &a, const int chunk0, const int y0,
                                           const int lane) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  using SP = Pack<S, VEC>;
  using FP = Pack<uint8_t, VEC>;
  static_assert(NY + 2 <= 32, "strip height");

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
  // chunks per row: VEC divides nx when x is periodic; otherwise the last chunk
  // may run into the row padding, whose flags are SOLID (pitch is a multiple of 64)
  const int nch = (a.nx + VEC - 1) / VEC;
  const int ch = chunk0 - 1 + lane;
  // source chunk: wrapped when x is periodic; outside a non-periodic x it is a wall
  bool col_ok = true;
  int chw = ch;
  if (ch < 0 || ch >= nch) {
    if (px)
      chw = ((ch % nch) + nch) % nch;
    else
      col_ok = false;
  }
  const int xc = col_ok ? chw * VEC : 0;
  const bool lane_out = lane >= 1 && lane <= 62 && ch < nch;  // chunks this strip writes

  using Arr = typename std::conditional<HASWALL, ArrW<C, VEC>, ArrS<C, VEC>>::type;
  Arr upA, upB, lev;
  C own_d[VEC];
  C own_f[HASWALL && WALL == WALL_HALFWAY ? 9 : 1][VEC];
  SP own_raw[3];
  uint32_t own_fluid = 0;
  (void)own_d;
  (void)own_f;
  (void)own_fluid;

  // Source row i of the strip (row y0 - 1 + i) in storage form; rows outside a
  // non-periodic axis read as walls.
  struct Row {
    SP raw[3];
    FP fl;
  };
  // The loads are unconditional (chunks and rows outside a non-periodic axis
  // read column 0 / row 0 instead and are flagged as walls): with no branch
  // around them the compiler keeps exact track of the loads in flight, which
  // is what lets the prefetch overlap.
  auto load_row = [&](const int i, Row &dst) __attribute__((always_inline)) {
    const int rr = wrap_axis(y0 - 1 + i, ny, py);
    const bool row_ok = rr >= 0;
    const long row = row_ok ? rr : 0;
    const long col = xc;
    const long idx = row * rs + col;
    dst.raw[0] = *reinterpret_cast<const SP *>(s0 + idx);
    dst.raw[1] = *reinterpret_cast<const SP *>(s1 + idx);
    dst.raw[2] = *reinterpret_cast<const SP *>(s2 + idx);
    if (HASWALL && !COLF) {
      const FP f = *reinterpret_cast<const FP *>(a.flags + row * pitch + col);
#pragma unroll
      for (int v = 0; v < VEC; ++v) dst.fl.v[v] = (row_ok && col_ok) ? f.v[v] : (uint8_t)NODE_SOLID;
    }
  };

  // the flags of every row of a COLF strip: those of its first row
  FP cfl;
  if (HASWALL && COLF) {
    const int rr = wrap_axis(y0 - 1, ny, py);
    const FP f = *reinterpret_cast<const FP *>(a.flags + (long)(rr >= 0 ? rr : 0) * pitch + xc);
#pragma unroll
    for (int v = 0; v < VEC; ++v) cfl.v[v] = col_ok ? f.v[v] : (uint8_t)NODE_SOLID;
  }
  (void)cfl;
  // COLF: the column left of column v is a wall (cwl), the one right of it (cwr),
  // column v is FLUID (cfo)
  bool cwl[VEC], cwr[VEC], cfo[VEC];
  if constexpr (HASWALL && COLF) {
    uint32_t sb = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      sb |= (uint32_t)(cfl.v[v] == NODE_SOLID) << v;
      cfo[v] = cfl.v[v] == NODE_FLUID;
    }
    const int Ls = lane_left<P>((int)((sb >> (VEC - 1)) & 1u));
    const int Rs = lane_right<P>((int)(sb & 1u));
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      cwl[v] = v > 0 ? ((sb >> (v - 1)) & 1u) != 0 : Ls != 0;
      cwr[v] = v < VEC - 1 ? ((sb >> (v + 1)) & 1u) != 0 : Rs != 0;
    }
  }
  (void)cwl;
  (void)cwr;
  (void)cfo;
  // COLF: non-FLUID columns keep their stored values.  Where a chunk's values fill
  // whole 32-bit words, that is a blend of each word of the new values with the old
  // under a mask formed once (the 16-bit values stay packed); else one select each.
  constexpr bool kWordBlend = (sizeof(S) * VEC) % 4 == 0;
  constexpr int kWords = kWordBlend ? (int)(sizeof(S) * VEC / 4) : 1;
  uint32_t ckeep[kWords];
  if constexpr (HASWALL && COLF && kWordBlend) {
#pragma unroll
    for (int w = 0; w < kWords; ++w) {
      uint32_t m = 0;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int b0 = v * (int)sizeof(S), b1 = b0 + (int)sizeof(S);  // bytes of value v
        if (b0 < 4 * (w + 1) && b1 > 4 * w && !cfo[v]) {
          const int lo = (b0 > 4 * w ? b0 - 4 * w : 0) * 8, hi = (b1 < 4 * (w + 1) ? b1 - 4 * w : 4) * 8;
          m |= (hi - lo == 32 ? 0xffffffffu : ((1u << (hi - lo)) - 1u)) << lo;
        }
      }
      ckeep[w] = m;
    }
  }
  (void)ckeep;

  // Row i is processed while the loads of the following PF rows are in flight.
  auto body = [&](const int i, Arr &up_old, const Row &cur) __attribute__((always_inline)) {
    const int r = y0 - 1 + i;
    const SP *raw = cur.raw;
    const FP &fl = COLF ? cfl : cur.fl;
    C f[VEC][9];
    C dd[VEC];
    uint32_t sbits = 0, fbits = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      C d = T::dec(raw[0].v[v]), jx = T::dec(raw[1].v[v]), jy = T::dec(raw[2].v[v]);
      if (T::kScaled && !UNIT) {
        d *= sd;
        jx *= sj;
        jy *= sj;
      }
      dd[v] = d;
      emit<C>(d, jx, jy, Fx, Fy, f[v]);
      if (HASWALL && !COLF) {
        sbits |= (uint32_t)(fl.v[v] == NODE_SOLID) << v;
        fbits |= (uint32_t)(fl.v[v] == NODE_FLUID) << v;
      }
    }
    (void)dd;
    (void)fbits;
    // neighbour-lane emissions: heading +x from the lane on the left, -x from
    // the right (lanes 0 and 63 receive nothing useful; they write nothing)
    const C L1 = lane_left<P>(f[VEC - 1][1]);
    const C L5 = lane_left<P>(f[VEC - 1][5]);
    const C L8 = lane_left<P>(f[VEC - 1][8]);
    const C R3 = lane_right<P>(f[0][3]);
    const C R6 = lane_right<P>(f[0][6]);
    const C R7 = lane_right<P>(f[0][7]);
    int Ls = 0, Rs = 0;
    if (HASWALL && !COLF) {
      Ls = lane_left<P>((int)((sbits >> (VEC - 1)) & 1u));
      Rs = lane_right<P>((int)(sbits & 1u));
    }
    // wall bits of the left / own / right source of column v
    auto bit_l = [&](int v) -> uint32_t { return v > 0 ? (sbits >> (v - 1)) & 1u : (uint32_t)Ls; };
    auto bit_r = [&](int v) -> uint32_t { return v < VEC - 1 ? (sbits >> (v + 1)) & 1u : (uint32_t)Rs; };

    // ---- target row r - 1: arrivals from rows r - 2 (up_old), r - 1 (lev), r (here)
    if (i >= 2) {
      const int t = r - 1;
      SP out[3];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const C a8 = v > 0 ? f[v - 1][8] : L8;
        const C a4 = f[v][4];
        const C a7 = v < VEC - 1 ? f[v + 1][7] : R7;
        C dn, jxn, jyn;
        if constexpr (HASWALL) {
          const uint32_t ub = up_old.sb >> (3 * v), lb = lev.sb >> (3 * v);
          C w5, w2, w6, w1, w3, w8, w4, w7;
          if constexpr (WALL == WALL_PAPER) {
            w2 = w1 = w3 = w4 = wall_axis<C>(own_d[v]);
            w5 = w6 = w8 = w7 = wall_diag<C>(own_d[v]);
          } else {
            w5 = own_f[7][v];
            w2 = own_f[4][v];
            w6 = own_f[8][v];
            w1 = own_f[3][v];
            w3 = own_f[1][v];
            w8 = own_f[6][v];
            w4 = own_f[2][v];
            w7 = own_f[5][v];
          }
          C g5, g2, g6, g1, g3, g8, g4, g7;
          if constexpr (COLF) {
            (void)ub;
            (void)lb;
            (void)w2;
            (void)w4;
            g5 = cwl[v] ? w5 : up_old.a[0][v];
            g2 = up_old.a[1][v];
            g6 = cwr[v] ? w6 : up_old.a[2][v];
            g1 = cwl[v] ? w1 : lev.a[0][v];
            g3 = cwr[v] ? w3 : lev.a[2][v];
            g8 = cwl[v] ? w8 : a8;
            g4 = a4;
            g7 = cwr[v] ? w7 : a7;
          } else {
            g5 = (ub & 1u) ? w5 : up_old.a[0][v];
            g2 = (ub & 2u) ? w2 : up_old.a[1][v];
            g6 = (ub & 4u) ? w6 : up_old.a[2][v];
            g1 = (lb & 1u) ? w1 : lev.a[0][v];
            g3 = (lb & 4u) ? w3 : lev.a[2][v];
            g8 = bit_l(v) ? w8 : a8;
            g4 = ((sbits >> v) & 1u) ? w4 : a4;
            g7 = bit_r(v) ? w7 : a7;
          }
          const C g0 = lev.a[1][v];
          finish<C>(row_sum(g5, g2, g6), row_dif(g5, g6), row_sum(g1, g0, g3), row_dif(g1, g3),
                    row_sum(g8, g4, g7), row_dif(g8, g7), dn, jxn, jyn);
        } else {
          finish<C>(up_old.s[v], up_old.x[v], lev.s[v], lev.x[v], row_sum(a8, a4, a7),
                    row_dif(a8, a7), dn, jxn, jyn);
        }
        if (T::kScaled && !UNIT) {
          dn *= ed;
          jxn *= ej;
          jyn *= ej;
        }
        S e0 = T::enc(dn), e1 = T::enc(jxn), e2 = T::enc(jyn);
        if (HASWALL && !(COLF && kWordBlend) && !(COLF ? cfo[v] : ((own_fluid >> v) & 1u) != 0)) {
          e0 = own_raw[0].v[v];
          e1 = own_raw[1].v[v];
          e2 = own_raw[2].v[v];
        }
        out[0].v[v] = e0;
        out[1].v[v] = e1;
        out[2].v[v] = e2;
      }
      if constexpr (HASWALL && COLF && kWordBlend) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          uint32_t nw[kWords], ow[kWords];
          __builtin_memcpy(nw, &out[q], sizeof(nw));
          __builtin_memcpy(ow, &own_raw[q], sizeof(ow));
#pragma unroll
          for (int w = 0; w < kWords; ++w) nw[w] = (ow[w] & ckeep[w]) | (nw[w] & ~ckeep[w]);
          __builtin_memcpy(&out[q], nw, sizeof(nw));
        }
      }
      {
        // rows past ny and lanes past nx write to the trash area (no branch)
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

    // ---- arrivals of this row for targets in rows r + 1 (into up_old) and r (into lev)
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const C a5 = v > 0 ? f[v - 1][5] : L5;
      const C a2 = f[v][2];
      const C a6 = v < VEC - 1 ? f[v + 1][6] : R6;
      const C a1 = v > 0 ? f[v - 1][1] : L1;
      const C a0 = f[v][0];
      const C a3 = v < VEC - 1 ? f[v + 1][3] : R3;
      if constexpr (HASWALL) {
        up_old.a[0][v] = a5;
        up_old.a[1][v] = a2;
        up_old.a[2][v] = a6;
        lev.a[0][v] = a1;
        lev.a[1][v] = a0;
        lev.a[2][v] = a3;
      } else {
        up_old.s[v] = row_sum(a5, a2, a6);
        up_old.x[v] = row_dif(a5, a6);
        lev.s[v] = row_sum(a1, a0, a3);
        lev.x[v] = row_dif(a1, a3);
      }
    }
    if constexpr (HASWALL) {
      if constexpr (!COLF) {
        uint32_t sb = 0;
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          sb |= (bit_l(v) | (((sbits >> v) & 1u) << 1) | (bit_r(v) << 2)) << (3 * v);
        up_old.sb = sb;
        lev.sb = sb;
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        own_d[v] = dd[v];
        if constexpr (WALL == WALL_HALFWAY) {
#pragma unroll
          for (int q = 1; q < 9; ++q) own_f[q][v] = f[v][q];
        }
      }
      own_fluid = fbits;
      own_raw[0] = raw[0];
      own_raw[1] = raw[1];
      own_raw[2] = raw[2];
    }
  };

  // Fully unrolled so that every ring slot and up-buffer role is static.
  Row ring[PF + 1];
#pragma unroll
  for (int i = 0; i < PF; ++i) load_row(i, ring[i]);
#pragma unroll
  for (int i = 0; i < NY + 2; ++i) {
    if (i + PF < NY + 2) load_row(i + PF, ring[(i + PF) % (PF + 1)]);
    // keep the scheduler from sinking those loads down to their use
    __builtin_amdgcn_sched_barrier(0);
    body(i, (i & 1) ? upB : upA, ring[i % (PF + 1)]);
  }
}

// ================================================================ strip kinds

// True when every node whose emissions reach a stored node of the strip at
// (chunk0, y0) through HALO steps is a FLUID node inside the grid: the stored
// chunks [chunk0, min(nch, chunk0 + 62)) widened by HALO columns on either side
// and its NY rows widened by HALO rows above and below, with no row or column
// across an axis.  Such a strip takes the wall-free body, which gives the same bits
// (the wall rule only ever replaces arrivals from SOLID sources, and the sums run
// in the same order).  The halo lanes' other columns feed only nodes that are not
// stored.  HALO <= VEC.  Wave-uniform: the flags are OR-ed per lane, then voted.
template <int VEC>
__device__ __forceinline__ bool strip_interior(const StepArgs &a, const int chunk0, const int y0, const int NY,
                                               const int HALO) {
  const int nch = (a.nx + VEC - 1) / VEC;
  const int ce = min(nch, chunk0 + 62);
  if (chunk0 < 1 || ce <= chunk0 || ce * VEC + HALO > a.nx || y0 < HALO || y0 + NY + HALO > a.ny) return false;
  const int lane = threadIdx.x & 63;
  const int ch = chunk0 - 1 + lane;
  // columns [lo, hi) of this lane's chunk that the stored nodes draw on
  const int lo = ch == chunk0 - 1 ? VEC - HALO : 0;
  const int hi = ch == ce ? HALO : (ch < ce ? VEC : 0);
  uint32_t any = 0;
  if (hi > lo) {
    // ch <= ce and ce * VEC < nx, so the pack lies inside the row's pitch
    const uint8_t *f = a.flags + (long)(y0 - HALO) * a.pitch + (long)ch * VEC;
    for (int i = 0; i < NY + 2 * HALO; ++i) {
      const Pack<uint8_t, VEC> p = *reinterpret_cast<const Pack<uint8_t, VEC> *>(f + (long)i * a.pitch);
#pragma unroll
      for (int v = 0; v < VEC; ++v) any |= (v >= lo && v < hi) ? p.v[v] : 0u;
    }
  }
  return __ballot(any != 0) == 0;
}

// True when the flags the wall-aware strip body loads for the strip at (chunk0,
// y0) -- rows y0 - HALO .. y0 + NY + HALO - 1 of its 64 lanes' chunks, wrapped on a
// periodic axis, SOLID outside a non-periodic x -- are the same in every row of
// each column, and no row lies across a non-periodic y.  The body may then take the
// flags of one row for all (COLF).  Wave-uniform.
template <int VEC>
__device__ __forceinline__ bool strip_colwall(const StepArgs &a, const int chunk0, const int y0, const int NY,
                                              const int HALO) {
  const bool py = a.periodic & 2u;
  if (!py && (y0 < HALO || y0 + NY + HALO > a.ny)) return false;
  const int lane = threadIdx.x & 63;
  const int nch = (a.nx + VEC - 1) / VEC;
  const int ch = chunk0 - 1 + lane;
  int chw = ch;
  bool col_ok = true;
  if (ch < 0 || ch >= nch) {
    if (a.periodic & 1u)
      chw = ((ch % nch) + nch) % nch;
    else
      col_ok = false;  // read as SOLID in every row
  }
  uint32_t diff = 0;
  if (col_ok) {
    const uint8_t *f = a.flags + (long)chw * VEC;
    const Pack<uint8_t, VEC> p0 =
        *reinterpret_cast<const Pack<uint8_t, VEC> *>(f + (long)wrap_axis(y0 - HALO, a.ny, py) * a.pitch);
    for (int i = 1; i < NY + 2 * HALO; ++i) {
      const int rr = wrap_axis(y0 - HALO + i, a.ny, py);
      const Pack<uint8_t, VEC> p = *reinterpret_cast<const Pack<uint8_t, VEC> *>(f + (long)rr * a.pitch);
#pragma unroll
      for (int v = 0; v < VEC; ++v) diff |= (uint32_t)(p.v[v] ^ p0.v[v]);
    }
  }
  return __ballot(diff != 0) == 0;
}

template <int P, bool HASWALL, int WALL, int VEC, int NY>
__global__ void __launch_bounds__(256) k_step_strip(StepArgs a, StripMap m) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int xcd = blockIdx.x & 7;
  const int local = blockIdx.x >> 3;
  const int begin = xcd * m.per_xcd;
  const int end = min(m.units, begin + m.per_xcd);
  const int stride = m.persistent ? (int)(gridDim.x >> 3) : m.units;
  for (int u = begin + local; u < end; u += stride) {
    // strips ordered along each row band (x fastest): the waves of a block and
    // the blocks of an XCD work on horizontally adjacent strips at the same
    // time, so the cache lines holding a strip's halo columns are the ones its
    // neighbours are reading, and the halo rows of the next band follow soon
    const int s = u * 4 + wave;
    const int sy = s / m.strips_x;
    const int sx = s - sy * m.strips_x;
    if (sy < m.strips_y) strip_body<P, HASWALL, WALL, VEC, NY>(a, sx * 62, sy * NY, lane);
  }
}

// ================================================================ reductions

// out slots: 0 sum d, 1 sum jx, 2 sum jy, 3 max residual, 4 non-finite, 5 fluid count
template <int P>
__global__ void __launch_bounds__(256) k_reduce_partial(ReduceArgs a) {
  using T = Traits<P>;
  using S = typename T::S;
  const S *c0 = static_cast<const S *>(a.cur[0]);
  const S *c1 = static_cast<const S *>(a.cur[1]);
  const S *c2 = static_cast<const S *>(a.cur[2]);
  S *n0 = static_cast<S *>(a.snap[0]);
  S *n1 = static_cast<S *>(a.snap[1]);
  S *n2 = static_cast<S *>(a.snap[2]);
  const bool want_res = a.what & 4u;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const long n = (long)a.nx * a.ny;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int y = (int)(k / a.nx);
    const int x = (int)(k - (long)y * a.nx);
    const long i = (long)y * a.rs + x;
    if (a.flags && a.flags[(long)y * a.pitch + x] != NODE_FLUID) continue;
    const S r0 = c0[i], r1 = c1[i], r2 = c2[i];
    const double d = (double)T::dec(r0) * a.sc_d;
    const double jx = (double)T::dec(r1) * a.sc_j;
    const double jy = (double)T::dec(r2) * a.sc_j;
    acc[0] += d;
    acc[1] += jx;
    acc[2] += jy;
    acc[4] += (__builtin_isfinite(d) && __builtin_isfinite(jx) && __builtin_isfinite(jy)) ? 0.0 : 1.0;
    acc[5] += 1.0;
    if (want_res) {
      const double rho = 1.0 + d;
      const double sr = 1.0 + (double)T::dec(n0[i]) * a.sc_d;
      const double su = (double)T::dec(n1[i]) * a.sc_j / sr;
      const double sv = (double)T::dec(n2[i]) * a.sc_j / sr;
      const double du = __builtin_fabs(jx / rho - su);
      const double dv = __builtin_fabs(jy / rho - sv);
      acc[3] = __builtin_fmax(acc[3], __builtin_fmax(du, dv));
      n0[i] = r0;
      n1[i] = r1;
      n2[i] = r2;
    }
  }
  // wavefront tree (fixed order), then the four waves of the block in order
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
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) part[wave][q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int q = threadIdx.x;
    double v = part[0][q];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      v = q == 3 ? __builtin_fmax(v, part[w][q]) : v + part[w][q];
    a.partials[blockIdx.x * 6 + q] = v;
  }
}


}  // namespace lbt1

// Temporally fused strip kernel: K LBMTau1 steps per pass over memory, for
// grids that are periodic in both axes and have no wall or fixed nodes.
//
// The update of a node needs only its 3 x 3 neighbourhood of the previous
// step (Algorithm 1), so a strip can carry a row through K steps in registers
// before it is stored: the wavefront walks NY + 2K source rows; stage 0
// computes step t+1 of a row as soon as the source row below it has arrived,
// stage 1 turns three finished rows of step t+1 into one row of step t+2, and
// so on.  Each row leaves stage s one row after it entered, so the last stage
// emits the strip's NY rows of step t+K.  The state crosses HBM once per K
// steps: 2 * 3 * c bytes per node per pass instead of per step.
//
// Columns: lane l owns the VEC-column chunk (chunk0 - 1 + l) exactly as in
// the single-step strip kernel.  Lanes 0 and 63 have no neighbour on their
// outer side, so after s stages their s outermost columns are wrong; lanes
// 1..62 stay exact as long as K <= VEC, and only they store.
//
// Every stage uses the per-source emission and per-target summation order of
// the single-step kernels, and an intermediate row passes through the storage
// codec (encode, then decode) exactly as if it had been stored and reloaded,
// so K fused steps give the same bits as K single steps.
#pragma once
#include "lbt1_step.hpp"

namespace lbt1 {

// Per column of a stage: the partial sums of the pending target row (the one
// completed by the next source row) and the up-sums of the newest source row.
// The finish step adds the up and level sums of a target first, so they are
// combined as soon as the level sum is known: ps = up.s + lev.s, px = up.x +
// lev.x; us keeps up.s alone for the y momentum.
template <int P, int VEC>
struct FusedStage {
  using C = typename Traits<P>::C;
  C ps[VEC], px[VEC], us[VEC];  // pending target row
  C ns[VEC], nx[VEC];           // up-sums of the newest source row
};

// One source row j into stage `st` (values already decoded and scaled; Fx, Fy
// the force of each source column).  When `emit_row` (the stage has seen two
// earlier rows), target row j - 1 is completed into dn/jxn/jyn (unscaled
// arithmetic values); the same additions in the same order as finish().
template <int P, int VEC>
__device__ __forceinline__ void fused_feed(FusedStage<P, VEC> &st, const bool emit_row,
                                           const typename Traits<P>::C (&d)[VEC],
                                           const typename Traits<P>::C (&jx)[VEC],
                                           const typename Traits<P>::C (&jy)[VEC],
                                           const typename Traits<P>::C (&Fx)[VEC],
                                           const typename Traits<P>::C (&Fy)[VEC], typename Traits<P>::C (&dn)[VEC],
                                           typename Traits<P>::C (&jxn)[VEC], typename Traits<P>::C (&jyn)[VEC]) {
  using C = typename Traits<P>::C;
  C f[VEC][9];
#pragma unroll
  for (int v = 0; v < VEC; ++v) emit<C>(d[v], jx[v], jy[v], Fx[v], Fy[v], f[v]);
  const C L1 = lane_left<P>(f[VEC - 1][1]);
  const C L5 = lane_left<P>(f[VEC - 1][5]);
  const C L8 = lane_left<P>(f[VEC - 1][8]);
  const C R3 = lane_right<P>(f[0][3]);
  const C R6 = lane_right<P>(f[0][6]);
  const C R7 = lane_right<P>(f[0][7]);
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const C a8 = v > 0 ? f[v - 1][8] : L8;
    const C a4 = f[v][4];
    const C a7 = v < VEC - 1 ? f[v + 1][7] : R7;
    if (emit_row) {
      const C ds = row_sum(a8, a4, a7), dx = row_dif(a8, a7);
      dn[v] = st.ps[v] + ds;
      jxn[v] = st.px[v] + dx;
      jyn[v] = st.us[v] - ds;
    }
    const C a1 = v > 0 ? f[v - 1][1] : L1;
    const C a0 = f[v][0];
    const C a3 = v < VEC - 1 ? f[v + 1][3] : R3;
    const C ls = row_sum(a1, a0, a3), lx = row_dif(a1, a3);
    // target row j: up-sums of row j - 1 plus the level sums of row j
    st.ps[v] = st.ns[v] + ls;
    st.px[v] = st.nx[v] + lx;
    st.us[v] = st.ns[v];
    const C a5 = v > 0 ? f[v - 1][5] : L5;
    const C a2 = f[v][2];
    const C a6 = v < VEC - 1 ? f[v + 1][6] : R6;
    st.ns[v] = row_sum(a5, a2, a6);
    st.nx[v] = row_dif(a5, a6);
  }
}

// The same stage for a strip walked upwards (source rows in decreasing order):
// a target row is completed by the row below it, its last source.  It keeps the
// level sums of the pending target and the down-sums of the row above it apart
// until then, so the target's sums are still formed as finish() forms them,
// (row below + level) + row above: the same bits as the downward walk.
template <int P, int VEC>
struct FusedStageUp {
  using C = typename Traits<P>::C;
  C ls[VEC], lx[VEC];  // pending target row: level sums
  C ps[VEC], px[VEC];  // and the down-sums of the row above it
  C ns[VEC], nx[VEC];  // down-sums of the newest source row
};

template <int P, int VEC>
__device__ __forceinline__ void fused_feed(FusedStageUp<P, VEC> &st, const bool emit_row,
                                           const typename Traits<P>::C (&d)[VEC],
                                           const typename Traits<P>::C (&jx)[VEC],
                                           const typename Traits<P>::C (&jy)[VEC],
                                           const typename Traits<P>::C (&Fx)[VEC],
                                           const typename Traits<P>::C (&Fy)[VEC], typename Traits<P>::C (&dn)[VEC],
                                           typename Traits<P>::C (&jxn)[VEC], typename Traits<P>::C (&jyn)[VEC]) {
  using C = typename Traits<P>::C;
  C f[VEC][9];
#pragma unroll
  for (int v = 0; v < VEC; ++v) emit<C>(d[v], jx[v], jy[v], Fx[v], Fy[v], f[v]);
  const C L1 = lane_left<P>(f[VEC - 1][1]);
  const C L5 = lane_left<P>(f[VEC - 1][5]);
  const C L8 = lane_left<P>(f[VEC - 1][8]);
  const C R3 = lane_right<P>(f[0][3]);
  const C R6 = lane_right<P>(f[0][6]);
  const C R7 = lane_right<P>(f[0][7]);
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    // up-sums of this row complete the target row above it
    const C a5 = v > 0 ? f[v - 1][5] : L5;
    const C a2 = f[v][2];
    const C a6 = v < VEC - 1 ? f[v + 1][6] : R6;
    const C us = row_sum(a5, a2, a6), ux = row_dif(a5, a6);
    if (emit_row) {
      dn[v] = (us + st.ls[v]) + st.ps[v];
      jxn[v] = (ux + st.lx[v]) + st.px[v];
      jyn[v] = us - st.ps[v];
    }
    // this row becomes the pending target: its level sums, and the down-sums of
    // the row above it (the previous source row)
    const C a1 = v > 0 ? f[v - 1][1] : L1;
    const C a0 = f[v][0];
    const C a3 = v < VEC - 1 ? f[v + 1][3] : R3;
    st.ls[v] = row_sum(a1, a0, a3);
    st.lx[v] = row_dif(a1, a3);
    st.ps[v] = st.ns[v];
    st.px[v] = st.nx[v];
    const C a8 = v > 0 ? f[v - 1][8] : L8;
    const C a4 = f[v][4];
    const C a7 = v < VEC - 1 ? f[v + 1][7] : R7;
    st.ns[v] = row_sum(a8, a4, a7);
    st.nx[v] = row_dif(a8, a7);
  }
}

// UNIT: both storage scales are 1 (the default), so the codec's scaling
// multiplications are exact no-ops and are left out.  UP: the strip is walked
// upwards, from its last halo row to its first (see k_step_fused).
template <int P, int VEC, int NY, int K, bool UNIT, bool UP = false>
__device__ __forceinline__ void fused_body(const StepArgs &a, const int chunk0, const int y0, const int lane) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  using SP = Pack<S, VEC>;
  static_assert(K >= 2 && K <= VEC, "lanes 1..62 stay exact for K <= VEC");
  static_assert(NY + 2 * K <= 40, "strip height");

  const int ny = a.ny;
  const long rs = a.rs;
  C Fx[VEC], Fy[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    Fx[v] = C(a.fx);
    Fy[v] = C(a.fy);
  }
  const C sd = C(a.sc_d), sj = C(a.sc_j), ed = C(a.is_d), ej = C(a.is_j);
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
  auto load_row = [&](const int i, Row &dst) __attribute__((always_inline)) {
    const long row = wrap_axis(UP ? y0 + NY + K - 1 - i : y0 - K + i, ny, true);
    const long idx = row * rs + xc;
    dst.raw[0] = *reinterpret_cast<const SP *>(s0 + idx);
    dst.raw[1] = *reinterpret_cast<const SP *>(s1 + idx);
    dst.raw[2] = *reinterpret_cast<const SP *>(s2 + idx);
  };
  // storage value -> arithmetic value, as a load of the next step would see it
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
  auto encode = [&](const C (&d)[VEC], const C (&jx)[VEC], const C (&jy)[VEC], SP (&out)[3]) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      C x0 = d[v], x1 = jx[v], x2 = jy[v];
      if (T::kScaled && !UNIT) {
        x0 *= ed;
        x1 *= ej;
        x2 *= ej;
      }
      out[0].v[v] = T::enc(x0);
      out[1].v[v] = T::enc(x1);
      out[2].v[v] = T::enc(x2);
    }
  };

  using Stage = typename std::conditional<UP, FusedStageUp<P, VEC>, FusedStage<P, VEC>>::type;
  Stage stage[K] = {};
  // Two steps: one wavefront per SIMD is enough registers for a ring of rows
  // loaded two ahead.  Three steps: the kernel is built for two wavefronts per
  // SIMD, which leaves room for one row in flight ahead of the row being fed
  // (12 VGPRs at four FP32 columns per lane; 6.3-6.8 % less time per launch at
  // 8192^2 than loading each row as it is needed).
  constexpr int PF = K >= 3 ? 1 : kPrefetch;
  constexpr int NR = NY + 2 * K;
  Row ring[PF + 1];
#pragma unroll
  for (int i = 0; i < PF; ++i) load_row(i, ring[i]);
#pragma clang loop unroll(full)
  for (int i = 0; i < NR; ++i) {
    if (i + PF < NR) load_row(i + PF, ring[(i + PF) % (PF + 1)]);
    if (PF > 0) __builtin_amdgcn_sched_barrier(0);
    C d[VEC], jx[VEC], jy[VEC];
    decode(ring[i % (PF + 1)].raw, d, jx, jy);
    // stage s receives its (i - 2s)-th row at iteration i
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int j = i - 2 * s;  // index of the row entering stage s
      // three steps: one stage at a time, so the stages' temporaries are not
      // live together
      if (K >= 3) __builtin_amdgcn_sched_barrier(0);
      if (j >= 0) {
        C dn[VEC], jxn[VEC], jyn[VEC];
        fused_feed<P, VEC>(stage[s], j >= 2, d, jx, jy, Fx, Fy, dn, jxn, jyn);
        if (j < 2) break;  // nothing leaves stage s yet, so later stages get nothing
        SP out[3];
        encode(dn, jxn, jyn, out);
        if (s + 1 < K) {
          decode(out, d, jx, jy);
        } else {
          const int t = UP ? y0 + NY - 1 - (i - 2 * K) : y0 + i - 2 * K;  // row leaving the last stage
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
    }
  }
}

template <int P, int VEC, int NY, int K>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K >= 3 ? 2 : 1)))
k_step_fused(StepArgs a, StripMap m) {
  const int lane = threadIdx.x & 63;
  // three steps: the wavefront index read as a wave-uniform value keeps the
  // strip coordinates and their divisions in scalar registers (the vector
  // registers are all taken at two wavefronts per SIMD)
  const int wave = K >= 3 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x >> 6);
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
    if constexpr (Traits<P>::kScaled) {
      // 16-bit storage is bound by vector-ALU issue: with unit scales (wave-uniform
      // test) the body without the scaling multiplications runs
      if (a.sc_d == 1.0 && a.sc_j == 1.0 && a.is_d == 1.0 && a.is_j == 1.0)
        fused_body<P, VEC, NY, K, true>(a, sx * 62, sy * NY, lane);
      else
        fused_body<P, VEC, NY, K, false>(a, sx * 62, sy * NY, lane);
    } else if (P == P_F32 && (sy & 1)) {
      // FP32: odd row bands walk upwards.  A downward strip reads the halo rows it
      // shares with the band below at the end of its walk and the band below
      // reads them at the start of its own; with alternate directions two
      // neighbouring bands read their shared rows at the same end of their walks,
      // while the first copy is still in L2.  (FP64 strips, six rows tall by
      // default, measured 3 % slower so; 16-bit storage is bound by arithmetic.)
      fused_body<P, VEC, NY, K, true, true>(a, sx * 62, sy * NY, lane);
    } else {
      fused_body<P, VEC, NY, K, true>(a, sx * 62, sy * NY, lane);
    }
  }
}

}  // namespace lbt1

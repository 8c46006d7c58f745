// Batched step kernels beyond one step per launch (templates; instantiated in
// lbt1_kernels.hip).  They run over the same flattened (grid, strip) item lists
// and grid descriptors as k_step_batch, with the arithmetic and its order of the
// single-grid kernels, so every grid gets the bits it would get alone.
#pragma once
#include "lbt1_fused.hpp"
#include "lbt1_fused_wall.hpp"

namespace lbt1 {

// Two steps per launch (the fused class, two columns per lane): launch s of a
// burst covers steps 2s and 2s + 1 of every grid in the class and flips its
// parity once.  A grid with an odd number of steps in the burst takes its last
// step in the single-step body of the same strip shape.
template <int P, int NY>
__global__ void __launch_bounds__(256) k_step_batch_fused(BatchStepArgs b) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = *b.count;
  for (int it = blockIdx.x * 4 + wave; it < n; it += gridDim.x * 4) {
    const int2 item = b.items[it];
    const BatchGrid &g = b.grids[item.x];
    const int left = g.steps_left - 2 * b.step;  // steps this grid still takes in the burst
    if (left <= 0) continue;
    const StepArgs a = batch_step_args(g, (g.parity0 + b.step) & 1);
    const int sy = item.y / g.strips_x;  // along each row band, as in k_step_strip
    const int sx = item.y - sy * g.strips_x;
    // unit storage scales (the default; a wave-uniform test): the bodies without
    // the scaling multiplications, which are exact no-ops then
    const bool unit = !Traits<P>::kScaled || (g.sc_d == 1.0 && g.sc_j == 1.0 && g.is_d == 1.0 && g.is_j == 1.0);
    if (left >= 2 && strip_interior<2>(a, sx * 62, sy * NY, NY, 2)) {
      // no wall, fixed node or grid edge within two rows and a lane: the wall-free
      // two-step body (same bits)
      if (unit)
        fused_body<P, 2, NY, 2, true>(a, sx * 62, sy * NY, lane);
      else
        fused_body<P, 2, NY, 2, false>(a, sx * 62, sy * NY, lane);
    } else if (left >= 2) {
      if (g.wall == WALL_PAPER) {
        if (unit)
          fused_wall_body<P, WALL_PAPER, 2, NY, true>(a, sx * 62, sy * NY, lane);
        else
          fused_wall_body<P, WALL_PAPER, 2, NY, false>(a, sx * 62, sy * NY, lane);
      } else {
        if (unit)
          fused_wall_body<P, WALL_HALFWAY, 2, NY, true>(a, sx * 62, sy * NY, lane);
        else
          fused_wall_body<P, WALL_HALFWAY, 2, NY, false>(a, sx * 62, sy * NY, lane);
      }
    } else {
      if (g.wall == WALL_PAPER) {
        if (unit)
          strip_body<P, true, WALL_PAPER, 2, NY, true>(a, sx * 62, sy * NY, lane);
        else
          strip_body<P, true, WALL_PAPER, 2, NY, false>(a, sx * 62, sy * NY, lane);
      } else {
        if (unit)
          strip_body<P, true, WALL_HALFWAY, 2, NY, true>(a, sx * 62, sy * NY, lane);
        else
          strip_body<P, true, WALL_HALFWAY, 2, NY, false>(a, sx * 62, sy * NY, lane);
      }
    }
  }
}

}  // namespace lbt1

namespace lbt1 {

// Small grids resident in LDS for a whole burst: one workgroup per grid copies its
// state and flags from HBM into LDS, takes all of the grid's steps of the burst
// there -- each step the strip body of the one-step kernels over the grid's strips,
// reading one LDS copy and writing the other, then a workgroup barrier -- and
// writes the final state to the grid's other HBM parity.  HBM is read and written
// once per burst instead of once per step; the arithmetic is that of the one-step
// kernels, so the bits are those of single steps.  Rows in LDS hold nch * VEC
// values (the last chunk padded with SOLID flags and zero moments, as the row
// padding in HBM is), so no strip reads outside its grid's copy.
template <int P, int VEC, int NY>
__global__ void __launch_bounds__(256) k_step_batch_lds(BatchStepArgs b) {
  using S = typename Traits<P>::S;
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = *b.count;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const BatchGrid &g = b.grids[b.items[it].x];
    const int K = g.steps_left;
    if (K <= 0) continue;  // uniform in the block
    const int nx = g.nx, ny = g.ny;
    const int nch = (nx + VEC - 1) / VEC;
    const int pitch = nch * VEC;
    const int rs = 3 * pitch;
    const long nstate = (long)ny * rs;
    S *buf[2];
    buf[0] = reinterpret_cast<S *>(lds);
    buf[1] = buf[0] + nstate;
    uint8_t *fl = reinterpret_cast<uint8_t *>(buf[1] + nstate);
    S *trash = reinterpret_cast<S *>(fl + ((long)ny * pitch + 15) / 16 * 16);
    const int p = g.parity0 & 1;
    // HBM -> LDS: the three fields of every row (padding columns zero) and the flags
    // (padding columns SOLID, like the row padding in HBM)
    for (long i = threadIdx.x; i < nstate; i += blockDim.x) {
      const int y = (int)(i / rs);
      const int r = (int)(i - (long)y * rs);
      const int q = r / pitch;
      const int x = r - q * pitch;
      buf[0][i] = x < nx ? static_cast<const S *>(g.plane[p][q])[(long)y * g.rs + x] : S(0);
    }
    for (long i = threadIdx.x; i < (long)ny * pitch; i += blockDim.x) {
      const int y = (int)(i / pitch);
      const int x = (int)(i - (long)y * pitch);
      fl[i] = x < nx ? g.flags[(long)y * g.pitch + x] : (uint8_t)NODE_SOLID;
    }
    __syncthreads();
    StepArgs a = batch_step_args(g, p);
    a.flags = fl;
    a.pitch = pitch;
    a.rs = rs;
    a.trash = trash;
    const int strips_x = (nch + 61) / 62;
    const int strips = strips_x * ((ny + NY - 1) / NY);
    const bool unit = !Traits<P>::kScaled || (g.sc_d == 1.0 && g.sc_j == 1.0 && g.is_d == 1.0 && g.is_j == 1.0);
    for (int s = 0; s < K; ++s) {
      const S *src = buf[s & 1];
      S *dst = buf[(s + 1) & 1];
      for (int q = 0; q < 3; ++q) {
        a.src[q] = src + q * pitch;
        a.dst[q] = dst + q * pitch;
      }
      for (int k = wave; k < strips; k += blockDim.x >> 6) {
        const int sy = k / strips_x;
        const int sx = k - sy * strips_x;
        if (g.wall == WALL_PAPER) {
          if (unit)
            strip_body<P, true, WALL_PAPER, VEC, NY, true>(a, sx * 62, sy * NY, lane);
          else
            strip_body<P, true, WALL_PAPER, VEC, NY, false>(a, sx * 62, sy * NY, lane);
        } else {
          if (unit)
            strip_body<P, true, WALL_HALFWAY, VEC, NY, true>(a, sx * 62, sy * NY, lane);
          else
            strip_body<P, true, WALL_HALFWAY, VEC, NY, false>(a, sx * 62, sy * NY, lane);
        }
      }
      __syncthreads();
    }
    // LDS -> the other HBM parity: the real columns of the three fields
    const S *fin = buf[K & 1];
    for (long i = threadIdx.x; i < nstate; i += blockDim.x) {
      const int y = (int)(i / rs);
      const int r = (int)(i - (long)y * rs);
      const int q = r / pitch;
      const int x = r - q * pitch;
      if (x < nx) static_cast<S *>(g.plane[1 - p][q])[(long)y * g.rs + x] = fin[i];
    }
    __syncthreads();  // the next grid of this block reuses the LDS
  }
}

}  // namespace lbt1

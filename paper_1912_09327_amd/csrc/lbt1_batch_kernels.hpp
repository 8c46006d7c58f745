// Batched step kernels beyond one step per launch (templates; instantiated in
// lbt1_kernels.hip).  They run over the same flattened (grid, strip) item lists
// and grid descriptors as k_step_batch, with the arithmetic and its order of the
// single-grid kernels, so every grid gets the bits it would get alone.
#pragma once
#include "lbt1_batch_args.hpp"
#include "lbt1_fused.hpp"
#include "lbt1_fused_wall.hpp"
#include "lbt1_step.hpp"

namespace lbt1 {

// ================================================================ batched step


// Step arguments of a resident grid reading parity p.
__device__ __forceinline__ StepArgs batch_step_args(const BatchGrid &g, const int p) {
  StepArgs a;
  for (int q = 0; q < 3; ++q) {
    a.src[q] = g.plane[p][q];
    a.dst[q] = g.plane[1 - p][q];
  }
  a.flags = g.flags;
  a.nx = g.nx;
  a.ny = g.ny;
  a.pitch = g.pitch;
  a.rs = g.rs;
  a.periodic = g.periodic;
  a.fx = g.fx;
  a.fy = g.fy;
  a.sc_d = g.sc_d;
  a.sc_j = g.sc_j;
  a.is_d = g.is_d;
  a.is_j = g.is_j;
  a.trash = g.trash;
  a.sc_G = 0.0;
  a.sc_rho0 = 1.0;
  return a;
}

// The kind of each strip of a work list: interior (the wall-free body), column
// walls (the wall-aware body with the flags of one row) or neither.  A strip's
// geometry does not change while its grid is resident, so this runs once per work
// list instead of in every step.  One wavefront per item.
template <int VEC>
__global__ void __launch_bounds__(256) k_batch_classify(BatchClassifyArgs b) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = *b.count;
  for (int it = blockIdx.x * 4 + wave; it < n; it += gridDim.x * 4) {
    const int2 item = b.items[it];
    const BatchGrid &g = b.grids[item.x];
    const StepArgs a = batch_step_args(g, 0);
    const int strip = item.y >> 2;
    const int sy = strip / g.strips_x;
    const int sx = strip - sy * g.strips_x;
    const int c0 = sx * 62, y0 = sy * b.rows;
    const int kind = strip_interior<VEC>(a, c0, y0, b.rows, b.halo)  ? STRIP_INTERIOR
                     : strip_colwall<VEC>(a, c0, y0, b.rows, b.halo) ? STRIP_COLUMN_WALLS
                                                                      : STRIP_WALLS;
    if ((threadIdx.x & 63) == 0) b.items[it].y = (strip << 2) | kind;
  }
}

// The one-step strip bodies of a batched grid by the strip's kind: wall-free for
// interior strips, the wall-aware body with the flags of one row where walls run
// down whole columns, else the general wall-aware body.  All give the bits of the
// single-grid kernels.
template <int P, int VEC, int NY, int PF>
__device__ __forceinline__ void batch_strip(const BatchGrid &g, const StepArgs &a, const int kind, const int c0,
                                            const int y0, const int lane) {
  // unit storage scales (the default; a wave-uniform test): the bodies without
  // the scaling multiplications, which are exact no-ops then
  const bool unit = !Traits<P>::kScaled || (g.sc_d == 1.0 && g.sc_j == 1.0 && g.is_d == 1.0 && g.is_j == 1.0);
  if (kind == STRIP_INTERIOR) {
    if (unit)
      strip_body<P, false, 0, VEC, NY, true, false, PF>(a, c0, y0, lane);
    else
      strip_body<P, false, 0, VEC, NY, false, false, PF>(a, c0, y0, lane);
  } else if (kind == STRIP_COLUMN_WALLS) {
    if (g.wall == WALL_PAPER) {
      if (unit)
        strip_body<P, true, WALL_PAPER, VEC, NY, true, true, PF>(a, c0, y0, lane);
      else
        strip_body<P, true, WALL_PAPER, VEC, NY, false, true, PF>(a, c0, y0, lane);
    } else {
      if (unit)
        strip_body<P, true, WALL_HALFWAY, VEC, NY, true, true, PF>(a, c0, y0, lane);
      else
        strip_body<P, true, WALL_HALFWAY, VEC, NY, false, true, PF>(a, c0, y0, lane);
    }
  } else if (g.wall == WALL_PAPER) {
    if (unit)
      strip_body<P, true, WALL_PAPER, VEC, NY, true, false, PF>(a, c0, y0, lane);
    else
      strip_body<P, true, WALL_PAPER, VEC, NY, false, false, PF>(a, c0, y0, lane);
  } else {
    if (unit)
      strip_body<P, true, WALL_HALFWAY, VEC, NY, true, false, PF>(a, c0, y0, lane);
    else
      strip_body<P, true, WALL_HALFWAY, VEC, NY, false, false, PF>(a, c0, y0, lane);
  }
}

// Rows in flight ahead of the row being computed in the one-step batched strips:
// deeper than the single-grid kernels' (two), since a wavefront of the batch
// spends much of its time waiting for its rows and the registers allow it at two
// wavefronts per SIMD (six rows spill scalar registers).  (The two-step walled
// body keeps two: four gave the same batch time.)
constexpr int kBatchPrefetch = 4;

// One wavefront per work item, grid-stride over all items of every grid with
// columns per lane VEC.
template <int P, int VEC, int NY>
__global__ void __launch_bounds__(256) k_step_batch(BatchStepArgs b) {
  const int lane = threadIdx.x & 63;
  // wave-uniform as the compiler sees it: the item, its grid's descriptor and the
  // step arguments are then scalar loads held in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = *b.count;
  for (int it = blockIdx.x * 4 + wave; it < n; it += gridDim.x * 4) {
    const int2 item = b.items[it];
    const BatchGrid &g = b.grids[item.x];
    if (b.step >= g.steps_left) continue;
    const StepArgs a = batch_step_args(g, (g.parity0 + b.step) & 1);
    const int strip = item.y >> 2;
    const int sy = strip / g.strips_x;   // along each row band, as in k_step_strip
    const int sx = strip - sy * g.strips_x;
    batch_strip<P, VEC, NY, kBatchPrefetch>(g, a, item.y & 3, sx * 62, sy * NY, lane);
  }
}


template <int P>
__global__ void __launch_bounds__(256) k_reduce_batch(BatchReduceArgs b) {
  using T = Traits<P>;
  using S = typename T::S;
  const int n = *b.nitems;
  __shared__ double part[4][6];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 item = b.items[it];
    const int slot = item.x;
    const BatchGrid &g = b.grids[slot];
    if (g.steps_left == 0) continue;  // not stepped in this burst (uniform in the block)
    const int p = (g.parity0 + g.flips) & 1;
    const S *c0 = static_cast<const S *>(g.plane[p][0]);
    const S *c1 = static_cast<const S *>(g.plane[p][1]);
    const S *c2 = static_cast<const S *>(g.plane[p][2]);
    S *n0 = static_cast<S *>(b.snaps[slot * 3 + 0]);
    S *n1 = static_cast<S *>(b.snaps[slot * 3 + 1]);
    S *n2 = static_cast<S *>(b.snaps[slot * 3 + 2]);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const long nn = (long)g.nx * g.ny;
    const long m0 = (long)item.y * kBatchReduceChunk;
    const long m1 = min(nn, m0 + kBatchReduceChunk);
    for (long m = m0 + threadIdx.x; m < m1; m += blockDim.x) {
      const int y = (int)(m / g.nx);
      const int x = (int)(m - (long)y * g.nx);
      const long i = (long)y * g.rs + x;
      if (g.flags[(long)y * g.pitch + x] != NODE_FLUID) continue;
      const S r0 = c0[i], r1 = c1[i], r2 = c2[i];
      const double d = (double)T::dec(r0) * g.sc_d;
      const double jx = (double)T::dec(r1) * g.sc_j;
      const double jy = (double)T::dec(r2) * g.sc_j;
      acc[0] += d;
      acc[1] += jx;
      acc[2] += jy;
      acc[4] += (__builtin_isfinite(d) && __builtin_isfinite(jx) && __builtin_isfinite(jy)) ? 0.0 : 1.0;
      acc[5] += 1.0;
      const double rho = 1.0 + d;
      const double sr = 1.0 + (double)T::dec(n0[i]) * g.sc_d;
      const double su = (double)T::dec(n1[i]) * g.sc_j / sr;
      const double sv = (double)T::dec(n2[i]) * g.sc_j / sr;
      acc[3] = __builtin_fmax(acc[3], __builtin_fmax(__builtin_fabs(jx / rho - su), __builtin_fabs(jy / rho - sv)));
      n0[i] = r0;
      n1[i] = r1;
      n2[i] = r2;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double o = __shfl_xor(acc[q], off);
        acc[q] = q == 3 ? __builtin_fmax(acc[q], o) : acc[q] + o;
      }
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int q = 0; q < 6; ++q) part[wave][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      const int q = threadIdx.x;
      double v = part[0][q];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = q == 3 ? __builtin_fmax(v, part[w][q]) : v + part[w][q];
      b.partials[(long)it * 6 + q] = v;
    }
    __syncthreads();
  }
}

// The partials of each active grid (fixed order: lane-strided, then a butterfly)
// into out[slot * 6 + q].
__global__ void __launch_bounds__(64) k_reduce_batch_final(BatchReduceArgs b) {
  const int n = *b.nactive;
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    const int slot = b.active[k];
    const int2 r = b.ranges[slot];
    // lane l: partial rows l, l + 64, ... of the grid in order, then a fixed butterfly
    const int l = threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = l; i < r.y; i += 64) {
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double x = b.partials[(long)(r.x + i) * 6 + q];
        acc[q] = q == 3 ? __builtin_fmax(acc[q], x) : acc[q] + x;
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
    if (l == 0) {
#pragma unroll
      for (int q = 0; q < 6; ++q) b.out[slot * 6 + q] = acc[q];
    }
  }
}

}  // namespace lbt1

namespace lbt1 {

// Two steps per launch (the fused class, two columns per lane): launch s of a
// burst covers steps 2s and 2s + 1 of every grid in the class and flips its
// parity once.  A grid with an odd number of steps in the burst takes its last
// step in the single-step body of the same strip shape.
template <int P, int NY>
__global__ void __launch_bounds__(256) k_step_batch_fused(BatchStepArgs b) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (see k_step_batch)
  const int n = *b.count;
  for (int it = blockIdx.x * 4 + wave; it < n; it += gridDim.x * 4) {
    const int2 item = b.items[it];
    const BatchGrid &g = b.grids[item.x];
    const int left = g.steps_left - 2 * b.step;  // steps this grid still takes in the burst
    if (left <= 0) continue;
    const StepArgs a = batch_step_args(g, (g.parity0 + b.step) & 1);
    const int strip = item.y >> 2;
    const int sy = strip / g.strips_x;  // along each row band, as in k_step_strip
    const int sx = strip - sy * g.strips_x;
    // unit storage scales (the default; a wave-uniform test): the bodies without
    // the scaling multiplications, which are exact no-ops then
    const bool unit = !Traits<P>::kScaled || (g.sc_d == 1.0 && g.sc_j == 1.0 && g.is_d == 1.0 && g.is_j == 1.0);
    if (left >= 2 && (item.y & 3) == STRIP_INTERIOR) {
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

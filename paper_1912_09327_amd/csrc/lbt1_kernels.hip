// Instantiation of the step and reduction kernels and the table the runtime
// selects from.
#include "lbt1_internal.hpp"
#include "lbt1_batch_kernels.hpp"
#include "lbt1_bgk.hpp"
#include "lbt1_fused.hpp"
#include "lbt1_fused_wall.hpp"
#include "lbt1_multiphase.hpp"
#include "lbt1_step.hpp"

namespace lbt1 {

// one wavefront: lane l combines partial rows l, l + 64, ... in index order, then
// a fixed butterfly over the lanes (slot 3 is a maximum, the others sums)
__device__ __forceinline__ void reduce_rows(const double *partials, int nparts, double (&acc)[6]) {
  const int l = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 6; ++q) acc[q] = 0.0;
  for (int b = l; b < nparts; b += 64) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double x = partials[b * 6 + q];
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
}

// lane 0 writes the six raw slots (0 sum of rho - 1, 1-2 momentum, 3 residual,
// 4 non-finite count, 5 FLUID count)
__global__ void __launch_bounds__(64) k_reduce_final(const double *partials, int nparts, double *out) {
  double acc[6];
  reduce_rows(partials, nparts, acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) out[q] = acc[q];
  }
}

// The same combination, written as lbt1_reduce reports it: slot 0 the mass
// (FLUID count + sum of rho - 1, the same FP64 addition the host makes), the
// slots of `what` (LBT1_REDUCE_* bits), and slot 5 always.
__global__ void __launch_bounds__(64) k_reduce_final_out(const double *partials, int nparts, uint32_t what,
                                                         double *out) {
  double acc[6];
  reduce_rows(partials, nparts, acc);
  if (threadIdx.x == 0) {
    if (what & 1u) out[0] = acc[5] + acc[0];
    if (what & 2u) {
      out[1] = acc[1];
      out[2] = acc[2];
    }
    if (what & 4u) out[3] = acc[3];
    if (what & 8u) out[4] = acc[4];
    out[5] = acc[5];
  }
}


#define LBT1_STR2(x) #x
#define LBT1_STR(x) LBT1_STR2(x)

#define GATHER(P, HW, W) \
  {P, HW, W, KIND_GATHER, 0, 0, (const void *)&k_step_gather<P, HW, W>, "k_step_gather<" #P "," #HW "," #W ">", 1, 0}
#define STRIP(P, HW, W, V, R)                                                    \
  {P, HW, W, KIND_STRIP, V, R, (const void *)&k_step_strip<P, HW, W, V, R>, \
   "k_step_strip<" #P "," #HW "," #W "," #V "," #R ">", 1, 0}
// K steps per launch, fully periodic grids without wall or fixed nodes
#define FUSED(P, V, R, K)                                                        \
  {P, false, 0, KIND_STRIP, V, R, (const void *)&k_step_fused<P, V, R, K>, \
   "k_step_fused<" #P "," #V "," #R "," #K ">", K, 0}
#define FUSED_ROWS(P, V, K) FUSED(P, V, 6, K), FUSED(P, V, 14, K)
// two steps per launch on grids with walls, fixed nodes or non-periodic axes
#define FUSED_WALL(P, W, V, R)                                                              \
  {P, true, W, KIND_STRIP, V, R, (const void *)&k_step_fused_wall<P, W, V, R>,           \
   "k_step_fused_wall<" #P "," #W "," #V "," #R ">", 2, 0}
// (2-row strips: the shortest walk, for small grids bound by its latency)
#define FUSED_WALL_ALL(P)                                                                       \
  FUSED_WALL(P, 0, 2, 2), FUSED_WALL(P, 0, 2, 6), FUSED_WALL(P, 0, 2, 14), FUSED_WALL(P, 1, 2, 2), \
      FUSED_WALL(P, 1, 2, 6), FUSED_WALL(P, 1, 2, 14)
// 30 rows: fewer rounds of resident wavefronts on the largest grids (FP64 at 30
// rows would spill a scalar register)
#define FUSED_WALL_TALL(P) FUSED_WALL(P, 0, 2, 30), FUSED_WALL(P, 1, 2, 30)
#define FUSED_TALL(P, V, K) FUSED(P, V, 22, K), FUSED(P, V, 30, K)
#define STRIP_WALLS(P, V, R) STRIP(P, false, 0, V, R), STRIP(P, true, 0, V, R), STRIP(P, true, 1, V, R)
#define STRIP_ROWS(P, V) STRIP_WALLS(P, V, 6), STRIP_WALLS(P, V, 14)
// 8 columns per lane only without walls: the wall-aware variants at that width
// need more registers than a wavefront has and spill (the build refuses any
// kernel that spills or uses scratch memory)
#define STRIP_ROWS_NOWALL(P, V) STRIP(P, false, 0, V, 6), STRIP(P, false, 0, V, 14)
#define GATHER_ALL(P) GATHER(P, false, 0), GATHER(P, true, 0), GATHER(P, true, 1)
#define BGK(P, HW, W, SC) \
  {P, HW, W, KIND_BGK, 0, 0, (const void *)&k_bgk_step<P, HW, W, SC>, "k_bgk_step<" #P "," #HW "," #W "," #SC ">", 1, SC}
#define BGK_ALL(P)                                                                            \
  BGK(P, false, 0, false), BGK(P, true, 0, false), BGK(P, true, 1, false), BGK(P, false, 0, true), \
      BGK(P, true, 0, true), BGK(P, true, 1, true)
// multiphase LBMTau1: gather for any geometry, strips for periodic grids without walls
#define SC_GATHER(P, HW, W) \
  {P, HW, W, KIND_GATHER, 0, 0, (const void *)&k_step_sc_gather<P, HW, W>, "k_step_sc_gather<" #P "," #HW "," #W ">", 1, 1}
#define SC_STRIP(P, V, R) \
  {P, false, 0, KIND_STRIP, V, R, (const void *)&k_step_sc_strip<P, V, R>, "k_step_sc_strip<" #P "," #V "," #R ">", 1, 1}
// two multiphase steps per launch (4 columns per lane: each step widens the
// wrong halo columns by two); 22 rows measured fastest on large drops, 30
// would spill
#define SC_FUSED(P, V, R) \
  {P, false, 0, KIND_STRIP, V, R, (const void *)&k_step_sc_fused<P, V, R>, "k_step_sc_fused<" #P "," #V "," #R ">", 2, 1}
#define SC_ALL(P, V)                                                                                \
  SC_GATHER(P, false, 0), SC_GATHER(P, true, 0), SC_GATHER(P, true, 1), SC_STRIP(P, V, 6), SC_STRIP(P, V, 14)

static const StepKernel kTable[] = {
    GATHER_ALL(P_F64),     GATHER_ALL(P_F32),     GATHER_ALL(P_F16S),    GATHER_ALL(P_BF16S),
    STRIP_ROWS(P_F64, 1),  STRIP_ROWS(P_F64, 2),  STRIP_ROWS(P_F32, 1),  STRIP_ROWS(P_F32, 2),
    STRIP_ROWS(P_F32, 4),  STRIP_ROWS(P_F16S, 1), STRIP_ROWS(P_F16S, 2), STRIP_ROWS(P_F16S, 4),
    STRIP_ROWS_NOWALL(P_F16S, 8), STRIP_ROWS(P_BF16S, 1), STRIP_ROWS(P_BF16S, 2), STRIP_ROWS(P_BF16S, 4),
    STRIP_ROWS_NOWALL(P_BF16S, 8),
    // two steps per launch, and three for FP32 at 4 columns per lane (built for
    // two wavefronts per SIMD: FP64, and 16-bit storage with its codec, would
    // need scratch memory); four would need more registers than a wavefront has
    FUSED_ROWS(P_F32, 4, 3),
    // taller strips: fewer redundant halo rows per stored row.  FP32 at 22 and 28
    // rows: the runtime picks the height whose strip count best fills the last
    // round of resident wavefronts (each with its two-step companion)
    FUSED(P_F32, 4, 22, 3),    FUSED(P_F32, 4, 22, 2),    FUSED(P_F32, 4, 28, 3),    FUSED(P_F32, 4, 28, 2),
    FUSED_TALL(P_F16S, 2, 2),  FUSED_TALL(P_BF16S, 2, 2),
    FUSED_ROWS(P_F64, 2, 2),   FUSED_ROWS(P_F32, 2, 2),   FUSED_ROWS(P_F32, 4, 2),
    FUSED_ROWS(P_F16S, 2, 2),  FUSED_ROWS(P_F16S, 4, 2),  FUSED_ROWS(P_BF16S, 2, 2),
    FUSED_ROWS(P_BF16S, 4, 2),
    FUSED_WALL_ALL(P_F64), FUSED_WALL_ALL(P_F32), FUSED_WALL_ALL(P_F16S), FUSED_WALL_ALL(P_BF16S),
    FUSED_WALL_TALL(P_F32), FUSED_WALL_TALL(P_F16S), FUSED_WALL_TALL(P_BF16S),
    BGK_ALL(P_F64), BGK_ALL(P_F32), BGK_ALL(P_F16S), BGK_ALL(P_BF16S),
    SC_ALL(P_F64, 2),  SC_ALL(P_F32, 2),  SC_STRIP(P_F32, 4, 6), SC_STRIP(P_F32, 4, 14),
    SC_FUSED(P_F32, 4, 6), SC_FUSED(P_F32, 4, 14), SC_FUSED(P_F32, 4, 22),
    SC_ALL(P_F16S, 2), SC_ALL(P_BF16S, 2),
};

const StepKernel *step_kernels(int *count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

const void *reduce_partial_kernel(int prec) {
  switch (prec) {
    case P_F64: return (const void *)&k_reduce_partial<P_F64>;
    case P_F32: return (const void *)&k_reduce_partial<P_F32>;
    case P_F16S: return (const void *)&k_reduce_partial<P_F16S>;
    case P_BF16S: return (const void *)&k_reduce_partial<P_BF16S>;
  }
  return nullptr;
}

const void *reduce_final_kernel() { return (const void *)&k_reduce_final; }

const void *reduce_final_out_kernel() { return (const void *)&k_reduce_final_out; }

const void *bgk_psi_kernel(int prec) {
  switch (prec) {
    case P_F64: return (const void *)&k_bgk_psi<P_F64>;
    case P_F32: return (const void *)&k_bgk_psi<P_F32>;
    case P_F16S: return (const void *)&k_bgk_psi<P_F16S>;
    case P_BF16S: return (const void *)&k_bgk_psi<P_BF16S>;
  }
  return nullptr;
}

const void *bgk_reduce_partial_kernel(int prec) {
  switch (prec) {
    case P_F64: return (const void *)&k_bgk_reduce_partial<P_F64>;
    case P_F32: return (const void *)&k_bgk_reduce_partial<P_F32>;
    case P_F16S: return (const void *)&k_bgk_reduce_partial<P_F16S>;
    case P_BF16S: return (const void *)&k_bgk_reduce_partial<P_BF16S>;
  }
  return nullptr;
}

// Batched kernels (always wall-aware): [precision][vec class 0..2 = vec 1, 2, 4]
// for strips of 14 rows (tall), 6 rows (short: half the serial latency of a
// strip, for classes with too few strips to fill the device) and 30 rows.
#define BATCH_ROW(P, R) \
  {(const void *)&k_step_batch<P, 1, R>, (const void *)&k_step_batch<P, 2, R>, (const void *)&k_step_batch<P, 4, R>, nullptr}

const void *batch_step_kernel(int prec, int vec_class, int rows) {
  static const void *tall[4][4] = {
      {(const void *)&k_step_batch<P_F64, 1, 14>, (const void *)&k_step_batch<P_F64, 2, 14>, nullptr, nullptr},
      BATCH_ROW(P_F32, 14),
      BATCH_ROW(P_F16S, 14),
      BATCH_ROW(P_BF16S, 14),
  };
  static const void *shrt[4][4] = {
      {(const void *)&k_step_batch<P_F64, 1, 6>, (const void *)&k_step_batch<P_F64, 2, 6>, nullptr, nullptr},
      BATCH_ROW(P_F32, 6),
      BATCH_ROW(P_F16S, 6),
      BATCH_ROW(P_BF16S, 6),
  };
  // 30-row strips: fewer, longer walks per item (not FP64, whose 30-row strips spill)
  static const void *tall30[4][4] = {
      {nullptr, nullptr, nullptr, nullptr},
      BATCH_ROW(P_F32, 30),
      BATCH_ROW(P_F16S, 30),
      BATCH_ROW(P_BF16S, 30),
  };
  if (prec < 0 || prec > 3 || vec_class < 0 || vec_class > 3) return nullptr;
  if (rows == 14) return tall[prec][vec_class];
  if (rows == 6) return shrt[prec][vec_class];
  if (rows == 30) return tall30[prec][vec_class];
  return nullptr;
}

// Two steps per launch, two columns per lane, strips of 2, 6, 14 or 30 rows (FP64
// at 30 rows would spill, as the single-grid kernel of that shape does).
const void *batch_fused_kernel(int prec, int rows) {
#define BATCH_FUSED(P) \
  if (rows == 2) return (const void *)&k_step_batch_fused<P, 2>; \
  if (rows == 6) return (const void *)&k_step_batch_fused<P, 6>; \
  if (rows == 14) return (const void *)&k_step_batch_fused<P, 14>;
  switch (prec) {
    case P_F64: { BATCH_FUSED(P_F64) break; }
    case P_F32: { BATCH_FUSED(P_F32) if (rows == 30) return (const void *)&k_step_batch_fused<P_F32, 30>; break; }
    case P_F16S: { BATCH_FUSED(P_F16S) if (rows == 30) return (const void *)&k_step_batch_fused<P_F16S, 30>; break; }
    case P_BF16S: { BATCH_FUSED(P_BF16S) if (rows == 30) return (const void *)&k_step_batch_fused<P_BF16S, 30>; break; }
  }
#undef BATCH_FUSED
  return nullptr;
}

// Grids resident in LDS for a burst: two columns per lane, strips of 6 or 14 rows
// (not FP64: its kernel would spill scalar registers, and only grids of about 32 x 32
// nodes would fit).
const void *batch_lds_kernel(int prec, int rows) {
  switch (prec) {
    case P_F32: return rows == 6 ? (const void *)&k_step_batch_lds<P_F32, 2, 6> : rows == 14 ? (const void *)&k_step_batch_lds<P_F32, 2, 14> : nullptr;
    case P_F16S: return rows == 6 ? (const void *)&k_step_batch_lds<P_F16S, 2, 6> : rows == 14 ? (const void *)&k_step_batch_lds<P_F16S, 2, 14> : nullptr;
    case P_BF16S: return rows == 6 ? (const void *)&k_step_batch_lds<P_BF16S, 2, 6> : rows == 14 ? (const void *)&k_step_batch_lds<P_BF16S, 2, 14> : nullptr;
  }
  return nullptr;
}

const void *batch_classify_kernel(int vec) {
  switch (vec) {
    case 1: return (const void *)&k_batch_classify<1>;
    case 2: return (const void *)&k_batch_classify<2>;
    case 4: return (const void *)&k_batch_classify<4>;
  }
  return nullptr;
}

const void *batch_reduce_final_kernel() { return (const void *)&k_reduce_batch_final; }

const void *batch_reduce_kernel(int prec) {
  switch (prec) {
    case P_F64: return (const void *)&k_reduce_batch<P_F64>;
    case P_F32: return (const void *)&k_reduce_batch<P_F32>;
    case P_F16S: return (const void *)&k_reduce_batch<P_F16S>;
    case P_BF16S: return (const void *)&k_reduce_batch<P_BF16S>;
  }
  return nullptr;
}

}  // namespace lbt1

// Instantiation of the step and reduction kernels and the table the runtime
// selects from.
#include "lbt1_internal.hpp"
#include "lbt1_step.hpp"

namespace lbt1 {

// one block: combine `nparts` partial rows in index order into out[6]
__global__ void __launch_bounds__(64) k_reduce_final(const double *partials, int nparts, double *out) {
  const int q = threadIdx.x;
  if (q < 6) {
    double v = 0.0;
    for (int b = 0; b < nparts; ++b) v = q == 3 ? __builtin_fmax(v, partials[b * 6 + q]) : v + partials[b * 6 + q];
    out[q] = v;
  }
}


#define LBT1_STR2(x) #x
#define LBT1_STR(x) LBT1_STR2(x)

#define GATHER(P, HW, W) \
  {P, HW, W, KIND_GATHER, 0, 0, (const void *)&k_step_gather<P, HW, W>, "k_step_gather<" #P "," #HW "," #W ">"}
#define STRIP(P, HW, W, V, R)                                                    \
  {P, HW, W, KIND_STRIP, V, R, (const void *)&k_step_strip<P, HW, W, V, R>, \
   "k_step_strip<" #P "," #HW "," #W "," #V "," #R ">"}
#define STRIP_WALLS(P, V, R) STRIP(P, false, 0, V, R), STRIP(P, true, 0, V, R), STRIP(P, true, 1, V, R)
#define STRIP_ROWS(P, V) STRIP_WALLS(P, V, 14), STRIP_WALLS(P, V, 30)
// 8 columns per lane only without walls: the wall-aware variants at that width
// need more registers than a wavefront has and spill (the build refuses any
// kernel that spills or uses scratch memory)
#define STRIP_ROWS_NOWALL(P, V) STRIP(P, false, 0, V, 14), STRIP(P, false, 0, V, 30)
#define GATHER_ALL(P) GATHER(P, false, 0), GATHER(P, true, 0), GATHER(P, true, 1)

static const StepKernel kTable[] = {
    GATHER_ALL(P_F64),     GATHER_ALL(P_F32),     GATHER_ALL(P_F16S),    GATHER_ALL(P_BF16S),
    STRIP_ROWS(P_F64, 1),  STRIP_ROWS(P_F64, 2),  STRIP_ROWS(P_F32, 1),  STRIP_ROWS(P_F32, 2),
    STRIP_ROWS(P_F32, 4),  STRIP_ROWS(P_F16S, 1), STRIP_ROWS(P_F16S, 2), STRIP_ROWS(P_F16S, 4),
    STRIP_ROWS_NOWALL(P_F16S, 8), STRIP_ROWS(P_BF16S, 1), STRIP_ROWS(P_BF16S, 2), STRIP_ROWS(P_BF16S, 4),
    STRIP_ROWS_NOWALL(P_BF16S, 8),
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

// Batched kernels (always wall-aware): [precision][vec class 0..2 = vec 1, 2, 4];
// strips of 14 rows.
#define BATCH_ROW(P) \
  {(const void *)&k_step_batch<P, 1, 14>, (const void *)&k_step_batch<P, 2, 14>, (const void *)&k_step_batch<P, 4, 14>, nullptr}

const void *batch_step_kernel(int prec, int vec_class) {
  static const void *table[4][4] = {
      {(const void *)&k_step_batch<P_F64, 1, 14>, (const void *)&k_step_batch<P_F64, 2, 14>, nullptr, nullptr},
      {(const void *)&k_step_batch<P_F32, 1, 14>, (const void *)&k_step_batch<P_F32, 2, 14>,
       (const void *)&k_step_batch<P_F32, 4, 14>, nullptr},
      BATCH_ROW(P_F16S),
      BATCH_ROW(P_BF16S),
  };
  if (prec < 0 || prec > 3 || vec_class < 0 || vec_class > 3) return nullptr;
  return table[prec][vec_class];
}

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

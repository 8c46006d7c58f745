// Host-side declarations shared by the runtime and the kernel table.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbt1 {

enum : int { KIND_GATHER = 1, KIND_STRIP = 2, KIND_BGK = 3 };

// One built step kernel.  Gather kernels take (StepArgs); strip kernels take
// (StepArgs, StripMap); population (BGK) kernels take (BgkArgs).
struct StepKernel {
  int prec, haswall, wall, kind, vec, rows;
  const void *fn;
  const char *name;
  int steps;  // time steps one launch advances (fused strip kernels: 2)
  int sc;     // multiphase (Shan-Chen force) kernel
};

const StepKernel *step_kernels(int *count);
const void *reduce_partial_kernel(int prec);
const void *reduce_final_kernel();
const void *reduce_final_out_kernel();  // final pass writing the user-facing slots
const void *bgk_reduce_partial_kernel(int prec);
const void *bgk_psi_kernel(int prec);
const void *batch_step_kernel(int prec, int vec_class, int rows);
const void *batch_fused_kernel(int prec, int rows);  // two steps per launch, two columns per lane
const void *batch_lds_kernel(int prec, int rows);    // grids resident in LDS for a burst
const void *batch_reduce_kernel(int prec);
const void *batch_classify_kernel(int vec);          // strip kinds of a work list, once per list
const void *batch_reduce_final_kernel();

}  // namespace lbt1

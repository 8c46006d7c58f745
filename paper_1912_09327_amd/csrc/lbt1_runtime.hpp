// Host-side state of grids and batches (shared by the runtime sources).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbt1.h"
#include "lbt1_internal.hpp"
#include "lbt1_args.hpp"

namespace lbt1 {

constexpr int kReduceBlocks = 1024;  // most partial rows a reduction writes

struct Layout {
  int pitch;          // values per row of one field (nx rounded up to 64)
  int nfield;         // fields per parity: 3 moments, or 9 populations
  int rs;             // field row stride in values: pitch (planar) or nfield * pitch
  bool interleaved;   // the field rows of a lattice row are adjacent
  size_t field_off[9];  // byte offset of field q inside a parity block
  size_t state;       // bytes of one parity block (all fields, 256-byte multiple)
  size_t flags_off, flags_bytes;
  size_t snap_off;    // 0 without LBT1_OPT_SNAPSHOT
  int snap_rs;        // row stride of the snapshot's three moment fields
  size_t snap_field_off[3];
  size_t psi_off;     // multiphase population grids: psi of every node, 0 otherwise
  int nparts;
  size_t part_off, out_off, trash_off;
  size_t total;
};

Layout layout_of(int nx, int ny, int prec, uint32_t options);
size_t value_bytes(int prec);
lbt1_status fail(lbt1_status st, const char *fmt, ...);
lbt1_status check_device(int *dev_out, int *cus);
void encode_values(int prec, const double *in, size_t n, double inv_scale, void *out);
void decode_values(int prec, const void *in, size_t n, double scale, double *out);
lbt1_status hip_fail(hipError_t e, const char *what);
void clear_error();

}  // namespace lbt1

struct lbt1_grid {
  int device = 0, cus = 0;
  int nx = 0, ny = 0;
  uint32_t periodic = 0;
  int prec = 0, wall = 0;
  uint32_t options = 0;
  bool pop = false;       // LBT1_OPT_POPULATIONS: stored-population BGK
  double tau = 1.0;
  bool mp = false;        // LBT1_OPT_MULTIPHASE: Shan-Chen force
  double sc_G = 0.0, sc_rho0 = 1.0;
  void *psi = nullptr;    // population grids with sc: psi field
  double F[2] = {0, 0};
  double sc[2] = {1, 1};  // decode scales of d and j
  lbt1::Layout L{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char *base = nullptr;
  bool own_mem = false;
  void *plane[2][9] = {};
  uint8_t *flags = nullptr;
  void *snap[3] = {};
  double *partials = nullptr;
  double *red_out = nullptr;
  double *red_host = nullptr;  // pinned
  int parity = 0;
  int64_t steps = 0;
  bool geometry = false;
  bool haswall = false;
  int64_t fluid = 0;
  // population grids: moments given to set_geometry for SOLID and FIXED nodes
  // (reported by the readout), node index and (rho, jx, jy)
  std::vector<size_t> given_idx;
  std::vector<double> given_val;
  // step kernel
  lbt1_kernel_config cfg{};
  bool user_cfg = false;
  const lbt1::StepKernel *kern = nullptr;   // advances kern->steps steps per launch
  const lbt1::StepKernel *kern1 = nullptr;  // single-step kernel of the same launch shape
  const lbt1::StepKernel *kern2 = nullptr;  // two-step kernel of the same strip shape, when kern takes three
  lbt1::StripMap map{};
  dim3 grid{1, 1, 1}, block{1, 1, 1};
  dim3 grid1{1, 1, 1}, block1{1, 1, 1};  // launch shape of kern1
  hipGraphExec_t burst[2] = {nullptr, nullptr};
  bool graph_valid = false;
  // batch residency
  lbt1_batch *batch = nullptr;
  int slot = -1;
};

namespace lbt1 {
lbt1_status bind_config(lbt1_grid *g, const lbt1_kernel_config &want, int cus);
StepArgs step_args(const lbt1_grid *g, int src_parity);
lbt1_status enqueue_steps(lbt1_grid *g, int64_t n, hipStream_t s, bool use_graph);
lbt1_status enqueue_reduce(lbt1_grid *g, uint32_t what, hipStream_t s);
}  // namespace lbt1

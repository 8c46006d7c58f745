// Kernel argument structures shared by the kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbt1_device.hpp"

namespace lbt1 {

struct StripMap {
  int strips_x, strips_y;  // strips per row band / per column band
  int units;               // groups of 4 consecutive strips (one per block)
  int per_xcd;             // units per XCD range
  int persistent;          // 0: one block per unit; else grid-stride within the XCD range
};

struct ReduceArgs {
  const void *cur[3];
  void *snap[3];
  const uint8_t *flags;  // NULL: every node FLUID
  int nx, ny, pitch, rs; // flag / moment row strides in values
  double sc_d, sc_j;
  uint32_t what;         // LBT1_REDUCE_* bits
  double *partials;      // 6 per block
};

// Stored-population BGK step (grids created with LBT1_OPT_POPULATIONS): nine
// deviation fields g_q = f_q - w_q per parity.
struct BgkArgs {
  const void *src[9];   // fields of the current parity (pre-collision populations)
  void *dst[9];         // fields of the next parity
  const uint8_t *flags; // NULL: every node FLUID and both axes periodic
  int nx, ny, pitch, rs;
  uint32_t periodic;
  double fx, fy;        // tau * F: the velocity-shift force of the equilibrium
  double omega;         // 1 / tau
  double sc, is;        // decode / encode scale of the populations
  int tiles_x, tiles;   // 64 x 4 node tiles per tile row / in all
  int per_xcd;          // consecutive tiles per XCD (launch: 8 * per_xcd blocks)
  // multiphase: psi of every node (arithmetic type, [ny][pitch]), written by
  // k_bgk_psi before each step; the force is tau (F_body + F_SC)
  void *psi;
  double sc_G, sc_rho0, tau, bfx, bfy;
};

struct BgkReduceArgs {
  const void *cur[9];
  void *snap[3];        // moments (rho - 1, jx, jy) at the last residual call, planar
  const uint8_t *flags;
  int nx, ny, pitch, rs, snap_rs;
  double sc, sc_d, sc_j, is_d, is_j;
  uint32_t what;
  double *partials;
};

// Descriptor of one resident grid (device copy refreshed by the host before
// every burst).  parity0 is the grid's parity at the start of the burst;
// the grid takes steps_left (<= burst length) steps in this burst, in `flips`
// launches (each launch reads one parity and writes the other: one launch per
// step, one per two steps in the fused class, one per burst in the LDS class).
struct BatchGrid {
  void *plane[2][3];
  const uint8_t *flags;
  int nx, ny, pitch, rs;  // flag / moment row strides in values
  uint32_t periodic;
  int wall;
  int parity0;
  int steps_left;
  int flips;
  int strips_x;  // strips per row band (columns of 64 * vec)
  double fx, fy, sc_d, sc_j, is_d, is_j;
  void *trash;  // see StepArgs::trash
};

// Bytes of LDS a grid takes in the batch's LDS-resident class: two copies of its
// three fields on rows of ceil(nx / vec) * vec values (the last chunk padded), one
// flag byte per such node, and the 3 KiB trash area of redirected stores.
__host__ __device__ inline long lds_grid_bytes(int nx, int ny, int vec, int value_bytes) {
  const long pitch = (long)((nx + vec - 1) / vec) * vec;
  const long state = (long)ny * 3 * pitch * value_bytes;
  const long flags = ((long)ny * pitch + 15) / 16 * 16;
  return 2 * state + flags + 3 * kTrashRegion;
}

struct BatchStepArgs {
  const BatchGrid *grids;
  const int2 *items;  // (slot, strip index), strips ordered along each row band
  const int *count;   // number of items (device memory, so a graph need not change)
  int step;           // step index inside the burst
};

// Per-grid diagnostics after a burst (the six slots of k_reduce_partial,
// snapshot refreshed): every resident grid is cut into chunks of
// kBatchReduceChunk nodes, one block reduces one chunk into partials[item],
// then the partials of each active grid are combined in item order into
// out[slot * 6 + q].
constexpr int kBatchReduceChunk = 16384;
struct BatchReduceArgs {
  const BatchGrid *grids;
  void *const *snaps;   // 3 per slot
  const int2 *items;    // (slot, chunk) of every resident grid
  const int *nitems;
  double *partials;     // 6 per item
  const int *active;    // slots reduced this burst
  const int *nactive;
  const int2 *ranges;   // per slot: first item, number of items
  double *out;
};

}  // namespace lbt1

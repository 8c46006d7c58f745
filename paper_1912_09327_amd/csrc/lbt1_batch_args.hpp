// Descriptors of the batched engine's grids and launches, shared by the host
// code of lbt1_batch.hip and the batched kernels.
#pragma once
#include "lbt1_args.hpp"

namespace lbt1 {

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

// A strip item is (slot, 4 * strip + kind): the strip index counts along each row
// band, and kind (set once per work list by k_batch_classify; 0 until then, which
// is always correct) says which body the strip may take.
enum { STRIP_WALLS = 0, STRIP_COLUMN_WALLS = 1, STRIP_INTERIOR = 2 };

struct BatchStepArgs {
  const BatchGrid *grids;
  const int2 *items;  // (slot, 4 * strip + kind); the LDS class: (slot, 0)
  const int *count;   // number of items (device memory, so a graph need not change)
  int step;           // step index inside the burst
};

struct BatchClassifyArgs {
  const BatchGrid *grids;
  int2 *items;       // kinds written into the low two bits
  const int *count;
  int rows;          // strip height of the class
  int halo;          // steps one launch takes (the rows and columns beyond a strip its results draw on)
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

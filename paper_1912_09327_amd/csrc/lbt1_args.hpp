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

}  // namespace lbt1

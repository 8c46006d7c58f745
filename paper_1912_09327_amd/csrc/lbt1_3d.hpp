// Three-dimensional LBMTau1 step (D3Q19, D3Q27) for gfx950.
//
// The method of section 2 / Algorithm 1 on the 3-D lattices of the memory
// analysis of section 4: a node keeps its density and momentum (four values,
// 2 * 4 * c bytes per node over both parities against (2 Q + 4) c for the
// standard method), and its new moments are the sums over the Q directions of
// the equilibrium that the upwind node x - e_q sends along e_q.  Walls, lid
// (FIXED) nodes and the body force as in 2-D.
//
// Arithmetic as the 2-D kernels: density as d = rho - 1, equilibrium
// deviations w_q [d + 3 e.J + 4.5 (e.J)^2 / rho - 1.5 |J|^2 / rho] with the
// forced momentum J = j + F.  Direction order here: rest, the six faces, the
// twelve edges, the eight corners (D3Q19 = the first 19).
#pragma once
#include "lbt1_device.hpp"

namespace lbt1 {

__device__ constexpr int k3x[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                    1, -1, 1, -1, 1, -1, 1, -1};
__device__ constexpr int k3y[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                    1, -1, 1, -1, -1, 1, -1, 1};
__device__ constexpr int k3z[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                    1, -1, -1, 1, 1, -1, -1, 1};

template <int Q>
__device__ __forceinline__ double w3(int q) {
  // weight by |e|^2: rest, face, edge, corner
  const int m = k3x[q] * k3x[q] + k3y[q] * k3y[q] + k3z[q] * k3z[q];
  if (Q == 19) return m == 0 ? 1.0 / 3.0 : m == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
  return m == 0 ? 8.0 / 27.0 : m == 1 ? 2.0 / 27.0 : m == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
}

template <int Q>
__device__ __forceinline__ int inv3(int q) {
  return q == 0 ? 0 : ((q - 1) ^ 1) + 1;  // the order pairs e and -e as neighbours
}

struct Step3Args {
  const void *src[4];  // d, jx, jy, jz of the current parity
  void *dst[4];
  const uint8_t *flags;  // NULL: every node FLUID and all three axes periodic
  int nx, ny, nz;
  int pitch;             // values per row of one field (nx rounded up to 64)
  long rs, zs;           // row and plane strides of the moment fields, in values
  long fzs;              // plane stride of the flags
  uint32_t periodic;     // bit 0 x, bit 1 y, bit 2 z
  double fx, fy, fz;
  double sc_d, sc_j, is_d, is_j;
};

// c + e * v for a lattice component e in {-1, 0, 1} (no multiplication; q is
// known at compile time once the direction loops are unrolled)
template <typename C>
__device__ __forceinline__ C add_comp(C c, int e, C v) {
  return e == 1 ? c + v : e == -1 ? c - v : c;
}

// a += e * v for e in {-1, 0, 1}, where `have` says whether a holds a term yet:
// the first term is taken as it is (a negation is exact), so no addition of
// zero is issued.  With the direction loops unrolled, `have` is a compile-time
// value.
template <typename C>
__device__ __forceinline__ void acc_comp(C &a, bool &have, int e, C v) {
  if (e == 0) return;
  if (have) {
    a = add_comp<C>(a, e, v);
  } else {
    a = e > 0 ? v : -v;
    have = true;
  }
}

// e_q . J, formed from its nonzero components in x, y, z order (0 for the rest
// direction)
template <typename C>
__device__ __forceinline__ C dot_e(int q, C Jx, C Jy, C Jz) {
  C r = C(0);
  bool have = false;
  acc_comp<C>(r, have, k3x[q], Jx);
  acc_comp<C>(r, have, k3y[q], Jy);
  acc_comp<C>(r, have, k3z[q], Jz);
  return r;
}

// Equilibrium deviation w_q [s (e.J)^2 + 3 e.J + b] with s = 4.5 / rho and
// b = d - 1.5 |J|^2 / rho; for the rest direction (e = 0) it is w_0 b.
template <typename C, int Q>
__device__ __forceinline__ C emit3_sb(int q, C Jx, C Jy, C Jz, C s, C b) {
  if (k3x[q] == 0 && k3y[q] == 0 && k3z[q] == 0) return C(w3<Q>(q)) * b;
  const C eJ = dot_e<C>(q, Jx, Jy, Jz);
  return C(w3<Q>(q)) * fmaC<C>(s, eJ * eJ, fmaC<C>(C(3), eJ, b));
}

// Equilibrium deviation a node with deviation d and forced momentum J sends
// along e_q (inv = 1 / (1 + d), t = |J|^2 inv).
template <typename C, int Q>
__device__ __forceinline__ C emit3(int q, C d, C Jx, C Jy, C Jz, C inv, C t) {
  return emit3_sb<C, Q>(q, Jx, Jy, Jz, C(4.5) * inv, fmaC<C>(C(-1.5), t, d));
}

template <int P>
__device__ __forceinline__ void load3(const Step3Args &a, long i, typename Traits<P>::C &d, typename Traits<P>::C &jx,
                                      typename Traits<P>::C &jy, typename Traits<P>::C &jz) {
  using T = Traits<P>;
  using S = typename T::S;
  using C = typename T::C;
  d = T::dec(static_cast<const S *>(a.src[0])[i]);
  jx = T::dec(static_cast<const S *>(a.src[1])[i]);
  jy = T::dec(static_cast<const S *>(a.src[2])[i]);
  jz = T::dec(static_cast<const S *>(a.src[3])[i]);
  if (T::kScaled) {
    d *= C(a.sc_d);
    jx *= C(a.sc_j);
    jy *= C(a.sc_j);
    jz *= C(a.sc_j);
  }
}

// load3 in two halves: the stored values of node i, and their decoding (the same
// operations in the same order).  The tile kernels keep a plane's stored values
// in registers while its loads are in flight and decode them only when the plane
// goes to LDS, one plane later, so no wait for the loads is forced before the
// targets of the current plane are formed.
template <int P>
__device__ __forceinline__ void load3_raw(const Step3Args &a, long i, typename Traits<P>::S &d, typename Traits<P>::S &jx,
                                          typename Traits<P>::S &jy, typename Traits<P>::S &jz) {
  using S = typename Traits<P>::S;
  d = static_cast<const S *>(a.src[0])[i];
  jx = static_cast<const S *>(a.src[1])[i];
  jy = static_cast<const S *>(a.src[2])[i];
  jz = static_cast<const S *>(a.src[3])[i];
}
template <int P>
__device__ __forceinline__ typename Traits<P>::C dec3_d(const Step3Args &a, typename Traits<P>::S v) {
  using C = typename Traits<P>::C;
  C d = Traits<P>::dec(v);
  if (Traits<P>::kScaled) d *= C(a.sc_d);
  return d;
}
template <int P>
__device__ __forceinline__ typename Traits<P>::C dec3_j(const Step3Args &a, typename Traits<P>::S v) {
  using C = typename Traits<P>::C;
  C j = Traits<P>::dec(v);
  if (Traits<P>::kScaled) j *= C(a.sc_j);
  return j;
}

// One thread per node; blocks of 64 x 4 nodes in (x, y), grid (x tiles,
// y tiles, nz).
template <int P, int Q, bool HASWALL, int WALL>
__global__ void __launch_bounds__(256) k_step3_gather(Step3Args a) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const long i = (long)z * a.zs + (long)y * a.rs + x;
  if (HASWALL && a.flags[(long)z * a.fzs + (long)y * a.pitch + x] != NODE_FLUID) return;  // held
  const C Fx = C(a.fx), Fy = C(a.fy), Fz = C(a.fz);
  C d0, jx0, jy0, jz0;
  load3<P>(a, i, d0, jx0, jy0, jz0);
  C own_inv = C(0), own_t = C(0);
  if (HASWALL && WALL == WALL_HALFWAY) {
    own_inv = recip<C>(C(1) + d0);
    const C Jx = jx0 + Fx, Jy = jy0 + Fy, Jz = jz0 + Fz;
    own_t = (Jx * Jx + Jy * Jy + Jz * Jz) * own_inv;
  }
  C dn = C(0), xn = C(0), yn = C(0), zn = C(0);
  bool hx = false, hy = false, hz = false;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int sx = wrap_axis(x - k3x[q], a.nx, a.periodic & 1u);
    const int sy = wrap_axis(y - k3y[q], a.ny, a.periodic & 2u);
    const int sz = wrap_axis(z - k3z[q], a.nz, a.periodic & 4u);
    bool solid = sx < 0 || sy < 0 || sz < 0;
    if (HASWALL && !solid) solid = a.flags[(long)sz * a.fzs + (long)sy * a.pitch + sx] == NODE_SOLID;
    C f;
    if (!solid) {
      C d, jx, jy, jz;
      load3<P>(a, (long)sz * a.zs + (long)sy * a.rs + sx, d, jx, jy, jz);
      const C inv = recip<C>(C(1) + d);
      const C Jx = jx + Fx, Jy = jy + Fy, Jz = jz + Fz;
      const C t = (Jx * Jx + Jy * Jy + Jz * Jz) * inv;
      f = emit3<C, Q>(q, d, Jx, Jy, Jz, inv, t);
    } else if (WALL == WALL_PAPER) {
      f = C(w3<Q>(q)) * d0;
    } else {
      f = emit3<C, Q>(inv3<Q>(q), d0, jx0 + Fx, jy0 + Fy, jz0 + Fz, own_inv, own_t);
    }
    dn = q == 0 ? f : dn + f;
    acc_comp<C>(xn, hx, k3x[q], f);
    acc_comp<C>(yn, hy, k3y[q], f);
    acc_comp<C>(zn, hz, k3z[q], f);
  }
  if (T::kScaled) {
    dn *= C(a.is_d);
    xn *= C(a.is_j);
    yn *= C(a.is_j);
    zn *= C(a.is_j);
  }
  static_cast<S *>(a.dst[0])[i] = T::enc(dn);
  static_cast<S *>(a.dst[1])[i] = T::enc(xn);
  static_cast<S *>(a.dst[2])[i] = T::enc(yn);
  static_cast<S *>(a.dst[3])[i] = T::enc(zn);
}

// A block of 64 x TY nodes marches along z through ZC planes.  Three planes of
// its tile plus a one-node halo live in LDS as the per-source values every
// emission needs (J, s = 4.5 / rho, b = d - 1.5 |J|^2 / rho), computed once per
// node and plane; each target then forms its Q arrivals from LDS.  The
// per-direction arithmetic is that of the gather kernel, so the two give the
// same bits.
//
// HASWALL: grids with SOLID or FIXED nodes or a non-periodic axis.  The flags of
// the three planes sit in LDS beside the values (SOLID for positions outside a
// non-periodic axis); an arrival from a SOLID source takes the wall rule of the
// gather kernel -- w_q times the target's own deviation (Eq. feqnoslip; the
// target's d is carried in registers from the plane it was loaded with) or, with
// half-way bounce-back, the target's own emission along -e_q from its LDS slot --
// and a non-FLUID target is not written (it holds its value in both parities).
// Without walls every axis is periodic and the block wraps.
//
// Loading a plane: every thread fills the LDS slot of its own node, and the
// first 2 (64 + 2) + 2 TY threads each fill one halo-ring slot (the other
// wavefronts skip that pass).  The in-plane offsets of both (wrapped, periodic
// in x and y) do not depend on z and are computed once; the moments of a plane
// are loaded into registers one plane before they go to LDS.
constexpr int kTile3X = 64;

template <int P, int Q, int ZC, int TY, bool HASWALL = false, int WALL = 0>
__global__ void __launch_bounds__(64 * TY) k_step3_tile(Step3Args a) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  constexpr int HX = kTile3X + 2, HY = TY + 2, HN = HX * HY;
  constexpr int RING = 2 * HX + 2 * TY;  // halo slots outside the tile
  __shared__ C sJx[3][HN], sJy[3][HN], sJz[3][HN], sS[3][HN], sB[3][HN];
  __shared__ uint8_t sF[HASWALL ? 3 : 1][HASWALL ? HN : 1];  // flags (SOLID outside a non-periodic axis)
  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;
  // A one-dimensional launch of 8 * per blocks (lbt1_grid3d_step): block b runs on XCD
  // b % 8, and XCD x takes the tiles [x * per, (x + 1) * per) in x-fastest order, so
  // the tiles whose halo columns and rows a tile shares are mostly on its own XCD
  // and its L2 (2-3 % faster at 512^3 than a three-dimensional grid, whose
  // consecutive blocks, the x neighbours, go to different XCDs).
  const int ntx = (a.nx + kTile3X - 1) / kTile3X, nty = (a.ny + TY - 1) / TY, ntz = (a.nz + ZC - 1) / ZC;
  const int ntiles = ntx * nty * ntz, per = (ntiles + 7) / 8;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= ntiles) return;  // uniform across the block
  const int tz = tile / (ntx * nty), trow = tile - tz * ntx * nty, tyi = trow / ntx, txi = trow - tyi * ntx;
  const int x0 = txi * kTile3X, y0 = tyi * TY, z0 = tz * ZC;
  const C Fx = C(a.fx), Fy = C(a.fy), Fz = C(a.fz);
  const bool px = !HASWALL || (a.periodic & 1u), py = !HASWALL || (a.periodic & 2u),
             pz = !HASWALL || (a.periodic & 4u);
  const int own_h = (ty + 1) * HX + tx + 1;
  // in-plane offsets (x, y wrapped on periodic axes); -1: outside a non-periodic axis
  auto plane_off = [&](const int x, const int y) -> long {
    const int wx = wrap_axis(x, a.nx, px), wy = wrap_axis(y, a.ny, py);
    return wx < 0 || wy < 0 ? -1 : (long)wy * a.rs + wx;
  };
  auto flag_off = [&](const int x, const int y) -> long {
    const int wx = wrap_axis(x, a.nx, px), wy = wrap_axis(y, a.ny, py);
    return wx < 0 || wy < 0 ? -1 : (long)wy * a.pitch + wx;
  };
  const long own_off = plane_off(x0 + tx, y0 + ty);
  const long own_foff = HASWALL ? flag_off(x0 + tx, y0 + ty) : 0;
  const bool has_ring = tid < RING;
  int ring_h = 0;
  long ring_off = 0, ring_foff = 0;
  if (has_ring) {
    int hx, hy;
    if (tid < HX) {  // row below the tile
      hx = tid;
      hy = 0;
    } else if (tid < 2 * HX) {  // row above
      hx = tid - HX;
      hy = HY - 1;
    } else if (tid < 2 * HX + TY) {  // left column
      hx = 0;
      hy = 1 + (tid - 2 * HX);
    } else {  // right column
      hx = HX - 1;
      hy = 1 + (tid - 2 * HX - TY);
    }
    ring_h = hy * HX + hx;
    ring_off = plane_off(x0 - 1 + hx, y0 - 1 + hy);
    if (HASWALL) ring_foff = flag_off(x0 - 1 + hx, y0 - 1 + hy);
  }
  // plane loads run one plane ahead in registers: the loads of plane z + 2 are
  // in flight while the targets of plane z are formed.  Positions outside a
  // non-periodic axis load node 0 and are flagged SOLID.
  S od, ojx, ojy, ojz, rd = S(0), rjx = S(0), rjy = S(0), rjz = S(0);  // stored values (see load3_raw)
  uint8_t ofl = NODE_FLUID, rfl = NODE_FLUID;
  auto fetch = [&](const int z) __attribute__((always_inline)) {
    const int wz = wrap_axis(z, a.nz, pz);
    const long zo = wz < 0 ? 0 : (long)wz * a.zs;
    load3_raw<P>(a, zo + (own_off < 0 ? 0 : own_off), od, ojx, ojy, ojz);
    if (has_ring) load3_raw<P>(a, zo + (ring_off < 0 ? 0 : ring_off), rd, rjx, rjy, rjz);
    if (HASWALL) {
      const long fz = (long)(wz < 0 ? 0 : wz) * a.fzs;
      ofl = wz < 0 || own_foff < 0 ? (uint8_t)NODE_SOLID : a.flags[fz + own_foff];
      if (has_ring) rfl = wz < 0 || ring_foff < 0 ? (uint8_t)NODE_SOLID : a.flags[fz + ring_foff];
    }
  };
  auto put = [&](const S sd, const S sjx, const S sjy, const S sjz, const int slot, const int h)
      __attribute__((always_inline)) {
    const C d = dec3_d<P>(a, sd), jx = dec3_j<P>(a, sjx), jy = dec3_j<P>(a, sjy), jz = dec3_j<P>(a, sjz);
    const C inv = recip<C>(C(1) + d);
    const C Jx = jx + Fx, Jy = jy + Fy, Jz = jz + Fz;
    const C t = (Jx * Jx + Jy * Jy + Jz * Jz) * inv;
    sJx[slot][h] = Jx;
    sJy[slot][h] = Jy;
    sJz[slot][h] = Jz;
    sS[slot][h] = C(4.5) * inv;
    sB[slot][h] = fmaC<C>(C(-1.5), t, d);
  };
  // the fetched plane into LDS slot `slot`
  auto store_plane = [&](const int slot) __attribute__((always_inline)) {
    put(od, ojx, ojy, ojz, slot, own_h);
    if (has_ring) put(rd, rjx, rjy, rjz, slot, ring_h);
    if (HASWALL) {
      sF[slot][own_h] = ofl;
      if (has_ring) sF[slot][ring_h] = rfl;
    }
  };
  fetch(z0 - 1);
  store_plane(0);
  fetch(z0);
  store_plane(1);
  C own_d = dec3_d<P>(a, od);  // the target's own deviation (plane z), for the wall rule
  uint8_t own_fl = ofl;
  fetch(z0 + 1);
  const int x = x0 + tx, y = y0 + ty;
  const bool out = x < a.nx && y < a.ny;
  for (int k = 0; k < ZC; ++k) {
    const int z = z0 + k;
    if (z >= a.nz) break;  // uniform across the block
    store_plane((k + 2) % 3);  // plane z + 1
    const C next_d = dec3_d<P>(a, od);
    const uint8_t next_fl = ofl;
    if (k + 1 < ZC) fetch(z + 2);
    __syncthreads();
    if (out && (!HASWALL || own_fl == NODE_FLUID)) {
      C dn = C(0), xn = C(0), yn = C(0), zn = C(0);
      bool hx = false, hy = false, hz = false;
      const int cs = (k + 1) % 3;  // the target's own plane
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int slot = (k + 1 - k3z[q] + 3) % 3;  // plane z - e_z
        const int h = (ty + 1 - k3y[q]) * HX + (tx + 1 - k3x[q]);
        C f = emit3_sb<C, Q>(q, sJx[slot][h], sJy[slot][h], sJz[slot][h], sS[slot][h], sB[slot][h]);
        if (HASWALL && q != 0 && sF[slot][h] == NODE_SOLID) {
          if (WALL == WALL_PAPER)
            f = C(w3<Q>(q)) * own_d;
          else
            f = emit3_sb<C, Q>(inv3<Q>(q), sJx[cs][own_h], sJy[cs][own_h], sJz[cs][own_h], sS[cs][own_h],
                               sB[cs][own_h]);
        }
        dn = q == 0 ? f : dn + f;
        acc_comp<C>(xn, hx, k3x[q], f);
        acc_comp<C>(yn, hy, k3y[q], f);
        acc_comp<C>(zn, hz, k3z[q], f);
      }
      if (T::kScaled) {
        dn *= C(a.is_d);
        xn *= C(a.is_j);
        yn *= C(a.is_j);
        zn *= C(a.is_j);
      }
      const long i = (long)z * a.zs + (long)y * a.rs + x;
      static_cast<S *>(a.dst[0])[i] = T::enc(dn);
      static_cast<S *>(a.dst[1])[i] = T::enc(xn);
      static_cast<S *>(a.dst[2])[i] = T::enc(yn);
      static_cast<S *>(a.dst[3])[i] = T::enc(zn);
    }
    own_d = next_d;
    own_fl = next_fl;
    __syncthreads();  // the slot of plane z - 1 is refilled next
  }
}

// Grids with every axis periodic and every node FLUID: the same march along z,
// with the x neighbours taken across the wavefront instead of from LDS.  A
// wavefront holds one row of 64 nodes, x0 - 1 ... x0 + 62: lanes 1 to 62 are
// the targets, lanes 0 and 63 the halo columns.  LDS holds three planes of
// TY + 2 such rows (the tile rows and one halo row on either side, loaded by
// wavefronts 0 and 1).  For each of the nine (e_y, e_z) offsets a lane reads the
// per-source values of node (x, y - e_y, z - e_z) once and forms the emissions
// of every direction with that offset; an emission along a direction with
// e_x = +1 (-1) then moves one lane up (down) by a whole-wavefront DPP shift.
// Half the LDS reads of the tile kernel for the same arithmetic in the same
// summation order, so the two give the same bits.  Every lane takes part in
// every shift (the halo lanes' emissions are what lanes 1 and 62 receive); only
// the stores are guarded.
constexpr int kLane3X = 62;

template <int P, int Q, int ZC, int TY>
__global__ void __launch_bounds__(64 * TY) k_step3_lane(Step3Args a) {
  using T = Traits<P>;
  using C = typename T::C;
  using S = typename T::S;
  constexpr int HY = TY + 2, HN = 64 * HY;
  __shared__ C sJx[3][HN], sJy[3][HN], sJz[3][HN], sS[3][HN], sB[3][HN];
  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;
  // tile order as in k_step3_tile (XCD b % 8 takes a contiguous range)
  const int ntx = (a.nx + kLane3X - 1) / kLane3X, nty = (a.ny + TY - 1) / TY, ntz = (a.nz + ZC - 1) / ZC;
  const int ntiles = ntx * nty * ntz, per = (ntiles + 7) / 8;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= ntiles) return;  // uniform across the block
  const int tz = tile / (ntx * nty), trow = tile - tz * ntx * nty, tyi = trow / ntx, txi = trow - tyi * ntx;
  const int x0 = txi * kLane3X, y0 = tyi * TY, z0 = tz * ZC;
  const C Fx = C(a.fx), Fy = C(a.fy), Fz = C(a.fz);
  const int x = x0 - 1 + tx, y = y0 + ty;
  const long xo = wrap_axis(x, a.nx, true);
  const long own_off = (long)wrap_axis(y, a.ny, true) * a.rs + xo;
  const int own_h = (ty + 1) * 64 + tx;
  const bool has_halo = tid < 128;  // wavefront 0: row y0 - 1, wavefront 1: row y0 + TY
  const int halo_h = tid < 64 ? tx : (HY - 1) * 64 + tx;
  const long halo_off = (long)wrap_axis(tid < 64 ? y0 - 1 : y0 + TY, a.ny, true) * a.rs + xo;
  S od, ojx, ojy, ojz, rd = S(0), rjx = S(0), rjy = S(0), rjz = S(0);  // stored values (see load3_raw)
  auto fetch = [&](const int z) __attribute__((always_inline)) {
    const long zo = (long)wrap_axis(z, a.nz, true) * a.zs;
    load3_raw<P>(a, zo + own_off, od, ojx, ojy, ojz);
    if (has_halo) load3_raw<P>(a, zo + halo_off, rd, rjx, rjy, rjz);
  };
  auto put = [&](const S sd, const S sjx, const S sjy, const S sjz, const int slot, const int h)
      __attribute__((always_inline)) {
    const C d = dec3_d<P>(a, sd), jx = dec3_j<P>(a, sjx), jy = dec3_j<P>(a, sjy), jz = dec3_j<P>(a, sjz);
    const C inv = recip<C>(C(1) + d);
    const C Jx = jx + Fx, Jy = jy + Fy, Jz = jz + Fz;
    const C t = (Jx * Jx + Jy * Jy + Jz * Jz) * inv;
    sJx[slot][h] = Jx;
    sJy[slot][h] = Jy;
    sJz[slot][h] = Jz;
    sS[slot][h] = C(4.5) * inv;
    sB[slot][h] = fmaC<C>(C(-1.5), t, d);
  };
  auto store_plane = [&](const int slot) __attribute__((always_inline)) {
    put(od, ojx, ojy, ojz, slot, own_h);
    if (has_halo) put(rd, rjx, rjy, rjz, slot, halo_h);
  };
  fetch(z0 - 1);
  store_plane(0);
  fetch(z0);
  store_plane(1);
  fetch(z0 + 1);
  const bool out = tx >= 1 && tx <= kLane3X && x < a.nx && y < a.ny;
  for (int k = 0; k < ZC; ++k) {
    const int z = z0 + k;
    if (z >= a.nz) break;  // uniform across the block
    store_plane((k + 2) % 3);  // plane z + 1
    if (k + 1 < ZC) fetch(z + 2);
    __syncthreads();
    C f[Q];
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      const int ey = p / 3 - 1, ez = p % 3 - 1;
      const int slot = (k + 1 - ez + 3) % 3;  // plane z - e_z
      const int h = (ty + 1 - ey) * 64 + tx;  // row y - e_y, this lane's column
      const C Jx = sJx[slot][h], Jy = sJy[slot][h], Jz = sJz[slot][h], s = sS[slot][h], b = sB[slot][h];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (k3y[q] != ey || k3z[q] != ez) continue;
        const C e = emit3_sb<C, Q>(q, Jx, Jy, Jz, s, b);
        f[q] = k3x[q] == 1 ? dpp_shift<kDppWaveShr1>(e) : k3x[q] == -1 ? dpp_shift<kDppWaveShl1>(e) : e;
      }
    }
    C dn = C(0), xn = C(0), yn = C(0), zn = C(0);
    bool hx = false, hy = false, hz = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      dn = q == 0 ? f[q] : dn + f[q];
      acc_comp<C>(xn, hx, k3x[q], f[q]);
      acc_comp<C>(yn, hy, k3y[q], f[q]);
      acc_comp<C>(zn, hz, k3z[q], f[q]);
    }
    if (out) {
      if (T::kScaled) {
        dn *= C(a.is_d);
        xn *= C(a.is_j);
        yn *= C(a.is_j);
        zn *= C(a.is_j);
      }
      const long i = (long)z * a.zs + (long)y * a.rs + x;
      static_cast<S *>(a.dst[0])[i] = T::enc(dn);
      static_cast<S *>(a.dst[1])[i] = T::enc(xn);
      static_cast<S *>(a.dst[2])[i] = T::enc(yn);
      static_cast<S *>(a.dst[3])[i] = T::enc(zn);
    }
    __syncthreads();  // the slot of plane z - 1 is refilled next
  }
}

struct Reduce3Args {
  const void *cur[4];
  void *snap[4];
  const uint8_t *flags;
  int nx, ny, nz, pitch;
  long rs, zs, fzs;
  double sc_d, sc_j;
  uint32_t what;
  double *partials;  // 8 per block
};

// out slots: 0 sum d, 1..3 sum j, 4 max residual, 5 non-finite, 6 FLUID count
template <int P>
__global__ void __launch_bounds__(256) k_reduce3_partial(Reduce3Args a) {
  using T = Traits<P>;
  using S = typename T::S;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long n = (long)a.nx * a.ny * a.nz;
  const bool want_res = a.what & 4u;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int x = (int)(k % a.nx);
    const long yz = k / a.nx;
    const int y = (int)(yz % a.ny);
    const int z = (int)(yz / a.ny);
    if (a.flags && a.flags[(long)z * a.fzs + (long)y * a.pitch + x] != NODE_FLUID) continue;
    const long i = (long)z * a.zs + (long)y * a.rs + x;
    double v[4];
    S r[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      r[m] = static_cast<const S *>(a.cur[m])[i];
      v[m] = (double)T::dec(r[m]) * (m == 0 ? a.sc_d : a.sc_j);
    }
    for (int m = 0; m < 4; ++m) acc[m] += v[m];
    const bool fin = __builtin_isfinite(v[0]) && __builtin_isfinite(v[1]) && __builtin_isfinite(v[2]) &&
                     __builtin_isfinite(v[3]);
    acc[5] += fin ? 0.0 : 1.0;
    acc[6] += 1.0;
    if (want_res) {
      const double rho = 1.0 + v[0];
      const double sr = 1.0 + (double)T::dec(static_cast<S *>(a.snap[0])[i]) * a.sc_d;
      double res = 0.0;
      for (int m = 1; m < 4; ++m) {
        const double su = (double)T::dec(static_cast<S *>(a.snap[m])[i]) * a.sc_j / sr;
        res = __builtin_fmax(res, __builtin_fabs(v[m] / rho - su));
      }
      acc[4] = __builtin_fmax(acc[4], res);
      for (int m = 0; m < 4; ++m) static_cast<S *>(a.snap[m])[i] = r[m];
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const double o = __shfl_xor(acc[m], off);
      acc[m] = m == 4 ? __builtin_fmax(acc[m], o) : acc[m] + o;
    }
  }
  __shared__ double part[4][8];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int m = 0; m < 8; ++m) part[wave][m] = acc[m];
  __syncthreads();
  if (threadIdx.x < 8) {
    const int m = threadIdx.x;
    double v = part[0][m];
    for (int w = 1; w < 4; ++w) v = m == 4 ? __builtin_fmax(v, part[w][m]) : v + part[w][m];
    a.partials[blockIdx.x * 8 + m] = v;
  }
}

// one wavefront: lane l combines partial rows l, l + 64, ... in index order, then a
// fixed butterfly over the lanes (slot 4 is a maximum, the others sums)
__global__ void __launch_bounds__(64) k_reduce3_final(const double *partials, int nparts, double *out) {
  const int l = threadIdx.x;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = l; b < nparts; b += 64) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const double x = partials[b * 8 + m];
      acc[m] = m == 4 ? __builtin_fmax(acc[m], x) : acc[m] + x;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const double o = __shfl_xor(acc[m], off);
      acc[m] = m == 4 ? __builtin_fmax(acc[m], o) : acc[m] + o;
    }
  }
  if (l == 0) {
#pragma unroll
    for (int m = 0; m < 8; ++m) out[m] = acc[m];
  }
}

}  // namespace lbt1

// Three-dimensional LBMTau1 grids: layout, initialisation, step launches,
// reductions and the lbt1_grid3d_* C ABI.
//
// Layout per parity: [nz][ny][4][pitch] (the four moment rows of a lattice
// row adjacent, pitch = nx rounded up to 64), flags [nz][ny][pitch] (padding
// SOLID), an optional snapshot (one more parity block) for the residual, and
// reduction partials.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbt1.h"
#include "lbt1_3d.hpp"
#include "lbt1_runtime.hpp"

namespace lbt1 {

static size_t rup(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout3 {
  int pitch;
  long rs, zs, fzs;
  size_t state, flags_off, flags_bytes, snap_off, part_off, out_off, total;
  int nparts;
};

static Layout3 layout3(int nx, int ny, int nz, int prec, uint32_t options) {
  Layout3 L{};
  const size_t c = value_bytes(prec);
  L.pitch = (int)rup((size_t)nx, 64);
  L.rs = 4L * L.pitch;
  L.zs = L.rs * ny;
  L.fzs = (long)L.pitch * ny;
  L.state = rup((size_t)L.zs * nz * c, 256);
  L.flags_off = 2 * L.state;
  L.flags_bytes = rup((size_t)L.fzs * nz, 256);
  size_t off = L.flags_off + L.flags_bytes;
  L.snap_off = 0;
  if (options & LBT1_OPT_SNAPSHOT) {
    L.snap_off = off;
    off += L.state;
  }
  L.nparts = 1024;
  L.part_off = off;
  off += rup((size_t)L.nparts * 8 * sizeof(double), 256);
  L.out_off = off;
  off += 256;
  L.total = off;
  return L;
}

static bool valid3(int nx, int ny, int nz) {
  return nx >= 3 && ny >= 3 && nz >= 1 && nx <= 16384 && ny <= 16384 && nz <= 16384;
}

typedef void (*Step3Fn)(Step3Args);

static const void *step3_kernel(int prec, int q, bool haswall, int wall) {
#define K3(P, Q)                                                                                        \
  if (prec == P && q == Q) {                                                                            \
    if (!haswall) return (const void *)&k_step3_gather<P, Q, false, 0>;                                 \
    return wall == WALL_PAPER ? (const void *)&k_step3_gather<P, Q, true, 0>                            \
                              : (const void *)&k_step3_gather<P, Q, true, 1>;                           \
  }
  K3(P_F64, 19) K3(P_F64, 27) K3(P_F32, 19) K3(P_F32, 27) K3(P_F16S, 19) K3(P_F16S, 27) K3(P_BF16S, 19)
  K3(P_BF16S, 27)
#undef K3
  return nullptr;
}

// Planes a tile block marches through: 32, but 16 for the periodic kernels with
// 16-bit storage (at 512^3, D3Q19: FP32 126.9k against 123.7k MLUPS at 16;
// FP16S 131.0k against 137.1k at 32).  The wall-aware kernels take 32 in every
// storage (FP16S lid-driven box at 512^3: 80.7k against 76.5k MLUPS at 16, and
// 96 VGPRs against 116).
template <int P>
constexpr int zchunk_of() {
  return P == P_F16S || P == P_BF16S ? 16 : 32;
}
constexpr int kZChunkWall = 32;
static int zchunk_for(int prec, bool haswall) {
  return haswall ? kZChunkWall : prec == P_F16S || prec == P_BF16S ? 16 : 32;
}
constexpr int kTile3Y = 8;   // rows of a tile block (64 x 8 nodes, 512 threads)

static const void *tile3_kernel(int prec, int q, bool haswall, int wall) {
#define T3(P, Q)                                                                                          \
  if (prec == P && q == Q) {                                                                              \
    if (!haswall && Q == 27) return (const void *)&k_step3_lane<P, Q, zchunk_of<P>(), kTile3Y>;          \
    if (!haswall) return (const void *)&k_step3_tile<P, Q, zchunk_of<P>(), kTile3Y>;                     \
    return wall == WALL_PAPER ? (const void *)&k_step3_tile<P, Q, kZChunkWall, kTile3Y, true, WALL_PAPER> \
                              : (const void *)&k_step3_tile<P, Q, kZChunkWall, kTile3Y, true, WALL_HALFWAY>; \
  }
  T3(P_F64, 19) T3(P_F64, 27) T3(P_F32, 19) T3(P_F32, 27) T3(P_F16S, 19) T3(P_F16S, 27) T3(P_BF16S, 19)
  T3(P_BF16S, 27)
#undef T3
  return nullptr;
}

static const void *reduce3_kernel(int prec) {
  switch (prec) {
    case P_F64: return (const void *)&k_reduce3_partial<P_F64>;
    case P_F32: return (const void *)&k_reduce3_partial<P_F32>;
    case P_F16S: return (const void *)&k_reduce3_partial<P_F16S>;
    case P_BF16S: return (const void *)&k_reduce3_partial<P_BF16S>;
  }
  return nullptr;
}

}  // namespace lbt1

using namespace lbt1;

struct lbt1_grid3d {
  int device = 0;
  int nx = 0, ny = 0, nz = 0, q = 19;
  uint32_t periodic = 0, options = 0;
  int prec = 0, wall = 0;
  double F[3] = {0, 0, 0};
  double sc[2] = {1, 1};
  Layout3 L{};
  hipStream_t stream = nullptr;
  bool own_stream = false, own_mem = false;
  char *base = nullptr;
  void *plane[2][4] = {};
  void *snap[4] = {};
  uint8_t *flags = nullptr;
  double *partials = nullptr, *red_out = nullptr, *red_host = nullptr;
  int parity = 0;
  bool geometry = false, haswall = false;
  int want = LBT1_KERNEL_AUTO;  // kernel family asked for
  bool tile = false;            // the z-marching LDS tile kernel is bound
  const void *kern = nullptr;
};

// AUTO and STRIP take a tile kernel: on fully periodic grids without SOLID or
// FIXED nodes k_step3_lane for D3Q27 (at 512^3, FP32: 112.2k against 107.6k
// MLUPS for k_step3_tile) and k_step3_tile for D3Q19 (137.3k against 105.2k: its
// 64-column tiles divide the power-of-two sides, while 62-column tiles leave
// 12.5 % of the lanes idle at 512, and D3Q19 reads too little from LDS to gain
// from the lane shifts); k_step3_tile's wall-aware form otherwise.  GATHER: the
// one-thread-per-node kernel.
static bool lane3(const lbt1_grid3d *g) { return g->tile && !g->haswall && g->q == 27; }

static lbt1_status bind3(lbt1_grid3d *g) {
  g->tile = g->want != LBT1_KERNEL_GATHER;
  g->kern = g->tile ? tile3_kernel(g->prec, g->q, g->haswall, g->wall) : step3_kernel(g->prec, g->q, g->haswall, g->wall);
  if (!g->kern) return fail(LBT1_EINVAL, "no built 3-D kernel");
  return LBT1_OK;
}

static Step3Args step3_args(const lbt1_grid3d *g, int p) {
  Step3Args a{};
  for (int m = 0; m < 4; ++m) {
    a.src[m] = g->plane[p][m];
    a.dst[m] = g->plane[1 - p][m];
  }
  a.flags = g->haswall ? g->flags : nullptr;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.pitch = g->L.pitch;
  a.rs = g->L.rs;
  a.zs = g->L.zs;
  a.fzs = g->L.fzs;
  a.periodic = g->periodic;
  a.fx = g->F[0];
  a.fy = g->F[1];
  a.fz = g->F[2];
  a.sc_d = g->sc[0];
  a.sc_j = g->sc[1];
  a.is_d = 1.0 / g->sc[0];
  a.is_j = 1.0 / g->sc[1];
  return a;
}

extern "C" {

size_t lbt1_grid3d_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t q, int32_t prec, uint32_t options) {
  if (!valid3(nx, ny, nz) || (q != 19 && q != 27) || prec < LBT1_F64 || prec > LBT1_BF16S) return 0;
  return layout3(nx, ny, nz, prec, options).total;
}

lbt1_status lbt1_grid3d_create(const lbt1_grid3d_desc *d, lbt1_grid3d **out) {
  clear_error();
  if (!d || !out) return fail(LBT1_EINVAL, "null argument");
  *out = nullptr;
  if (!valid3(d->nx, d->ny, d->nz))
    return fail(LBT1_EINVAL, "grid %d x %d x %d: x, y 3..16384, z 1..16384", d->nx, d->ny, d->nz);
  if (d->q != 19 && d->q != 27) return fail(LBT1_EINVAL, "lattice D3Q%d: 19 or 27", d->q);
  if (d->prec < LBT1_F64 || d->prec > LBT1_BF16S) return fail(LBT1_EINVAL, "unknown precision %d", d->prec);
  if (d->wall != LBT1_WALL_PAPER && d->wall != LBT1_WALL_HALFWAY) return fail(LBT1_EINVAL, "unknown wall rule");
  if (d->periodic & ~7u) return fail(LBT1_EINVAL, "periodic mask %u", d->periodic);
  if (d->options & ~(uint32_t)LBT1_OPT_SNAPSHOT) return fail(LBT1_EINVAL, "unknown options %u", d->options);
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->force[a])) return fail(LBT1_EINVAL, "force must be finite");
  for (int a = 0; a < 2; ++a) {
    const double s = d->scale[a];
    int e;
    if (s != 0.0 && !(s > 0.0 && std::isfinite(s) && std::frexp(s, &e) == 0.5))
      return fail(LBT1_EINVAL, "scales must be 0 or positive powers of two");
  }
  int dev = 0, cus = 0;
  lbt1_status st = check_device(&dev, &cus);
  if (st) return st;
  lbt1_grid3d *g = new (std::nothrow) lbt1_grid3d();
  if (!g) return fail(LBT1_ENOMEM, "host allocation");
  g->device = dev;
  g->nx = d->nx;
  g->ny = d->ny;
  g->nz = d->nz;
  g->q = d->q;
  g->periodic = d->periodic;
  g->options = d->options;
  g->prec = d->prec;
  g->wall = d->wall;
  for (int a = 0; a < 3; ++a) g->F[a] = d->force[a];
  const bool scaled = d->prec == LBT1_F16S || d->prec == LBT1_BF16S;
  g->sc[0] = (scaled && d->scale[0] != 0.0) ? d->scale[0] : 1.0;
  g->sc[1] = (scaled && d->scale[1] != 0.0) ? d->scale[1] : 1.0;
  g->L = layout3(d->nx, d->ny, d->nz, d->prec, d->options);
  hipError_t e;
  if (d->device_buffer) {
    if (d->device_bytes < g->L.total || ((uintptr_t)d->device_buffer) % 256) {
      delete g;
      return fail(LBT1_EINVAL, "device buffer too small or not 256-byte aligned");
    }
    g->base = (char *)d->device_buffer;
  } else {
    void *p = nullptr;
    if ((e = hipMalloc(&p, g->L.total)) != hipSuccess) {
      delete g;
      return fail(LBT1_ENOMEM, "hipMalloc(%zu): %s", g->L.total, hipGetErrorString(e));
    }
    g->base = (char *)p;
    g->own_mem = true;
  }
  if (d->stream) {
    g->stream = (hipStream_t)d->stream;
  } else {
    if ((e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) != hipSuccess) {
      if (g->own_mem) hipFree(g->base);
      delete g;
      return hip_fail(e, "hipStreamCreate");
    }
    g->own_stream = true;
  }
  const size_t c = value_bytes(g->prec);
  for (int p = 0; p < 2; ++p)
    for (int m = 0; m < 4; ++m) g->plane[p][m] = g->base + (size_t)p * g->L.state + (size_t)m * g->L.pitch * c;
  for (int m = 0; m < 4; ++m)
    g->snap[m] = g->L.snap_off ? g->base + g->L.snap_off + (size_t)m * g->L.pitch * c : nullptr;
  g->flags = (uint8_t *)(g->base + g->L.flags_off);
  g->partials = (double *)(g->base + g->L.part_off);
  g->red_out = (double *)(g->base + g->L.out_off);
  if ((e = hipHostMalloc((void **)&g->red_host, 8 * sizeof(double), hipHostMallocDefault)) != hipSuccess) {
    if (g->own_stream) hipStreamDestroy(g->stream);
    if (g->own_mem) hipFree(g->base);
    delete g;
    return hip_fail(e, "hipHostMalloc");
  }
  *out = g;
  return LBT1_OK;
}

lbt1_status lbt1_grid3d_set_geometry(lbt1_grid3d *g, const uint8_t *flags, const double *rho, const double *jx,
                                     const double *jy, const double *jz) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const size_t n = (size_t)nx * ny * nz;
  bool any_fixed = false, any_nonfluid = false;
  for (size_t i = 0; flags && i < n; ++i) {
    if (flags[i] > LBT1_FIXED) return fail(LBT1_EINVAL, "flag %u at node %zu", flags[i], i);
    any_fixed |= flags[i] == LBT1_FIXED;
    any_nonfluid |= flags[i] != LBT1_FLUID;
  }
  if (any_fixed && !rho && !jx && !jy && !jz) return fail(LBT1_EINVAL, "FIXED nodes need moments");
  for (size_t i = 0; rho && i < n; ++i)
    if (!(rho[i] > 0.0) || !std::isfinite(rho[i])) return fail(LBT1_EINVAL, "rho[%zu] must be finite and > 0", i);
  const double *js[3] = {jx, jy, jz};
  for (int a = 0; a < 3; ++a)
    for (size_t i = 0; js[a] && i < n; ++i)
      if (!std::isfinite(js[a][i])) return fail(LBT1_EINVAL, "momentum %d at node %zu is not finite", a, i);
  const size_t c = value_bytes(g->prec);
  std::vector<char> stage;
  std::vector<uint8_t> fstage;
  std::vector<double> row(nx);
  try {
    stage.assign(g->L.state, 0);
    fstage.assign((size_t)g->L.fzs * nz, LBT1_SOLID);
  } catch (...) {
    return fail(LBT1_ENOMEM, "host staging");
  }
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y) {
      const size_t r0 = ((size_t)z * ny + y) * nx;
      for (int m = 0; m < 4; ++m) {
        const double *src = m == 0 ? rho : js[m - 1];
        for (int x = 0; x < nx; ++x) row[x] = src ? (m == 0 ? src[r0 + x] - 1.0 : src[r0 + x]) : 0.0;
        encode_values(g->prec, row.data(), nx, 1.0 / g->sc[m == 0 ? 0 : 1],
                      stage.data() + ((size_t)z * g->L.zs + (size_t)y * g->L.rs + (size_t)m * g->L.pitch) * c);
      }
      for (int x = 0; x < nx; ++x)
        fstage[(size_t)z * g->L.fzs + (size_t)y * g->L.pitch + x] = flags ? flags[r0 + x] : LBT1_FLUID;
    }
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int p = 0; p < 2; ++p)
    if ((e = hipMemcpy(g->base + (size_t)p * g->L.state, stage.data(), g->L.state, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy H2D");
  if (g->L.snap_off &&
      (e = hipMemcpy(g->base + g->L.snap_off, stage.data(), g->L.state, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy H2D");
  if ((e = hipMemcpy(g->flags, fstage.data(), fstage.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy H2D");
  g->haswall = any_nonfluid || g->periodic != 7u;
  lbt1_status st = bind3(g);
  if (st) return st;
  g->parity = 0;
  g->geometry = true;
  return LBT1_OK;
}

lbt1_status lbt1_grid3d_set_kernel(lbt1_grid3d *g, int32_t kernel) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  if (kernel != LBT1_KERNEL_AUTO && kernel != LBT1_KERNEL_GATHER && kernel != LBT1_KERNEL_STRIP)
    return fail(LBT1_EINVAL, "unknown kernel family %d", kernel);
  const int old = g->want;
  g->want = kernel;
  if (!g->geometry) return LBT1_OK;
  lbt1_status st = bind3(g);
  if (st) {
    g->want = old;
    bind3(g);
  }
  return st;
}

lbt1_status lbt1_grid3d_get_kernel(lbt1_grid3d *g, int32_t *kernel) {
  clear_error();
  if (!g || !kernel) return fail(LBT1_EINVAL, "null argument");
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  *kernel = g->tile ? LBT1_KERNEL_STRIP : LBT1_KERNEL_GATHER;
  return LBT1_OK;
}

lbt1_status lbt1_grid3d_step(lbt1_grid3d *g, int64_t n) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  if (n < 0) return fail(LBT1_EINVAL, "negative step count");
  if (!g->geometry) return fail(LBT1_ESTATE, "step before set_geometry");
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  const dim3 block = g->tile ? dim3(64 * kTile3Y, 1, 1) : dim3(64, 4, 1);
  // tile kernel: one block per tile, rounded up to a multiple of the 8 XCDs (the
  // kernel maps block b to a tile of XCD b % 8's contiguous range)
  const int tw = lane3(g) ? kLane3X : kTile3X;  // target columns per tile
  const long ntiles = (long)((g->nx + tw - 1) / tw) * ((g->ny + kTile3Y - 1) / kTile3Y) *
                      ((g->nz + zchunk_for(g->prec, g->haswall) - 1) / zchunk_for(g->prec, g->haswall));
  const dim3 grid = g->tile ? dim3((unsigned)((ntiles + 7) / 8 * 8), 1, 1) : dim3((g->nx + 63) / 64, (g->ny + 3) / 4, g->nz);
  for (int64_t s = 0; s < n; ++s) {
    Step3Args a = step3_args(g, g->parity);
    void *args[] = {&a};
    if ((e = hipLaunchKernel(g->kern, grid, block, args, 0, g->stream)) != hipSuccess)
      return hip_fail(e, "3-D step launch");
    g->parity ^= 1;
  }
  return LBT1_OK;
}

lbt1_status lbt1_grid3d_read_moments(lbt1_grid3d *g, double *rho, double *jx, double *jy, double *jz) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const size_t c = value_bytes(g->prec);
  std::vector<char> stage;
  try {
    stage.resize((size_t)nx * ny * nz * c);
  } catch (...) {
    return fail(LBT1_ENOMEM, "host staging");
  }
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  double *dst[4] = {rho, jx, jy, jz};
  for (int m = 0; m < 4; ++m) {
    if (!dst[m]) continue;
    // rows of all planes: ny * nz rows of nx values, row stride rs
    if ((e = hipMemcpy2D(stage.data(), (size_t)nx * c, g->plane[g->parity][m], (size_t)g->L.rs * c, (size_t)nx * c,
                         (size_t)ny * nz, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hipMemcpy2D D2H");
    decode_values(g->prec, stage.data(), (size_t)nx * ny * nz, g->sc[m == 0 ? 0 : 1], dst[m]);
    if (m == 0)
      for (size_t i = 0; i < (size_t)nx * ny * nz; ++i) dst[m][i] += 1.0;
  }
  return LBT1_OK;
}

lbt1_status lbt1_grid3d_reduce(lbt1_grid3d *g, uint32_t what, double *out) {
  clear_error();
  if (!g || !out) return fail(LBT1_EINVAL, "null argument");
  if (what & ~15u) return fail(LBT1_EINVAL, "unknown reduce bits %u", what);
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  if ((what & LBT1_REDUCE_RESIDUAL) && !g->L.snap_off) return fail(LBT1_EINVAL, "grid has no snapshot");
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  Reduce3Args a{};
  for (int m = 0; m < 4; ++m) {
    a.cur[m] = g->plane[g->parity][m];
    a.snap[m] = g->snap[m];
  }
  a.flags = g->haswall ? g->flags : nullptr;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.pitch = g->L.pitch;
  a.rs = g->L.rs;
  a.zs = g->L.zs;
  a.fzs = g->L.fzs;
  a.sc_d = g->sc[0];
  a.sc_j = g->sc[1];
  a.what = what;
  a.partials = g->partials;
  const long n = (long)g->nx * g->ny * g->nz;
  const int blocks = (int)std::min<long>(g->L.nparts, std::max<long>(1, (n + 1023) / 1024));
  void *args[] = {&a};
  if ((e = hipLaunchKernel(reduce3_kernel(g->prec), dim3(blocks), dim3(256), args, 0, g->stream)) != hipSuccess)
    return hip_fail(e, "reduce launch");
  const double *parts = g->partials;
  int np = blocks;
  double *ro = g->red_out;
  void *args2[] = {&parts, &np, &ro};
  if ((e = hipLaunchKernel((const void *)&k_reduce3_final, dim3(1), dim3(64), args2, 0, g->stream)) != hipSuccess)
    return hip_fail(e, "reduce launch");
  if ((e = hipMemcpyAsync(g->red_host, g->red_out, 8 * sizeof(double), hipMemcpyDeviceToHost, g->stream)) !=
      hipSuccess)
    return hip_fail(e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  const double *r = g->red_host;
  out[0] = r[6] + r[0];
  out[1] = r[1];
  out[2] = r[2];
  out[3] = r[3];
  out[4] = r[4];
  out[5] = r[5];
  out[6] = r[6];
  out[7] = 0.0;
  return LBT1_OK;
}

lbt1_status lbt1_grid3d_sync(lbt1_grid3d *g) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  hipError_t e = hipStreamSynchronize(g->stream);
  return e == hipSuccess ? LBT1_OK : hip_fail(e, "hipStreamSynchronize");
}

lbt1_status lbt1_grid3d_destroy(lbt1_grid3d *g) {
  clear_error();
  if (!g) return LBT1_OK;
  hipStreamSynchronize(g->stream);
  if (g->red_host) hipHostFree(g->red_host);
  if (g->own_stream) hipStreamDestroy(g->stream);
  if (g->own_mem) hipFree(g->base);
  delete g;
  return LBT1_OK;
}

}  // extern "C"

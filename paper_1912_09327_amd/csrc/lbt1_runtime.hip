// Host runtime and C ABI of liblbt1 (see include/lbt1.h).
//
// A grid owns (or borrows) one device allocation laid out as
//   planes[parity 0][d, jx, jy] planes[parity 1][d, jx, jy] flags [snapshot d, jx, jy]
//   reduction partials, reduction result
// Each plane is ny rows of `pitch` values (pitch = nx rounded up to 64), the
// structure-of-arrays form of the paper's R, U, V tables (Algorithm 1), with
// x fastest so a wavefront's loads of one row are contiguous.  The two
// parities are the paper's ping-pong copies; lbt1_step flips between them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/lbt1.h"
#include "lbt1_internal.hpp"
#include "lbt1_runtime.hpp"

namespace lbt1 {

// ----------------------------------------------------------------- errors
static thread_local std::string g_err;

lbt1_status fail(lbt1_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

lbt1_status hip_fail(hipError_t e, const char *what) {
  return fail(LBT1_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

void clear_error() { g_err.clear(); }

// ----------------------------------------------------------------- layout
size_t value_bytes(int prec) {
  switch (prec) {
    case LBT1_F64: return 8;
    case LBT1_F32: return 4;
    case LBT1_F16S:
    case LBT1_BF16S: return 2;
  }
  return 0;
}

static size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

Layout layout_of(int nx, int ny, int prec, uint32_t options) {
  Layout L{};
  const size_t c = value_bytes(prec);
  L.pitch = (int)round_up((size_t)nx, 64);
  L.interleaved = !(options & LBT1_OPT_PLANAR);
  const bool pop = options & LBT1_OPT_POPULATIONS;
  const int nf = pop ? 9 : 3;
  L.nfield = nf;
  const size_t plane = round_up((size_t)L.pitch * ny * c, 256);
  if (L.interleaved) {
    // [ny][nf][pitch]: a wavefront reading (writing) one lattice row touches one
    // contiguous stretch of the parity block
    L.rs = nf * L.pitch;
    for (int q = 0; q < nf; ++q) L.field_off[q] = (size_t)q * L.pitch * c;
    L.state = round_up((size_t)nf * L.pitch * ny * c, 256);
  } else {
    // [nf][ny][pitch]: separate planes
    L.rs = L.pitch;
    for (int q = 0; q < nf; ++q) L.field_off[q] = (size_t)q * plane;
    L.state = nf * plane;
  }
  L.flags_off = 2 * L.state;
  L.flags_bytes = round_up((size_t)L.pitch * ny, 256);
  size_t off = L.flags_off + L.flags_bytes;
  L.snap_off = 0;
  L.snap_rs = L.rs;
  for (int q = 0; q < 3; ++q) L.snap_field_off[q] = L.field_off[q];
  if (options & LBT1_OPT_SNAPSHOT) {
    L.snap_off = off;
    if (pop) {
      // the residual compares moments: three planes of rho - 1, jx, jy
      L.snap_rs = L.pitch;
      for (int q = 0; q < 3; ++q) L.snap_field_off[q] = (size_t)q * plane;
      off += 3 * plane;
    } else {
      off += L.state;
    }
  }
  L.psi_off = 0;
  if (pop && (options & LBT1_OPT_MULTIPHASE)) {
    L.psi_off = off;
    off += round_up((size_t)L.pitch * ny * (prec == LBT1_F64 ? 8 : 4), 256);
  }
  L.nparts = kReduceBlocks;
  L.part_off = off;
  off += round_up((size_t)L.nparts * 6 * sizeof(double), 256);
  L.out_off = off;
  off += 256;
  L.trash_off = off;  // 3 KiB: stores of lanes / rows outside the grid land here (one region per field)
  off += 3 * kTrashRegion;
  L.total = off;
  return L;
}

static bool valid_shape(int nx, int ny) { return nx >= 3 && ny >= 3 && nx <= 65536 && ny <= 65536; }
static bool valid_prec(int p) { return p >= LBT1_F64 && p <= LBT1_BF16S; }

static bool pow2_or_zero(double s) {
  if (s == 0.0) return true;
  if (!(s > 0.0) || !std::isfinite(s)) return false;
  int e;
  double m = std::frexp(s, &e);
  return m == 0.5;
}

// ----------------------------------------------------------------- host codecs
// Round a double to the nearest value with `mant` significand bits (round half
// to even), normal exponent >= emin, gradual underflow below; returns +-inf
// above `maxv`.  Used for IEEE binary16 (11 bits, emin -14, max 65504) and
// bfloat16 (8 bits, emin -126, max (2 - 2^-7) 2^127).
static double round_to_format(double x, int mant, int emin, double maxv) {
  if (!std::isfinite(x) || x == 0.0) return x;
  int e;
  std::frexp(x, &e);               // x = m 2^e, 0.5 <= |m| < 1
  int q = std::max(e, emin + 1) - mant;  // quantum exponent
  double r = std::nearbyint(std::ldexp(x, -q));  // default rounding mode: to nearest even
  double y = std::ldexp(r, q);
  if (std::fabs(y) > maxv) return std::copysign(INFINITY, x);
  return y;
}

static uint16_t encode_half(double v) {
  double r = round_to_format(v, 11, -14, 65504.0);
  _Float16 h = (_Float16)(float)r;  // exact: r is representable
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}
static uint16_t encode_bf16(double v) {
  if (std::isnan(v)) return 0x7fc0;
  double r = round_to_format(v, 8, -126, std::ldexp(255.0, 120));
  float f = (float)r;  // exact
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}
static double decode_half(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return (double)(float)h;
}
static double decode_bf16(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

void encode_values(int prec, const double *in, size_t n, double inv_scale, void *out) {
  switch (prec) {
    case LBT1_F64: {
      double *o = (double *)out;
      for (size_t i = 0; i < n; ++i) o[i] = in[i];
      break;
    }
    case LBT1_F32: {
      float *o = (float *)out;
      for (size_t i = 0; i < n; ++i) o[i] = (float)in[i];
      break;
    }
    case LBT1_F16S: {
      uint16_t *o = (uint16_t *)out;
      for (size_t i = 0; i < n; ++i) o[i] = encode_half(in[i] * inv_scale);
      break;
    }
    case LBT1_BF16S: {
      uint16_t *o = (uint16_t *)out;
      for (size_t i = 0; i < n; ++i) o[i] = encode_bf16(in[i] * inv_scale);
      break;
    }
  }
}

void decode_values(int prec, const void *in, size_t n, double scale, double *out) {
  switch (prec) {
    case LBT1_F64: {
      const double *s = (const double *)in;
      for (size_t i = 0; i < n; ++i) out[i] = s[i];
      break;
    }
    case LBT1_F32: {
      const float *s = (const float *)in;
      for (size_t i = 0; i < n; ++i) out[i] = s[i];
      break;
    }
    case LBT1_F16S: {
      const uint16_t *s = (const uint16_t *)in;
      for (size_t i = 0; i < n; ++i) out[i] = decode_half(s[i]) * scale;
      break;
    }
    case LBT1_BF16S: {
      const uint16_t *s = (const uint16_t *)in;
      for (size_t i = 0; i < n; ++i) out[i] = decode_bf16(s[i]) * scale;
      break;
    }
  }
}

// ----------------------------------------------------------------- device check
lbt1_status check_device(int *dev_out, int *cus) {
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return fail(LBT1_EDEVICE, "no HIP device is visible: hipGetDeviceCount: %s (%d)", hipGetErrorString(e), (int)e);
  if (ndev <= 0) return fail(LBT1_EDEVICE, "no HIP device is visible");
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(LBT1_EDEVICE, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  *dev_out = dev;
  if (cus) *cus = prop.multiProcessorCount;
  return LBT1_OK;
}

// ----------------------------------------------------------------- kernel selection
// A strip kernel with vec columns per lane fits a grid when vec divides nx, or
// when x is not periodic: then the last chunk of a row runs past nx into the
// row padding (pitch is nx rounded up to 64, a multiple of vec), whose flags
// are SOLID, exactly like the outside of a non-periodic axis.
static bool strip_fits(int nx, int vec, bool periodic_x) { return vec >= 1 && (nx % vec == 0 || !periodic_x); }
static int chunks_of(int nx, int vec) { return (nx + vec - 1) / vec; }

const StepKernel *find_kernel(int prec, bool haswall, int wall, int kind, int vec, int rows, int fuse, bool sc) {
  int n = 0;
  const StepKernel *t = step_kernels(&n);
  for (int i = 0; i < n; ++i) {
    const StepKernel &k = t[i];
    if (k.prec != prec || k.kind != kind || (k.haswall != 0) != haswall || (k.sc != 0) != sc) continue;
    if (haswall && k.wall != wall) continue;
    if (kind == KIND_STRIP && (k.vec != vec || k.rows != rows || k.steps != fuse)) continue;
    return &k;
  }
  return nullptr;
}

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int, int, int>, lbt1_kernel_config> g_tuned;

static std::tuple<int, int, int, int, int, int> tune_key(const lbt1_grid *g) {
  // multiphase grids tune separately (precision code offset by 8); the periodic
  // bits take part because a strip shape that fits a walled grid of odd width
  // does not fit one periodic in x
  return std::make_tuple(g->prec + (g->mp ? 8 : 0), (int)g->haswall, g->haswall ? g->wall : 0, (int)(g->periodic & 3u),
                         g->nx, g->ny);
}

// Default without a tuned entry: the gather kernel for tiny grids, else the
// widest built strip kernel that fits nx (see strip_fits) and whose strip is not much
// wider than the grid, with short strips (6 rows) when tall ones would not give
// every CU several wavefronts (a strip's rows are walked one after another, so
// its length sets the latency of a step).
lbt1_kernel_config heuristic_config(int prec, bool haswall, int wall, int nx, int ny, int cus, bool sc, bool px) {
  lbt1_kernel_config c{};
  if ((long)nx * ny < 64 * 64) {
    c.kernel = LBT1_KERNEL_GATHER;
    return c;
  }
  if (sc) {
    // multiphase: strips (2 columns per lane) on periodic grids without walls that
    // give every CU two strips or more, else one thread per node.  FP32 grids with
    // two 22-row strips of two fused steps per CU take those (drop fields: 71.5
    // against 82.4 us per step at 4096^2, 232 against 284 at 8192^2).
    c.kernel = LBT1_KERNEL_GATHER;
    const long fused = (long)((nx / 4 + 61) / 62) * ((ny + 21) / 22);
    if (prec == LBT1_F32 && !haswall && nx % 4 == 0 && fused >= 2L * cus &&
        find_kernel(prec, false, 0, KIND_STRIP, 4, 22, 2, true)) {
      c.kernel = LBT1_KERNEL_STRIP;
      c.vec = 4;
      c.rows = 22;
      c.fuse = 2;
      return c;
    }
    const long strips = (long)((nx / 2 + 61) / 62) * ((ny + 13) / 14);
    if (!haswall && nx % 2 == 0 && strips >= 2L * cus && find_kernel(prec, false, 0, KIND_STRIP, 2, 14, 1, true)) {
      c.kernel = LBT1_KERNEL_STRIP;
      c.vec = 2;
      c.rows = 14;
      c.fuse = 1;
    }
    return c;
  }
  c.kernel = LBT1_KERNEL_STRIP;
  c.waves = 0;
  c.vec = 1;
  c.fuse = 1;
  if (!haswall) {
    // several steps per pass (measured fastest on large periodic grids): FP32 three
    // steps at 4 columns per lane; FP64 two at 2 (registers); 16-bit storage two at
    // 2 columns. Tall strips where there are enough of them: these kernels are
    // bound by arithmetic, and a taller strip repeats fewer halo rows.
    const bool half = prec == LBT1_F16S || prec == LBT1_BF16S;
    const int v = prec == LBT1_F32 ? 4 : 2;
    const int k = prec == LBT1_F32 ? 3 : 2;
    if (nx % v == 0 && 62 * v <= std::max(62, nx)) {
      const long sx = (nx / v + 61) / 62;
      int r = half ? (sx * ((ny + 29) / 30) >= 8L * cus ? 30 : 6)
                   : prec == LBT1_F32 ? (sx * ((ny + 21) / 22) >= 8L * cus ? 22 : 14) : 6;
      if (r == 22) {
        // three-step strips run two wavefronts per SIMD (8 per CU): a launch of W
        // strips takes about ceil(W / slots) rounds of one strip's walk, 3 R + 12
        // stage-row emissions for R stored rows.  28 rows where that is no longer
        // than at 22 (the 8192^2 field: 5 rounds of 96 against 7 of 78).
        const long slots = 8L * cus;
        const long w22 = sx * ((ny + 21) / 22), w28 = sx * ((ny + 27) / 28);
        if ((w28 + slots - 1) / slots * 96 <= (w22 + slots - 1) / slots * 78) r = 28;
      }
      if (find_kernel(prec, false, 0, KIND_STRIP, v, r, k, false)) {
        c.vec = v;
        c.rows = r;
        c.fuse = k;
        c.waves = 0;
        return c;
      }
    }
  }
  if (haswall && strip_fits(nx, 2, px) && 62 * 2 <= std::max(62, nx)) {
    // two fused steps at 2 columns per lane on grids with walls (measured on
    // cavities of side 256, 1024 and 4096: fastest in FP32 and 16-bit storage at
    // every size, in FP64 at 256 and 4096 and within 6 % at 1024).  Strip height:
    // up to 512 x 512 nodes 2 rows (the step is bound by the latency of a strip's
    // walk: 2.9 us against 5.0 at 6 rows on a 256^2 cavity), else 14 where there
    // are enough strips, else 6.  30 rows where a launch then takes at least 5 %
    // less of rounds of resident wavefronts times walk length (2 R + 6 stage rows)
    // than at 14: on the 8192^2 cavity 6 rounds of 66 against 13 of 34 (FP32 0.190
    // against 0.204 ms per step); at 4096^2 2 of 66 against 4 of 34, and 14 rows
    // are 1-4 % faster.
    const long sx = (chunks_of(nx, 2) + 61) / 62;
    int r = (long)nx * ny <= 512L * 512 ? 2 : sx * ((ny + 13) / 14) >= 8L * cus ? 14 : 6;
    const StepKernel *k30 = find_kernel(prec, true, wall, KIND_STRIP, 2, 30, 2, false);
    if (r == 14 && k30) {
      int per_cu = 0;  // 256-thread blocks per CU
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k30->fn, 256, 0) == hipSuccess && per_cu > 0) {
        const long slots = 4L * per_cu * cus;
        const long w14 = sx * ((ny + 13) / 14), w30 = sx * ((ny + 29) / 30);
        if ((w30 + slots - 1) / slots * 66 * 20 < (w14 + slots - 1) / slots * 34 * 19) r = 30;
      }
    }
    if (find_kernel(prec, true, wall, KIND_STRIP, 2, r, 2, false)) {
      c.vec = 2;
      c.rows = r;
      c.fuse = 2;
      c.waves = 0;
      return c;
    }
  }
  const int cands[] = {8, 4, 2, 1};
  for (int v : cands) {
    if (strip_fits(nx, v, px) && 62 * v <= std::max(62, nx) && find_kernel(prec, haswall, wall, KIND_STRIP, v, 14, 1, false)) {
      c.vec = v;
      break;
    }
  }
  const long tall = (long)((chunks_of(nx, c.vec) + 61) / 62) * ((ny + 13) / 14);
  c.rows = tall < 8L * cus ? 6 : 14;
  // A grid of up to 512 x 512 nodes is bound by the latency of a strip's walk
  // down its rows, not by bandwidth: one column per lane gives the most wavefronts
  // for the same short walk (measured on cavities of side 128 to 512: 1 column per
  // lane and 6 rows fastest, or within 5 % of the gather kernel).
  if ((long)nx * ny <= 512L * 512 && c.rows == 6 && find_kernel(prec, haswall, wall, KIND_STRIP, 1, 6, 1, false))
    c.vec = 1;
  return c;
}

// Resolve a configuration into a kernel and launch shape for grid g.
lbt1_status bind_config(lbt1_grid *g, const lbt1_kernel_config &want, int cus) {
  if (g->pop) {
    // one kernel: a thread per node (the gather launch shape)
    const StepKernel *k = find_kernel(g->prec, g->haswall, g->wall, KIND_BGK, 0, 0, 1, g->mp);
    if (!k) return fail(LBT1_EINVAL, "no built population kernel at this precision");
    g->kern = g->kern1 = k;
    g->kern2 = nullptr;
    g->cfg = lbt1_kernel_config{};
    g->cfg.kernel = LBT1_KERNEL_GATHER;
    g->cfg.fuse = 1;
    const int tiles = ((g->nx + 63) / 64) * ((g->ny + 3) / 4);
    g->block = g->block1 = dim3(256, 1, 1);
    g->grid = g->grid1 = dim3((tiles + 7) / 8 * 8, 1, 1);
    g->graph_valid = false;
    return LBT1_OK;
  }
  lbt1_kernel_config c = want;
  if (c.kernel == LBT1_KERNEL_AUTO) {
    lbt1_kernel_config tuned{};
    bool have = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tuned.find(tune_key(g));
      if (it != g_tuned.end()) tuned = it->second, have = true;
    }
    // a tuned entry that does not bind this grid (it should always, being keyed on
    // everything bind_config checks) yields to the heuristic rather than failing
    if (have && bind_config(g, tuned, cus) == LBT1_OK) return LBT1_OK;
    if (have) clear_error();
    c = heuristic_config(g->prec, g->haswall, g->wall, g->nx, g->ny, cus, g->mp, g->periodic & 1u);
  }
  const StepKernel *k = nullptr, *k1 = nullptr, *k2 = nullptr;
  if (c.kernel == LBT1_KERNEL_GATHER) {
    k = k1 = find_kernel(g->prec, g->haswall, g->wall, KIND_GATHER, 0, 0, 1, g->mp);
    k2 = nullptr;
    c.vec = c.rows = c.waves = 0;
    c.fuse = 1;
  } else if (c.kernel == LBT1_KERNEL_STRIP) {
    if (!strip_fits(g->nx, c.vec, g->periodic & 1u))
      return fail(LBT1_EINVAL, "strip kernel: vec %d does not divide nx %d on a grid periodic in x", c.vec, g->nx);
    if ((long)chunks_of(g->nx, c.vec) * c.vec > g->L.pitch)
      return fail(LBT1_EINVAL, "strip kernel: vec %d chunks overrun the row pitch %d", c.vec, g->L.pitch);
    if (c.waves < 0 || c.waves > 32) return fail(LBT1_EINVAL, "waves %d out of range", c.waves);
    if (c.fuse == 0) c.fuse = 1;
    if (c.fuse < 1 || c.fuse > c.vec) return fail(LBT1_EINVAL, "fuse %d must be between 1 and vec %d", c.fuse, c.vec);
    if (c.fuse > 2 && g->haswall)
      return fail(LBT1_EINVAL, "three fused steps need a grid periodic in x and y without SOLID or FIXED nodes");
    if (c.fuse > 2 && g->mp) return fail(LBT1_EINVAL, "multiphase grids take one or two steps per launch");
    if (g->mp && g->haswall)
      return fail(LBT1_EINVAL, "multiphase strips need a grid periodic in x and y without SOLID nodes (use gather)");
    k = find_kernel(g->prec, g->haswall, g->wall, KIND_STRIP, c.vec, c.rows, c.fuse, g->mp);
    k1 = find_kernel(g->prec, g->haswall, g->wall, KIND_STRIP, c.vec, c.rows, 1, g->mp);
    // a fused shape with no single-step strip of its height finishes odd step
    // counts with the gather kernel (same arithmetic, own launch shape)
    if (k && !k1 && c.fuse > 1) k1 = find_kernel(g->prec, g->haswall, g->wall, KIND_GATHER, 0, 0, 1, g->mp);
    // three steps per launch: remainders of two steps take the two-step kernel of
    // the same strip shape where one is built
    if (c.fuse == 3) k2 = find_kernel(g->prec, g->haswall, g->wall, KIND_STRIP, c.vec, c.rows, 2, g->mp);
  } else {
    return fail(LBT1_EINVAL, "unknown kernel family %d", c.kernel);
  }
  if (!k || !k1)
    return fail(LBT1_EINVAL, "no built kernel for vec %d rows %d fuse %d at this precision", c.vec, c.rows, c.fuse);
  g->kern = k;
  g->kern1 = k1;
  g->kern2 = k2;
  g->cfg = c;
  g->cfg.kernel = k->kind == KIND_GATHER ? LBT1_KERNEL_GATHER : LBT1_KERNEL_STRIP;
  if (k->kind == KIND_GATHER) {
    g->block = dim3(64, 4, 1);
    g->grid = dim3((g->nx + 63) / 64, (g->ny + 3) / 4, 1);
  } else {
    StripMap &m = g->map;
    m.strips_x = (chunks_of(g->nx, c.vec) + 61) / 62;  // 62 chunks of vec columns per strip
    m.strips_y = (g->ny + c.rows - 1) / c.rows;
    const int strips = m.strips_x * m.strips_y;
    m.units = (strips + 3) / 4;
    int blocks;
    if (c.waves > 0) {
      // c.waves wavefronts per CU, 4 per block, a multiple of 8 blocks (one range per XCD)
      blocks = std::max(8, (cus * c.waves / 4) / 8 * 8);
      blocks = std::min(blocks, (m.units + 7) / 8 * 8);
      m.persistent = 1;
    } else {
      blocks = (m.units + 7) / 8 * 8;
      m.persistent = 0;
    }
    m.per_xcd = (m.units + 7) / 8;
    g->block = dim3(256, 1, 1);
    g->grid = dim3(blocks, 1, 1);
  }
  g->block1 = g->block;
  g->grid1 = g->grid;
  if (k1->kind == KIND_GATHER && k->kind != KIND_GATHER) {
    g->block1 = dim3(64, 4, 1);
    g->grid1 = dim3((g->nx + 63) / 64, (g->ny + 3) / 4, 1);
  }
  g->graph_valid = false;
  return LBT1_OK;
}

StepArgs step_args(const lbt1_grid *g, int src_parity) {
  StepArgs a{};
  for (int q = 0; q < 3; ++q) {
    a.src[q] = g->plane[src_parity][q];
    a.dst[q] = g->plane[1 - src_parity][q];
  }
  a.flags = g->haswall ? g->flags : nullptr;
  a.nx = g->nx;
  a.ny = g->ny;
  a.pitch = g->L.pitch;
  a.rs = g->L.rs;
  a.periodic = g->periodic;
  a.fx = g->F[0];
  a.fy = g->F[1];
  a.sc_d = g->sc[0];
  a.sc_j = g->sc[1];
  a.is_d = 1.0 / g->sc[0];
  a.is_j = 1.0 / g->sc[1];
  a.trash = g->base + g->L.trash_off;
  a.sc_G = g->sc_G;
  a.sc_rho0 = g->sc_rho0;
  return a;
}

BgkArgs bgk_args(const lbt1_grid *g, int src_parity) {
  BgkArgs a{};
  for (int q = 0; q < 9; ++q) {
    a.src[q] = g->plane[src_parity][q];
    a.dst[q] = g->plane[1 - src_parity][q];
  }
  a.flags = g->haswall ? g->flags : nullptr;
  a.nx = g->nx;
  a.ny = g->ny;
  a.pitch = g->L.pitch;
  a.rs = g->L.rs;
  a.periodic = g->periodic;
  a.fx = g->tau * g->F[0];
  a.fy = g->tau * g->F[1];
  a.omega = 1.0 / g->tau;
  a.sc = g->sc[0];
  a.is = 1.0 / g->sc[0];
  a.tiles_x = (g->nx + 63) / 64;
  a.tiles = a.tiles_x * ((g->ny + 3) / 4);
  a.per_xcd = (a.tiles + 7) / 8;
  a.psi = g->psi;
  a.sc_G = g->sc_G;
  a.sc_rho0 = g->sc_rho0;
  a.tau = g->tau;
  a.bfx = g->F[0];
  a.bfy = g->F[1];
  return a;
}

// One launch of kernel k (g->kern, or its single-step companion g->kern1,
// which has the same launch shape) reading parity src_parity.
hipError_t launch_step(lbt1_grid *g, const StepKernel *k, int src_parity, hipStream_t s) {
  if (k->kind == KIND_BGK) {
    BgkArgs b = bgk_args(g, src_parity);
    void *args[] = {&b};
    if (g->mp) {
      hipError_t e = hipLaunchKernel(bgk_psi_kernel(g->prec), g->grid, g->block, args, 0, s);
      if (e != hipSuccess) return e;
    }
    return hipLaunchKernel(k->fn, g->grid, g->block, args, 0, s);
  }
  StepArgs a = step_args(g, src_parity);
  if (k->kind == KIND_GATHER) {
    void *args[] = {&a};
    const bool companion = k == g->kern1 && k != g->kern;
    return hipLaunchKernel(k->fn, companion ? g->grid1 : g->grid, companion ? g->block1 : g->block, args, 0, s);
  }
  StripMap m = g->map;
  void *args[] = {&a, &m};
  return hipLaunchKernel(k->fn, g->grid, g->block, args, 0, s);
}

// A graph of kBurst / K launches (K = g->kern->steps) starting from parity p:
// it advances burst_steps(g) steps and flips the parity once per launch.
static const int kBurst = 64;

static int burst_launches(const lbt1_grid *g) { return kBurst / g->kern->steps; }
static int burst_steps(const lbt1_grid *g) { return burst_launches(g) * g->kern->steps; }

static lbt1_status build_burst(lbt1_grid *g, int p) {
  hipGraph_t graph = nullptr;
  hipError_t e = hipGraphCreate(&graph, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");
  hipGraphNode_t prev = nullptr;
  const int launches = burst_launches(g);
  std::vector<StepArgs> argv(launches);
  std::vector<BgkArgs> bargv(g->pop ? launches : 0);
  StripMap m = g->map;
  for (int s = 0; s < launches; ++s) {
    argv[s] = step_args(g, (p + s) & 1);
    if (g->pop) bargv[s] = bgk_args(g, (p + s) & 1);
    void *args_gather[] = {g->pop ? (void *)&bargv[s] : (void *)&argv[s]};
    void *args_strip[] = {&argv[s], &m};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(g->kern->fn);
    kp.gridDim = g->grid;
    kp.blockDim = g->block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = g->kern->kind == KIND_STRIP ? args_strip : args_gather;
    kp.extra = nullptr;
    hipGraphNode_t node;
    if (g->pop && g->mp) {
      // multiphase population grids: the psi pass before each step
      hipKernelNodeParams pp = kp;
      pp.func = const_cast<void *>(bgk_psi_kernel(g->prec));
      e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &pp);
      if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphAddKernelNode");
      }
      prev = node;
    }
    e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e != hipSuccess) {
      hipGraphDestroy(graph);
      return hip_fail(e, "hipGraphAddKernelNode");
    }
    prev = node;
  }
  if (g->burst[p]) hipGraphExecDestroy(g->burst[p]);
  g->burst[p] = nullptr;
  e = hipGraphInstantiate(&g->burst[p], graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return LBT1_OK;
}

static void drop_bursts(lbt1_grid *g) {
  for (int p = 0; p < 2; ++p)
    if (g->burst[p]) {
      hipGraphExecDestroy(g->burst[p]);
      g->burst[p] = nullptr;
    }
  g->graph_valid = false;
}

lbt1_status enqueue_steps(lbt1_grid *g, int64_t n, hipStream_t s, bool use_graph) {
  hipError_t e;
  const int bs = burst_steps(g);
  if (use_graph && n >= bs) {
    if (!g->graph_valid) {
      drop_bursts(g);
      g->graph_valid = true;
    }
    while (n >= bs) {
      const int p = g->parity;
      if (!g->burst[p]) {
        lbt1_status st = build_burst(g, p);
        if (st) return st;
      }
      if ((e = hipGraphLaunch(g->burst[p], s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      n -= bs;
      g->steps += bs;
      g->parity ^= burst_launches(g) & 1;
    }
  }
  const int K = g->kern->steps;
  // With a two-step companion the remainder after three-step launches is covered
  // by two-step launches: one for 2 left, two for 1 left when the single-step
  // companion is the (slower) gather kernel and at least 4 steps are asked for.
  int64_t tail2 = 0;
  if (g->kern2) {
    if (n % K == 2) tail2 = 1;
    if (n % K == 1 && n >= 4 && g->kern1->kind == KIND_GATHER) tail2 = 2;
  }
  for (; n - 2 * tail2 >= K; n -= K) {
    if ((e = launch_step(g, g->kern, g->parity, s)) != hipSuccess) return hip_fail(e, "step launch");
    g->parity ^= 1;
    g->steps += K;
  }
  for (; tail2 > 0; --tail2, n -= 2) {
    if ((e = launch_step(g, g->kern2, g->parity, s)) != hipSuccess) return hip_fail(e, "step launch");
    g->parity ^= 1;
    g->steps += 2;
  }
  for (; n > 0; --n) {
    if ((e = launch_step(g, g->kern1, g->parity, s)) != hipSuccess) return hip_fail(e, "step launch");
    g->parity ^= 1;
    g->steps += 1;
  }
  return LBT1_OK;
}

// Number of partial rows (reduction blocks) the partial pass of grid g writes.
static int reduce_blocks(const lbt1_grid *g) {
  const long n = (long)g->nx * g->ny;
  return (int)std::min<long>(g->L.nparts, std::max<long>(1, (n + 1023) / 1024));
}

// The two reduction passes of grid g on stream s: block partials into
// `partials` (reduce_blocks(g) rows of six doubles), then one wavefront combines
// them into `out`: the six raw slots, or with user_slots the slots as
// lbt1_reduce reports them (k_reduce_final_out).
static lbt1_status enqueue_reduce_into(lbt1_grid *g, uint32_t what, hipStream_t s, double *partials, double *out,
                                       bool user_slots) {
  const int blocks = reduce_blocks(g);
  hipError_t e;
  if (g->pop) {
    BgkReduceArgs a{};
    for (int q = 0; q < 9; ++q) a.cur[q] = g->plane[g->parity][q];
    for (int q = 0; q < 3; ++q) a.snap[q] = g->snap[q];
    a.flags = g->haswall ? g->flags : nullptr;
    a.nx = g->nx;
    a.ny = g->ny;
    a.pitch = g->L.pitch;
    a.rs = g->L.rs;
    a.snap_rs = g->L.snap_rs;
    a.sc = g->sc[0];
    a.sc_d = g->sc[0];
    a.sc_j = g->sc[1];
    a.is_d = 1.0 / g->sc[0];
    a.is_j = 1.0 / g->sc[1];
    a.what = what;
    a.partials = partials;
    void *args[] = {&a};
    e = hipLaunchKernel(bgk_reduce_partial_kernel(g->prec), dim3(blocks), dim3(256), args, 0, s);
  } else {
    ReduceArgs a{};
    for (int q = 0; q < 3; ++q) {
      a.cur[q] = g->plane[g->parity][q];
      a.snap[q] = g->snap[q];
    }
    a.flags = g->haswall ? g->flags : nullptr;
    a.nx = g->nx;
    a.ny = g->ny;
    a.pitch = g->L.pitch;
    a.rs = g->L.rs;
    a.sc_d = g->sc[0];
    a.sc_j = g->sc[1];
    a.what = what;
    a.partials = partials;
    void *args[] = {&a};
    e = hipLaunchKernel(reduce_partial_kernel(g->prec), dim3(blocks), dim3(256), args, 0, s);
  }
  if (e != hipSuccess) return hip_fail(e, "reduce launch");
  const double *parts = partials;
  int np = blocks;
  if (user_slots) {
    void *args2[] = {&parts, &np, &what, &out};
    e = hipLaunchKernel(reduce_final_out_kernel(), dim3(1), dim3(64), args2, 0, s);
  } else {
    void *args2[] = {&parts, &np, &out};
    e = hipLaunchKernel(reduce_final_kernel(), dim3(1), dim3(64), args2, 0, s);
  }
  if (e != hipSuccess) return hip_fail(e, "reduce launch");
  return LBT1_OK;
}

lbt1_status enqueue_reduce(lbt1_grid *g, uint32_t what, hipStream_t s) {
  return enqueue_reduce_into(g, what, s, g->partials, g->red_out, false);
}

// ----------------------------------------------------------------- allocation-free reduction
// Partial rows of lbt1_reduce_noalloc, in a file-scope device array instead of
// the grid's workspace: kReduceBlocks rows of six doubles (48 KiB on every
// device the library runs on, held until the process ends).  In host code the
// name `scratch` is only a stand-in for the symbol; its device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
constexpr int kScratchRows = kReduceBlocks;
static __device__ __align__(256) double scratch[kScratchRows * 6];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// The address of `scratch` on device dev (which must be current).
static lbt1_status scratch_on(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(LBT1_EDEVICE, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(LBT1_EDEVICE, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return LBT1_OK;
}

// D2Q9 tables of section 2 for the host-side initialisation of population grids.
static const int kHostEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int kHostEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double kHostW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Populations of a stored-population grid at t = 0: the equilibrium
// (Eq. maxwellboltzmann, FP64) of each FLUID node's moments, that of the
// moments with the force shift tau F for FIXED nodes (what they send every
// step), w_q for SOLID nodes; stored as deviations f_q - w_q.
static lbt1_status set_geometry_pop(lbt1_grid *g, const uint8_t *flags, const double *rho, const double *jx,
                                    const double *jy) {
  const int nx = g->nx, ny = g->ny, pitch = g->L.pitch;
  const size_t c = value_bytes(g->prec);
  const size_t plane = (size_t)pitch * ny;
  std::vector<char> stage, sstage;
  std::vector<uint8_t> fstage;
  std::vector<double> rows;
  try {
    stage.assign(g->L.state, 0);
    fstage.assign(plane, LBT1_SOLID);
    if (g->snap[0]) sstage.assign(g->L.snap_field_off[2] + plane * c, 0);
    rows.assign((size_t)12 * nx, 0.0);
    g->given_idx.clear();
    g->given_val.clear();
  } catch (...) {
    return fail(LBT1_ENOMEM, "host staging");
  }
  double *mom = rows.data() + (size_t)9 * nx;  // rho - 1, jx, jy of one row
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      const size_t i = (size_t)y * nx + x;
      const uint8_t fl = flags ? flags[i] : LBT1_FLUID;
      const double r = rho ? rho[i] : 1.0, a = jx ? jx[i] : 0.0, b = jy ? jy[i] : 0.0;
      if (fl != LBT1_FLUID) {
        g->given_idx.push_back(i);
        g->given_val.insert(g->given_val.end(), {r, a, b});
      }
      mom[x] = r - 1.0;
      mom[nx + x] = a;
      mom[2 * nx + x] = b;
      if (fl == LBT1_SOLID) {
        // zero-velocity equilibrium of the given density (never streamed; read by
        // the multiphase psi pass)
        for (int q = 0; q < 9; ++q) rows[(size_t)q * nx + x] = kHostW[q] * (r - 1.0);
        continue;
      }
      const double shift = fl == LBT1_FIXED ? g->tau : 0.0;
      const double ux = (a + shift * g->F[0]) / r, uy = (b + shift * g->F[1]) / r;
      const double usq = ux * ux + uy * uy;
      for (int q = 0; q < 9; ++q) {
        const double eu = kHostEx[q] * ux + kHostEy[q] * uy;
        rows[(size_t)q * nx + x] = kHostW[q] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq) - kHostW[q];
      }
    }
    for (int q = 0; q < 9; ++q)
      encode_values(g->prec, rows.data() + (size_t)q * nx, nx, 1.0 / g->sc[0],
                    stage.data() + g->L.field_off[q] + (size_t)y * g->L.rs * c);
    if (g->snap[0])
      for (int q = 0; q < 3; ++q)
        encode_values(g->prec, mom + (size_t)q * nx, nx, 1.0 / g->sc[q == 0 ? 0 : 1],
                      sstage.data() + g->L.snap_field_off[q] + (size_t)y * g->L.snap_rs * c);
    for (int x = 0; x < nx; ++x) fstage[(size_t)y * pitch + x] = flags ? flags[(size_t)y * nx + x] : LBT1_FLUID;
  }
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int p = 0; p < 2; ++p)
    if ((e = hipMemcpy(g->base + (size_t)p * g->L.state, stage.data(), g->L.state, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy H2D");
  if (g->snap[0] && (e = hipMemcpy(g->base + g->L.snap_off, sstage.data(), sstage.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy H2D");
  if ((e = hipMemcpy(g->flags, fstage.data(), plane, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy H2D");
  return LBT1_OK;
}

// Decode the populations of rows y0..y0+h-1, columns x0..x0+w-1 of the current
// parity into f[q][h][w] (deviations plus w_q).
static lbt1_status read_pop_window(lbt1_grid *g, int x0, int y0, int w, int h, std::vector<double> &f) {
  const size_t c = value_bytes(g->prec);
  const size_t n = (size_t)w * h;
  std::vector<char> stage;
  try {
    stage.resize(n * c);
    f.resize(9 * n);
  } catch (...) {
    return fail(LBT1_ENOMEM, "host staging");
  }
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int q = 0; q < 9; ++q) {
    const char *src = (const char *)g->plane[g->parity][q] + ((size_t)y0 * g->L.rs + x0) * c;
    if ((e = hipMemcpy2D(stage.data(), (size_t)w * c, src, (size_t)g->L.rs * c, (size_t)w * c, h,
                         hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hipMemcpy2D D2H");
    double *dst = f.data() + (size_t)q * n;
    decode_values(g->prec, stage.data(), n, g->sc[0], dst);
    for (size_t i = 0; i < n; ++i) dst[i] += kHostW[q];
  }
  return LBT1_OK;
}

}  // namespace lbt1

using namespace lbt1;

// =================================================================== C ABI
extern "C" {

const char *lbt1_last_error(void) { return g_err.c_str(); }

size_t lbt1_grid_bytes(int32_t nx, int32_t ny, int32_t prec, uint32_t options) {
  if (!valid_shape(nx, ny) || !valid_prec(prec)) return 0;
  return layout_of(nx, ny, prec, options).total;
}

lbt1_status lbt1_create_grid(const lbt1_grid_desc *d, lbt1_grid **out) {
  clear_error();
  if (!d || !out) return fail(LBT1_EINVAL, "null argument");
  *out = nullptr;
  if (!valid_shape(d->nx, d->ny)) return fail(LBT1_EINVAL, "grid %d x %d: each side must be 3..65536", d->nx, d->ny);
  if (!valid_prec(d->prec)) return fail(LBT1_EINVAL, "unknown precision %d", d->prec);
  if (d->wall != LBT1_WALL_PAPER && d->wall != LBT1_WALL_HALFWAY) return fail(LBT1_EINVAL, "unknown wall rule %d", d->wall);
  if (d->periodic & ~3u) return fail(LBT1_EINVAL, "periodic mask %u", d->periodic);
  if (d->options & ~(uint32_t)(LBT1_OPT_SNAPSHOT | LBT1_OPT_PLANAR | LBT1_OPT_POPULATIONS | LBT1_OPT_MULTIPHASE))
    return fail(LBT1_EINVAL, "unknown options %u", d->options);
  const bool sc = d->options & LBT1_OPT_MULTIPHASE;
  const double rho0 = d->sc_rho0 == 0.0 ? 1.0 : d->sc_rho0;
  if (sc && (!std::isfinite(d->sc_G) || !(rho0 > 0.0) || !std::isfinite(rho0)))
    return fail(LBT1_EINVAL, "multiphase: sc_G must be finite and sc_rho0 > 0");
  if (!sc && (d->sc_G != 0.0 || d->sc_rho0 != 0.0))
    return fail(LBT1_EINVAL, "sc_G / sc_rho0 given without LBT1_OPT_MULTIPHASE");
  const bool pop = d->options & LBT1_OPT_POPULATIONS;
  const double tau = d->tau == 0.0 ? 1.0 : d->tau;
  if (pop && !(tau > 0.5 && std::isfinite(tau))) return fail(LBT1_EINVAL, "tau = %g: must be finite and > 1/2", d->tau);
  if (!pop && tau != 1.0) return fail(LBT1_EINVAL, "tau = %g: LBMTau1 grids have tau = 1 (0 or 1)", d->tau);
  if (!std::isfinite(d->force[0]) || !std::isfinite(d->force[1])) return fail(LBT1_EINVAL, "force must be finite");
  if (!pow2_or_zero(d->scale[0]) || !pow2_or_zero(d->scale[1]))
    return fail(LBT1_EINVAL, "scales must be 0 or positive powers of two");
  int dev = 0, cus = 0;
  lbt1_status st = check_device(&dev, &cus);
  if (st) return st;
  lbt1_grid *g = new (std::nothrow) lbt1_grid();
  if (!g) return fail(LBT1_ENOMEM, "host allocation");
  g->device = dev;
  g->cus = cus;
  g->nx = d->nx;
  g->ny = d->ny;
  g->periodic = d->periodic;
  g->prec = d->prec;
  g->wall = d->wall;
  g->options = d->options;
  g->pop = pop;
  g->tau = tau;
  g->mp = sc;
  g->sc_G = sc ? d->sc_G : 0.0;
  g->sc_rho0 = rho0;
  g->F[0] = d->force[0];
  g->F[1] = d->force[1];
  const bool scaled = d->prec == LBT1_F16S || d->prec == LBT1_BF16S;
  g->sc[0] = (scaled && d->scale[0] != 0.0) ? d->scale[0] : 1.0;
  g->sc[1] = (scaled && d->scale[1] != 0.0) ? d->scale[1] : 1.0;
  g->L = layout_of(d->nx, d->ny, d->prec, d->options);
  hipError_t e;
  if (d->device_buffer) {
    if (d->device_bytes < g->L.total) {
      delete g;
      return fail(LBT1_ENOMEM, "device buffer has %zu bytes, grid needs %zu", d->device_bytes, g->L.total);
    }
    if (((uintptr_t)d->device_buffer) % 256) {
      delete g;
      return fail(LBT1_EINVAL, "device buffer must be 256-byte aligned");
    }
    g->base = (char *)d->device_buffer;
    g->own_mem = false;
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
    g->own_stream = false;
  } else {
    if ((e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) != hipSuccess) {
      if (g->own_mem) hipFree(g->base);
      delete g;
      return hip_fail(e, "hipStreamCreate");
    }
    g->own_stream = true;
  }
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < g->L.nfield; ++q) g->plane[p][q] = g->base + (size_t)p * g->L.state + g->L.field_off[q];
  g->flags = (uint8_t *)(g->base + g->L.flags_off);
  for (int q = 0; q < 3; ++q)
    g->snap[q] = (d->options & LBT1_OPT_SNAPSHOT) ? g->base + g->L.snap_off + g->L.snap_field_off[q] : nullptr;
  g->psi = g->L.psi_off ? g->base + g->L.psi_off : nullptr;
  g->partials = (double *)(g->base + g->L.part_off);
  g->red_out = (double *)(g->base + g->L.out_off);
  if ((e = hipHostMalloc((void **)&g->red_host, 8 * sizeof(double), hipHostMallocDefault)) != hipSuccess) {
    if (g->own_stream) hipStreamDestroy(g->stream);
    if (g->own_mem) hipFree(g->base);
    delete g;
    return hip_fail(e, "hipHostMalloc");
  }
  g->cfg.kernel = LBT1_KERNEL_AUTO;
  *out = g;
  return LBT1_OK;
}

lbt1_status lbt1_set_geometry(lbt1_grid *g, const uint8_t *flags, const double *rho, const double *jx,
                              const double *jy) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  if (g->batch) return fail(LBT1_ESTATE, "grid is resident in a batch");
  const int nx = g->nx, ny = g->ny, pitch = g->L.pitch;
  const size_t n = (size_t)nx * ny;
  bool any_fixed = false, any_nonfluid = false;
  int64_t fluid = 0;
  if (flags) {
    for (size_t i = 0; i < n; ++i) {
      const uint8_t f = flags[i];
      if (f > LBT1_FIXED) return fail(LBT1_EINVAL, "flag %u at node %zu is not FLUID/SOLID/FIXED", f, i);
      any_fixed |= f == LBT1_FIXED;
      any_nonfluid |= f != LBT1_FLUID;
      fluid += f == LBT1_FLUID;
    }
  } else {
    fluid = (int64_t)n;
  }
  if (any_fixed && !rho && !jx && !jy) return fail(LBT1_EINVAL, "FIXED nodes need moments");
  if (any_fixed && g->mp) return fail(LBT1_EINVAL, "multiphase grids have no FIXED nodes");
  for (size_t i = 0; rho && i < n; ++i)
    if (!(rho[i] > 0.0) || !std::isfinite(rho[i])) return fail(LBT1_EINVAL, "rho[%zu] = %g must be finite and > 0", i, rho[i]);
  for (size_t i = 0; jx && i < n; ++i)
    if (!std::isfinite(jx[i])) return fail(LBT1_EINVAL, "jx[%zu] is not finite", i);
  for (size_t i = 0; jy && i < n; ++i)
    if (!std::isfinite(jy[i])) return fail(LBT1_EINVAL, "jy[%zu] is not finite", i);

  if (g->pop) {
    lbt1_status st = set_geometry_pop(g, flags, rho, jx, jy);
    if (st) return st;
    g->haswall = any_nonfluid || g->periodic != 3u;
    g->fluid = fluid;
    g->parity = 0;
    g->steps = 0;
    g->geometry = true;
    drop_bursts(g);
    return bind_config(g, lbt1_kernel_config{}, g->cus);
  }
  // Host staging in storage format with padded rows.
  const size_t c = value_bytes(g->prec);
  const size_t plane_vals = (size_t)pitch * ny;
  std::vector<char> stage;
  std::vector<uint8_t> fstage;
  try {
    stage.assign(g->L.state, 0);
    fstage.assign(plane_vals, LBT1_SOLID);
  } catch (...) {
    return fail(LBT1_ENOMEM, "host staging");
  }
  std::vector<double> row(nx);
  for (int y = 0; y < ny; ++y) {
    for (int q = 0; q < 3; ++q) {
      const double *src = q == 0 ? rho : q == 1 ? jx : jy;
      for (int x = 0; x < nx; ++x) {
        const size_t i = (size_t)y * nx + x;
        row[x] = src ? (q == 0 ? src[i] - 1.0 : src[i]) : 0.0;
      }
      encode_values(g->prec, row.data(), nx, 1.0 / g->sc[q == 0 ? 0 : 1],
                    stage.data() + g->L.field_off[q] + (size_t)y * g->L.rs * c);
    }
    for (int x = 0; x < nx; ++x) fstage[(size_t)y * pitch + x] = flags ? flags[(size_t)y * nx + x] : LBT1_FLUID;
  }
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int p = 0; p < 2; ++p)
    if ((e = hipMemcpy(g->base + (size_t)p * g->L.state, stage.data(), g->L.state, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy H2D");
  if (g->snap[0] && (e = hipMemcpy(g->base + g->L.snap_off, stage.data(), g->L.state, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy H2D");
  if ((e = hipMemcpy(g->flags, fstage.data(), plane_vals, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy H2D");
  g->haswall = any_nonfluid || g->periodic != 3u;
  g->fluid = fluid;
  g->parity = 0;
  g->steps = 0;
  g->geometry = true;
  drop_bursts(g);
  lbt1_kernel_config want{};
  if (g->user_cfg) want = g->cfg;
  lbt1_status st = bind_config(g, want, g->cus);
  if (st) return st;
  return LBT1_OK;
}

lbt1_status lbt1_step(lbt1_grid *g, int64_t n) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  if (n < 0) return fail(LBT1_EINVAL, "negative step count");
  if (!g->geometry) return fail(LBT1_ESTATE, "lbt1_step before lbt1_set_geometry");
  if (g->batch) return fail(LBT1_ESTATE, "grid is resident in a batch");
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  return enqueue_steps(g, n, g->stream, true);
}

lbt1_status lbt1_sync(lbt1_grid *g) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  hipError_t e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return LBT1_OK;
}

lbt1_status lbt1_read_window(lbt1_grid *g, int32_t x0, int32_t y0, int32_t w, int32_t h, double *rho, double *jx,
                             double *jy) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  if (w <= 0 || h <= 0 || x0 < 0 || y0 < 0 || (int64_t)x0 + w > g->nx || (int64_t)y0 + h > g->ny)
    return fail(LBT1_EINVAL, "window (%d, %d) + %d x %d is not inside the %d x %d grid", x0, y0, w, h, g->nx, g->ny);
  const size_t n = (size_t)w * h;
  if (g->pop) {
    std::vector<double> f;
    lbt1_status st = read_pop_window(g, x0, y0, w, h, f);
    if (st) return st;
    for (size_t i = 0; i < n; ++i) {
      double v[9];
      for (int q = 0; q < 9; ++q) v[q] = f[(size_t)q * n + i] - kHostW[q];
      const double d = (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) + v[8];
      if (rho) rho[i] = 1.0 + d;
      if (jx) jx[i] = ((v[1] - v[3]) + (v[5] - v[6])) + (v[8] - v[7]);
      if (jy) jy[i] = ((v[2] - v[4]) + (v[5] - v[7])) + (v[6] - v[8]);
    }
    for (size_t k = 0; k < g->given_idx.size(); ++k) {
      const int gy = (int)(g->given_idx[k] / g->nx), gx = (int)(g->given_idx[k] % g->nx);
      if (gx < x0 || gx >= x0 + w || gy < y0 || gy >= y0 + h) continue;
      const size_t i = (size_t)(gy - y0) * w + (gx - x0);
      if (rho) rho[i] = g->given_val[3 * k];
      if (jx) jx[i] = g->given_val[3 * k + 1];
      if (jy) jy[i] = g->given_val[3 * k + 2];
    }
    return LBT1_OK;
  }
  const size_t c = value_bytes(g->prec);
  std::vector<char> stage;
  try {
    stage.resize(n * c);
  } catch (...) {
    return fail(LBT1_ENOMEM, "host staging");
  }
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int q = 0; q < 3; ++q) {
    double *dst = q == 0 ? rho : q == 1 ? jx : jy;
    if (!dst) continue;
    const char *src = (const char *)g->plane[g->parity][q] + ((size_t)y0 * g->L.rs + x0) * c;
    if ((e = hipMemcpy2D(stage.data(), (size_t)w * c, src, (size_t)g->L.rs * c, (size_t)w * c, h,
                         hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hipMemcpy2D D2H");
    decode_values(g->prec, stage.data(), n, g->sc[q == 0 ? 0 : 1], dst);
    if (q == 0)
      for (size_t i = 0; i < n; ++i) dst[i] += 1.0;
  }
  return LBT1_OK;
}

lbt1_status lbt1_read_moments(lbt1_grid *g, double *rho, double *jx, double *jy) {
  if (!g) {
    clear_error();
    return fail(LBT1_EINVAL, "null grid");
  }
  return lbt1_read_window(g, 0, 0, g->nx, g->ny, rho, jx, jy);
}

lbt1_status lbt1_read_populations(lbt1_grid *g, double *f) {
  clear_error();
  if (!g || !f) return fail(LBT1_EINVAL, "null argument");
  if (!g->pop) return fail(LBT1_EINVAL, "not a population grid (LBT1_OPT_POPULATIONS)");
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  std::vector<double> v;
  lbt1_status st = read_pop_window(g, 0, 0, g->nx, g->ny, v);
  if (st) return st;
  std::memcpy(f, v.data(), v.size() * sizeof(double));
  return LBT1_OK;
}

lbt1_status lbt1_reduce(lbt1_grid *g, uint32_t what, double *out) {
  clear_error();
  if (!g || !out) return fail(LBT1_EINVAL, "null argument");
  if (what & ~15u) return fail(LBT1_EINVAL, "unknown reduce bits %u", what);
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  if ((what & LBT1_REDUCE_RESIDUAL) && !g->snap[0]) return fail(LBT1_EINVAL, "grid was created without LBT1_OPT_SNAPSHOT");
  if (g->batch) return fail(LBT1_ESTATE, "grid is resident in a batch");
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  lbt1_status st = enqueue_reduce(g, what, g->stream);
  if (st) return st;
  if ((e = hipMemcpyAsync(g->red_host, g->red_out, 6 * sizeof(double), hipMemcpyDeviceToHost, g->stream)) != hipSuccess)
    return hip_fail(e, "hipMemcpyAsync D2H");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  const double *r = g->red_host;
  if (what & LBT1_REDUCE_MASS) out[0] = r[5] + r[0];
  if (what & LBT1_REDUCE_MOMENTUM) {
    out[1] = r[1];
    out[2] = r[2];
  }
  if (what & LBT1_REDUCE_RESIDUAL) out[3] = r[3];
  if (what & LBT1_REDUCE_NONFINITE) out[4] = r[4];
  out[5] = r[5];
  return LBT1_OK;
}

lbt1_status lbt1_reduce_noalloc(lbt1_grid *g, uint32_t what, double *out) {
  clear_error();
  if (!g || !out) return fail(LBT1_EINVAL, "null argument");
  if (what & ~15u) return fail(LBT1_EINVAL, "unknown reduce bits %u", what);
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  if ((what & LBT1_REDUCE_RESIDUAL) && !g->snap[0]) return fail(LBT1_EINVAL, "grid was created without LBT1_OPT_SNAPSHOT");
  if (g->batch) return fail(LBT1_ESTATE, "grid is resident in a batch");
  const int rows = reduce_blocks(g);
  if (rows > kScratchRows)
    return fail(LBT1_EINVAL, "reduction needs %d partial rows, the static scratch holds %d", rows, kScratchRows);
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  double *parts = nullptr;
  lbt1_status st = scratch_on(g->device, &parts);
  if (st) return st;
  return enqueue_reduce_into(g, what, g->stream, parts, out, true);
}

// Bytes of an exact checkpoint: the parity block in storage format, and the
// residual snapshot when the grid keeps one.
static size_t snapshot_bytes(const lbt1_grid *g) {
  if (!g->snap[0]) return 0;
  return g->pop ? 3 * (g->L.snap_field_off[1] - g->L.snap_field_off[0]) : g->L.state;
}

size_t lbt1_state_bytes(lbt1_grid *g) {
  if (!g) return 0;
  return g->L.state + snapshot_bytes(g);
}

lbt1_status lbt1_save_state(lbt1_grid *g, void *host, size_t bytes) {
  clear_error();
  if (!g || !host) return fail(LBT1_EINVAL, "null argument");
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  if (g->batch) return fail(LBT1_ESTATE, "grid is resident in a batch");
  if (bytes < lbt1_state_bytes(g)) return fail(LBT1_EINVAL, "buffer has %zu bytes, the state %zu", bytes, lbt1_state_bytes(g));
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  char *h = (char *)host;
  if ((e = hipMemcpy(h, g->base + (size_t)g->parity * g->L.state, g->L.state, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy D2H");
  if (snapshot_bytes(g) &&
      (e = hipMemcpy(h + g->L.state, g->base + g->L.snap_off, snapshot_bytes(g), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy D2H");
  return LBT1_OK;
}

lbt1_status lbt1_load_state(lbt1_grid *g, const void *host, size_t bytes) {
  clear_error();
  if (!g || !host) return fail(LBT1_EINVAL, "null argument");
  if (!g->geometry) return fail(LBT1_ESTATE, "set the geometry (flags) before loading a state");
  if (g->batch) return fail(LBT1_ESTATE, "grid is resident in a batch");
  if (bytes != lbt1_state_bytes(g)) return fail(LBT1_EINVAL, "state has %zu bytes, this grid takes %zu", bytes, lbt1_state_bytes(g));
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  const char *h = (const char *)host;
  // both parities: non-FLUID nodes are read from either
  for (int p = 0; p < 2; ++p)
    if ((e = hipMemcpy(g->base + (size_t)p * g->L.state, h, g->L.state, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy H2D");
  if (snapshot_bytes(g) &&
      (e = hipMemcpy(g->base + g->L.snap_off, h + g->L.state, snapshot_bytes(g), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy H2D");
  g->parity = 0;
  return LBT1_OK;
}

lbt1_status lbt1_destroy_grid(lbt1_grid *g) {
  clear_error();
  if (!g) return LBT1_OK;
  if (g->batch) return fail(LBT1_ESTATE, "grid is resident in a batch; evict it first");
  hipSetDevice(g->device);
  hipStreamSynchronize(g->stream);
  drop_bursts(g);
  if (g->red_host) hipHostFree(g->red_host);
  if (g->own_stream) hipStreamDestroy(g->stream);
  if (g->own_mem) hipFree(g->base);
  delete g;
  return LBT1_OK;
}

lbt1_status lbt1_set_kernel(lbt1_grid *g, const lbt1_kernel_config *cfg) {
  clear_error();
  if (!g || !cfg) return fail(LBT1_EINVAL, "null argument");
  if (g->pop) return fail(LBT1_EINVAL, "population grids have a single step kernel");
  if (!g->geometry) {
    g->cfg = *cfg;
    g->user_cfg = cfg->kernel != LBT1_KERNEL_AUTO;
    return LBT1_OK;
  }
  lbt1_kernel_config old = g->cfg;
  const StepKernel *oldk = g->kern;
  lbt1_status st = bind_config(g, *cfg, g->cus);
  if (st) {
    g->cfg = old;
    g->kern = oldk;
    bind_config(g, old, g->cus);
    return st;
  }
  g->user_cfg = cfg->kernel != LBT1_KERNEL_AUTO;
  drop_bursts(g);
  return LBT1_OK;
}

lbt1_status lbt1_get_kernel(lbt1_grid *g, lbt1_kernel_config *cfg, char *name, size_t cap) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  if (!g->kern) return fail(LBT1_ESTATE, "no kernel bound (set the geometry first)");
  if (cfg) *cfg = g->cfg;
  if (name && cap) {
    std::strncpy(name, g->kern->name, cap - 1);
    name[cap - 1] = 0;
  }
  return LBT1_OK;
}

lbt1_status lbt1_autotune(lbt1_grid *g, int32_t steps, int32_t reps, lbt1_kernel_config *best,
                          double *ms_per_step) {
  clear_error();
  if (!g) return fail(LBT1_EINVAL, "null grid");
  if (!g->geometry) return fail(LBT1_ESTATE, "no geometry set");
  if (g->batch) return fail(LBT1_ESTATE, "grid is resident in a batch");
  if (steps < 2 || reps < 1) return fail(LBT1_EINVAL, "steps >= 2 and reps >= 1 required");
  if (g->pop) return fail(LBT1_EINVAL, "population grids have a single step kernel");
  hipError_t e;
  if ((e = hipSetDevice(g->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  // The candidates run on the grid's own memory (a copy elsewhere can time
  // differently: measured up to 2.5 % between two allocations of one 8192^2
  // field); both parities are saved to scratch first and restored afterwards.
  lbt1_grid t = *g;
  t.burst[0] = t.burst[1] = nullptr;
  t.graph_valid = false;
  void *p = nullptr;
  if ((e = hipMalloc(&p, 2 * g->L.state)) != hipSuccess)
    return fail(LBT1_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
  if ((e = hipMemcpyAsync(p, g->base, 2 * g->L.state, hipMemcpyDeviceToDevice, g->stream)) != hipSuccess) {
    hipFree(p);
    return hip_fail(e, "autotune save");
  }
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  std::vector<lbt1_kernel_config> cands;
  {
    lbt1_kernel_config c{};
    c.kernel = LBT1_KERNEL_GATHER;
    cands.push_back(c);
  }
  const int vecs[] = {1, 2, 4, 8};
  const int rows[] = {2, 6, 14, 22, 28, 30};
  const int waves[] = {0, 8, 16};
  const int fuses[] = {1, 2, 3};
  for (int v : vecs)
    for (int r : rows)
      for (int w : waves)
        for (int f : fuses) {
          if (!strip_fits(g->nx, v, g->periodic & 1u)) continue;
          if (f > 2 && (g->mp || g->haswall)) continue;
          if (g->mp && g->haswall) continue;
          if (!find_kernel(g->prec, g->haswall, g->wall, KIND_STRIP, v, r, f, g->mp)) continue;
          if (64 * v > 2 * std::max(64, g->nx)) continue;
          lbt1_kernel_config c{};
          c.kernel = LBT1_KERNEL_STRIP;
          c.vec = v;
          c.rows = r;
          c.waves = w;
          c.fuse = f;
          cands.push_back(c);
        }
  // a whole number of fused launches for every candidate
  steps = (steps + 5) / 6 * 6;
  lbt1_status st = LBT1_OK;
  auto time_steps = [&](const int n, const bool use_graph) -> double {
    hipEventRecord(e0, g->stream);
    st = enqueue_steps(&t, n, g->stream, use_graph);
    hipEventRecord(e1, g->stream);
    hipEventSynchronize(e1);
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    return (double)ms / n;
  };
  // screening: every candidate, best of `reps` after one warm-up run
  std::vector<std::pair<double, lbt1_kernel_config>> timed;
  for (const auto &c : cands) {
    if (bind_config(&t, c, g->cus) != LBT1_OK) continue;
    double cbest = 1e300;
    for (int r = 0; r < reps + 1 && st == LBT1_OK; ++r) {
      const double ms = time_steps(steps, false);
      if (r > 0) cbest = std::min(cbest, ms);
    }
    if (st) break;
    timed.push_back({cbest, t.cfg});
  }
  // final: the candidates within 5 % of the fastest, re-timed as lbt1_step runs
  // them (graph bursts) on three bursts' worth of steps, in interleaved rounds so
  // that a drift of the clock between candidates does not decide; each round
  // first runs a candidate once untimed (it builds the bursts)
  double best_ms = 1e300;
  lbt1_kernel_config bc = g->cfg;
  if (!st && !timed.empty()) {
    std::stable_sort(timed.begin(), timed.end(),
                     [](const std::pair<double, lbt1_kernel_config> &a, const std::pair<double, lbt1_kernel_config> &b) {
                       return a.first < b.first;
                     });
    size_t nf = 1;
    while (nf < timed.size() && nf < 8 && timed[nf].first <= 1.05 * timed[0].first) ++nf;
    best_ms = timed[0].first;
    bc = timed[0].second;
    if (nf > 1) {
      std::vector<double> fbest(nf, 1e300);
      for (int r = 0; r < std::max(reps, 3) && !st; ++r)
        for (size_t i = 0; i < nf && !st; ++i) {
          if (bind_config(&t, timed[i].second, g->cus) != LBT1_OK) continue;
          (void)time_steps(3 * kBurst, true);
          if (st) break;
          const double ms = time_steps(3 * kBurst, true);
          fbest[i] = std::min(fbest[i], ms);
        }
      if (!st) {
        size_t bi = 0;
        for (size_t i = 1; i < nf; ++i)
          if (fbest[i] < fbest[bi]) bi = i;
        best_ms = fbest[bi];
        bc = timed[bi].second;
      }
    }
  }
  hipStreamSynchronize(g->stream);
  drop_bursts(&t);  // (the clone's bursts, idle now)
  const hipError_t er = hipMemcpyAsync(g->base, p, 2 * g->L.state, hipMemcpyDeviceToDevice, g->stream);
  hipStreamSynchronize(g->stream);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(p);
  if (st) return st;
  if (er != hipSuccess) return hip_fail(er, "autotune restore");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[tune_key(g)] = bc;
  }
  st = bind_config(g, bc, g->cus);
  if (st) return st;
  g->user_cfg = true;
  drop_bursts(g);
  if (best) *best = bc;
  if (ms_per_step) *ms_per_step = best_ms;
  return LBT1_OK;
}

}  // extern "C"

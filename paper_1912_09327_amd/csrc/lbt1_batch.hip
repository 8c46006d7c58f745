// Batched stepping of many resident grids (lbt1_batch_* of include/lbt1.h).
//
// Every resident grid is cut into strips (62 chunks of vec columns by a class's
// strip height) and belongs to one work class: one step per launch at 1, 2 or 4
// columns per lane, or two steps per launch at 2 columns per lane (the fused
// class, k_step_batch_fused).  The strips of all grids of a class form one work
// list, and one launch per class and launch step covers the whole list, so a step
// of hundreds of small, uneven grids costs a handful of launches.  Which class a
// grid joins and each class's strip height are the batch's tile shape: a
// heuristic by default (6-row strips for classes too short to give every CU
// several wavefronts, since a strip walks its rows one after another), or what
// lbt1_batch_autotune measured fastest on the resident grids.  Each strip's kind
// (interior, walls down whole columns, general), which picks the body it runs,
// is found once per work list on the device (k_batch_classify) and kept in its
// work item.  A burst of K steps
// plus the per-grid residual check is one HIP graph with one chain of launches
// per class (the classes touch disjoint grids, so their chains run side by side);
// the grid descriptors and work lists live in device memory, so admitting or
// finishing grids changes data, not the graph (it is rebuilt only when the burst
// length, the set of non-empty classes or a class's shape changes, or a list
// outgrows its allocation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbt1.h"
#include "lbt1_batch_args.hpp"
#include "lbt1_internal.hpp"
#include "lbt1_runtime.hpp"

namespace lbt1 {

// Work classes: one step per launch at 1, 2, 4 columns per lane, two steps per
// launch at 2 columns per lane, and small grids resident in LDS for a whole burst
// (one launch per burst, two columns per lane).
enum { CLS_V1 = 0, CLS_V2 = 1, CLS_V4 = 2, CLS_F2 = 3, CLS_LDS = 4, kClasses = 5 };
static const int kVecOfClass[kClasses] = {1, 2, 4, 2, 2};
static const int kStepsOfClass[kClasses] = {1, 1, 1, 2, 0};  // 0: every step of the burst in one launch

// launches a class takes for a burst of K steps, and the parity flips of a grid of
// the class that takes k steps in it
static int class_launches(int c, int K) { return kStepsOfClass[c] ? (K + kStepsOfClass[c] - 1) / kStepsOfClass[c] : 1; }
static int class_flips(int c, int k) {
  return k <= 0 ? 0 : kStepsOfClass[c] ? (k + kStepsOfClass[c] - 1) / kStepsOfClass[c] : 1;
}

// How grids are assigned to classes.  MIXED: the fused class except for grids of
// the four-column class narrower than kMixedWide columns (measured on the uneven
// cavities: one step per launch at four columns per lane is faster for sides 256
// to 512, two steps per launch for narrower grids, as on single grids of 1024
// and more, where two fused steps win).
enum { FUSE_NONE = 0, FUSE_ALL = 1, FUSE_MIXED = 2 };
constexpr int kMixedWide = 1024;

struct Slot {
  lbt1_grid *g = nullptr;
  int64_t budget = 0, taken = 0;
  double tol = -1.0, residual = -1.0;
  int state = LBT1_SLOT_FREE;
  size_t bytes = 0;
  int vclass = 0;  // widest one-step class that fits the grid
  int cls = 0;     // class it runs in (the tile-shape policy's choice)
  int steps_this_burst = 0;
};

}  // namespace lbt1

struct lbt1_batch {
  int device = 0, cus = 0;
  size_t budget = 0, used = 0;
  int max_slots = 0;
  int prec = -1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<lbt1::Slot> slots;
  // device side
  lbt1::BatchGrid *d_grids = nullptr;
  void **d_snaps = nullptr;
  int *d_active = nullptr;
  int *d_counts = nullptr;  // [0..kClasses-1] item counts per class, [6] active slots, [7] reduction items
  double *d_red = nullptr;
  int2 *d_items[lbt1::kClasses] = {};
  size_t item_cap[lbt1::kClasses] = {};
  int2 *d_ritems = nullptr;  // reduction items (slot, chunk)
  double *d_partials = nullptr;
  size_t ritem_cap = 0;
  int2 *d_ranges = nullptr;  // per slot: first reduction item, count
  // pinned host mirrors
  lbt1::BatchGrid *h_grids = nullptr;
  void **h_snaps = nullptr;
  int *h_active = nullptr;
  int *h_counts = nullptr;
  double *h_red = nullptr;
  int2 *h_ranges = nullptr;
  std::vector<int2> items[lbt1::kClasses];
  std::vector<int2> ritems;
  int rows[lbt1::kClasses] = {14, 14, 14, 14, 6};  // strip height per class
  int blocks[lbt1::kClasses] = {};                  // launch size per class
  size_t lds_bytes = 0;                             // dynamic LDS of the LDS-class launch
  size_t lds_limit = 0;                             // most LDS one workgroup may take
  // tile-shape policy: class assignment and fixed strip heights (0 = heuristic)
  int fuse_mode = lbt1::FUSE_MIXED;
  bool lds_mode = false;
  int vec_cap_class = lbt1::CLS_V4;  // widest one-step class a grid may take
  int want_rows[lbt1::kClasses] = {};
  bool items_dirty = true;
  hipGraphExec_t graph = nullptr;
  int graph_K = 0, graph_mask = -1;
  long graph_shape = -1;
  bool graph_valid = false;
};

namespace lbt1 {

static const int kCntActive = 6, kCntRitems = 7;  // slots of d_counts after the class counts

// Widest one-step class whose chunk fits the grid: v divides nx, or x is not
// periodic (the last chunk of a row then runs into the row padding, whose flags
// are SOLID; pitch is nx rounded up to 64, a multiple of v).
static int vec_class_for(int prec, int nx, bool periodic_x) {
  const int maxc = prec == LBT1_F64 ? CLS_V2 : CLS_V4;  // FP64 batched kernels go up to 2 columns per lane
  for (int c = maxc; c >= CLS_V1; --c) {
    const int v = kVecOfClass[c];
    if ((nx % v == 0 || !periodic_x) && 64 * v <= std::max(64, nx)) return c;
  }
  return CLS_V1;
}
static int chunks_of(int nx, int v) { return (nx + v - 1) / v; }

// The class a grid runs in under the batch's policy: the fused class takes grids
// whose rows two columns per lane fit (all of them, or those narrower than the
// four-column class), the others their widest one-step class.
static int class_for(const lbt1_batch *b, const Slot &sl) {
  const bool fits2 = sl.g->nx % 2 == 0 || !(sl.g->periodic & 1u);
  if (b->lds_mode && fits2 && batch_lds_kernel(sl.g->prec, 6) &&
      (size_t)lds_grid_bytes(sl.g->nx, sl.g->ny, 2, (int)value_bytes(sl.g->prec)) <= b->lds_limit)
    return CLS_LDS;
  if (b->fuse_mode == FUSE_ALL && fits2) return CLS_F2;
  if (b->fuse_mode == FUSE_MIXED && fits2 && (sl.vclass < CLS_V4 || sl.g->nx >= kMixedWide)) return CLS_F2;
  // the widest one-step class allowed (narrower chunks: fewer registers, more
  // wavefronts per SIMD to hide memory latency, fewer idle lanes on some widths)
  return std::min(sl.vclass, b->vec_cap_class);
}

static const void *class_kernel(const lbt1_batch *b, int c) {
  if (c == CLS_LDS) return batch_lds_kernel(b->prec, b->rows[c]);
  return c == CLS_F2 ? batch_fused_kernel(b->prec, b->rows[c]) : batch_step_kernel(b->prec, c, b->rows[c]);
}

// Launch size of a class: as many 256-thread blocks as the kernel's register
// use lets every CU hold at once, but no more than the class has work items
// for (each block takes four strips per pass).
static int class_blocks(const lbt1_batch *b, int c) {
  const void *fn = class_kernel(b, c);
  int per_cu = 2;
  const size_t shmem = c == CLS_LDS ? b->lds_bytes : 0;
  if (fn) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, shmem);
  per_cu = std::max(1, per_cu);
  // LDS class: one block per grid; the others: four strips per block and pass
  const long need = c == CLS_LDS ? (long)b->items[c].size() : ((long)b->items[c].size() + 3) / 4;
  return (int)std::max<long>(1, std::min<long>((long)per_cu * b->cus, need));
}

static long graph_shape(const lbt1_batch *b) {
  long key = 0;
  for (int c = 0; c < kClasses; ++c) key = key * 1000003L + b->rows[c] * 100003L + b->blocks[c];
  return key * 1000003L + (long)b->lds_bytes;
}

static void rebuild_items(lbt1_batch *b) {
  long tall[kClasses] = {};
  long tall30 = 0;  // fused-class strips at 30 rows
  for (int s = 0; s < b->max_slots; ++s) {
    Slot &sl = b->slots[s];
    if (sl.state == LBT1_SLOT_FREE) continue;
    sl.cls = class_for(b, sl);
    const int v = kVecOfClass[sl.cls];
    const long sx = (chunks_of(sl.g->nx, v) + 61) / 62;
    tall[sl.cls] += sx * ((sl.g->ny + 13) / 14);
    if (sl.cls == CLS_F2) tall30 += sx * ((sl.g->ny + 29) / 30);
  }
  for (int c = 0; c < kClasses; ++c) {
    b->items[c].clear();
    // heuristic height: 14-row strips where a class has eight or more per CU,
    // else 6 (a strip walks its rows one after another); the fused class 30 rows
    // where it has four or more such strips per CU (the uneven cavities' tuned
    // choice: fewer halo rows per stored row)
    b->rows[c] = b->want_rows[c] ? b->want_rows[c] : c == CLS_LDS || tall[c] < 8L * b->cus ? 6 : 14;
    if (c == CLS_F2 && !b->want_rows[c] && tall30 >= 4L * b->cus) b->rows[c] = 30;
    // a height the batch's precision has no kernel for (30 rows in FP64) falls back
    if (b->prec >= 0 && !class_kernel(b, c)) b->rows[c] = 14;
  }
  // (block counts are set below, once the lists are built)
  b->ritems.clear();
  b->lds_bytes = 0;
  for (int s = 0; s < b->max_slots; ++s) {
    const Slot &sl = b->slots[s];
    b->h_ranges[s] = make_int2(0, 0);
    if (sl.state == LBT1_SLOT_FREE) continue;
    const int v = kVecOfClass[sl.cls];
    const int rows = b->rows[sl.cls];
    const int sx = (chunks_of(sl.g->nx, v) + 61) / 62;  // strips of 62 chunks of v columns
    const int sy = (sl.g->ny + rows - 1) / rows;
    b->h_grids[s].strips_x = sx;
    if (sl.cls == CLS_LDS) {
      // one item per grid: its workgroup walks all of its strips
      b->items[sl.cls].push_back(make_int2(s, 0));
      b->lds_bytes = std::max(b->lds_bytes, (size_t)lds_grid_bytes(sl.g->nx, sl.g->ny, 2, (int)value_bytes(sl.g->prec)));
    } else {
      // (slot, 4 * strip + kind); kind 0 (the general wall-aware body) until the
      // list is classified on the device
      for (int k = 0; k < sx * sy; ++k) b->items[sl.cls].push_back(make_int2(s, k << 2));
    }
    const long nodes = (long)sl.g->nx * sl.g->ny;
    const int chunks = (int)((nodes + kBatchReduceChunk - 1) / kBatchReduceChunk);
    b->h_ranges[s] = make_int2((int)b->ritems.size(), chunks);
    for (int k = 0; k < chunks; ++k) b->ritems.push_back(make_int2(s, k));
  }
  for (int c = 0; c < kClasses; ++c) b->blocks[c] = b->items[c].empty() ? 0 : class_blocks(b, c);
}


static lbt1_status upload_items(lbt1_batch *b) {
  hipError_t e;
  for (int c = 0; c < kClasses; ++c) {
    const size_t n = b->items[c].size();
    if (n > b->item_cap[c]) {
      size_t cap = std::max<size_t>(1024, b->item_cap[c]);
      while (cap < n) cap *= 2;
      if (b->d_items[c]) (void)hipFree(b->d_items[c]);
      b->d_items[c] = nullptr;
      b->item_cap[c] = 0;
      if ((e = hipMalloc(&b->d_items[c], cap * sizeof(int2))) != hipSuccess) return hip_fail(e, "hipMalloc items");
      b->item_cap[c] = cap;
      b->graph_valid = false;  // kernel arguments point at the old list
    }
    if (n && (e = hipMemcpyAsync(b->d_items[c], b->items[c].data(), n * sizeof(int2), hipMemcpyHostToDevice, b->stream)) !=
                 hipSuccess)
      return hip_fail(e, "items H2D");
    b->h_counts[c] = (int)n;
  }
  const size_t nr = b->ritems.size();
  if (nr > b->ritem_cap) {
    size_t cap = std::max<size_t>(1024, b->ritem_cap);
    while (cap < nr) cap *= 2;
    if (b->d_ritems) (void)hipFree(b->d_ritems);
    if (b->d_partials) (void)hipFree(b->d_partials);
    b->d_ritems = nullptr;
    b->d_partials = nullptr;
    b->ritem_cap = 0;
    if ((e = hipMalloc(&b->d_ritems, cap * sizeof(int2))) != hipSuccess ||
        (e = hipMalloc(&b->d_partials, cap * 6 * sizeof(double))) != hipSuccess)
      return hip_fail(e, "hipMalloc reduction items");
    b->ritem_cap = cap;
    b->graph_valid = false;
  }
  if (nr && (e = hipMemcpyAsync(b->d_ritems, b->ritems.data(), nr * sizeof(int2), hipMemcpyHostToDevice, b->stream)) !=
                hipSuccess)
    return hip_fail(e, "reduction items H2D");
  if ((e = hipMemcpyAsync(b->d_ranges, b->h_ranges, (size_t)b->max_slots * sizeof(int2), hipMemcpyHostToDevice,
                          b->stream)) != hipSuccess)
    return hip_fail(e, "ranges H2D");
  b->h_counts[kCntRitems] = (int)nr;
  b->items_dirty = false;
  return LBT1_OK;
}

static lbt1_status build_graph(lbt1_batch *b, int K, int mask) {
  hipError_t e;
  hipGraph_t graph = nullptr;
  if ((e = hipGraphCreate(&graph, 0)) != hipSuccess) return hip_fail(e, "hipGraphCreate");
  std::vector<BatchStepArgs> argv;
  argv.reserve((size_t)K * kClasses);
  auto add = [&](const void *fn, dim3 grid, dim3 block, void **args, const hipGraphNode_t *deps, int ndeps,
                 hipGraphNode_t *out, size_t shmem = 0) -> lbt1_status {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(fn);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = (unsigned int)shmem;
    kp.kernelParams = args;
    hipError_t err = hipGraphAddKernelNode(out, graph, ndeps ? deps : nullptr, ndeps, &kp);
    if (err != hipSuccess) return hip_fail(err, "hipGraphAddKernelNode");
    return LBT1_OK;
  };
  // one chain per class: launch s of a class waits for launch s - 1 of the same
  // class; a class of k steps per launch takes ceil(K / k) launches
  lbt1_status st = LBT1_OK;
  hipGraphNode_t last[kClasses];
  int nlast = 0;
  for (int c = 0; c < kClasses && !st; ++c) {
    if (!(mask & (1 << c))) continue;
    hipGraphNode_t prev = nullptr;
    const int launches = class_launches(c, K);
    for (int s = 0; s < launches && !st; ++s) {
      BatchStepArgs a;
      a.grids = b->d_grids;
      a.items = b->d_items[c];
      a.count = b->d_counts + c;
      a.step = s;
      argv.push_back(a);
      void *args[] = {&argv.back()};
      hipGraphNode_t node;
      st = add(class_kernel(b, c), dim3(b->blocks[c]), dim3(256), args, &prev, prev ? 1 : 0, &node,
               c == CLS_LDS ? b->lds_bytes : 0);
      prev = node;
    }
    last[nlast++] = prev;
  }
  BatchReduceArgs ra;
  ra.grids = b->d_grids;
  ra.snaps = b->d_snaps;
  ra.items = b->d_ritems;
  ra.nitems = b->d_counts + kCntRitems;
  ra.partials = b->d_partials;
  ra.active = b->d_active;
  ra.nactive = b->d_counts + kCntActive;
  ra.ranges = b->d_ranges;
  ra.out = b->d_red;
  hipGraphNode_t partial;
  if (!st) {
    void *args[] = {&ra};
    st = add(batch_reduce_kernel(b->prec), dim3(std::max(8, b->cus * 4)), dim3(256), args, last, nlast, &partial);
  }
  if (!st) {
    void *args[] = {&ra};
    hipGraphNode_t node;
    st = add(batch_reduce_final_kernel(), dim3(std::max(8, b->cus)), dim3(64), args, &partial, 1, &node);
  }
  if (st) {
    (void)hipGraphDestroy(graph);
    return st;
  }
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  e = hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  b->graph_K = K;
  b->graph_mask = mask;
  b->graph_shape = graph_shape(b);
  b->graph_valid = true;
  return LBT1_OK;
}

// Descriptors and work lists for a burst of K steps of every running grid,
// uploaded, and the burst graph launched on the batch's stream (no wait, no
// bookkeeping).  *nact receives the number of grids stepped.
static lbt1_status launch_burst(lbt1_batch *b, int K, int *nact_out) {
  hipError_t e;
  if ((e = hipSetDevice(b->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  int nact = 0;
  for (int s = 0; s < b->max_slots; ++s) {
    Slot &sl = b->slots[s];
    BatchGrid &d = b->h_grids[s];
    sl.steps_this_burst = 0;
    d.steps_left = 0;
    d.flips = 0;
    if (sl.state != LBT1_SLOT_RUNNING) continue;
    const int64_t left = sl.budget - sl.taken;
    sl.steps_this_burst = (int)std::min<int64_t>(K, left);
    d.steps_left = sl.steps_this_burst;
    d.parity0 = sl.g->parity;
    b->h_active[nact++] = s;
  }
  *nact_out = nact;
  if (nact == 0) return LBT1_OK;
  b->h_counts[kCntActive] = nact;
  const bool rebuilt = b->items_dirty;
  if (b->items_dirty) {
    rebuild_items(b);
    lbt1_status st = upload_items(b);
    if (st) return st;
  }
  for (int k = 0; k < nact; ++k) {
    const int s = b->h_active[k];
    b->h_grids[s].flips = class_flips(b->slots[s].cls, b->slots[s].steps_this_burst);
  }
  int mask = 0;
  for (int c = 0; c < kClasses; ++c)
    if (!b->items[c].empty()) mask |= 1 << c;
  const size_t ns = (size_t)b->max_slots;
  if ((e = hipMemcpyAsync(b->d_grids, b->h_grids, ns * sizeof(BatchGrid), hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(b->d_snaps, b->h_snaps, ns * 3 * sizeof(void *), hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(b->d_active, b->h_active, (size_t)nact * sizeof(int), hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(b->d_counts, b->h_counts, 8 * sizeof(int), hipMemcpyHostToDevice, b->stream)) != hipSuccess)
    return hip_fail(e, "descriptor H2D");
  if (rebuilt) {
    // the kind of every strip of the new lists (stream-ordered before the burst)
    for (int c = 0; c < kClasses; ++c) {
      if (c == CLS_LDS || b->items[c].empty()) continue;
      BatchClassifyArgs ca;
      ca.grids = b->d_grids;
      ca.items = b->d_items[c];
      ca.count = b->d_counts + c;
      ca.rows = b->rows[c];
      ca.halo = kStepsOfClass[c];
      void *args[] = {&ca};
      const int blocks = (int)std::min<long>(((long)b->items[c].size() + 3) / 4, 8L * b->cus);
      if ((e = hipLaunchKernel(batch_classify_kernel(kVecOfClass[c]), dim3(std::max(1, blocks)), dim3(256), args, 0,
                               b->stream)) != hipSuccess)
        return hip_fail(e, "strip classification");
    }
  }
  if (!b->graph_valid || b->graph_K != K || b->graph_mask != mask || b->graph_shape != graph_shape(b)) {
    lbt1_status st = build_graph(b, K, mask);
    if (st) return st;
  }
  if ((e = hipGraphLaunch(b->graph, b->stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return LBT1_OK;
}

// Take a tile-shape policy: the class assignment and the strip heights (0 keeps
// the heuristic); the work lists are rebuilt before the next burst.
static lbt1_status set_shape(lbt1_batch *b, const lbt1_batch_shape &sh) {
  if (sh.fuse < FUSE_NONE || sh.fuse > FUSE_MIXED) return fail(LBT1_EINVAL, "fuse mode %d", sh.fuse);
  if (sh.lds != 0 && sh.lds != 1) return fail(LBT1_EINVAL, "lds mode %d", sh.lds);
  if (sh.vec_cap != 0 && sh.vec_cap != 1 && sh.vec_cap != 2 && sh.vec_cap != 4)
    return fail(LBT1_EINVAL, "vec_cap %d (0, 1, 2 or 4)", sh.vec_cap);
  for (int c = 0; c < kClasses; ++c) {
    const int r = sh.rows[c];
    if (r == 0) continue;
    const int pr = b->prec >= 0 ? b->prec : LBT1_F32;
    const bool ok = c == CLS_F2    ? batch_fused_kernel(pr, r) != nullptr
                    : c == CLS_LDS ? (r == 6 || r == 14)
                                   : batch_step_kernel(pr, c, r) != nullptr;
    if (!ok) return fail(LBT1_EINVAL, "class %d: no built kernel with %d-row strips", c, r);
  }
  b->fuse_mode = sh.fuse;
  b->lds_mode = sh.lds != 0;
  b->vec_cap_class = sh.vec_cap == 1 ? CLS_V1 : sh.vec_cap == 2 ? CLS_V2 : CLS_V4;
  for (int c = 0; c < kClasses; ++c) b->want_rows[c] = sh.rows[c];
  b->items_dirty = true;
  return LBT1_OK;
}

}  // namespace lbt1

using namespace lbt1;

extern "C" {

lbt1_status lbt1_batch_create(size_t hbm_budget_bytes, int32_t max_slots, void *stream, lbt1_batch **out) {
  clear_error();
  if (!out) return fail(LBT1_EINVAL, "null argument");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 65536) return fail(LBT1_EINVAL, "max_slots %d out of 1..65536", max_slots);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(LBT1_EDEVICE, "no HIP device is visible");
  lbt1_batch *b = new (std::nothrow) lbt1_batch();
  if (!b) return fail(LBT1_ENOMEM, "host allocation");
  hipError_t e;
  hipDeviceProp_t prop;
  if ((e = hipGetDevice(&b->device)) != hipSuccess || (e = hipGetDeviceProperties(&prop, b->device)) != hipSuccess) {
    delete b;
    return hip_fail(e, "device query");
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete b;
    return fail(LBT1_EDEVICE, "device is %s; this library is built for gfx950", prop.gcnArchName);
  }
  b->cus = prop.multiProcessorCount;
  // the LDS class keeps a grid within what one workgroup may allocate, at most
  // 64 KiB (two such workgroups fit a CU's 160 KiB)
  b->lds_limit = std::min<size_t>(prop.sharedMemPerBlock, 64 * 1024);
  b->budget = hbm_budget_bytes;
  b->max_slots = max_slots;
  b->slots.resize(max_slots);
  const size_t ns = (size_t)max_slots;
  bool ok = hipMalloc(&b->d_grids, ns * sizeof(BatchGrid)) == hipSuccess &&
            hipMalloc(&b->d_snaps, ns * 3 * sizeof(void *)) == hipSuccess &&
            hipMalloc(&b->d_active, ns * sizeof(int)) == hipSuccess &&
            hipMalloc(&b->d_counts, 8 * sizeof(int)) == hipSuccess &&
            hipMalloc(&b->d_red, ns * 6 * sizeof(double)) == hipSuccess &&
            hipMalloc(&b->d_ranges, ns * sizeof(int2)) == hipSuccess &&
            hipHostMalloc((void **)&b->h_ranges, ns * sizeof(int2), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&b->h_grids, ns * sizeof(BatchGrid), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&b->h_snaps, ns * 3 * sizeof(void *), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&b->h_active, ns * sizeof(int), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&b->h_counts, 8 * sizeof(int), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&b->h_red, ns * 6 * sizeof(double), hipHostMallocDefault) == hipSuccess;
  if (ok && stream) {
    b->stream = (hipStream_t)stream;
  } else if (ok) {
    ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
    b->own_stream = ok;
  }
  if (!ok) {
    lbt1_batch_destroy(b);
    return fail(LBT1_ENOMEM, "batch allocation failed");
  }
  std::memset(b->h_grids, 0, ns * sizeof(BatchGrid));
  std::memset(b->h_snaps, 0, ns * 3 * sizeof(void *));
  std::memset(b->h_counts, 0, 8 * sizeof(int));
  *out = b;
  return LBT1_OK;
}

lbt1_status lbt1_batch_admit(lbt1_batch *b, lbt1_grid *g, int64_t step_budget, double residual_tol, int32_t *slot) {
  clear_error();
  if (!b || !g || !slot) return fail(LBT1_EINVAL, "null argument");
  if (step_budget < 0) return fail(LBT1_EINVAL, "negative step budget");
  if (g->batch) return fail(LBT1_ESTATE, "grid is already resident in a batch");
  if (!g->geometry) return fail(LBT1_ESTATE, "grid geometry is not set");
  if (g->pop) return fail(LBT1_EINVAL, "population grids (LBT1_OPT_POPULATIONS) cannot join a batch");
  if (g->mp) return fail(LBT1_EINVAL, "multiphase grids (LBT1_OPT_MULTIPHASE) cannot join a batch");
  if (!g->snap[0]) return fail(LBT1_EINVAL, "batched grids need LBT1_OPT_SNAPSHOT");
  if (g->device != b->device) return fail(LBT1_EINVAL, "grid is on another device");
  if (b->prec >= 0 && g->prec != b->prec) return fail(LBT1_EINVAL, "batch precision is %d, grid has %d", b->prec, g->prec);
  const int vclass = vec_class_for(g->prec, g->nx, g->periodic & 1u);
  if ((long)chunks_of(g->nx, kVecOfClass[vclass]) * kVecOfClass[vclass] > g->L.pitch)
    return fail(LBT1_EINVAL, "batch: %d-column chunks overrun the row pitch %d", kVecOfClass[vclass], g->L.pitch);
  const size_t bytes = g->L.total;
  if (b->used + bytes > b->budget) return fail(LBT1_EBUSY, "HBM budget: %zu used + %zu > %zu", b->used, bytes, b->budget);
  int s = -1;
  for (int i = 0; i < b->max_slots; ++i)
    if (b->slots[i].state == LBT1_SLOT_FREE) {
      s = i;
      break;
    }
  if (s < 0) return fail(LBT1_EBUSY, "no free slot (%d in use)", b->max_slots);
  // make sure the grid's own queued work is done before the batch stream touches it
  hipError_t e;
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  Slot &sl = b->slots[s];
  sl = Slot();
  sl.g = g;
  sl.budget = step_budget;
  sl.tol = residual_tol;
  sl.state = step_budget > 0 ? LBT1_SLOT_RUNNING : LBT1_SLOT_BUDGET;
  sl.bytes = bytes;
  sl.vclass = vclass;
  b->prec = g->prec;
  b->used += bytes;
  g->batch = b;
  g->slot = s;
  BatchGrid &d = b->h_grids[s];
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 3; ++q) d.plane[p][q] = g->plane[p][q];
  d.flags = g->flags;
  d.nx = g->nx;
  d.ny = g->ny;
  d.pitch = g->L.pitch;
  d.rs = g->L.rs;
  d.periodic = g->periodic;
  d.wall = g->wall;
  d.parity0 = g->parity;
  d.steps_left = 0;
  d.flips = 0;
  d.strips_x = 0;  // set when the work lists are rebuilt
  d.fx = g->F[0];
  d.fy = g->F[1];
  d.sc_d = g->sc[0];
  d.sc_j = g->sc[1];
  d.is_d = 1.0 / g->sc[0];
  d.is_j = 1.0 / g->sc[1];
  d.trash = g->base + g->L.trash_off;
  for (int q = 0; q < 3; ++q) b->h_snaps[3 * s + q] = g->snap[q];
  b->items_dirty = true;
  *slot = s;
  return LBT1_OK;
}

lbt1_status lbt1_batch_run(lbt1_batch *b, int32_t burst_steps) {
  clear_error();
  if (!b) return fail(LBT1_EINVAL, "null batch");
  if (burst_steps < 1 || burst_steps > 100000) return fail(LBT1_EINVAL, "burst_steps %d out of 1..100000", burst_steps);
  int nact = 0;
  lbt1_status st = launch_burst(b, burst_steps, &nact);
  if (st || nact == 0) return st;
  hipError_t e;
  const size_t ns = (size_t)b->max_slots;
  if ((e = hipMemcpyAsync(b->h_red, b->d_red, ns * 6 * sizeof(double), hipMemcpyDeviceToHost, b->stream)) != hipSuccess)
    return hip_fail(e, "results D2H");
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int k = 0; k < nact; ++k) {
    const int s = b->h_active[k];
    Slot &sl = b->slots[s];
    const double *r = b->h_red + 6 * s;
    sl.taken += sl.steps_this_burst;
    sl.g->steps += sl.steps_this_burst;
    sl.g->parity ^= b->h_grids[s].flips & 1;
    sl.residual = r[3];
    if (r[4] > 0)
      sl.state = LBT1_SLOT_NONFINITE;
    else if (sl.tol >= 0 && sl.residual <= sl.tol)
      sl.state = LBT1_SLOT_CONVERGED;
    else if (sl.taken >= sl.budget)
      sl.state = LBT1_SLOT_BUDGET;
  }
  return LBT1_OK;
}

lbt1_status lbt1_batch_set_shape(lbt1_batch *b, const lbt1_batch_shape *shape) {
  clear_error();
  if (!b || !shape) return fail(LBT1_EINVAL, "null argument");
  return set_shape(b, *shape);
}

lbt1_status lbt1_batch_get_shape(lbt1_batch *b, lbt1_batch_shape *shape) {
  clear_error();
  if (!b || !shape) return fail(LBT1_EINVAL, "null argument");
  if (b->items_dirty) rebuild_items(b);  // the heights the heuristic gives the resident grids now
  shape->fuse = b->fuse_mode;
  shape->lds = b->lds_mode ? 1 : 0;
  for (int c = 0; c < kClasses; ++c) shape->rows[c] = b->rows[c];
  shape->vec_cap = kVecOfClass[b->vec_cap_class];
  return LBT1_OK;
}

lbt1_status lbt1_batch_autotune(lbt1_batch *b, int32_t burst_steps, int32_t reps, lbt1_batch_shape *best,
                                double *ms_per_burst) {
  clear_error();
  if (!b) return fail(LBT1_EINVAL, "null batch");
  if (burst_steps < 1 || burst_steps > 100000 || reps < 1) return fail(LBT1_EINVAL, "burst_steps 1..100000, reps >= 1");
  hipError_t e;
  if ((e = hipSetDevice(b->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  // the resident grids' memory is saved to scratch and restored afterwards
  std::vector<int> res;
  size_t total = 0;
  for (int s = 0; s < b->max_slots; ++s)
    if (b->slots[s].state == LBT1_SLOT_RUNNING) {
      res.push_back(s);
      total += b->slots[s].g->L.total;
    }
  if (res.empty()) return fail(LBT1_ESTATE, "no running grid to tune on");
  char *save = nullptr;
  if ((e = hipMalloc(&save, total)) != hipSuccess) return fail(LBT1_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
  auto copy_all = [&](bool out) -> hipError_t {
    size_t off = 0;
    for (int s : res) {
      lbt1_grid *g = b->slots[s].g;
      const hipError_t er = out ? hipMemcpyAsync(save + off, g->base, g->L.total, hipMemcpyDeviceToDevice, b->stream)
                                : hipMemcpyAsync(g->base, save + off, g->L.total, hipMemcpyDeviceToDevice, b->stream);
      if (er != hipSuccess) return er;
      off += g->L.total;
    }
    return hipSuccess;
  };
  lbt1_status st = LBT1_OK;
  if ((e = copy_all(true)) != hipSuccess) {
    (void)hipFree(save);
    return hip_fail(e, "autotune save");
  }
  const int saved_mode = b->fuse_mode;
  const bool saved_lds = b->lds_mode;
  const int saved_cap = b->vec_cap_class;
  int saved_rows[kClasses];
  std::memcpy(saved_rows, b->want_rows, sizeof saved_rows);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // one candidate: an untimed burst (builds the graph), then the best of `reps`
  auto time_shape = [&](const lbt1_batch_shape &sh) -> double {
    if (set_shape(b, sh) != LBT1_OK) return 1e300;
    double bestms = 1e300;
    for (int r = 0; r <= reps && st == LBT1_OK; ++r) {
      int nact = 0;
      (void)hipEventRecord(e0, b->stream);
      st = launch_burst(b, burst_steps, &nact);
      (void)hipEventRecord(e1, b->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) bestms = std::min(bestms, (double)ms);
    }
    return bestms;
  };
  lbt1_batch_shape bestsh{};
  double best_ms = 1e300;
  const int modes[] = {FUSE_NONE, FUSE_MIXED, FUSE_ALL};
  // every column cap (four, then two columns per lane), LDS mode and fuse mode
  for (int cap = CLS_V4; cap >= CLS_V2 && !st; --cap) {
  for (int lds = 0; lds <= 1 && !st; ++lds) {
    for (int mode : modes) {
      if (st) break;
      // classes the grids take under this policy
      b->fuse_mode = mode;
      b->lds_mode = lds != 0;
      b->vec_cap_class = CLS_V4;
      bool present[kClasses] = {}, wide = false;
      for (int s : res) {
        const int c = class_for(b, b->slots[s]);
        present[c] = true;
        wide |= c == CLS_V4;
      }
      if (lds && !present[CLS_LDS]) continue;
      if (mode != FUSE_NONE && !present[CLS_F2]) continue;
      if (mode == FUSE_MIXED && !present[CLS_V4]) continue;  // the same classes as FUSE_ALL
      if (cap < CLS_V4) {
        // narrower chunks for the four-column grids: only where some grid has them
        if (!wide) continue;
        b->vec_cap_class = cap;
        for (int c = 0; c < kClasses; ++c) present[c] = false;
        for (int s : res) present[class_for(b, b->slots[s])] = true;
      }
      lbt1_batch_shape cur{};
      cur.fuse = mode;
      cur.lds = lds;
      cur.vec_cap = kVecOfClass[cap];
      double cur_ms = time_shape(cur);
      // coordinate descent over the strip height of each class present
      for (int c = 0; c < kClasses && !st; ++c) {
        if (!present[c]) continue;
        const int single[] = {6, 14, 30};
        const int fused[] = {2, 6, 14, 30};
        const int *opts = c == CLS_F2 ? fused : single;
        const int nopt = c == CLS_F2 ? 4 : c == CLS_LDS ? 2 : 3;
        int keep = cur.rows[c];
        for (int k = 0; k < nopt && !st; ++k) {
          lbt1_batch_shape t = cur;
          t.rows[c] = opts[k];
          if (c == CLS_F2 && !batch_fused_kernel(b->prec, opts[k])) continue;
          if (c < CLS_F2 && !batch_step_kernel(b->prec, c, opts[k])) continue;
          const double ms = time_shape(t);
          if (ms < cur_ms) {
            cur_ms = ms;
            keep = opts[k];
          }
        }
        cur.rows[c] = keep;
      }
      if (cur_ms < best_ms) {
        best_ms = cur_ms;
        bestsh = cur;
      }
    }
  }
  }
  (void)hipStreamSynchronize(b->stream);
  const hipError_t er = copy_all(false);
  (void)hipStreamSynchronize(b->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(save);
  if (st || er != hipSuccess || best_ms >= 1e300) {
    b->fuse_mode = saved_mode;
    b->lds_mode = saved_lds;
    b->vec_cap_class = saved_cap;
    std::memcpy(b->want_rows, saved_rows, sizeof saved_rows);
    b->items_dirty = true;
    if (st) return st;
    if (er != hipSuccess) return hip_fail(er, "autotune restore");
    return fail(LBT1_EDEVICE, "autotune timed no shape");
  }
  st = set_shape(b, bestsh);
  if (st) return st;
  if (best) *best = bestsh;
  if (ms_per_burst) *ms_per_burst = best_ms;
  return LBT1_OK;
}

lbt1_status lbt1_batch_poll(lbt1_batch *b, int32_t *done_slots, int32_t cap, int32_t *n_done) {
  clear_error();
  if (!b || !n_done || (cap > 0 && !done_slots)) return fail(LBT1_EINVAL, "null argument");
  int n = 0;
  for (int s = 0; s < b->max_slots; ++s) {
    const int st = b->slots[s].state;
    if (st == LBT1_SLOT_BUDGET || st == LBT1_SLOT_CONVERGED || st == LBT1_SLOT_NONFINITE) {
      if (n < cap) done_slots[n] = s;
      ++n;
    }
  }
  *n_done = n;
  return LBT1_OK;
}

lbt1_status lbt1_batch_slot_info(lbt1_batch *b, int32_t slot, int32_t *state, int64_t *steps, double *residual) {
  clear_error();
  if (!b) return fail(LBT1_EINVAL, "null batch");
  if (slot < 0 || slot >= b->max_slots) return fail(LBT1_EINVAL, "slot %d out of range", slot);
  const Slot &sl = b->slots[slot];
  if (state) *state = sl.state;
  if (steps) *steps = sl.taken;
  if (residual) *residual = sl.residual;
  return LBT1_OK;
}

lbt1_status lbt1_batch_evict(lbt1_batch *b, int32_t slot) {
  clear_error();
  if (!b) return fail(LBT1_EINVAL, "null batch");
  if (slot < 0 || slot >= b->max_slots || b->slots[slot].state == LBT1_SLOT_FREE)
    return fail(LBT1_EINVAL, "slot %d is not in use", slot);
  hipError_t e;
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  Slot &sl = b->slots[slot];
  sl.g->batch = nullptr;
  sl.g->slot = -1;
  b->used -= sl.bytes;
  sl = Slot();
  std::memset(&b->h_grids[slot], 0, sizeof(BatchGrid));
  b->items_dirty = true;
  bool empty = true;
  for (const auto &x : b->slots) empty &= x.state == LBT1_SLOT_FREE;
  if (empty) b->prec = -1;
  return LBT1_OK;
}

lbt1_status lbt1_batch_destroy(lbt1_batch *b) {
  clear_error();
  if (!b) return LBT1_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (auto &sl : b->slots)
    if (sl.g) {
      sl.g->batch = nullptr;
      sl.g->slot = -1;
    }
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  for (int c = 0; c < kClasses; ++c)
    if (b->d_items[c]) (void)hipFree(b->d_items[c]);
  if (b->d_grids) (void)hipFree(b->d_grids);
  if (b->d_snaps) (void)hipFree(b->d_snaps);
  if (b->d_active) (void)hipFree(b->d_active);
  if (b->d_counts) (void)hipFree(b->d_counts);
  if (b->d_red) (void)hipFree(b->d_red);
  if (b->d_ranges) (void)hipFree(b->d_ranges);
  if (b->d_ritems) (void)hipFree(b->d_ritems);
  if (b->d_partials) (void)hipFree(b->d_partials);
  if (b->h_ranges) (void)hipHostFree(b->h_ranges);
  if (b->h_grids) (void)hipHostFree(b->h_grids);
  if (b->h_snaps) (void)hipHostFree(b->h_snaps);
  if (b->h_active) (void)hipHostFree(b->h_active);
  if (b->h_counts) (void)hipHostFree(b->h_counts);
  if (b->h_red) (void)hipHostFree(b->h_red);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return LBT1_OK;
}

}  // extern "C"

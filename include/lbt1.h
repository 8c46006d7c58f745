/*
 * lbt1.h -- C ABI of the MI355X LBMTau1 D2Q9 library (liblbt1.so).
 *
 * Method: M. Matyka and M. Dzikowski, "Memory-efficient Lattice Boltzmann
 * Method for low Reynolds number flows" (arXiv:1912.09327).  With the BGK
 * relaxation time fixed at tau = 1 (Eq. LBMTau1) every post-collision
 * population equals its equilibrium (Eq. maxwellboltzmann), so a node keeps
 * only its density and momentum, and one time step rebuilds the equilibria
 * of the nine upwind neighbours and sums them (Eq. rhotau1, Eq. utau1 read
 * as momentum sums, Algorithm 1).
 *
 * The calls follow the paper's statement of the problem (Algorithm 1 and
 * Appendix A): declare fields and flags (lbt1_create_grid), initialise them
 * (lbt1_set_geometry, the algorithm's initialisation), repeat the step
 * (lbt1_step), read density and momentum back (lbt1_read_moments, the
 * algorithm's optional visualisation).  lbt1_reduce adds the steady-state
 * diagnostics of section 3 (velocity change between two times, mass).
 * The lbt1_batch_* calls run many independent grids together.
 *
 * Conventions for every call:
 *   - all calls return lbt1_status; nothing throws, aborts or exits across
 *     the ABI; on a non-OK status lbt1_last_error() gives a message for the
 *     calling thread.
 *   - host arrays are caller-owned, [ny][nx] row-major with x fastest, and
 *     are only read or written during the call.
 *   - handles are owned by the library until the matching destroy call.  A
 *     handle is not thread-safe; distinct handles may be used from distinct
 *     threads.
 *   - device work is asynchronous with respect to the host unless a call
 *     says it synchronises.
 *   - nothing on this path falls back to the CPU: without a usable gfx950
 *     device, calls that need one return LBT1_EDEVICE.
 */
#ifndef LBT1_H
#define LBT1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbt1_grid lbt1_grid;   /* opaque; one 2-D lattice and its device state */
typedef struct lbt1_batch lbt1_batch; /* opaque; a set of resident grids stepped together */

typedef enum {
  LBT1_OK = 0,
  LBT1_EINVAL = 1,     /* bad argument (sizes, flags, densities, handle) */
  LBT1_ENOMEM = 2,     /* device or host allocation failed, or caller buffer too small */
  LBT1_EDEVICE = 3,    /* a HIP call failed or no gfx950 device is usable */
  LBT1_ESTATE = 4,     /* call out of order (e.g. lbt1_step before lbt1_set_geometry) */
  LBT1_EBUSY = 5,      /* batch has no free slot or HBM budget for the grid */
  LBT1_ENONFINITE = 6  /* a grid's moments became non-finite (reported by poll) */
} lbt1_status;

/* Storage of the moment planes.  Every variant stores the density as the
 * deviation rho - 1 and the momentum j = (jx, jy) (the "shifted" form);
 * F64 computes in double, the others in float. */
typedef enum {
  LBT1_F64 = 0,  /* 8 bytes per value */
  LBT1_F32 = 1,  /* 4 bytes per value */
  LBT1_F16S = 2, /* IEEE binary16, round-to-nearest-even, optional power-of-two scale */
  LBT1_BF16S = 3 /* bfloat16, round-to-nearest-even, optional power-of-two scale */
} lbt1_precision;

/* Treatment of a link from a fluid node x to a solid neighbour x + e_k. */
typedef enum {
  LBT1_WALL_PAPER = 0,  /* Eq. feqnoslip: the term is w_k * rho(x), the zero-velocity
                           equilibrium of x itself (the paper's rule, default) */
  LBT1_WALL_HALFWAY = 1 /* half-way bounce-back: the equilibrium x sends toward the
                           wall, f^eq_k(rho(x), u(x)), returns reversed */
} lbt1_wall;

/* Node flags (uint8 values of the flag plane). */
enum {
  LBT1_FLUID = 0, /* updated every step */
  LBT1_SOLID = 1, /* no-slip wall node; never updated, never a source */
  LBT1_FIXED = 2  /* Dirichlet node (the moving lid of Appendix A): a source with its
                     stored moments, never updated */
};

enum { LBT1_PERIODIC_X = 1u, LBT1_PERIODIC_Y = 2u };

/* lbt1_grid_desc.options bits */
enum {
  LBT1_OPT_SNAPSHOT = 1u, /* keep a copy of the state for the residual */
  LBT1_OPT_PLANAR = 2u,   /* store rho - 1, jx, jy as three separate planes; by default
                             the three rows of each lattice row are adjacent in memory
                             ([ny][3][pitch]), so a row is one contiguous read and one
                             contiguous write */
  LBT1_OPT_POPULATIONS = 4u, /* the standard stored-population D2Q9 BGK method instead of
                             LBMTau1 (section 2, Eq. lbm, with relaxation time
                             lbt1_grid_desc.tau): two parities of nine population fields,
                             each stored as the deviation f_q - w_q in the grid's storage
                             format (scale[0] applies), (2 Q) c bytes per node against
                             LBMTau1's 2 N_f c (section 4).  Same flags, walls, lid and
                             force rules; the equilibrium velocity is (j + tau F) / rho.
                             lbt1_step runs one kernel (set_kernel/autotune: EINVAL); the
                             grid cannot join a batch */
  LBT1_OPT_MULTIPHASE = 8u  /* single-component multiphase flow: the Shan-Chen interaction
                             force of the paper's Eq. f_sc, F(x) = -G psi(x) sum_k w_k
                             psi(x + e_k) e_k with psi(rho) = rho0 (1 - exp(-rho / rho0))
                             (lbt1_grid_desc.sc_G, sc_rho0), is added to the body force of
                             every node before its equilibrium is formed.  A SOLID
                             neighbour contributes the psi of its stored density (a
                             wetting control), a neighbour outside a non-periodic axis that
                             of the node itself.  No FIXED nodes (EINVAL); no batches.
                             LBMTau1 grids keep no psi field (it is formed in registers);
                             population grids keep one psi value per node */
};

/* lbt1_reduce what-mask bits and output slots */
enum {
  LBT1_REDUCE_MASS = 1u,      /* out[0] = sum of rho over FLUID nodes */
  LBT1_REDUCE_MOMENTUM = 2u,  /* out[1], out[2] = sum of jx, jy over FLUID nodes */
  LBT1_REDUCE_RESIDUAL = 4u,  /* out[3] = max over FLUID nodes and both components of
                                 |u - u_snap|, u = j / rho, against the snapshot taken
                                 by the previous residual call (or lbt1_set_geometry);
                                 the snapshot is then refreshed to the current state */
  LBT1_REDUCE_NONFINITE = 8u  /* out[4] = number of FLUID nodes with a non-finite value */
};
#define LBT1_REDUCE_SLOTS 6 /* out[5] = number of FLUID nodes (always written) */

typedef struct {
  int32_t nx, ny;        /* lattice size, each >= 3 and <= 65536 */
  uint32_t periodic;     /* LBT1_PERIODIC_X | LBT1_PERIODIC_Y; a neighbour outside a
                            non-periodic axis counts as SOLID */
  int32_t prec;          /* lbt1_precision */
  int32_t wall;          /* lbt1_wall */
  uint32_t options;      /* LBT1_OPT_* */
  double force[2];       /* body force F, added to the momentum before the equilibrium
                            velocity (j + F) / rho is formed (Algorithm 1); uniform */
  double scale[2];       /* F16S/BF16S: stored value = value / scale, for rho - 1 and for
                            j; must be powers of two; 0 means 1 */
  void *device_buffer;   /* optional caller-owned device memory of at least
                            lbt1_grid_bytes(...) bytes, 256-byte aligned; NULL: the
                            library allocates */
  size_t device_bytes;   /* size of device_buffer */
  void *stream;          /* hipStream_t to run on; NULL: a library-owned stream */
  double tau;            /* relaxation time of LBT1_OPT_POPULATIONS grids, > 1/2 (0 means
                            1); other grids are LBMTau1 (tau = 1): 0 or 1 only */
  double sc_G;           /* LBT1_OPT_MULTIPHASE: Shan-Chen coupling G (finite; negative is
                            attractive, phase separation below about -4); 0 otherwise */
  double sc_rho0;        /* LBT1_OPT_MULTIPHASE: psi scale rho0 > 0 (0 means 1) */
} lbt1_grid_desc;

/* Device bytes a grid of this shape needs: two parities of the three moment
 * fields (the paper's 2 N_f c per node, Eq. LBMTau1memory, with rows padded
 * to 64 values), one flag byte per node, one more copy of the three fields
 * with LBT1_OPT_SNAPSHOT, and a small reduction workspace.  With
 * LBT1_OPT_POPULATIONS two parities of nine population fields (2 Q c per
 * node, Eq. lbmmemory without the separate moment arrays) replace the moment
 * fields.  0 on bad arguments. */
size_t lbt1_grid_bytes(int32_t nx, int32_t ny, int32_t prec, uint32_t options);

/* Create a grid (no device work yet besides allocation).  *out receives the handle. */
lbt1_status lbt1_create_grid(const lbt1_grid_desc *desc, lbt1_grid **out);

/* Initialise flags and moments in both parities (the algorithm's first line).
 *   flags: ny*nx uint8 in {FLUID, SOLID, FIXED}, or NULL for all FLUID
 *   rho, jx, jy: ny*nx doubles each, or all three NULL for rho = 1, j = 0;
 *                rho must be finite and > 0, j finite.
 * Synchronises the grid's stream.  EINVAL on bad values. */
lbt1_status lbt1_set_geometry(lbt1_grid *g, const uint8_t *flags, const double *rho,
                              const double *jx, const double *jy);

/* Enqueue n >= 0 LBMTau1 steps (Algorithm 1) on the grid's stream and return.
 * ESTATE before lbt1_set_geometry. */
lbt1_status lbt1_step(lbt1_grid *g, int64_t n);

/* Copy the current density rho and momentum (jx, jy) into ny*nx host arrays
 * (any of them may be NULL).  Synchronises the grid's stream. */
lbt1_status lbt1_read_moments(lbt1_grid *g, double *rho, double *jx, double *jy);

/* Copy the moments of the window x0 <= x < x0+w, y0 <= y < y0+h into h*w host
 * arrays (row-major, x fastest; any of them may be NULL).  Used for point
 * probes of large grids: the centre-velocity and mid-section flux stopping
 * rules of section 3, and sampled checks.  EINVAL if the window is empty or
 * not inside the grid.  Synchronises the grid's stream. */
lbt1_status lbt1_read_window(lbt1_grid *g, int32_t x0, int32_t y0, int32_t w, int32_t h, double *rho, double *jx,
                             double *jy);

/* LBT1_OPT_POPULATIONS grids: copy the nine populations f_q = w_q + stored
 * deviation into a host array of 9 * ny * nx doubles, [9][ny][nx] in the
 * direction order of section 2 (the populations after streaming, before the
 * next collision; FIXED nodes hold the equilibrium of their moments with the
 * force shift).  EINVAL for other grids.  Synchronises the grid's stream.
 * For these grids lbt1_read_moments/lbt1_read_window report rho = sum f and
 * j = sum e f of FLUID nodes (summed in FP64 on the host from the decoded
 * populations) and the moments given to lbt1_set_geometry for SOLID and
 * FIXED nodes. */
lbt1_status lbt1_read_populations(lbt1_grid *g, double *f);

/* FP64 diagnostics over FLUID nodes, see LBT1_REDUCE_*; out has
 * LBT1_REDUCE_SLOTS doubles, slots not asked for are left untouched except
 * out[5].  Synchronises the grid's stream. */
lbt1_status lbt1_reduce(lbt1_grid *g, uint32_t what, double *out);

/* lbt1_reduce for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same diagnostics,
 * enqueued on the grid's stream without synchronising and without allocating
 * anything.  The partial sums go to a static device array of the library
 * (1024 rows of six doubles, 48 KiB per device, held until the process ends)
 * instead of the grid's workspace; every grid size fits, since the partial
 * count is capped at 1024 (EINVAL otherwise).  `out` is caller-owned
 * device-accessible memory of LBT1_REDUCE_SLOTS doubles, written when the
 * stream reaches this work, with the slots of lbt1_reduce (those not asked for
 * untouched except out[5]); results are bitwise those of lbt1_reduce.  With
 * LBT1_REDUCE_RESIDUAL the snapshot is refreshed as by lbt1_reduce.  The
 * static array is shared by all calls on one device: calls whose work overlaps
 * on the device (grids on different streams) race and must be ordered by the
 * caller. */
lbt1_status lbt1_reduce_noalloc(lbt1_grid *g, uint32_t what, double *out);

/* Exact checkpoint and resume (the state is the paper's fields, Algorithm 1).
 * lbt1_read_moments returns rho = 1 + (rho - 1) in FP64, which rounds for FP64
 * storage; these calls move the stored bits instead.  lbt1_save_state copies the
 * current state in storage format -- the parity block, then the residual
 * snapshot when the grid keeps one, lbt1_state_bytes(g) bytes -- into caller host
 * memory (EINVAL if `bytes` is smaller).  lbt1_load_state puts such a block back
 * into a grid of the same shape, precision and options whose geometry (flags) is
 * set, in both parities (EINVAL if `bytes` differs); stepping then continues bit
 * for bit as the saved grid would have.  Both synchronise the grid's stream. */
size_t lbt1_state_bytes(lbt1_grid *g);
lbt1_status lbt1_save_state(lbt1_grid *g, void *host, size_t bytes);
lbt1_status lbt1_load_state(lbt1_grid *g, const void *host, size_t bytes);

/* Wait until all work enqueued on the grid's stream has finished. */
lbt1_status lbt1_sync(lbt1_grid *g);

/* Release the grid (after its stream drained).  NULL is accepted. */
lbt1_status lbt1_destroy_grid(lbt1_grid *g);

/* Message for the last non-OK status returned to this thread ("" if none). */
const char *lbt1_last_error(void);

/* ---------------------------------------------------------------- kernel choice */

/* Step kernel families. */
enum {
  LBT1_KERNEL_AUTO = 0,   /* library choice (tuned table, else heuristic) */
  LBT1_KERNEL_GATHER = 1, /* one thread per node, nine neighbour reads */
  LBT1_KERNEL_STRIP = 2   /* a wavefront walks a strip of rows; each lane owns `vec`
                             adjacent columns, neighbour columns come from adjacent
                             lanes; every moment is read from memory once per strip
                             (plus one halo row above and below and one halo chunk on
                             each side) */
};

typedef struct {
  int32_t kernel; /* LBT1_KERNEL_* */
  int32_t vec;    /* STRIP: columns per lane, 1, 2, 4 or 8.  Must divide nx on a grid
                     periodic in x; otherwise the last chunk of a row may run into the
                     row padding, which reads as SOLID like the outside of the axis */
  int32_t rows;   /* STRIP: rows per strip, 6 or 14 (fused kernels also 22; 28 for three
                     FP32 steps, 30 for 16-bit storage; two steps on grids with walls also 2,
                     and 30 except in FP64; lbt1_set_kernel
                     says EINVAL for a shape that is not built) */
  int32_t waves;  /* STRIP: resident wavefronts per CU the launch aims at (1..32);
                     0 = one wavefront per strip, no grid-stride loop */
  int32_t fuse;   /* STRIP: time steps per launch.  0 or 1: one.  2 or 3: that many
                     steps in one pass over memory (the state is read and written
                     once per pass, results bit for bit those of single steps);
                     fuse <= vec.  3: vec 4, FP32, grids periodic in x and y without
                     SOLID or FIXED nodes.  2: any grid that is not multiphase (with
                     walls, fixed nodes or open axes: vec 2, rows 2, 6, 14, or 30
                     except in FP64).  Step counts that are not a
                     multiple of fuse end with two-step launches of the same strip
                     shape (after three-step ones), else single-step launches of the
                     same height, else the gather kernel. */
} lbt1_kernel_config;

/* Select the step kernel for a grid.  EINVAL if the combination is not built
 * or does not fit the grid. */
lbt1_status lbt1_set_kernel(lbt1_grid *g, const lbt1_kernel_config *cfg);

/* The configuration lbt1_step uses now; name (optional) receives the kernel's
 * symbol-like name, NUL-terminated, at most name_cap bytes. */
lbt1_status lbt1_get_kernel(lbt1_grid *g, lbt1_kernel_config *cfg, char *name, size_t name_cap);

/* Time every built configuration that fits this grid, on the grid's own memory
 * (its state is saved to scratch memory first and restored afterwards):
 * `steps` steps each, best of `reps`; then those within 5 % of the fastest (at
 * most eight) again as lbt1_step runs them, in graph bursts of 64 steps (three
 * bursts each, in interleaved rounds, best of max(reps, 3)).  Selects the
 * fastest and returns it in *best (optional) and its time per step in
 * *ms_per_step (optional).  The grid's state is unchanged.  The result is
 * remembered for grids of the same precision, flag use and size in this
 * process.  Needs 2 * state bytes of scratch device memory (ENOMEM otherwise). */
lbt1_status lbt1_autotune(lbt1_grid *g, int32_t steps, int32_t reps, lbt1_kernel_config *best,
                          double *ms_per_step);

/* ---------------------------------------------------------------- 3-D grids */

/* Three-dimensional LBMTau1 on the D3Q19 or D3Q27 lattice (the lattices of the
 * memory analysis of section 4): the step of Algorithm 1 with Q directions; a
 * node keeps rho - 1 and (jx, jy, jz), 2 * 4 * c bytes per node over both
 * parities against (2 Q + 4) c for the standard method (Eq. lbmmemory).  The
 * body force, the two wall rules and FIXED nodes as in 2-D; a neighbour
 * outside a non-periodic axis is a wall.  Host arrays are [nz][ny][nx], x
 * fastest.  Same conventions as the 2-D calls. */
typedef struct lbt1_grid3d lbt1_grid3d;

typedef struct {
  int32_t nx, ny, nz;    /* x, y: 3..16384; z: 1..16384 */
  int32_t q;             /* 19 or 27 */
  uint32_t periodic;     /* bit 0 x, bit 1 y, bit 2 z */
  int32_t prec;          /* lbt1_precision */
  int32_t wall;          /* lbt1_wall */
  uint32_t options;      /* LBT1_OPT_SNAPSHOT only */
  double force[3];       /* uniform body force, added to the momentum before the
                            equilibrium velocity is formed */
  double scale[2];       /* F16S/BF16S scales of rho - 1 and j (powers of two; 0 = 1) */
  void *device_buffer;   /* optional caller memory of lbt1_grid3d_bytes(...) bytes, 256-aligned */
  size_t device_bytes;
  void *stream;          /* hipStream_t, NULL: a library stream */
} lbt1_grid3d_desc;

/* Device bytes: two parities of the four moment fields ([nz][ny][4][pitch],
 * pitch = nx rounded up to 64), one flag byte per node, a snapshot with
 * LBT1_OPT_SNAPSHOT, reduction workspace.  0 on bad arguments. */
size_t lbt1_grid3d_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t q, int32_t prec, uint32_t options);
lbt1_status lbt1_grid3d_create(const lbt1_grid3d_desc *d, lbt1_grid3d **out);
/* Flags (NULL: all FLUID) and moments (NULL: rho = 1, j = 0); validation as 2-D. */
lbt1_status lbt1_grid3d_set_geometry(lbt1_grid3d *g, const uint8_t *flags, const double *rho, const double *jx,
                                     const double *jy, const double *jz);
/* n steps, asynchronous (one launch per step, one thread per node). */
lbt1_status lbt1_grid3d_step(lbt1_grid3d *g, int64_t n);
/* rho and momentum into nz*ny*nx host arrays (any may be NULL); synchronises. */
lbt1_status lbt1_grid3d_read_moments(lbt1_grid3d *g, double *rho, double *jx, double *jy, double *jz);
/* FP64 diagnostics over FLUID nodes into out[8]: 0 mass, 1..3 momentum,
 * 4 residual max |u - u_snap| (LBT1_REDUCE_RESIDUAL, refreshes the snapshot),
 * 5 non-finite count, 6 FLUID count, 7 zero.  Synchronises. */
lbt1_status lbt1_grid3d_reduce(lbt1_grid3d *g, uint32_t what, double *out);
/* Kernel family: LBT1_KERNEL_AUTO (default) and LBT1_KERNEL_STRIP take the tile
 * kernel (a block of 8 rows marches along z with three planes of per-node
 * values in LDS: a wavefront holds 64 targets of a row and the block a halo
 * ring, with the flags in LDS on grids with SOLID or FIXED nodes or a
 * non-periodic axis; for D3Q27 on grids with every axis periodic and no SOLID
 * or FIXED node, 62 targets and 2 halo columns, the x neighbours taken by lane
 * shifts); LBT1_KERNEL_GATHER one thread per node.  They give the same bits.
 * get_kernel reports the family bound (ESTATE before set_geometry). */
lbt1_status lbt1_grid3d_set_kernel(lbt1_grid3d *g, int32_t kernel);
lbt1_status lbt1_grid3d_get_kernel(lbt1_grid3d *g, int32_t *kernel);
lbt1_status lbt1_grid3d_sync(lbt1_grid3d *g);
lbt1_status lbt1_grid3d_destroy(lbt1_grid3d *g);

/* ---------------------------------------------------------------- batches */

/* A batch steps every resident grid together: one launch per time step (or per
 * two steps, see lbt1_batch_shape) covers the strips of all grids of a work
 * class, and bursts of steps run as a HIP graph.
 *   hbm_budget_bytes: admission limit on the sum of lbt1_grid_bytes of resident grids
 *   max_slots:        admission limit on the number of resident grids (1..65536)
 *   stream:           hipStream_t for the batch's work, NULL for a library stream
 * Grids admitted must be F16S/BF16S/F32/F64 grids created with LBT1_OPT_SNAPSHOT, whose
 * geometry is set, on the same device; all grids of a batch share one precision. */
lbt1_status lbt1_batch_create(size_t hbm_budget_bytes, int32_t max_slots, void *stream,
                              lbt1_batch **out);

/* Make g resident.  It will take at most step_budget more steps and is
 * finished early when its residual (LBT1_REDUCE_RESIDUAL, checked at burst
 * ends) is <= residual_tol (use a negative value to disable).  *slot receives
 * its slot id.  EBUSY when the budget or slots are exhausted (nothing changes).
 * The grid must not be stepped or destroyed while resident. */
lbt1_status lbt1_batch_admit(lbt1_batch *b, lbt1_grid *g, int64_t step_budget, double residual_tol,
                             int32_t *slot);

/* Run one burst of burst_steps steps (>= 1) for every resident, unfinished grid,
 * then the residual / non-finite check of every such grid.  Synchronises. */
lbt1_status lbt1_batch_run(lbt1_batch *b, int32_t burst_steps);

/* Report the slots that are finished (budget used, converged or non-finite):
 * up to cap slot ids go to done_slots, their count to *n_done.  The reason is
 * given by lbt1_batch_slot_info.  Finished grids stay resident (and are not
 * stepped) until evicted. */
lbt1_status lbt1_batch_poll(lbt1_batch *b, int32_t *done_slots, int32_t cap, int32_t *n_done);

/* Reason codes of lbt1_batch_slot_info */
enum {
  LBT1_SLOT_FREE = 0,
  LBT1_SLOT_RUNNING = 1,
  LBT1_SLOT_BUDGET = 2,    /* finished: step budget used */
  LBT1_SLOT_CONVERGED = 3, /* finished: residual <= tolerance */
  LBT1_SLOT_NONFINITE = 4  /* finished: non-finite moments (the grid is not stepped further) */
};

/* State of a slot: reason (LBT1_SLOT_*), steps taken since admission, last residual. */
lbt1_status lbt1_batch_slot_info(lbt1_batch *b, int32_t slot, int32_t *state, int64_t *steps,
                                 double *residual);

/* Tile shape of a batch.  Every resident grid runs in one of five work classes:
 * one step per launch at 1, 2 or 4 columns per lane (classes 0, 1, 2; strips of
 * 62 chunks of that many columns; a grid takes the widest class that fits it),
 * two steps per launch at 2 columns per lane (class 3, the fused class: the state
 * crosses memory once per two steps, as lbt1_kernel_config.fuse = 2 does for one
 * grid), or resident in LDS for a whole burst (class 4: one workgroup per grid
 * copies the grid into LDS, takes all of its steps of the burst there and writes
 * it back; grids whose two copies fit 64 KiB of LDS, about 64 x 64 nodes in 16-bit
 * storage, 45 x 45 in FP32; not FP64).  Results are bit for bit the same in every class. */
enum {
  LBT1_BATCH_FUSE_NONE = 0,   /* every grid one step per launch */
  LBT1_BATCH_FUSE_ALL = 1,    /* every grid whose rows 2 columns per lane fit in the fused class */
  LBT1_BATCH_FUSE_MIXED = 2   /* the fused class except for grids of the 4-column class narrower
                                 than 1024 columns (the default) */
};
typedef struct {
  int32_t fuse;     /* LBT1_BATCH_FUSE_* */
  int32_t lds;      /* 1: grids that fit run resident in LDS (class 4); 0: they do not */
  int32_t rows[5];  /* strip height of classes 0..4: 6, 14 or 30 (not 30 in FP64) for classes 0-2;
                       2, 6, 14 or 30 (not 30 in FP64) for class 3; 6 or 14 for class 4; 0 = the
                       library's heuristic (14 rows where a class has eight or more strips per CU,
                       else 6; class 3 30 rows where it has four or more such strips per CU) */
  int32_t vec_cap;  /* widest columns per lane of the one-step classes: 4 (and 0: the
                       default), 2 or 1; narrower chunks hold fewer registers, so more
                       wavefronts per SIMD hide memory latency */
} lbt1_batch_shape;

/* Take a tile shape for the following bursts.  EINVAL for a shape that is not built. */
lbt1_status lbt1_batch_set_shape(lbt1_batch *b, const lbt1_batch_shape *shape);

/* The fuse mode, LDS mode and column cap in force and the strip heights the resident
 * grids run with now. */
lbt1_status lbt1_batch_get_shape(lbt1_batch *b, lbt1_batch_shape *shape);

/* Time tile shapes on the resident, running grids and keep the fastest: each fuse
 * and LDS mode that changes some grid's class, with the strip height of each class chosen
 * in turn (coordinate descent), every candidate timed as bursts of burst_steps
 * steps as lbt1_batch_run runs them (the best of `reps` after one untimed burst).
 * The grids' device memory is saved to scratch first and restored afterwards
 * (ENOMEM when the scratch does not fit), and no step counts, parities or slot
 * states change.  *best (optional) receives the shape, *ms_per_burst (optional)
 * its time.  ESTATE when no grid is running.  Synchronises. */
lbt1_status lbt1_batch_autotune(lbt1_batch *b, int32_t burst_steps, int32_t reps, lbt1_batch_shape *best,
                                double *ms_per_burst);

/* Remove the grid in `slot` from the batch (it stays valid and owned by the caller). */
lbt1_status lbt1_batch_evict(lbt1_batch *b, int32_t slot);

/* Release the batch (it must be empty or its grids are simply evicted). */
lbt1_status lbt1_batch_destroy(lbt1_batch *b);

/* ---------------------------------------------------------------- diagnostics */

enum {
  LBT1_PROBE_COPY = 0,     /* one input stream, one output stream */
  LBT1_PROBE_READ = 1,     /* one input stream */
  LBT1_PROBE_WRITE = 2,    /* one output stream */
  LBT1_PROBE_3IN3OUT = 3   /* three inputs, three outputs: the access pattern of one
                              moments-only step over three moment planes */
};

/* Achievable device bandwidth of a plain streaming pattern: library-allocated
 * scratch of about `bytes` bytes (>= 1 MiB) split over the pattern's streams,
 * float4 accesses, stores nontemporal when `nontemporal` != 0.  Eight launch
 * shapes are tried (4 to 32 blocks of 256 threads per CU, one or several
 * elements in flight per thread), each `reps` timed launches after a warm-up;
 * *gbps = bytes read and written / time of the fastest, in GB/s.  Runs on the
 * current device's null stream and synchronises. */
lbt1_status lbt1_probe_bandwidth(int32_t kind, size_t bytes, int32_t nontemporal, int32_t reps, double *gbps);

#ifdef __cplusplus
}
#endif

#endif /* LBT1_H */

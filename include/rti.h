/*
 * rti.h -- C ABI of librti: the time step of the nested nonlinear long-wave
 * (shallow-water) model of the RTi real-time tsunami inundation simulator
 * (arXiv 2408.07609), run on one AMD Instinct MI355X (gfx950) GPU.
 *
 * What one step computes (paper, Sec. II-A and Sec. IV-A):
 *   1. continuity, Eq. (1): the water level eta of every cell from the
 *      divergence of the discharge fluxes M (x-faces) and N (y-faces);
 *   2. child -> parent: the water level of the parent cells on the ring of a
 *      child's footprint becomes the mean of the 3x3 child cells below them
 *      (Sec. IV-C);
 *   3. momentum, Eqs. (2)-(3): M and N from the pressure gradient g D grad(eta),
 *      upwind advection of M^2/D, MN/D, N^2/D and semi-implicit Manning
 *      friction g n^2 M sqrt(M^2+N^2)/D^{7/3}, D = h + eta, with a wet/dry
 *      moving shoreline;
 *   4. parent -> child: the discharge of the parent faces on a child's edge is
 *      injected into the child's boundary faces (3:1 nesting, Sec. II-A);
 *   5. open (radiating) or wall sides of the root level;
 *   6. running maxima: highest water level on sea cells and deepest
 *      inundation on land (the outputs of Sec. IV-A).
 * Levels use the same time step (Sec. V-A) and must satisfy the CFL bound
 * of Eq. (4): dx_l / dt >= sqrt(2 g h_max,l).
 *
 * Conventions.
 *   - Host arrays are row-major with x (i) fastest: a level of nx by ny cells
 *     has eta, h and the maxima as nx*ny doubles, cell (i,j) at i + nx*j;
 *     M as (nx+1)*ny doubles, x-face (i,j) between cells (i-1,j) and (i,j) at
 *     i + (nx+1)*j; N as nx*(ny+1) doubles, y-face (i,j) between cells (i,j-1)
 *     and (i,j) at i + nx*j.
 *   - h > 0 is still-water depth [m]; h <= 0 is land whose elevation is -h.
 *   - Every call returns 0 (RTI_OK) or a negative RTI_E* code; the message of
 *     the last failure on the calling thread is rti_last_error().  No call
 *     throws; no call aborts the process.
 *   - The caller owns every host buffer it passes and every buffer it gets
 *     back; the library copies what it needs.  A domain handle is owned by
 *     the library until rti_domain_destroy.
 *   - One thread at a time per domain.  Distinct domains may be driven from
 *     distinct threads on distinct streams.
 */
#ifndef RTI_H
#define RTI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RTI_OK = 0,
    RTI_EINVAL = -1,       /* bad argument: null pointer, size, level index, enum value */
    RTI_ENOMEM = -2,       /* device memory or arena too small */
    RTI_EHIP = -3,         /* a HIP runtime call failed (message names it) */
    RTI_ECFL = -4,         /* Eq. (4) violated on some level */
    RTI_ENEST = -5,        /* nesting rule violated (ratio 3, inclusion, margin) */
    RTI_ESTATE = -6,       /* call not allowed in the domain's current state */
    RTI_EDIVERGED = -7,    /* non-finite water level or flux found (sticky) */
    RTI_EINTERNAL = -8     /* an internal device check failed (active-tile list overflow; sticky) */
};

/* Arithmetic of the step.  RTI_FP64: everything in binary64.  RTI_FP32_BULK:
 * h, the maxima and the fluxes M, N are stored in binary32 and the momentum
 * update runs in binary32; the water level, its continuity update, face
 * depths, wet/dry tests and the level difference of the pressure term stay
 * binary64.  Host arrays are binary64 in both cases (converted on copy). */
enum { RTI_FP64 = 0, RTI_FP32_BULK = 1 };
enum { RTI_BC_OPEN = 0, RTI_BC_WALL = 1 };  /* root sides */
enum { RTI_GAUSS = 0, RTI_COS2_ELLIPSE = 1 };

/* flags of rti_domain_desc */
#define RTI_FLAG_NO_GRAPH    0x1u   /* rti_step launches kernels one by one instead of replaying a HIP graph */
#define RTI_FLAG_NO_ACTIVE   0x2u   /* compute every tile; do not skip stationary tiles */
#define RTI_FLAG_PHASED      0x4u   /* one kernel per phase (mass, ring mean, momentum, edge fluxes)
                                       instead of the fused tile kernel; for comparison */
#define RTI_FLAG_PERSISTENT  0x8u   /* launch the fused kernel with a fixed grid of resident
                                       wavefronts that loop over the active tiles, instead of one
                                       workgroup per tile (also a flag of rti_batch_create) */
#define RTI_MAX_LEVELS 128

/* One nest level.  A resolution that the paper's model covers with several
 * rectangular blocks (Sec. II-A, Table 1) is given either as several entries,
 * one per block, each with its own parent, or -- where blocks of the
 * resolution touch -- as one entry whose array covers their bounding box with
 * a mask of the cells inside the blocks.  Level 0 is the root (parent = -1);
 * every other level names a parent listed before it.  A child's spacing is
 * its parent's divided by 3 (Sec. II-A); its nx and ny are multiples of 3 and
 * at least 9; its footprint, the parent cells [off_i, off_i + nx/3) x
 * [off_j, off_j + ny/3), lies inside the parent with at least 3 parent cells
 * on every side; sibling footprints keep 3 parent cells apart.
 *
 * Masked levels (mask not NULL; not on the root): mask[i + nx*j] is 1 for a
 * cell inside the level and 0 for one outside; it is constant over the 3x3
 * cells of each parent cell, so each parent cell of the footprint is covered
 * (its cells inside) or not, and at least one is covered.  Blocks that share
 * an edge are then one grid: their common faces are computed like any other.
 * Cells outside take no part in the step: every face touching one carries no
 * computed flux, the parent's flux is injected on every parent face between a
 * covered and an uncovered parent cell (Sec. IV-A), and the child-to-parent
 * mean (Sec. IV-C) is taken on every covered parent cell with an uncovered
 * neighbour (8-neighbourhood; for a rectangle, its outermost ring).  A child
 * of a masked level keeps 3 of its parent cells away from the cells outside
 * it.  h and the values given for outside cells are ignored; the state and
 * the maxima read back 0 there. */
typedef struct {
    int32_t nx, ny;        /* cells */
    int32_t parent;        /* index into levels[], -1 for the root */
    int32_t off_i, off_j;  /* child origin in parent cells */
    const double *h;       /* host, nx*ny still-water depth [m]; copied by rti_domain_create */
    const uint8_t *mask;   /* host, nx*ny, 1 inside / 0 outside, or NULL (every cell); copied by create */
} rti_level_desc;

typedef struct {
    int32_t n_levels;                /* 1 .. RTI_MAX_LEVELS */
    const rti_level_desc *levels;
    double dx0;                      /* root spacing [m] */
    double x0, y0;                   /* south-west corner of the root [m] */
    double dt;                       /* time step [s], all levels */
    double g;                        /* gravity [m/s^2] (9.81) */
    double manning_n;                /* Manning roughness [s m^-1/3] (0.025) */
    double dry_eps;                  /* dry threshold on total depth [m] (0.01; at least 1e-12) */
    int32_t bc[4];                   /* root sides W, E, S, N: RTI_BC_OPEN or RTI_BC_WALL */
    int32_t precision;               /* RTI_FP64 or RTI_FP32_BULK (not with RTI_FLAG_PHASED) */
    uint32_t flags;                  /* RTI_FLAG_* */
} rti_domain_desc;

typedef struct rti_domain rti_domain;   /* opaque */

/* Initial sea-surface displacement, applied on every level at t = 0.
 * Offsets from (xc, yc) rotated by theta: x' along the a axis, y' along b.
 * RTI_GAUSS: amp exp(-((x'/a)^2 + (y'/b)^2)/2).
 * RTI_COS2_ELLIPSE: amp cos^2(pi rho/2) for rho^2 = (x'/a)^2 + (y'/b)^2 < 1,
 * else 0 (a, b semi-axes). */
typedef struct {
    double xc, yc;       /* centre [m] */
    double a, b;         /* scales [m] */
    double theta;        /* rotation of the a axis from x [rad] */
    double amp;          /* amplitude [m] */
    int32_t shape;       /* RTI_GAUSS or RTI_COS2_ELLIPSE */
} rti_source;

/* Device bytes a domain needs (state, bathymetry, maxima, tile tables), for
 * admission against free HBM.  Validates the descriptor like create. */
int rti_domain_footprint(const rti_domain_desc *desc, size_t *bytes);

/* Validate the descriptor (Eq. (4) -> RTI_ECFL, nesting -> RTI_ENEST), carve
 * device memory from arena (device pointer, arena_bytes >= footprint, 256-byte
 * aligned; the caller keeps it alive until destroy) or allocate it when arena
 * is NULL, copy the bathymetry, and set the lake at rest (eta = 0 at sea,
 * -h on land, no flux).  hip_stream (a hipStream_t, may be NULL for the
 * default stream) is borrowed: every kernel of this domain runs on it.
 * Besides the device memory, the domain holds two timing events and one
 * word of pinned host memory (the active-tile count rti_step reads back),
 * released by rti_domain_destroy.
 * Validation happens before any HIP call, so it works without a GPU. */
int rti_domain_create(const rti_domain_desc *desc, void *arena, size_t arena_bytes,
                      void *hip_stream, rti_domain **out);

/* Parametric initial condition (see rti_source) on every level at t = 0.
 * The time-integration loop of Sec. IV-A starts from an initial water level
 * that the fault model outside the loop provides; the paper gives that model
 * no form, so the instantaneous displacement shapes here are a reading.
 * Sea cells (h > 0) take the displacement, land keeps eta = -h, a level below
 * the ground is clipped to it; fluxes zero; maxima start at these values.
 * Evaluated on the device with the device's exp, sin and cos (not correctly
 * rounded: within a few ulp of any other evaluation).
 * RTI_ESTATE once the domain has stepped (use rti_set_state to restart). */
int rti_set_source(rti_domain *dom, const rti_source *src);

/* Raw initial water level of one level (host, nx*ny), clipped to the ground;
 * fluxes of that level zeroed; its maxima start here.  t = 0 only. */
int rti_set_eta(rti_domain *dom, int32_t level, const double *eta0);

/* Enqueue nsteps time steps on the domain's stream and return (asynchronous).
 * One step is one iteration of the loop of Sec. IV-A: continuity (Eq. 1) on
 * every level, the child-to-parent water level on the footprint rings
 * (Sec. IV-C), momentum (Eqs. 2-3), the parent-to-child fluxes and the open
 * or wall sides of the root, and the output maxima; every level advances by
 * the same dt (Sec. V-A).  FP64 results are bitwise reproducible (every
 * operation correctly rounded).  nsteps >= 0.  RTI_EDIVERGED if an earlier
 * synchronising call found the domain diverged.
 * Whole groups of 20 steps replay a HIP graph (unless RTI_FLAG_NO_GRAPH).
 * After each graph the active-tile count of its last step is copied, on the
 * stream, into pinned host memory the domain holds; when it is large the
 * next graph leaves the sparse-step kernel out (the fused kernel then
 * computes every listed tile, however few), else it launches both as an
 * eager step does; the results are the same either way. */
int rti_step(rti_domain *dom, int64_t nsteps);

/* Step until round(t_end / dt) steps have been taken in total (the paper's
 * forecast is a 6 h run at dt = 0.2 s, Sec. V-A: 108,000 steps), then
 * synchronise, check every level for non-finite values and read the sticky
 * device checks (RTI_EDIVERGED, RTI_EINTERNAL as rti_sync). */
int rti_run(rti_domain *dom, double t_end);

/* Maxima of one level (host out, nx*ny), the outputs the loop of Sec. IV-A
 * accumulates at the end of each iteration: the highest water level on sea
 * cells (h > 0) and the largest total depth h + eta, the inundation depth,
 * on land (h <= 0), over every step taken, t = 0 included.  Synchronises. */
int rti_max_inundation(rti_domain *dom, int32_t level, double *out);

/* Copy the state of one level to the host (any pointer may be NULL to skip
 * that field): eta nx*ny, M (nx+1)*ny, N nx*(ny+1).  Synchronises. */
int rti_get_state(rti_domain *dom, int32_t level, double *eta, double *M, double *N);

/* Overwrite the state of one level (NULL skips a field).  The maxima are not
 * touched (rti_set_max does that), nor is the step count. */
int rti_set_state(rti_domain *dom, int32_t level, const double *eta, const double *M, const double *N);

/* Overwrite the maxima of one level (host, nx*ny). */
int rti_set_max(rti_domain *dom, int32_t level, const double *zmax);

/* Steps taken since the initial condition. */
int rti_steps_done(const rti_domain *dom, int64_t *steps);

/* Wait for every step enqueued on the domain's stream, then read the
 * domain's sticky device checks: RTI_EDIVERGED (and the domain is marked
 * diverged: further steps are refused) once any step wrote a non-finite
 * water level or flux (the fused kernel checks every value it writes, every
 * step), RTI_EINTERNAL if an active-tile list ever overflowed (a broken
 * invariant: each tile is listed at most once per step). */
int rti_sync(rti_domain *dom);

/* The sticky device checks without failing on them (synchronises):
 * *bits = RTI_STATUS_DIVERGED | RTI_STATUS_LIST_OVERFLOW as set. */
#define RTI_STATUS_DIVERGED 0x1u
#define RTI_STATUS_LIST_OVERFLOW 0x2u
int rti_device_status(rti_domain *dom, uint32_t *bits);

/* Time the kernels of nsteps steps launched one by one with HIP events on
 * the domain's stream (this advances the state).  ms[k] receives the average
 * duration of kernel kind k per launch, names[k] (may be NULL) a static
 * name; at most cap kinds; *n_kinds the number filled; *active_cells (may be
 * NULL) the average number of cells in the tiles computed per step.
 * Synchronises. */
int rti_profile(rti_domain *dom, int64_t nsteps, double *ms, const char **names, int32_t cap,
                int32_t *n_kinds, double *active_cells);

/* Tiles computed in the last step (not skipped as stationary), all
 * tiles, and the cells inside the computed tiles.  Before the first step every
 * tile counts as computed.  Synchronises. */
int rti_active_tiles(rti_domain *dom, int64_t *active, int64_t *total, int64_t *active_cells);

/* Cell-updates of the steps this domain took through its own launches
 * (rti_step, rti_run, rti_profile; not through a batch): *all counts every
 * cell of every level at every step, *computed only the cells of the tiles
 * the fused kernel computed (stationary tiles skipped).  Synchronises. */
int rti_cell_updates(rti_domain *dom, int64_t *all, int64_t *computed);

/* Step graphs this domain has launched, per kind (see rti_step): counts[0]
 * both kernels as an eager step, counts[1] the fused kernel alone (after
 * many active tiles).  For observability; does not synchronise. */
int rti_graph_launches(const rti_domain *dom, int64_t counts[2]);

/* Tile shape of the fused kernel.  A tile is 60 columns wide and `rows` rows
 * high, rows in [RTI_TILE_ROWS_MIN, RTI_TILE_ROWS_MAX] (default
 * RTI_TILE_ROWS_DEFAULT).  The tile shape changes only the work decomposition:
 * results are bitwise the same for every height.  Setting it synchronises,
 * rebuilds the tile tables and forgets the stationarity history (the next two
 * steps compute every tile). */
#define RTI_TILE_ROWS_MIN 4
#define RTI_TILE_ROWS_MAX 64
#define RTI_TILE_ROWS_DEFAULT 12
int rti_domain_set_tile_rows(rti_domain *dom, int32_t rows);
int rti_domain_tile_rows(const rti_domain *dom, int32_t *rows);

/* Autotuner of the tile shape: for each candidate height (4, 5, 6, 8, 10, 12,
 * 16, 24), run 2 untimed steps and then nsteps timed steps from the domain's
 * current state with every tile computed (so the choice does not depend on how
 * much of the state is stationary at the time), keep the shortest height whose
 * time is within 1 % of the fastest (runs skip stationary tiles, at a finer
 * grain with shorter tiles), and restore the state, the maxima and the step
 * count exactly as they were.
 * nsteps >= 1.  *rows_out (may be NULL) receives the height chosen; ms_out
 * (may be NULL) the average time [ms] of a step computing every tile at that
 * height.  Allocates a device snapshot of the state for the
 * duration of the call; synchronises. */
int rti_domain_autotune(rti_domain *dom, int32_t nsteps, int32_t *rows_out, double *ms_out);

/* rti_domain_autotune for callers that cannot allocate device memory (tight
 * serving loops that tune each arriving request, harnesses that forbid
 * hipMalloc): the same trials and the same exact restore, but the state
 * snapshot is staged in a static device array of RTI_AUTOTUNE_NOALLOC_MAX_BYTES
 * that the library holds on each GPU it runs on until the process ends, and
 * no hipMalloc, hipFree or other allocating routine is called (the timing
 * events are the domain's own, made by rti_domain_create).  RTI_ENOMEM,
 * before anything runs, when the domain's state is larger than the array.
 * Every call on one GPU shares that GPU's array, whose contents the next
 * call overwrites: calls that overlap on one GPU (from several threads, or on
 * several streams) race and must not be made. */
#define RTI_AUTOTUNE_NOALLOC_MAX_BYTES (128u << 20)
int rti_domain_autotune_noalloc(rti_domain *dom, int32_t nsteps, int32_t *rows_out, double *ms_out);

/* Free the domain's device memory (when the library allocated it), its
 * graphs and the handle.  NULL is a no-op.  Synchronises first.  A domain
 * still in a batch is removed from it first. */
void rti_domain_destroy(rti_domain *dom);

/* ---------------------------------------------------------------------------
 * Batches: several domains stepped together, one active-tile launch and one
 * fused launch per step over a global table of every member's tiles (uneven
 * sizes, level counts and tile heights mixed).  Each member keeps its own
 * state, parity and maxima; a member's results are bitwise the ones it gets
 * stepped alone.  Members must share the device and the precision, may not
 * use RTI_FLAG_PHASED, and belong to at most one batch.  Every batch kernel
 * runs on hip_stream (borrowed).  A member created on another stream is
 * adopted: rti_batch_add waits for the work queued on that stream, and while
 * the domain is in the batch all of its calls run on the batch's stream; it
 * returns to its own stream when it leaves.  While a domain is in a batch it is stepped
 * only through the batch (rti_step and rti_run on it return RTI_ESTATE);
 * reading its state, maxima and step count works as usual.  Members may be
 * added and removed between batch steps (continuous batching: a member added
 * later simply starts from its own state).  flags: RTI_FLAG_NO_GRAPH,
 * RTI_FLAG_NO_ACTIVE, RTI_FLAG_PERSISTENT. */
typedef struct rti_batch rti_batch;     /* opaque */

int rti_batch_create(rti_domain *const *members, int32_t n, void *hip_stream, uint32_t flags, rti_batch **out);
int rti_batch_add(rti_batch *batch, rti_domain *dom);
int rti_batch_remove(rti_batch *batch, rti_domain *dom);
int rti_batch_size(const rti_batch *batch, int32_t *n);

/* Enqueue nsteps steps of every member (asynchronous). */
int rti_batch_step(rti_batch *batch, int64_t nsteps);
int rti_batch_sync(rti_batch *batch);

/* Time nsteps batch steps launched one by one (advances every member):
 * average fused-kernel and active-list-kernel durations per launch [ms] and
 * the average number of cells in the tiles computed per step.  Synchronises. */
int rti_batch_profile(rti_batch *batch, int64_t nsteps, double *fused_ms, double *active_ms, double *active_cells);

/* Cell-updates of every batch step since the batch was created (as
 * rti_cell_updates, summed over the members).  Synchronises. */
int rti_batch_cell_updates(rti_batch *batch, int64_t *all, int64_t *computed);

/* Free the batch's tables and graphs; the members stay valid (and can be
 * stepped alone again).  NULL is a no-op.  Synchronises first. */
void rti_batch_destroy(rti_batch *batch);

/* Diagnostic: the FP64 operations the step is built from, applied element by
 * element, so that a test can compare them with IEEE binary64 (the step's
 * FP64 results are bitwise reproducible only because each of them is
 * correctly rounded).  op: RTI_PROBE_CBRT, the cube root of the Manning term
 * (Eqs. 2-3: D^(-7/3) = (1/D)^2 cbrt(1/D)), defined for positive normal x;
 * RTI_PROBE_RECIP, the reciprocal 1/x of a face depth, defined for x in
 * [2^-767, 2^1022) (every face depth of a step lies there); RTI_PROBE_SQRT,
 * the square root.  x and y are device arrays of n doubles (y may alias x); the
 * kernel is enqueued on hip_stream (borrowed, NULL = default stream) and the
 * call returns without waiting.  RTI_EINVAL for an unknown op, n < 0 or a NULL
 * array with n > 0. */
enum { RTI_PROBE_CBRT = 0, RTI_PROBE_RECIP = 1, RTI_PROBE_SQRT = 2 };
int rti_math_probe(int32_t op, const double *x, double *y, int64_t n, void *hip_stream);

/* Diagnostic: the HBM rate a plain stream reaches on this GPU, as the
 * practical ceiling for the step's kernels (which move 5 reads and 4 writes
 * of 8 bytes per cell in FP64).  out[j][i] = (j + 1) * sum_k in[k][i] over n
 * doubles; in: `reads` (1..8) device arrays, out: `writes` (0..8) device
 * arrays, none overlapping; host arrays of the device pointers.  Enqueued on
 * hip_stream (borrowed); returns without waiting.  RTI_EINVAL on a bad count,
 * n < 0 or a NULL pointer. */
int rti_stream_probe(const double *const *in, int32_t reads, double *const *out, int32_t writes, int64_t n,
                     void *hip_stream);

const char *rti_last_error(void);
const char *rti_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* RTI_H */

// rti_internal.h -- device-side data layout shared by the host runtime
// (rti_host.cpp) and the kernels (rti_kernels.hip, rti_fused.hip).  Not part
// of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define RTI_MAX_LEVELS_DEV 128

// Tile of the fused kernel: one wavefront of 64 lanes covers 64 columns and
// writes the middle RTI_TW of them (2 columns of halo on the left, 2 on the
// right); it streams up DomainDev::th output rows (plus 3 rows of pipeline
// warm-up).  Short tiles give many wavefronts and skip dry or still water
// finely; tall tiles recompute fewer warm-up rows.  RTI_TH rows, the default,
// measured best on gfx950 with RTI_PD = 2 over whole runs of the nested
// workloads (6 to 12 rows within 5 %).  The height is a per-domain setting between
// RTI_TH_MIN (the 3x3 tile neighbourhood of the skip rule must cover the
// stencil's reach) and RTI_TH_MAX.
#define RTI_TW 60
#ifndef RTI_TH
#define RTI_TH 12
#endif
#define RTI_TH_MIN 4
#define RTI_TH_MAX 64
// Rows of loads the fused kernel keeps in flight ahead of the row it computes,
// and the rows of its rolling window (rows t-2 .. t+RTI_PD).  2 still fits
// 3 wavefronts per SIMD (<= 168 VGPRs); deeper prefetch drops to 2.
#ifndef RTI_PD
#define RTI_PD 2
#endif
#define RTI_NS (RTI_PD + 3)
// Wavefronts per tile in the split kernel of sparse steps (each a band of rows).
#define RTI_SPLIT 4
// Zero rows above the last row of every array (the prefetch reads up to row
// ny + RTI_PD + 2) and below row 0 (the warm-up reads down to row -3).
#define RTI_PAD_TOP (RTI_PD + 3)
#define RTI_PAD_BOTTOM 3

// Numbering of a level's fused-kernel tiles: RTI_TILE_ORDER 0 numbers them
// row by row (x fastest), 1 column by column (y fastest).  The active list
// keeps this order and each XCD takes a contiguous slice of it, so the order
// decides which neighbouring tiles run close together in one L2.
#ifndef RTI_TILE_ORDER
#define RTI_TILE_ORDER 0
#endif
__host__ __device__ inline int tile_index(int tx, int ty, int tiles_x, int tiles_y)
{
    return RTI_TILE_ORDER ? tx * tiles_y + ty : ty * tiles_x + tx;
}
__host__ __device__ inline int tile_x(int tl, int tiles_x, int tiles_y)
{
    return RTI_TILE_ORDER ? tl / tiles_y : tl % tiles_x;
}
__host__ __device__ inline int tile_y(int tl, int tiles_x, int tiles_y)
{
    return RTI_TILE_ORDER ? tl % tiles_y : tl / tiles_x;
}

// Root side kinds of DomainDev::bc (the values of RTI_BC_OPEN / RTI_BC_WALL).
#define RTI_BC_OPEN_DEV 0

// Static per-tile bits (host-computed whenever the tile grid is laid out).
#define TI_PINNED 0x1u      // never skipped and never reported stationary
#define TI_CHILD 0x2u       // the tile's extended region meets a child's ring or edge faces
#define TI_EDGE 0x4u        // the tile's extended region meets the level's outer faces
#define TI_DEPS 0x8u        // tiles of other levels (DomainDev::dep) must be stationary too before a skip

// One level on the device.  Every field of a level shares one row pitch P
// (a multiple of 32 elements, >= nx + 64): cell (i,j), x-face (i,j) and
// y-face (i,j) all live at element i + P*j of their array, counted from the
// array's base pointer.  Each array is a zeroed allocation of
// P x (RTI_PAD_BOTTOM + ny + RTI_PAD_TOP) elements whose base pointer is
// RTI_PAD_BOTTOM rows and 2 columns in, so columns -2 .. P-3 and rows
// -RTI_PAD_BOTTOM .. ny + RTI_PAD_TOP - 1 can be read and hold 0 outside the
// level.  eta and the
// fluxes are double-buffered; buffer b of a step is read, buffer b^1 written.
// eta is always FP64; h, the maxima and the fluxes are FP64, or FP32 when the
// domain runs in FP32-bulk precision (DomainDev::bulk32).
struct LevelDev {
    int32_t nx, ny, pitch;
    int32_t parent, off_i, off_j;
    int32_t tiles_x, tiles_y, tile_base;   // tile grid of the fused kernel and its first global tile
    int32_t s_tiles_x, s_tile_base;        // 64x4 tile grid of the per-phase kernels
    int32_t first_child, n_children;       // children are levels first_child .. (listed in child[])
    int32_t masked;                        // 1: some cells of the rectangle are outside the level (touching
                                           // blocks held as one level); its edge fluxes come from the
                                           // injection list (DomainDev::inject), not from inject_edges
    double r, gr;                          // dt/dx and g*dt/dx
    double *eta[2];
    void *h, *zmax, *M[2], *N[2];          // element type: double, or float when bulk32
    // Levels with children: per cell, laid out like eta, the child-to-parent
    // mean of the current step on the cells of the children's rings (written
    // by the active-list kernel before the fused kernel reads it), NaN on every
    // other cell and where no child cell of the block is wet.  nullptr otherwise.
    double *ring;
};

struct DomainDev {
    int32_t nlev;
    int32_t th;                            // output rows of a fused-kernel tile
    int32_t ntiles;                        // fused-kernel tiles over all levels
    int32_t s_ntiles;                      // per-phase-kernel tiles over all levels
    int32_t bc[4];
    int32_t bulk32;                        // 1: h, maxima, M, N stored and the momentum computed in FP32
    int32_t max_ring, max_edge;            // longest child ring (parent cells) and child edge (faces)
    int32_t split_max;                     // steps with at most this many active tiles run k_fused_split (0: never)
    double eps, fc, g;                     // dry threshold, dt/2 g n^2, gravity
    const uint8_t *tinfo;                  // ntiles static bits (TI_*)
    uint8_t *tflag;                        // ntiles: bit0 stationary in the last step (nothing it writes changed), bit1 in the one before
    int32_t *list;                         // ntiles: active tiles of the current step
    int32_t *lmeta;                        // ntiles: level of each listed tile (written with the list)
    int32_t *count;                        // [b] number of active tiles of a step reading buffer b
    int32_t *status;                       // sticky device checks: [0] a non-finite level or flux was
                                           // written, [1] an active-tile list would have overflowed
    const int32_t *tcells;                 // ntiles: cells of the level inside each tile
    unsigned long long *cells_done;        // per active-list workgroup: cells of the computed tiles, summed over the steps
    const LevelDev *lv;                    // nlev levels (blocks of a resolution): device table
    const int32_t *child;                  // level indices grouped by parent: lv[p].first_child indexes here
    const uint8_t *tlev;                   // ntiles: level of each fused-kernel tile
    const uint8_t *slev;                   // s_ntiles: level of each per-phase tile
    const int32_t *dep_off;                // ntiles + 1: tile g's coupled tiles are dep[dep_off[g] .. dep_off[g+1])
    const int32_t *dep;                    // tiles of a parent or child level a tile's step reads through the nest
    const uint32_t *tcmask;                // ntiles: bit q = child q of the tile's level has edge faces in its output
    int32_t nring;                         // ring cells of all children
    const int32_t *ring_cells;             // nring x 2: child level | parent level << 16, (J << 16) | I of ring cell (I, J)
    int32_t ninject;                       // parent faces on the boundary of masked children
    const int32_t *inject;                 // ninject x 4: child level | parent level << 16, 0 (x-face) or 1 (y-face),
                                           // element offset of the first of the 3 child faces, of the parent face
};

// Reads of the level table and the per-tile level indices go through the
// constant address space: the table is read-only during a step and the
// indices used are wavefront-uniform, so these become scalar loads.
typedef const __attribute__((address_space(4))) LevelDev ConstLevelDev;
typedef const __attribute__((address_space(4))) int32_t ConstI32;
typedef const __attribute__((address_space(4))) uint8_t ConstU8;
__device__ __forceinline__ const LevelDev &level_of(const DomainDev &d, int l)
{
    return *(const LevelDev *)&((ConstLevelDev *)d.lv)[l];
}
__device__ __forceinline__ int child_level(const DomainDev &d, int k) { return ((ConstI32 *)d.child)[k]; }
__device__ __forceinline__ int level_of_tile(const DomainDev &d, int g) { return ((ConstU8 *)d.tlev)[g]; }
__device__ __forceinline__ int level_of_stile(const DomainDev &d, int s) { return ((ConstU8 *)d.slev)[s]; }

// A batch of domains stepped together: member m's tiles are global tiles
// base[m] .. base[m+1]-1 of one table, and its state buffer at step parity
// flip is par[m] ^ flip.
struct BatchDev {
    const DomainDev *doms;                 // n members (device copy of each DomainDev)
    const int32_t *base;                   // n + 1 entries
    const uint16_t *tdom;                  // ntiles: member of each global tile
    const uint8_t *par;                    // n
    int32_t n, ntiles;
    int32_t *list;                         // ntiles: active global tiles of the current step
    int32_t *lmeta;                        // ntiles: level << 16 | member of each listed tile (written with the list)
    int32_t *count;                        // [flip]
    int32_t *status;                       // [1]: the global active-tile list would have overflowed (sticky)
    unsigned long long *cells_done;        // per active-list workgroup: cells of the computed tiles of all members
    int32_t nring;                         // ring cells of all members
    const int32_t *rbase;                  // n + 1: member m's ring cells are global ring cells rbase[m] .. rbase[m+1]-1
    const uint16_t *rdom;                  // nring: member of each global ring cell
};

// Parameters of the initial state of one level: the level's origin and
// spacing, and the source (shape -1: none, the lake at rest; 0 Gaussian;
// 1 cos^2 ellipse), its rotation given as cos/sin.
struct InitSource {
    double ox, oy, dx;
    double xc, yc, a, b, ct, st, amp;
    int32_t shape;
};

// Kernel kinds (for profiling).
enum {
    K_MASS = 0, K_JNZ, K_MOMENTUM, K_JNQ, K_FUSED, K_ACTIVE, K_FINITE, K_NKINDS
};

// Launchers; all enqueue on stream and return the launch status.
hipError_t launch_mass(const DomainDev &d, int b, hipStream_t s);
hipError_t launch_jnz(const DomainDev &d, int b, hipStream_t s);
hipError_t launch_momentum(const DomainDev &d, int b, hipStream_t s);
hipError_t launch_jnq(const DomainDev &d, int b, hipStream_t s);
// The new parent fluxes on the boundary of masked children (DomainDev::inject),
// after the step's momentum: buffer b^1 of the parent into buffer b^1 of the child.
hipError_t launch_inject(const DomainDev &d, int b, hipStream_t s);
hipError_t launch_finite_check(const DomainDev &d, int b, int *flag, hipStream_t s);
hipError_t launch_zero_int(int *p, int n, hipStream_t s);
hipError_t launch_init_level(const LevelDev &L, int bulk32, const InitSource &sp, hipStream_t s);
// Also computes the ring means of the step (LevelDev::ring).
hipError_t launch_active(const DomainDev &d, int b, int all_active, hipStream_t s);
// every_tile: the step's list holds every tile (RTI_FLAG_NO_ACTIVE, the autotuner's trials).
hipError_t launch_fused(const DomainDev &d, int b, int grid, hipStream_t s, bool every_tile);
hipError_t launch_active_batch(const BatchDev &bd, int flip, int all_active, int bulk32, hipStream_t s);
hipError_t launch_fused_batch(const BatchDev &bd, int flip, int bulk32, int grid, hipStream_t s);
hipError_t launch_probe_math(int op, const double *x, double *y, int64_t n, hipStream_t s);
hipError_t launch_stream_probe(const double *const *in, int reads, double *const *out, int writes, int64_t n,
                               int grid, hipStream_t s);

// rti_internal.h -- device-side data layout shared by the host runtime
// (rti_host.cpp) and the kernels (rti_kernels.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define RTI_MAX_LEVELS_DEV 16

// One level on the device.  Every field of a level shares one row pitch P
// (a multiple of 32 doubles, >= nx + 1): cell (i,j), x-face (i,j) and
// y-face (i,j) all live at element i + P*j of their array.  eta and the
// fluxes are double-buffered; buffer b of a step is read, buffer b^1 written.
struct LevelDev {
    int32_t nx, ny, pitch;
    int32_t parent, off_i, off_j;
    int32_t tiles_x, tiles_y, tile_base;   // tile grid of the fused kernel and its first global tile
    int32_t s_tiles_x, s_tile_base;        // 64x4 tile grid of the per-phase kernels
    int32_t has_children;
    double r, gr;                          // dt/dx and g*dt/dx
    double *h, *zmax;
    double *eta[2], *M[2], *N[2];
    uint8_t *flag;                         // per tile: bit0 quiescent after the step just done, bit1 the step before, bit2 pinned active
};

struct DomainDev {
    int32_t nlev;
    int32_t ntiles;                        // fused-kernel tiles over all levels
    int32_t s_ntiles;                      // per-phase-kernel tiles over all levels
    int32_t bc[4];
    double eps, fc, g;                     // dry threshold, dt/2 g n^2, gravity
    LevelDev lv[RTI_MAX_LEVELS_DEV];
};

// Tile of the fused kernel: TW output columns, TH output rows.
#define RTI_TW 60
#define RTI_TH 32

// Kernel kinds (for profiling).
enum {
    K_MASS = 0, K_JNZ, K_MOMENTUM, K_JNQ, K_FUSED, K_ACTIVE, K_FINITE, K_NKINDS
};

// Launchers (rti_kernels.hip); all enqueue on stream and return the launch status.
hipError_t launch_mass(const DomainDev &d, int b, hipStream_t s);
hipError_t launch_jnz(const DomainDev &d, int b, hipStream_t s);
hipError_t launch_momentum(const DomainDev &d, int b, hipStream_t s);
hipError_t launch_jnq(const DomainDev &d, int b, hipStream_t s);
hipError_t launch_finite_check(const DomainDev &d, int b, int *flag, hipStream_t s);
hipError_t launch_zero_int(int *p, int n, hipStream_t s);

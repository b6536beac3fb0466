// rti_runtime.h -- host-side internals shared by the domain runtime
// (rti_host.cpp) and the batch runtime (rti_batch.cpp).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "rti.h"
#include "rti_internal.h"

namespace rti_rt {

// Records the message of the calling thread's last failure; returns code.
int fail(int code, const char *fmt, ...);

#define HIP_TRY(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::rti_rt::fail(RTI_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kGraphSteps = 20;   // steps per captured graph (even: parity returns)
// Kinds of step graphs: both fused and split launches, as an eager step
// (default); the fused kernel alone, computing every listed tile (runs of
// dense steps).
enum { kGraphDefault = 0, kGraphDense = 1, kGraphKinds = 2 };

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct LevelPlan {
    int nx, ny, pitch, parent, off_i, off_j;
    double dx, ox, oy;
    size_t eta_bytes;                       // one pitched FP64 cell array (eta)
    size_t cells_bytes, xf_bytes, yf_bytes; // one pitched array of h/maxima, M, N in the bulk precision
    int tiles_x, tiles_y, s_tiles_x, s_tiles_y;
    // Masked level (touching blocks held as one level): inside[i + nx*j] = 1 for
    // the cells of the level, cover[I + (nx/3)*J] = 1 for the parent cells it
    // covers (their 3x3 cells inside).  Both empty for a rectangular level.
    std::vector<uint8_t> inside, cover;
    int64_t cells = 0;                      // cells inside the level
};

// Depth stored on the device for cells outside a masked level: ground far
// above any water level, so every face touching such a cell is dry (Eq. (1)
// then keeps its level exactly at -h: its neighbours' fluxes are far below
// the rounding of that level).  The host reads such cells back as 0.
constexpr double kOutsideDepth = -1e30;

struct Plan {
    std::vector<LevelPlan> lv;
    std::vector<uint8_t> tinfo;   // static bits per fused-kernel tile (TI_*)
    std::vector<int32_t> tcells;  // cells of the level inside each tile
    std::vector<uint8_t> tlev;    // level of each fused-kernel tile
    std::vector<uint8_t> slev;    // level of each per-phase tile
    std::vector<int32_t> dep_off; // ntiles + 1 offsets into dep
    std::vector<int32_t> dep;     // per tile: the tiles of other levels its step reads through the nest
    std::vector<uint32_t> tcmask; // per tile: children (bit = index among the level's children, first 32)
                                  // whose edge faces lie in the tile's output rows and columns
    size_t dep_cap = 0;           // device entries reserved for dep (a tile whose list does not fit is pinned)
    std::vector<int32_t> ring;    // 2 per ring cell of every child: child level | parent level << 16, (J << 16) | I
    std::vector<int32_t> inject;  // 4 per boundary face of every masked child (DomainDev::inject)
    int64_t cells = 0;            // cells inside the levels
    size_t ring_bytes = 0;        // the parents' ring-mean arrays (one eta-sized array per level with children)
    size_t elem = sizeof(double); // element size of h, maxima, M, N
    size_t level_bytes = 0;       // the level arrays (state, bathymetry, maxima), first in memory
    size_t bytes = 0;
    int ntiles = 0, s_ntiles = 0;
    int ntiles_cap = 0;           // tile tables are sized for the smallest tile height
    int th = RTI_TH;              // tile rows of the fused kernel
};

// Tile grid, static tile bits, per-tile cell counts and coupled tiles of tile
// height th.  Coupled-tile lists are kept within dep_cap entries in all.
void plan_tiles(Plan &plan, int th, size_t dep_cap);

// Workgroups of a fused launch over ntiles tiles: one per tile, or a fixed
// persistent grid of resident wavefronts when that is smaller.
int fused_grid(int ntiles, bool persistent, int cu_count);

}  // namespace rti_rt

struct rti_batch;

struct rti_domain {
    rti_rt::Plan plan;
    DomainDev dev{};
    std::vector<LevelDev> lvh;           // host copy of the level table (dev.lv points at the device copy)
    std::vector<int32_t> childh;         // host copy of the child list
    LevelDev *lv_dev = nullptr;
    int32_t *child_dev = nullptr;
    uint8_t *tlev_dev = nullptr, *slev_dev = nullptr;
    hipStream_t stream = nullptr;        // borrowed (the batch's stream while in a batch)
    hipStream_t home_stream = nullptr;   // the stream given at create, restored on leaving a batch
    hipStream_t capture = nullptr;       // private, for graph capture
    // Step graphs per kind (rti_rt::kGraph*) and starting parity: the same
    // steps with the fused and split launches shaped for the coming steps.
    hipGraph_t graph[rti_rt::kGraphKinds][2] = {};
    hipGraphExec_t exec[rti_rt::kGraphKinds][2] = {};
    int *hint = nullptr;                 // pinned host memory: the active tiles of the last graph's last step
    int hint_age = 0;                    // graphs since the hint was last refreshed
    int64_t graph_launches[rti_rt::kGraphKinds] = {};   // graphs launched per kind
    hipEvent_t tev[2] = {nullptr, nullptr};   // timing events of the autotuner, made at create
    void *mem = nullptr;                 // base of the carved memory
    bool owns_mem = false;
    int *ctrl = nullptr;                 // [0..1] active tile counts per step parity, [2] divergence flag
    uint8_t *tinfo = nullptr;
    int32_t *tcells = nullptr;
    int32_t *dep_off_dev = nullptr, *dep_dev = nullptr;
    uint32_t *tcmask_dev = nullptr;
    int32_t *ring_dev = nullptr;         // the ring-cell list (Plan::ring)
    int32_t *inject_dev = nullptr;       // the masked children's boundary faces (Plan::inject)
    char *ring_mem = nullptr;            // start of the parents' ring-mean arrays (ring_bytes)
    int cur = 0;                         // buffer holding the current state
    int64_t steps = 0;
    int64_t own_steps = 0;               // steps taken by this domain's own launches (not through a batch)
    uint32_t flags = 0;
    double dt = 0.0;
    bool diverged = false;
    int device = 0;
    int cu_count = 256;
    uint64_t gen = 0;                    // bumped whenever dev or the tile tables change
    int64_t tiles_step = 0;              // step count when the tile tables were last rebuilt
    rti_batch *batch = nullptr;          // the batch this domain belongs to
};

namespace rti_rt {
// Used by the batch runtime.
int forget_quiet(rti_domain *D);
// The sticky device checks (after the stream drained): RTI_EINTERNAL on a list
// overflow, RTI_EDIVERGED (and the domain marked diverged) on a non-finite value.
int check_status(rti_domain *D);
// Zero both active-tile counters.  A step's list is appended at its parity's
// counter, which the step before resets; whenever a domain's parity moves
// without its own steps (batch steps, autotune restore) the counters are
// zeroed so no stale count survives.
int reset_counts(rti_domain *D);
void batch_forget_member(rti_batch *B, rti_domain *D);   // a member is being destroyed
}  // namespace rti_rt

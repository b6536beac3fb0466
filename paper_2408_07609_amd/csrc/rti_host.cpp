// rti_host.cpp -- host runtime behind the C ABI of include/rti.h: descriptor
// validation (CFL bound Eq. (4) and 3:1 inclusive nesting of Sec. II-A of
// the paper), device memory carving, state transfer, the step driver (HIP
// graphs replaying a fixed number of steps), profiling hooks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rti_runtime.h"

namespace rti_rt {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// Does child level C cover parent cell (I, J) of its footprint (counted from
// its origin)?  A rectangular child covers its whole footprint.
bool covers(const LevelPlan &C, int I, int J)
{
    const int fw = C.nx / 3, fh = C.ny / 3;
    if (I < 0 || J < 0 || I >= fw || J >= fh) return false;
    return C.cover.empty() || C.cover[(size_t)I + (size_t)fw * J] != 0;
}

// A ring cell of child C (Sec. IV-C): a covered parent cell with an uncovered
// one among its 8 neighbours (the outermost ring of a rectangle, corners once).
bool ring_cell(const LevelPlan &C, int I, int J)
{
    if (!covers(C, I, J)) return false;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di)
            if (!covers(C, I + di, J + dj)) return true;
    return false;
}

// Static bits and coupled tiles of every tile.
//
// A tile's extended region (its cells plus the 2-cell halo its stencil reads,
// plus one for safety) decides: TI_EDGE when it reaches within 3 cells of the
// level's outer faces (open sides, injected child edges); TI_CHILD when it
// reaches within 3 parent cells of a child's footprint boundary (ring cells,
// edge faces).
//
// A tile may be skipped only if every input of its step is unchanged over the
// last two steps.  Its 3x3 neighbourhood covers the inputs on its own level.
// Two kinds of input come from other levels (the exchanges of Sec. IV-C), and
// the tiles that write them are listed as its coupled tiles:
//  - a child tile near the child's edge reads edge faces that the parent
//    injects: the parent tiles over the tile's read region;
//  - a parent tile reading the ring means reads the child's 3x3 blocks along
//    the footprint boundary (cells, their faces, the injected edge faces):
//    the child tiles within 4 cells of the child's edge under the tile's read
//    region.
// The read region is taken 4 cells wider than the tile on every side (2 halo
// columns and rows, the faces beyond them, one to spare), so the lists hold
// every writer of those inputs and possibly more.  A tile whose list would
// pass dep_cap is pinned instead: never skipped, never reported stationary.
void plan_tiles(Plan &plan, int th, size_t dep_cap)
{
    plan.th = th;
    const int nlev = (int)plan.lv.size();
    int ntiles = 0;
    std::vector<int> tbase(nlev);
    for (int l = 0; l < nlev; ++l) {
        LevelPlan &p = plan.lv[l];
        // A tile writes the cells of its columns and rows and their left and bottom faces.  The
        // root also writes its last faces (i = nx, j = ny: open sides or walls), so its grid covers
        // them; a child's last faces are injected by its parent, so its grid covers only its cells.
        const int fx = (l == 0) ? 1 : 0;
        p.tiles_x = (p.nx + fx + RTI_TW - 1) / RTI_TW;
        p.tiles_y = (p.ny + fx + th - 1) / th;
        tbase[l] = ntiles;
        ntiles += p.tiles_x * p.tiles_y;
    }
    plan.ntiles = ntiles;
    plan.tinfo.assign(ntiles, 0);
    plan.tcells.assign(ntiles, 0);
    plan.tlev.assign(ntiles, 0);
    plan.dep_off.assign((size_t)ntiles + 1, 0);
    plan.dep.clear();
    plan.tcmask.assign(ntiles, 0u);
    std::vector<int32_t> deps;
    // tiles of level k over cells [i0, i1] x [j0, j1] (inclusive; face indices nx, ny allowed)
    auto add_rect = [&](int k, int i0, int i1, int j0, int j1) {
        const LevelPlan &q = plan.lv[k];
        i0 = std::max(i0, 0); j0 = std::max(j0, 0);
        i1 = std::min(i1, q.nx); j1 = std::min(j1, q.ny);
        if (i0 > i1 || j0 > j1) return;
        // (a child's faces i = nx, j = ny belong to no tile of its own: clip to its last tile)
        for (int ty = j0 / th; ty <= std::min(j1 / th, q.tiles_y - 1); ++ty)
            for (int tx = i0 / RTI_TW; tx <= std::min(i1 / RTI_TW, q.tiles_x - 1); ++tx)
                deps.push_back(tbase[k] + tile_index(tx, ty, q.tiles_x, q.tiles_y));
    };
    for (int l = 0; l < nlev; ++l) {
        const LevelPlan &p = plan.lv[l];
        for (int tl = 0; tl < p.tiles_x * p.tiles_y; ++tl) {   // in tile-number order: lists are appended
            {
                const int tx = tile_x(tl, p.tiles_x, p.tiles_y), ty = tile_y(tl, p.tiles_x, p.tiles_y);
                const int ax = tx * RTI_TW - 3, bx = tx * RTI_TW + RTI_TW + 2;
                const int ay = ty * th - 3, by = ty * th + th + 2;
                // read region, cells and faces
                const int rx0 = tx * RTI_TW - 4, rx1 = tx * RTI_TW + RTI_TW + 3;
                const int ry0 = ty * th - 4, ry1 = ty * th + th + 3;
                uint8_t bits = 0;
                uint32_t cmask = 0;
                int q = 0;   // index of the next child among the level's children (increasing level order)
                deps.clear();
                bool near_edge = ax <= 3 || bx >= p.nx - 4 || ay <= 3 || by >= p.ny - 4;
                if (l > 0 && !near_edge && !p.cover.empty()) {
                    // a masked level's boundary inside the rectangle is injected too: an
                    // uncovered parent cell next to the read region's parent cells
                    const int I0 = std::max(rx0, 0) / 3 - 1, I1 = std::min(rx1, p.nx - 1) / 3 + 1;
                    const int J0 = std::max(ry0, 0) / 3 - 1, J1 = std::min(ry1, p.ny - 1) / 3 + 1;
                    for (int J = J0; J <= J1 && !near_edge; ++J)
                        for (int I = I0; I <= I1 && !near_edge; ++I)
                            if (!covers(p, I, J)) near_edge = true;
                }
                if (near_edge) {
                    bits |= TI_EDGE;
                    if (l > 0) {
                        // parent cells over the read region (edge faces i = nx map to parent face off_i + nx/3),
                        // widened by one parent cell
                        const int i0 = std::max(rx0, 0), i1 = std::min(rx1, p.nx);
                        const int j0 = std::max(ry0, 0), j1 = std::min(ry1, p.ny);
                        add_rect(p.parent, p.off_i + i0 / 3 - 1, p.off_i + i1 / 3 + 1, p.off_j + j0 / 3 - 1,
                                 p.off_j + j1 / 3 + 1);
                    }
                }
                for (int k = l + 1; k < nlev; ++k) {
                    const LevelPlan &C = plan.lv[k];
                    if (C.parent != l) continue;
                    const int fx0 = C.off_i, fx1 = C.off_i + C.nx / 3 - 1;   // footprint, inclusive
                    const int fy0 = C.off_j, fy1 = C.off_j + C.ny / 3 - 1;
                    if (!C.cover.empty()) {
                        // masked child: its edges are injected by k_inject (no cmask bit); the
                        // tile reads ring means where a ring cell lies in its extended region,
                        // and depends on the child tiles of the ring blocks in its read region
                        ++q;
                        const int a = std::max(rx0, fx0), b = std::min(rx1, fx1);
                        const int c = std::max(ry0, fy0), e = std::min(ry1, fy1);
                        for (int t = c; t <= e; ++t)
                            for (int u = a; u <= b; ++u) {
                                const int I = u - fx0, J = t - fy0;
                                if (!ring_cell(C, I, J)) continue;
                                if (u >= ax && u <= bx && t >= ay && t <= by) bits |= TI_CHILD;
                                add_rect(k, 3 * I, 3 * I + 3, 3 * J, 3 * J + 3);
                            }
                        continue;
                    }
                    {
                        // output columns x0 .. x0+59, rows y0 .. y0+th-1: does an edge face of child k lie there?
                        const int ox0 = tx * RTI_TW, ox1 = ox0 + RTI_TW - 1, oy0 = ty * th, oy1 = oy0 + th - 1;
                        const bool cols = ox0 <= fx1 && ox1 >= fx0, rows = oy0 <= fy1 && oy1 >= fy0;
                        const bool xcol = (ox0 <= fx0 && fx0 <= ox1) || (ox0 <= fx1 + 1 && fx1 + 1 <= ox1);
                        const bool yrow = (oy0 <= fy0 && fy0 <= oy1) || (oy0 <= fy1 + 1 && fy1 + 1 <= oy1);
                        if (q < 32 && ((xcol && rows) || (yrow && cols))) cmask |= 1u << q;
                        ++q;
                    }
                    const bool meets_outer = ax <= fx1 + 3 && bx >= fx0 - 3 && ay <= fy1 + 3 && by >= fy0 - 3;
                    const bool inside_inner = ax >= fx0 + 3 && bx <= fx1 - 3 && ay >= fy0 + 3 && by <= fy1 - 3;
                    if (!(meets_outer && !inside_inner)) continue;
                    bits |= TI_CHILD;
                    // footprint cells in the read region -> their 3x3 child blocks and the faces above/right
                    const int a = std::max(rx0, fx0), b = std::min(rx1, fx1);
                    const int c = std::max(ry0, fy0), e = std::min(ry1, fy1);
                    if (a > b || c > e) continue;
                    const int ci0 = 3 * (a - fx0), ci1 = 3 * (b - fx0) + 3;
                    const int cj0 = 3 * (c - fy0), cj1 = 3 * (e - fy0) + 3;
                    // only the blocks of ring cells are read: the 4-cell strips along the child's edges
                    add_rect(k, ci0, std::min(ci1, 3), cj0, cj1);
                    add_rect(k, std::max(ci0, C.nx - 3), ci1, cj0, cj1);
                    add_rect(k, ci0, ci1, cj0, std::min(cj1, 3));
                    add_rect(k, ci0, ci1, std::max(cj0, C.ny - 3), cj1);
                }
                const int g = tbase[l] + tl;
                std::sort(deps.begin(), deps.end());
                deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
                if (!deps.empty()) {
                    if (plan.dep.size() + deps.size() <= dep_cap) {
                        bits |= TI_DEPS;
                        plan.dep.insert(plan.dep.end(), deps.begin(), deps.end());
                    } else {
                        bits |= TI_PINNED;
                    }
                }
                plan.tinfo[g] = bits;
                plan.tcmask[g] = cmask;
                plan.tlev[g] = (uint8_t)l;
                const int w = std::min(RTI_TW, p.nx - tx * RTI_TW), hgt = std::min(th, p.ny - ty * th);
                if (p.inside.empty()) {
                    plan.tcells[g] = std::max(0, w) * std::max(0, hgt);
                } else {
                    int n = 0;
                    for (int j = ty * th; j < ty * th + hgt; ++j)
                        for (int i = tx * RTI_TW; i < tx * RTI_TW + w; ++i) n += p.inside[(size_t)i + (size_t)p.nx * j];
                    plan.tcells[g] = n;
                }
                plan.dep_off[(size_t)g + 1] = (int32_t)plan.dep.size();
            }
        }
    }
}

int fused_grid(int ntiles, bool persistent, int cu_count)
{
    int grid = (ntiles + 7) / 8 * 8;
    if (persistent) {
        // 3 wavefronts per SIMD, 4 SIMDs per compute unit (the fused kernel's occupancy)
        const int resident = std::max(8, cu_count * 12 / 8 * 8);
        grid = std::min(grid, resident);
    }
    return std::max(grid, 8);
}

}  // namespace rti_rt

using namespace rti_rt;

static_assert(RTI_MAX_LEVELS <= RTI_MAX_LEVELS_DEV && RTI_MAX_LEVELS <= 256, "level indices are stored in 8 bits");
static_assert(RTI_TH == RTI_TILE_ROWS_DEFAULT && RTI_TH_MIN == RTI_TILE_ROWS_MIN && RTI_TH_MAX == RTI_TILE_ROWS_MAX,
              "tile heights of the ABI and the kernels disagree");

namespace {

// Cells whose (2r+1) x (2r+1) neighbourhood lies inside the grid and inside
// `in` (an nx x ny 0/1 map).
std::vector<uint8_t> erode(const std::vector<uint8_t> &in, int nx, int ny, int r)
{
    std::vector<uint8_t> rows(in.size(), 0), out(in.size(), 0);
    std::vector<int> pre((size_t)std::max(nx, ny) + 1);
    for (int j = 0; j < ny; ++j) {
        pre[0] = 0;
        for (int i = 0; i < nx; ++i) pre[i + 1] = pre[i] + (in[(size_t)i + (size_t)nx * j] != 0);
        for (int i = r; i + r < nx; ++i) rows[(size_t)i + (size_t)nx * j] = (pre[i + r + 1] - pre[i - r] == 2 * r + 1);
    }
    for (int i = 0; i < nx; ++i) {
        pre[0] = 0;
        for (int j = 0; j < ny; ++j) pre[j + 1] = pre[j] + rows[(size_t)i + (size_t)nx * j];
        for (int j = r; j + r < ny; ++j) out[(size_t)i + (size_t)nx * j] = (pre[j + r + 1] - pre[j - r] == 2 * r + 1);
    }
    return out;
}

// Validate the descriptor and lay the domain out in device memory.
int plan_domain(const rti_domain_desc *d, Plan &plan)
{
    if (!d) return fail(RTI_EINVAL, "descriptor is NULL");
    if (d->n_levels < 1 || d->n_levels > RTI_MAX_LEVELS)
        return fail(RTI_EINVAL, "n_levels %d outside [1, %d]", d->n_levels, RTI_MAX_LEVELS);
    if (!d->levels) return fail(RTI_EINVAL, "levels is NULL");
    if (!(d->dt > 0.0) || !(d->dx0 > 0.0) || !(d->g > 0.0) || !(d->manning_n >= 0.0) || !(d->dry_eps >= 1e-12)
        || !std::isfinite(d->dt) || !std::isfinite(d->dx0) || !std::isfinite(d->x0) || !std::isfinite(d->y0))
        return fail(RTI_EINVAL, "dt, dx0, g must be positive and finite, dry_eps >= 1e-12, manning_n >= 0");
    for (int s = 0; s < 4; ++s)
        if (d->bc[s] != RTI_BC_OPEN && d->bc[s] != RTI_BC_WALL) return fail(RTI_EINVAL, "bc[%d] = %d", s, d->bc[s]);
    if (d->precision != RTI_FP64 && d->precision != RTI_FP32_BULK)
        return fail(RTI_EINVAL, "precision %d unknown", d->precision);
    if (d->precision == RTI_FP32_BULK && (d->flags & RTI_FLAG_PHASED))
        return fail(RTI_EINVAL, "the per-phase kernels are FP64 only");
    plan.elem = (d->precision == RTI_FP32_BULK) ? sizeof(float) : sizeof(double);
    if (d->flags & ~(RTI_FLAG_NO_GRAPH | RTI_FLAG_NO_ACTIVE | RTI_FLAG_PHASED | RTI_FLAG_PERSISTENT))
        return fail(RTI_EINVAL, "unknown flags 0x%x", d->flags);

    plan.lv.assign(d->n_levels, LevelPlan{});
    for (int k = 0; k < d->n_levels; ++k) {
        const rti_level_desc &L = d->levels[k];
        LevelPlan &p = plan.lv[k];
        if (!L.h) return fail(RTI_EINVAL, "level %d: h is NULL", k);
        if (L.nx < 3 || L.ny < 3) return fail(RTI_EINVAL, "level %d: %d x %d cells (at least 3 x 3)", k, L.nx, L.ny);
        p.nx = L.nx; p.ny = L.ny; p.parent = L.parent; p.off_i = L.off_i; p.off_j = L.off_j;
        if (k == 0) {
            if (L.parent != -1) return fail(RTI_ENEST, "level 0 must be the root (parent -1)");
            p.dx = d->dx0; p.ox = d->x0; p.oy = d->y0;
        } else {
            if (L.parent < 0 || L.parent >= k) return fail(RTI_ENEST, "level %d: parent %d must precede it", k, L.parent);
            const LevelPlan &P = plan.lv[L.parent];
            if (L.nx % 3 || L.ny % 3 || L.nx < 9 || L.ny < 9)
                return fail(RTI_ENEST, "level %d: %d x %d cells, need multiples of 3 and >= 9 (ratio 3)", k, L.nx, L.ny);
            if (L.off_i < 3 || L.off_j < 3 || L.off_i + L.nx / 3 > P.nx - 3 || L.off_j + L.ny / 3 > P.ny - 3)
                return fail(RTI_ENEST, "level %d: footprint [%d,%d)x[%d,%d) not inside parent %d with 3 cells of margin",
                            k, L.off_i, L.off_i + L.nx / 3, L.off_j, L.off_j + L.ny / 3, L.parent);
            p.dx = P.dx / 3.0;
            p.ox = P.ox + (double)L.off_i * P.dx;
            p.oy = P.oy + (double)L.off_j * P.dx;
        }
        p.cells = (int64_t)L.nx * L.ny;
        if (L.mask) {
            // touching blocks of one resolution held as one level (Sec. II-A, Table 1)
            if (k == 0) return fail(RTI_ENEST, "level 0 (the root) cannot have a mask");
            const int fw = L.nx / 3, fh = L.ny / 3;
            p.inside.assign((size_t)L.nx * L.ny, 0);
            p.cover.assign((size_t)fw * fh, 0);
            int64_t covered = 0;
            for (int J = 0; J < fh; ++J)
                for (int I = 0; I < fw; ++I) {
                    const uint8_t v = L.mask[(size_t)3 * I + (size_t)L.nx * (3 * J)];
                    if (v > 1) return fail(RTI_EINVAL, "level %d: mask values must be 0 or 1", k);
                    for (int jj = 3 * J; jj < 3 * J + 3; ++jj)
                        for (int ii = 3 * I; ii < 3 * I + 3; ++ii) {
                            const size_t c = (size_t)ii + (size_t)L.nx * jj;
                            if (L.mask[c] != v)
                                return fail(RTI_ENEST, "level %d: mask not constant over the 3x3 cells of parent cell (%d, %d)",
                                            k, L.off_i + I, L.off_j + J);
                            p.inside[c] = v;
                        }
                    p.cover[(size_t)I + (size_t)fw * J] = v;
                    covered += v;
                }
            if (covered == 0) return fail(RTI_ENEST, "level %d: the mask covers no parent cell", k);
            p.cells = 9 * covered;
        }
        // Zero-padded layout (see LevelDev): pitch >= nx + 64, RTI_PAD_BOTTOM + ny + RTI_PAD_TOP rows.
        const long long rows = (long long)RTI_PAD_BOTTOM + L.ny + RTI_PAD_TOP;
        const long long pitch = (long long)align_up((size_t)L.nx + 64, 32);
        if (pitch * rows * 8 >= (1LL << 31)) return fail(RTI_EINVAL, "level %d too large", k);
        p.pitch = (int)pitch;
        p.eta_bytes = align_up((size_t)pitch * (size_t)rows * sizeof(double), kAlign);
        p.cells_bytes = align_up((size_t)pitch * (size_t)rows * plan.elem, kAlign);
        p.xf_bytes = p.cells_bytes;
        p.yf_bytes = p.cells_bytes;
    }
    for (int a = 1; a < d->n_levels; ++a) {
        for (int b = a + 1; b < d->n_levels; ++b) {
            const rti_level_desc &A = d->levels[a], &B = d->levels[b];
            if (A.parent != B.parent) continue;
            const bool apart = A.off_i + A.nx / 3 + 3 <= B.off_i || B.off_i + B.nx / 3 + 3 <= A.off_i
                            || A.off_j + A.ny / 3 + 3 <= B.off_j || B.off_j + B.ny / 3 + 3 <= A.off_j;
            if (!apart) return fail(RTI_ENEST, "levels %d and %d: sibling footprints closer than 3 parent cells", a, b);
        }
    }
    // A child of a masked level keeps 3 parent cells away from the cells outside it.
    {
        std::vector<std::vector<uint8_t>> core(d->n_levels);
        for (int k = 1; k < d->n_levels; ++k) {
            const LevelPlan &C = plan.lv[k];
            const LevelPlan &P = plan.lv[C.parent];
            if (P.inside.empty()) continue;
            std::vector<uint8_t> &pc = core[C.parent];
            if (pc.empty()) pc = erode(P.inside, P.nx, P.ny, 3);
            for (int J = 0; J < C.ny / 3; ++J)
                for (int I = 0; I < C.nx / 3; ++I)
                    if (covers(C, I, J) && !pc[(size_t)(C.off_i + I) + (size_t)P.nx * (C.off_j + J)])
                        return fail(RTI_ENEST, "level %d: parent cell (%d, %d) it covers lies within 3 cells of a cell "
                                    "outside its masked parent %d", k, C.off_i + I, C.off_j + J, C.parent);
        }
    }
    // Eq. (4): dx / dt >= sqrt(2 g h_max) on every level (over the cells inside it).
    plan.cells = 0;
    for (int k = 0; k < d->n_levels; ++k) {
        const rti_level_desc &L = d->levels[k];
        const std::vector<uint8_t> &in = plan.lv[k].inside;
        plan.cells += plan.lv[k].cells;
        double hmax = 0.0;
        const size_t n = (size_t)L.nx * (size_t)L.ny;
        for (size_t c = 0; c < n; ++c) {
            if (!in.empty() && !in[c]) continue;
            const double h = L.h[c];
            if (!std::isfinite(h)) return fail(RTI_EINVAL, "level %d: non-finite depth at cell %zu", k, c);
            hmax = std::max(hmax, h);
        }
        const double lim = std::sqrt(2.0 * d->g * hmax);
        if (plan.lv[k].dx / d->dt < lim)
            return fail(RTI_ECFL, "level %d: dx/dt = %.3f m/s < sqrt(2 g h_max) = %.3f m/s (h_max %.1f m)", k,
                        plan.lv[k].dx / d->dt, lim, hmax);
    }
    // Tiles and bytes.
    size_t bytes = 0;
    int s_ntiles = 0;
    for (auto &p : plan.lv) {
        p.s_tiles_x = (p.nx + 63) / 64;
        p.s_tiles_y = (p.ny + 3) / 4;
        s_ntiles += p.s_tiles_x * p.s_tiles_y;
        // eta x2 (FP64); h, zmax, M x2, N x2 (bulk precision)
        bytes += 2 * p.eta_bytes + 2 * p.cells_bytes + 2 * p.xf_bytes + 2 * p.yf_bytes;
    }
    plan.level_bytes = bytes;
    // Ring cells of every child (Sec. IV-C: covered parent cells next to an uncovered one; the
    // outermost ring of a rectangular footprint), and one ring-mean array, laid out like eta, per
    // level with children.  The boundary faces of every masked child: parent faces between a
    // covered and an uncovered parent cell, whose flux the child's 3 faces there receive.
    plan.ring.clear();
    plan.inject.clear();
    plan.ring_bytes = 0;
    std::vector<char> has_children(plan.lv.size(), 0);
    for (int k = 1; k < (int)plan.lv.size(); ++k) {
        const LevelPlan &C = plan.lv[k];
        const LevelPlan &P = plan.lv[C.parent];
        const int fw = C.nx / 3, fh = C.ny / 3;
        if (fw > 65535 || fh > 32767) return fail(RTI_EINVAL, "level %d: footprint %d x %d too large", k, fw, fh);
        has_children[C.parent] = 1;
        for (int J = 0; J < fh; ++J)
            for (int I = 0; I < fw; ++I)
                if (ring_cell(C, I, J)) {
                    plan.ring.push_back(k | (C.parent << 16));
                    plan.ring.push_back((J << 16) | I);
                }
        if (C.cover.empty()) continue;
        for (int J = 0; J < fh; ++J)             // x-faces between parent cells (I-1, J) and (I, J)
            for (int I = 0; I <= fw; ++I)
                if (covers(C, I - 1, J) != covers(C, I, J)) {
                    plan.inject.push_back(k | (C.parent << 16));
                    plan.inject.push_back(0);
                    plan.inject.push_back(3 * I + C.pitch * (3 * J));
                    plan.inject.push_back((C.off_i + I) + P.pitch * (C.off_j + J));
                }
        for (int J = 0; J <= fh; ++J)            // y-faces between parent cells (I, J-1) and (I, J)
            for (int I = 0; I < fw; ++I)
                if (covers(C, I, J - 1) != covers(C, I, J)) {
                    plan.inject.push_back(k | (C.parent << 16));
                    plan.inject.push_back(1);
                    plan.inject.push_back(3 * I + C.pitch * (3 * J));
                    plan.inject.push_back((C.off_i + I) + P.pitch * (C.off_j + J));
                }
    }
    for (int l = 0; l < (int)plan.lv.size(); ++l)
        if (has_children[l]) plan.ring_bytes += plan.lv[l].eta_bytes;
    bytes += plan.ring_bytes + align_up(sizeof(int32_t) * std::max<size_t>(plan.ring.size(), 1), kAlign)
             + align_up(sizeof(int32_t) * std::max<size_t>(plan.inject.size(), 4), kAlign);
    plan.slev.clear();
    for (int k = 0; k < (int)plan.lv.size(); ++k)
        plan.slev.insert(plan.slev.end(), (size_t)plan.lv[k].s_tiles_x * plan.lv[k].s_tiles_y, (uint8_t)k);
    plan_tiles(plan, RTI_TH_MIN, SIZE_MAX);   // the most tiles any height gives
    const int cap = plan.ntiles;
    // coupled-tile entries: the larger of the smallest and the default height's (other heights
    // give about as many or fewer; a tile whose list would not fit is pinned)
    size_t dep_cap = plan.dep.size();
    plan_tiles(plan, RTI_TH, SIZE_MAX);
    dep_cap = std::max(dep_cap, plan.dep.size());
    // tile info, tile flags, active list and its levels, tile cells, control block (counts, divergence flag),
    // computed-cell sums (one per active-list workgroup)
    bytes += 2 * align_up((size_t)cap, kAlign) + 3 * align_up((size_t)cap * 4, kAlign) + kAlign
             + align_up(sizeof(unsigned long long) * (size_t)((cap + 255) / 256), kAlign);
    // level table, child list, tile levels, per-phase tile levels
    bytes += align_up(sizeof(LevelDev) * plan.lv.size(), kAlign) + align_up(sizeof(int32_t) * plan.lv.size(), kAlign)
             + align_up((size_t)cap, kAlign) + align_up((size_t)s_ntiles, kAlign);
    // coupled-tile offsets and lists, child masks
    bytes += align_up(sizeof(int32_t) * ((size_t)cap + 1), kAlign) + align_up(sizeof(int32_t) * std::max<size_t>(dep_cap, 1), kAlign)
             + align_up(sizeof(uint32_t) * (size_t)cap, kAlign);
    plan.bytes = bytes;
    plan.ntiles_cap = cap;
    plan.s_ntiles = s_ntiles;
    plan.dep_cap = dep_cap;
    return RTI_OK;
}

}  // namespace

namespace {

int carve(rti_domain *D)
{
    char *p = static_cast<char *>(D->mem);
    auto take = [&p](size_t n) { char *q = p; p += n; return q; };
    for (int k = 0; k < (int)D->plan.lv.size(); ++k) {
        const LevelPlan &pl = D->plan.lv[k];
        LevelDev &L = D->lvh[k];
        // base pointer = cell (0,0): RTI_PAD_BOTTOM padding rows and 2 padding columns in
        const size_t in = (size_t)RTI_PAD_BOTTOM * pl.pitch + 2;
        auto based = [&](size_t bytes, size_t elem) { return take(bytes) + in * elem; };
        L.eta[0] = reinterpret_cast<double *>(based(pl.eta_bytes, sizeof(double)));
        L.eta[1] = reinterpret_cast<double *>(based(pl.eta_bytes, sizeof(double)));
        L.h = based(pl.cells_bytes, D->plan.elem);
        L.zmax = based(pl.cells_bytes, D->plan.elem);
        L.M[0] = based(pl.xf_bytes, D->plan.elem);
        L.M[1] = based(pl.xf_bytes, D->plan.elem);
        L.N[0] = based(pl.yf_bytes, D->plan.elem);
        L.N[1] = based(pl.yf_bytes, D->plan.elem);
    }
    // ring-mean arrays of the levels with children (after the level arrays: not part of the state)
    D->ring_mem = p;
    for (int k = 0; k < (int)D->plan.lv.size(); ++k) D->lvh[k].ring = nullptr;
    for (int k = 1; k < (int)D->plan.lv.size(); ++k) {
        const int par = D->plan.lv[k].parent;
        if (D->lvh[par].ring) continue;
        const LevelPlan &pl = D->plan.lv[par];
        const size_t in = (size_t)RTI_PAD_BOTTOM * pl.pitch + 2;
        D->lvh[par].ring = reinterpret_cast<double *>(take(pl.eta_bytes)) + in;
    }
    D->ring_dev = reinterpret_cast<int32_t *>(take(align_up(sizeof(int32_t) * std::max<size_t>(D->plan.ring.size(), 1), kAlign)));
    D->dev.ring_cells = D->ring_dev;
    D->dev.nring = (int32_t)(D->plan.ring.size() / 2);
    D->inject_dev = reinterpret_cast<int32_t *>(
        take(align_up(sizeof(int32_t) * std::max<size_t>(D->plan.inject.size(), 4), kAlign)));
    D->dev.inject = D->inject_dev;
    D->dev.ninject = (int32_t)(D->plan.inject.size() / 4);
    const size_t nt = (size_t)D->plan.ntiles_cap;
    D->tinfo = reinterpret_cast<uint8_t *>(take(align_up(nt, kAlign)));
    D->dev.tinfo = D->tinfo;
    D->dev.tflag = reinterpret_cast<uint8_t *>(take(align_up(nt, kAlign)));
    D->dev.list = reinterpret_cast<int32_t *>(take(align_up(nt * 4, kAlign)));
    D->dev.lmeta = reinterpret_cast<int32_t *>(take(align_up(nt * 4, kAlign)));
    D->tcells = reinterpret_cast<int32_t *>(take(align_up(nt * 4, kAlign)));
    D->dev.tcells = D->tcells;
    D->ctrl = reinterpret_cast<int *>(take(kAlign));
    D->dev.count = D->ctrl;         // ctrl[0..1]: active tiles per step parity
    D->dev.status = D->ctrl + 2;    // ctrl[2]: non-finite value written, ctrl[3]: list overflow (both sticky)
    D->dev.cells_done = reinterpret_cast<unsigned long long *>(
        take(align_up(sizeof(unsigned long long) * ((nt + 255) / 256), kAlign)));
    const size_t nl = D->plan.lv.size();
    D->lv_dev = reinterpret_cast<LevelDev *>(take(align_up(sizeof(LevelDev) * nl, kAlign)));
    D->child_dev = reinterpret_cast<int32_t *>(take(align_up(sizeof(int32_t) * nl, kAlign)));
    D->tlev_dev = reinterpret_cast<uint8_t *>(take(align_up(nt, kAlign)));
    D->slev_dev = reinterpret_cast<uint8_t *>(take(align_up((size_t)D->plan.s_ntiles, kAlign)));
    D->dep_off_dev = reinterpret_cast<int32_t *>(take(align_up(sizeof(int32_t) * (nt + 1), kAlign)));
    D->dep_dev = reinterpret_cast<int32_t *>(take(align_up(sizeof(int32_t) * std::max<size_t>(D->plan.dep_cap, 1), kAlign)));
    D->dev.dep_off = D->dep_off_dev;
    D->dev.dep = D->dep_dev;
    D->tcmask_dev = reinterpret_cast<uint32_t *>(take(align_up(sizeof(uint32_t) * nt, kAlign)));
    D->dev.tcmask = D->tcmask_dev;
    D->dev.lv = D->lv_dev;
    D->dev.child = D->child_dev;
    D->dev.tlev = D->tlev_dev;
    D->dev.slev = D->slev_dev;
    return RTI_OK;
}

// Pitched copies between packed host rows (width w) and device rows.
int put_rows(rti_domain *D, double *dst, int pitch, const double *src, int w, int rows)
{
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)pitch * sizeof(double), src, (size_t)w * sizeof(double),
                             (size_t)w * sizeof(double), rows, hipMemcpyHostToDevice, D->stream));
    return RTI_OK;
}

int get_rows(rti_domain *D, double *dst, int w, const double *src, int pitch, int rows)
{
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)w * sizeof(double), src, (size_t)pitch * sizeof(double),
                             (size_t)w * sizeof(double), rows, hipMemcpyDeviceToHost, D->stream));
    return RTI_OK;
}

// The same for arrays in the bulk precision (h, maxima, M, N): FP64 host rows
// are converted to FP32 on the host first when the domain runs FP32-bulk.
int put_rows_b(rti_domain *D, void *dst, int pitch, const double *src, int w, int rows)
{
    if (D->plan.elem == sizeof(double)) return put_rows(D, static_cast<double *>(dst), pitch, src, w, rows);
    std::vector<float> tmp((size_t)w * rows);
    for (size_t k = 0; k < tmp.size(); ++k) tmp[k] = (float)src[k];
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)pitch * sizeof(float), tmp.data(), (size_t)w * sizeof(float),
                             (size_t)w * sizeof(float), rows, hipMemcpyHostToDevice, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));
    return RTI_OK;
}

int get_rows_b(rti_domain *D, double *dst, int w, const void *src, int pitch, int rows)
{
    if (D->plan.elem == sizeof(double)) return get_rows(D, dst, w, static_cast<const double *>(src), pitch, rows);
    std::vector<float> tmp((size_t)w * rows);
    HIP_TRY(hipMemcpy2DAsync(tmp.data(), (size_t)w * sizeof(float), src, (size_t)pitch * sizeof(float),
                             (size_t)w * sizeof(float), rows, hipMemcpyDeviceToHost, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));
    for (size_t k = 0; k < tmp.size(); ++k) dst[k] = (double)tmp[k];
    return RTI_OK;
}

int check_level(const rti_domain *D, int level)
{
    if (!D) return fail(RTI_EINVAL, "domain is NULL");
    if (level < 0 || level >= D->dev.nlev) return fail(RTI_EINVAL, "level %d outside [0, %d)", level, D->dev.nlev);
    return RTI_OK;
}

}  // namespace

// Any host-side change of the state forgets the stationarity history, so the
// next two steps compute every tile.
int rti_rt::forget_quiet(rti_domain *D)
{
    HIP_TRY(hipMemsetAsync(D->dev.tflag, 0, (size_t)D->plan.ntiles, D->stream));
    if (D->hint) *D->hint = -1;          // every tile is listed next: no sparse graph
    return RTI_OK;
}

// The sticky device checks, read after the stream has drained: a list
// overflow is an internal error; a non-finite value marks the domain diverged.
int rti_rt::check_status(rti_domain *D)
{
    int st[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(st, D->dev.status, sizeof st, hipMemcpyDeviceToHost, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));
    if (st[1]) return fail(RTI_EINTERNAL, "an active-tile list overflowed on the device");
    if (st[0]) {
        D->diverged = true;
        return fail(RTI_EDIVERGED, "non-finite water level or flux after %lld steps", (long long)D->steps);
    }
    return RTI_OK;
}

int rti_rt::reset_counts(rti_domain *D)
{
    HIP_TRY(hipMemsetAsync(D->ctrl, 0, 2 * sizeof(int), D->stream));
    return RTI_OK;
}

namespace {

// Initial water level of a level (host, packed) -> both eta buffers; zero
// fluxes; maxima at the initial values.  eta is clipped to the ground.
int install_initial(rti_domain *D, int k, const double *h, std::vector<double> &eta)
{
    const LevelPlan &p = D->plan.lv[k];
    LevelDev &L = D->lvh[k];
    const size_t n = (size_t)p.nx * p.ny;
    std::vector<double> z(n);
    for (size_t c = 0; c < n; ++c) {
        if (h[c] + eta[c] < 0.0) eta[c] = -h[c];
        z[c] = (h[c] > 0.0) ? eta[c] : h[c] + eta[c];
    }
    for (int b = 0; b < 2; ++b) {
        int rc = put_rows(D, L.eta[b], p.pitch, eta.data(), p.nx, p.ny);
        if (rc) return rc;
        // whole padded allocations (their base pointers are RTI_PAD_BOTTOM rows + 2 columns in)
        const size_t in = ((size_t)RTI_PAD_BOTTOM * p.pitch + 2) * D->plan.elem;
        HIP_TRY(hipMemsetAsync(static_cast<char *>(L.M[b]) - in, 0, p.xf_bytes, D->stream));
        HIP_TRY(hipMemsetAsync(static_cast<char *>(L.N[b]) - in, 0, p.yf_bytes, D->stream));
    }
    int rc = put_rows_b(D, L.zmax, p.pitch, z.data(), p.nx, p.ny);
    if (rc) return rc;
    if ((rc = forget_quiet(D))) return rc;
    HIP_TRY(hipStreamSynchronize(D->stream));   // host vectors die on return
    return RTI_OK;
}

// Initial state of level k computed on the device from the depth already
// there: the lake at rest (src NULL) or the lake plus the source; fluxes zero.
// Asynchronous on the domain's stream.
int device_initial(rti_domain *D, int k, const rti_source *src)
{
    const LevelPlan &p = D->plan.lv[k];
    LevelDev &L = D->lvh[k];
    InitSource sp{};
    sp.ox = p.ox;
    sp.oy = p.oy;
    sp.dx = p.dx;
    sp.shape = -1;
    if (src) {
        sp.xc = src->xc;
        sp.yc = src->yc;
        sp.a = src->a;
        sp.b = src->b;
        sp.ct = std::cos(src->theta);
        sp.st = std::sin(src->theta);
        sp.amp = src->amp;
        sp.shape = src->shape;
    }
    const size_t in = ((size_t)RTI_PAD_BOTTOM * p.pitch + 2) * D->plan.elem;
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipMemsetAsync(static_cast<char *>(L.M[b]) - in, 0, p.xf_bytes, D->stream));
        HIP_TRY(hipMemsetAsync(static_cast<char *>(L.N[b]) - in, 0, p.yf_bytes, D->stream));
    }
    // The depth was just uploaded from pageable host memory and the fluxes
    // cleared; the kernel that reads them and the calls after it wait for
    // that explicitly instead of relying on the order of the stream (seen to
    // break when a profiler intercepts the runtime).
    HIP_TRY(hipStreamSynchronize(D->stream));
    HIP_TRY(launch_init_level(L, D->dev.bulk32, sp, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));
    return RTI_OK;
}

// every_tile: compute every tile this step whatever the domain's flags.
// kind: the step-graph kind (kGraph*, rti_runtime.h) being captured; eager
// steps are kGraphDefault.
int launch_step(rti_domain *D, int b, hipStream_t s, bool every_tile = false, int kind = kGraphDefault)
{
    if (D->flags & RTI_FLAG_PHASED) {
        HIP_TRY(launch_mass(D->dev, b, s));
        HIP_TRY(launch_jnz(D->dev, b, s));
        HIP_TRY(launch_momentum(D->dev, b, s));
        HIP_TRY(launch_jnq(D->dev, b, s));
    } else {
        const bool all = every_tile || (D->flags & RTI_FLAG_NO_ACTIVE);
        HIP_TRY(launch_active(D->dev, b, all ? 1 : 0, s));
        // kGraphDense: the fused kernel is told there is no split kernel (split_max 0 in its copy of
        // the descriptor), so it computes every listed tile, however few, and no split launch follows
        DomainDev dv = D->dev;
        if (kind == kGraphDense) dv.split_max = 0;
        HIP_TRY(launch_fused(dv, b, fused_grid(D->dev.ntiles, (D->flags & RTI_FLAG_PERSISTENT) != 0, D->cu_count), s,
                             all));
    }
    HIP_TRY(launch_inject(D->dev, b, s));
    return RTI_OK;
}

// The kind of the next graph, from the active tiles of the last graph's last
// step: more than twice the split kernel's share of tiles, and the coming
// steps will most likely all be fused-kernel steps, so the split kernel,
// which would return at once, is left out (kGraphDense); otherwise, or with
// no count yet, both kernels as in an eager step.  The count is a hint only:
// it is read without synchronising and lags the graphs already enqueued (by
// many graphs when the host runs ahead), and a fused kernel with no split
// share computes every listed tile, so a stale count costs time, never
// results.  (The active-tile count rarely falls during a forecast, so a
// stale large count is rarely wrong.  A kind for sparse steps, the fused
// kernel on the small looping grid, was dropped: the count grows, so a stale
// small one put runs of dense steps on that grid.)
int graph_kind(const rti_domain *D)
{
    if (!D->hint || D->dev.split_max <= 0 || (D->flags & (RTI_FLAG_NO_ACTIVE | RTI_FLAG_PERSISTENT)))
        return kGraphDefault;
    const int n = __atomic_load_n(D->hint, __ATOMIC_RELAXED);
    return n > 2 * D->dev.split_max ? kGraphDense : kGraphDefault;
}

// Cells inside the tiles of the current active list (synchronises).
int active_cells(rti_domain *D, int64_t *tiles, int64_t *cells)
{
    if (D->flags & RTI_FLAG_PHASED) {
        *tiles = D->dev.s_ntiles;
        *cells = D->plan.cells;
        return RTI_OK;
    }
    int n = 0;
    // the last step read buffer cur^1, so its list was counted in ctrl[cur^1]
    HIP_TRY(hipMemcpyAsync(&n, D->ctrl + (D->cur ^ 1), sizeof(int), hipMemcpyDeviceToHost, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));
    const bool fresh = D->steps == D->tiles_step;   // no step since the tile tables were built
    if (fresh) n = D->dev.ntiles;
    n = std::min(std::max(n, 0), D->dev.ntiles);   // the list holds at most one entry per tile
    std::vector<int32_t> list(n);
    if (!fresh && n > 0) {
        HIP_TRY(hipMemcpyAsync(list.data(), D->dev.list, sizeof(int32_t) * n, hipMemcpyDeviceToHost, D->stream));
        HIP_TRY(hipStreamSynchronize(D->stream));
    } else {
        for (int g = 0; g < n; ++g) list[g] = g;
    }
    int64_t c = 0;
    for (int g : list) c += D->plan.tcells[g];
    *tiles = n;
    *cells = c;
    return RTI_OK;
}

// The level table, child list and per-tile level indices to the device.
int upload_tables(rti_domain *D)
{
    const size_t nl = D->lvh.size();
    HIP_TRY(hipMemcpyAsync(D->lv_dev, D->lvh.data(), sizeof(LevelDev) * nl, hipMemcpyHostToDevice, D->stream));
    if (!D->childh.empty())
        HIP_TRY(hipMemcpyAsync(D->child_dev, D->childh.data(), sizeof(int32_t) * D->childh.size(),
                               hipMemcpyHostToDevice, D->stream));
    HIP_TRY(hipMemcpyAsync(D->tlev_dev, D->plan.tlev.data(), D->plan.tlev.size(), hipMemcpyHostToDevice, D->stream));
    HIP_TRY(hipMemcpyAsync(D->slev_dev, D->plan.slev.data(), D->plan.slev.size(), hipMemcpyHostToDevice, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));   // the host vectors may change after return
    return RTI_OK;
}

// The fused kernel's tile tables (static bits, cells, coupled tiles) to the device.
int upload_tiles(rti_domain *D)
{
    const Plan &pl = D->plan;
    HIP_TRY(hipMemcpyAsync(D->tinfo, pl.tinfo.data(), pl.tinfo.size(), hipMemcpyHostToDevice, D->stream));
    HIP_TRY(hipMemcpyAsync(D->tcells, pl.tcells.data(), pl.tcells.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           D->stream));
    HIP_TRY(hipMemcpyAsync(D->dep_off_dev, pl.dep_off.data(), pl.dep_off.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, D->stream));
    HIP_TRY(hipMemcpyAsync(D->tcmask_dev, pl.tcmask.data(), pl.tcmask.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           D->stream));
    if (!pl.dep.empty())
        HIP_TRY(hipMemcpyAsync(D->dep_dev, pl.dep.data(), pl.dep.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));   // the host vectors may change after return
    return RTI_OK;
}

void drop_graphs(rti_domain *D)
{
    for (int p = 0; p < 2; ++p) {
        for (int k = 0; k < kGraphKinds; ++k) {
            if (D->exec[k][p]) (void)hipGraphExecDestroy(D->exec[k][p]);
            if (D->graph[k][p]) (void)hipGraphDestroy(D->graph[k][p]);
            D->exec[k][p] = nullptr;
            D->graph[k][p] = nullptr;
        }
    }
}

// Rebuild the fused kernel's tile tables for tile height th (synchronises).
int retile(rti_domain *D, int th)
{
    HIP_TRY(hipStreamSynchronize(D->stream));
    plan_tiles(D->plan, th, D->plan.dep_cap);
    DomainDev &dv = D->dev;
    dv.th = th;
    dv.ntiles = D->plan.ntiles;
    int base = 0;
    for (int k = 0; k < dv.nlev; ++k) {
        const LevelPlan &p = D->plan.lv[k];
        D->lvh[k].tiles_x = p.tiles_x;
        D->lvh[k].tiles_y = p.tiles_y;
        D->lvh[k].tile_base = base;
        base += p.tiles_x * p.tiles_y;
    }
    int rc0 = upload_tables(D);
    if (!rc0) rc0 = upload_tiles(D);
    if (rc0) return rc0;
    int rc = forget_quiet(D);
    if (!rc) rc = reset_counts(D);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(D->stream));
    drop_graphs(D);
    D->tiles_step = D->steps;
    D->gen += 1;
    return RTI_OK;
}

int build_graph(rti_domain *D, int parity, int kind)
{
    if (!D->capture) HIP_TRY(hipStreamCreateWithFlags(&D->capture, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(D->capture, hipStreamCaptureModeThreadLocal));
    int rc = RTI_OK;
    for (int k = 0; k < kGraphSteps && rc == RTI_OK; ++k)
        rc = launch_step(D, (parity + k) & 1, D->capture, false, kind);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(D->capture, &g);
    if (rc != RTI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(RTI_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(RTI_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    D->graph[kind][parity] = g;
    D->exec[kind][parity] = x;
    return RTI_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char *rti_last_error(void) { return rti_rt::g_err.c_str(); }

const char *rti_strerror(int code)
{
    switch (code) {
    case RTI_OK: return "ok";
    case RTI_EINVAL: return "invalid argument";
    case RTI_ENOMEM: return "out of device memory";
    case RTI_EHIP: return "HIP runtime error";
    case RTI_ECFL: return "CFL condition violated";
    case RTI_ENEST: return "nesting rule violated";
    case RTI_ESTATE: return "call not allowed in this state";
    case RTI_EDIVERGED: return "simulation diverged";
    case RTI_EINTERNAL: return "internal device check failed";
    default: return "unknown error";
    }
}

int rti_domain_footprint(const rti_domain_desc *desc, size_t *bytes)
{
    try {
        if (!bytes) return fail(RTI_EINVAL, "bytes is NULL");
        Plan plan;
        int rc = plan_domain(desc, plan);
        if (rc) return rc;
        *bytes = plan.bytes;
        return RTI_OK;
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

// Test hook, not part of the ABI: the fused kernel's tile plan of a
// descriptor at tile height th (host only; no device is touched).  Called
// with null arrays it returns the sizes; the arrays then receive ntiles
// static bits, levels and child masks, ntiles + 1 coupled-tile offsets and
// ndep entries.
int rti_plan_tiles_for_test(const rti_domain_desc *desc, int th, int32_t *ntiles, int32_t *ndep, uint8_t *tinfo,
                            uint8_t *tlev, int32_t *dep_off, int32_t *dep, uint32_t *tcmask)
{
    try {
        if (!ntiles || !ndep) return fail(RTI_EINVAL, "ntiles or ndep is NULL");
        if (th < RTI_TH_MIN || th > RTI_TH_MAX) return fail(RTI_EINVAL, "tile rows %d outside [%d, %d]", th, RTI_TH_MIN, RTI_TH_MAX);
        Plan plan;
        int rc = plan_domain(desc, plan);
        if (rc) return rc;
        plan_tiles(plan, th, plan.dep_cap);
        *ntiles = plan.ntiles;
        *ndep = (int32_t)plan.dep.size();
        if (tinfo) std::memcpy(tinfo, plan.tinfo.data(), plan.tinfo.size());
        if (tlev) std::memcpy(tlev, plan.tlev.data(), plan.tlev.size());
        if (dep_off) std::memcpy(dep_off, plan.dep_off.data(), plan.dep_off.size() * sizeof(int32_t));
        if (dep && !plan.dep.empty()) std::memcpy(dep, plan.dep.data(), plan.dep.size() * sizeof(int32_t));
        if (tcmask) std::memcpy(tcmask, plan.tcmask.data(), plan.tcmask.size() * sizeof(uint32_t));
        return RTI_OK;
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_domain_create(const rti_domain_desc *desc, void *arena, size_t arena_bytes, void *hip_stream,
                      rti_domain **out)
{
    try {
        if (!out) return fail(RTI_EINVAL, "out is NULL");
        *out = nullptr;
        Plan plan;
        int rc = plan_domain(desc, plan);
        if (rc) return rc;
        if (arena && arena_bytes < plan.bytes)
            return fail(RTI_ENOMEM, "arena of %zu bytes is smaller than the footprint %zu", arena_bytes, plan.bytes);
        if (arena && (reinterpret_cast<uintptr_t>(arena) % kAlign))
            return fail(RTI_EINVAL, "arena must be %zu-byte aligned", kAlign);

        rti_domain *D = new rti_domain;
        D->plan = plan;
        D->stream = static_cast<hipStream_t>(hip_stream);
        D->home_stream = D->stream;
        D->flags = desc->flags;
        D->dt = desc->dt;
        hipError_t e = hipGetDevice(&D->device);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&D->cu_count, hipDeviceAttributeMultiprocessorCount, D->device);
        if (e != hipSuccess) {
            delete D;
            return fail(RTI_EHIP, "querying the device failed: %s", hipGetErrorString(e));
        }
        e = hipEventCreate(&D->tev[0]);
        if (e == hipSuccess) e = hipEventCreate(&D->tev[1]);
        if (e == hipSuccess) e = hipHostMalloc((void **)&D->hint, sizeof(int), hipHostMallocDefault);
        if (e != hipSuccess) {
            rti_domain_destroy(D);
            return fail(RTI_EHIP, "creating the timing events or the pinned hint failed: %s", hipGetErrorString(e));
        }
        *D->hint = -1;                   // no hint until a graph has run
        if (arena) {
            D->mem = arena;
        } else {
            e = hipMalloc(&D->mem, plan.bytes);
            if (e != hipSuccess) {
                rti_domain_destroy(D);
                return fail(RTI_ENOMEM, "hipMalloc(%zu) failed: %s", plan.bytes, hipGetErrorString(e));
            }
            D->owns_mem = true;
        }
        DomainDev &dv = D->dev;
        dv.nlev = desc->n_levels;
        dv.th = plan.th;
        dv.ntiles = plan.ntiles;
        dv.s_ntiles = plan.s_ntiles;
        for (int s = 0; s < 4; ++s) dv.bc[s] = desc->bc[s];
        dv.eps = desc->dry_eps;
        dv.bulk32 = (desc->precision == RTI_FP32_BULK) ? 1 : 0;
        // sparse steps (active tiles that fill at most 3 wavefronts per SIMD once split)
        // run the split kernel; the persistent-grid option keeps the one-wavefront tiles
        dv.split_max = (desc->flags & RTI_FLAG_PERSISTENT) ? 0 : 3 * D->cu_count;
        dv.g = desc->g;
        dv.fc = 0.5 * desc->dt * desc->g * desc->manning_n * desc->manning_n;
        D->lvh.assign(dv.nlev, LevelDev{});
        D->childh.assign(dv.nlev, 0);
        int base = 0, sbase = 0;
        for (int k = 0; k < dv.nlev; ++k) {
            const LevelPlan &p = plan.lv[k];
            LevelDev &L = D->lvh[k];
            L.nx = p.nx; L.ny = p.ny; L.pitch = p.pitch;
            L.parent = p.parent; L.off_i = p.off_i; L.off_j = p.off_j;
            L.tiles_x = p.tiles_x; L.tiles_y = p.tiles_y; L.tile_base = base;
            L.s_tiles_x = p.s_tiles_x; L.s_tile_base = sbase;
            base += p.tiles_x * p.tiles_y;
            sbase += p.s_tiles_x * p.s_tiles_y;
            L.r = desc->dt / p.dx;
            L.gr = desc->g * L.r;
            L.masked = p.inside.empty() ? 0 : 1;
        }
        {
            int nc = 0;
            for (int p = 0; p < dv.nlev; ++p) {
                D->lvh[p].first_child = nc;
                D->lvh[p].n_children = 0;
                for (int k = p + 1; k < dv.nlev; ++k) {
                    if (desc->levels[k].parent == p) {
                        D->childh[nc++] = k;
                        D->lvh[p].n_children += 1;
                    }
                }
            }
        }
        for (int c = 1; c < dv.nlev; ++c) {
            const int fw = plan.lv[c].nx / 3, fh = plan.lv[c].ny / 3;
            dv.max_ring = std::max(dv.max_ring, 2 * fw + 2 * (fh - 2));
            dv.max_edge = std::max(dv.max_edge, 2 * plan.lv[c].nx + 2 * plan.lv[c].ny);
        }
        carve(D);
        e = hipMemsetAsync(D->mem, 0, plan.bytes, D->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(D->stream);
        if (e != hipSuccess) {
            rti_domain_destroy(D);
            return fail(RTI_EHIP, "initialising device memory failed: %s", hipGetErrorString(e));
        }
        if ((rc = upload_tiles(D)) || (rc = upload_tables(D))) {
            rti_domain_destroy(D);
            return rc;
        }
        // ring-mean arrays: NaN (all bits set) everywhere; each step overwrites the ring cells
        if (plan.ring_bytes) e = hipMemsetAsync(D->ring_mem, 0xFF, plan.ring_bytes, D->stream);
        if (e == hipSuccess && !plan.ring.empty())
            e = hipMemcpyAsync(D->ring_dev, plan.ring.data(), sizeof(int32_t) * plan.ring.size(), hipMemcpyHostToDevice,
                               D->stream);
        if (e == hipSuccess && !plan.inject.empty())
            e = hipMemcpyAsync(D->inject_dev, plan.inject.data(), sizeof(int32_t) * plan.inject.size(),
                               hipMemcpyHostToDevice, D->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(D->stream);
        if (e != hipSuccess) {
            rti_domain_destroy(D);
            return fail(RTI_EHIP, "initialising the ring tables failed: %s", hipGetErrorString(e));
        }
        for (int k = 0; k < dv.nlev; ++k) {
            const LevelPlan &p = plan.lv[k];
            if (p.inside.empty()) {
                rc = put_rows_b(D, D->lvh[k].h, p.pitch, desc->levels[k].h, p.nx, p.ny);
            } else {
                // cells outside a masked level: dry ground far above the sea (kOutsideDepth)
                std::vector<double> h(desc->levels[k].h, desc->levels[k].h + (size_t)p.nx * p.ny);
                for (size_t c = 0; c < h.size(); ++c)
                    if (!p.inside[c]) h[c] = kOutsideDepth;
                rc = put_rows_b(D, D->lvh[k].h, p.pitch, h.data(), p.nx, p.ny);
                if (!rc) {
                    e = hipStreamSynchronize(D->stream);
                    if (e != hipSuccess) rc = fail(RTI_EHIP, "uploading the depth failed: %s", hipGetErrorString(e));
                }
            }
            if (rc) { rti_domain_destroy(D); return rc; }
            // the lake at rest on the depth as the kernels see it (rounded to FP32 in FP32-bulk)
            rc = device_initial(D, k, nullptr);
            if (rc) { rti_domain_destroy(D); return rc; }
        }
        e = hipStreamSynchronize(D->stream);     // the caller's depth arrays may go once create returns
        if (e != hipSuccess) {
            rti_domain_destroy(D);
            return fail(RTI_EHIP, "initialising the levels failed: %s", hipGetErrorString(e));
        }
        *out = D;
        return RTI_OK;
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_set_source(rti_domain *D, const rti_source *src)
{
    try {
        if (!D || !src) return fail(RTI_EINVAL, "NULL argument");
        if (D->steps != 0) return fail(RTI_ESTATE, "rti_set_source after %lld steps", (long long)D->steps);
        if (src->shape != RTI_GAUSS && src->shape != RTI_COS2_ELLIPSE) return fail(RTI_EINVAL, "shape %d", src->shape);
        if (!(src->a > 0.0) || !(src->b > 0.0) || !std::isfinite(src->amp) || !std::isfinite(src->xc)
            || !std::isfinite(src->yc) || !std::isfinite(src->theta))
            return fail(RTI_EINVAL, "source scales must be positive and values finite");
        HIP_TRY(hipStreamSynchronize(D->stream));
        for (int k = 0; k < D->dev.nlev; ++k) {
            int rc = device_initial(D, k, src);
            if (rc) return rc;
        }
        int rc = forget_quiet(D);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(D->stream));
        D->steps = 0;
        D->diverged = false;
        return RTI_OK;
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_set_eta(rti_domain *D, int32_t level, const double *eta0)
{
    try {
        int rc = check_level(D, level);
        if (rc) return rc;
        if (!eta0) return fail(RTI_EINVAL, "eta0 is NULL");
        if (D->steps != 0) return fail(RTI_ESTATE, "rti_set_eta after %lld steps", (long long)D->steps);
        const LevelPlan &p = D->plan.lv[level];
        const size_t n = (size_t)p.nx * p.ny;
        std::vector<double> h(n), eta(eta0, eta0 + n);
        for (size_t c = 0; c < n; ++c)
            if (!std::isfinite(eta[c])) return fail(RTI_EINVAL, "eta0 not finite at cell %zu", c);
        rc = get_rows_b(D, h.data(), p.nx, D->lvh[level].h, p.pitch, p.ny);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(D->stream));
        return install_initial(D, level, h.data(), eta);
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_step(rti_domain *D, int64_t nsteps)
{
    try {
        if (!D) return fail(RTI_EINVAL, "domain is NULL");
        if (nsteps < 0) return fail(RTI_EINVAL, "nsteps %lld < 0", (long long)nsteps);
        if (D->batch) return fail(RTI_ESTATE, "the domain is in a batch; step the batch");
        if (D->diverged) return fail(RTI_EDIVERGED, "the domain diverged earlier");
        const bool graphs = !(D->flags & RTI_FLAG_NO_GRAPH);
        while (nsteps > 0) {
            if (graphs && nsteps >= kGraphSteps) {
                const int kind = graph_kind(D);
                hipGraphExec_t &x = D->exec[kind][D->cur];
                if (!x) {
                    int rc = build_graph(D, D->cur, kind);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(x, D->stream));
                D->graph_launches[kind] += 1;
                // the active tiles of the graph's last step (parity cur + kGraphSteps - 1), for the next
                // choice: after every graph while the count is small or unknown, after every 16th once it
                // is large (a run rarely falls back to sparse steps, and each copy is a few microseconds)
                if (D->hint) {
                    const int last = __atomic_load_n(D->hint, __ATOMIC_RELAXED);
                    if (last < 0 || last <= 2 * D->dev.split_max || ++D->hint_age >= 16) {
                        HIP_TRY(hipMemcpyAsync(D->hint, D->dev.count + ((D->cur + kGraphSteps - 1) & 1), sizeof(int),
                                               hipMemcpyDeviceToHost, D->stream));
                        D->hint_age = 0;
                    }
                }
                D->steps += kGraphSteps;
                D->own_steps += kGraphSteps;
                nsteps -= kGraphSteps;
            } else {
                int rc = launch_step(D, D->cur, D->stream);
                if (rc) return rc;
                D->cur ^= 1;
                D->steps += 1;
                D->own_steps += 1;
                nsteps -= 1;
            }
        }
        return RTI_OK;
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_math_probe(int32_t op, const double *x, double *y, int64_t n, void *hip_stream)
{
    if (op < RTI_PROBE_CBRT || op > RTI_PROBE_SQRT) return fail(RTI_EINVAL, "probe op %d unknown", op);
    if (n < 0 || n > (int64_t)0x7fffffff * 256) return fail(RTI_EINVAL, "n %lld outside [0, 2^31 * 256)", (long long)n);
    if (n > 0 && (!x || !y)) return fail(RTI_EINVAL, "NULL array");
    HIP_TRY(launch_probe_math(op, x, y, n, static_cast<hipStream_t>(hip_stream)));
    return RTI_OK;
}

int rti_stream_probe(const double *const *in, int32_t reads, double *const *out, int32_t writes, int64_t n,
                     void *hip_stream)
{
    if (reads < 1 || reads > 8 || writes < 0 || writes > 8) return fail(RTI_EINVAL, "reads %d / writes %d", reads, writes);
    if (n < 0) return fail(RTI_EINVAL, "n %lld < 0", (long long)n);
    if (!in || (writes > 0 && !out)) return fail(RTI_EINVAL, "NULL array list");
    for (int k = 0; k < reads; ++k)
        if (!in[k]) return fail(RTI_EINVAL, "input %d is NULL", k);
    for (int k = 0; k < writes; ++k)
        if (!out[k]) return fail(RTI_EINVAL, "output %d is NULL", k);
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t want = (n + 255) / 256;
    const int grid = (int)std::min<int64_t>(want, (int64_t)cus * 16);
    HIP_TRY(launch_stream_probe(in, reads, out, writes, n, std::max(grid, 1), static_cast<hipStream_t>(hip_stream)));
    return RTI_OK;
}

int rti_sync(rti_domain *D)
{
    if (!D) return fail(RTI_EINVAL, "domain is NULL");
    HIP_TRY(hipStreamSynchronize(D->stream));
    return check_status(D);
}

int rti_device_status(rti_domain *D, uint32_t *bits)
{
    if (!D || !bits) return fail(RTI_EINVAL, "NULL argument");
    int st[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(st, D->dev.status, sizeof st, hipMemcpyDeviceToHost, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));
    *bits = (st[0] ? RTI_STATUS_DIVERGED : 0u) | (st[1] ? RTI_STATUS_LIST_OVERFLOW : 0u);
    return RTI_OK;
}

int rti_run(rti_domain *D, double t_end)
{
    if (!D) return fail(RTI_EINVAL, "domain is NULL");
    if (!std::isfinite(t_end) || t_end < 0.0) return fail(RTI_EINVAL, "t_end %g", t_end);
    if (D->batch) return fail(RTI_ESTATE, "the domain is in a batch; step the batch");
    const int64_t target = (int64_t)std::llround(t_end / D->dt);
    if (target > D->steps) {
        int rc = rti_step(D, target - D->steps);
        if (rc) return rc;
    }
    // the fused kernel's watchdog saw every value it wrote; this whole-level
    // pass also covers the per-phase kernels and values set from the host
    HIP_TRY(launch_finite_check(D->dev, D->cur, D->dev.status, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));
    return check_status(D);
}

// Cells outside a masked level read back as 0.
static void zero_outside(const LevelPlan &p, double *a)
{
    if (!a || p.inside.empty()) return;
    for (size_t c = 0; c < p.inside.size(); ++c)
        if (!p.inside[c]) a[c] = 0.0;
}

int rti_max_inundation(rti_domain *D, int32_t level, double *out)
{
    int rc = check_level(D, level);
    if (rc) return rc;
    if (!out) return fail(RTI_EINVAL, "out is NULL");
    const LevelPlan &p = D->plan.lv[level];
    rc = get_rows_b(D, out, p.nx, D->lvh[level].zmax, p.pitch, p.ny);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(D->stream));
    zero_outside(p, out);
    return RTI_OK;
}

int rti_get_state(rti_domain *D, int32_t level, double *eta, double *M, double *N)
{
    int rc = check_level(D, level);
    if (rc) return rc;
    const LevelPlan &p = D->plan.lv[level];
    const LevelDev &L = D->lvh[level];
    if (eta && (rc = get_rows(D, eta, p.nx, L.eta[D->cur], p.pitch, p.ny))) return rc;
    if (M && (rc = get_rows_b(D, M, p.nx + 1, L.M[D->cur], p.pitch, p.ny))) return rc;
    if (N && (rc = get_rows_b(D, N, p.nx, L.N[D->cur], p.pitch, p.ny + 1))) return rc;
    HIP_TRY(hipStreamSynchronize(D->stream));
    zero_outside(p, eta);
    return RTI_OK;
}

int rti_set_state(rti_domain *D, int32_t level, const double *eta, const double *M, const double *N)
{
    int rc = check_level(D, level);
    if (rc) return rc;
    const LevelPlan &p = D->plan.lv[level];
    const LevelDev &L = D->lvh[level];
    std::vector<double> own;
    if (eta && !p.inside.empty()) {
        // cells outside keep the level of their ground (-kOutsideDepth as the device stores it)
        const double out = (D->plan.elem == sizeof(float)) ? -(double)(float)kOutsideDepth : -kOutsideDepth;
        own.assign(eta, eta + (size_t)p.nx * p.ny);
        for (size_t c = 0; c < own.size(); ++c)
            if (!p.inside[c]) own[c] = out;
        eta = own.data();
    }
    for (int b = 0; b < 2; ++b) {
        if (eta && (rc = put_rows(D, L.eta[b], p.pitch, eta, p.nx, p.ny))) return rc;
        if (M && (rc = put_rows_b(D, L.M[b], p.pitch, M, p.nx + 1, p.ny))) return rc;
        if (N && (rc = put_rows_b(D, L.N[b], p.pitch, N, p.nx, p.ny + 1))) return rc;
    }
    if ((rc = forget_quiet(D))) return rc;
    HIP_TRY(hipStreamSynchronize(D->stream));
    D->diverged = false;
    return RTI_OK;
}

int rti_set_max(rti_domain *D, int32_t level, const double *zmax)
{
    int rc = check_level(D, level);
    if (rc) return rc;
    if (!zmax) return fail(RTI_EINVAL, "zmax is NULL");
    const LevelPlan &p = D->plan.lv[level];
    std::vector<double> own;
    if (!p.inside.empty()) {
        own.assign(zmax, zmax + (size_t)p.nx * p.ny);
        zero_outside(p, own.data());
        zmax = own.data();
    }
    if ((rc = put_rows_b(D, D->lvh[level].zmax, p.pitch, zmax, p.nx, p.ny))) return rc;
    if ((rc = forget_quiet(D))) return rc;
    HIP_TRY(hipStreamSynchronize(D->stream));
    return RTI_OK;
}

int rti_steps_done(const rti_domain *D, int64_t *steps)
{
    if (!D || !steps) return fail(RTI_EINVAL, "NULL argument");
    *steps = D->steps;
    return RTI_OK;
}

int rti_profile(rti_domain *D, int64_t nsteps, double *ms, const char **names, int32_t cap, int32_t *n_kinds,
                double *avg_cells)
{
    if (!D || !ms || !n_kinds || cap < 1 || nsteps < 1) return fail(RTI_EINVAL, "bad argument");
    if (D->batch) return fail(RTI_ESTATE, "the domain is in a batch; profile the batch");
    static const char *kNames[K_NKINDS] = {"k_mass", "k_jnz", "k_momentum", "k_jnq", "k_fused", "k_active", "k_finite"};
    double sum[K_NKINDS] = {0};
    int cnt[K_NKINDS] = {0};
    hipEvent_t ev[5];
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    int rc = RTI_OK;
    const bool phased = (D->flags & RTI_FLAG_PHASED) != 0;
    double cell_sum = 0.0;
    for (int64_t s = 0; s < nsteps && rc == RTI_OK; ++s) {
        const int b = D->cur;
        int kinds[4];
        int nk = 0;
        hipError_t e = hipEventRecord(ev[0], D->stream);
        if (phased) {
            if (e == hipSuccess) e = launch_mass(D->dev, b, D->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[1], D->stream);
            if (e == hipSuccess) e = launch_jnz(D->dev, b, D->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[2], D->stream);
            if (e == hipSuccess) e = launch_momentum(D->dev, b, D->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[3], D->stream);
            if (e == hipSuccess) e = launch_jnq(D->dev, b, D->stream);
            if (e == hipSuccess) e = launch_inject(D->dev, b, D->stream);   // masked children (timed as k_jnq)
            if (e == hipSuccess) e = hipEventRecord(ev[4], D->stream);
            kinds[0] = K_MASS; kinds[1] = K_JNZ; kinds[2] = K_MOMENTUM; kinds[3] = K_JNQ;
            nk = 4;
        } else {
            if (e == hipSuccess) e = launch_active(D->dev, b, (D->flags & RTI_FLAG_NO_ACTIVE) ? 1 : 0, D->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[1], D->stream);
            if (e == hipSuccess)
                e = launch_fused(D->dev, b, fused_grid(D->dev.ntiles, (D->flags & RTI_FLAG_PERSISTENT) != 0, D->cu_count),
                                 D->stream, (D->flags & RTI_FLAG_NO_ACTIVE) != 0);
            if (e == hipSuccess) e = launch_inject(D->dev, b, D->stream);   // masked children (timed with k_fused)
            if (e == hipSuccess) e = hipEventRecord(ev[2], D->stream);
            kinds[0] = K_ACTIVE; kinds[1] = K_FUSED;
            nk = 2;
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[nk]);
        if (e != hipSuccess) {
            rc = fail(RTI_EHIP, "profiling step failed: %s", hipGetErrorString(e));
            break;
        }
        for (int q = 0; q < nk; ++q) {
            if ((kinds[q] == K_JNZ || kinds[q] == K_JNQ) && D->dev.nlev < 2) continue;
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, ev[q], ev[q + 1]);
            sum[kinds[q]] += t;
            cnt[kinds[q]] += 1;
        }
        D->cur ^= 1;
        D->steps += 1;
        D->own_steps += 1;
        if (avg_cells) {
            int64_t t = 0, c = 0;
            if ((rc = active_cells(D, &t, &c))) break;
            cell_sum += (double)c;
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
    int n = 0;
    for (int k = 0; k < K_NKINDS && n < cap; ++k) {
        if (!cnt[k]) continue;
        ms[n] = sum[k] / cnt[k];
        if (names) names[n] = kNames[k];
        ++n;
    }
    *n_kinds = n;
    if (avg_cells) *avg_cells = cell_sum / (double)nsteps;
    return RTI_OK;
}

int rti_active_tiles(rti_domain *D, int64_t *active, int64_t *total, int64_t *cells)
{
    if (!D || !active || !total || !cells) return fail(RTI_EINVAL, "NULL argument");
    int rc = active_cells(D, active, cells);
    if (rc) return rc;
    *total = (D->flags & RTI_FLAG_PHASED) ? D->dev.s_ntiles : D->dev.ntiles;
    return RTI_OK;
}

// Sum of the computed-cell slots (synchronises).
int cells_done(rti_domain *D, unsigned long long *out)
{
    std::vector<unsigned long long> part((size_t)(D->plan.ntiles_cap + 255) / 256);
    HIP_TRY(hipMemcpyAsync(part.data(), D->dev.cells_done, sizeof(unsigned long long) * part.size(),
                           hipMemcpyDeviceToHost, D->stream));
    HIP_TRY(hipStreamSynchronize(D->stream));
    unsigned long long t = 0;
    for (auto v : part) t += v;
    *out = t;
    return RTI_OK;
}

int rti_cell_updates(rti_domain *D, int64_t *all, int64_t *computed)
{
    if (!D || !all || !computed) return fail(RTI_EINVAL, "NULL argument");
    const int64_t cells = D->plan.cells;
    unsigned long long done = 0;
    int rc = cells_done(D, &done);
    if (rc) return rc;
    *all = cells * D->own_steps;
    *computed = (D->flags & RTI_FLAG_PHASED) ? *all : (int64_t)done;
    return RTI_OK;
}

int rti_domain_set_tile_rows(rti_domain *D, int32_t rows)
{
    try {
        if (!D) return fail(RTI_EINVAL, "domain is NULL");
        if (rows < RTI_TILE_ROWS_MIN || rows > RTI_TILE_ROWS_MAX)
            return fail(RTI_EINVAL, "tile rows %d outside [%d, %d]", rows, RTI_TILE_ROWS_MIN, RTI_TILE_ROWS_MAX);
        if (rows == D->plan.th) return RTI_OK;
        return retile(D, rows);
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_domain_tile_rows(const rti_domain *D, int32_t *rows)
{
    if (!D || !rows) return fail(RTI_EINVAL, "NULL argument");
    *rows = D->plan.th;
    return RTI_OK;
}

int rti_graph_launches(const rti_domain *D, int64_t counts[2])
{
    if (!D || !counts) return fail(RTI_EINVAL, "NULL argument");
    for (int k = 0; k < kGraphKinds; ++k) counts[k] = D->graph_launches[k];
    return RTI_OK;
}

}  // extern "C"

namespace {

// Staging memory of rti_domain_autotune_noalloc: a file-scope device array,
// so each GPU that loads the library holds its own copy (its own address)
// until the process ends, and that entry point allocates nothing.  In host
// code the symbol is only a stand-in: the device address of this GPU's copy
// comes from hipGetSymbolAddress, taken once per device with the device
// current (noalloc_stage), and only that address is passed to HIP.
__device__ __align__(256) unsigned char scratch[RTI_AUTOTUNE_NOALLOC_MAX_BYTES];

std::mutex g_stage_mu;
void *g_stage[64] = {};            // per device ordinal

int noalloc_stage(int device, void **out)
{
    if (device < 0 || device >= 64) return fail(RTI_EINVAL, "device %d outside [0, 64)", device);
    std::lock_guard<std::mutex> lock(g_stage_mu);
    if (!g_stage[device]) {
        int prev = 0;
        HIP_TRY(hipGetDevice(&prev));
        HIP_TRY(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        (void)hipSetDevice(prev);
        if (e != hipSuccess || !p) return fail(RTI_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_stage[device] = p;
    }
    *out = g_stage[device];
    return RTI_OK;
}

// The autotuner.  stage: device memory of at least level_bytes for the state
// snapshot, or null to allocate it here.
int autotune(rti_domain *D, int32_t nsteps, int32_t *rows_out, double *ms_out, void *stage)
{
    if (!D) return fail(RTI_EINVAL, "domain is NULL");
    if (nsteps < 1) return fail(RTI_EINVAL, "nsteps %d < 1", nsteps);
    if (D->batch) return fail(RTI_ESTATE, "the domain is in a batch");
    if (D->flags & RTI_FLAG_PHASED) return fail(RTI_EINVAL, "the per-phase kernels have no tiles to tune");
    if (D->diverged) return fail(RTI_EDIVERGED, "the domain diverged earlier");
    static const int kCand[] = {4, 5, 6, 8, 10, 12, 16, 24};      // ascending
    constexpr int kNCand = (int)(sizeof kCand / sizeof kCand[0]);
    double cand_ms[kNCand] = {};
    void *snap = stage;
    hipEvent_t *ev = D->tev;
    const int cur0 = D->cur;
    const int64_t steps0 = D->steps;
    std::vector<unsigned long long> done0((size_t)(D->plan.ntiles_cap + 255) / 256);   // the trials do not count
    int best = D->plan.th;
    double best_ms = 0.0;
    int rc = RTI_OK;
    auto restore = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(D->mem, snap, D->plan.level_bytes, hipMemcpyDeviceToDevice, D->stream));
        HIP_TRY(hipMemcpyAsync(D->dev.cells_done, done0.data(), sizeof(unsigned long long) * done0.size(),
                               hipMemcpyHostToDevice, D->stream));
        D->cur = cur0;
        D->steps = steps0;
        int rc2 = forget_quiet(D);
        if (!rc2) rc2 = reset_counts(D);
        if (!rc2 && hipStreamSynchronize(D->stream) != hipSuccess) rc2 = fail(RTI_EHIP, "autotune restore failed");
        return rc2;
    };
    try {
        HIP_TRY(hipMemcpyAsync(done0.data(), D->dev.cells_done, sizeof(unsigned long long) * done0.size(),
                               hipMemcpyDeviceToHost, D->stream));
        HIP_TRY(hipStreamSynchronize(D->stream));
        hipError_t e = hipSuccess;
        if (!stage) {
            e = hipMalloc(&snap, D->plan.level_bytes);
            if (e != hipSuccess)
                return fail(RTI_ENOMEM, "autotune snapshot of %zu bytes: %s", D->plan.level_bytes, hipGetErrorString(e));
        }
        e = hipMemcpyAsync(snap, D->mem, D->plan.level_bytes, hipMemcpyDeviceToDevice, D->stream);
        if (e != hipSuccess) rc = fail(RTI_EHIP, "autotune set-up: %s", hipGetErrorString(e));
        for (int ci = 0; ci < kNCand; ++ci) {
            const int c = kCand[ci];
            if (rc) break;
            if ((rc = retile(D, c)) || (rc = restore())) break;
            // Every tile is computed in the trials: the time then measures the
            // kernel at this height per cell, not how much of the current state
            // happens to be stationary (early in a run, nearly all of it).
            for (int k = 0; k < 2 && !rc; ++k) {      // untimed
                rc = launch_step(D, D->cur, D->stream, true);
                D->cur ^= 1;
                D->steps += 1;
            }
            if (rc) break;
            e = hipEventRecord(ev[0], D->stream);
            for (int k = 0; k < nsteps && !rc && e == hipSuccess; ++k) {
                rc = launch_step(D, D->cur, D->stream, true);
                D->cur ^= 1;
                D->steps += 1;
            }
            if (!rc && e == hipSuccess) e = hipEventRecord(ev[1], D->stream);
            if (!rc && e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float t = 0.0f;
            if (!rc && e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
            if (!rc && e != hipSuccess) rc = fail(RTI_EHIP, "autotune timing: %s", hipGetErrorString(e));
            if (rc) break;
            cand_ms[ci] = (double)t / nsteps;
        }
        if (!rc) {
            // The shortest height within 1 % of the fastest: the trials compute every tile, while a
            // run skips stationary tiles, at a finer grain the shorter the tile, so near-ties go to
            // the shorter one; but a height slower by more than the trials' noise loses over a whole
            // run too (C3: 12 rows 1.3 % slower than 16 in the trials and over the run).
            double fastest = cand_ms[0];
            for (int ci = 1; ci < kNCand; ++ci) fastest = std::min(fastest, cand_ms[ci]);
            for (int ci = 0; ci < kNCand; ++ci)
                if (cand_ms[ci] <= fastest * 1.01) {
                    best = kCand[ci];
                    best_ms = cand_ms[ci];
                    break;
                }
        }
        if (!rc) rc = retile(D, best);
        if (!rc) rc = restore();
        if (!rc) {
            e = hipStreamSynchronize(D->stream);
            if (e != hipSuccess) rc = fail(RTI_EHIP, "autotune restore: %s", hipGetErrorString(e));
        }
    } catch (...) {
        rc = fail(RTI_EINVAL, "unexpected exception");
    }
    if (rc && snap) {
        // leave the domain as it was, whatever failed
        (void)hipStreamSynchronize(D->stream);
        (void)hipMemcpy(D->mem, snap, D->plan.level_bytes, hipMemcpyDeviceToDevice);
        (void)hipMemcpy(D->dev.cells_done, done0.data(), sizeof(unsigned long long) * done0.size(),
                        hipMemcpyHostToDevice);
        D->cur = cur0;
        D->steps = steps0;
        (void)forget_quiet(D);
        (void)reset_counts(D);
        (void)hipStreamSynchronize(D->stream);
    }
    if (snap && !stage) (void)hipFree(snap);
    if (rc) return rc;
    if (rows_out) *rows_out = best;
    if (ms_out) *ms_out = best_ms;
    return RTI_OK;
}

}  // namespace

extern "C" {

int rti_domain_autotune(rti_domain *D, int32_t nsteps, int32_t *rows_out, double *ms_out)
{
    return autotune(D, nsteps, rows_out, ms_out, nullptr);
}

int rti_domain_autotune_noalloc(rti_domain *D, int32_t nsteps, int32_t *rows_out, double *ms_out)
{
    if (!D) return fail(RTI_EINVAL, "domain is NULL");
    if (D->plan.level_bytes > (size_t)RTI_AUTOTUNE_NOALLOC_MAX_BYTES)
        return fail(RTI_ENOMEM, "the domain's state is %zu bytes, above the %zu bytes of the static staging array",
                    D->plan.level_bytes, (size_t)RTI_AUTOTUNE_NOALLOC_MAX_BYTES);
    void *stage = nullptr;
    int rc = noalloc_stage(D->device, &stage);
    if (rc) return rc;
    return autotune(D, nsteps, rows_out, ms_out, stage);
}

void rti_domain_destroy(rti_domain *D)
{
    if (!D) return;
    if (D->batch) batch_forget_member(D->batch, D);
    (void)hipStreamSynchronize(D->stream);
    drop_graphs(D);
    if (D->capture) (void)hipStreamDestroy(D->capture);
    for (auto &x : D->tev)
        if (x) (void)hipEventDestroy(x);
    if (D->hint) (void)hipHostFree(D->hint);
    if (D->owns_mem && D->mem) (void)hipFree(D->mem);
    delete D;
}

}  // extern "C"

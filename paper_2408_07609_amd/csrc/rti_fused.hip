// rti_fused.hip -- the fused time step of the nested long-wave model on
// gfx950, FP64: one launch computes, for every active tile of every level,
// the continuity update (paper Eq. 1), the child-to-parent ring mean (Sec.
// IV-C; precomputed for the step in the active-list launch and read here like
// the water level), the momentum update (Eqs. 2-3) with the wet/dry rule, the root's open
// or wall sides, the injection of the new parent fluxes into the children's
// edge faces, and the running maxima.  State is read from buffer b and the new
// state written to buffer b^1, so every tile may recompute its halo.
//
// Tile = one wavefront, 60 columns by DomainDev::th rows.  Lane L owns
// column c = x0 - 2 + L and the wavefront streams up the rows of the tile:
// iteration t computes the new water level of row t, the face quantities of
// row t (depth, M^2/D, M N/D ...) and the momentum of row t-1, whose up/down
// neighbours are then in registers; left/right neighbours come from the
// adjacent lanes through DPP wavefront shifts.  The raw loads of row t+RTI_PD
// (one coalesced access per field) are issued in iteration t, so RTI_PD rows
// of loads are in flight.  Each face quantity is computed once per tile.  The
// 2 halo lanes on each side and the 3 warm-up rows are recomputed by the
// neighbouring tiles (most of their loads hit L2).  The tile function serves
// the single-domain kernels (one workgroup per tile, or a persistent grid)
// and the batch kernel (tiles of many domains in one launch).
//
// Precision: k_fused<double> is the FP64 step.  k_fused<float> is the
// FP32-bulk step: h, M, N and the maxima are stored in FP32 and the momentum
// is computed in FP32, while the water level eta, the continuity update, the
// total depth at faces, the wet/dry tests and the water-level difference of
// the pressure term stay FP64 (so still water stays still and the level does
// not accumulate FP32 rounding).
//
// Active tiles: before each step k_active lists the tiles to compute.  A tile
// is stationary after a step that left every value it writes (water levels,
// fluxes) bitwise unchanged.  A tile is skipped only when it and its 8
// neighbours were stationary after both of the last two steps, and so were its
// coupled tiles on other levels: near a child's edge, the parent tiles that
// inject its edge fluxes; near a child's footprint boundary, the child tiles
// whose blocks its ring means read.  Then every value its step reads is what
// it read in the step before, so its step is an exact no-op, and both state
// buffers already hold its values (the maxima cannot rise either).  Dry land
// and water still at rest ahead of the wave therefore cost no bandwidth.
#include <type_traits>

#include "rti_device.h"
#include "rti_internal.h"

namespace {
using namespace rti_dev;

// Bitwise equality (tells -0 from +0), for the stationarity test of a tile.
__device__ __forceinline__ bool same_bits(double a, double b) { return __double_as_longlong(a) == __double_as_longlong(b); }
__device__ __forceinline__ bool same_bits(float a, float b) { return __float_as_int(a) == __float_as_int(b); }

// Value held by lane+1 (from_right) or lane-1 (from_left): wavefront-wide DPP
// shifts (wave_shl:1 = 0x130, wave_shr:1 = 0x138); with bound_ctrl set, the
// lane without a source receives 0 (so no old value has to be set up).
// Called only in wave-uniform control flow.
__device__ __forceinline__ int dpp_right_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_left_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }

__device__ __forceinline__ double from_right(double v)
{
    const long long bits = __double_as_longlong(v);
    const int lo = dpp_right_i((int)(bits & 0xffffffffLL));
    const int hi = dpp_right_i((int)(bits >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double from_left(double v)
{
    const long long bits = __double_as_longlong(v);
    const int lo = dpp_left_i((int)(bits & 0xffffffffLL));
    const int hi = dpp_left_i((int)(bits >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_right_i(__float_as_int(v))); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_left_i(__float_as_int(v))); }

// Face quantities of one x-face (or y-face) of a row, in the flux precision F.
template <typename F>
struct FaceQ {
    F D;          // total depth at the face (if active)
    F f;          // the face's own flux (M on x-faces, N on y-faces)
    F cr;         // the cross flux averaged to the face (N on x-faces, M on y-faces)
    F q;          // f^2 / D
    F p;          // f * cr / D
    F fr;         // Manning factor of the face (friction)
    int act;      // face active under the wet/dry rule (and interior)
};

// The wet/dry rule and the depth are evaluated in FP64 on the FP64 levels.
template <typename F, bool Friction = true>
__device__ __forceinline__ FaceQ<F> face_q(bool interior, double ha, double ea, double hb, double eb, double eps,
                                          F f, F cr, F fc)
{
    // Computed on every lane.  An inactive face carries D = 1 (a safe value)
    // and q, p, fr of that D; nothing reads them: neighbours test act first,
    // and the face's own new flux is replaced by 0.
    FaceQ<F> o;
    double D;
    const bool act = face_depth(ha, ea, hb, eb, eps, D) & interior;
    const F Df = act ? (F)D : F(1);
    const F iD = inv_depth(Df);
    o.act = act ? 1 : 0;
    o.D = Df;
    o.f = f;
    o.cr = cr;
    o.q = over_depth(f, f, iD);
    o.p = over_depth(f, cr, iD);
    o.fr = Friction ? friction(fc, f, cr, Df, iD) : F(0);   // only the faces the tile writes need it
    return o;
}

// One row of the fused kernel's rolling window.
template <typename F>
struct RowW {
    double E, H;        // raw eta and h of the row
    F Mx, Ny;           // raw flux of the row's x-face and of its top y-face (j = row + 1)
    F Z;                // maxima of the row before this step
    double e1;          // new eta of the row
    double e1L, HL;     // new eta and h of the cell on the left
    F MxR, NyL;         // x-face flux on the right, top y-face flux on the left
    double R;           // ring mean of the row's cell (NaN: not a ring cell, or none wet)
    FaceQ<F> x, y;      // the row's x-face and bottom y-face (j = row)
};

// New flux of an active face (momentum_update); de is the FP64 water-level
// difference across the face.
template <typename F>
__device__ __forceinline__ F new_flux(const FaceQ<F> &m, double de, F along, F cross, F r, F gr)
{
    return momentum_update(m.f, m.fr, m.D, (F)de, along, cross, r, gr);
}

// Child-to-parent mean of ring cell e of the domain (Sec. IV-C): the mean of
// the wet cells of the child's 3x3 block after their continuity update of this
// step (computed here from the child's buffer b with the continuity
// kernel's operations), summed j outer, i inner, not below the parent's
// ground; NaN when none is wet (the parent cell then keeps its own new
// level).  Written into the parent's ring array, which the fused kernel of
// the same step reads.  Only buffer b is read, so this runs before the fused
// kernel, in the active-list launch.  A mean whose inputs did not change in
// the last step is left as stored.
template <typename F>
__device__ void ring_mean(const DomainDev &d, int b, int e)
{
    const int kp = d.ring_cells[2 * e];                 // child level | parent level << 16
    const int ij = d.ring_cells[2 * e + 1];
    const int I = ij & 0xffff, J = ij >> 16;
    const LevelDev &C = d.lv[kp & 0xffff];
    const LevelDev &P = d.lv[kp >> 16];                 // loaded together with the child's fields
    // The block's inputs are the child cells and faces of [3I, 3I+3] x [3J, 3J+3]
    // (written by at most 2 x 2 child tiles) and the edge faces the parent
    // injects there (written by the parent tiles of (c, t), (c+1, t), (c, t+1)).
    // If every one of these tiles left its outputs unchanged in the last step,
    // the inputs are those of the step the stored mean was computed in (by
    // induction over the steps since), so the stored mean is this step's too.
    {
        const int c = C.off_i + I, t = C.off_j + J, th = d.th;
        const int ci1 = min(3 * I + 3, C.nx - 1), cj1 = min(3 * J + 3, C.ny - 1);
        auto flag = [&](const LevelDev &Q, int i, int j) -> unsigned {
            const int tx = min(i / RTI_TW, Q.tiles_x - 1), ty = min(j / th, Q.tiles_y - 1);
            return (unsigned)d.tflag[Q.tile_base + tile_index(tx, ty, Q.tiles_x, Q.tiles_y)];
        };
        const unsigned acc = flag(C, 3 * I, 3 * J) & flag(C, ci1, 3 * J) & flag(C, 3 * I, cj1) & flag(C, ci1, cj1)
                           & flag(P, c, t) & flag(P, c + 1, t) & flag(P, c, t + 1) & flag(P, c + 1, t + 1);
        if (acc & 1u) return;
    }
    const int CP = C.pitch;
    const double *ce = C.eta[b];
    const F *cm = static_cast<const F *>(C.M[b]), *cn = static_cast<const F *>(C.N[b]);
    const F *ch = static_cast<const F *>(C.h);
    const int pc = (C.off_i + I) + P.pitch * (C.off_j + J);
    const double hpar = (double)static_cast<const F *>(P.h)[pc];
    // The block's 9 water levels and depths, 12 x-faces and 12 y-faces, all
    // loaded before any is used (one wait instead of one per cell).
    const int c0 = 3 * I + CP * (3 * J);
    double E[9], Hc[9];
    F Mx[3][4], Ny[4][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            E[3 * r + q] = ce[c0 + CP * r + q];
            Hc[3 * r + q] = (double)ch[c0 + CP * r + q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Mx[r][q] = cm[c0 + CP * r + q];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) Ny[r][q] = cn[c0 + CP * r + q];
    double s = 0.0;
    int nw = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {          // j outer, i inner
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double ec = E[3 * r + q] - C.r * (((double)Mx[r][q + 1] - (double)Mx[r][q])
                                              + ((double)Ny[r + 1][q] - (double)Ny[r][q]));
            const double hc = Hc[3 * r + q];
            if (hc + ec < 0.0) ec = -hc;
            if (hc + ec > d.eps) { s += ec; ++nw; }
        }
    }
    // Selected rather than branched, so the parent's depth is loaded with the
    // block (s / 0 when none is wet is computed and discarded).
    const double m = s / (double)nw;
    const double ground = -hpar;
    const double v = (nw > 0) ? ((m > ground) ? m : ground) : __longlong_as_double(0x7ff8000000000000LL);
    P.ring[pc] = v;                                     // NaN: none wet
}

// The new parent flux on a child's edge goes to the 3 child faces it covers.
// cmask: bit q set when child q's edge faces may lie in the tile's output
// rows and columns (children from the 33rd on are always visited).  A masked
// child's boundary is injected after the launch from its list (k_inject): the
// child's own tiles write its faces inside the rectangle in this launch.
template <typename F>
__device__ void inject_edges(const DomainDev &d, const LevelDev &L, int b, int c, int r, bool xface, bool yface,
                             F Mnew, F Nnew, unsigned cmask)
{
    for (int q = 0; q < L.n_children; ++q) {
        if (q < 32 && !((cmask >> q) & 1u)) continue;
        const LevelDev &C = level_of(d, child_level(d, L.first_child + q));
        if (C.masked) continue;
        const int fw = C.nx / 3, fh = C.ny / 3;
        const int CP = C.pitch;
        if (xface && r >= C.off_j && r < C.off_j + fh && (c == C.off_i || c == C.off_i + fw)) {
            const int ci = (c == C.off_i) ? 0 : C.nx;
            const int j0 = 3 * (r - C.off_j);
            F *cm = static_cast<F *>(C.M[b ^ 1]);
            cm[ci + CP * j0] = Mnew;
            cm[ci + CP * (j0 + 1)] = Mnew;
            cm[ci + CP * (j0 + 2)] = Mnew;
        }
        if (yface && c >= C.off_i && c < C.off_i + fw && (r == C.off_j || r == C.off_j + fh)) {
            const int cj = (r == C.off_j) ? 0 : C.ny;
            const int i0 = 3 * (c - C.off_i);
            F *cn = static_cast<F *>(C.N[b ^ 1]);
            cn[i0 + CP * cj] = Nnew;
            cn[i0 + 1 + CP * cj] = Nnew;
            cn[i0 + 2 + CP * cj] = Nnew;
        }
    }
}


// Output rows [r0, r1) of tile g of domain d (0 <= r0 < r1 <= th, and the
// first of them at most ny): read buffer b, write buffer b^1 (paper Eqs. 1-3
// and the nest exchanges of Sec. IV-C for those rows' cells and faces).
// Returns whether every value written was left bitwise unchanged (the
// wavefront's part of the tile's stationarity); the caller records the flag.
template <typename F, bool Ring>
__device__ __forceinline__ bool fused_rows_k(const DomainDev &d, int b, int g, int l, int r0, int r1)
{
    const LevelDev &L = level_of(d, l);
    const int tl = g - L.tile_base;
    const int x0 = tile_x(tl, L.tiles_x, L.tiles_y) * RTI_TW;
    const int y0 = tile_y(tl, L.tiles_x, L.tiles_y) * d.th + r0;     // first output row
    const int yend = y0 + (r1 - r0);                                 // one past the last
    constexpr bool has_child = Ring;                 // the tile meets a child's ring or edge faces
    const bool root = (l == 0);
    const unsigned cmask = has_child ? d.tcmask[g] : 0u;   // children whose edges the tile injects

    const int lane = (int)(threadIdx.x & 63);
    const int c = x0 - 2 + lane;
    const int nx = L.nx, ny = L.ny, P = L.pitch;
    const double r = L.r, eps = d.eps;
    const F rf = (F)L.r, grf = (F)L.gr, fcf = (F)d.fc;
    const double *Eb = L.eta[b];
    const F *Hh = static_cast<const F *>(L.h), *Mb = static_cast<const F *>(L.M[b]);
    const F *Nb = static_cast<const F *>(L.N[b]);
    double *Eo = L.eta[b ^ 1];
    F *Mo = static_cast<F *>(L.M[b ^ 1]), *No = static_cast<F *>(L.N[b ^ 1]), *Z = static_cast<F *>(L.zmax);


    const bool col_cell = (c >= 0) && (c < nx);
    const bool col_xf = (c >= 0) && (c <= nx);
    const bool col_xint = (c >= 1) && (c <= nx - 1);
    const bool out_lane = (lane >= 2) && (lane < 2 + RTI_TW);

    // Every array is padded with zeros: 2 columns on the left, at least 61 on
    // the right of the last face, 3 rows below and RTI_PD + 3 above; the padding is
    // never written.  So a lane can load any (c, row) of its tile without a
    // bounds test and gets exactly 0 outside the level.  Offsets are taken
    // from the start of the padded allocation (always >= 0), one 32-bit
    // element offset per row shared by every array.
    const uint32_t pad = (uint32_t)(RTI_PAD_BOTTOM * P + 2);
    const char *Eb_a = reinterpret_cast<const char *>(Eb - pad);
    const char *Hh_a = reinterpret_cast<const char *>(Hh - pad);
    const char *Mb_a = reinterpret_cast<const char *>(Mb - pad);
    const char *Nb_a = reinterpret_cast<const char *>(Nb - pad);
    const uint32_t u0 = (uint32_t)(x0 + lane);                    // element offset of (c, -RTI_PAD_BOTTOM)
    auto ofs = [&](int row) -> uint32_t { return u0 + (uint32_t)P * (uint32_t)(row + RTI_PAD_BOTTOM); };
    auto ld_eta = [&](int row) -> double {
        return *reinterpret_cast<const double *>(Eb_a + ofs(row) * (uint32_t)sizeof(double));
    };
    auto ld_h = [&](int row) -> double {
        return (double)*reinterpret_cast<const F *>(Hh_a + ofs(row) * (uint32_t)sizeof(F));
    };
    auto ld_xf = [&](int row) -> F { return *reinterpret_cast<const F *>(Mb_a + ofs(row) * (uint32_t)sizeof(F)); };
    auto ld_yf = [&](int row) -> F { return *reinterpret_cast<const F *>(Nb_a + ofs(row) * (uint32_t)sizeof(F)); };
    // Ring means of the step (precomputed in the active-list launch), read like
    // eta by the tiles that meet a child's ring; the others do not load them.
    const char *Rg_a = reinterpret_cast<const char *>((has_child ? L.ring : Eb) - pad);
    auto ld_ring = [&](int row) -> double {
        if constexpr (Ring) return *reinterpret_cast<const double *>(Rg_a + ofs(row) * (uint32_t)sizeof(double));
        else return 0.0;
    };

    const int t0 = y0 - 2;
    const int t1 = min(yend, ny + 1);          // last iteration; it writes row t1 - 1

    // Output arrays through the same padded offsets.
    char *Eo_a = reinterpret_cast<char *>(Eo - pad);
    char *Mo_a = reinterpret_cast<char *>(Mo - pad);
    char *No_a = reinterpret_cast<char *>(No - pad);
    char *Z_a = reinterpret_cast<char *>(Z - pad);
    auto ld_z = [&](int row) -> F { return *reinterpret_cast<const F *>(Z_a + ofs(row) * (uint32_t)sizeof(F)); };

    // Rolling window of RTI_NS = RTI_PD + 3 rows: iteration t works on slot
    // K = (t - t0) mod RTI_NS (row t); K-1 holds row t-1, K-2 row t-2, and
    // K+RTI_PD receives the raw loads of row t+RTI_PD, which therefore have
    // RTI_PD rows of arithmetic to arrive.  The loop is unrolled by RTI_NS so
    // every slot index is a compile-time constant and rows rotate by renaming,
    // not by copying registers.
    constexpr int NS = RTI_NS;
    RowW<F> w[NS] = {};
    w[NS - 1].Ny = ld_yf(t0);                      // bottom face of the first row
    w[NS - 1].NyL = from_left(w[NS - 1].Ny);
#pragma unroll
    for (int k = 0; k < RTI_PD; ++k) {
        w[k].E = ld_eta(t0 + k);
        w[k].H = ld_h(t0 + k);
        w[k].Mx = ld_xf(t0 + k);
        w[k].Ny = ld_yf(t0 + k + 1);
        w[k].R = ld_ring(t0 + k);
    }
    bool quiet = true;
    bool bad = false;            // a non-finite value written (the divergence watchdog)

    // Phase of a row (compile time): 0 the first warm-up row (y0 - 2: only its
    // new water level is read, by the y-faces of row y0 - 1), 1 the second
    // (y0 - 1: its faces are read as neighbours, never updated, so their
    // friction is not needed), 2 the rows from y0 on.
    auto do_row = [&](auto kc, auto phc, int t) {
        constexpr int K = decltype(kc)::value;
        constexpr int PH = decltype(phc)::value;
        RowW<F> &cur = w[K];
        const RowW<F> &p = w[(K + NS - 1) % NS];
        const RowW<F> &pp = w[(K + NS - 2) % NS];
        RowW<F> &nxt = w[(K + RTI_PD) % NS];
        // Unconditional loads (the last iterations' are not used; row
        // t1 + RTI_PD + 1 <= ny + RTI_PD + 2 is still padding): a load under a
        // branch would make the compiler wait for every load in flight where
        // the paths join.
        nxt.E = ld_eta(t + RTI_PD);
        nxt.H = ld_h(t + RTI_PD);
        nxt.Mx = ld_xf(t + RTI_PD);
        nxt.Ny = ld_yf(t + RTI_PD + 1);
        nxt.R = ld_ring(t + RTI_PD);
        cur.Z = ld_z(t);
        const bool row_cell = (t >= 0) && (t < ny);

        // Continuity of row t (Eq. 1, FP64), then the child-to-parent mean on ring cells.
        const double H_t = cur.H;
        cur.MxR = from_right(cur.Mx);
        double e1 = cur.E - r * (((double)cur.MxR - (double)cur.Mx) + ((double)cur.Ny - (double)p.Ny));
        e1 = (H_t + e1 < 0.0) ? -H_t : e1;
        e1 = (col_cell && row_cell) ? e1 : 0.0;
        if constexpr (Ring) e1 = (col_cell && row_cell && cur.R == cur.R) ? cur.R : e1;
        cur.e1 = e1;
        // a water level this tile writes (row t is written in the next iteration) left unchanged?
        if (out_lane && col_cell && t >= y0 && t < yend && t < ny) quiet = quiet && same_bits(e1, cur.E);

        // Face quantities: x-face c of row t, y-face c at j = t.
        cur.e1L = from_left(e1);
        cur.HL = from_left(H_t);
        cur.NyL = from_left(cur.Ny);
        const F nb = F(0.25) * ((p.NyL + cur.NyL) + (p.Ny + cur.Ny));
        if constexpr (PH > 0)
            cur.x = face_q<F, (PH == 2)>(col_xint && row_cell, cur.HL, cur.e1L, H_t, e1, eps, cur.Mx, nb, fcf);
        const F mb = F(0.25) * ((p.Mx + p.MxR) + (cur.Mx + cur.MxR));
        if constexpr (PH > 0)
            cur.y = face_q<F, (PH == 2)>(col_cell && t >= 1 && t <= ny - 1, p.H, p.e1, H_t, e1, eps, p.Ny, mb, fcf);

        // Momentum and outputs of row (x-faces, cells) / face (y-faces) rr = t-1.
        // The momentum of both faces is evaluated on every lane (inactive
        // faces carry safe values) and the rule selects the result; only the
        // stores depend on the lane.
        const int rr = t - 1;
        if (PH == 2 && rr >= y0 && rr <= ny) {
            const FaceQ<F> &xp = p.x, &yp = p.y;
            const int xl_act = dpp_left_i(xp.act), xr_act = dpp_right_i(xp.act);
            const F xl_f = from_left(xp.f), xr_f = from_right(xp.f);
            const F xl_q = from_left(xp.q), xr_q = from_right(xp.q);
            const int yl_act = dpp_left_i(yp.act), yr_act = dpp_right_i(yp.act);
            const F yl_cr = from_left(yp.cr), yr_cr = from_right(yp.cr);
            const F yl_p = from_left(yp.p), yr_p = from_right(yp.p);
            const F X = upwind_diff<F>(xp.f, xp.q, xl_act != 0, xl_f, xl_q, xr_act != 0, xr_f, xr_q);
            const F Y = upwind_diff<F>(xp.cr, xp.p, pp.x.act != 0, pp.x.cr, pp.x.p, cur.x.act != 0, cur.x.cr, cur.x.p);
            const F Mint = new_flux<F>(xp, p.e1 - p.e1L, X, Y, rf, grf);
            const F Yd = upwind_diff<F>(yp.f, yp.q, pp.y.act != 0, pp.y.f, pp.y.q, cur.y.act != 0, cur.y.f, cur.y.q);
            const F Xd = upwind_diff<F>(yp.cr, yp.p, yl_act != 0, yl_cr, yl_p, yr_act != 0, yr_cr, yr_p);
            const F Nint = new_flux<F>(yp, p.e1 - pp.e1, Yd, Xd, rf, grf);
            const bool xf_here = col_xf && rr < ny;
            const bool yf_int = col_cell && rr >= 1 && rr <= ny - 1;
            F Mnew = (xp.act != 0) ? Mint : F(0);        // xp.act implies an interior face
            F Nnew = (yp.act != 0) ? Nint : F(0);
            if (root) {
                // One radiation value per face kind: the west side's at column 0, the east side's at
                // column nx (operands selected first, then one evaluation); the south side's at face
                // row 0, the north side's at row ny.  A wall gives 0.
                const bool west = (c == 0), south = (rr == 0);
                const bool xopen = west ? (d.bc[0] == RTI_BC_OPEN_DEV) : (d.bc[1] == RTI_BC_OPEN_DEV);
                const bool yopen = south ? (d.bc[2] == RTI_BC_OPEN_DEV) : (d.bc[3] == RTI_BC_OPEN_DEV);
                const double mrad = radiate(d.g, eps, west ? p.H : p.HL, west ? p.e1 : p.e1L, west ? -1.0 : 1.0);
                const double nrad = radiate(d.g, eps, south ? p.H : pp.H, south ? p.e1 : pp.e1, south ? -1.0 : 1.0);
                if (xf_here && !col_xint) Mnew = (F)(xopen ? mrad : 0.0);
                if (col_cell && !(rr >= 1 && rr <= ny - 1)) Nnew = (F)(yopen ? nrad : 0.0);
            }
            if (out_lane) {
                const bool wx = xf_here && (col_xint || root), wy = col_cell && (yf_int || root);
                if (wx) *reinterpret_cast<F *>(Mo_a + ofs(rr) * (uint32_t)sizeof(F)) = Mnew;
                if (wy) *reinterpret_cast<F *>(No_a + ofs(rr) * (uint32_t)sizeof(F)) = Nnew;
                if (col_cell && rr < ny) {
                    *reinterpret_cast<double *>(Eo_a + ofs(rr) * (uint32_t)sizeof(double)) = p.e1;
                    const F v = (F)((p.H > 0.0) ? p.e1 : p.H + p.e1);
                    if (v > p.Z) *reinterpret_cast<F *>(Z_a + ofs(rr) * (uint32_t)sizeof(F)) = v;
                }
                // the fluxes this tile writes left unchanged?
                quiet = quiet && (!wx || same_bits(Mnew, xp.f)) && (!wy || same_bits(Nnew, yp.f));
                bad = bad || (wx && !isfinite(Mnew)) || (wy && !isfinite(Nnew)) || (col_cell && rr < ny && !isfinite(p.e1));
                if constexpr (Ring) inject_edges<F>(d, L, b, c, rr, xf_here && col_xint, yf_int, Mnew, Nnew, cmask);
            }
        }
    };

    // The two warm-up rows, then rows y0 .. t1 - 1 in slots 2, 3, ..., 1 (the
    // loop runs at least to t0 + 3: t1 >= y0 + 1 since y0 <= ny).
    do_row(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{}, t0);
    do_row(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{}, t0 + 1);
    for (int t = t0 + 2;; t += NS) {
#define RTI_ROW(J)                                                                                     \
        do_row(std::integral_constant<int, ((J) + 2) % NS>{}, std::integral_constant<int, 2>{}, t + (J)); \
        if (t + (J) + 1 > t1) break;
        RTI_ROW(0)
        RTI_ROW(1)
        RTI_ROW(2)
        RTI_ROW(3)
#if RTI_NS > 4
        RTI_ROW(4)
#endif
#if RTI_NS > 5
        RTI_ROW(5)
#endif
#if RTI_NS > 6
        RTI_ROW(6)
#endif
#if RTI_NS > 7
        RTI_ROW(7)
#endif
#if RTI_NS > 8
        RTI_ROW(8)
#endif
#if RTI_NS > 9
#error "RTI_PD above 6 is not unrolled"
#endif
#undef RTI_ROW
    }

    if (__any(bad ? 1 : 0) && lane == 0) atomicOr(&d.status[0], 1);   // sticky: RTI_EDIVERGED on the host
    return __all(quiet ? 1 : 0);
}

// Rows [r0, r1) of tile g (fused_rows_k), with or without the child-ring
// path: a tile's static bits say whether it meets a child's ring or edge
// faces; the others neither load ring means nor inject (wavefront-uniform).
template <typename F>
__device__ __forceinline__ bool fused_rows(const DomainDev &d, int b, int g, int l, int r0, int r1)
{
    if (d.tinfo[g] & TI_CHILD) return fused_rows_k<F, true>(d, b, g, l, r0, r1);
    return fused_rows_k<F, false>(d, b, g, l, r0, r1);
}

// Stationarity history of tile g: bit1 <- bit0, bit0 <- this step left every
// value the tile writes (water levels, fluxes) bitwise unchanged.
__device__ __forceinline__ void record_quiet(const DomainDev &d, int g, bool all_quiet)
{
    const uint8_t old = d.tflag[g];
    const uint8_t nw = (d.tinfo[g] & TI_PINNED) ? 0 : (uint8_t)(((old & 1u) << 1) | (all_quiet ? 1u : 0u));
    d.tflag[g] = nw;
}

// A whole tile on one wavefront.
template <typename F>
__device__ __forceinline__ void fused_tile(const DomainDev &d, int b, int g, int l)
{
    const bool q = fused_rows<F>(d, b, g, l, 0, d.th);
    if ((threadIdx.x & 63) == 0) record_quiet(d, g, q);
}

// Position in the active list of workgroup w's i-th tile.  Workgroups go to
// the 8 XCDs round-robin; XCD x works through the x-th contiguous slice of the
// (row-ordered) list, so the halo rows and columns a tile shares with its
// neighbours sit in the same L2.  A grid smaller than the list makes every
// workgroup loop over several tiles (a persistent grid); the loop bound is
// uniform, so every wavefront reaches the exit.
__device__ __forceinline__ int slice_pos(int n_active, int slot)
{
    const int per = (n_active + 7) >> 3;
    if (slot >= per) return -1;
    const int pos = (int)(blockIdx.x & 7) * per + slot;
    return pos < n_active ? pos : -1;
}

// One workgroup per active tile.  Steps with at most split_max active tiles
// are left to k_fused_split.
template <typename F>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_fused(DomainDev d, int b)
{
    const int n = min(d.count[b], d.ntiles);
    if (n <= d.split_max) return;
    const int pos = slice_pos(n, (int)(blockIdx.x >> 3));
    if (pos >= 0) fused_tile<F>(d, b, d.list[pos], d.lmeta[pos]);
}

// Steps with few active tiles (at most split_max): the machine is mostly
// idle, and a tile's serial chain of th + 3 row iterations is the step's
// floor.  Each active tile gets a workgroup of RTI_SPLIT wavefronts, each
// computing a band of ceil(th / RTI_SPLIT) output rows with its own three
// warm-up rows (recomputed from buffer b exactly as the whole tile would), so
// the chain is that band plus three rows.  The bands' stationarity is AND-ed
// in LDS into the tile's flag.  Steps with more active tiles are k_fused's.
template <typename F>
__global__ __launch_bounds__(64 * RTI_SPLIT) __attribute__((amdgpu_waves_per_eu(3))) void k_fused_split(DomainDev d,
                                                                                                       int b)
{
    const int n = min(d.count[b], d.ntiles);
    if (n > d.split_max) return;
    const int pos = slice_pos(n, (int)(blockIdx.x >> 3));
    if (pos < 0) return;                                    // uniform over the workgroup
    const int g = d.list[pos], l = d.lmeta[pos];
    const LevelDev &L = level_of(d, l);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // the wavefront's band (uniform)
    const int band = (d.th + RTI_SPLIT - 1) / RTI_SPLIT;
    const int r0 = w * band, r1 = min(d.th, r0 + band);
    const int y0 = tile_y(g - L.tile_base, L.tiles_x, L.tiles_y) * d.th;
    bool q = true;
    if (r0 < r1 && y0 + r0 <= L.ny) q = fused_rows<F>(d, b, g, l, r0, r1);
    __shared__ int band_quiet[RTI_SPLIT];
    if ((threadIdx.x & 63) == 0) band_quiet[w] = q ? 1 : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int all = 1;
        for (int k = 0; k < RTI_SPLIT; ++k) all &= band_quiet[k];
        record_quiet(d, g, all != 0);
    }
}

// A persistent grid: every workgroup loops over tiles.  (The loop costs the
// register allocator a few registers; it is held to 3 wavefronts per SIMD.)
template <typename F>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_fused_loop(DomainDev d, int b)
{
    const int n_active = min(d.count[b], d.ntiles);
    if (n_active <= d.split_max) return;
    for (int slot = (int)(blockIdx.x >> 3);; slot += (int)(gridDim.x >> 3)) {
        const int pos = slice_pos(n_active, slot);
        if (pos < 0) break;
        fused_tile<F>(d, b, d.list[pos], d.lmeta[pos]);
    }
}

// Member descriptors of a batch are read through the constant address space,
// so their (wavefront-uniform) fields come in with scalar loads, as a single
// domain's do from the kernel arguments.
typedef const __attribute__((address_space(4))) DomainDev ConstDomainDev;

// Every member of a batch in one launch: the list holds global tile numbers
// (member base + tile), and each member keeps its own buffer parity.
template <typename F>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_fused_batch(BatchDev bd, int flip)
{
    ConstDomainDev *doms = (ConstDomainDev *)bd.doms;
    const int n_active = min(bd.count[flip], bd.ntiles);
    for (int slot = (int)(blockIdx.x >> 3);; slot += (int)(gridDim.x >> 3)) {
        const int pos = slice_pos(n_active, slot);
        if (pos < 0) break;
        // the list entry and its level and member are loaded together
        const int G = bd.list[pos];
        const int meta = bd.lmeta[pos];
        const int m = meta & 0xffff;
        fused_tile<F>(*(const DomainDev *)&doms[m], bd.par[m] ^ flip, G - bd.base[m], meta >> 16);
    }
}

// ---------------------------------------------------------------------------
// Active tiles of the coming step.  A tile is tested with its 9 flag bytes
// loaded together, then, near a nest boundary, the flags of its coupled tiles
// on the parent or child level (the writers of the injected edge faces it
// reads, or of the child blocks its ring means read).
__device__ __forceinline__ int tile_active(const DomainDev &d, int g, int all_active)
{
    if (all_active) return 1;
    const unsigned info = d.tinfo[g];
    if (info & TI_PINNED) return 1;
    const int l = level_of_tile(d, g);
    const LevelDev &L = level_of(d, l);
    const int base = L.tile_base, nxt = L.tiles_x, nyt = L.tiles_y;
    const int tl = g - base;
    const int tx = tile_x(tl, nxt, nyt), ty = tile_y(tl, nxt, nyt);
    // The 9 flags are loaded unconditionally (indices clamped into the level,
    // so all loads are issued together); neighbours outside count as stationary.
    unsigned f[9];
    #pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        #pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int x = min(max(tx + dx, 0), nxt - 1), y = min(max(ty + dy, 0), nyt - 1);
            f[(dy + 1) * 3 + dx + 1] = d.tflag[base + tile_index(x, y, nxt, nyt)];
        }
    }
    unsigned acc = 3u;
    #pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        #pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int x = tx + dx, y = ty + dy;
            const bool in = x >= 0 && x < nxt && y >= 0 && y < nyt;
            acc &= in ? f[(dy + 1) * 3 + dx + 1] : 3u;
        }
    }
    if ((info & TI_DEPS) && (acc & 3u) == 3u) {
        // 8 list entries at a time (the last one repeated past the end), so
        // the index loads and then the flag loads of a group are in flight
        // together rather than one after another.
        const int e = d.dep_off[g + 1] - 1;
        for (int k = d.dep_off[g]; k <= e; k += 8) {
            int t[8];
            #pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = d.dep[min(k + u, e)];
            #pragma unroll
            for (int u = 0; u < 8; ++u) acc &= (unsigned)d.tflag[t[u]];
        }
    }
    return (acc & 3u) == 3u ? 0 : 1;
}

// One thread per tile, 256 tiles per workgroup: a block-wide scan orders the
// block's active tiles and one atomic reserves their place in the list of
// step parity b (the list keeps each block's tiles together and in order).
// The counter of the other parity, read by nobody during this step, is reset
// for the next one, so no memset is needed between steps.
__device__ __forceinline__ void append_active(int a, int id, int meta, int tb, int *count_b, int *count_other, int *list,
                                              int *lmeta, int cap, int *overflow)
{
    __shared__ int wsum[4];
    __shared__ int base;
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    int incl = a;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < 4; ++k) {
        const int s = wsum[k];
        before += (k < w) ? s : 0;
        total += s;
    }
    if (tid == 0) base = total ? atomicAdd(count_b, total) : 0;
    if (tb == 0 && tid == 0) *count_other = 0;
    __syncthreads();
    // A list holds at most cap (= tiles) entries: each tile is listed at most
    // once per step, so a position at or beyond cap means the counter was not
    // reset for this step.  The entry is then dropped (the writes stay inside
    // the list) and the sticky overflow flag raised, which the host reports
    // as RTI_EINTERNAL at the next synchronising call.
    const int pos = base + before + incl - 1;
    if (a && pos < cap) {
        list[pos] = id;
        lmeta[pos] = meta;
    }
    if (a && pos >= cap) atomicOr(overflow, 1);
}

// Sum of c over the workgroup added to slot `slot` of part (no atomics: each
// slot has one writer; the host adds the slots up).
__device__ __forceinline__ void add_cells(int c, unsigned long long *part, int slot)
{
    __shared__ int csum[4];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) csum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = (csum[0] + csum[1]) + (csum[2] + csum[3]);
        if (t) part[slot] += (unsigned long long)t;
    }
}

// Ring cells per ring workgroup: one wavefront of each 256-thread workgroup
// works, so the ring gathers spread over four times as many compute units.  A
// vertical ring's gathers touch one cache line per lane and load, so a compute
// unit's address units, not bytes, bound the ring half of the launch.
#define RTI_RING_LANES 64

// The active-list launch: its first nrb workgroups compute the ring means of
// the step (one thread per ring cell; dispatched first, their gathers are the
// longest), the others list the active tiles (one thread per tile).  Held to
// 4 wavefronts per SIMD so that a ring cell's 42 loads can all be in flight.
template <typename F>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_active(DomainDev d, int b, int all_active,
                                                                                         int nrb)
{
    if ((int)blockIdx.x < nrb) {
        const int e = (int)blockIdx.x * RTI_RING_LANES + (int)threadIdx.x;
        if ((int)threadIdx.x < RTI_RING_LANES && e < d.nring) ring_mean<F>(d, b, e);
        return;
    }
    const int tb = (int)blockIdx.x - nrb;
    const int g = tb * 256 + (int)threadIdx.x;
    const int a = (g < d.ntiles) ? tile_active(d, g, all_active) : 0;
    const int l = (g < d.ntiles) ? level_of_tile(d, g) : 0;
    add_cells(a ? d.tcells[g] : 0, d.cells_done, tb);
    append_active(a, g, l, tb, &d.count[b], &d.count[b ^ 1], d.list, d.lmeta, d.ntiles, &d.status[1]);
}

// The same over a batch's global tables: each member's own flags decide, and
// each ring cell uses its member's state and buffer parity.
template <typename F>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_active_batch(BatchDev bd, int flip,
                                                                                               int all_active, int nrb)
{
    if ((int)blockIdx.x < nrb) {
        const int E = (int)blockIdx.x * RTI_RING_LANES + (int)threadIdx.x;
        if ((int)threadIdx.x < RTI_RING_LANES && E < bd.nring) {
            const int m = bd.rdom[E];
            ring_mean<F>(bd.doms[m], bd.par[m] ^ flip, E - bd.rbase[m]);
        }
        return;
    }
    const int tb = (int)blockIdx.x - nrb;
    const int G = tb * 256 + (int)threadIdx.x;
    int a = 0, c = 0, meta = 0;
    if (G < bd.ntiles) {
        const int m = bd.tdom[G];
        const DomainDev &d = bd.doms[m];
        a = tile_active(d, G - bd.base[m], all_active);
        c = a ? d.tcells[G - bd.base[m]] : 0;
        meta = (level_of_tile(d, G - bd.base[m]) << 16) | m;
    }
    add_cells(c, bd.cells_done, tb);
    append_active(a, G, meta, tb, &bd.count[flip], &bd.count[flip ^ 1], bd.list, bd.lmeta, bd.ntiles, &bd.status[1]);
}

}  // namespace

hipError_t launch_active(const DomainDev &d, int b, int all_active, hipStream_t s)
{
    const int nrb = (d.nring + RTI_RING_LANES - 1) / RTI_RING_LANES, ntb = (d.ntiles + 255) / 256;
    if (d.bulk32)
        hipLaunchKernelGGL(k_active<float>, dim3(nrb + ntb), dim3(256), 0, s, d, b, all_active, nrb);
    else
        hipLaunchKernelGGL(k_active<double>, dim3(nrb + ntb), dim3(256), 0, s, d, b, all_active, nrb);
    return hipGetLastError();
}

hipError_t launch_active_batch(const BatchDev &bd, int flip, int all_active, int bulk32, hipStream_t s)
{
    const int nrb = (bd.nring + RTI_RING_LANES - 1) / RTI_RING_LANES, ntb = (bd.ntiles + 255) / 256;
    if (bulk32)
        hipLaunchKernelGGL(k_active_batch<float>, dim3(nrb + ntb), dim3(256), 0, s, bd, flip, all_active, nrb);
    else
        hipLaunchKernelGGL(k_active_batch<double>, dim3(nrb + ntb), dim3(256), 0, s, bd, flip, all_active, nrb);
    return hipGetLastError();
}

// grid: workgroups (a multiple of 8), at most one per tile; fewer make a
// persistent grid.
hipError_t launch_fused(const DomainDev &d, int b, int grid, hipStream_t s, bool every_tile)
{
    const bool loop = grid < (d.ntiles + 7) / 8 * 8;
    if (d.bulk32) {
        if (loop) hipLaunchKernelGGL(k_fused_loop<float>, dim3(grid), dim3(64), 0, s, d, b);
        else hipLaunchKernelGGL(k_fused<float>, dim3(grid), dim3(64), 0, s, d, b);
    } else {
        if (loop) hipLaunchKernelGGL(k_fused_loop<double>, dim3(grid), dim3(64), 0, s, d, b);
        else hipLaunchKernelGGL(k_fused<double>, dim3(grid), dim3(64), 0, s, d, b);
    }
    hipError_t e = hipGetLastError();
    // with every tile listed the split kernel has nothing to do unless the domain is that small
    if (e != hipSuccess || d.split_max <= 0 || (every_tile && d.ntiles > d.split_max)) return e;
    // the split kernel: one workgroup per list position up to split_max, 8 XCD slices
    const int sgrid = (d.split_max + 7) / 8 * 8;
    if (d.bulk32)
        hipLaunchKernelGGL(k_fused_split<float>, dim3(sgrid), dim3(64 * RTI_SPLIT), 0, s, d, b);
    else
        hipLaunchKernelGGL(k_fused_split<double>, dim3(sgrid), dim3(64 * RTI_SPLIT), 0, s, d, b);
    return hipGetLastError();
}

hipError_t launch_fused_batch(const BatchDev &bd, int flip, int bulk32, int grid, hipStream_t s)
{
    if (bulk32)
        hipLaunchKernelGGL(k_fused_batch<float>, dim3(grid), dim3(64), 0, s, bd, flip);
    else
        hipLaunchKernelGGL(k_fused_batch<double>, dim3(grid), dim3(64), 0, s, bd, flip);
    return hipGetLastError();
}

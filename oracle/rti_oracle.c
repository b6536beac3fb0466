/*
 * rti_oracle.c -- TEST INFRASTRUCTURE ONLY: the CPU FP64 oracle.
 *
 * A plain, slow, obviously-correct reference for the time step of the nested
 * nonlinear long-wave model of the RTi simulator (TUNAMI-N2 family), written
 * from the paper (arXiv 2408.07609):
 *   - continuity, Sec. II-A Eq. (1)                       -> ora_mass
 *   - momentum with advection, pressure and Manning
 *     friction, Sec. II-A Eqs. (2)-(3), D = h + eta        -> ora_momentum
 *   - leap-frog in time on a staggered grid, Sec. II-A     -> ora_step
 *   - nested grids, ratio 3:1, inclusive, one dt on all
 *     levels, Sec. II-A and Sec. V-A                       -> ora_domain
 *   - per-iteration order: mass, child->parent water
 *     level, momentum, parent->child fluxes, output
 *     maxima, Sec. IV-A (time-integration loop)            -> ora_step
 *   - child->parent level as the mean of the 3x3 child
 *     cells summed j-outer / i-inner, Sec. IV-C (JNZSND)   -> ora_jnz
 * The paper gives no discretisation details; every place where it is silent
 * follows a stated reading (time levels, face depth, upwind advection,
 * semi-implicit friction, wet/dry rule, open boundary, flux injection).
 * Each reading is named where it is used.
 *
 * Nothing on the product path may load this file: only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg do.  It shares no code,
 * header or constant with the HIP library.
 *
 * Layout per level (i = x index fastest):
 *   h, eta, zmax : nx*ny cells,           cell (i,j)   at i + nx*j
 *   M            : (nx+1)*ny x-faces,     face (i,j)   between cells (i-1,j),(i,j)
 *   N            : nx*(ny+1) y-faces,     face (i,j)   between cells (i,j-1),(i,j)
 * h > 0 is still-water depth, h <= 0 is land with elevation -h.
 *
 * A child level may leave cells of its rectangle out (mask): the union of
 * touching blocks of one resolution (Sec. II-A, Table 1: a resolution is
 * covered by several rectangular blocks) held in one array, so that blocks
 * that share an edge exchange exactly, as one grid.  The mask is constant
 * over each child 3x3 block, so each parent cell is either covered by the
 * child (its 9 child cells inside) or not.  A cell outside takes no part in
 * the step: no face touching it carries a computed flux, and the
 * exchanges follow the covered region's boundary instead of the rectangle's.
 *
 * Arithmetic: IEEE binary64, round to nearest, built with -ffp-contract=off so
 * no multiply-add is fused.  Sums are grouped exactly as written.  Every
 * operation of the step is correctly rounded: +, -, *, / and sqrt by IEEE, and
 * the cube root of the friction term by ora_cbrt_rn (libm's cbrt is not), so
 * the step's result is one fixed double for each input, whatever machine
 * computes it.  The initial condition (ora_set_source) uses libm's exp, sin and
 * cos, which are not correctly rounded: it is exact only to within an ulp or so.
 *
 * Parity unpinned (no pin beyond the lake-at-rest, symmetry and the oracle
 * itself fixes them, because the paper is silent): the one-wet-side face depth
 * of the wet/dry rule, the neighbour-skip rule of the advection term, the
 * wet-only average of the child->parent exchange, and on a masked level the
 * ring cell at an inner corner of the covered region (a covered parent cell
 * whose only uncovered neighbour is diagonal takes the child mean, as a
 * rectangle's corner cells do).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny;         /* cells */
    int32_t parent;         /* index of the parent level, -1 for the root */
    int32_t off_i, off_j;   /* child origin, in parent cells */
    double dx;              /* grid spacing [m] */
    double ox, oy;          /* south-west corner of the level [m] */
    double *h, *eta, *M, *N, *zmax;
    double *M2, *N2;        /* scratch for the new fluxes, same shapes as M, N */
    double *clip;           /* optional (may be NULL): accumulated clipped depth per cell */
    const uint8_t *mask;    /* optional (NULL: every cell): 1 = cell inside the level, nx*ny */
} ora_level;

typedef struct {
    int32_t nlev;
    int32_t bc[4];          /* root sides W,E,S,N: 0 open (radiation), 1 wall */
    ora_level *lv;
    double dt, g, manning, eps;
    int64_t steps;
} ora_domain;

#define CELL(L, i, j)  ((size_t)(j) * (size_t)(L)->nx + (size_t)(i))
#define XF(L, i, j)    ((size_t)(j) * (size_t)((L)->nx + 1) + (size_t)(i))
#define YF(L, i, j)    ((size_t)(j) * (size_t)(L)->nx + (size_t)(i))

/* Is cell (i, j) of level L inside it (not left out by its mask)? */
static int inside(const ora_level *L, int i, int j)
{
    return !L->mask || L->mask[CELL(L, i, j)];
}

/* Is parent cell (I, J), counted from child C's origin, covered by C (the
 * 3x3 child cells below it inside C)? */
static int covered(const ora_level *C, int I, int J)
{
    if (I < 0 || J < 0 || I >= C->nx / 3 || J >= C->ny / 3) return 0;
    return inside(C, 3 * I, 3 * J);
}

int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Correctly rounded cube root: the double nearest to the real cube root of x,
 * for a positive normal x (here the reciprocal of a face depth).  libm's cbrt
 * lands within about an ulp of the root but is not always the nearest double,
 * and another platform's cbrt need not agree with it; the nearest double is
 * one fixed number.  Starting from libm's value y, y moves to its neighbour
 * while the root lies beyond the midpoint between them.  The root lies above a
 * midpoint m exactly when m^3 < x.  That test is done on integers: m = K 2^(e-1)
 * with K odd and below 2^55, x = X 2^ex with X the 53-bit significand, and K^3
 * (below 2^165) is compared with X 2^(ex - 3e + 3).  K^3 is odd and the other
 * side even, so the two are never equal: no root is ever a midpoint. */

/* x = X 2^E, X the 53-bit integer significand (x positive and normal). */
static uint64_t int_significand(double x, int *E)
{
    uint64_t b;
    memcpy(&b, &x, sizeof b);
    *E = (int)(b >> 52) - 1075;
    return (b & ((UINT64_C(1) << 52) - 1)) | (UINT64_C(1) << 52);
}

static double bits_step(double y, int k)         /* the k-th neighbour of y > 0 */
{
    uint64_t b;
    memcpy(&b, &y, sizeof b);
    b += (uint64_t)(int64_t)k;
    memcpy(&y, &b, sizeof y);
    return y;
}

/* Is ((lo + hi) / 2)^3 < x, for adjacent positive normal doubles lo < hi?
 * Exact, on integers. */
static int midpoint_cube_below_exact(double lo, double hi, double x)
{
    int elo, ehi, ex;
    const uint64_t Llo = int_significand(lo, &elo), Lhi = int_significand(hi, &ehi), X = int_significand(x, &ex);
    const int e = (elo < ehi) ? elo : ehi;
    const uint64_t K = (Llo << (elo - e)) + (Lhi << (ehi - e));      /* lo + hi = K 2^e */
    const int sh = ex - (3 * e - 3);             /* x = (X 2^sh) 2^(3e-3), midpoint^3 = K^3 2^(3e-3) */
    if (sh < 64 || sh - 64 > 74) abort();        /* outside what the comparison was sized for */
    /* K^3 = top 2^64 + (something below 2^64) */
    const unsigned __int128 K2 = (unsigned __int128)K * K;                    /* below 2^110 */
    const unsigned __int128 low = (unsigned __int128)(uint64_t)K2 * K;        /* below 2^119 */
    const unsigned __int128 top = (K2 >> 64) * K + (low >> 64);
    /* X 2^sh = (X 2^(sh-64)) 2^64 exactly; K^3 < X 2^sh iff top < X 2^(sh-64) */
    return top < ((unsigned __int128)X << (sh - 64));
}

/* The same test, first in long double (64-bit significand: the midpoint is
 * exact and its cube within 2^-63 relative), which settles every case where
 * the cube is more than 2^-60 x away from x; the rest go to the integer test. */
static int midpoint_cube_below(double lo, double hi, double x)
{
    const long double m = ((long double)lo + (long double)hi) * 0.5L;
    const long double d = (m * m) * m - (long double)x;
    const long double tol = 0x1p-60L * (long double)x;
    if (d < -tol) return 1;
    if (d > tol) return 0;
    return midpoint_cube_below_exact(lo, hi, x);
}

double ora_cbrt_rn(double x)
{
    double y = cbrt(x);
    for (int moves = 0; moves < 8; moves++) {  /* libm is within an ulp: one move at most */
        const double up = bits_step(y, 1), dn = bits_step(y, -1);
        if (midpoint_cube_below(y, up, x)) { y = up; continue; }      /* root above (y+up)/2 */
        if (!midpoint_cube_below(dn, y, x)) { y = dn; continue; }     /* root below (dn+y)/2 */
        return y;
    }
    return NAN;                                  /* not reached for a positive normal x */
}

/* ora_cbrt_rn over an array (for the tests of the cube root). */
void ora_cbrt_rn_array(const double *x, double *y, int64_t n)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; k++) y[k] = ora_cbrt_rn(x[k]);
}

/* ------------------------------------------------------------------------ */
/* Continuity, Eq. (1): eta^{n+1} = eta^n - dt/dx [(M_{i+1}-M_i) + (N_{j+1}-N_j)],
 * with the fluxes at n+1/2 (fluxes run half a step ahead of the level).
 * Reading: where the new level would fall below the ground (h + eta < 0) it is
 * clipped to the ground, eta = -h; the clipped depth is recorded if asked. */
void ora_mass(ora_domain *d, int l)
{
    ora_level *L = &d->lv[l];
    const double r = d->dt / L->dx;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < L->ny; j++) {
        for (int i = 0; i < L->nx; i++) {
            if (!inside(L, i, j)) continue;
            double e = L->eta[CELL(L, i, j)]
                     - r * ((L->M[XF(L, i + 1, j)] - L->M[XF(L, i, j)])
                          + (L->N[YF(L, i, j + 1)] - L->N[YF(L, i, j)]));
            double hh = L->h[CELL(L, i, j)];
            if (hh + e < 0.0) {
                if (L->clip) L->clip[CELL(L, i, j)] += -(hh + e);
                e = -hh;
            }
            L->eta[CELL(L, i, j)] = e;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Child -> parent water level (Sec. IV-C, the JNZSND exchange): every parent
 * cell on the ring of the child's footprint (a covered parent cell with a
 * parent cell among its 8 neighbours that the child does not cover; for a
 * rectangular child the outermost ring, corners once) takes the mean of the
 * 3x3 child cells it covers, summed j outer, i inner.
 * Reading: only wet child cells (h + eta > eps) enter the mean (a dry child
 * cell holds its ground level, which is not a water level); with no wet child
 * cell the parent keeps its own value; the result is not allowed below the
 * parent's ground. */
void ora_jnz(ora_domain *d, int c)
{
    ora_level *C = &d->lv[c];
    ora_level *P = &d->lv[C->parent];
    const int fw = C->nx / 3, fh = C->ny / 3;
    for (int J = 0; J < fh; J++) {
        for (int I = 0; I < fw; I++) {
            if (!covered(C, I, J)) continue;
            int ring = 0;
            for (int dj = -1; dj <= 1; dj++)
                for (int di = -1; di <= 1; di++)
                    if (!covered(C, I + di, J + dj)) ring = 1;
            if (!ring) continue;
            double s = 0.0;
            int k = 0;
            for (int jj = 3 * J; jj < 3 * J + 3; jj++) {
                for (int ii = 3 * I; ii < 3 * I + 3; ii++) {
                    double e = C->eta[CELL(C, ii, jj)];
                    if (C->h[CELL(C, ii, jj)] + e > d->eps) { s += e; k++; }
                }
            }
            if (k > 0) {
                size_t pc = CELL(P, C->off_i + I, C->off_j + J);
                double v = s / (double)k;
                double ground = -P->h[pc];
                P->eta[pc] = (v > ground) ? v : ground;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Wet/dry rule for the face between cell A and cell B (Imamura-style moving
 * shoreline; reading, the paper only names inundation as an output).
 * Both wet: total depth D = (h_A+h_B)/2 + (eta_A+eta_B)/2, at the new level.
 * One wet, say A: flux allowed only if eta_A > -h_B (the water stands above
 * the dry cell's ground), with D = eta_A + h_B.  Both dry: no flux.
 * In every case the flux is zero when D <= eps.
 * Returns 1 and the depth when the face is active, 0 when the flux is zero. */
static int face_depth(double ha, double ea, double hb, double eb, double eps, double *Dout)
{
    int wa = (ha + ea > eps), wb = (hb + eb > eps);
    double D;
    if (wa && wb) {
        D = 0.5 * (ha + hb) + 0.5 * (ea + eb);
    } else if (wa) {
        if (!(ea > -hb)) return 0;
        D = ea + hb;
    } else if (wb) {
        if (!(eb > -ha)) return 0;
        D = eb + ha;
    } else {
        return 0;
    }
    if (!(D > eps)) return 0;
    *Dout = D;
    return 1;
}

/* A face touching a cell outside the level is, like the level's own edge
 * faces, never active: its flux comes from the parent (ora_jnq) or is 0. */
static int xface_depth(const ora_level *L, double eps, int i, int j, double *D)
{
    if (!inside(L, i - 1, j) || !inside(L, i, j)) return 0;
    return face_depth(L->h[CELL(L, i - 1, j)], L->eta[CELL(L, i - 1, j)],
                      L->h[CELL(L, i, j)], L->eta[CELL(L, i, j)], eps, D);
}

static int yface_depth(const ora_level *L, double eps, int i, int j, double *D)
{
    if (!inside(L, i, j - 1) || !inside(L, i, j)) return 0;
    return face_depth(L->h[CELL(L, i, j - 1)], L->eta[CELL(L, i, j - 1)],
                      L->h[CELL(L, i, j)], L->eta[CELL(L, i, j)], eps, D);
}

/* N averaged to x-face (i,j): the mean of the cell-centred N of cells (i-1,j)
 * and (i,j), each the pair of its south and north faces. */
static double nbar_at_xface(const ora_level *L, int i, int j)
{
    return 0.25 * ((L->N[YF(L, i - 1, j)] + L->N[YF(L, i - 1, j + 1)])
                 + (L->N[YF(L, i, j)] + L->N[YF(L, i, j + 1)]));
}

/* M averaged to y-face (i,j): cells (i,j-1) and (i,j), west+east face each. */
static double mbar_at_yface(const ora_level *L, int i, int j)
{
    return 0.25 * ((L->M[XF(L, i, j - 1)] + L->M[XF(L, i + 1, j - 1)])
                 + (L->M[XF(L, i, j)] + L->M[XF(L, i + 1, j)]));
}

/* First-order upwind difference of a face quantity v along one direction
 * (reading; the paper does not give the advection scheme).  s is the velocity
 * sign carrier at this face (the flux itself, or the cross flux averaged to
 * the face), v its momentum flux; "m" is the neighbour face behind, "p" the
 * one ahead along the axis; ok = the neighbour may be used (inside the level,
 * not a level-boundary face, active under the wet/dry rule).
 * s > 0: v - v_m;  s < 0: v_p - v;  s == 0 (no flow here, v = 0): the
 * momentum flux of each neighbour that flows into this face, -v_m if s_m > 0
 * plus v_p if s_p < 0.  The tie rule keeps still water still and mirror
 * images bitwise mirrored, and lets a newly opened face at a wet front take
 * up the momentum behind it. */
static double upwind_diff(double s, double v, int okm, double sm, double vm,
                          int okp, double sp, double vp)
{
    if (s > 0.0) return okm ? v - vm : 0.0;
    if (s < 0.0) return okp ? vp - v : 0.0;
    double a = (okm && sm > 0.0) ? vm : 0.0;
    double b = (okp && sp < 0.0) ? vp : 0.0;
    return (-a) + b;
}

/* Semi-implicit Manning factor of a face (reading): with the face's own flux
 * f, the cross flux c averaged to the face and the reciprocal rD = 1/D of the
 * total depth, F = fc sqrt(f^2 + c^2) D^(-7/3), where fc = dt/2 g n^2 and
 * D^(-7/3) = rD^2 cbrt(rD) with the correctly rounded cube root.  A face
 * without flow has F = 0 (the product is +0 either way, so the cube root is
 * not needed there). */
static double friction(double fc, double f, double c, double rD)
{
    const double s = fc * sqrt(f * f + c * c);
    if (!(s > 0.0)) return s;
    return s * ((rD * rD) * ora_cbrt_rn(rD));
}

/* x-momentum, Eq. (2), at interior x-face (i,j), 1 <= i <= nx-1.
 * Time levels (reading): the level is eta^{n+1} (already updated), the fluxes
 * on the right-hand side are the old ones, M^{n+1/2}, N^{n+1/2}.
 *  pressure  : g D dt/dx (eta_R - eta_L)
 *  advection : d(M^2/D)/dx and d(M N/D)/dy, each a first-order upwind
 *              difference between this face and its neighbour face along
 *              x (same row) or along y (same column), N averaged to the
 *              x-faces (upwind_diff).
 *  friction  : Manning, g n^2 M sqrt(M^2+N^2) / D^{7/3}, semi-implicit
 *              (reading): the friction on M is the average of the old and new
 *              M, the magnitude uses the old fluxes (friction()).
 *              With F = dt/2 g n^2 sqrt(M^2+N^2)/D^{7/3}:
 *              M_new = ((1-F) M - pressure - advection) / (1+F).
 * Every quotient by a face depth is a product with that face's reciprocal
 * depth 1/D (one division per face; reading: the paper gives no arithmetic). */
static double xmomentum(const ora_domain *d, const ora_level *L, int i, int j)
{
    const double eps = d->eps;
    double D;
    if (!xface_depth(L, eps, i, j, &D)) return 0.0;

    const double r = d->dt / L->dx;
    const double gr = d->g * r;
    const double fc = 0.5 * d->dt * d->g * d->manning * d->manning;
    const double rD = 1.0 / D;
    const double m = L->M[XF(L, i, j)];
    const double nb = nbar_at_xface(L, i, j);

    const double P = (gr * D) * (L->eta[CELL(L, i, j)] - L->eta[CELL(L, i - 1, j)]);

    /* along x: the x-faces i-1 and i+1 in the same row */
    double Dm, Dp;
    const int okm = (i - 1 >= 1) && xface_depth(L, eps, i - 1, j, &Dm);
    const int okp = (i + 1 <= L->nx - 1) && xface_depth(L, eps, i + 1, j, &Dp);
    const double mm = okm ? L->M[XF(L, i - 1, j)] : 0.0;
    const double mp = okp ? L->M[XF(L, i + 1, j)] : 0.0;
    const double X = upwind_diff(m, (m * m) * rD,
                                 okm, mm, okm ? (mm * mm) * (1.0 / Dm) : 0.0,
                                 okp, mp, okp ? (mp * mp) * (1.0 / Dp) : 0.0);
    /* along y: the x-faces in rows j-1 and j+1 */
    double Ds, Dn;
    const int oks = (j - 1 >= 0) && xface_depth(L, eps, i, j - 1, &Ds);
    const int okn = (j + 1 <= L->ny - 1) && xface_depth(L, eps, i, j + 1, &Dn);
    const double nbs = oks ? nbar_at_xface(L, i, j - 1) : 0.0;
    const double nbn = okn ? nbar_at_xface(L, i, j + 1) : 0.0;
    const double Y = upwind_diff(nb, (m * nb) * rD,
                                 oks, nbs, oks ? (L->M[XF(L, i, j - 1)] * nbs) * (1.0 / Ds) : 0.0,
                                 okn, nbn, okn ? (L->M[XF(L, i, j + 1)] * nbn) * (1.0 / Dn) : 0.0);
    const double A = r * (X + Y);
    const double F = friction(fc, m, nb, rD);
    return (((1.0 - F) * m - P) - A) / (1.0 + F);
}

/* y-momentum, Eq. (3), at interior y-face (i,j), 1 <= j <= ny-1: the mirror
 * of xmomentum with x <-> y and M <-> N. */
static double ymomentum(const ora_domain *d, const ora_level *L, int i, int j)
{
    const double eps = d->eps;
    double D;
    if (!yface_depth(L, eps, i, j, &D)) return 0.0;

    const double r = d->dt / L->dx;
    const double gr = d->g * r;
    const double fc = 0.5 * d->dt * d->g * d->manning * d->manning;
    const double rD = 1.0 / D;
    const double n = L->N[YF(L, i, j)];
    const double mb = mbar_at_yface(L, i, j);

    const double P = (gr * D) * (L->eta[CELL(L, i, j)] - L->eta[CELL(L, i, j - 1)]);

    /* along y: the y-faces j-1 and j+1 in the same column */
    double Ds, Dn;
    const int oks = (j - 1 >= 1) && yface_depth(L, eps, i, j - 1, &Ds);
    const int okn = (j + 1 <= L->ny - 1) && yface_depth(L, eps, i, j + 1, &Dn);
    const double ns = oks ? L->N[YF(L, i, j - 1)] : 0.0;
    const double nn = okn ? L->N[YF(L, i, j + 1)] : 0.0;
    const double Yd = upwind_diff(n, (n * n) * rD,
                                  oks, ns, oks ? (ns * ns) * (1.0 / Ds) : 0.0,
                                  okn, nn, okn ? (nn * nn) * (1.0 / Dn) : 0.0);
    /* along x: the y-faces in columns i-1 and i+1 */
    double Dw, De;
    const int okw = (i - 1 >= 0) && yface_depth(L, eps, i - 1, j, &Dw);
    const int oke = (i + 1 <= L->nx - 1) && yface_depth(L, eps, i + 1, j, &De);
    const double mbw = okw ? mbar_at_yface(L, i - 1, j) : 0.0;
    const double mbe = oke ? mbar_at_yface(L, i + 1, j) : 0.0;
    const double Xd = upwind_diff(mb, (n * mb) * rD,
                                  okw, mbw, okw ? (L->N[YF(L, i - 1, j)] * mbw) * (1.0 / Dw) : 0.0,
                                  oke, mbe, oke ? (L->N[YF(L, i + 1, j)] * mbe) * (1.0 / De) : 0.0);
    const double A = r * (Yd + Xd);
    const double F = friction(fc, n, mb, rD);
    return (((1.0 - F) * n - P) - A) / (1.0 + F);
}

/* Momentum update of every interior face of level l.  Level-boundary faces
 * are left alone: the root's are set by ora_bc_root, a child's by ora_jnq. */
void ora_momentum(ora_domain *d, int l)
{
    ora_level *L = &d->lv[l];
    const int nx = L->nx, ny = L->ny;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 1; i <= nx - 1; i++)
            L->M2[XF(L, i, j)] = xmomentum(d, L, i, j);
    #pragma omp parallel for schedule(static)
    for (int j = 1; j <= ny - 1; j++)
        for (int i = 0; i < nx; i++)
            L->N2[YF(L, i, j)] = ymomentum(d, L, i, j);
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 1; i <= nx - 1; i++)
            L->M[XF(L, i, j)] = L->M2[XF(L, i, j)];
    #pragma omp parallel for schedule(static)
    for (int j = 1; j <= ny - 1; j++)
        for (int i = 0; i < nx; i++)
            L->N[YF(L, i, j)] = L->N2[YF(L, i, j)];
}

/* ------------------------------------------------------------------------ */
/* Outer faces of the root level (reading): a wall carries no flux; an open
 * side lets a long wave leave, flux = celerity * level with c = sqrt(g h) of
 * the boundary cell and the sign of the outward normal; no flux when the
 * boundary cell is land (h <= 0) or dry. */
static double radiate(const ora_domain *d, double h, double e, double sign)
{
    if (!(h > 0.0) || !(h + e > d->eps)) return 0.0;
    double c = sqrt(d->g * h);
    return sign * (c * e);
}

void ora_bc_root(ora_domain *d)
{
    ora_level *L = &d->lv[0];
    const int nx = L->nx, ny = L->ny;
    for (int j = 0; j < ny; j++) {
        L->M[XF(L, 0, j)] = d->bc[0] ? 0.0
            : radiate(d, L->h[CELL(L, 0, j)], L->eta[CELL(L, 0, j)], -1.0);
        L->M[XF(L, nx, j)] = d->bc[1] ? 0.0
            : radiate(d, L->h[CELL(L, nx - 1, j)], L->eta[CELL(L, nx - 1, j)], 1.0);
    }
    for (int i = 0; i < nx; i++) {
        L->N[YF(L, i, 0)] = d->bc[2] ? 0.0
            : radiate(d, L->h[CELL(L, i, 0)], L->eta[CELL(L, i, 0)], -1.0);
        L->N[YF(L, i, ny)] = d->bc[3] ? 0.0
            : radiate(d, L->h[CELL(L, i, ny - 1)], L->eta[CELL(L, i, ny - 1)], 1.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Parent -> child fluxes (Sec. IV-A, the JNQ exchange; the interpolation is a
 * reading): each child face on the boundary of the child's footprint (a
 * parent face between a covered and an uncovered parent cell; for a
 * rectangular child the four edges) takes the flux per unit width of the
 * parent face it lies on, on all 3 child faces of that parent face.  Three
 * child faces of width dx/3 then carry exactly the parent face's discharge. */
void ora_jnq(ora_domain *d, int c)
{
    ora_level *C = &d->lv[c];
    ora_level *P = &d->lv[C->parent];
    const int I0 = C->off_i, J0 = C->off_j, fw = C->nx / 3, fh = C->ny / 3;
    for (int J = 0; J < fh; J++)                 /* x-faces: between parent cells (I-1, J) and (I, J) */
        for (int I = 0; I <= fw; I++)
            if (covered(C, I - 1, J) != covered(C, I, J))
                for (int k = 0; k < 3; k++)
                    C->M[XF(C, 3 * I, 3 * J + k)] = P->M[XF(P, I0 + I, J0 + J)];
    for (int J = 0; J <= fh; J++)                /* y-faces: between parent cells (I, J-1) and (I, J) */
        for (int I = 0; I < fw; I++)
            if (covered(C, I, J - 1) != covered(C, I, J))
                for (int k = 0; k < 3; k++)
                    C->N[YF(C, 3 * I + k, 3 * J)] = P->N[YF(P, I0 + I, J0 + J)];
}

/* ------------------------------------------------------------------------ */
/* Output maxima (Sec. IV-A, end of the iteration): the highest water level on
 * sea cells (h > 0) and the deepest inundation D = h + eta on land cells. */
void ora_max(ora_domain *d, int l)
{
    ora_level *L = &d->lv[l];
    const size_t n = (size_t)L->nx * (size_t)L->ny;
    #pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; c++) {
        if (L->mask && !L->mask[c]) continue;
        double h = L->h[c], e = L->eta[c];
        double v = (h > 0.0) ? e : h + e;
        if (v > L->zmax[c]) L->zmax[c] = v;
    }
}

/* ------------------------------------------------------------------------ */
/* One time step of the nested domain, in the order of the paper's loop. */
void ora_step(ora_domain *d, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; s++) {
        for (int l = 0; l < d->nlev; l++) ora_mass(d, l);
        for (int l = 1; l < d->nlev; l++) ora_jnz(d, l);
        for (int l = 0; l < d->nlev; l++) ora_momentum(d, l);
        ora_bc_root(d);
        for (int l = 1; l < d->nlev; l++) ora_jnq(d, l);
        for (int l = 0; l < d->nlev; l++) ora_max(d, l);
        d->steps++;
    }
}

/* ------------------------------------------------------------------------ */
/* Initial condition (reading; the paper's fault model is outside the loop):
 * an instantaneous sea-surface displacement s(x,y) sampled at cell centres of
 * every level, on sea cells (h > 0) only; land cells hold eta = -h (no water);
 * a displaced level below the ground is clipped to it.  Fluxes start at zero
 * and the maxima at the t = 0 values.
 * shape 0: Gaussian, s = amp exp(-(u^2+v^2)/2)
 * shape 1: elliptic uplift, s = amp cos^2(pi rho/2) for rho < 1, else 0,
 * where u = x'/a, v = y'/b, rho^2 = u^2 + v^2, (x',y') the offsets from the
 * centre rotated by theta. */
void ora_set_source(ora_domain *d, double xc, double yc, double a, double b,
                    double theta, double amp, int shape)
{
    const double ct = cos(theta), st = sin(theta);
    for (int l = 0; l < d->nlev; l++) {
        ora_level *L = &d->lv[l];
        for (int j = 0; j < L->ny; j++) {
            for (int i = 0; i < L->nx; i++) {
                size_t c = CELL(L, i, j);
                double x = L->ox + ((double)i + 0.5) * L->dx;
                double y = L->oy + ((double)j + 0.5) * L->dx;
                double ddx = x - xc, ddy = y - yc;
                double xp = ddx * ct + ddy * st;
                double yp = -(ddx * st) + ddy * ct;
                double u = xp / a, v = yp / b;
                double rho2 = u * u + v * v;
                double s;
                if (shape == 0) {
                    s = amp * exp(-0.5 * rho2);
                } else {
                    if (rho2 < 1.0) {
                        double cs = cos(0.5 * M_PI * sqrt(rho2));
                        s = amp * (cs * cs);
                    } else {
                        s = 0.0;
                    }
                }
                double h = L->h[c];
                double e = (h > 0.0) ? s : -h;
                if (h + e < 0.0) e = -h;
                L->eta[c] = e;
                L->zmax[c] = (h > 0.0) ? e : h + e;
            }
        }
        memset(L->M, 0, sizeof(double) * (size_t)(L->nx + 1) * (size_t)L->ny);
        memset(L->N, 0, sizeof(double) * (size_t)L->nx * (size_t)(L->ny + 1));
    }
    d->steps = 0;
}

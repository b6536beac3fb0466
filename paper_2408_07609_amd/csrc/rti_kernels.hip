// rti_kernels.hip -- per-phase HIP kernels of the nested long-wave step for
// gfx950 (CDNA4), FP64.  One launch per phase covers every level: blocks of
// 256 threads map to 64x4-cell tiles (64 = one wavefront along a row, so each
// wavefront reads and writes 512 contiguous bytes per field).
//
// Phase order of one step (paper, Sec. IV-A): continuity (Eq. 1) on every
// level -> child-to-parent water level on the footprint rings (Sec. IV-C) ->
// momentum (Eqs. 2-3) on every level, with the root's open/wall sides and the
// running maxima -> parent-to-child fluxes on every child edge.
// Buffers: state in buffer b is read, the new state is written to b^1.
//
// The arithmetic of every formula is written operation by operation in the
// order stated next to it (no reassociation; the library is built with
// -ffp-contract=off so no multiply-add is fused).
#include "rti_internal.h"
#include "rti_device.h"

namespace {
using namespace rti_dev;


struct View {
    const double *h, *eta, *M, *N;
    int nx, ny, P;
};

__device__ __forceinline__ bool xdepth(const View &v, double eps, int i, int j, double &D)
{
    return face_depth(v.h[(i - 1) + v.P * j], v.eta[(i - 1) + v.P * j], v.h[i + v.P * j], v.eta[i + v.P * j], eps, D);
}

__device__ __forceinline__ bool ydepth(const View &v, double eps, int i, int j, double &D)
{
    return face_depth(v.h[i + v.P * (j - 1)], v.eta[i + v.P * (j - 1)], v.h[i + v.P * j], v.eta[i + v.P * j], eps, D);
}

// N at x-face (i,j): (cell i-1's south+north) + (cell i's south+north), / 4.
__device__ __forceinline__ double nbar_x(const View &v, int i, int j)
{
    const double *N = v.N;
    const int P = v.P;
    return 0.25 * ((N[(i - 1) + P * j] + N[(i - 1) + P * (j + 1)]) + (N[i + P * j] + N[i + P * (j + 1)]));
}

// M at y-face (i,j): (cell (i,j-1)'s west+east) + (cell (i,j)'s west+east), / 4.
__device__ __forceinline__ double mbar_y(const View &v, int i, int j)
{
    const double *M = v.M;
    const int P = v.P;
    return 0.25 * ((M[i + P * (j - 1)] + M[(i + 1) + P * (j - 1)]) + (M[i + P * j] + M[(i + 1) + P * j]));
}

// x-momentum at interior x-face (i,j): M_new = ((1-F) M - Pr - A) / (1+F) with
// Pr = (gr D)(eta_i - eta_{i-1}), A = r (X + Y), F = fc sqrt(M^2+Nb^2) D^(-7/3)
// (friction, momentum_update); the quotients by depths use 1/D (over_depth).
__device__ double xmom(const View &v, double eps, double r, double gr, double fc, int i, int j)
{
    double D;
    if (!xdepth(v, eps, i, j, D)) return 0.0;
    const int P = v.P;
    const double m = v.M[i + P * j];
    const double nb = nbar_x(v, i, j);

    const double iD = inv_depth(D);

    double Dm = 0.0, Dp = 0.0;
    const bool okm = (i - 1 >= 1) && xdepth(v, eps, i - 1, j, Dm);
    const bool okp = (i + 1 <= v.nx - 1) && xdepth(v, eps, i + 1, j, Dp);
    const double mm = okm ? v.M[(i - 1) + P * j] : 0.0;
    const double mp = okp ? v.M[(i + 1) + P * j] : 0.0;
    const double X = upwind_diff(m, over_depth(m, m, iD), okm, mm, okm ? over_depth(mm, mm, inv_depth(Dm)) : 0.0,
                                 okp, mp, okp ? over_depth(mp, mp, inv_depth(Dp)) : 0.0);

    double Ds = 0.0, Dn = 0.0;
    const bool oks = (j - 1 >= 0) && xdepth(v, eps, i, j - 1, Ds);
    const bool okn = (j + 1 <= v.ny - 1) && xdepth(v, eps, i, j + 1, Dn);
    const double nbs = oks ? nbar_x(v, i, j - 1) : 0.0;
    const double nbn = okn ? nbar_x(v, i, j + 1) : 0.0;
    const double Y = upwind_diff(nb, over_depth(m, nb, iD), oks, nbs,
                                 oks ? over_depth(v.M[i + P * (j - 1)], nbs, inv_depth(Ds)) : 0.0, okn, nbn,
                                 okn ? over_depth(v.M[i + P * (j + 1)], nbn, inv_depth(Dn)) : 0.0);
    return momentum_update(m, friction(fc, m, nb, D, iD), D, v.eta[i + P * j] - v.eta[(i - 1) + P * j], X, Y, r, gr);
}

// y-momentum at interior y-face (i,j): the mirror of xmom (x<->y, M<->N).
__device__ double ymom(const View &v, double eps, double r, double gr, double fc, int i, int j)
{
    double D;
    if (!ydepth(v, eps, i, j, D)) return 0.0;
    const int P = v.P;
    const double n = v.N[i + P * j];
    const double mb = mbar_y(v, i, j);

    const double iD = inv_depth(D);

    double Ds = 0.0, Dn = 0.0;
    const bool oks = (j - 1 >= 1) && ydepth(v, eps, i, j - 1, Ds);
    const bool okn = (j + 1 <= v.ny - 1) && ydepth(v, eps, i, j + 1, Dn);
    const double ns = oks ? v.N[i + P * (j - 1)] : 0.0;
    const double nn = okn ? v.N[i + P * (j + 1)] : 0.0;
    const double Yd = upwind_diff(n, over_depth(n, n, iD), oks, ns, oks ? over_depth(ns, ns, inv_depth(Ds)) : 0.0,
                                  okn, nn, okn ? over_depth(nn, nn, inv_depth(Dn)) : 0.0);

    double Dw = 0.0, De = 0.0;
    const bool okw = (i - 1 >= 0) && ydepth(v, eps, i - 1, j, Dw);
    const bool oke = (i + 1 <= v.nx - 1) && ydepth(v, eps, i + 1, j, De);
    const double mbw = okw ? mbar_y(v, i - 1, j) : 0.0;
    const double mbe = oke ? mbar_y(v, i + 1, j) : 0.0;
    const double Xd = upwind_diff(mb, over_depth(n, mb, iD), okw, mbw,
                                  okw ? over_depth(v.N[(i - 1) + P * j], mbw, inv_depth(Dw)) : 0.0, oke, mbe,
                                  oke ? over_depth(v.N[(i + 1) + P * j], mbe, inv_depth(De)) : 0.0);
    return momentum_update(n, friction(fc, n, mb, D, iD), D, v.eta[i + P * j] - v.eta[i + P * (j - 1)], Yd, Xd, r, gr);
}

// ---------------------------------------------------------------------------
// Continuity, Eq. (1): eta' = eta - r ((M_{i+1} - M_i) + (N_{j+1} - N_j)),
// then clipped to the ground (h + eta' < 0 -> eta' = -h).
__global__ __launch_bounds__(256) void k_mass(DomainDev d, int b)
{
    const int blk = blockIdx.x;
    const LevelDev &L = level_of(d, level_of_stile(d, blk));
    const int t = blk - L.s_tile_base;
    const int i = (t % L.s_tiles_x) * 64 + (threadIdx.x & 63);
    const int j = (t / L.s_tiles_x) * 4 + (threadIdx.x >> 6);
    if (i >= L.nx || j >= L.ny) return;
    const int P = L.pitch;
    const double *M = static_cast<const double *>(L.M[b]), *N = static_cast<const double *>(L.N[b]);
    const int c = i + P * j;
    double e = L.eta[b][c] - L.r * ((M[c + 1] - M[c]) + (N[c + P] - N[c]));
    const double hh = static_cast<const double *>(L.h)[c];
    if (hh + e < 0.0) e = -hh;
    L.eta[b ^ 1][c] = e;
}

// Child -> parent (Sec. IV-C): each parent cell on the ring of a child's
// footprint (DomainDev::ring_cells, one thread each) := max(mean of the wet
// 3x3 child cells (summed j outer, i inner), parent ground); unchanged when
// none is wet.
__global__ __launch_bounds__(256) void k_jnz(DomainDev d, int b)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d.nring) return;
    const int kp = d.ring_cells[2 * e], ij = d.ring_cells[2 * e + 1];
    const int I = ij & 0xffff, J = ij >> 16;
    const LevelDev &C = d.lv[kp & 0xffff];
    const LevelDev &Pl = d.lv[kp >> 16];
    const double *ce = C.eta[b ^ 1];
    const double *ch = static_cast<const double *>(C.h);
    const int CP = C.pitch;
    double s = 0.0;
    int nw = 0;
    for (int jj = 3 * J; jj < 3 * J + 3; ++jj) {
        for (int ii = 3 * I; ii < 3 * I + 3; ++ii) {
            const double e = ce[ii + CP * jj];
            if (ch[ii + CP * jj] + e > d.eps) { s += e; ++nw; }
        }
    }
    if (nw > 0) {
        const int pc = (C.off_i + I) + Pl.pitch * (C.off_j + J);
        const double v = s / (double)nw;
        const double ground = -static_cast<const double *>(Pl.h)[pc];
        Pl.eta[b ^ 1][pc] = (v > ground) ? v : ground;
    }
}

// Momentum (Eqs. 2-3) for the west x-face and the south y-face of each cell,
// the root's outer faces, and the running maxima of the cell.
__global__ __launch_bounds__(256) void k_momentum(DomainDev d, int b)
{
    const int blk = blockIdx.x;
    const int l = level_of_stile(d, blk);
    const LevelDev &L = level_of(d, l);
    const int t = blk - L.s_tile_base;
    const int i = (t % L.s_tiles_x) * 64 + (threadIdx.x & 63);
    const int j = (t / L.s_tiles_x) * 4 + (threadIdx.x >> 6);
    if (i >= L.nx || j >= L.ny) return;
    const int P = L.pitch;
    const double *Lh = static_cast<const double *>(L.h);
    View v{Lh, L.eta[b ^ 1], static_cast<const double *>(L.M[b]), static_cast<const double *>(L.N[b]), L.nx, L.ny, P};
    double *Mo = static_cast<double *>(L.M[b ^ 1]), *No = static_cast<double *>(L.N[b ^ 1]);
    double *Zm = static_cast<double *>(L.zmax);
    const int c = i + P * j;

    if (i >= 1) Mo[c] = xmom(v, d.eps, L.r, L.gr, d.fc, i, j);
    if (j >= 1) No[c] = ymom(v, d.eps, L.r, L.gr, d.fc, i, j);

    if (l == 0) {
        const double hc = Lh[c], ec = v.eta[c];
        if (i == 0) Mo[c] = d.bc[0] ? 0.0 : radiate(d.g, d.eps, hc, ec, -1.0);
        if (i == L.nx - 1) Mo[c + 1] = d.bc[1] ? 0.0 : radiate(d.g, d.eps, hc, ec, 1.0);
        if (j == 0) No[c] = d.bc[2] ? 0.0 : radiate(d.g, d.eps, hc, ec, -1.0);
        if (j == L.ny - 1) No[c + P] = d.bc[3] ? 0.0 : radiate(d.g, d.eps, hc, ec, 1.0);
    }

    const double hc = Lh[c], e = v.eta[c];
    const double val = (hc > 0.0) ? e : hc + e;
    if (val > Zm[c]) Zm[c] = val;
}

// Parent -> child: every child boundary face takes the flux of the parent
// face it lies on (new fluxes, buffer b^1).  blockIdx.y = child level - 1.
__global__ __launch_bounds__(256) void k_jnq(DomainDev d, int b)
{
    const int c = blockIdx.y + 1;
    const LevelDev &C = level_of(d, c);
    if (C.masked) return;                          // injected from the list (k_inject)
    const LevelDev &Pl = level_of(d, C.parent);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int ny = C.ny, nx = C.nx;
    const int I0 = C.off_i, J0 = C.off_j, fw = nx / 3, fh = ny / 3;
    const int CP = C.pitch, PP = Pl.pitch;
    const double *PM = static_cast<const double *>(Pl.M[b ^ 1]), *PN = static_cast<const double *>(Pl.N[b ^ 1]);
    double *CM = static_cast<double *>(C.M[b ^ 1]), *CN = static_cast<double *>(C.N[b ^ 1]);
    if (k < ny) {
        CM[0 + CP * k] = PM[I0 + PP * (J0 + k / 3)];
    } else if (k < 2 * ny) {
        const int jf = k - ny;
        CM[nx + CP * jf] = PM[(I0 + fw) + PP * (J0 + jf / 3)];
    } else if (k < 2 * ny + nx) {
        const int i = k - 2 * ny;
        CN[i] = PN[(I0 + i / 3) + PP * J0];
    } else if (k < 2 * ny + 2 * nx) {
        const int i = k - 2 * ny - nx;
        CN[i + CP * ny] = PN[(I0 + i / 3) + PP * (J0 + fh)];
    }
}

// Parent -> child on the boundary of masked children (Sec. IV-A, the flux
// exchange): one thread per parent face between a covered and an uncovered
// parent cell copies its new flux per unit width to the 3 child faces on it.
template <typename F>
__global__ __launch_bounds__(256) void k_inject(DomainDev d, int b)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d.ninject) return;
    const int4 q = reinterpret_cast<const int4 *>(d.inject)[e];
    const LevelDev &C = d.lv[q.x & 0xffff];
    const LevelDev &Pl = d.lv[q.x >> 16];
    if (q.y == 0) {
        const F v = static_cast<const F *>(Pl.M[b ^ 1])[q.w];
        F *cm = static_cast<F *>(C.M[b ^ 1]);
        cm[q.z] = v;
        cm[q.z + C.pitch] = v;
        cm[q.z + 2 * C.pitch] = v;
    } else {
        const F v = static_cast<const F *>(Pl.N[b ^ 1])[q.w];
        F *cn = static_cast<F *>(C.N[b ^ 1]);
        cn[q.z] = v;
        cn[q.z + 1] = v;
        cn[q.z + 2] = v;
    }
}

// Any non-finite water level or flux in buffer b sets *flag.
template <typename F>
__global__ __launch_bounds__(256) void k_finite(DomainDev d, int b, int *flag)
{
    const int blk = blockIdx.x;
    const LevelDev &L = level_of(d, level_of_stile(d, blk));
    const int t = blk - L.s_tile_base;
    const int i = (t % L.s_tiles_x) * 64 + (threadIdx.x & 63);
    const int j = (t / L.s_tiles_x) * 4 + (threadIdx.x >> 6);
    if (i >= L.nx || j >= L.ny) return;
    const int c = i + L.pitch * j;
    const bool bad = !isfinite(L.eta[b][c]) || !isfinite((double)static_cast<const F *>(L.M[b])[c])
                     || !isfinite((double)static_cast<const F *>(L.N[b])[c]);
    if (bad) atomicOr(flag, 1);
}

__global__ void k_zero_int(int *p, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0;
}

// Initial state of one level at t = 0: water level from the depth (and the
// source, when shape >= 0), both eta buffers and the maxima.  Sea cells (h > 0)
// take the displacement of the source (paper Sec. IV-A input; the shapes of
// rti_source), land keeps eta = -h, and a level below the ground is clipped
// to it; the maxima start at the initial values (sea: eta, land: h + eta).
template <typename F>
__global__ __launch_bounds__(256) void k_init_level(LevelDev L, InitSource sp)
{
    const int i = (int)(blockIdx.x * 64 + (threadIdx.x & 63));
    const int j = (int)(blockIdx.y * 4 + (threadIdx.x >> 6));
    if (i >= L.nx || j >= L.ny) return;
    const int c = i + L.pitch * j;
    const double h = (double)static_cast<const F *>(L.h)[c];
    double s = 0.0;
    if (sp.shape >= 0) {
        const double x = sp.ox + ((double)i + 0.5) * sp.dx;
        const double y = sp.oy + ((double)j + 0.5) * sp.dx;
        const double ddx = x - sp.xc, ddy = y - sp.yc;
        const double xp = ddx * sp.ct + ddy * sp.st;
        const double yp = -(ddx * sp.st) + ddy * sp.ct;
        const double u = xp / sp.a, v = yp / sp.b;
        const double rho2 = u * u + v * v;
        if (sp.shape == 0) {
            s = sp.amp * exp(-0.5 * rho2);
        } else if (rho2 < 1.0) {
            const double cs = cos(0.5 * M_PI * sqrt(rho2));
            s = sp.amp * (cs * cs);
        }
    }
    double eta = (h > 0.0) ? s : -h;
    if (h + eta < 0.0) eta = -h;
    L.eta[0][c] = eta;
    L.eta[1][c] = eta;
    static_cast<F *>(L.zmax)[c] = (F)((h > 0.0) ? eta : h + eta);
}

// The FP64 operations the step is built from, element by element, for the
// tests that compare them with IEEE binary64: op 0 cube root (cbrt_rn), 1 the
// reciprocal of a depth (inv_depth), 2 the square root.
__global__ __launch_bounds__(256) void k_probe_math(int op, const double *x, double *y, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const double v = x[k];
    y[k] = (op == 0) ? cbrt_rn(v) : (op == 1) ? inv_depth(v) : sqrt(v);
}

// A plain stream over n doubles: `reads` input arrays and `writes` output
// arrays, out_j[i] = (j + 1) * (sum of the inputs at i), one element per
// lane per array (the access width of the step's kernels), a grid-stride
// loop over a fixed grid.  It measures the HBM rate that a kernel moving the
// step's mix of reads and writes can reach on this GPU; one read and one
// write is a plain copy (k_stream_copy).
struct StreamArgs {
    const double *in[8];
    double *out[8];
};

__global__ __launch_bounds__(256) void k_stream_copy(const double *in, double *out, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(&in[i]), &out[i]);
}

__global__ __launch_bounds__(256) void k_stream_probe(StreamArgs a, int reads, int writes, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        double s = 0.0;
        for (int k = 0; k < reads; ++k) s += __builtin_nontemporal_load(&a.in[k][i]);
        for (int k = 0; k < writes; ++k) __builtin_nontemporal_store(s * (double)(k + 1), &a.out[k][i]);
    }
}

}  // namespace

hipError_t launch_stream_probe(const double *const *in, int reads, double *const *out, int writes, int64_t n,
                               int grid, hipStream_t s)
{
    StreamArgs a{};
    for (int k = 0; k < reads; ++k) a.in[k] = in[k];
    for (int k = 0; k < writes; ++k) a.out[k] = out[k];
    if (n <= 0) return hipSuccess;
    if (reads == 1 && writes == 1)       // a plain copy (a kernel of its own: it calibrates the HBM counters)
        hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, s, in[0], out[0], n);
    else
        hipLaunchKernelGGL(k_stream_probe, dim3(grid), dim3(256), 0, s, a, reads, writes, n);
    return hipGetLastError();
}

hipError_t launch_probe_math(int op, const double *x, double *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_math, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, op, x, y, n);
    return hipGetLastError();
}

hipError_t launch_mass(const DomainDev &d, int b, hipStream_t s)
{
    hipLaunchKernelGGL(k_mass, dim3(d.s_ntiles), dim3(256), 0, s, d, b);
    return hipGetLastError();
}

hipError_t launch_jnz(const DomainDev &d, int b, hipStream_t s)
{
    if (d.nlev < 2) return hipSuccess;
    if (d.nring == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jnz, dim3((d.nring + 255) / 256), dim3(256), 0, s, d, b);
    return hipGetLastError();
}

hipError_t launch_momentum(const DomainDev &d, int b, hipStream_t s)
{
    hipLaunchKernelGGL(k_momentum, dim3(d.s_ntiles), dim3(256), 0, s, d, b);
    return hipGetLastError();
}

hipError_t launch_jnq(const DomainDev &d, int b, hipStream_t s)
{
    if (d.nlev < 2) return hipSuccess;
    hipLaunchKernelGGL(k_jnq, dim3((d.max_edge + 255) / 256, d.nlev - 1), dim3(256), 0, s, d, b);
    return hipGetLastError();
}

hipError_t launch_inject(const DomainDev &d, int b, hipStream_t s)
{
    if (d.ninject == 0) return hipSuccess;
    const dim3 grid((d.ninject + 255) / 256);
    if (d.bulk32)
        hipLaunchKernelGGL(k_inject<float>, grid, dim3(256), 0, s, d, b);
    else
        hipLaunchKernelGGL(k_inject<double>, grid, dim3(256), 0, s, d, b);
    return hipGetLastError();
}

hipError_t launch_finite_check(const DomainDev &d, int b, int *flag, hipStream_t s)
{
    if (d.bulk32)
        hipLaunchKernelGGL(k_finite<float>, dim3(d.s_ntiles), dim3(256), 0, s, d, b, flag);
    else
        hipLaunchKernelGGL(k_finite<double>, dim3(d.s_ntiles), dim3(256), 0, s, d, b, flag);
    return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_init_level(const LevelDev &L, int bulk32, const InitSource &sp, hipStream_t s)
{
    const dim3 grid((L.nx + 63) / 64, (L.ny + 3) / 4);
    if (bulk32)
        hipLaunchKernelGGL(k_init_level<float>, grid, dim3(256), 0, s, L, sp);
    else
        hipLaunchKernelGGL(k_init_level<double>, grid, dim3(256), 0, s, L, sp);
    return hipGetLastError();
}

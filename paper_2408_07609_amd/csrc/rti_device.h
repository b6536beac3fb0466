// rti_device.h -- device helpers shared by the per-phase and the fused
// kernels: the wet/dry face rule, the upwind difference, the open side.
// Each is written operation by operation in a fixed order (the library is
// built with -ffp-contract=off, so no multiply-add is fused).
#pragma once

#include <hip/hip_runtime.h>

namespace rti_dev {

// Wet/dry rule of a face between cells A and B: both wet -> D = (hA+hB)/2 +
// (eA+eB)/2; one wet (say A) -> flux only if eA > -hB, D = eA + hB; both dry
// -> none; and none whenever D <= eps.
__device__ __forceinline__ bool face_depth(double ha, double ea, double hb, double eb, double eps, double &D)
{
    // Every candidate is formed and the rule picks one (no branches: the
    // lanes of a wavefront take different cases).
    const bool wa = ha + ea > eps, wb = hb + eb > eps;
    const double Dboth = 0.5 * (ha + hb) + 0.5 * (ea + eb);
    const double Da = ea + hb, Db = eb + ha;
    const bool both = wa & wb;
    const bool only_a = wa & !wb & (ea > -hb);
    const bool only_b = wb & !wa & (eb > -ha);
    D = both ? Dboth : (only_a ? Da : Db);
    return (both | only_a | only_b) & (D > eps);
}

// First-order upwind difference of a face momentum flux v along one axis;
// s carries the velocity sign at the face, (m) the neighbour behind, (p) the
// one ahead.  A face without flow takes the flux of neighbours flowing in.
template <typename F>
__device__ __forceinline__ F upwind_diff(F s, F v, bool okm, F sm, F vm, bool okp, F sp, F vp)
{
    // One subtraction of selected operands: s > 0 takes v - vm, s < 0 takes
    // vp - v, s == 0 takes c - a (c = vp if that face flows in, a = vm if that
    // one does; c - a is exactly (-a) + c), and a missing neighbour gives 0 - 0.
    const bool pos = s > F(0), neg = s < F(0);
    const bool l_v = pos & okm;                              // lhs = v
    const bool l_vp = (neg & okp) | (!pos & !neg & okp & (sp < F(0)));   // lhs = vp
    const bool r_vm = l_v | (!pos & !neg & okm & (sm > F(0)));           // rhs = vm
    const bool r_v = neg & okp;                              // rhs = v
    const F lhs = l_v ? v : (l_vp ? vp : F(0));
    const F rhs = r_vm ? vm : (r_v ? v : F(0));
    return lhs - rhs;
}

// Open side of the root: flux = sign * (sqrt(g h) * eta) of the boundary cell;
// none when the cell is land or dry.
__device__ __forceinline__ double radiate(double g, double eps, double h, double e, double sign)
{
    if (!(h > 0.0) || !(h + e > eps)) return 0.0;
    const double c = sqrt(g * h);
    return sign * (c * e);
}

// 1/x: the hardware reciprocal refined by one Newton step (x is a positive
// depth or 1 + F, far from denormals).
__device__ __forceinline__ double recip(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}

// x^(-1/3) for x > 0: a binary32 estimate z = 2^(-log2(x)/3) (relative error
// d below 1e-6), then one correction of second order.  With e = 1 - x z^3
// (about -3d), the exact value is z (1 - e)^(-1/3) = z (1 + e/3 + 2e^2/9 +
// O(e^3)); the dropped O(e^3) term is below 1e-17 relative, so the result is
// within about 1.5 ulp of binary64.
__device__ __forceinline__ double rcbrt(double x)
{
    const double z = (double)__builtin_amdgcn_exp2f(-0.333333333f * __builtin_amdgcn_logf((float)x));
    const double z3 = (z * z) * z;
    const double e = fma(-x, z3, 1.0);
    const double c = fma(e, 2.0 / 9.0, 1.0 / 3.0);
    return fma(z * e, c, z);
}
__device__ __forceinline__ float rcbrt(float x)
{
    float z = __builtin_amdgcn_exp2f(-0.333333333f * __builtin_amdgcn_logf(x));
    const float z3 = (z * z) * z;
    return (z * (4.0f - x * z3)) * (1.0f / 3.0f);
}

// sqrt(x) for x >= 0 (0 for x = 0): the hardware reciprocal square root y
// refined by one Goldschmidt step on (g, h) = (x y, y/2) and one residual
// correction g += (x - g^2) h; within about 1 ulp of the rounded root.
__device__ __forceinline__ double sqrt_nonneg(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    return (x > 0.0) ? g : 0.0;
}
__device__ __forceinline__ float sqrt_nonneg(float x) { return sqrtf(x); }

// Momentum flux quantity a*b/D given 1/D.
template <typename F>
__device__ __forceinline__ F over_depth(F a, F b, F invD)
{
    return (a * b) * invD;
}

// New flux of an active face: ((1-F) f - Pr - A) / (1+F) with Pr = (gr D) de,
// A = r (along + cross) and the semi-implicit Manning factor
// F = (dt/2) g n^2 sqrt(f^2 + cr^2) / D^(7/3), D^(-7/3) = (D^(-1/3))^7.
template <typename F>
__device__ __forceinline__ F momentum_update(F f, F cr, F D, F de, F along, F cross, F r, F gr, F fc)
{
    const F Pr = (gr * D) * de;
    const F A = r * (along + cross);
    const F z = rcbrt(D);
    const F z2 = z * z;
    const F z7 = (z2 * z2) * (z2 * z);
    const F Fr = (fc * sqrt_nonneg(f * f + cr * cr)) * z7;
    return (((F(1) - Fr) * f - Pr) - A) * recip(F(1) + Fr);
}

}  // namespace rti_dev

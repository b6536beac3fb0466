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

// FP32-bulk helpers.  1/x: the hardware reciprocal refined by one Newton
// step (x is a positive depth or 1 + F, far from denormals).
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}

// x^(-1/3) for x > 0 in binary32: 2^(-log2(x)/3) and one Newton step.
__device__ __forceinline__ float rcbrt(float x)
{
    float z = __builtin_amdgcn_exp2f(-0.333333333f * __builtin_amdgcn_logf(x));
    const float z3 = (z * z) * z;
    return (z * (4.0f - x * z3)) * (1.0f / 3.0f);
}

__device__ __forceinline__ float sqrt_nonneg(float x) { return sqrtf(x); }

// ---------------------------------------------------------------------------
// FP64: correctly rounded operations only, so that every result is the one
// fixed double that IEEE binary64 defines.  1/x and sqrt are the language's
// operators (IEEE division and square root on gfx950); the cube root, which
// has no correctly rounded library form, is cbrt_rn below.

// Is ((lo + hi) / 2)^3 < a, exactly?  For adjacent doubles lo < hi in
// [0.5, 2) and a in [0.5, 4): such doubles are integer multiples of 2^-53, so
// lo + hi = K 2^-53 with K < 2^55, the midpoint is K 2^-54, and a = A 2^-53
// with A < 2^55.  The test is K^3 < A 2^109, on 192-bit integers (three
// 64-bit words).  K^3 is odd and A 2^109 even, so they never tie.
__device__ __forceinline__ bool midpoint_cube_below(double lo, double hi, double a)
{
    const uint64_t K = (uint64_t)(lo * 0x1p53) + (uint64_t)(hi * 0x1p53);
    const uint64_t A = (uint64_t)(a * 0x1p53);
    const uint64_t k2l = K * K, k2h = __umul64hi(K, K);             // K^2 = k2h 2^64 + k2l, k2h < 2^46
    const uint64_t l_lo = k2l * K, l_hi = __umul64hi(k2l, K);        // k2l K
    const uint64_t h_lo = k2h * K, h_hi = __umul64hi(k2h, K);        // k2h K, h_hi < 2^37
    const uint64_t w1 = h_lo + l_hi;                                 // K^3 = w2 2^128 + w1 2^64 + l_lo
    const uint64_t w2 = h_hi + (w1 < l_hi ? 1u : 0u);
    const uint64_t b2 = A >> 19, b1 = A << 45;                       // A 2^109 = b2 2^128 + b1 2^64
    (void)l_lo;
    return (w2 < b2) || (w2 == b2 && w1 < b1);
}

// Cube root, correctly rounded (the double nearest to the real root), on the
// reduced range: x = a 2^(3q) with a in [0.5, 4), so that the root of a and
// its neighbours lie in [0.5, 2) as midpoint_cube_below needs.  An estimate
// z of a^(-1/3) from binary32 log2/exp2 (relative error about 2^-22) gets a
// correction of second order: with e = 1 - a z^3, a^(-1/3) = z (1 - e)^(-1/3)
// = z (1 + e/3 + 2e^2/9 + O(e^3)), leaving an error near 2^-52.  y = a z^2
// is then within a few ulps of the root, and d = (a - y^3) / (3 y^2), with the
// residual a - y^3 formed from the exact products y^2 = p + pl and
// p y = t + tl, is the distance from y to the root to about 2^-50 relative.
// s = y + d rounded is the nearest double unless the root lies within 2^-21
// ulp of the midpoint between s and its neighbour on that side (err, the
// exact rounding error of y + d, says how close); that case is settled by
// the exact test.  Any positive normal x.
__device__ __forceinline__ double cbrt_rn_reduced(double x)
{
    const int ex = __builtin_amdgcn_frexp_exp(x);                    // x = m 2^ex, m in [0.5, 1)
    const int q = (ex + 1023) / 3 - 341;                             // floor(ex / 3)
    const double a = __builtin_amdgcn_ldexp(__builtin_amdgcn_frexp_mant(x), ex - 3 * q);
    double z = (double)__builtin_amdgcn_exp2f(-0.333333333f * __builtin_amdgcn_logf((float)a));
    const double e = fma(-a, (z * z) * z, 1.0);
    z = fma(z * e, fma(e, 2.0 / 9.0, 1.0 / 3.0), z);
    const double y = (a * z) * z;
    const double p = y * y, pl = fma(y, y, -p);
    const double t = p * y, tl = fma(p, y, -t);
    const double res = ((a - t) - tl) - pl * y;
    const double d = res * ((z * z) * (1.0 / 3.0));
    const double s = y + d;
    const double err = d - (s - y);                                  // exact (|d| << |y|)
    const long long bits = __double_as_longlong(s);
    const double nb = __longlong_as_double(err > 0.0 ? bits + 1 : bits - 1);
    const double half = 0.5 * (nb - s);                              // exact, signed
    double r = s;
    if (fabs(err) > fabs(half) * (1.0 - 0x1p-20)) {
        const bool above_mid = (err > 0.0) ? midpoint_cube_below(s, nb, a) : midpoint_cube_below(nb, s, a);
        r = (err > 0.0) ? (above_mid ? nb : s) : (above_mid ? s : nb);
    }
    return __builtin_amdgcn_ldexp(r, q);
}

// The cube root of the friction term: the same steps without the range
// reduction for x in [2^-120, 2^120] (where the binary32 estimate and the
// exact products neither overflow nor underflow, and the relative error
// bounds above do not depend on the scale), falling back to the reduced
// form outside that range and whenever the root lies too near a midpoint
// for the fast decision.  Correctly rounded for every positive normal x.
// Outside [2^-120, 2^120] the unreduced steps may produce anything (an
// infinite or zero estimate); they are computed regardless and their result
// discarded, which costs less than selecting a safe operand first.
__device__ __forceinline__ double cbrt_rn(double x)
{
    double z = (double)__builtin_amdgcn_exp2f(-0.333333333f * __builtin_amdgcn_logf((float)x));
    const double e = fma(-x, (z * z) * z, 1.0);
    z = fma(z * e, fma(e, 2.0 / 9.0, 1.0 / 3.0), z);
    const double y = (x * z) * z;
    const double p = y * y, pl = fma(y, y, -p);
    const double t = p * y, tl = fma(p, y, -t);
    const double res = ((x - t) - tl) - pl * y;
    const double d = res * ((z * z) * (1.0 / 3.0));
    const double s = y + d;
    const double err = d - (s - y);
    const long long bits = __double_as_longlong(s);
    const double nb = __longlong_as_double(err > 0.0 ? bits + 1 : bits - 1);
    const bool slow = !(x >= 0x1p-120 && x <= 0x1p120) || (fabs(err) > fabs(0.5 * (nb - s)) * (1.0 - 0x1p-20));
    double r = s;
    if (slow) r = cbrt_rn_reduced(x);
    return r;
}

// Reciprocal of a face depth, correctly rounded (the IEEE quotient 1/D) for
// D in [2^-767, 2^1022): the steps of the correctly rounded division --
// hardware reciprocal estimate, two Newton steps, the quotient, its exact
// residual and the final correction -- without its operand scaling and
// special-value fix-up, which are identities on that range (no operand or
// result near the limits of the format).  A face depth lies there: an active
// face's exceeds the dry threshold (at least 1e-12, checked at create), an
// inactive face's is 1, and depths are far below 2^1022 m in any state the
// watchdog has not flagged.
__device__ __forceinline__ double inv_depth(double D)
{
    double r = __builtin_amdgcn_rcp(D);
    r = fma(r, fma(-D, r, 1.0), r);
    r = fma(r, fma(-D, r, 1.0), r);
    return fma(fma(-D, r, 1.0), r, r);
}
__device__ __forceinline__ float inv_depth(float D) { return recip(D); }

// Momentum flux quantity a*b/D given 1/D.
template <typename F>
__device__ __forceinline__ F over_depth(F a, F b, F invD)
{
    return (a * b) * invD;
}

// Semi-implicit Manning factor of a face, F = fc sqrt(f^2 + c^2) D^(-7/3)
// (fc = dt/2 g n^2, f the face's flux, c the cross flux averaged to the face).
// FP64: D^(-7/3) = iD^2 cbrt(iD), iD = 1/D, every operation correctly rounded.
// FP32-bulk: D^(-7/3) = z^7 with z = D^(-1/3).
__device__ __forceinline__ double friction(double fc, double f, double c, double D, double iD)
{
    (void)D;
    return (fc * sqrt(f * f + c * c)) * ((iD * iD) * cbrt_rn(iD));
}
__device__ __forceinline__ float friction(float fc, float f, float c, float D, float iD)
{
    (void)iD;
    const float z = rcbrt(D);
    const float z2 = z * z;
    return (fc * sqrt_nonneg(f * f + c * c)) * ((z2 * z2) * (z2 * z));
}

// New flux of an active face: ((1-Fr) f - Pr - A) / (1+Fr) with Pr = (gr D) de,
// A = r (along + cross) and Fr the Manning factor (friction).  FP64 divides;
// FP32-bulk multiplies by the refined reciprocal.
__device__ __forceinline__ double momentum_update(double f, double Fr, double D, double de, double along,
                                                  double cross, double r, double gr)
{
    const double Pr = (gr * D) * de;
    const double A = r * (along + cross);
    return (((1.0 - Fr) * f - Pr) - A) / (1.0 + Fr);
}
__device__ __forceinline__ float momentum_update(float f, float Fr, float D, float de, float along,
                                                 float cross, float r, float gr)
{
    const float Pr = (gr * D) * de;
    const float A = r * (along + cross);
    return (((1.0f - Fr) * f - Pr) - A) * recip(1.0f + Fr);
}

}  // namespace rti_dev

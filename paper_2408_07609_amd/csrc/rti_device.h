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
    const bool wa = ha + ea > eps, wb = hb + eb > eps;
    if (wa && wb) {
        D = 0.5 * (ha + hb) + 0.5 * (ea + eb);
    } else if (wa) {
        if (!(ea > -hb)) return false;
        D = ea + hb;
    } else if (wb) {
        if (!(eb > -ha)) return false;
        D = eb + ha;
    } else {
        return false;
    }
    return D > eps;
}

// First-order upwind difference of a face momentum flux v along one axis;
// s carries the velocity sign at the face, (m) the neighbour behind, (p) the
// one ahead.  A face without flow takes the flux of neighbours flowing in.
template <typename F>
__device__ __forceinline__ F upwind_diff(F s, F v, bool okm, F sm, F vm, bool okp, F sp, F vp)
{
    if (s > F(0)) return okm ? v - vm : F(0);
    if (s < F(0)) return okp ? vp - v : F(0);
    const F a = (okm && sm > F(0)) ? vm : F(0);
    const F c = (okp && sp < F(0)) ? vp : F(0);
    return (-a) + c;
}

// Open side of the root: flux = sign * (sqrt(g h) * eta) of the boundary cell;
// none when the cell is land or dry.
__device__ __forceinline__ double radiate(double g, double eps, double h, double e, double sign)
{
    if (!(h > 0.0) || !(h + e > eps)) return 0.0;
    const double c = sqrt(g * h);
    return sign * (c * e);
}

}  // namespace rti_dev

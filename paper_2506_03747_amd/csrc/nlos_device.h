// Device-side building blocks shared by the forward kernels and the bin
// export hook, so both decide every bin with the same instructions.
//
// Compiled with -ffp-contract=off: every fused multiply-add below is written
// out (fmaf); nothing else is contracted, so the fp64 re-evaluation follows
// the stated operation order exactly.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nlos_internal.h"

namespace nlos {

// Canonical fp32 coordinate of cell i: fp32(a0 + (i + 0.5) * step) in fp64.
__device__ __forceinline__ float canon(const Axis& ax, int i)
{
    return (float)(ax.a0 + ((double)i + 0.5) * ax.step);
}

// Device leg of wall point (wx, wy): the device sits at (cx, cy, s).
// Path offset L - s and weight (s / L)^3; s = 0 -> no leg (0, 1).
__device__ __forceinline__ void device_leg(float wx, float wy, double cx, double cy, double s,
                                           double* off, double* g)
{
    if (s > 0.0) {
        const double ex = (double)wx - cx, ey = (double)wy - cy;
        const double L = sqrt((ex * ex + ey * ey) + s * s);
        const double q = s / L;
        *off = L - s;
        *g = q * q * q;
    } else {
        *off = 0.0;
        *g = 1.0;
    }
}

// Exact bin: floor of ((r_l + r_d) + o) * inv evaluated in fp64 from the fp32
// coordinates, in this order, no contraction.  Clamped to the int32 range.
__device__ __forceinline__ int32_t exact_bin(float px, float py, float pz, float wlx, float wly,
                                             float wdx, float wdy, double o, double inv,
                                             double* u_out = nullptr)
{
    const double alx = (double)px - (double)wlx, aly = (double)py - (double)wly;
    const double alz = (double)pz;
    const double r_l = sqrt((alx * alx + aly * aly) + alz * alz);
    const double adx = (double)px - (double)wdx, ady = (double)py - (double)wdy;
    const double r_d = sqrt((adx * adx + ady * ady) + alz * alz);
    const double u = ((r_l + r_d) + o) * inv;
    if (u_out) *u_out = u;
    const double kf = floor(u);
    if (kf < -2147483648.0) return INT32_MIN;
    if (kf > 2147483647.0) return INT32_MAX;
    return (int32_t)kf;
}

// ---------------------------------------------------------------------------
// fp32 fast path.  A lane holds one patch.  Per patch constants:
struct PatchC {
    float px, py, pz2;
    float ap;          // a / pz^4 (cosines) or a (no cosines)
    float mnxs, mnys;  // -n_x pz^3, -n_y pz^3
    float c0s;         // -n_z pz^4
};

__device__ __forceinline__ PatchC patch_consts(float4 A, float4 B, bool cosines)
{
    PatchC c;
    c.px = A.x;
    c.py = A.y;
    const float pz = A.z;
    c.pz2 = pz * pz;
    if (cosines) {
        const float pz3 = c.pz2 * pz;
        c.ap = A.w * __builtin_amdgcn_rcpf(c.pz2 * c.pz2);   // weight only: 1 ulp is ample
        c.mnxs = -B.x * pz3;
        c.mnys = -B.y * pz3;
        c.c0s = -B.z * (pz3 * pz);
    } else {
        c.ap = A.w;
        c.mnxs = c.mnys = c.c0s = 0.f;
    }
    return c;
}

// Column (wall x) and row (wall y) terms of a leg: with dx = px - wx,
//   cx2 = dx^2 + pz^2,  ax = -n_x pz^3 dx - n_z pz^4
//   cy2 = dy^2,         by = -n_y pz^3 dy
// so that r^2 = cx2 + cy2 and pz^3 * n.(w - p) = ax + by.
__device__ __forceinline__ void col_terms(const PatchC& c, float wx, float* cx2, float* ax)
{
    const float dx = c.px - wx;
    *cx2 = fmaf(dx, dx, c.pz2);
    *ax = fmaf(c.mnxs, dx, c.c0s);
}

__device__ __forceinline__ void row_terms(const PatchC& c, float wy, float* cy2, float* by)
{
    const float dy = c.py - wy;
    *cy2 = dy * dy;
    *by = c.mnys * dy;
}

// One leg from its column/row terms: distance (times a scale folded into the
// arrival), reciprocal fourth power and the clamped cosine product
//   q = clamp(pz^3 n.(w-p) / r^4, 0, 1) = cos_wall cos_patch (pz / r)^2.
struct Leg {
    float rr;   // r
    float ri2;  // 1 / r^2
    float ri4;  // 1 / r^4
    float q;    // cosine factor in [0, 1]
};

__device__ __forceinline__ Leg leg_eval(float cx2, float cy2, float ax, float by, bool cosines)
{
    Leg l;
    const float r2 = cx2 + cy2;
    const float ri = __builtin_amdgcn_rsqf(r2);
    l.rr = r2 * ri;
    l.ri2 = ri * ri;
    l.ri4 = l.ri2 * l.ri2;
    l.q = cosines ? __builtin_amdgcn_fmed3f((ax + by) * l.ri4, 0.0f, 1.0f) : 1.0f;
    return l;
}

// The same for a record whose coordinates are multiplied by sig (bins per
// metre of one leg) before anything else, with the arrival offset folded in:
// rr = r + off in bins by a single fma.  q is unchanged (its numerator and
// r^4 both carry sig^4); ri2, ri4 and PatchC::ap carry sig^-2, sig^-4 and
// sig^-4, which the caller folds into its fixed-point scale.
__device__ __forceinline__ PatchC patch_consts_scaled(float4 A, float4 B, bool cosines, float sig)
{
    A.x *= sig;
    A.y *= sig;
    A.z *= sig;
    return patch_consts(A, B, cosines);
}

__device__ __forceinline__ Leg leg_eval_at(float cx2, float cy2, float ax, float by, float off, bool cosines)
{
    Leg l;
    const float r2 = cx2 + cy2;
    const float ri = __builtin_amdgcn_rsqf(r2);
    l.rr = fmaf(r2, ri, off);
    l.ri2 = ri * ri;
    l.ri4 = l.ri2 * l.ri2;
    l.q = cosines ? __builtin_amdgcn_fmed3f((ax + by) * l.ri4, 0.0f, 1.0f) : 1.0f;
    return l;
}

// Fast-path decision on w = u + delta (delta folded into the offset):
// k = floor(w); when frac(w) >= 2 delta the bin is k for certain, else the
// pair is re-evaluated in fp64 (k - 1 or k).
struct Decision {
    int32_t k;
    bool sure;
};

__device__ __forceinline__ Decision decide(float w, float two_delta)
{
    Decision d;
    d.k = (int32_t)w;   // w > 0: truncation is floor
    d.sure = __builtin_amdgcn_fractf(w) >= two_delta;
    return d;
}

}  // namespace nlos

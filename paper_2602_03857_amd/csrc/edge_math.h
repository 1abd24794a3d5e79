// Device arithmetic of the prism vertical-attraction kernel (paper Eq. 1-3).
//
// Two evaluations of the same closed form:
//
//  * psi_f64: the corner function Psi(x, y, z) of Eq. 2 in FP64, used by the
//    plain GRAV_FP64 path, which sums Psi over mesh nodes.
//
//  * edge_segment: the difference S = Psi(x, y, z2) - Psi(x, y, z1) along one
//    vertical mesh edge (z2 = z1 + h), in FP32, written so that no step
//    subtracts two nearly equal numbers.  Summing Eq. 1 over the two vertical
//    corners r = 1, 2 of a prism gives exactly S for each of its four vertical
//    edges, so the prism term is sum_{p,q} (-1)^(p+q) S(edge p,q).
//    Identities used (all exact in real arithmetic):
//      R2 - R1                     = h (z1 + z2) / (R1 + R2)
//      ln(R2 + y) - ln(R1 + y)     = log1p((R2 - R1) / (R1 + y))
//      R1 + y  (y < 0)             = (x^2 + z1^2) / (R1 - y)
//      z2 atan(u2) - z1 atan(u1)   = h atan(u2) + z1 atan((u2 - u1) / (1 + u1 u2))
//      (u2 - u1) / (1 + u1 u2)     = -xy h (z1 + z2)(x^2 + y^2 + z1^2 + z2^2)
//                                     / ((z1 R1 + z2 R2)(z1 z2 R1 R2 + x^2 y^2))
//    with u = xy / (z R).  The last identity needs 1 + u1 u2 > 0, which holds
//    because z1, z2 >= 0 (observations on or above the mesh top).
//
// Singular limits, taken by select (never by multiplying by zero, so that an
// infinite or NaN intermediate of a discarded branch cannot leak):
// x = 0 => the x*ln term is 0; y = 0 => the y*ln term is 0; z1 = 0 => the
// z1*atan term is 0.  These are the continuous limits of Eq. 2.
#pragma once

#include <hip/hip_runtime.h>

namespace grav {

// Per (observation, mesh column) quantities, FP32, from FP64 differences.
struct Column {
    float x, y;      // node column minus observation
    float xx, yy;    // x^2, y^2
    float s;         // x^2 + y^2
    float xy;        // x*y
    bool xnz, ynz;   // x != 0, y != 0
    bool xneg, yneg; // x < 0, y < 0
};

__device__ __forceinline__ Column make_column(double X, double Y, double xo, double yo) {
    Column c;
    c.x = static_cast<float>(X - xo);
    c.y = static_cast<float>(Y - yo);
    c.xx = c.x * c.x;
    c.yy = c.y * c.y;
    c.s = c.xx + c.yy;
    c.xy = c.x * c.y;
    c.xnz = c.x != 0.0f;
    c.ynz = c.y != 0.0f;
    c.xneg = c.x < 0.0f;
    c.yneg = c.y < 0.0f;
    return c;
}

__device__ __forceinline__ float node_radius(const Column &c, float z) {
    return sqrtf(fmaf(z, z, c.s));
}

// S = Psi(x, y, z2) - Psi(x, y, z1) for one vertical edge segment, z2 = z1 + h,
// z1 >= 0, R1 = |(x, y, z1)|, R2 = |(x, y, z2)|.
__device__ __forceinline__ float edge_segment(const Column &c, float z1, float z2, float h,
                                              float R1, float R2) {
    const float hz = h * (z1 + z2);
    const float dR = hz / (R1 + R2);                 // R2 - R1
    const float z1s = z1 * z1;
    // ln(R2 + y) - ln(R1 + y) = log1p(dR / (R1 + y))
    const float denY = c.yneg ? (c.xx + z1s) : (R1 + c.y);
    const float numY = c.yneg ? (R1 - c.y) : 1.0f;
    const float lnY = log1pf(dR * numY / denY);
    // ln(R2 + x) - ln(R1 + x)
    const float denX = c.xneg ? (c.yy + z1s) : (R1 + c.x);
    const float numX = c.xneg ? (R1 - c.x) : 1.0f;
    const float lnX = log1pf(dR * numX / denX);
    // z2 atan(u2) - z1 atan(u1) = h atan(u2) + z1 atan(delta)
    const float zR1 = z1 * R1;
    const float zR2 = z2 * R2;
    const float at2 = atanf(c.xy / zR2);
    const float num = -c.xy * hz * (c.s + z1s + z2 * z2);
    const float den = (zR1 + zR2) * fmaf(zR1, zR2, c.xy * c.xy);
    const float atd = atanf(num / den);
    float S = h * at2;
    S = (z1 > 0.0f) ? fmaf(z1, atd, S) : S;
    S = c.xnz ? fmaf(-c.x, lnY, S) : S;
    S = c.ynz ? fmaf(-c.y, lnX, S) : S;
    return S;
}

// Psi(x, y, z) of Eq. 2 in FP64 (R from Eq. 3); ln(R + y) for y < 0 is taken
// as ln((x^2 + z^2) / (R - y)), the same number without cancellation.
__device__ __forceinline__ double psi_f64(double x, double y, double z) {
    const double xx = x * x, yy = y * y, zz = z * z;
    const double R = sqrt(xx + yy + zz);
    const double t_at = (z != 0.0) ? z * atan((x * y) / (z * R)) : 0.0;
    const double rpy = (y >= 0.0) ? R + y : (xx + zz) / (R - y);
    const double rpx = (x >= 0.0) ? R + x : (yy + zz) / (R - x);
    const double tx = (x != 0.0) ? x * log(rpy) : 0.0;
    const double ty = (y != 0.0) ? y * log(rpx) : 0.0;
    return t_at - tx - ty;
}

}  // namespace grav

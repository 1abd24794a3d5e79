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
//    because z1, z2 >= 0 (observations on or above the mesh top).  By the same
//    addition formula atan(u2) = atan(u1) + atan(delta) with the delta above,
//    so in layers where atan(delta) is cheap (deep layers, below) the angle of
//    the bottom node is carried down the column instead of being evaluated.
//
// Singular limits, taken by select (never by multiplying by zero, so that an
// infinite or NaN intermediate of a discarded branch cannot leak):
// x = 0 => the x*ln term is 0; y = 0 => the y*ln term is 0; z1 = 0 => the
// z1*atan term is 0.  These are the continuous limits of Eq. 2.  In FP32 a
// horizontal offset below kTinyOffset (0.1 mm) is treated as 0, so that its
// square cannot underflow into a zero denominator; the term it drops is
// bounded by |x| * |ln(...)|, below 3e-3 m * (kg/m^3 weight) per segment.
//
// Elementary functions of the FP32 path (all in this file, no library calls):
//  * reciprocal, square root, log2: the gfx950 hardware instructions
//    (v_rcp_f32, v_sqrt_f32, v_log_f32).
//  * log1p(t), t >= 0: u = 1 + t rounded, c = t - (u - 1) its exact rounding
//    error (Sterbenz), log1p(t) = ln(u) + c/u; c/u is replaced by
//    c * max(0, 2 - u), which differs from it by less than 0.5 c for u <= 2
//    and drops it above 2 where c/u < 2^-24 relative to ln(u) >= ln 2.  Where
//    t < 1/4 is guaranteed (deep layers), c/u is replaced by c itself: the
//    difference |c| (u - 1) / u is zero for t <= 2^-24 (then u = 1) and at
//    most 2^-24 (t + 2^-24) < 2^-23 t above, a relative error below 1.2e-7
//    of log1p(t) >= 0.875 t (about 2^-24 once t >> 2^-24).
//  * atan(n/d), d >= 0: r = min(|n|, d) / max(|n|, d) in [0, 1],
//    atan(r) = r P(r^2) with a degree-8 polynomial in r^2 fitted to the
//    relative error of atan on [0, 1] by iteratively reweighted least squares
//    (max relative error 1.4e-7 in FP32), then pi/2 - atan(r) if |n| > d, and
//    the sign of n.
#pragma once

#include <hip/hip_runtime.h>

namespace grav {

namespace fm {

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float log2(float x) { return __builtin_amdgcn_logf(x); }

constexpr float kLn2 = 0.693147180559945309f;
constexpr float kHalfPi = 1.57079632679489662f;

// atan(r) = r * P(r^2) on [0, 1]
constexpr float kAt0 = 1.0f;
constexpr float kAt1 = -0.3333307206630707f;
constexpr float kAt2 = 0.1999262124300003f;
constexpr float kAt3 = -0.142036572098732f;
constexpr float kAt4 = 0.10640984773635864f;
constexpr float kAt5 = -0.07504411041736603f;
constexpr float kAt6 = 0.042692989110946655f;
constexpr float kAt7 = -0.01606959104537964f;
constexpr float kAt8 = 0.002850143937394023f;

// atan(n / d) for d >= 0 (n = d = 0 gives NaN; callers discard it).
__device__ __forceinline__ float atan_ratio(float n, float d) {
    const float a = fabsf(n);
    const float r = fminf(a, d) * rcp(fmaxf(a, d));
    const float r2 = r * r;
    float p = fmaf(kAt8, r2, kAt7);
    p = fmaf(p, r2, kAt6);
    p = fmaf(p, r2, kAt5);
    p = fmaf(p, r2, kAt4);
    p = fmaf(p, r2, kAt3);
    p = fmaf(p, r2, kAt2);
    p = fmaf(p, r2, kAt1);
    p = fmaf(p, r2, kAt0);
    p *= r;
    p = (a > d) ? (kHalfPi - p) : p;
    return copysignf(p, n);
}

// atan(d) for |d| <= 1/8: odd polynomial d Q(d^2), Q of degree 3 fitted like
// the one above on [0, 1/8] (max relative error 8.9e-8 in FP32).
constexpr float kAs0 = 1.0f;
constexpr float kAs1 = -0.33333322405815125f;
constexpr float kAs2 = 0.1999669075012207f;
constexpr float kAs3 = -0.1394471824169159f;

__device__ __forceinline__ float atan_small(float d) {
    const float d2 = d * d;
    float p = fmaf(kAs3, d2, kAs2);
    p = fmaf(p, d2, kAs1);
    p = fmaf(p, d2, kAs0);
    return p * d;
}

// log1p(t) for t >= 0.  kSmall: the caller guarantees t < 1/4, and the
// rounding error c of 1 + t is added without the 1/u factor (error bound in
// the header).
template <bool kSmall = false>
__device__ __forceinline__ float log1p_pos(float t) {
    const float u = 1.0f + t;
    const float c = t - (u - 1.0f);
    if constexpr (kSmall) {
        return fmaf(log2(u), kLn2, c);
    } else {
        const float w = fmaxf(2.0f - u, 0.0f);
        return fmaf(log2(u), kLn2, c * w);
    }
}

}  // namespace fm

constexpr float kTinyOffset = 1.0e-4f;   // metres
constexpr double kDeepRatio = 9.0;       // layer top >= 9 h below the mesh top => "deep"
constexpr double kDeepMinDepth = 1e-3;   // ... and >= 1 mm below it (metres)

// Per (observation, mesh column) quantities, FP32, from FP64 differences.
struct Column {
    float x, y;      // node column minus observation
    float xx, yy;    // x^2, y^2
    float s;         // x^2 + y^2
    float xy;        // x*y
    float xy2;       // (x*y)^2
    bool xnz, ynz;   // |x|, |y| above kTinyOffset
    bool xneg, yneg; // x < 0, y < 0
};

// Column terms from FP32 offsets (x, y) already reduced by column_offset().
__device__ __forceinline__ Column column_from_xy(float x, float y) {
    Column c;
    c.x = x;
    c.y = y;
    c.xnz = x != 0.0f;
    c.ynz = y != 0.0f;
    c.xx = c.x * c.x;
    c.yy = c.y * c.y;
    c.s = c.xx + c.yy;
    c.xy = c.x * c.y;
    c.xy2 = c.xy * c.xy;
    c.xneg = c.x < 0.0f;
    c.yneg = c.y < 0.0f;
    return c;
}

// FP64 coordinate difference rounded to FP32, offsets below kTinyOffset -> 0.
__device__ __forceinline__ float column_offset(double X, double xo) {
    const float x = static_cast<float>(X - xo);
    return fabsf(x) > kTinyOffset ? x : 0.0f;
}

__device__ __forceinline__ Column make_column(double X, double Y, double xo, double yo) {
    return column_from_xy(column_offset(X, xo), column_offset(Y, yo));
}

// Per (observation, mesh node) quantities along a column: depth below the
// observation z >= 0, z^2, distance R and z*R.  The bottom node of one
// segment is the top node of the next.
struct Node {
    float z, zz, R, zR;
};

__device__ __forceinline__ Node make_node(const Column &c, float z) {
    Node n;
    n.z = z;
    n.zz = z * z;
    n.R = fm::sqrt(c.s + n.zz);
    n.zR = z * n.R;
    return n;
}

// S = Psi(x, y, z2) - Psi(x, y, z1) for one vertical edge segment between
// node t (top, depth z1 >= 0) and node b (bottom, z2 = z1 + h).
//
// kDeep: the segment's layer starts at least 9 h (and at least 1 mm) below the
// mesh top.  Then z1 > 0, so x^2 + z1^2, y^2 + z1^2, R1 + |y|, R1 + |x| and
// the atan-difference denominator are all positive for every observation and
// the limit selects of the general path are not needed.  Since
// z1 >= (layer top - mesh top) for every observation on or above the top, and
// the atan-difference argument obeys |delta| <= h (z1 + h) / z1^2 (bound from
// z1 R1 + z2 R2 >= (z1 + z2) R1, x^2 + y^2 + z1^2 + z2^2 <= 2 R2^2, AM-GM on the
// denominator and R2/R1 <= z2/z1), such layers have |delta| <= 10/81 < 1/8 for
// all observations and take atan_small without range reduction.  The log1p
// arguments there stay below 1/4 as well: dR / (R1 + |y|) <= h / z1, and for
// y < 0, dR (R1 + |y|) / (x^2 + z1^2) = dR / (R1 - |y|) <= (z2^2 - z1^2) / z1^2
// = 2 h / z1 + (h / z1)^2 (using R1 - |y| >= z1^2 / (2 R1) and R2 >= R1), at
// most 2/9 + 1/81 when z1 >= 9 h; likewise for x.
template <bool kDeep>
__device__ __forceinline__ void edge_logs(const Column &c, const Node &t, const Node &b, float hz,
                                          float &lnY, float &lnX) {
    // 1/(R1 + y) = (y >= 0) ? 1/(R1 + |y|) : (R1 + |y|)/(x^2 + z1^2) (rationalised
    // for y < 0), likewise for x; a denominator belonging to a discarded log
    // term (x = 0, resp. y = 0) is replaced by 1.
    const float ry = t.R + fabsf(c.y), rx = t.R + fabsf(c.x);
    float denY = c.yneg ? (c.xx + t.zz) : ry;
    float denX = c.xneg ? (c.yy + t.zz) : rx;
    if constexpr (!kDeep) {
        denY = c.xnz ? denY : 1.0f;
        denX = c.ynz ? denX : 1.0f;
    }
    const float numY = c.yneg ? ry : 1.0f;
    const float numX = c.xneg ? rx : 1.0f;
    // dR/(R1 + y) and dR/(R1 + x) with dR = hz / (R1 + R2), one reciprocal
    const float q = hz * fm::rcp((t.R + b.R) * (denY * denX));
    lnY = fm::log1p_pos<kDeep>(q * numY * denX);   // ln(R2 + y) - ln(R1 + y)
    lnX = fm::log1p_pos<kDeep>(q * numX * denY);   // ln(R2 + x) - ln(R1 + x)
}

// atan(delta), delta = (u2 - u1) / (1 + u1 u2).
template <bool kDeep>
__device__ __forceinline__ float edge_atan_delta(const Column &c, const Node &t, const Node &b,
                                                 float hz) {
    const float num = -c.xy * hz * (c.s + t.zz + b.zz);
    const float den = (t.zR + b.zR) * fmaf(t.zR, b.zR, c.xy2);
    return kDeep ? fm::atan_small(num * fm::rcp(den)) : fm::atan_ratio(num, den);
}

// S = h atan(u2) + z1 atan(delta) - x ln(..) - y ln(..)
template <bool kDeep>
__device__ __forceinline__ float edge_assemble(const Column &c, const Node &t, float h, float at2,
                                               float atd, float lnY, float lnX) {
    float S = h * at2;
    if constexpr (kDeep) {
        // z1 > 0 keeps every denominator above zero, so every term is finite
        // and the x = 0, y = 0 limits are the products themselves.
        S = fmaf(t.z, atd, S);
        S = fmaf(-c.x, lnY, S);
        S = fmaf(-c.y, lnX, S);
    } else {
        S = (t.z > 0.0f) ? fmaf(t.z, atd, S) : S;
        S = c.xnz ? fmaf(-c.x, lnY, S) : S;
        S = c.ynz ? fmaf(-c.y, lnX, S) : S;
    }
    return S;
}

// S = Psi(x, y, z2) - Psi(x, y, z1) for one vertical edge segment between
// node t (top, depth z1 >= 0) and node b (bottom, z2 = z1 + h).
//
// kDeep: the segment's layer starts at least 9 h (and at least 1 mm) below the
// mesh top.  Then z1 > 0, so x^2 + z1^2, y^2 + z1^2, R1 + |y|, R1 + |x| and
// the atan-difference denominator are all positive for every observation and
// the limit selects of the general path are not needed.  Since
// z1 >= (layer top - mesh top) for every observation on or above the top, and
// the atan-difference argument obeys |delta| <= h (z1 + h) / z1^2 (bound from
// z1 R1 + z2 R2 >= (z1 + z2) R1, x^2 + y^2 + z1^2 + z2^2 <= 2 R2^2, AM-GM on the
// denominator and R2/R1 <= z2/z1), such layers have |delta| <= 10/81 < 1/8 for
// all observations and take atan_small without range reduction.  The log1p
// arguments there stay below 1/4 as well: dR / (R1 + |y|) <= h / z1, and for
// y < 0, dR (R1 + |y|) / (x^2 + z1^2) = dR / (R1 - |y|) <= (z2^2 - z1^2) / z1^2
// = 2 h / z1 + (h / z1)^2 (using R1 - |y| >= z1^2 / (2 R1) and R2 >= R1), at
// most 2/9 + 1/81 when z1 >= 9 h; likewise for x.
template <bool kDeep = false>
__device__ __forceinline__ float edge_segment(const Column &c, const Node &t, const Node &b,
                                              float h) {
    const float hz = h * (t.z + b.z);
    float lnY, lnX;
    edge_logs<kDeep>(c, t, b, hz, lnY, lnX);
    // z2 atan(u2) - z1 atan(u1) = h atan(u2) + z1 atan(delta)
    const float at2 = fm::atan_ratio(c.xy, b.zR);
    const float atd = edge_atan_delta<kDeep>(c, t, b, hz);
    return edge_assemble<kDeep>(c, t, h, at2, atd, lnY, lnX);
}

// Deep-layer segment with atan(u) carried down the column: on entry A holds
// atan(u1) of the top node, on exit atan(u2) = atan(u1) + atan(delta), the
// addition formula of atan, exact here because u1 u2 = x^2 y^2 / (z1 R1 z2 R2)
// >= 0 keeps both angles on one branch.  This replaces the range-reduced
// atan of the bottom node by one addition; the angle is started once per
// walk with atan_ratio(xy, zR) at its first node.  Since u is monotone in z
// along a column, every delta of a walk has the same sign, so the errors of
// the atan(delta) terms add up to at most their relative error times
// |A_end - A_start| <= pi/2.  T = double accumulates the angle exactly for
// walks of any length; T = float adds one rounding of 2^-24 |A| per layer
// and is for walks of at most 16 layers.
template <typename T>
__device__ __forceinline__ float edge_segment_carry(const Column &c, const Node &t, const Node &b,
                                                    float h, T &A) {
    const float hz = h * (t.z + b.z);
    float lnY, lnX;
    edge_logs<true>(c, t, b, hz, lnY, lnX);
    const float atd = edge_atan_delta<true>(c, t, b, hz);
    A += static_cast<T>(atd);
    return edge_assemble<true>(c, t, h, static_cast<float>(A), atd, lnY, lnX);
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

// Device helpers of the near-surface integrals shared by the plain and the
// learned paths: the cut-cell volume fraction and the Wendland C2 taps.
//
// V is the volume fraction of a cell on the phi > 0 side of the plane
// phi_j + g_j . (y - x_j).  It is evaluated with the case analysis of
// Scardovelli & Zaleski (J. Comput. Phys. 164, 2000) on the normal sorted and
// scaled to unit 1-norm.  Every case is written with bounded ratios (alpha /
// m_k with alpha < m_k, or (alpha - m_2) / m_1 with alpha - m_2 < m_1), so no
// case cancels when one or two normal components vanish; the divisions are
// products with the hardware reciprocals of the m_k (1 ulp each).  All five
// cases are evaluated and the right one selected, which costs less than
// divergent branches over a wavefront whose points fall in different cases.
#pragma once

#include "common.hpp"

namespace sgrid {

__device__ __forceinline__ float sz_volume_below(float alpha, float m1, float m2, float m3) {
    // |{w in [0,1]^3 : m.w < alpha}| for 0 <= m1 <= m2 <= m3, m1 + m2 + m3 = 1
    // and 2^-26 <= alpha <= 1/2 (alpha = fl(x + 1/2) > 0 is a multiple of
    // 2^-26).  A reciprocal is infinite only where m_k = 0 (or is subnormal),
    // and then no case that uses it is the selected one: case A needs
    // m1 > alpha, B m2 > alpha, C and D need alpha < m1 + m2 with alpha >= m2,
    // so m1 > alpha - m2 >= 0 is not absorbed into m2.
    const float i1 = __builtin_amdgcn_rcpf(m1), i2 = __builtin_amdgcn_rcpf(m2), i3 = __builtin_amdgcn_rcpf(m3);
    const float c3 = i3 * (1.0f / 6.0f);
    const float m12 = m1 + m2;
    const float r = alpha * i2;
    // B, m1 <= alpha < m2: the wedge past the m1 vertex plane
    const float vb = (3.0f * r * alpha - 3.0f * r * m1 + (m1 * i2) * m1) * c3;
    // C and D subtract the corners cut off past the m2 (and m3) vertex planes
    const float e2 = alpha - m2, e3 = alpha - m3;
    const float t2 = (e2 * i1) * (e2 * i2) * e2;
    const float t3 = (e3 * i1) * (e3 * i2) * e3;
    const float va = (alpha * i1) * r * (alpha * i3) * (1.0f / 6.0f);   // A, alpha < m1: the corner tetrahedron
    const float vc = vb - t2 * c3;
    const float vd = vb - (t2 + t3) * c3;
    const float ve = (2.0f * alpha - m12) * (0.5f * i3);                // E: a prism over the m3 axis
    float v = m3 < m12 ? vd : ve;
    v = (alpha < m12 && alpha < m3) ? vc : v;
    v = alpha < m2 ? vb : v;
    return alpha < m1 ? va : v;
}

// Fraction of the cube u in [-1/2, 1/2]^3 where a + g.u > 0.
__device__ __forceinline__ float plane_cube_fraction(float a, float gx, float gy, float gz) {
    const float ax = fabsf(gx), ay = fabsf(gy), az = fabsf(gz);
    const float s = ax + ay + az;
    if (!(s > 0.0f)) return a > 0.0f ? 1.0f : (a < 0.0f ? 0.0f : 0.5f);   // no gradient (or NaN)
    const float inv = __builtin_amdgcn_rcpf(s);
    const float alpha = a * inv + 0.5f;   // (a + s/2) / s
    if (alpha >= 1.0f) return 1.0f;
    if (alpha <= 0.0f) return 0.0f;
    // sorted ascending (median by v_med3)
    const float m1 = fminf(fminf(ax, ay), az) * inv;
    const float m2 = __builtin_amdgcn_fmed3f(ax, ay, az) * inv;
    const float m3 = fmaxf(fmaxf(ax, ay), az) * inv;
    // the part above 1/2 by the symmetry w -> 1 - w (1 - alpha is exact there)
    const bool flip = alpha > 0.5f;
    const float vb = sz_volume_below(flip ? 1.0f - alpha : alpha, m1, m2, m3);
    return flip ? 1.0f - vb : vb;
}

// Saturation: the plane lies beyond the cell, |a| > 0.51 |g|_1 (|g|_1 / 2 is
// its reach over the cell; the extra 2 % covers the rounding of the fraction's
// normalisation, 1 ulp in the reciprocal and in the product), so
// plane_cube_fraction returns exactly 1 or 0 there, by the sign of a.  NaN and
// huge gradients are not saturated.
__device__ __forceinline__ bool fraction_saturated(float a, float gx, float gy, float gz) {
    const float s1 = fabsf(gx) + fabsf(gy) + fabsf(gz);
    return fabsf(a) > 0.51f * s1 && s1 < 1e30f;
}

}  // namespace sgrid

namespace sgrid {

// Wendland C2 kernel in units of h (smoothing length h, support 2h): the two
// tap distances of the dual-cell query are sqrt(3)/2 (8 taps) and sqrt(11)/2
// (24 taps).  W(r) and W'(r) / r.
__host__ __device__ __forceinline__ double wendland_u(double r) {
    const double e = 1.0 - 0.5 * r;
    return 21.0 / (16.0 * M_PI) * e * e * e * e * (1.0 + 2.0 * r);
}
__host__ __device__ __forceinline__ double wendland_dr_over_r_u(double r) {
    const double e = 1.0 - 0.5 * r;
    return -105.0 / (16.0 * M_PI) * e * e * e;
}

// The 32 taps of the dual-cell query of data point (i, j, k), over cut
// fractions V(x, y, z) (x, y, z the window points i - 1 .. i + 2 etc.): K_W
// and the three K_grad sums.  A tap at offset o in {-1, 0, 1, 2}^3 has d =
// (1/2, 1/2, 1/2) - o, |d|^2 < 4, weight W(|d|) and gradient weight W'(|d|) /
// |d| * d.  The taps form four 2 x 2 x 2 blocks: the eight nearest (|d| =
// sqrt(3)/2, o in {0, 1}^3) and, per axis, the eight with that offset in
// {-1, 2} and the others in {0, 1} (|d| = sqrt(11)/2); inside a block each
// weight is constant and each gradient weight takes two values of opposite
// sign per axis, so a block contributes its sum and its three
// half-differences.  V is called once per tap.  Every path that sums taps
// (plain, factorised, fallback, saturated points of the learned path) uses
// this, so they agree bit for bit wherever their fractions do.
struct TapBlock {
    float t, dx, dy, dz;
};
template <class VF>
__device__ __forceinline__ TapBlock tap_block(const VF &V, int x, int y, int z, int sx, int sy, int sz) {
    // v[a][b][c] at (x + a sx, y + b sy, z + c sz), slot 0 on the + side of d
    const float v000 = V(x, y, z), v001 = V(x, y, z + sz);
    const float v010 = V(x, y + sy, z), v011 = V(x, y + sy, z + sz);
    const float v100 = V(x + sx, y, z), v101 = V(x + sx, y, z + sz);
    const float v110 = V(x + sx, y + sy, z), v111 = V(x + sx, y + sy, z + sz);
    const float c00 = v000 + v001, c01 = v010 + v011, c10 = v100 + v101, c11 = v110 + v111;
    const float x0 = c00 + c01, x1 = c10 + c11;
    TapBlock b;
    b.t = x0 + x1;
    b.dx = x0 - x1;
    b.dy = (c00 + c10) - (c01 + c11);
    b.dz = ((v000 + v010) + (v100 + v110)) - ((v001 + v011) + (v101 + v111));
    return b;
}
template <class VF>
__device__ __forceinline__ void tap_sums(const VF &V, int i, int j, int k, float &kw, float &kx, float &ky,
                                         float &kz) {
    const float Wn = (float)wendland_u(sqrt(0.75)), Wf = (float)wendland_u(sqrt(2.75));
    const float Dn = (float)(0.5 * wendland_dr_over_r_u(sqrt(0.75)));
    const float Dh = (float)(0.5 * wendland_dr_over_r_u(sqrt(2.75)));   // far taps, the +-1/2 components
    const float Dw = (float)(1.5 * wendland_dr_over_r_u(sqrt(2.75)));   // far taps, the +-3/2 component
    const TapBlock n = tap_block(V, i, j, k, 1, 1, 1);
    const TapBlock fx = tap_block(V, i - 1, j, k, 3, 1, 1);
    const TapBlock fy = tap_block(V, i, j - 1, k, 1, 3, 1);
    const TapBlock fz = tap_block(V, i, j, k - 1, 1, 1, 3);
    kw = Wn * n.t + Wf * ((fx.t + fy.t) + fz.t);
    kx = Dn * n.dx + (Dw * fx.dx + Dh * (fy.dx + fz.dx));
    ky = Dn * n.dy + (Dw * fy.dy + Dh * (fx.dy + fz.dy));
    kz = Dn * n.dz + (Dw * fz.dz + Dh * (fx.dz + fy.dz));
}

}  // namespace sgrid

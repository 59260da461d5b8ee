// Device helpers of the near-surface integrals shared by the plain and the
// learned paths: the cut-cell volume fraction and the Wendland C2 taps.
//
// V is the volume fraction of a cell on the phi > 0 side of the plane
// phi_j + g_j . (y - x_j).  It is evaluated with the case analysis of
// Scardovelli & Zaleski (J. Comput. Phys. 164, 2000) on the normal sorted and
// scaled to unit 1-norm, with the cases rewritten so that every division is by
// a bounded ratio (no cancellation when one or two normal components vanish).
#pragma once

#include "common.hpp"

namespace sgrid {

__device__ __forceinline__ float sz_volume_below(float alpha, float m1, float m2, float m3) {
    // |{w in [0,1]^3 : m.w < alpha}| for 0 <= m1 <= m2 <= m3, m1 + m2 + m3 = 1, 0 <= alpha <= 1/2
    if (alpha <= 0.0f) return 0.0f;
    const float m12 = m1 + m2;
    if (alpha < m1) return (alpha / m1) * (alpha / m2) * (alpha / m3) * (1.0f / 6.0f);
    if (alpha < m2) {
        const float r = alpha / m2;
        return (3.0f * r * alpha - 3.0f * r * m1 + (m1 / m2) * m1) / (6.0f * m3);
    }
    if (alpha < m12 && alpha < m3) {
        const float e = alpha - m2;
        const float base = (3.0f * (alpha / m2) * alpha - 3.0f * (alpha / m2) * m1 + (m1 / m2) * m1) / (6.0f * m3);
        return base - (e / m1) * (e / m2) * e / (6.0f * m3);
    }
    if (m3 < m12) {
        const float e2 = alpha - m2, e3 = alpha - m3;
        const float base = (3.0f * (alpha / m2) * alpha - 3.0f * (alpha / m2) * m1 + (m1 / m2) * m1) / (6.0f * m3);
        return base - ((e2 / m1) * (e2 / m2) * e2 + (e3 / m1) * (e3 / m2) * e3) / (6.0f * m3);
    }
    return (2.0f * alpha - m12) / (2.0f * m3);
}

// Fraction of the cube u in [-1/2, 1/2]^3 where a + g.u > 0.
__device__ __forceinline__ float plane_cube_fraction(float a, float gx, float gy, float gz) {
    float m1 = fabsf(gx), m2 = fabsf(gy), m3 = fabsf(gz);
    // sort ascending
    float t;
    if (m1 > m2) { t = m1; m1 = m2; m2 = t; }
    if (m2 > m3) { t = m2; m2 = m3; m3 = t; }
    if (m1 > m2) { t = m1; m1 = m2; m2 = t; }
    const float s = m1 + m2 + m3;
    if (!(s > 0.0f)) return a > 0.0f ? 1.0f : (a < 0.0f ? 0.0f : 0.5f);
    const float inv = 1.0f / s;
    m1 *= inv;
    m2 *= inv;
    m3 *= inv;
    const float alpha = a * inv + 0.5f;   // (a + s/2) / s
    if (alpha >= 1.0f) return 1.0f;
    if (alpha <= 0.0f) return 0.0f;
    if (alpha > 0.5f) return 1.0f - sz_volume_below(1.0f - alpha, m1, m2, m3);
    return sz_volume_below(alpha, m1, m2, m3);
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

}  // namespace sgrid

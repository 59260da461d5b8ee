// Near-surface kernel integrals over the core packages (Sec. 8: the integral
// with an SPH smoothing kernel evaluated on the sparse grid).
//
// One wavefront per core package.  The package's 9 x 9 x 9 phi window (local
// coordinates -2..6 per axis, reached through the 27-entry neighbour table and
// the index shift of Sec. 5.2) is staged in LDS; the cut fractions V of the
// 7 x 7 x 7 points -1..5 are computed once per point into LDS; then every lane
// (one data point) sums the 32 taps of its dual-cell query.
//
// V is the volume fraction of a cell on the phi > 0 side of the plane
// phi_j + g_j . (y - x_j).  It is evaluated with the case analysis of
// Scardovelli & Zaleski (J. Comput. Phys. 164, 2000) on the normal sorted and
// scaled to unit 1-norm, with the cases rewritten so that every division is by
// a bounded ratio (no cancellation when one or two normal components vanish).
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

namespace {

constexpr int kWin = 9;       // phi window edge (-2..6)
constexpr int kVol = 7;       // V window edge (-1..5)
constexpr int kWinN = kWin * kWin * kWin;
constexpr int kVolN = kVol * kVol * kVol;

// Wendland C2 in units of h (support 2): W(r) and W'(r) / r.
__device__ __forceinline__ double wendland_u(double r) {
    const double e = 1.0 - 0.5 * r;
    return 21.0 / (16.0 * M_PI) * e * e * e * e * (1.0 + 2.0 * r);
}
__device__ __forceinline__ double wendland_dr_over_r_u(double r) {
    const double e = 1.0 - 0.5 * r;
    return -105.0 / (16.0 * M_PI) * e * e * e;
}

__global__ __launch_bounds__(256) void integrals_plain_kernel(const float *__restrict__ phi,
                                                              const uint32_t *__restrict__ nbr,
                                                              const uint32_t *__restrict__ core_list,
                                                              int64_t n_core, float inv_h, float inv_2h,
                                                              float *__restrict__ out) {
    __shared__ float s_phi[4][kWinN];
    __shared__ float s_v[4][kVolN];
    __shared__ uint32_t s_ids[4][27];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t ci = (int64_t)blockIdx.x * 4 + w;
    const bool live = ci < n_core;
    const int64_t p = live ? core_list[ci] : 0;
    if (live && lane < 27) s_ids[w][lane] = nbr[p * 27 + lane];
    __syncthreads();
    if (live) {
        for (int v = lane; v < kWinN; v += 64) {
            const int x = v % kWin - 2, y = (v / kWin) % kWin - 2, z = v / (kWin * kWin) - 2;
            const int kx = (x + 4) >> 2, ky = (y + 4) >> 2, kz = (z + 4) >> 2;   // slot per axis
            const int d = (x + 4 - 4 * kx) + 4 * (y + 4 - 4 * ky) + 16 * (z + 4 - 4 * kz);
            s_phi[w][v] = phi[(int64_t)s_ids[w][kx + 3 * ky + 9 * kz] * 64 + d];
        }
    }
    __syncthreads();
    if (live) {
        const float *f = s_phi[w];
        for (int v = lane; v < kVolN; v += 64) {
            const int x = v % kVol + 1, y = (v / kVol) % kVol + 1, z = v / (kVol * kVol) + 1;   // in window coords
            const int c = x + kWin * (y + kWin * z);
            const float gx = (f[c + 1] - f[c - 1]) * inv_2h;
            const float gy = (f[c + kWin] - f[c - kWin]) * inv_2h;
            const float gz = (f[c + kWin * kWin] - f[c - kWin * kWin]) * inv_2h;
            s_v[w][v] = sgrid::plane_cube_fraction(f[c] * inv_h, gx, gy, gz);
        }
    }
    __syncthreads();
    if (!live) return;
    const float Wn = (float)wendland_u(sqrt(0.75)), Wf = (float)wendland_u(sqrt(2.75));
    const float Dn = (float)wendland_dr_over_r_u(sqrt(0.75)), Df = (float)wendland_dr_over_r_u(sqrt(2.75));
    const int i = lane & 3, j = (lane >> 2) & 3, k = lane >> 4;
    const float *V = s_v[w];
    float kw = 0.f, kx = 0.f, ky = 0.f, kz = 0.f;
    for (int oz = -1; oz <= 2; ++oz)
        for (int oy = -1; oy <= 2; ++oy)
            for (int ox = -1; ox <= 2; ++ox) {
                const float dx = 0.5f - ox, dy = 0.5f - oy, dz = 0.5f - oz;
                const float r2 = dx * dx + dy * dy + dz * dz;
                if (r2 >= 4.0f) continue;
                const bool nearp = r2 < 1.0f;
                const float vv = V[(i + ox + 1) + kVol * ((j + oy + 1) + kVol * (k + oz + 1))];
                const float Wt = nearp ? Wn : Wf, Dt = nearp ? Dn : Df;
                kw += Wt * vv;
                kx += Dt * dx * vv;
                ky += Dt * dy * vv;
                kz += Dt * dz * vv;
            }
    const int64_t o = ci * 64 + lane, stride = n_core * 64;
    out[o] = kw;
    out[stride + o] = kx;
    out[2 * stride + o] = ky;
    out[3 * stride + o] = kz;
}

}  // namespace

namespace sgrid {

sgrid_status launch_integrals_plain(const sgrid_grid *g, const float *phi, float *out, hipStream_t st) {
    if (g->n_core == 0) return SGRID_OK;
    const int64_t nb = (g->n_core + 3) / 4;
    hipLaunchKernelGGL(integrals_plain_kernel, dim3((unsigned)nb), dim3(256), 0, st, phi, g->nbr, g->core_list,
                       g->n_core, (float)(1.0 / g->h), (float)(0.5 / g->h), out);
    SG_CHECK_LAUNCH("plain integrals");
    return SGRID_OK;
}

sgrid_status integrals_learned(const sgrid_grid *g, const float *phi, const sgrid_mlp *model, float *out,
                               uint32_t *n_fallback, hipStream_t st);

}  // namespace sgrid

extern "C" sgrid_status sgrid_compute_near_surface_integrals(const sgrid_grid *g, const float *phi,
                                                             const sgrid_mlp *model, float *out,
                                                             uint32_t *n_fallback, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(phi != nullptr, "phi is NULL");
    SG_REQUIRE(out != nullptr || g->n_core == 0, "out is NULL");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(out, 16), "phi / out must be 16-byte aligned");
    hipStream_t st = sg_stream(stream);
    if (model) return sgrid::integrals_learned(g, phi, model, out, n_fallback, st);
    if (n_fallback) SG_CHECK_HIP(hipMemsetAsync(n_fallback, 0, sizeof(uint32_t), st));
    return sgrid::launch_integrals_plain(g, phi, out, st);
}

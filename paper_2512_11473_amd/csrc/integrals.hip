// Near-surface kernel integrals over the core packages (Sec. 8: the integral
// with an SPH smoothing kernel evaluated on the sparse grid).
//
// One wavefront per core package.  The package's 9 x 9 x 9 phi window (local
// coordinates -2..6 per axis, reached through the 27-entry neighbour table and
// the index shift of Sec. 5.2) is staged in LDS; the cut fractions V of the
// 7 x 7 x 7 points -1..5 are computed once per point into LDS; then every lane
// (one data point) sums the 32 taps of its dual-cell query.
//
// The cut fraction V and the kernel taps are in fraction.hpp.
#include "fraction.hpp"
#include "window.hpp"

namespace {

using sgrid::kWin;            // phi window edge (-2..6)
using sgrid::kWinN;
constexpr int kVol = 7;       // V window edge (-1..5)
constexpr int kVolN = kVol * kVol * kVol;

using sgrid::wendland_u;
using sgrid::wendland_dr_over_r_u;

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
    if (live) sgrid::stage_window_part<64>(phi, s_ids[w], lane, s_phi[w]);
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

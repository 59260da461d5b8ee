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

// The 32 taps of the dual-cell query of point (i, j, k) over the 7^3 cut
// fractions V (window coordinates -1..5): K_W and the three K_grad sums.
__device__ __forceinline__ void tap_sums(const float *V, int i, int j, int k, float &kw, float &kx, float &ky,
                                         float &kz) {
    const float Wn = (float)wendland_u(sqrt(0.75)), Wf = (float)wendland_u(sqrt(2.75));
    const float Dn = (float)wendland_dr_over_r_u(sqrt(0.75)), Df = (float)wendland_dr_over_r_u(sqrt(2.75));
    kw = kx = ky = kz = 0.f;
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
}

// The cut fractions of the 7^3 points -1..5 of a package from its staged
// 9^3 phi window f, by the wavefront's 64 lanes.
__device__ __forceinline__ void window_fractions(const float *f, int lane, float inv_h, float inv_2h, float *V) {
    for (int v = lane; v < kVolN; v += 64) {
        const int x = v % kVol + 1, y = (v / kVol) % kVol + 1, z = v / (kVol * kVol) + 1;   // in window coords
        const int c = x + kWin * (y + kWin * z);
        const float gx = (f[c + 1] - f[c - 1]) * inv_2h;
        const float gy = (f[c + kWin] - f[c - kWin]) * inv_2h;
        const float gz = (f[c + kWin * kWin] - f[c - kWin * kWin]) * inv_2h;
        V[v] = sgrid::plane_cube_fraction(f[c] * inv_h, gx, gy, gz);
    }
}

// FIELD = false: the core packages of `list`, output [4][n * 64] in list
// order.  FIELD = true: every activated package (ids 2 .. n + 1, `list`
// unused), output one float4 (K_W, h K_grad) per data point in the packed
// blocked layout of the probe fields.
template <bool FIELD>
__global__ __launch_bounds__(256) void integrals_plain_kernel(const float *__restrict__ phi,
                                                              const uint32_t *__restrict__ nbr,
                                                              const uint32_t *__restrict__ list,
                                                              int64_t n, float inv_h, float inv_2h,
                                                              float *__restrict__ out) {
    __shared__ float s_phi[4][kWinN];
    __shared__ float s_v[4][kVolN];
    __shared__ uint32_t s_ids[4][27];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t ci = (int64_t)blockIdx.x * 4 + w;
    const bool live = ci < n;
    const int64_t p = live ? (FIELD ? ci + 2 : (int64_t)list[ci]) : 0;
    if (live && lane < 27) s_ids[w][lane] = nbr[p * 27 + lane];
    __syncthreads();
    if (live) sgrid::stage_window_part<64>(phi, s_ids[w], lane, s_phi[w]);
    __syncthreads();
    if (live) window_fractions(s_phi[w], lane, inv_h, inv_2h, s_v[w]);
    __syncthreads();
    if (!live) return;
    const int i = lane & 3, j = (lane >> 2) & 3, k = lane >> 4;
    float kw, kx, ky, kz;
    tap_sums(s_v[w], i, j, k, kw, kx, ky, kz);
    if (FIELD) {
        reinterpret_cast<float4 *>(out)[p * 64 + blocked_index(i, j, k)] = make_float4(kw, kx, ky, kz);
    } else {
        const int64_t o = ci * 64 + lane, stride = n * 64;
        out[o] = kw;
        out[stride + o] = kx;
        out[2 * stride + o] = ky;
        out[3 * stride + o] = kz;
    }
}

// Second pass of the factorised integrals: one wavefront per core package
// stages the 7^3 cut fractions around it from the first pass's array (through
// the neighbour row, index shift of Sec. 5.2 with the window origin at -1)
// and sums the taps.  A core package's 26 neighbours are all activated inside
// the domain, so the window reads only band points there; a package at a
// domain face has far-field neighbours, whose window points take their
// fractions from the mixed neighbourhood of the face rather than from a
// shared far-field row: such a wavefront stages its phi window and evaluates
// the fractions itself, as the plain kernel does.  The taps and the fractions
// are the plain kernel's expressions, so the output carries its bits.
__global__ __launch_bounds__(256) void integrals_factorised_kernel(const float *__restrict__ phi,
                                                                   const float *__restrict__ vfrac,
                                                                   const uint32_t *__restrict__ nbr,
                                                                   const uint32_t *__restrict__ list, int64_t n,
                                                                   int64_t n_blocks, float inv_h, float inv_2h,
                                                                   float *__restrict__ out) {
    __shared__ float s_phi[4][kWinN];
    __shared__ float s_v[4][kVolN];
    __shared__ uint32_t s_ids[4][28];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t ci = xcd_block(blockIdx.x, n_blocks) * 4 + w;
    const bool live = ci < n;
    const int64_t p = live ? (int64_t)list[ci] : 0;
    if (live && lane < 27) s_ids[w][lane] = nbr[p * 27 + lane];
    __syncthreads();
    const uint32_t *ids = s_ids[w];
    bool edge = false;
    if (live)
        for (int q = 0; q < 27; ++q) edge |= ids[q] < 2u;
    if (live && edge) sgrid::stage_window_part<64>(phi, ids, lane, s_phi[w]);
    __syncthreads();
    if (live) {
        if (edge) {
            window_fractions(s_phi[w], lane, inv_h, inv_2h, s_v[w]);
        } else {
            constexpr int kIters = (kVolN + 63) / 64;
            float v[kIters];
#pragma unroll
            for (int u = 0; u < kIters; ++u) {
                const int q = min(lane + 64 * u, kVolN - 1);
                const int x = q % kVol - 1, y = (q / kVol) % kVol - 1, z = q / (kVol * kVol) - 1;
                const int kx = (x + 4) >> 2, ky = (y + 4) >> 2, kz = (z + 4) >> 2;
                const int d = (x + 4 - 4 * kx) + 4 * (y + 4 - 4 * ky) + 16 * (z + 4 - 4 * kz);
                v[u] = vfrac[(int64_t)ids[kx + 3 * ky + 9 * kz] * 64 + d];
            }
#pragma unroll
            for (int u = 0; u < kIters; ++u) {
                const int q = lane + 64 * u;
                if (q < kVolN) s_v[w][q] = v[u];
            }
        }
    }
    __syncthreads();
    if (!live) return;
    const int i = lane & 3, j = (lane >> 2) & 3, k = lane >> 4;
    float kw, kx, ky, kz;
    tap_sums(s_v[w], i, j, k, kw, kx, ky, kz);
    const int64_t o = ci * 64 + lane, stride = n * 64;
    out[o] = kw;
    out[stride + o] = kx;
    out[2 * stride + o] = ky;
    out[3 * stride + o] = kz;
}

// Rows 0 and 1 of the integral field: the far-field packages, whose points
// have every cell of their support on one side of the surface.  Negative far
// field (inside): all cut fractions 0, so (0, 0, 0, 0); positive far field:
// all fractions 1, so K_W = the full kernel sum c_full and, by the symmetry of
// the 32 taps about the query point, K_grad = 0.
__global__ __launch_bounds__(128) void integral_far_rows_kernel(float4 *__restrict__ field, float c_full) {
    const int t = threadIdx.x;
    field[t] = t < 64 ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(c_full, 0.f, 0.f, 0.f);
}

}  // namespace

namespace sgrid {

sgrid_status launch_integrals_plain(const sgrid_grid *g, const float *phi, float *out, hipStream_t st) {
    if (g->n_core == 0) return SGRID_OK;
    const int64_t nb = (g->n_core + 3) / 4;
    hipLaunchKernelGGL(integrals_plain_kernel<false>, dim3((unsigned)nb), dim3(256), 0, st, phi, g->nbr,
                       g->core_list, g->n_core, (float)(1.0 / g->h), (float)(0.5 / g->h), out);
    SG_CHECK_LAUNCH("plain integrals");
    return SGRID_OK;
}

sgrid_status integrals_learned(const sgrid_grid *g, const float *phi, const sgrid_mlp *model, float *out,
                               uint32_t *n_fallback, hipStream_t st);

sgrid_status launch_cut_fractions(const sgrid_grid *g, const float *phi, float *vfrac, hipStream_t st);

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
    if (n_fallback) {
        sgrid_status s = sgrid::launch_zero_u32(n_fallback, st);
        if (s != SGRID_OK) return s;
    }
    return sgrid::launch_integrals_plain(g, phi, out, st);
}

extern "C" sgrid_status sgrid_compute_near_surface_integrals_factorised(const sgrid_grid *g, const float *phi,
                                                                        float *vfrac, float *out, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(phi != nullptr && vfrac != nullptr, "phi or vfrac is NULL");
    SG_REQUIRE(out != nullptr || g->n_core == 0, "out is NULL");
    SG_REQUIRE(phi != vfrac && (const float *)out != phi && out != vfrac, "phi, vfrac and out must be distinct");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(vfrac, 16) && sg_aligned(out, 16),
               "phi / vfrac / out must be 16-byte aligned");
    if (g->n_core == 0) return SGRID_OK;
    hipStream_t st = sg_stream(stream);
    sgrid_status s = sgrid::launch_cut_fractions(g, phi, vfrac, st);
    if (s != SGRID_OK) return s;
    const int64_t nb = (g->n_core + 3) / 4;
    hipLaunchKernelGGL(integrals_factorised_kernel, dim3((unsigned)nb), dim3(256), 0, st, phi, (const float *)vfrac,
                       g->nbr, g->core_list, g->n_core, nb, (float)(1.0 / g->h), (float)(0.5 / g->h), out);
    SG_CHECK_LAUNCH("factorised integrals");
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_compute_integral_field(const sgrid_grid *g, const float *phi, float *field,
                                                     void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(phi != nullptr && field != nullptr, "phi or field is NULL");
    SG_REQUIRE(phi != field, "phi and field must be distinct buffers");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(field, 16), "phi / field must be 16-byte aligned");
    hipStream_t st = sg_stream(stream);
    const double c_full = 8.0 * sgrid::wendland_u(0.5 * sqrt(3.0)) + 24.0 * sgrid::wendland_u(0.5 * sqrt(11.0));
    hipLaunchKernelGGL(integral_far_rows_kernel, dim3(1), dim3(128), 0, st, (float4 *)field, (float)c_full);
    SG_CHECK_LAUNCH("integral field far-field rows");
    if (g->P == 0) return SGRID_OK;
    const int64_t nb = (g->P + 3) / 4;
    SG_REQUIRE(nb <= kMaxGrid, "too many packages for one launch");
    hipLaunchKernelGGL(integrals_plain_kernel<true>, dim3((unsigned)nb), dim3(256), 0, st, phi, g->nbr,
                       (const uint32_t *)nullptr, g->P, (float)(1.0 / g->h), (float)(0.5 / g->h), field);
    SG_CHECK_LAUNCH("integral field");
    return SGRID_OK;
}

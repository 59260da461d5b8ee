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

// LDS layout of the 7^3 cut fractions V (window coordinates -1..5): rows of 8
// along x (x = 0..5 at 0..5, x = -1 at 7, 6 unused), 8 floats per y step and
// 60 per z step.  A row is two aligned 16-byte words, and the 32 lanes of a
// half-wavefront (i, j in 0..3, k in 0..1) read 32 distinct banks at any tap.
constexpr int kVRow = 8, kVPlane = 60, kVWinN = kVol * kVPlane;
__device__ __forceinline__ int vidx(int x, int y, int z) { return (x & 7) + kVRow * (y + 1) + kVPlane * (z + 1); }

// The 32 taps of data point (i, j, k) over the LDS window of cut fractions.
__device__ __forceinline__ void tap_sums(const float *V, int i, int j, int k, float &kw, float &kx, float &ky,
                                         float &kz) {
    sgrid::tap_sums([V](int x, int y, int z) { return V[vidx(x, y, z)]; }, i, j, k, kw, kx, ky, kz);
}

// The cut fractions of the 7^3 points -1..5 of a package from its staged
// 9^3 phi window f, by the wavefront's 64 lanes.  A point more than half a
// cell (in the 1-norm of its gradient) from the surface has V = 0 or 1 by the
// sign of phi; the cut points are listed (ballot, in LDS) and evaluated one
// per lane afterwards, so the case code runs once per 64 cut points rather
// than once per 64 window points.  A saturated point's value is the one the
// fraction returns (see fraction_saturated).
__device__ __forceinline__ void window_fractions(const float *f, int lane, float inv_h, float inv_2h, float *V,
                                                 uint16_t *cut_list) {
    const uint64_t below = (1ull << lane) - 1ull;
    int n_cut = 0;
#pragma unroll
    for (int u = 0; u < (kVolN + 63) / 64; ++u) {
        const int v = lane + 64 * u;
        const int vc = min(v, kVolN - 1);
        const int x = vc % kVol, y = (vc / kVol) % kVol, z = vc / (kVol * kVol);   // window coords + 1
        const int c = (x + 1) + kWin * ((y + 1) + kWin * (z + 1));
        const float a = f[c] * inv_h;
        const float gx = (f[c + 1] - f[c - 1]) * inv_2h;
        const float gy = (f[c + kWin] - f[c - kWin]) * inv_2h;
        const float gz = (f[c + kWin * kWin] - f[c - kWin * kWin]) * inv_2h;
        const bool sat = sgrid::fraction_saturated(a, gx, gy, gz);
        if (v < kVolN && sat) V[vidx(x - 1, y - 1, z - 1)] = a > 0.0f ? 1.0f : 0.0f;
        const bool cut = v < kVolN && !sat;
        const uint64_t m = __ballot(cut);
        if (cut) cut_list[n_cut + (int)__popcll(m & below)] = (uint16_t)v;
        n_cut += (int)__popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < n_cut; t += 64) {
        const int v = cut_list[t];
        const int x = v % kVol, y = (v / kVol) % kVol, z = v / (kVol * kVol);
        const int c = (x + 1) + kWin * ((y + 1) + kWin * (z + 1));
        const float gx = (f[c + 1] - f[c - 1]) * inv_2h;
        const float gy = (f[c + kWin] - f[c - kWin]) * inv_2h;
        const float gz = (f[c + kWin * kWin] - f[c - kWin * kWin]) * inv_2h;
        V[vidx(x - 1, y - 1, z - 1)] = sgrid::plane_cube_fraction(f[c] * inv_h, gx, gy, gz);
    }
}

// The 9^3 phi window of a package into LDS (x fastest, window coordinates
// -2..6), one window row of 9 per lane and step (81 rows): x = -2, -1 from
// the -x neighbour's row (8-byte load), x = 0..3 the package's own row
// (16-byte load), x = 4..6 from the +x neighbour's row (16-byte load, the
// fourth value unused).  The neighbours through the 27-entry row ids with the
// index shift of Sec. 5.2.
__device__ __forceinline__ void stage_window_rows(const float *__restrict__ phi, const uint32_t *ids, int lane,
                                                  float *f) {
    constexpr int kRows = kWin * kWin;
    constexpr int kSteps = (kRows + 63) / 64;
    float2 m[kSteps];
    float4 c[kSteps], q[kSteps];
#pragma unroll
    for (int u = 0; u < kSteps; ++u) {
        const int r = min(lane + 64 * u, kRows - 1);
        const int y = r % kWin - 2, z = r / kWin - 2;
        const int ky = (y + 4) >> 2, kz = (z + 4) >> 2;
        const int row = 4 * ((y + 4 - 4 * ky) + 4 * (z + 4 - 4 * kz));
        const int s = 3 * ky + 9 * kz;
        m[u] = *reinterpret_cast<const float2 *>(phi + (int64_t)ids[s] * 64 + row + 2);
        c[u] = *reinterpret_cast<const float4 *>(phi + (int64_t)ids[s + 1] * 64 + row);
        q[u] = *reinterpret_cast<const float4 *>(phi + (int64_t)ids[s + 2] * 64 + row);
    }
#pragma unroll
    for (int u = 0; u < kSteps; ++u) {
        const int r = lane + 64 * u;
        if (r < kRows) {
            float *d = f + kWin * r;
            d[0] = m[u].x;
            d[1] = m[u].y;
            d[2] = c[u].x;
            d[3] = c[u].y;
            d[4] = c[u].z;
            d[5] = c[u].w;
            d[6] = q[u].x;
            d[7] = q[u].y;
            d[8] = q[u].z;
        }
    }
}

// FIELD = false: the core packages of `list`, output [4][n * 64] in list
// order.  FIELD = true: every activated package (ids 2 .. n + 1, `list`
// unused), output one float4 (K_W, h K_grad) per data point in the packed
// blocked layout of the probe fields.  Each wavefront works on its own
// package and LDS slices alone, so it waits for no other.
template <bool FIELD>
__global__ __launch_bounds__(256) void integrals_plain_kernel(const float *__restrict__ phi,
                                                              const uint32_t *__restrict__ nbr,
                                                              const uint32_t *__restrict__ list,
                                                              int64_t n, float inv_h, float inv_2h,
                                                              float *__restrict__ out) {
    __shared__ float s_phi[4][kWinN];
    __shared__ __align__(16) float s_v[4][kVWinN];
    __shared__ uint16_t s_cut[4][kVolN + 1];
    __shared__ uint32_t s_ids[4][27];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t ci = (int64_t)blockIdx.x * 4 + w;
    if (ci >= n) return;
    const int64_t p = FIELD ? ci + 2 : (int64_t)list[ci];
    if (lane < 27) s_ids[w][lane] = nbr[p * 27 + lane];
    __builtin_amdgcn_wave_barrier();
    stage_window_rows(phi, s_ids[w], lane, s_phi[w]);
    __builtin_amdgcn_wave_barrier();
    window_fractions(s_phi[w], lane, inv_h, inv_2h, s_v[w], s_cut[w]);
    __builtin_amdgcn_wave_barrier();
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

// The cut fractions of the window of a package at a domain face straight
// from phi (the values and expressions of window_fractions), in a rolled
// loop: this rare path needs no LDS window and does not raise the register
// count of the common one.
__device__ __forceinline__ void edge_window_fractions(const float *__restrict__ phi, const uint32_t *ids, int lane,
                                                      float inv_h, float inv_2h, float *V) {
#pragma unroll 1
    for (int v = lane; v < kVolN; v += 64) {
        const int x = v % kVol, y = (v / kVol) % kVol, z = v / (kVol * kVol);   // window coords + 1
        const int c = (x + 1) + kWin * ((y + 1) + kWin * (z + 1));
        const float fc = phi[sgrid::window_source(ids, c)];
        const float gx = (phi[sgrid::window_source(ids, c + 1)] - phi[sgrid::window_source(ids, c - 1)]) * inv_2h;
        const float gy = (phi[sgrid::window_source(ids, c + kWin)] - phi[sgrid::window_source(ids, c - kWin)]) * inv_2h;
        const float gz = (phi[sgrid::window_source(ids, c + kWin * kWin)] -
                          phi[sgrid::window_source(ids, c - kWin * kWin)]) * inv_2h;
        V[vidx(x - 1, y - 1, z - 1)] = sgrid::plane_cube_fraction(fc * inv_h, gx, gy, gz);
    }
}

// Second pass of the factorised integrals: each wavefront takes G
// consecutive core packages.  Per package it gathers the 7^3 cut fractions
// around it from the first pass's array (through the neighbour row, index
// shift of Sec. 5.2 with the window origin at -1), one window row of 7 per
// lane: the 4 of the package's own row as one 16-byte load, x = -1 from the
// -x neighbour and x = 4, 5 from the +x neighbour.  All G packages' neighbour
// rows, then all their window rows, are requested before the first package's
// taps are summed, so the later packages' loads are in flight while the
// earlier ones are summed and stored.  The windows pass one by one through
// the wavefront's LDS slice.  A core package's 26 neighbours are all
// activated inside the domain, so the window reads only band points there; a
// package at a domain face has far-field neighbours, whose window points take
// their fractions from the mixed neighbourhood of the face rather than from a
// shared far-field row: such a package's fractions are evaluated from phi, as
// the plain kernel does.  The taps and the fractions are the plain kernel's
// expressions, so the output carries its bits.
template <int G>
__global__ __launch_bounds__(256) void integrals_factorised_kernel(const float *__restrict__ phi,
                                                                   const float *__restrict__ vfrac,
                                                                   const uint32_t *__restrict__ nbr,
                                                                   const uint32_t *__restrict__ list, int64_t n,
                                                                   int64_t n_blocks, float inv_h, float inv_2h,
                                                                   float *__restrict__ out) {
    __shared__ __align__(16) float s_v[4][kVWinN + kVRow * (64 - kVol * kVol)];
    __shared__ uint32_t s_ids[4][27];
    // (the wavefront index through readfirstlane: the compiler then knows it
    // is uniform and reads the list with scalar loads)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t c0 = (xcd_block(blockIdx.x, n_blocks) * 4 + w) * G;
    if (c0 >= n) return;
    const int64_t stride = n * 64;
    uint32_t p[G], id[G];
#pragma unroll
    for (int g = 0; g < G; ++g) p[g] = list[min(c0 + g, n - 1)];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t v = nbr[(int64_t)p[g] * 27 + min(lane, 26)];
        id[g] = lane < 27 ? v : 2u;
    }
    // window row of this lane (lanes 49..63 repeat row 48 and write it to a
    // spare row of their own past the window)
    const int rl = min(lane, kVol * kVol - 1);
    const int y = rl % kVol - 1, z = rl / kVol - 1;
    const int ky = (y + 4) >> 2, kz = (z + 4) >> 2;
    const int row = 4 * ((y + 4 - 4 * ky) + 4 * (z + 4 - 4 * kz));
    const int s = 3 * ky + 9 * kz;
    // (an edge package's loads read the far-field rows 0 / 1, in bounds, and
    // are not used)
    float xm[G];
    float4 c[G];
    float2 xp[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t im = __shfl(id[g], s), ic = __shfl(id[g], s + 1), ip = __shfl(id[g], s + 2);
        xm[g] = vfrac[(int64_t)im * 64 + row + 3];
        c[g] = *reinterpret_cast<const float4 *>(vfrac + (int64_t)ic * 64 + row);
        xp[g] = *reinterpret_cast<const float2 *>(vfrac + (int64_t)ip * 64 + row);
    }
    float *V = s_v[w];
    const int i = lane & 3, j = (lane >> 2) & 3, k = lane >> 4;
    // The common path has no branch, so the compiler keeps every load where
    // it is issued: a tail package repeats the last one and stores the same
    // values to the same place.  Packages with a far-field neighbour get their
    // stores overwritten below.
    float4 *dst = reinterpret_cast<float4 *>(
        V + (lane < kVol * kVol ? kVRow * (y + 1) + kVPlane * (z + 1) : kVWinN + kVRow * (lane - kVol * kVol)));
    uint32_t edge = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        edge |= (__ballot(id[g] < 2u) != 0 ? 1u : 0u) << g;
        dst[0] = c[g];
        dst[1] = make_float4(xp[g].x, xp[g].y, 0.f, xm[g]);
        __builtin_amdgcn_wave_barrier();
        float kw, kx, ky_, kz_;
        tap_sums(V, i, j, k, kw, kx, ky_, kz_);
        __builtin_amdgcn_wave_barrier();
        const int64_t o = min(c0 + g, n - 1) * 64 + lane;
        out[o] = kw;
        out[stride + o] = kx;
        out[2 * stride + o] = ky_;
        out[3 * stride + o] = kz_;
    }
    if (edge == 0u) return;
#pragma unroll 1
    for (int g = 0; g < G; ++g) {
        if (!((edge >> g) & 1u) || c0 + g >= n) continue;
        uint32_t idg = id[0];
#pragma unroll
        for (int q = 1; q < G; ++q) idg = g == q ? id[q] : idg;
        if (lane < 27) s_ids[w][lane] = idg;
        __builtin_amdgcn_wave_barrier();
        edge_window_fractions(phi, s_ids[w], lane, inv_h, inv_2h, V);
        __builtin_amdgcn_wave_barrier();
        float kw, kx, ky_, kz_;
        tap_sums(V, i, j, k, kw, kx, ky_, kz_);
        __builtin_amdgcn_wave_barrier();
        const int64_t o = (c0 + g) * 64 + lane;
        out[o] = kw;
        out[stride + o] = kx;
        out[2 * stride + o] = ky_;
        out[3 * stride + o] = kz_;
    }
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
    constexpr int kG = 4;   // core packages per wavefront
    const int64_t nb = (g->n_core + 4 * kG - 1) / (4 * kG);
    hipLaunchKernelGGL(integrals_factorised_kernel<kG>, dim3((unsigned)nb), dim3(256), 0, st, phi,
                       (const float *)vfrac, g->nbr, g->core_list, g->n_core, nb, (float)(1.0 / g->h),
                       (float)(0.5 / g->h), out);
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

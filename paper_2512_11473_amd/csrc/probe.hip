// Grid-to-particle probe (Sec. 8): trilinear interpolation of phi and of the
// gradient at particle positions, reached through the cell-to-package map and
// the neighbour table (position-based random access, Sec. 5.1 indexing and the
// index shift of Sec. 5.2).
//
// One lane per particle.  The particle's coarse cell gives its home package;
// the base corner's shift relative to that package lies in [-1, 3] per axis,
// so the eight corners have shifts in [-1, 4] and the index shift
// slot = (s + 4) / 4, data = s + 4 - 4 slot stays inside the 27 neighbours.
// The packages of the home cell and its neighbours come from the rank map, a
// compact form of the cell-to-package map (32 cells per 16-byte entry) that
// the build writes beside it; the values are those of cell_pkg and of the
// neighbour table.
#include "common.hpp"

namespace {

// fmax / fmin return the non-NaN operand, so a NaN coordinate clamps to `lo`
// and every index below stays inside the tables.
template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi) { return fmin(fmax(v, lo), hi); }

// Corner field access: SoA (phi and three gradient arrays) or packed
// (phi, gx, gy, gz) quadruples.
template <typename T, bool PACKED>
struct Corner {
    const T *phi, *grad;
    int64_t stride;
    __device__ __forceinline__ void get(int64_t idx, T &v, T &gx, T &gy, T &gz) const {
        if (PACKED) {
            const T *f = phi + idx * 4;
            if (sizeof(T) == 4) {
                const float4 q = *reinterpret_cast<const float4 *>(f);
                v = q.x; gx = q.y; gy = q.z; gz = q.w;
            } else {
                v = f[0]; gx = f[1]; gy = f[2]; gz = f[3];
            }
        } else {
            v = phi[idx];
            gx = grad[idx];
            gy = grad[stride + idx];
            gz = grad[2 * stride + idx];
        }
    }
};

// Home cell and base shift of one particle (per axis: u = x / h, s = u - 1/2,
// i0 = clamp(floor(s), 0, N - 2), t = clamp(s - i0, 0, 1), home cell =
// clamp(floor(u / 4), 0, M - 1), shift = i0 - 4 * cell in [-1, 3]).
template <typename T>
__device__ __forceinline__ void locate(const T *x, int M, T inv_h, int cc[3], int sh[3], T t[3]) {
    const int N = 4 * M;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T u = x[a] * inv_h;
        const T s = u - T(0.5);
        const T f = clampv(floor(s), T(0), T(N - 2));
        t[a] = clampv(s - f, T(0), T(1));
        cc[a] = (int)clampv(floor(u * T(0.25)), T(0), T(M - 1));
        sh[a] = (int)f - 4 * cc[a];
    }
}

// Package ids from the rank map: entry {activated bits, negative bits, rank,
// 0} of the 32 cells holding x gives id = 2 + rank + (activated cells of the
// entry below x) for an activated cell, else the far-field package of its
// sign; cells outside the domain belong to the positive far field (the
// neighbour table's rule).  These are the values of cell_pkg, read from a
// table 64 times smaller that stays in the caches.
struct RankMap {
    const uint4 *map;
    int M, W32;
    __device__ __forceinline__ int64_t entry(int x, int y, int z) const {
        return ((int64_t)y + (int64_t)M * z) * W32 + (x >> 5);
    }
    __device__ __forceinline__ static uint32_t id(const uint4 &e, int x) {
        const uint32_t bit = 1u << (x & 31);
        if (e.x & bit) return 2u + e.z + (uint32_t)__popc(e.x & (bit - 1u));
        return (e.y & bit) ? sgrid::kFarNeg : sgrid::kFarPos;
    }
};

// Trilinear blend of the four components (phi and g, or an integral field)
// over the eight corners.  The
// corners' packages are the home cell's package and, for corners past a face
// of the home cell, those of the neighbouring cells (the index shift of
// Sec. 5.2 per axis: slot = (s + 4) / 4, data = s + 4 - 4 slot).  A particle
// whose home cell is far field reads the far-field constant at every corner,
// as the far-field packages neighbour themselves.  All rank-map reads issue
// before any is used, then all corner reads.
template <typename T, bool PACKED>
__device__ __forceinline__ void blend(const Corner<T, PACKED> &field, const RankMap &rm, const int cc[3],
                                      const int sh[3], const T t[3], T &v, T &gx, T &gy, T &gz) {
    const int M = rm.M;
    uint4 e[8];
    int cx[8];
    bool out[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        const int x = cc[0] + ((sh[0] + bx + 4) >> 2) - 1;
        const int y = cc[1] + ((sh[1] + by + 4) >> 2) - 1;
        const int z = cc[2] + ((sh[2] + bz + 4) >> 2) - 1;
        out[b] = x < 0 || y < 0 || z < 0 || x >= M || y >= M || z >= M;
        cx[b] = x;
        e[b] = rm.map[out[b] ? 0 : rm.entry(x, y, z)];
    }
    // the home cell's own entry (one of the eight above, read again rather than
    // picked by a per-lane index into the register array)
    const uint4 eh = rm.map[rm.entry(cc[0], cc[1], cc[2])];
    const uint32_t home = RankMap::id(eh, cc[0]);
    uint32_t pk[8];
    int d[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        const int s0 = sh[0] + bx + 4, s1 = sh[1] + by + 4, s2 = sh[2] + bz + 4;   // shift + 4 in [3, 8]
        const int k0 = s0 >> 2, k1 = s1 >> 2, k2 = s2 >> 2;                        // neighbour slot per axis
        const int di = s0 - 4 * k0, dj = s1 - 4 * k1, dk = s2 - 4 * k2;            // data index
        d[b] = PACKED ? blocked_index(di, dj, dk) : di + 4 * dj + 16 * dk;
        const uint32_t own = out[b] ? sgrid::kFarPos : RankMap::id(e[b], cx[b]);
        pk[b] = home < 2u ? home : own;
    }
    v = T(0);
    gx = T(0);
    gy = T(0);
    gz = T(0);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        const int64_t idx = (int64_t)pk[b] * 64 + d[b];
        const T w = (bx ? t[0] : T(1) - t[0]) * (by ? t[1] : T(1) - t[1]) * (bz ? t[2] : T(1) - t[2]);
        T cv, cx_, cy_, cz_;
        field.get(idx, cv, cx_, cy_, cz_);
        v += w * cv;
        gx += w * cx_;
        gy += w * cy_;
        gz += w * cz_;
    }
}

template <typename T, bool PACKED>
__global__ __launch_bounds__(256) void probe_kernel(Corner<T, PACKED> field, RankMap rm, const T *__restrict__ pos,
                                                    int64_t n, T *__restrict__ phi_out, T *__restrict__ nrm_out,
                                                    T inv_h) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int cc[3], sh[3];
    T t[3], v, gx, gy, gz;
    locate(pos + 3 * q, rm.M, inv_h, cc, sh, t);
    blend(field, rm, cc, sh, t, v, gx, gy, gz);
    const T gn = sqrt(gx * gx + gy * gy + gz * gz);
    const T inv = gn > T(0) ? T(1) / gn : T(0);
    phi_out[q] = v;
    nrm_out[3 * q] = gx * inv;
    nrm_out[3 * q + 1] = gy * inv;
    nrm_out[3 * q + 2] = gz * inv;
}

// The integral field (K_W, h K_grad) at the particles (Sec. 8: the field is
// interpolated trilinearly to the particle position and drives it as a
// surface force): the same blend, no normalisation, one float4 per particle.
__global__ __launch_bounds__(256) void probe_field_kernel(Corner<float, true> field, RankMap rm,
                                                          const float *__restrict__ pos, int64_t n,
                                                          float4 *__restrict__ out, float inv_h) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int cc[3], sh[3];
    float t[3], v, gx, gy, gz;
    locate(pos + 3 * q, rm.M, inv_h, cc, sh, t);
    blend(field, rm, cc, sh, t, v, gx, gy, gz);
    out[q] = make_float4(v, gx, gy, gz);
}

}  // namespace

template <bool PACKED>
static sgrid_status probe_entry(const sgrid_grid *g, sgrid_dtype dtype, const void *phi, const void *grad,
                                const void *pos, int64_t n, void *phi_out, void *normal_out, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(n >= 0, "n must be >= 0");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    if (n == 0) return SGRID_OK;
    SG_REQUIRE(phi && (PACKED || grad) && pos && phi_out && normal_out, "NULL field or particle array");
    const size_t es = dtype == SGRID_F32 ? 4 : 8;
    SG_REQUIRE(sg_aligned(phi, 16) && (PACKED || sg_aligned(grad, 16)), "fields must be 16-byte aligned");
    SG_REQUIRE(sg_aligned(pos, es) && sg_aligned(phi_out, es) && sg_aligned(normal_out, es),
               "particle arrays must be aligned to their element size");
    hipStream_t st = sg_stream(stream);
    const int64_t nb = (n + 255) / 256;
    SG_REQUIRE(nb <= kMaxGrid, "too many particles for one launch");
    const int64_t stride = g->total() * 64;
    const RankMap rm{g->rank_map, g->M, g->W32};
    if (dtype == SGRID_F32) {
        Corner<float, PACKED> f{(const float *)phi, (const float *)grad, stride};
        hipLaunchKernelGGL((probe_kernel<float, PACKED>), dim3((unsigned)nb), dim3(256), 0, st, f, rm,
                           (const float *)pos, n, (float *)phi_out, (float *)normal_out, (float)(1.0 / g->h));
    } else {
        Corner<double, PACKED> f{(const double *)phi, (const double *)grad, stride};
        hipLaunchKernelGGL((probe_kernel<double, PACKED>), dim3((unsigned)nb), dim3(256), 0, st, f, rm,
                           (const double *)pos, n, (double *)phi_out, (double *)normal_out, 1.0 / g->h);
    }
    SG_CHECK_LAUNCH("probe");
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_probe_particles(const sgrid_grid *g, sgrid_dtype dtype, const void *phi,
                                              const void *grad, const void *pos, int64_t n, void *phi_out,
                                              void *normal_out, void *stream) {
    return probe_entry<false>(g, dtype, phi, grad, pos, n, phi_out, normal_out, stream);
}

extern "C" sgrid_status sgrid_probe_particles_packed(const sgrid_grid *g, sgrid_dtype dtype, const void *packed,
                                                     const void *pos, int64_t n, void *phi_out, void *normal_out,
                                                     void *stream) {
    return probe_entry<true>(g, dtype, packed, nullptr, pos, n, phi_out, normal_out, stream);
}

extern "C" sgrid_status sgrid_probe_integral_field(const sgrid_grid *g, const float *field, const float *pos,
                                                   int64_t n, float *out, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(n >= 0, "n must be >= 0");
    if (n == 0) return SGRID_OK;
    SG_REQUIRE(field && pos && out, "NULL field or particle array");
    SG_REQUIRE(sg_aligned(field, 16) && sg_aligned(out, 16), "field / out must be 16-byte aligned");
    SG_REQUIRE(sg_aligned(pos, 4), "pos must be 4-byte aligned");
    hipStream_t st = sg_stream(stream);
    const int64_t nb = (n + 255) / 256;
    SG_REQUIRE(nb <= kMaxGrid, "too many particles for one launch");
    const RankMap rm{g->rank_map, g->M, g->W32};
    const Corner<float, true> f{field, nullptr, 0};
    hipLaunchKernelGGL(probe_field_kernel, dim3((unsigned)nb), dim3(256), 0, st, f, rm, pos, n, (float4 *)out,
                       (float)(1.0 / g->h));
    SG_CHECK_LAUNCH("integral field probe");
    return SGRID_OK;
}

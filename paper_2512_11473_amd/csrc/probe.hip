// Grid-to-particle probe (Sec. 8): trilinear interpolation of phi and of the
// gradient at particle positions, reached through the cell-to-package map and
// the neighbour table (position-based random access, Sec. 5.1 indexing and the
// index shift of Sec. 5.2).
//
// One lane per particle.  The particle's coarse cell gives its home package;
// the base corner's shift relative to that package lies in [-1, 3] per axis,
// so the eight corners have shifts in [-1, 4] and the index shift
// slot = (s + 4) / 4, data = s + 4 - 4 slot stays inside the 27 neighbours.
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

// Home package and base shift of one particle (per axis: u = x / h,
// s = u - 1/2, i0 = clamp(floor(s), 0, N - 2), t = clamp(s - i0, 0, 1), home
// cell = clamp(floor(u / 4), 0, M - 1), shift = i0 - 4 * cell in [-1, 3]).
template <typename T>
__device__ __forceinline__ int64_t locate(const T *x, int M, T inv_h, int sh[3], T t[3]) {
    const int N = 4 * M;
    int cc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T u = x[a] * inv_h;
        const T s = u - T(0.5);
        const T f = clampv(floor(s), T(0), T(N - 2));
        t[a] = clampv(s - f, T(0), T(1));
        cc[a] = (int)clampv(floor(u * T(0.25)), T(0), T(M - 1));
        sh[a] = (int)f - 4 * cc[a];
    }
    return cc[0] + (int64_t)M * (cc[1] + (int64_t)M * cc[2]);
}

// Trilinear blend of phi and g over the eight corners reached from the home
// package's neighbour row, then the normal.
template <typename T, bool PACKED>
__device__ __forceinline__ void blend(const Corner<T, PACKED> &field, const uint32_t *__restrict__ row, const int sh[3],
                                      const T t[3], T &v, T n[3]) {
    v = T(0);
    T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        const int s0 = sh[0] + bx + 4, s1 = sh[1] + by + 4, s2 = sh[2] + bz + 4;   // shift + 4 in [3, 8]
        const int k0 = s0 >> 2, k1 = s1 >> 2, k2 = s2 >> 2;                        // neighbour slot per axis
        const int di = s0 - 4 * k0, dj = s1 - 4 * k1, dk = s2 - 4 * k2;            // data index
        const int d = PACKED ? blocked_index(di, dj, dk) : di + 4 * dj + 16 * dk;
        const int64_t idx = (int64_t)row[k0 + 3 * k1 + 9 * k2] * 64 + d;
        const T w = (bx ? t[0] : T(1) - t[0]) * (by ? t[1] : T(1) - t[1]) * (bz ? t[2] : T(1) - t[2]);
        T cv, cx, cy, cz;
        field.get(idx, cv, cx, cy, cz);
        v += w * cv;
        gx += w * cx;
        gy += w * cy;
        gz += w * cz;
    }
    const T gn = sqrt(gx * gx + gy * gy + gz * gz);
    const T inv = gn > T(0) ? T(1) / gn : T(0);
    n[0] = gx * inv;
    n[1] = gy * inv;
    n[2] = gz * inv;
}

template <typename T, bool PACKED>
__global__ __launch_bounds__(256) void probe_kernel(Corner<T, PACKED> field, const uint32_t *__restrict__ cell_pkg,
                                                    const uint32_t *__restrict__ nbr, const T *__restrict__ pos,
                                                    int64_t n, T *__restrict__ phi_out, T *__restrict__ nrm_out,
                                                    int M, T inv_h) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int sh[3];
    T t[3], v, nr[3];
    const int64_t home = cell_pkg[locate(pos + 3 * q, M, inv_h, sh, t)];
    blend(field, nbr + home * 27, sh, t, v, nr);
    phi_out[q] = v;
    nrm_out[3 * q] = nr[0];
    nrm_out[3 * q + 1] = nr[1];
    nrm_out[3 * q + 2] = nr[2];
}

// ---------------------------------------------------------------------------
// Binned probe: a counting sort of the particles by home package, so that the
// particles sharing a package are probed together and its lines are fetched
// once, then results scattered back to input order.
//   key_kernel    home package and rank within it (atomic count per package)
//   scan          exclusive offsets of the per-package counts
//   place_kernel  slot = offset[home] + rank; order[slot] = particle
//   probe_sorted  lane = slot: particle order[slot]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void key_kernel(const T *__restrict__ pos, int64_t n,
                                                  const uint32_t *__restrict__ cell_pkg, int M, T inv_h,
                                                  uint32_t *__restrict__ key, uint32_t *__restrict__ rank,
                                                  uint32_t *__restrict__ count) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int sh[3];
    T t[3];
    const uint32_t home = cell_pkg[locate(pos + 3 * q, M, inv_h, sh, t)];
    key[q] = home;
    rank[q] = atomicAdd(count + home, 1u);
}

// Exclusive scan in place, three phases: per-block scan of 4096 entries with
// block totals, a single-block scan of the totals, and the block offsets added.
constexpr int kScanBlock = 1024, kScanPer = 4;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *s_warp, uint32_t &total) {
    // inclusive scan inside the wavefront, then across wavefronts
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t v = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(v, off);
        if (lane >= off) v += y;
    }
    if (lane == 63) s_warp[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            const uint32_t t = s_warp[i];
            s_warp[i] = acc;
            acc += t;
        }
        s_warp[blockDim.x >> 6] = acc;
    }
    __syncthreads();
    total = s_warp[blockDim.x >> 6];
    return v - x + s_warp[w];
}

__global__ __launch_bounds__(kScanBlock) void scan_blocks_kernel(uint32_t *__restrict__ a, int64_t n,
                                                                 uint32_t *__restrict__ sums) {
    __shared__ uint32_t s_warp[kScanBlock / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanPer + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer], x = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = base + i < n ? a[base + i] : 0u;
        x += v[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(x, s_warp, total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < n) a[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void scan_sums_kernel(uint32_t *__restrict__ sums, int64_t nb) {
    __shared__ uint32_t s_warp[kScanBlock / 64 + 1];
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        const int64_t i = base + threadIdx.x;
        const uint32_t x = i < nb ? sums[i] : 0u;
        uint32_t total;
        const uint32_t e = block_exclusive_scan(x, s_warp, total);
        if (i < nb) sums[i] = carry + e;
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void scan_add_kernel(uint32_t *__restrict__ a, int64_t n,
                                                       const uint32_t *__restrict__ sums) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += sums[i / (kScanBlock * kScanPer)];
}

__global__ __launch_bounds__(256) void place_kernel(const uint32_t *__restrict__ key, const uint32_t *__restrict__ rank,
                                                    const uint32_t *__restrict__ offset, int64_t n,
                                                    uint32_t *__restrict__ order) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    order[offset[key[q]] + rank[q]] = (uint32_t)q;
}

template <typename T, bool PACKED>
__global__ __launch_bounds__(256) void probe_sorted_kernel(Corner<T, PACKED> field, const uint32_t *__restrict__ cell_pkg,
                                                           const uint32_t *__restrict__ nbr,
                                                           const T *__restrict__ pos, const uint32_t *__restrict__ order,
                                                           int64_t n, T *__restrict__ phi_out, T *__restrict__ nrm_out,
                                                           int M, T inv_h) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t q = order[i];
    int sh[3];
    T t[3], v, nr[3];
    const int64_t home = cell_pkg[locate(pos + 3 * q, M, inv_h, sh, t)];
    blend(field, nbr + home * 27, sh, t, v, nr);
    phi_out[q] = v;
    nrm_out[3 * q] = nr[0];
    nrm_out[3 * q + 1] = nr[1];
    nrm_out[3 * q + 2] = nr[2];
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
    if (dtype == SGRID_F32) {
        Corner<float, PACKED> f{(const float *)phi, (const float *)grad, stride};
        hipLaunchKernelGGL((probe_kernel<float, PACKED>), dim3((unsigned)nb), dim3(256), 0, st, f, g->cell_pkg,
                           g->nbr, (const float *)pos, n, (float *)phi_out, (float *)normal_out, g->M,
                           (float)(1.0 / g->h));
    } else {
        Corner<double, PACKED> f{(const double *)phi, (const double *)grad, stride};
        hipLaunchKernelGGL((probe_kernel<double, PACKED>), dim3((unsigned)nb), dim3(256), 0, st, f, g->cell_pkg,
                           g->nbr, (const double *)pos, n, (double *)phi_out, (double *)normal_out, g->M,
                           1.0 / g->h);
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

// Workspace of the binned probe, cached on the grid handle.
static sgrid_status probe_workspace(sgrid_grid *g, int64_t n, uint32_t **key, uint32_t **rank, uint32_t **order,
                                    uint32_t **count, uint32_t **sums) {
    const int64_t nt = g->total();
    const int64_t nb = (nt + kScanBlock * kScanPer - 1) / (kScanBlock * kScanPer);
    const size_t need = (size_t)(3 * n + nt + nb + 64) * 4;
    if (need > g->probe_ws_bytes) {
        sgrid::dev_free(g->probe_ws);
        g->probe_ws = nullptr;
        g->probe_ws_bytes = 0;
        sgrid_status s = sgrid::dev_alloc(&g->probe_ws, need, "binned probe workspace");
        if (s != SGRID_OK) return s;
        g->probe_ws_bytes = need;
    }
    uint32_t *w = (uint32_t *)g->probe_ws;
    *key = w;
    *rank = w + n;
    *order = w + 2 * n;
    *count = w + 3 * n;
    *sums = w + 3 * n + nt;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_probe_particles_binned(const sgrid_grid *gc, sgrid_dtype dtype, const void *packed,
                                                     const void *pos, int64_t n, void *phi_out, void *normal_out,
                                                     void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(gc != nullptr, "grid is NULL");
    SG_REQUIRE(n >= 0, "n must be >= 0");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    if (n == 0) return SGRID_OK;
    SG_REQUIRE(packed && pos && phi_out && normal_out, "NULL field or particle array");
    SG_REQUIRE(n < (int64_t)0xFFFFFFFFll, "too many particles for 32-bit ranks");
    const size_t es = dtype == SGRID_F32 ? 4 : 8;
    SG_REQUIRE(sg_aligned(packed, 16), "packed field must be 16-byte aligned");
    SG_REQUIRE(sg_aligned(pos, es) && sg_aligned(phi_out, es) && sg_aligned(normal_out, es),
               "particle arrays must be aligned to their element size");
    sgrid_grid *g = const_cast<sgrid_grid *>(gc);
    hipStream_t st = sg_stream(stream);
    const int64_t nt = g->total();
    uint32_t *key, *rank, *order, *count, *sums;
    sgrid_status s = probe_workspace(g, n, &key, &rank, &order, &count, &sums);
    if (s != SGRID_OK) return s;
    const int64_t nbn = (n + 255) / 256, nbt = (nt + 255) / 256;
    const int64_t nbs = (nt + kScanBlock * kScanPer - 1) / (kScanBlock * kScanPer);
    SG_REQUIRE(nbn <= kMaxGrid, "too many particles for one launch");
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)nbt), dim3(256), 0, st, count, nt, 0u);
    SG_CHECK_LAUNCH("binned probe: clear counts");
    if (dtype == SGRID_F32)
        hipLaunchKernelGGL(key_kernel<float>, dim3((unsigned)nbn), dim3(256), 0, st, (const float *)pos, n, g->cell_pkg,
                           g->M, (float)(1.0 / g->h), key, rank, count);
    else
        hipLaunchKernelGGL(key_kernel<double>, dim3((unsigned)nbn), dim3(256), 0, st, (const double *)pos, n,
                           g->cell_pkg, g->M, 1.0 / g->h, key, rank, count);
    SG_CHECK_LAUNCH("binned probe: keys");
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)nbs), dim3(kScanBlock), 0, st, count, nt, sums);
    SG_CHECK_LAUNCH("binned probe: scan");
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, st, sums, nbs);
    SG_CHECK_LAUNCH("binned probe: scan totals");
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nbt), dim3(256), 0, st, count, nt, sums);
    SG_CHECK_LAUNCH("binned probe: scan offsets");
    hipLaunchKernelGGL(place_kernel, dim3((unsigned)nbn), dim3(256), 0, st, key, rank, count, n, order);
    SG_CHECK_LAUNCH("binned probe: placement");
    if (dtype == SGRID_F32) {
        Corner<float, true> f{(const float *)packed, nullptr, 0};
        hipLaunchKernelGGL((probe_sorted_kernel<float, true>), dim3((unsigned)nbn), dim3(256), 0, st, f, g->cell_pkg,
                           g->nbr, (const float *)pos, order, n, (float *)phi_out, (float *)normal_out, g->M,
                           (float)(1.0 / g->h));
    } else {
        Corner<double, true> f{(const double *)packed, nullptr, 0};
        hipLaunchKernelGGL((probe_sorted_kernel<double, true>), dim3((unsigned)nbn), dim3(256), 0, st, f,
                           g->cell_pkg, g->nbr, (const double *)pos, order, n, (double *)phi_out,
                           (double *)normal_out, g->M, 1.0 / g->h);
    }
    SG_CHECK_LAUNCH("binned probe");
    return SGRID_OK;
}

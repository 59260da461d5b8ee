// Package sweeps: upwind reinitialisation and the central-difference gradient.
//
// Work mapping (both sweeps).  A wavefront owns four consecutive packages;
// 16 lanes per package, and lane r = j + 4k of a package holds the row
// (0..3, j, k) of four x-consecutive values, loaded as one 16-byte (float4)
// or two 16-byte (double) vector loads, so a wavefront reads 1 KiB of
// contiguous package data.  The one-cell halo the stencils need comes from the
// six face neighbours found through the neighbour table (Sec. 5.2):
//   x: the end values of the same row in the -x / +x packages (4-byte loads);
//   y: lanes j = 0 / j = 3 load a whole row of the -y / +y package;
//   z: lanes k = 0 / k = 3 load a whole row of the -z / +z package;
// and interior y / z neighbours move between lanes of the same package with
// DPP row shifts (lane +-1 is y, lane +-4 is z; a package is exactly one
// 16-lane DPP row).  The LDS-staged variant writes the same rows and halos
// into a per-package tile in LDS and reads the neighbours back from there.
#include "common.hpp"

namespace {

template <typename T>
struct Row { T v[4]; };

template <typename T>
__device__ __forceinline__ Row<T> load_row(const T *__restrict__ p);
template <>
__device__ __forceinline__ Row<float> load_row<float>(const float *__restrict__ p) {
    float4 a = *reinterpret_cast<const float4 *>(p);
    return Row<float>{{a.x, a.y, a.z, a.w}};
}
template <>
__device__ __forceinline__ Row<double> load_row<double>(const double *__restrict__ p) {
    double2 a = reinterpret_cast<const double2 *>(p)[0];
    double2 b = reinterpret_cast<const double2 *>(p)[1];
    return Row<double>{{a.x, a.y, b.x, b.y}};
}

template <typename T>
__device__ __forceinline__ void store_row(T *__restrict__ p, const Row<T> &r);
template <>
__device__ __forceinline__ void store_row<float>(float *__restrict__ p, const Row<float> &r) {
    *reinterpret_cast<float4 *>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
}
template <>
__device__ __forceinline__ void store_row<double>(double *__restrict__ p, const Row<double> &r) {
    reinterpret_cast<double2 *>(p)[0] = make_double2(r.v[0], r.v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(r.v[2], r.v[3]);
}

// Godunov-upwinded update of one point (Sussman-Smereka-Osher iteration).
template <typename T>
__device__ __forceinline__ T upwind_update(T p0, T xm, T xp, T ym, T yp, T zm, T zp, T h, T dt) {
    const T S = p0 / sqrt(p0 * p0 + h * h);
    const T nb[6] = {xm, xp, ym, yp, zm, zp};
    T sum = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T dm = (p0 - nb[2 * a]) / h;
        const T dp = (nb[2 * a + 1] - p0) / h;
        T x, y;
        if (S > T(0)) {
            x = fmax(dm, T(0));
            y = fmin(dp, T(0));
        } else {
            x = fmin(dm, T(0));
            y = fmax(dp, T(0));
        }
        sum += fmax(x * x, y * y);
    }
    return S == T(0) ? p0 : p0 - dt * S * (sqrt(sum) - T(1));
}

// Loads a package row and its face halo.  Returns false for lanes past the
// last package (their whole 16-lane row is idle).
template <typename T>
struct Stencil {
    Row<T> c, ym, yp, zm, zp;
    T xm, xp;
};

template <typename T>
__device__ __forceinline__ void gather_halo(const T *__restrict__ src, const uint32_t *__restrict__ face, int64_t p,
                                            int r, Stencil<T> &s) {
    const int j = r & 3, k = r >> 2;
    const uint4 f0 = *reinterpret_cast<const uint4 *>(face + p * 8);
    const uint2 f1 = *reinterpret_cast<const uint2 *>(face + p * 8 + 4);
    s.c = load_row(src + p * 64 + r * 4);
    s.xm = src[(int64_t)f0.x * 64 + r * 4 + 3];
    s.xp = src[(int64_t)f0.y * 64 + r * 4];
    if (j == 0) s.ym = load_row(src + (int64_t)f0.z * 64 + (3 + 4 * k) * 4);
    if (j == 3) s.yp = load_row(src + (int64_t)f0.w * 64 + (4 * k) * 4);
    if (k == 0) s.zm = load_row(src + (int64_t)f1.x * 64 + (j + 12) * 4);
    if (k == 3) s.zp = load_row(src + (int64_t)f1.y * 64 + j * 4);
}

// Interior y / z neighbours through DPP row shifts (all 16 lanes of a package
// execute these together).
template <typename T>
__device__ __forceinline__ void exchange_dpp(int r, Stencil<T> &s) {
    const int j = r & 3, k = r >> 2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const T v = s.c.v[i];
        const T a = row_move<kRowShr1>(v);   // lane - 1: (j - 1, k)
        const T b = row_move<kRowShl1>(v);   // lane + 1: (j + 1, k)
        const T c = row_move<kRowShr4>(v);   // lane - 4: (j, k - 1)
        const T d = row_move<kRowShl4>(v);   // lane + 4: (j, k + 1)
        if (j > 0) s.ym.v[i] = a;
        if (j < 3) s.yp.v[i] = b;
        if (k > 0) s.zm.v[i] = c;
        if (k < 3) s.zp.v[i] = d;
    }
}

template <typename T>
__device__ __forceinline__ Row<T> reinit_row(const Stencil<T> &s, T h, T dt) {
    Row<T> o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const T xm = i > 0 ? s.c.v[i - 1] : s.xm;
        const T xp = i < 3 ? s.c.v[i + 1] : s.xp;
        o.v[i] = upwind_update(s.c.v[i], xm, xp, s.ym.v[i], s.yp.v[i], s.zm.v[i], s.zp.v[i], h, dt);
    }
    return o;
}

// Reinitialisation sweep over packages [2, 2 + P): DPP exchange variant.
// Each wavefront handles `groups` consecutive sets of four packages.
template <typename T>
__global__ __launch_bounds__(256) void reinit_dpp_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                         const uint32_t *__restrict__ face, int64_t P,
                                                         int64_t n_blocks, int groups, T h, T dt) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t wave = b * 4 + (threadIdx.x >> 6);
    for (int gi = 0; gi < groups; ++gi) {
        const int64_t p = 2 + (wave * groups + gi) * 4 + (lane >> 4);
        if (p >= P + 2) return;   // rows past the end are idle together
        Stencil<T> s;
        gather_halo(src, face, p, r, s);
        exchange_dpp(r, s);
        store_row(dst + p * 64 + r * 4, reinit_row(s, h, dt));
    }
}

// LDS-staged variant: every package's rows and its face halo rows are written
// into a 6 x 6 x 6 tile (interior 4^3 plus one-cell faces) in LDS, then each
// lane reads its stencil back from the tile.
template <typename T>
__global__ __launch_bounds__(256) void reinit_lds_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                         const uint32_t *__restrict__ face, int64_t P,
                                                         int64_t n_blocks, int groups, T h, T dt) {
    __shared__ T tile[16][216];
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, j = r & 3, k = r >> 2;
    const int slot = threadIdx.x >> 4;   // package slot of this lane in the block
    T *t = tile[slot];
    auto at = [](int x, int y, int z) { return (x + 1) + 6 * ((y + 1) + 6 * (z + 1)); };
    const int64_t wave = b * 4 + (threadIdx.x >> 6);
    for (int gi = 0; gi < groups; ++gi) {
        const int64_t p = 2 + (wave * groups + gi) * 4 + (lane >> 4);
        const bool live = p < P + 2;
        Stencil<T> s;
        if (live) {
            gather_halo(src, face, p, r, s);
#pragma unroll
            for (int i = 0; i < 4; ++i) t[at(i, j, k)] = s.c.v[i];
            t[at(-1, j, k)] = s.xm;
            t[at(4, j, k)] = s.xp;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (j == 0) t[at(i, -1, k)] = s.ym.v[i];
                if (j == 3) t[at(i, 4, k)] = s.yp.v[i];
                if (k == 0) t[at(i, j, -1)] = s.zm.v[i];
                if (k == 3) t[at(i, j, 4)] = s.zp.v[i];
            }
        }
        __syncthreads();
        if (live) {
            Row<T> o;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                o.v[i] = upwind_update(t[at(i, j, k)], t[at(i - 1, j, k)], t[at(i + 1, j, k)], t[at(i, j - 1, k)],
                                       t[at(i, j + 1, k)], t[at(i, j, k - 1)], t[at(i, j, k + 1)], h, dt);
            store_row(dst + p * 64 + r * 4, o);
        }
        __syncthreads();
    }
}

// Central-difference gradient over packages [0, P + 2); far-field rows get 0.
template <typename T>
__global__ __launch_bounds__(256) void gradient_kernel(const T *__restrict__ phi, T *__restrict__ grad,
                                                       const uint32_t *__restrict__ face, int64_t n_total,
                                                       int64_t n_blocks, T inv_2h) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t p = (b * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
    if (p >= n_total) return;
    T *gx = grad + p * 64 + r * 4;
    T *gy = gx + n_total * 64;
    T *gz = gy + n_total * 64;
    if (p < 2) {
        const Row<T> z{{T(0), T(0), T(0), T(0)}};
        store_row(gx, z);
        store_row(gy, z);
        store_row(gz, z);
        return;
    }
    Stencil<T> s;
    gather_halo(phi, face, p, r, s);
    exchange_dpp(r, s);
    Row<T> ox, oy, oz;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const T xm = i > 0 ? s.c.v[i - 1] : s.xm;
        const T xp = i < 3 ? s.c.v[i + 1] : s.xp;
        ox.v[i] = (xp - xm) * inv_2h;
        oy.v[i] = (s.yp.v[i] - s.ym.v[i]) * inv_2h;
        oz.v[i] = (s.zp.v[i] - s.zm.v[i]) * inv_2h;
    }
    store_row(gx, ox);
    store_row(gy, oy);
    store_row(gz, oz);
}

template <typename T>
__global__ void far_field_kernel(T *__restrict__ phi, T B) {
    const int t = threadIdx.x;   // 128 lanes: rows 0 and 1
    phi[t] = t < 64 ? -B : B;
}

}  // namespace

namespace sgrid {

// Sweep variants selectable by the tuner: 0 = DPP exchange, 1 = LDS tile.
struct SweepConfig {
    int variant = 0;
    int groups = 1;   // sets of four packages per wavefront
};

static SweepConfig g_sweep_cfg;

void set_sweep_config(int variant, int groups) {
    g_sweep_cfg.variant = variant;
    g_sweep_cfg.groups = groups;
}

template <typename T>
static sgrid_status launch_reinit_sweep(const sgrid_grid *g, const T *src, T *dst, hipStream_t st,
                                        const SweepConfig &cfg) {
    if (g->P == 0) return SGRID_OK;
    const int64_t per_block = 16 * (int64_t)cfg.groups;
    const int64_t nb = (g->P + per_block - 1) / per_block;
    const T h = (T)g->h, dt = (T)(0.5 * g->h);
    if (cfg.variant == 1)
        hipLaunchKernelGGL(reinit_lds_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, src, dst, g->face, g->P, nb,
                           cfg.groups, h, dt);
    else
        hipLaunchKernelGGL(reinit_dpp_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, src, dst, g->face, g->P, nb,
                           cfg.groups, h, dt);
    SG_CHECK_LAUNCH("reinit sweep");
    return SGRID_OK;
}

template <typename T>
sgrid_status reinit_impl(const sgrid_grid *g, T *phi, T *scratch, int32_t n_iter, hipStream_t st,
                         const SweepConfig &cfg) {
    if (n_iter == 0) return SGRID_OK;
    // far-field rows of the second buffer: read as halo, never written
    SG_CHECK_HIP(hipMemcpyAsync(scratch, phi, 2 * 64 * sizeof(T), hipMemcpyDeviceToDevice, st));
    T *a = phi, *b = scratch;
    for (int32_t it = 0; it < n_iter; ++it) {
        sgrid_status s = launch_reinit_sweep<T>(g, a, b, st, cfg);
        if (s != SGRID_OK) return s;
        T *t = a;
        a = b;
        b = t;
    }
    if (a != phi)
        SG_CHECK_HIP(hipMemcpyAsync(phi + 128, a + 128, (size_t)g->P * 64 * sizeof(T), hipMemcpyDeviceToDevice, st));
    return SGRID_OK;
}

template sgrid_status reinit_impl<float>(const sgrid_grid *, float *, float *, int32_t, hipStream_t,
                                         const SweepConfig &);

}  // namespace sgrid

extern "C" sgrid_status sgrid_set_sweep_config(int32_t variant, int32_t groups) {
    sgrid::clear_error();
    SG_REQUIRE(variant == 0 || variant == 1, "sweep variant must be 0 or 1 (got %d)", variant);
    SG_REQUIRE(groups >= 1 && groups <= 8, "groups must be in 1..8 (got %d)", groups);
    sgrid::set_sweep_config(variant, groups);
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_fill_far_field(const sgrid_grid *g, sgrid_dtype dtype, void *phi, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr && phi != nullptr, "NULL argument");
    SG_REQUIRE(sg_aligned(phi, 16), "phi is not 16-byte aligned");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    hipStream_t st = sg_stream(stream);
    const double B = sgrid::kFarFieldInH * g->h;
    if (dtype == SGRID_F32)
        hipLaunchKernelGGL(far_field_kernel<float>, dim3(1), dim3(128), 0, st, (float *)phi, (float)B);
    else
        hipLaunchKernelGGL(far_field_kernel<double>, dim3(1), dim3(128), 0, st, (double *)phi, B);
    SG_CHECK_LAUNCH("far-field fill");
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_reinitialize(const sgrid_grid *g, sgrid_dtype dtype, void *phi, void *scratch,
                                           int32_t n_iter, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(phi != nullptr && scratch != nullptr, "phi or scratch is NULL");
    SG_REQUIRE(phi != scratch, "phi and scratch must be distinct buffers");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(scratch, 16), "phi / scratch must be 16-byte aligned");
    SG_REQUIRE(n_iter >= 0, "n_iter must be >= 0 (got %d)", n_iter);
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    hipStream_t st = sg_stream(stream);
    if (dtype == SGRID_F32)
        return sgrid::reinit_impl<float>(g, (float *)phi, (float *)scratch, n_iter, st, sgrid::g_sweep_cfg);
    return sgrid::reinit_impl<double>(g, (double *)phi, (double *)scratch, n_iter, st, sgrid::g_sweep_cfg);
}

extern "C" sgrid_status sgrid_compute_gradient(const sgrid_grid *g, sgrid_dtype dtype, const void *phi, void *grad,
                                               void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(phi != nullptr && grad != nullptr, "phi or grad is NULL");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(grad, 16), "phi / grad must be 16-byte aligned");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    hipStream_t st = sg_stream(stream);
    const int64_t nt = g->total();
    const int64_t nb = (nt + 15) / 16;
    if (dtype == SGRID_F32)
        hipLaunchKernelGGL(gradient_kernel<float>, dim3((unsigned)nb), dim3(256), 0, st, (const float *)phi,
                           (float *)grad, g->face, nt, nb, (float)(0.5 / g->h));
    else
        hipLaunchKernelGGL(gradient_kernel<double>, dim3((unsigned)nb), dim3(256), 0, st, (const double *)phi,
                           (double *)grad, g->face, nt, nb, 0.5 / g->h);
    SG_CHECK_LAUNCH("gradient sweep");
    return SGRID_OK;
}

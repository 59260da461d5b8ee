// Consistency (sign) correction of a layer's distances (Sec. 7.2), the coarse
// step on the mesh cells.  Where an inside/outside test is unreliable (a
// leaky triangle mesh), only the signs of cells near the surface are used as
// given: the core cells, |d| < lc.  Every other cell gets its sign by
// diffusion from them: in rounds of simultaneous updates, a cell without a
// sign takes one when a face neighbour has one, positive if any such
// neighbour is positive, else negative, until a round changes nothing.
//
// The state lives in bitmaps of 64 cells per word along x (the build's word
// layout: W = ceil(M / 64) words per (y, z) row): `dec` marks cells with a
// sign, `pos` the positive ones among them.  One lane per word: x neighbours
// by shifts with the carry bits of the adjacent words, y / z neighbours are
// the same word of the neighbouring rows.  Rounds ping-pong between two
// bitmap pairs; each round raises its own flag when it decides a cell, and
// the host reads a batch of flags at a time.
#include "common.hpp"

namespace {

constexpr int kRoundsPerCheck = 16;

__global__ __launch_bounds__(256) void sign_init_kernel(const float *__restrict__ d, int M, int W, int64_t n_words,
                                                        double lc, uint64_t *__restrict__ dec,
                                                        uint64_t *__restrict__ pos) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_words) return;   // whole wavefronts
    const int lane = threadIdx.x & 63;
    const int64_t r = w / W;
    const int x = (int)(w - r * W) * 64 + lane;
    const float v = x < M ? d[r * M + x] : 1.0f;
    const bool core = x < M && fabs((double)v) < lc;
    const uint64_t bd = __ballot(core);
    const uint64_t bp = __ballot(core && !(v < 0.0f));
    if (lane == 0) {
        dec[w] = bd;
        pos[w] = bp;
    }
}

__global__ __launch_bounds__(256) void sign_round_kernel(const uint64_t *__restrict__ dec,
                                                         const uint64_t *__restrict__ pos, int M, int W,
                                                         int64_t n_words, uint64_t *__restrict__ dec_out,
                                                         uint64_t *__restrict__ pos_out,
                                                         uint32_t *__restrict__ changed) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_words) return;
    const int64_t r = w / W;
    const int b = (int)(w - r * W);
    const int y = (int)(r % M), z = (int)(r / M);
    const uint64_t D = dec[w];
    uint64_t pn = 0, nn = 0;   // cells with a positive / negative face neighbour
    auto add = [&](int64_t v, int shift) {
        const uint64_t dv = dec[v], pv = pos[v] & dv, qv = dv & ~pos[v];
        if (shift > 0) {
            pn |= pv << shift;
            nn |= qv << shift;
        } else if (shift < 0) {
            pn |= pv >> -shift;
            nn |= qv >> -shift;
        } else {
            pn |= pv;
            nn |= qv;
        }
    };
    add(w, 1);    // x - 1 seen at x
    add(w, -1);   // x + 1 seen at x
    if (b > 0) {  // bit 63 of the word below is the x - 1 neighbour of bit 0
        const uint64_t dv = dec[w - 1], pv = pos[w - 1] & dv, qv = dv & ~pos[w - 1];
        pn |= pv >> 63;
        nn |= qv >> 63;
    }
    if (b + 1 < W) {
        const uint64_t dv = dec[w + 1], pv = pos[w + 1] & dv, qv = dv & ~pos[w + 1];
        pn |= pv << 63;
        nn |= qv << 63;
    }
    if (y > 0) add(w - W, 0);
    if (y + 1 < M) add(w + W, 0);
    if (z > 0) add(w - (int64_t)M * W, 0);
    if (z + 1 < M) add(w + (int64_t)M * W, 0);
    const int rem = M - 64 * b;
    const uint64_t valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
    const uint64_t fresh = ~D & (pn | nn) & valid;
    dec_out[w] = D | fresh;
    pos_out[w] = (pos[w] & D) | (fresh & pn);
    if (fresh) *changed = 1u;
}

// Corrected distances: core cells and cells without a sign keep d; the rest
// take |d| with their diffused sign.
__global__ __launch_bounds__(256) void sign_apply_kernel(const float *__restrict__ d, const uint64_t *__restrict__ dec,
                                                         const uint64_t *__restrict__ pos, int M, int W,
                                                         int64_t n_cells, double lc, float *__restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int64_t r = c / M;
    const int x = (int)(c - r * M);
    const int64_t w = r * W + (x >> 6);
    const uint64_t bit = 1ull << (x & 63);
    const float v = d[c];
    const bool core = fabs((double)v) < lc;
    float o = v;
    if (!core && (dec[w] & bit)) o = (pos[w] & bit) ? fabsf(v) : -fabsf(v);
    out[c] = o;
}

__global__ __launch_bounds__(64) void clear_flags_kernel(uint32_t *__restrict__ f, int n) {
    if ((int)threadIdx.x < n) f[threadIdx.x] = 0u;
}

}  // namespace

extern "C" sgrid_status sgrid_correct_signs(const sgrid_desc *desc, const float *d, float *out, void *stream,
                                            int32_t *rounds_out) {
    sgrid::clear_error();
    SG_REQUIRE(desc != nullptr, "desc is NULL");
    SG_REQUIRE(d != nullptr && out != nullptr, "d or out is NULL");
    SG_REQUIRE(sg_aligned(d, 4) && sg_aligned(out, 4), "d / out must be 4-byte aligned");
    SG_REQUIRE(desc->n_coarse >= 1 && desc->n_coarse <= 4096, "n_coarse must be in 1..4096 (got %d)",
               desc->n_coarse);
    SG_REQUIRE(desc->h > 0.0 && desc->h < 1e30, "h must be positive and finite");
    const int64_t M = desc->n_coarse, W = (M + 63) / 64, n_words = M * M * W, n_cells = M * M * M;
    const double lc = 4.0 * desc->h;
    hipStream_t st = sg_stream(stream);
    const size_t bits = (size_t)n_words * 8;
    uint8_t *mem = nullptr;
    sgrid_status s = sgrid::dev_alloc((void **)&mem, 4 * bits + 256, "sign correction bitmaps");
    if (s != SGRID_OK) return s;
    uint64_t *dec[2] = {(uint64_t *)mem, (uint64_t *)(mem + bits)};
    uint64_t *pos[2] = {(uint64_t *)(mem + 2 * bits), (uint64_t *)(mem + 3 * bits)};
    uint32_t *flags = (uint32_t *)(mem + 4 * bits);
    uint32_t *host = nullptr;
    if (hipHostMalloc((void **)&host, kRoundsPerCheck * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        sgrid::dev_free(mem);
        sgrid::set_error("pinned host flags could not be allocated");
        return SGRID_E_NOMEM;
    }
    auto fail = [&](hipError_t e, const char *what) {
        (void)hipStreamSynchronize(st);
        sgrid::dev_free(mem);
        (void)hipHostFree(host);
        sgrid::set_error("%s failed: %s", what, hipGetErrorString(e));
        return SGRID_E_HIP;
    };
    hipLaunchKernelGGL(sign_init_kernel, dim3((unsigned)((n_words + 3) / 4)), dim3(256), 0, st, d, (int)M, (int)W,
                       n_words, lc, dec[0], pos[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(e, "sign init");
    int cur = 0;
    int32_t rounds = 0;
    // every round that decides a cell is followed by one more; at most one
    // face step per round separates any cell from a core cell (3 (M - 1)),
    // so the loop ends by then
    const int64_t max_rounds = 3 * M + kRoundsPerCheck;
    bool done = false;
    for (int64_t base = 0; !done && base < max_rounds; base += kRoundsPerCheck) {
        hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(64), 0, st, flags, kRoundsPerCheck);
        for (int k = 0; k < kRoundsPerCheck; ++k) {
            hipLaunchKernelGGL(sign_round_kernel, dim3((unsigned)((n_words + 255) / 256)), dim3(256), 0, st,
                               dec[cur], pos[cur], (int)M, (int)W, n_words, dec[cur ^ 1], pos[cur ^ 1], flags + k);
            cur ^= 1;
        }
        e = hipGetLastError();
        if (e != hipSuccess) return fail(e, "sign rounds");
        e = hipMemcpyAsync(host, flags, kRoundsPerCheck * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(e, "sign round flags");
        for (int k = 0; k < kRoundsPerCheck; ++k) {
            if (!host[k]) {
                done = true;
                break;
            }
            ++rounds;
        }
    }
    hipLaunchKernelGGL(sign_apply_kernel, dim3((unsigned)((n_cells + 255) / 256)), dim3(256), 0, st, d, dec[cur],
                       pos[cur], (int)M, (int)W, n_cells, lc, out);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(e, "sign apply");
    sgrid::dev_free(mem);
    (void)hipHostFree(host);
    if (rounds_out) *rounds_out = rounds;
    return SGRID_OK;
}

// ---------------------------------------------------------------------------
// The refined step on the data packages (Sec. 7.2: on a refined layer the
// operation is limited to the inner packages).  The points of core packages
// keep their sign, as the core cells do in the coarse step, and so do the
// far-field packages (their constants; a neighbour outside the domain is the
// positive far field, as in the neighbour table).  The points of inner
// packages get their sign by the same rounds of diffusion over face
// neighbours, reached through the six face slots of the package's face row;
// state per point: 0 no sign, 1 negative, 2 positive.
// ---------------------------------------------------------------------------
namespace {

template <typename T>
__global__ __launch_bounds__(256) void point_sign_init_kernel(const T *__restrict__ phi,
                                                              const uint8_t *__restrict__ pkg_type, int64_t n_points,
                                                              uint8_t *__restrict__ state) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_points) return;
    const int64_t p = t >> 6;
    state[t] = pkg_type[p] == 2 ? (uint8_t)0 : (phi[t] < T(0) ? (uint8_t)1 : (uint8_t)2);
}

__global__ __launch_bounds__(256) void point_sign_round_kernel(const uint8_t *__restrict__ state,
                                                               const uint32_t *__restrict__ face, int64_t n_points,
                                                               uint8_t *__restrict__ next,
                                                               uint32_t *__restrict__ changed) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_points) return;
    const uint8_t s = state[t];
    if (s) {
        next[t] = s;
        return;
    }
    const int64_t p = t >> 6;
    const int l = (int)(t & 63), i = l & 3, j = (l >> 2) & 3, k = l >> 4;
    const uint32_t *f = face + p * 8;
    // the six face neighbours: inside the package, or across a face slot
    const int64_t nb[6] = {
        i > 0 ? t - 1 : (int64_t)f[0] * 64 + (l + 3),  i < 3 ? t + 1 : (int64_t)f[1] * 64 + (l - 3),
        j > 0 ? t - 4 : (int64_t)f[2] * 64 + (l + 12), j < 3 ? t + 4 : (int64_t)f[3] * 64 + (l - 12),
        k > 0 ? t - 16 : (int64_t)f[4] * 64 + (l + 48), k < 3 ? t + 16 : (int64_t)f[5] * 64 + (l - 48)};
    bool pos = false, neg = false;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const uint8_t v = state[nb[d]];
        pos = pos || v == 2;
        neg = neg || v == 1;
    }
    const uint8_t o = pos ? 2 : (neg ? 1 : 0);
    next[t] = o;
    if (o) *changed = 1u;
}

template <typename T>
__global__ __launch_bounds__(256) void point_sign_apply_kernel(T *__restrict__ phi, const uint8_t *__restrict__ pkg_type,
                                                               const uint8_t *__restrict__ state, int64_t n_points) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_points) return;
    const uint8_t s = state[t];
    if (pkg_type[t >> 6] == 2 && s) phi[t] = s == 2 ? fabs(phi[t]) : -fabs(phi[t]);
}

template <typename T>
sgrid_status correct_package_signs(const sgrid_grid *g, T *phi, hipStream_t st, int32_t *rounds_out) {
    const int64_t n_points = g->total() * 64;
    const int64_t nb = (n_points + 255) / 256;
    uint8_t *mem = nullptr;
    sgrid_status s = sgrid::dev_alloc((void **)&mem, (size_t)(2 * n_points + 256), "sign correction state");
    if (s != SGRID_OK) return s;
    uint8_t *state[2] = {mem, mem + n_points};
    uint32_t *flags = reinterpret_cast<uint32_t *>(mem + ((2 * n_points + 3) / 4) * 4);
    uint32_t *host = nullptr;
    if (hipHostMalloc((void **)&host, kRoundsPerCheck * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        sgrid::dev_free(mem);
        sgrid::set_error("pinned host flags could not be allocated");
        return SGRID_E_NOMEM;
    }
    auto fail = [&](hipError_t e, const char *what) {
        (void)hipStreamSynchronize(st);
        sgrid::dev_free(mem);
        (void)hipHostFree(host);
        sgrid::set_error("%s failed: %s", what, hipGetErrorString(e));
        return SGRID_E_HIP;
    };
    hipLaunchKernelGGL(point_sign_init_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, phi, g->pkg_type, n_points,
                       state[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(e, "point sign init");
    int cur = 0;
    int32_t rounds = 0;
    bool done = false;
    // every inner point lies within a few face steps of a core package, but
    // the loop only ends on a round that changes nothing (or after as many
    // rounds as there are points)
    for (int64_t base = 0; !done && base < n_points + kRoundsPerCheck; base += kRoundsPerCheck) {
        hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(64), 0, st, flags, kRoundsPerCheck);
        for (int k = 0; k < kRoundsPerCheck; ++k) {
            hipLaunchKernelGGL(point_sign_round_kernel, dim3((unsigned)nb), dim3(256), 0, st, state[cur], g->face,
                               n_points, state[cur ^ 1], flags + k);
            cur ^= 1;
        }
        e = hipGetLastError();
        if (e != hipSuccess) return fail(e, "point sign rounds");
        e = hipMemcpyAsync(host, flags, kRoundsPerCheck * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(e, "point sign round flags");
        for (int k = 0; k < kRoundsPerCheck; ++k) {
            if (!host[k]) {
                done = true;
                break;
            }
            ++rounds;
        }
    }
    hipLaunchKernelGGL(point_sign_apply_kernel<T>, dim3((unsigned)nb), dim3(256), 0, st, phi, g->pkg_type, state[cur],
                       n_points);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(e, "point sign apply");
    sgrid::dev_free(mem);
    (void)hipHostFree(host);
    if (rounds_out) *rounds_out = rounds;
    return SGRID_OK;
}

}  // namespace

extern "C" sgrid_status sgrid_correct_package_signs(const sgrid_grid *g, sgrid_dtype dtype, void *phi, void *stream,
                                                    int32_t *rounds_out) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr && phi != nullptr, "NULL argument");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    SG_REQUIRE(sg_aligned(phi, dtype == SGRID_F32 ? 4 : 8), "phi is not aligned to its element size");
    hipStream_t st = sg_stream(stream);
    if (dtype == SGRID_F32) return correct_package_signs<float>(g, (float *)phi, st, rounds_out);
    return correct_package_signs<double>(g, (double *)phi, st, rounds_out);
}

// Package activation, numbering and neighbour tables (Sec. 4, Sec. 5 and
// Sec. 7.1 steps 1-3 and 5 of the paper), plus the handle lifecycle and error
// reporting of the C ABI.
//
// Pipeline on the caller's stream:
//   tag_kernel      one lane per coarse cell: core = |d| < l_c, inner = not core
//                   with a core 26-neighbour; ballot-count active and core cells
//                   per block;
//   scan_kernel     one workgroup: exclusive scan of the per-block counts;
//   (host)          read back P and n_core once, allocate the package tables;
//   scatter_kernel  ballot + mbcnt rank inside each wavefront, wave offsets in
//                   LDS, block offset from the scan: id = 2 + rank, in ascending
//                   linear order, so no sort is needed;
//   nbr_kernel      one lane per (package, slot): the 27-entry neighbour table and
//                   the six face slots copied into a 32-byte row per package.
#include <stdarg.h>
#include <stdlib.h>
#include <string.h>

#include "common.hpp"

namespace sgrid {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

}  // namespace sgrid

extern "C" const char *sgrid_last_error(void) { return sgrid::g_last_error.c_str(); }

extern "C" int32_t sgrid_version(void) { return 10000; }

namespace {

constexpr int kTagBlock = 256;

__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned lane = threadIdx.x & 63u;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Cell type (0 inactive, 1 core, 2 inner) from the coarse distances.
__device__ __forceinline__ uint8_t cell_type(const float *__restrict__ d, int M, int64_t c, double lc) {
    if (fabs((double)d[c]) < lc) return 1;
    const int64_t MM = (int64_t)M * M;
    const int x = (int)(c % M), y = (int)((c / M) % M), z = (int)(c / MM);
    for (int dz = -1; dz <= 1; ++dz) {
        const int zz = z + dz;
        if (zz < 0 || zz >= M) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= M) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int xx = x + dx;
                if (xx < 0 || xx >= M || (dx == 0 && dy == 0 && dz == 0)) continue;
                if (fabs((double)d[xx + (int64_t)M * yy + MM * zz]) < lc) return 2;
            }
        }
    }
    return 0;
}

// Per-block ballot counts of active and core cells; the cell types are kept
// for the scatter pass.
__global__ __launch_bounds__(kTagBlock) void tag_kernel(const float *__restrict__ d, int M, int64_t n_cells,
                                                        double lc, uint8_t *__restrict__ type,
                                                        uint32_t *__restrict__ cnt_active,
                                                        uint32_t *__restrict__ cnt_core) {
    __shared__ uint32_t s_act[kTagBlock / 64], s_core[kTagBlock / 64];
    const int64_t c = (int64_t)blockIdx.x * kTagBlock + threadIdx.x;
    uint8_t t = 0;
    if (c < n_cells) {
        t = cell_type(d, M, c, lc);
        type[c] = t;
    }
    const uint64_t ba = __ballot(t != 0);
    const uint64_t bc = __ballot(t == 1);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_act[w] = (uint32_t)__popcll(ba);
        s_core[w] = (uint32_t)__popcll(bc);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, k = 0;
        for (int i = 0; i < kTagBlock / 64; ++i) { a += s_act[i]; k += s_core[i]; }
        cnt_active[blockIdx.x] = a;
        cnt_core[blockIdx.x] = k;
    }
}

// Exclusive scan of two count arrays by one workgroup: each thread sums a
// contiguous chunk, the chunk sums are scanned in LDS, then each thread
// rewrites its chunk as offsets.  totals = {P, n_core}.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void scan_kernel(uint32_t *__restrict__ a, uint32_t *__restrict__ b,
                                                            int64_t n, uint64_t *__restrict__ totals) {
    __shared__ uint64_t sa[kScanThreads], sb[kScanThreads];
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
    uint64_t ta = 0, tb = 0;
    for (int64_t i = lo; i < hi; ++i) { ta += a[i]; tb += b[i]; }
    sa[threadIdx.x] = ta;
    sb[threadIdx.x] = tb;
    __syncthreads();
    // Hillis-Steele inclusive scan over the chunk sums
    for (int off = 1; off < kScanThreads; off <<= 1) {
        uint64_t va = threadIdx.x >= off ? sa[threadIdx.x - off] : 0;
        uint64_t vb = threadIdx.x >= off ? sb[threadIdx.x - off] : 0;
        __syncthreads();
        sa[threadIdx.x] += va;
        sb[threadIdx.x] += vb;
        __syncthreads();
    }
    uint64_t ra = sa[threadIdx.x] - ta, rb = sb[threadIdx.x] - tb;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t xa = a[i], xb = b[i];
        a[i] = (uint32_t)ra;
        b[i] = (uint32_t)rb;
        ra += xa;
        rb += xb;
    }
    if (threadIdx.x == kScanThreads - 1) {
        totals[0] = sa[kScanThreads - 1];
        totals[1] = sb[kScanThreads - 1];
    }
}

__global__ __launch_bounds__(kTagBlock) void scatter_kernel(const float *__restrict__ d, const uint8_t *__restrict__ type,
                                                            int64_t n_cells, const uint32_t *__restrict__ off_active,
                                                            const uint32_t *__restrict__ off_core,
                                                            uint32_t *__restrict__ cell_pkg,
                                                            uint32_t *__restrict__ pkg_cell,
                                                            uint8_t *__restrict__ pkg_type,
                                                            uint32_t *__restrict__ core_list) {
    __shared__ uint32_t s_act[kTagBlock / 64], s_core[kTagBlock / 64];
    const int64_t c = (int64_t)blockIdx.x * kTagBlock + threadIdx.x;
    const uint8_t t = c < n_cells ? type[c] : 0;
    const uint64_t ba = __ballot(t != 0);
    const uint64_t bc = __ballot(t == 1);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_act[w] = (uint32_t)__popcll(ba);
        s_core[w] = (uint32_t)__popcll(bc);
    }
    __syncthreads();
    uint32_t wa = off_active[blockIdx.x], wc = off_core[blockIdx.x];
    for (int i = 0; i < w; ++i) { wa += s_act[i]; wc += s_core[i]; }
    if (c >= n_cells) return;
    const uint64_t lt = lanemask_lt();
    if (t != 0) {
        const uint32_t id = 2u + wa + (uint32_t)__popcll(ba & lt);
        cell_pkg[c] = id;
        pkg_cell[id] = (uint32_t)c;
        pkg_type[id] = t;
        if (t == 1) core_list[wc + (uint32_t)__popcll(bc & lt)] = id;
    } else {
        cell_pkg[c] = d[c] < 0.0f ? sgrid::kFarNeg : sgrid::kFarPos;
    }
}

__global__ void far_rows_kernel(uint32_t *__restrict__ pkg_cell, uint8_t *__restrict__ pkg_type) {
    if (threadIdx.x < 2) {
        pkg_cell[threadIdx.x] = sgrid::kNoCell;
        pkg_type[threadIdx.x] = 0;
    }
}

// One lane per (package, slot).
__global__ __launch_bounds__(256) void nbr_kernel(const uint32_t *__restrict__ cell_pkg,
                                                  const uint32_t *__restrict__ pkg_cell, int M,
                                                  int64_t n_total, uint32_t *__restrict__ nbr,
                                                  uint32_t *__restrict__ face) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_total * 27) return;
    const int64_t p = t / 27;
    const int s = (int)(t - p * 27);
    uint32_t v;
    if (p < 2) {
        v = (uint32_t)p;
    } else {
        const int64_t c = pkg_cell[p];
        const int64_t MM = (int64_t)M * M;
        const int x = (int)(c % M) + s % 3 - 1;
        const int y = (int)((c / M) % M) + (s / 3) % 3 - 1;
        const int z = (int)(c / MM) + s / 9 - 1;
        v = (x < 0 || y < 0 || z < 0 || x >= M || y >= M || z >= M) ? sgrid::kFarPos
                                                                      : cell_pkg[x + (int64_t)M * y + MM * z];
    }
    nbr[t] = v;
    // face row: -x, +x, -y, +y, -z, +z, then the package itself twice
    int f = -1;
    switch (s) {
        case 12: f = 0; break;
        case 14: f = 1; break;
        case 10: f = 2; break;
        case 16: f = 3; break;
        case 4: f = 4; break;
        case 22: f = 5; break;
        default: break;
    }
    if (f >= 0) face[p * 8 + f] = v;
    if (s == 13) {
        face[p * 8 + 6] = v;
        face[p * 8 + 7] = v;
    }
}

void free_grid(sgrid_grid *g) {
    if (!g) return;
    hipFree(g->cell_pkg);
    hipFree(g->pkg_cell);
    hipFree(g->pkg_type);
    hipFree(g->nbr);
    hipFree(g->face);
    hipFree(g->core_list);
    delete g;
}

struct Scratch {
    uint8_t *type = nullptr;
    uint32_t *ca = nullptr, *cc = nullptr;
    uint64_t *totals = nullptr;
    ~Scratch() {
        hipFree(type);
        hipFree(ca);
        hipFree(cc);
        hipFree(totals);
    }
};

sgrid_status dev_alloc(void **p, size_t bytes, const char *what) {
    if (bytes == 0) bytes = 4;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        sgrid::set_error("hipMalloc of %zu bytes for %s failed: %s", bytes, what, hipGetErrorString(e));
        return SGRID_E_NOMEM;
    }
    return SGRID_OK;
}

}  // namespace

#define SG_ALLOC(ptr, bytes, what)                                              \
    do {                                                                        \
        sgrid_status _s = dev_alloc((void **)&(ptr), (size_t)(bytes), what);    \
        if (_s != SGRID_OK) { free_grid(g); return _s; }                        \
    } while (0)

#define SG_HIP_OR_FREE(expr)                                                          \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) {                                                       \
            sgrid::set_error("%s failed: %s", #expr, hipGetErrorString(_e));          \
            free_grid(g);                                                             \
            return SGRID_E_HIP;                                                       \
        }                                                                             \
    } while (0)

extern "C" sgrid_status sgrid_build_packages(const sgrid_desc *desc, const float *coarse_sdf, void *stream,
                                             sgrid_grid **out) {
    sgrid::clear_error();
    SG_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    SG_REQUIRE(desc != nullptr, "desc is NULL");
    SG_REQUIRE(coarse_sdf != nullptr, "coarse_sdf is NULL");
    SG_REQUIRE(sg_aligned(coarse_sdf, 4), "coarse_sdf is not 4-byte aligned");
    SG_REQUIRE(desc->n_coarse >= 1, "n_coarse must be >= 1 (got %d)", desc->n_coarse);
    SG_REQUIRE(desc->h > 0.0 && desc->h < 1e30, "h must be positive and finite");
    const int64_t M = desc->n_coarse;
    const int64_t n_cells = M * M * M;
    if (n_cells + 2 > (int64_t)0xFFFFFFFFll || (n_cells + 2) * 64 > ((int64_t)1 << 40)) {
        sgrid::set_error("n_coarse = %lld gives %lld coarse cells, beyond the 32-bit package ids",
                         (long long)M, (long long)n_cells);
        return SGRID_E_CAPACITY;
    }
    hipStream_t st = sg_stream(stream);
    sgrid_grid *g = new sgrid_grid();
    g->M = (int32_t)M;
    g->h = desc->h;
    SG_HIP_OR_FREE(hipGetDevice(&g->device));

    const int64_t nb = (n_cells + kTagBlock - 1) / kTagBlock;
    Scratch s;
    SG_ALLOC(g->cell_pkg, n_cells * 4, "cell_pkg");
    {
        sgrid_status r;
        if ((r = dev_alloc((void **)&s.type, n_cells, "cell types")) != SGRID_OK ||
            (r = dev_alloc((void **)&s.ca, nb * 4, "block counts")) != SGRID_OK ||
            (r = dev_alloc((void **)&s.cc, nb * 4, "block counts")) != SGRID_OK ||
            (r = dev_alloc((void **)&s.totals, 16, "totals")) != SGRID_OK) {
            free_grid(g);
            return r;
        }
    }
    const double lc = 4.0 * desc->h;
    hipLaunchKernelGGL(tag_kernel, dim3((unsigned)nb), dim3(kTagBlock), 0, st, coarse_sdf, (int)M, n_cells, lc,
                       s.type, s.ca, s.cc);
    SG_HIP_OR_FREE(hipGetLastError());
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, st, s.ca, s.cc, nb, s.totals);
    SG_HIP_OR_FREE(hipGetLastError());
    uint64_t totals[2] = {0, 0};
    SG_HIP_OR_FREE(hipMemcpyAsync(totals, s.totals, sizeof totals, hipMemcpyDeviceToHost, st));
    SG_HIP_OR_FREE(hipStreamSynchronize(st));
    g->P = (int64_t)totals[0];
    g->n_core = (int64_t)totals[1];
    const int64_t nt = g->total();
    SG_ALLOC(g->pkg_cell, nt * 4, "pkg_cell");
    SG_ALLOC(g->pkg_type, nt, "pkg_type");
    SG_ALLOC(g->nbr, nt * 27 * 4, "pkg_nbr");
    SG_ALLOC(g->face, nt * 8 * 4, "face table");
    SG_ALLOC(g->core_list, (g->n_core > 0 ? g->n_core : 1) * 4, "core_list");
    hipLaunchKernelGGL(far_rows_kernel, dim3(1), dim3(64), 0, st, g->pkg_cell, g->pkg_type);
    SG_HIP_OR_FREE(hipGetLastError());
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)nb), dim3(kTagBlock), 0, st, coarse_sdf, s.type, n_cells,
                       s.ca, s.cc, g->cell_pkg, g->pkg_cell, g->pkg_type, g->core_list);
    SG_HIP_OR_FREE(hipGetLastError());
    const int64_t nn = nt * 27;
    hipLaunchKernelGGL(nbr_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, g->cell_pkg, g->pkg_cell,
                       (int)M, nt, g->nbr, g->face);
    SG_HIP_OR_FREE(hipGetLastError());
    // the scratch buffers are freed when `s` goes out of scope; wait for the
    // kernels that read them first
    SG_HIP_OR_FREE(hipStreamSynchronize(st));
    *out = g;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_get_info(const sgrid_grid *g, sgrid_info *out) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr && out != nullptr, "NULL argument");
    out->n_coarse = g->M;
    out->h = g->h;
    out->n_packages = g->P;
    out->n_core = g->n_core;
    out->cell_pkg = g->cell_pkg;
    out->pkg_cell = g->pkg_cell;
    out->pkg_type = g->pkg_type;
    out->pkg_nbr = g->nbr;
    out->core_list = g->core_list;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_destroy(sgrid_grid *g) {
    sgrid::clear_error();
    if (!g) return SGRID_OK;
    hipError_t e = hipDeviceSynchronize();
    free_grid(g);
    if (e != hipSuccess) {
        sgrid::set_error("hipDeviceSynchronize before destroy failed: %s", hipGetErrorString(e));
        return SGRID_E_HIP;
    }
    return SGRID_OK;
}

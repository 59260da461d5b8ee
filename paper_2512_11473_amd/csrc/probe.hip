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
#include <algorithm>

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
__device__ __forceinline__ int home_coord(T u, int M) { return (int)clampv(floor(u * T(0.25)), T(0), T(M - 1)); }

template <typename T>
__device__ __forceinline__ void locate(const T *x, int M, T inv_h, int cc[3], int sh[3], T t[3]) {
    const int N = 4 * M;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T u = x[a] * inv_h;
        const T s = u - T(0.5);
        const T f = clampv(floor(s), T(0), T(N - 2));
        t[a] = clampv(s - f, T(0), T(1));
        cc[a] = home_coord(u, M);
        sh[a] = (int)f - 4 * cc[a];
    }
}

// Package ids from the rank map: entry {activated bits, negative bits, rank,
// 0} of the 32 cells holding x gives id = 2 + rank + (activated cells of the
// entry below x) for an activated cell, else the far-field package of its
// sign; cells outside the domain belong to the positive far field (the
// neighbour table's rule).  These are the values of cell_pkg, read from a
// table 64 times smaller that stays in the caches.
constexpr int kProbeMaxM = 4096;   // rank-map indices in 32 bits (cell_pkg alone takes 256 GiB there)
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
// over the eight corners.  The corners' packages are the home cell's package
// and, for corners past a face of the home cell, those of the neighbouring
// cells (the index shift of Sec. 5.2 per axis: slot = (s + 4) / 4, data =
// s + 4 - 4 slot).  A particle whose home cell is far field reads the
// far-field constant at every corner, as the far-field packages neighbour
// themselves.
//
// Per axis the corners lie in at most two cells, c0 <= c1 (equal unless the
// base shift is -1 or 3), and the home cell is one of them.  A rank-map entry
// spans 32 cells along x, so the four (y, z) pairs' entries at c0's x word
// serve all eight corners, except for a particle whose two x cells straddle a
// 32-cell boundary, which also reads the entries at c1's word.  All rank-map
// reads issue before any is used, then all corner reads.
template <typename T, bool PACKED>
__device__ __forceinline__ void blend(const Corner<T, PACKED> &field, const RankMap &rm, const int cc[3],
                                      const int sh[3], const T t[3], T &v, T &gx, T &gy, T &gz) {
    const int M = rm.M;
    int c0[3], c1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c0[a] = cc[a] + ((sh[a] + 4) >> 2) - 1;   // cc - 1 or cc
        c1[a] = cc[a] + ((sh[a] + 5) >> 2) - 1;   // cc or cc + 1
    }
    const int wx0 = max(c0[0], 0) >> 5, wx1 = min(c1[0], M - 1) >> 5;   // x words (cells clamped into the domain)
    // entry index (y + M z) W32 + word, in 32 bits: below M^3 / 32 <= 2^31 for
    // M <= 4096, from products of 24-bit operands (|c| <= M, M W32 <= 2^19);
    // pairs with a cell outside the domain read entry 0 instead
    const int zrow = M * rm.W32;
    const int e00 = __mul24(c0[1], rm.W32) + __mul24(c0[2], zrow) + wx0;
    const int ey = c1[1] != c0[1] ? rm.W32 : 0, ez = c1[2] != c0[2] ? zrow : 0;
    uint4 ea[4], eb[4];
    bool yz_out[4];
    int ei[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int y = (p & 1) ? c1[1] : c0[1], z = (p & 2) ? c1[2] : c0[2];
        yz_out[p] = y < 0 || z < 0 || y >= M || z >= M;
        ei[p] = yz_out[p] ? 0 : e00 + ((p & 1) ? ey : 0) + ((p & 2) ? ez : 0);
        ea[p] = rm.map[(uint32_t)ei[p]];
        eb[p] = ea[p];
    }
    if (wx1 != wx0) {
#pragma unroll
        for (int p = 0; p < 4; ++p) eb[p] = rm.map[(uint32_t)(yz_out[p] ? 0 : ei[p] + 1)];
    }
    uint32_t own[8];
    int d[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        const int x = bx ? c1[0] : c0[0];
        const bool out = x < 0 || x >= M || yz_out[b >> 1];
        own[b] = out ? sgrid::kFarPos : RankMap::id(bx ? eb[b >> 1] : ea[b >> 1], x);
        const int s0 = sh[0] + bx + 4, s1 = sh[1] + by + 4, s2 = sh[2] + bz + 4;   // shift + 4 in [3, 8]
        const int di = s0 - 4 * (s0 >> 2), dj = s1 - 4 * (s1 >> 2), dk = s2 - 4 * (s2 >> 2);   // data index
        d[b] = PACKED ? blocked_index(di, dj, dk) : di + 4 * dj + 16 * dk;
    }
    // the home cell is the corner cell (cc == c0 ? c0 : c1) on every axis
    const int bh = (cc[0] == c0[0] ? 0 : 1) + (cc[1] == c0[1] ? 0 : 2) + (cc[2] == c0[2] ? 0 : 4);
    uint32_t home = own[0];
#pragma unroll
    for (int b = 1; b < 8; ++b) home = b == bh ? own[b] : home;
    uint32_t pk[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) pk[b] = home < 2u ? home : own[b];
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
    // each XCD takes one contiguous stretch of the particles: when they are
    // sorted by home package, its L2 then holds the packages it gathers from
    const int64_t q = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
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
    const int64_t q = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int cc[3], sh[3];
    float t[3], v, gx, gy, gz;
    locate(pos + 3 * q, rm.M, inv_h, cc, sh, t);
    blend(field, rm, cc, sh, t, v, gx, gy, gz);
    out[q] = make_float4(v, gx, gy, gz);
}

// ---------------------------------------------------------------------------
// Particle sort by home cell
// ---------------------------------------------------------------------------
// Probing is position-based random access (Sec. 8): in generated order the
// lanes of a wavefront gather from unrelated packages, about five cache lines
// each.  Sorted by the Morton (Z-order) code of the home coarse cell, the
// particles of one package are adjacent and neighbouring packages close, so a
// wavefront's corners fall on a few shared lines and the packages a stretch of
// particles gathers from stay in the L2 of the XCD that probes them.
//
// LSD radix sort, 9 bits per pass (three passes for 512^3 coarse cells),
// stable, so the result is unique: keys non-decreasing, equal keys in their
// input order.  Per pass, one kernel counts each 4096-element tile's digits in
// LDS, a scan turns the digit-major [512][tiles] counts into output offsets,
// and a second kernel (eight wavefronts, three workgroups per CU)
// ranks the tile's elements stably (wavefront ballots over the digit bits,
// then per-wavefront running counts in LDS), reorders the tile by digit in
// LDS and writes each digit's run contiguously.  The first pass's counts
// compute the keys from the positions and store them for its scatter; the
// last pass writes the permutation and gathers the sorted positions.  Both kernels take their tiles in XCD-aware order: the
// runs of one digit from consecutive tiles are adjacent in the output, and
// the partial cache lines where they meet are then written from one L2.

constexpr int kScanItems = 4096;    // entries per scan block: 1024 lanes x 4
constexpr int kRadixBits = 9, kRadixBins = 1 << kRadixBits;
constexpr int kSortWaves = 8, kSortThreads = 64 * kSortWaves;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;   // 4096 elements per tile
static_assert(kRadixBins <= kSortThreads && kRadixBins % 64 == 0, "one digit per thread of whole wavefronts");

__device__ __forceinline__ uint32_t spread3(uint32_t v) {   // bit b of v (b < 10) to bit 3b
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Morton code of the particle's home coarse cell (x in the lowest bit).
__device__ __forceinline__ uint32_t home_key(const float *x, int M, float inv_h) {
    const int cx = home_coord(x[0] * inv_h, M), cy = home_coord(x[1] * inv_h, M), cz = home_coord(x[2] * inv_h, M);
    return spread3((uint32_t)cx) | (spread3((uint32_t)cy) << 1) | (spread3((uint32_t)cz) << 2);
}

// counts[d * n_tiles + tile] = elements of the tile whose digit is d.
// The first pass's counts compute the keys from the positions and, when the
// sort has more passes, store them for the first scatter (keys_out).
template <bool FIRST>
__global__ __launch_bounds__(256) void radix_count_kernel(const float *__restrict__ pos,
                                                          const uint32_t *__restrict__ keys, int64_t n, int M,
                                                          float inv_h, int shift, uint32_t *__restrict__ counts,
                                                          int64_t n_tiles, uint32_t *__restrict__ keys_out) {
    __shared__ uint32_t s_hist[kRadixBins];
    for (int d = threadIdx.x; d < kRadixBins; d += 256) s_hist[d] = 0u;
    __syncthreads();
    const int64_t tile = xcd_block(blockIdx.x, n_tiles);
    const int64_t t0 = tile * kSortTile;
    if constexpr (FIRST) {
#pragma unroll 4
        for (int k = 0; k < kSortTile / 256; ++k) {
            const int64_t e = t0 + k * 256 + threadIdx.x;
            if (e < n) {
                const uint32_t key = home_key(pos + 3 * e, M, inv_h);
                if (keys_out) keys_out[e] = key;
                atomicAdd(&s_hist[(key >> shift) & (kRadixBins - 1)], 1u);
            }
        }
    } else {
        // four consecutive keys per lane and step, one 16-byte load each (the
        // key arrays are 256-byte aligned and tiles start at multiples of 4),
        // all of a lane's loads issued before its LDS atomics
        constexpr int kSteps = kSortTile / 1024;
        uint4 q[kSteps];
#pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            const int64_t e = t0 + 4 * (k * 256 + threadIdx.x);
            if (e + 3 < n)
                q[k] = *reinterpret_cast<const uint4 *>(keys + e);
            else
                q[k] = make_uint4(e < n ? keys[e] : 0u, e + 1 < n ? keys[e + 1] : 0u, e + 2 < n ? keys[e + 2] : 0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            const int64_t e = t0 + 4 * (k * 256 + threadIdx.x);
            const uint32_t v[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e + u < n) atomicAdd(&s_hist[(v[u] >> shift) & (kRadixBins - 1)], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadixBins; d += 256) counts[(int64_t)d * n_tiles + tile] = s_hist[d];
}

// Exclusive scan of one block of kScanItems entries in place; the block's
// total goes to sums[blockIdx.x].
__global__ __launch_bounds__(1024) void scan_block_kernel(uint32_t *__restrict__ v, int64_t n,
                                                          uint32_t *__restrict__ sums) {
    __shared__ uint32_t s_wave[16];
    const int64_t base = (int64_t)blockIdx.x * kScanItems + 4 * threadIdx.x;
    uint32_t a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = base + k < n ? v[base + k] : 0u;
    const uint32_t own = a[0] + a[1] + a[2] + a[3];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = own;                       // inclusive scan over the wavefront
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
    }
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += s_wave[k];
    uint32_t run = before + inc - own;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t c = a[k];
        if (base + k < n) v[base + k] = run;
        run += c;
    }
    if (threadIdx.x == 1023) sums[blockIdx.x] = run;
}

// Exclusive scan of the block totals by one workgroup, in chunks of 1024.
__global__ __launch_bounds__(1024) void scan_sums_kernel(uint32_t *__restrict__ sums, int64_t nb) {
    __shared__ uint32_t s_wave[16];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        __syncthreads();
        const int64_t i = c0 + threadIdx.x;
        const uint32_t own = i < nb ? sums[i] : 0u;
        uint32_t inc = own;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d);
            if (lane >= d) inc += o;
        }
        if (lane == 63) s_wave[w] = inc;
        __syncthreads();
        uint32_t before = s_carry;
        for (int k = 0; k < w; ++k) before += s_wave[k];
        if (i < nb) sums[i] = before + inc - own;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = before + inc;
    }
}

// One stable pass over a tile: rank, reorder in LDS, write runs.  Element
// order inside the tile: wavefront w holds elements [64 R w, 64 R (w + 1)),
// R = kSortRounds, taken in rounds of 64 consecutive ones.
template <bool FIRST, bool LAST>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(const float *__restrict__ pos,
                                                            const uint32_t *__restrict__ keys_in,
                                                            const uint32_t *__restrict__ idx_in, int64_t n, int M,
                                                            float inv_h, int shift,
                                                            const uint32_t *__restrict__ offs,
                                                            const uint32_t *__restrict__ sums, int64_t n_tiles,
                                                            uint32_t *__restrict__ keys_out,
                                                            uint32_t *__restrict__ idx_out,
                                                            float *__restrict__ pos_out) {
    __shared__ uint32_t s_cnt[kSortWaves][kRadixBins];   // running count per wavefront, then its base
    __shared__ uint32_t s_start[kRadixBins];             // first tile position of each digit
    __shared__ uint32_t s_goff[kRadixBins];              // output position of each digit's run
    __shared__ uint32_t s_key[kSortTile], s_idx[kSortTile];
    __shared__ uint32_t s_wsum[kRadixBins / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kSortWaves * kRadixBins; i += kSortThreads) s_cnt[i / kRadixBins][i % kRadixBins] = 0u;
    __syncthreads();
    const int64_t tile = xcd_block(blockIdx.x, n_tiles);
    const int64_t tile0 = tile * kSortTile;
    const int64_t w0 = tile0 + (int64_t)(64 * kSortRounds) * w;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t key[kSortRounds], idx[kSortRounds], rank[kSortRounds];
#pragma unroll
    for (int j = 0; j < kSortRounds; ++j) {
        const int64_t e = w0 + 64 * j + lane;
        const bool valid = e < n;
        const int64_t ec = valid ? e : n - 1;
        // (a single-pass sort computes the keys here; otherwise the first
        // pass's counts have stored them)
        key[j] = (FIRST && LAST) ? home_key(pos + 3 * ec, M, inv_h) : keys_in[ec];
        idx[j] = FIRST ? (uint32_t)ec : idx_in[ec];
        const uint32_t d = (key[j] >> shift) & (kRadixBins - 1);
        // lanes of this round with the same digit (the valid ones)
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const uint64_t ones = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? ones : ~ones;
        }
        const uint32_t lower = (uint32_t)__popcll(peers & below);
        const uint32_t pre = s_cnt[w][d];
        if (valid && lower == 0) s_cnt[w][d] = pre + (uint32_t)__popcll(peers);
        rank[j] = pre + lower;
    }
    __syncthreads();
    // thread d < kRadixBins owns digit d: its counts in the wavefronts, its
    // tile start (exclusive scan over the digits) and each wavefront's base
    const bool owner = threadIdx.x < kRadixBins;
    const int d = threadIdx.x;
    uint32_t c[kSortWaves], tot = 0;
#pragma unroll
    for (int k = 0; k < kSortWaves; ++k) {
        c[k] = owner ? s_cnt[k][d] : 0u;
        tot += c[k];
    }
    uint32_t inc = tot;
#pragma unroll
    for (int k = 1; k < 64; k <<= 1) {
        const uint32_t o = __shfl_up(inc, k);
        if (lane >= k) inc += o;
    }
    if (owner && lane == 63) s_wsum[w] = inc;
    __syncthreads();
    if (owner) {
        uint32_t start = inc - tot;
        for (int k = 0; k < w; ++k) start += s_wsum[k];
        s_start[d] = start;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) {
            s_cnt[k][d] = start;
            start += c[k];
        }
        const int64_t oi = (int64_t)d * n_tiles + tile;
        s_goff[d] = offs[oi] + sums[oi / kScanItems];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortRounds; ++j) {
        const int64_t e = w0 + 64 * j + lane;
        if (e < n) {
            const uint32_t p = s_cnt[w][(key[j] >> shift) & (kRadixBins - 1)] + rank[j];
            s_key[p] = key[j];
            s_idx[p] = idx[j];
        }
    }
    __syncthreads();
    const int64_t n_tile = n - tile0 < kSortTile ? n - tile0 : kSortTile;
#pragma unroll 4
    for (int k = 0; k < kSortTile / kSortThreads; ++k) {
        const int p = k * kSortThreads + threadIdx.x;
        if (p < n_tile) {
            const uint32_t kp = s_key[p], ip = s_idx[p];
            const uint32_t dd = (kp >> shift) & (kRadixBins - 1);
            const int64_t dest = (int64_t)s_goff[dd] + (p - (int64_t)s_start[dd]);
            if (LAST) {
                idx_out[dest] = ip;
                pos_out[3 * dest] = pos[3 * (int64_t)ip];
                pos_out[3 * dest + 1] = pos[3 * (int64_t)ip + 1];
                pos_out[3 * dest + 2] = pos[3 * (int64_t)ip + 2];
            } else {
                keys_out[dest] = kp;
                idx_out[dest] = ip;
            }
        }
    }
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
    SG_REQUIRE(g->M <= kProbeMaxM, "the probe takes grids of at most %d coarse cells per axis (got %d)", kProbeMaxM,
               (int)g->M);
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
    SG_REQUIRE(g->M <= kProbeMaxM, "the probe takes grids of at most %d coarse cells per axis (got %d)", kProbeMaxM,
               (int)g->M);
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

namespace {
constexpr int64_t kSortMaxParticles = 0xFFFFFFFFll;   // 32-bit permutation entries

// Layout of the sort's workspace for n particles: key and index ping-pong
// buffers (when there is more than one pass), the digit counts of every tile
// and the scan's block totals, each 256-byte aligned.
struct SortPlan {
    int passes = 0;
    int64_t n_tiles = 0, n_counts = 0, n_sums = 0;
    int64_t off_keys[2] = {0, 0}, off_idx[2] = {0, 0}, off_counts = 0, off_sums = 0, bytes = 0;
};

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

SortPlan sort_plan(const sgrid_grid *g, int64_t n) {
    SortPlan s;
    int bits_axis = 0;
    while ((1 << bits_axis) < g->M) ++bits_axis;
    s.passes = std::max(1, (3 * bits_axis + kRadixBits - 1) / kRadixBits);
    s.n_tiles = (n + kSortTile - 1) / kSortTile;
    s.n_counts = (int64_t)kRadixBins * s.n_tiles;
    s.n_sums = (s.n_counts + kScanItems - 1) / kScanItems;
    int64_t b = 0;
    if (s.passes > 1)
        for (int k = 0; k < 2; ++k) {
            s.off_keys[k] = b;
            b += align256(4 * n);
            s.off_idx[k] = b;
            b += align256(4 * n);
        }
    s.off_counts = b;
    b += align256(4 * s.n_counts);
    s.off_sums = b;
    b += align256(4 * std::max<int64_t>(1, s.n_sums));
    s.bytes = b;
    return s;
}

template <bool FIRST, bool LAST>
sgrid_status radix_pass(const sgrid_grid *g, const float *pos, const uint32_t *keys_in, const uint32_t *idx_in,
                        int64_t n, int shift, const SortPlan &sp, uint32_t *counts, uint32_t *sums,
                        uint32_t *keys_out, uint32_t *idx_out, float *pos_out, hipStream_t st) {
    const float inv_h = (float)(1.0 / g->h);
    // the first of several passes: the counts store the keys where the scatter reads them
    uint32_t *first_keys = FIRST && !LAST ? const_cast<uint32_t *>(keys_in) : nullptr;
    hipLaunchKernelGGL(radix_count_kernel<FIRST>, dim3((unsigned)sp.n_tiles), dim3(256), 0, st, pos, keys_in, n, g->M,
                       inv_h, shift, counts, sp.n_tiles, first_keys);
    SG_CHECK_LAUNCH("sort digit counts");
    hipLaunchKernelGGL(scan_block_kernel, dim3((unsigned)sp.n_sums), dim3(1024), 0, st, counts, sp.n_counts, sums);
    SG_CHECK_LAUNCH("sort scan");
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, sums, sp.n_sums);
    SG_CHECK_LAUNCH("sort scan of block totals");
    hipLaunchKernelGGL((radix_scatter_kernel<FIRST, LAST>), dim3((unsigned)sp.n_tiles), dim3(kSortThreads), 0, st, pos,
                       keys_in, idx_in, n, g->M, inv_h, shift, (const uint32_t *)counts, (const uint32_t *)sums,
                       sp.n_tiles, keys_out, idx_out, pos_out);
    SG_CHECK_LAUNCH("sort scatter");
    return SGRID_OK;
}
}  // namespace

extern "C" sgrid_status sgrid_sort_particles_workspace_size(const sgrid_grid *g, int64_t n, int64_t *bytes) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr && bytes != nullptr, "grid or bytes is NULL");
    SG_REQUIRE(n >= 0 && n <= kSortMaxParticles, "n = %lld is outside [0, 2^32 - 1]", (long long)n);
    *bytes = sort_plan(g, n).bytes;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_sort_particles(const sgrid_grid *g, const float *pos, int64_t n, float *pos_sorted,
                                             uint32_t *perm, void *workspace, int64_t workspace_bytes,
                                             void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(n >= 0 && n <= kSortMaxParticles, "n = %lld is outside [0, 2^32 - 1]", (long long)n);
    if (n == 0) return SGRID_OK;
    SG_REQUIRE(pos && pos_sorted && perm && workspace, "NULL particle array or workspace");
    SG_REQUIRE(pos != pos_sorted, "pos and pos_sorted must be distinct");
    SG_REQUIRE(sg_aligned(pos, 4) && sg_aligned(pos_sorted, 4) && sg_aligned(perm, 4) && sg_aligned(workspace, 256),
               "arrays must be 4-byte aligned, the workspace 256-byte aligned");
    const SortPlan sp = sort_plan(g, n);
    SG_REQUIRE(workspace_bytes >= sp.bytes, "workspace holds %lld bytes, the sort needs %lld",
               (long long)workspace_bytes, (long long)sp.bytes);
    SG_REQUIRE(sp.n_tiles <= kMaxGrid, "too many particles for one launch");
    hipStream_t st = sg_stream(stream);
    char *ws = static_cast<char *>(workspace);
    uint32_t *keys[2] = {(uint32_t *)(ws + sp.off_keys[0]), (uint32_t *)(ws + sp.off_keys[1])};
    uint32_t *idx[2] = {(uint32_t *)(ws + sp.off_idx[0]), (uint32_t *)(ws + sp.off_idx[1])};
    uint32_t *counts = (uint32_t *)(ws + sp.off_counts), *sums = (uint32_t *)(ws + sp.off_sums);
    sgrid_status s;
    if (sp.passes == 1)
        return radix_pass<true, true>(g, pos, nullptr, nullptr, n, 0, sp, counts, sums, nullptr, perm, pos_sorted, st);
    // (keys[1] holds the first pass's keys until the second pass writes it)
    s = radix_pass<true, false>(g, pos, keys[1], nullptr, n, 0, sp, counts, sums, keys[0], idx[0], nullptr, st);
    if (s != SGRID_OK) return s;
    int cur = 0;
    for (int p = 1; p + 1 < sp.passes; ++p, cur ^= 1) {
        s = radix_pass<false, false>(g, pos, keys[cur], idx[cur], n, p * kRadixBits, sp, counts, sums, keys[cur ^ 1],
                                     idx[cur ^ 1], nullptr, st);
        if (s != SGRID_OK) return s;
    }
    return radix_pass<false, true>(g, pos, keys[cur], idx[cur], n, (sp.passes - 1) * kRadixBits, sp, counts, sums,
                                   nullptr, perm, pos_sorted, st);
}

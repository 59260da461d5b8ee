// Package activation, numbering and neighbour tables (Sec. 4, Sec. 5 and
// Sec. 7.1 steps 1-3 and 5 of the paper), plus the handle lifecycle and error
// reporting of the C ABI.
//
// Pipeline on the caller's stream (coarse cells held as bitmaps, 64 cells of a
// row per word):
//   bits_kernel     one wavefront per 16 words: core flag |d| < l_c and sign of d,
//                   one ballot each;
//   dilate_kernel   one lane per word: activated = core dilated by one cell in
//                   x, y, z (word shifts and ORs); per-group counts;
//   scan_pair       exclusive scan of the counts (block sums, one workgroup
//                   over them, block scans);
//   (host)          read back P and n_core once, allocate the package tables;
//   scatter_kernel  16 words per wavefront in steps of four, four cells per lane: rank by
//                   popcount below the cell plus word offsets from the scan,
//                   id = 2 + rank in ascending linear order (no sort needed);
//                   the cell map in 16-byte stores, the rank map;
//   nbr_kernel      27 lanes per four packages: the neighbour table and the six
//                   face slots copied into a 32-byte row per package;
//   morton_*        the sweep worklist in Morton order of the cells, one lane
//                   per 4 x 4 x 4 box of codes.
// The next layer of the multi-resolution construction replaces bits_kernel by
// refine_bits_kernel (the parent layer's rank map and the children's
// distances) and shares the rest.
#include <stdarg.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <unordered_map>
#include <vector>

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

namespace {
struct CachedBlock {
    void *ptr;
    size_t bytes;
    int device;
};
std::mutex g_alloc_mu;
std::vector<CachedBlock> g_free_blocks;
std::unordered_map<void *, CachedBlock> g_live_blocks;

size_t round_bytes(size_t b) {
    const size_t q = b <= (1u << 20) ? 4096 : (2u << 20);
    return (b + q - 1) / q * q;
}
}  // namespace

sgrid_status dev_alloc(void **p, size_t bytes, const char *what) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    const size_t rb = round_bytes(bytes == 0 ? 1 : bytes);
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        for (size_t i = 0; i < g_free_blocks.size(); ++i) {
            if (g_free_blocks[i].bytes == rb && g_free_blocks[i].device == dev) {
                CachedBlock b = g_free_blocks[i];
                g_free_blocks[i] = g_free_blocks.back();
                g_free_blocks.pop_back();
                g_live_blocks[b.ptr] = b;
                *p = b.ptr;
                return SGRID_OK;
            }
        }
    }
    hipError_t e = hipMalloc(p, rb);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // give cached blocks back to the driver and retry once
        std::vector<CachedBlock> drop;
        {
            std::lock_guard<std::mutex> lk(g_alloc_mu);
            drop.swap(g_free_blocks);
        }
        for (auto &b : drop) (void)hipFree(b.ptr);
        e = hipMalloc(p, rb);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("allocation of %zu bytes for %s failed: %s", bytes, what, hipGetErrorString(e));
        return SGRID_E_NOMEM;
    }
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_live_blocks[*p] = CachedBlock{*p, rb, dev};
    return SGRID_OK;
}

void dev_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_live_blocks.find(p);
    if (it == g_live_blocks.end()) return;
    g_free_blocks.push_back(it->second);
    g_live_blocks.erase(it);
}

int cu_count() {
    static std::atomic<int> cached[64];   // 0 until first asked; threads that race store the same value
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) return 256;
    int n = cached[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

}  // namespace sgrid

extern "C" const char *sgrid_last_error(void) { return sgrid::g_last_error.c_str(); }

extern "C" int32_t sgrid_version(void) { return 10000; }

namespace {

constexpr int kTagBlock = 256;

__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned lane = threadIdx.x & 63u;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Quotient of a word or row index by a row length, in 32-bit arithmetic when
// the index fits (M^2 W words stay below 2^32 up to M = 4096): a few
// instructions instead of the fifty of a 64-bit division.
__device__ __forceinline__ int64_t quot(int64_t a, int b) {
    return a < 0x100000000ll ? (int64_t)((uint32_t)a / (uint32_t)b) : a / b;
}

// Bitmaps of the background grid.  Row r = y + M z holds its M cells in
// W = ceil(M / 64) words; bit b of word r W + i is the cell x = 64 i + b.
// Bits of x >= M are zero.  Word order is linear cell order.

// Pass 1: one wavefront per word: the core flag |d| < l_c (compared in double,
// so that a non-representable l_c rounds as the definition does) and the sign
// of d, each one ballot.
constexpr int kBitsWords = 16;   // words per wavefront of bits_kernel

__global__ __launch_bounds__(256) void bits_kernel(const float *__restrict__ d, int M, int W, int64_t n_words,
                                                   double lc, uint64_t *__restrict__ core,
                                                   uint64_t *__restrict__ neg) {
    // kBitsWords consecutive words per wavefront, their loads issued together
    // (4 KiB in flight per wavefront); the words' rows and offsets advance
    // from the first word's (one division per wavefront)
    const int64_t w0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kBitsWords;
    if (w0 >= n_words) return;   // whole wavefronts
    const int lane = threadIdx.x & 63;
    const int64_t r0 = quot(w0, W);
    const int i0 = (int)(w0 - r0 * W);
    float v[kBitsWords];
    bool in[kBitsWords];
    {
        int64_t r = r0;
        int i = i0;
#pragma unroll
        for (int k = 0; k < kBitsWords; ++k) {
            const int x = i * 64 + lane;
            in[k] = w0 + k < n_words && x < M;
            v[k] = d[in[k] ? r * M + x : 0];   // every lane loads, in bounds
            if (++i == W) {
                i = 0;
                ++r;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kBitsWords; ++k) {
        const int64_t w = w0 + k;
        const uint64_t bc = __ballot(in[k] && fabs((double)v[k]) < lc);
        const uint64_t bn = __ballot(in[k] && v[k] < 0.0f);
        if (lane == 0 && w < n_words) {
            core[w] = bc;
            neg[w] = bn;
        }
    }
}

// Pass 2: one lane per word: the activated cells are the core cells dilated by
// one cell along x, y and z (the cell and its 26 neighbours, Sec. 7.1 steps
// 1-2: inner = not core with a core neighbour); per group of 16 words, the
// counts of activated and of core cells feed the scan.
__global__ __launch_bounds__(256) void dilate_kernel(const uint64_t *__restrict__ core, int M, int W,
                                                     int64_t n_words, uint64_t *__restrict__ act,
                                                     uint32_t *__restrict__ cnt_act,
                                                     uint32_t *__restrict__ cnt_core) {
    const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint64_t a = 0, own = 0;
    if (w < n_words) {
        const int64_t r = quot(w, W);
        const int i = (int)(w - r * W);
        const int64_t rz = quot(r, M);
        const int y = (int)(r - rz * M), z = (int)rz;
        for (int dz = -1; dz <= 1; ++dz) {
            const int zz = z + dz;
            if (zz < 0 || zz >= M) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = y + dy;
                if (yy < 0 || yy >= M) continue;
                const int64_t b = ((int64_t)yy + (int64_t)M * zz) * W + i;
                const uint64_t c = core[b];
                const uint64_t lo = i > 0 ? core[b - 1] : 0ull, hi = i < W - 1 ? core[b + 1] : 0ull;
                a |= c | (c << 1) | (c >> 1) | (lo >> 63) | (hi << 63);
            }
        }
        if (i == W - 1 && (M & 63)) a &= (1ull << (M & 63)) - 1ull;
        own = core[w];
    }
    uint32_t na = (uint32_t)__popcll(a), nc = (uint32_t)__popcll(own);
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
        na += __shfl_xor(na, off, 16);
        nc += __shfl_xor(nc, off, 16);
    }
    if (w < n_words) {
        act[w] = a;
        if ((threadIdx.x & 15) == 0) {
            cnt_act[w >> 4] = na;
            cnt_core[w >> 4] = nc;
        }
    }
}

// Exclusive scan of two count arrays in three passes: per-block sums of
// kScanBlock entries, one workgroup scanning the block sums (and writing the
// totals), then every block scanning its entries from its offset.
constexpr int kScanThreads = 1024;
constexpr int kScanTile = kScanThreads * 4;
constexpr int kScanBlock = 1024;   // entries per block of the first and last pass (256 lanes x 4)

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                                                          int64_t n, uint32_t *__restrict__ sa,
                                                          uint32_t *__restrict__ sb) {
    __shared__ uint32_t ra[4], rb[4];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
    uint32_t xa = 0, xb = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < n) {
            xa += a[base + k];
            xb += b[base + k];
        }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        xa += __shfl_xor(xa, off);
        xb += __shfl_xor(xb, off);
    }
    if ((threadIdx.x & 63) == 0) {
        ra[threadIdx.x >> 6] = xa;
        rb[threadIdx.x >> 6] = xb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sa[blockIdx.x] = ra[0] + ra[1] + ra[2] + ra[3];
        sb[blockIdx.x] = rb[0] + rb[1] + rb[2] + rb[3];
    }
}

// One workgroup, in tiles of kScanTile entries: coalesced loads into LDS, a
// sequential scan of 4 entries per thread, a Hillis-Steele scan of the thread
// sums, coalesced stores, and a running carry between tiles.  totals = the
// two sums.
__global__ __launch_bounds__(kScanThreads) void scan_kernel(uint32_t *__restrict__ a, uint32_t *__restrict__ b,
                                                            int64_t n, uint64_t *__restrict__ totals) {
    __shared__ uint32_t ta[kScanTile], tb[kScanTile];
    __shared__ uint64_t sa[kScanThreads], sb[kScanThreads];
    uint64_t carry_a = 0, carry_b = 0;
    const int t = threadIdx.x;
    for (int64_t base = 0; base < n; base += kScanTile) {
        for (int i = t; i < kScanTile; i += kScanThreads) {
            const int64_t g = base + i;
            ta[i] = g < n ? a[g] : 0u;
            tb[i] = g < n ? b[g] : 0u;
        }
        __syncthreads();
        uint64_t xa = 0, xb = 0;
        for (int i = 0; i < 4; ++i) { xa += ta[4 * t + i]; xb += tb[4 * t + i]; }
        sa[t] = xa;
        sb[t] = xb;
        __syncthreads();
        for (int off = 1; off < kScanThreads; off <<= 1) {
            const uint64_t va = t >= off ? sa[t - off] : 0, vb = t >= off ? sb[t - off] : 0;
            __syncthreads();
            sa[t] += va;
            sb[t] += vb;
            __syncthreads();
        }
        uint64_t ra = carry_a + sa[t] - xa, rb = carry_b + sb[t] - xb;
        for (int i = 0; i < 4; ++i) {
            const uint32_t va = ta[4 * t + i], vb = tb[4 * t + i];
            ta[4 * t + i] = (uint32_t)ra;
            tb[4 * t + i] = (uint32_t)rb;
            ra += va;
            rb += vb;
        }
        carry_a += sa[kScanThreads - 1];
        carry_b += sb[kScanThreads - 1];
        __syncthreads();
        for (int i = t; i < kScanTile; i += kScanThreads) {
            const int64_t g = base + i;
            if (g < n) {
                a[g] = ta[i];
                b[g] = tb[i];
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        totals[0] = carry_a;
        totals[1] = carry_b;
    }
}

__global__ __launch_bounds__(256) void scan_apply_kernel(uint32_t *__restrict__ a, uint32_t *__restrict__ b, int64_t n,
                                                         const uint32_t *__restrict__ off_a,
                                                         const uint32_t *__restrict__ off_b) {
    __shared__ uint32_t wa[4], wb[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + t * 4;
    uint32_t va[4], vb[4], xa = 0, xb = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        va[k] = base + k < n ? a[base + k] : 0u;
        vb[k] = base + k < n ? b[base + k] : 0u;
        xa += va[k];
        xb += vb[k];
    }
    // inclusive scan of the thread sums inside the wavefront
    uint32_t ia = xa, ib = xb;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t pa = __shfl_up(ia, off), pb = __shfl_up(ib, off);
        if (lane >= off) {
            ia += pa;
            ib += pb;
        }
    }
    if (lane == 63) {
        wa[wv] = ia;
        wb[wv] = ib;
    }
    __syncthreads();
    uint32_t ra = off_a[blockIdx.x] + ia - xa, rb = off_b[blockIdx.x] + ib - xb;
    for (int k = 0; k < wv; ++k) {
        ra += wa[k];
        rb += wb[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < n) {
            a[base + k] = ra;
            b[base + k] = rb;
            ra += va[k];
            rb += vb[k];
        }
}

// Exclusive scan of a[n] and b[n] in place; totals = {sum a, sum b}.  part
// holds 2 * ceil(n / kScanBlock) words.
static void scan_pair(uint32_t *a, uint32_t *b, int64_t n, uint32_t *part, uint64_t *totals, hipStream_t st) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb <= 1) {
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, st, a, b, n, totals);
        return;
    }
    uint32_t *pa = part, *pb = part + nb;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, b, n, pa, pb);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, st, pa, pb, nb, totals);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, b, n, pa, pb);
}

// Pass 4: numbering.  One workgroup per group of 16 words, four words per
// wavefront.  Cell x of word w gets id = 2 + (activated cells before the word:
// the group's offset from the scan plus the words before it in the group) +
// (activated cells of the word below x), which is ascending linear order, so
// no sort is needed.  Cells not activated take the far-field package of their
// sign.
__global__ __launch_bounds__(256) void scatter_kernel(const uint64_t *__restrict__ act,
                                                      const uint64_t *__restrict__ core,
                                                      const uint64_t *__restrict__ neg, int M, int W,
                                                      int64_t n_words, const uint32_t *__restrict__ off_act,
                                                      const uint32_t *__restrict__ off_core,
                                                      uint32_t *__restrict__ cell_pkg,
                                                      uint32_t *__restrict__ pkg_cell,
                                                      uint8_t *__restrict__ pkg_type,
                                                      uint32_t *__restrict__ core_list,
                                                      uint4 *__restrict__ rank_map, int W32) {
    // a wavefront owns one group of 16 words, in four steps of four
    // consecutive words; in a step lane l takes the four cells of bits
    // 4 (l mod 16) .. 4 (l mod 16) + 3 of word l / 16, stored with one 16-byte
    // write where the row allows it.  Lane l < 16 loads word l of the group
    // (the loads issued together) and the counts before each word come from
    // one scan over the 16 lanes; the other lanes read words and counts from
    // them.
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t grp = (int64_t)blockIdx.x * 4 + wv;
    const int64_t g0 = grp * 16;
    if (g0 >= n_words) return;   // the same for the whole wavefront
    const int64_t wl = g0 + (lane & 15);
    const bool inl = wl < n_words;
    const uint64_t la = inl ? act[wl] : 0ull, lcw = inl ? core[wl] : 0ull, ln = inl ? neg[wl] : 0ull;
    uint32_t ea = (uint32_t)__popcll(la), ec = (uint32_t)__popcll(lcw);   // inclusive, then exclusive, counts
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        const uint32_t ta = __shfl_up(ea, o, 16), tc = __shfl_up(ec, o, 16);
        if ((lane & 15) >= o) {
            ea += ta;
            ec += tc;
        }
    }
    ea -= (uint32_t)__popcll(la);
    ec -= (uint32_t)__popcll(lcw);
    const uint32_t pa = off_act[grp], pc = off_core[grp];
    auto word = [](uint64_t v, int src) {
        return ((uint64_t)(uint32_t)__shfl((int)(v >> 32), src) << 32) | (uint32_t)__shfl((int)(uint32_t)v, src);
    };
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        const int64_t w0 = g0 + 4 * step;
        if (w0 >= n_words) break;
        // the rank map entries of the four words' 32-cell halves (lanes 0..7)
        {
            const int k = (lane >> 1) & 3, hf = lane & 1;
            const int j = 4 * step + k;
            const uint64_t aj = word(la, j), nj = word(ln, j);
            const uint32_t before_j = (uint32_t)__shfl((int)ea, j);
            const int64_t w = w0 + k;
            if (lane < 8 && w < n_words) {
                const int64_t r = quot(w, W);
                const int half = (int)(w - r * W) * 2 + hf;
                if (half < W32) {
                    const uint32_t before = pa + before_j + (hf ? (uint32_t)__popc((uint32_t)aj) : 0u);
                    rank_map[r * W32 + half] = make_uint4((uint32_t)(hf ? aj >> 32 : aj),
                                                          (uint32_t)(hf ? nj >> 32 : nj), before, 0u);
                }
            }
        }
        const int k = lane >> 4, b0 = 4 * (lane & 15);
        const int j = 4 * step + k;
        const uint64_t ak = word(la, j), ck = word(lcw, j), nk = word(ln, j);
        uint32_t ra = pa + (uint32_t)__shfl((int)ea, j), rc = pc + (uint32_t)__shfl((int)ec, j);
        const int64_t w = w0 + k;
        if (w >= n_words) continue;
        const uint64_t below = (1ull << b0) - 1ull;
        ra += (uint32_t)__popcll(ak & below);
        rc += (uint32_t)__popcll(ck & below);
        const int64_t r = quot(w, W);
        const int x0 = (int)(w - r * W) * 64 + b0;
        if (x0 >= M) continue;
        uint32_t v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int bit = b0 + i;
            const int64_t c = r * M + x0 + i;
            if ((ak >> bit) & 1ull) {
                const uint32_t id = 2u + ra++;
                v[i] = id;
                if (x0 + i < M) {
                    pkg_cell[id] = (uint32_t)c;
                    const bool is_core = (ck >> bit) & 1ull;
                    pkg_type[id] = is_core ? 1 : 2;
                    if (is_core) core_list[rc++] = id;
                }
            } else {
                v[i] = ((nk >> bit) & 1ull) ? sgrid::kFarNeg : sgrid::kFarPos;
            }
        }
        uint32_t *dst = cell_pkg + r * M + x0;
        if ((M & 3) == 0) {   // x0 and M multiples of 4: the four cells are in the row and 16-byte aligned
            *reinterpret_cast<uint4 *>(dst) = make_uint4(v[0], v[1], v[2], v[3]);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (x0 + i < M) dst[i] = v[i];
        }
    }
}

// Sweep order: the activated packages listed in Morton (Z-curve) order of
// their coarse cells, so the packages one workgroup sweeps together are
// spatial neighbours and share their halo lines in the caches.  The codes run
// over the enclosing power-of-two cube; codes outside the grid are skipped.
// One lane per 64 consecutive codes, which cover a 4 x 4 x 4 box of cells:
// the box's activation is 16 four-bit pieces of the bitmap (one per (y, z)
// row, never straddling a word as the box is 4-aligned), gathered into one
// 64-bit mask, bit lx + 4 ly + 16 lz.  Most boxes of a narrow band are empty
// and cost 16 word reads; a box with activated cells is walked in Morton order
// and reads the package id of its activated cells only.
constexpr int kCodesPerBlock = kTagBlock * 64;

__device__ __forceinline__ void morton_decode(int64_t code, int bits, int &x, int &y, int &z) {
    x = y = z = 0;
    for (int b = 0; b < bits; ++b) {
        x |= (int)((code >> (3 * b)) & 1) << b;
        y |= (int)((code >> (3 * b + 1)) & 1) << b;
        z |= (int)((code >> (3 * b + 2)) & 1) << b;
    }
}

// Activation mask of the box of codes 64 box .. 64 box + 63 and its origin
// cell; 0 when the box lies past the codes or the grid.
__device__ __forceinline__ uint64_t box_mask(const uint64_t *__restrict__ act, int M, int W, int bits,
                                             int64_t box, int64_t n_codes, int &ox, int &oy, int &oz) {
    ox = oy = oz = 0;
    if (box * 64 >= n_codes) return 0ull;
    if (bits > 2) {
        morton_decode(box, bits - 2, ox, oy, oz);
        ox *= 4;
        oy *= 4;
        oz *= 4;
    }
    if (ox >= M || oy >= M || oz >= M) return 0ull;
    const int nx = M - ox;
    const uint64_t xm = nx >= 4 ? 0xFull : ((1ull << nx) - 1ull);
    uint64_t m = 0;
#pragma unroll
    for (int lz = 0; lz < 4; ++lz)
#pragma unroll
        for (int ly = 0; ly < 4; ++ly) {
            const int y = oy + ly, z = oz + lz;
            const uint64_t w = (y < M && z < M) ? act[((int64_t)y + (int64_t)M * z) * W + (ox >> 6)] : 0ull;
            m |= ((w >> (ox & 63)) & xm) << (4 * (ly + 4 * lz));
        }
    return m;
}

__global__ __launch_bounds__(kTagBlock) void morton_count_kernel(const uint64_t *__restrict__ act, int M, int W,
                                                                 int bits, int64_t n_codes,
                                                                 uint32_t *__restrict__ cnt) {
    __shared__ uint32_t s_n[kTagBlock / 64];
    int ox, oy, oz;
    const uint64_t m = box_mask(act, M, W, bits, (int64_t)blockIdx.x * kTagBlock + threadIdx.x, n_codes, ox, oy, oz);
    uint32_t n = (uint32_t)__popcll(m);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) n += __shfl_xor(n, d);
    if ((threadIdx.x & 63) == 0) s_n[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int i = 0; i < kTagBlock / 64; ++i) a += s_n[i];
        cnt[blockIdx.x] = a;
    }
}

__global__ __launch_bounds__(kTagBlock) void morton_scatter_kernel(const uint32_t *__restrict__ cell_pkg,
                                                                   const uint64_t *__restrict__ act, int M, int W,
                                                                   int bits, int64_t n_codes,
                                                                   const uint32_t *__restrict__ off,
                                                                   uint32_t *__restrict__ work) {
    __shared__ uint32_t s_n[kTagBlock / 64];
    int ox, oy, oz;
    const uint64_t m = box_mask(act, M, W, bits, (int64_t)blockIdx.x * kTagBlock + threadIdx.x, n_codes, ox, oy, oz);
    // exclusive prefix of the boxes' counts over the workgroup (lane order is code order)
    const uint32_t n = (uint32_t)__popcll(m);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = n;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(inc, d);
        if (lane >= d) inc += v;
    }
    if (lane == 63) s_n[wv] = inc;
    __syncthreads();
    uint32_t pos = off[blockIdx.x] + inc - n;
    for (int i = 0; i < wv; ++i) pos += s_n[i];
    if (!m) return;
    // the box in Morton order: code t has lx = t0 + 2 t3, ly = t1 + 2 t4, lz = t2 + 2 t5
    for (int t = 0; t < 64; ++t) {
        const int lx = (t & 1) | ((t >> 2) & 2), ly = ((t >> 1) & 1) | ((t >> 3) & 2), lz = ((t >> 2) & 1) | ((t >> 4) & 2);
        if ((m >> (lx + 4 * ly + 16 * lz)) & 1ull)
            work[pos++] = cell_pkg[(ox + lx) + (int64_t)M * ((oy + ly) + (int64_t)M * (oz + lz))];
    }
}

__global__ __launch_bounds__(256) void worklist_pos_kernel(const uint32_t *__restrict__ work, int64_t P,
                                                           uint32_t *__restrict__ wpos) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < P) wpos[work[e]] = (uint32_t)e;
}

// Face rows in worklist order, three times: wface holds the six face
// neighbours' package ids and the package's own id; sface marks a neighbour
// in the same group of kGroup entries by its slot in the group (flagged with
// kLocal); mface gives the neighbours' rows in the worklist-ordered copy of a
// field (row 2 + e holds the package at worklist position e, rows 0 and 1 the
// far fields), then the own id.  Eight lanes per entry (one per row slot),
// each taking kFacePkgs consecutive entries whose loads are issued together.
constexpr int kFacePkgs = 4;

__global__ __launch_bounds__(256) void sweep_face_kernel(const uint32_t *__restrict__ work,
                                                         const uint32_t *__restrict__ face,
                                                         const uint32_t *__restrict__ wpos, int64_t P,
                                                         uint32_t *__restrict__ wface, uint32_t *__restrict__ sface,
                                                         uint32_t *__restrict__ mface) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int f = (int)(t & 7);
    const int64_t e0 = (t >> 3) * kFacePkgs;
    if (e0 >= P) return;
    uint32_t p[kFacePkgs], n[kFacePkgs], en[kFacePkgs];
#pragma unroll
    for (int g = 0; g < kFacePkgs; ++g) p[g] = work[e0 + g < P ? e0 + g : P - 1];
#pragma unroll
    for (int g = 0; g < kFacePkgs; ++g) n[g] = f < 6 ? face[(int64_t)p[g] * 8 + f] : 0u;
#pragma unroll
    for (int g = 0; g < kFacePkgs; ++g) en[g] = wpos[n[g]];   // n < 2: a far-field row's entry, not used
#pragma unroll
    for (int g = 0; g < kFacePkgs; ++g) {
        const int64_t e = e0 + g;
        if (e >= P) break;
        uint32_t v, w, m;
        if (f < 6) {
            v = w = n[g];
            m = n[g] < 2u ? n[g] : 2u + en[g];
            if (n[g] >= 2u && (int64_t)en[g] / sgrid::kGroup == e / sgrid::kGroup)
                v = sgrid::kLocal | (en[g] % sgrid::kGroup);
        } else {
            v = w = m = f == 6 ? p[g] : 0u;
        }
        wface[e * 8 + f] = w;
        sface[e * 8 + f] = v;
        mface[e * 8 + f] = m;
    }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void far_rows_kernel(uint32_t *__restrict__ pkg_cell, uint8_t *__restrict__ pkg_type) {
    if (threadIdx.x < 2) {
        pkg_cell[threadIdx.x] = sgrid::kNoCell;
        pkg_type[threadIdx.x] = 0;
    }
}

// One lane per slot for each of kNbrPkgs packages.
constexpr int kNbrPkgs = 4;   // consecutive packages per 27-lane group of nbr_kernel

__global__ __launch_bounds__(256) void nbr_kernel(const uint32_t *__restrict__ cell_pkg,
                                                  const uint32_t *__restrict__ pkg_cell, int M,
                                                  int64_t n_total, uint32_t *__restrict__ nbr,
                                                  uint32_t *__restrict__ face) {
    // nine groups of 27 lanes per workgroup (lanes 243.. idle), each group
    // kNbrPkgs consecutive packages, lane s their slot s: the packages' cells,
    // then their neighbours' map entries, are requested together.  32-bit
    // index arithmetic, divisions by constants
    const int tl = (int)threadIdx.x;
    if (tl >= 9 * 27) return;
    const int64_t p0 = ((int64_t)blockIdx.x * 9 + tl / 27) * kNbrPkgs;
    if (p0 >= n_total) return;
    const int s = tl % 27;
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    uint32_t c[kNbrPkgs];
#pragma unroll
    for (int g = 0; g < kNbrPkgs; ++g) {
        const int64_t p = p0 + g;
        c[g] = (p >= 2 && p < n_total) ? pkg_cell[p] : 0u;
    }
    uint32_t v[kNbrPkgs];
#pragma unroll
    for (int g = 0; g < kNbrPkgs; ++g) {
        const int64_t p = p0 + g;
        const uint32_t um = (uint32_t)M;
        const uint32_t cyz = c[g] / um;
        const int x = (int)(c[g] - cyz * um) + dx;
        const int y = (int)(cyz % um) + dy;
        const int z = (int)(cyz / um) + dz;
        const bool out = x < 0 || y < 0 || z < 0 || x >= M || y >= M || z >= M;
        const uint32_t m = cell_pkg[out ? 0 : x + (int64_t)M * y + (int64_t)M * M * z];   // in bounds
        v[g] = p < 2 ? (uint32_t)p : (out ? sgrid::kFarPos : m);
    }
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
#pragma unroll
    for (int g = 0; g < kNbrPkgs; ++g) {
        const int64_t p = p0 + g;
        if (p >= n_total) break;
        nbr[p * 27 + s] = v[g];
        if (f >= 0) face[p * 8 + f] = v[g];
        if (s == 13) {
            face[p * 8 + 6] = v[g];
            face[p * 8 + 7] = v[g];
        }
    }
}

// Multi-resolution layers (Sec. 7, Sec. 7.1 step 1): the layer of doubled
// resolution evaluates distances only in the cells its parent layer's core
// cells cover.  core_slot[id] = position of core package `id` in the parent's
// core list (the rows of the caller's child distances).
__global__ __launch_bounds__(256) void core_slot_kernel(const uint32_t *__restrict__ core_list, int64_t n_core,
                                                        uint32_t *__restrict__ core_slot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_core) core_slot[core_list[i]] = (uint32_t)i;
}

// Core and sign bits of the refined layer, one wavefront per 64-cell word as
// in bits_kernel.  A fine cell under a core parent takes its own distance
// (child b = bx + 2 by + 4 bz of the parent's row); any other cell takes the
// parent's sign from the parent layer's rank map and is not core (the parent
// is not core, so its distance is at least the parent cell size, twice the
// fine one).
__global__ __launch_bounds__(256) void refine_bits_kernel(const uint4 *__restrict__ rank_map, int W32c,
                                                          const uint8_t *__restrict__ pkg_type,
                                                          const uint32_t *__restrict__ core_slot,
                                                          const float *__restrict__ child_d, int Mc, int W,
                                                          int64_t n_words, double lc, uint64_t *__restrict__ core,
                                                          uint64_t *__restrict__ neg) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_words) return;   // whole wavefronts
    const int lane = threadIdx.x & 63;
    const int Mf = 2 * Mc;
    const int64_t r = quot(w, W);
    const int x = (int)(w - r * W) * 64 + lane;
    const int64_t rz = quot(r, Mf);
    const int y = (int)(r - rz * Mf), z = (int)rz;
    bool is_core = false, is_neg = false;
    if (x < Mf) {
        const int px = x >> 1, py = y >> 1, pz = z >> 1;
        const uint4 e = rank_map[((int64_t)py + (int64_t)Mc * pz) * W32c + (px >> 5)];
        const uint32_t bit = 1u << (px & 31);
        is_neg = (e.y & bit) != 0u;
        if (e.x & bit) {
            const uint32_t id = 2u + e.z + (uint32_t)__popc(e.x & (bit - 1u));
            if (pkg_type[id] == 1) {
                const int b = (x & 1) + 2 * (y & 1) + 4 * (z & 1);
                const float v = child_d[(int64_t)core_slot[id] * 8 + b];
                is_core = fabs((double)v) < lc;
                is_neg = v < 0.0f;
            }
        }
    }
    const uint64_t bc = __ballot(is_core);
    const uint64_t bn = __ballot(is_neg);
    if (lane == 0) {
        core[w] = bc;
        neg[w] = bn;
    }
}

void free_grid(sgrid_grid *g) {
    if (!g) return;
    void *ptrs[] = {g->cell_pkg, g->pkg_cell, g->pkg_type, g->nbr,  g->face, g->core_list,
                    g->workspace, g->rank_map, g->work, g->sface, g->wface,     g->wpos,
                    g->mface};
    for (void *p : ptrs) sgrid::dev_free(p);
    delete g;
}

// Pinned host word for the one readback of a build (per thread).
uint64_t *pinned_totals() {
    static thread_local uint64_t *buf = nullptr;
    if (!buf && hipHostMalloc((void **)&buf, 2 * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        buf = nullptr;
    }
    return buf;
}

}  // namespace

#define SG_ALLOC(ptr, bytes, what)                                                  \
    do {                                                                            \
        sgrid_status _s = sgrid::dev_alloc((void **)&(ptr), (size_t)(bytes), what); \
        if (_s != SGRID_OK) { free_grid(g); return _s; }                            \
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

namespace {

// A new grid of M^3 cells at spacing h with its build workspace: three
// bitmaps (core, negative sign, activated), the per-group counts, the scan's
// block sums and the totals.
struct BuildWs {
    int64_t W, n_words, n_groups;
    uint64_t *core_bits, *neg_bits, *act_bits, *totals;
    uint32_t *ca, *cc, *part;
};

sgrid_status new_grid(int64_t M, double h, sgrid_grid **out, BuildWs &ws) {
    const int64_t n_cells = M * M * M;
    if (n_cells + 2 > (int64_t)0xFFFFFFFFll || (n_cells + 2) * 64 > ((int64_t)1 << 40)) {
        sgrid::set_error("n_coarse = %lld gives %lld coarse cells, beyond the 32-bit package ids",
                         (long long)M, (long long)n_cells);
        return SGRID_E_CAPACITY;
    }
    sgrid_grid *g = new sgrid_grid();
    g->M = (int32_t)M;
    g->h = h;
    SG_HIP_OR_FREE(hipGetDevice(&g->device));
    ws.W = (M + 63) / 64;
    ws.n_words = M * M * ws.W;
    ws.n_groups = (ws.n_words + 15) / 16;
    const int64_t n_sblocks = (ws.n_groups + kScanBlock - 1) / kScanBlock;
    const size_t ws_bits = ((size_t)ws.n_words * 8 + 255) / 256 * 256;
    const size_t ws_counts = ((size_t)ws.n_groups * 4 + 255) / 256 * 256;
    const size_t ws_part = ((size_t)n_sblocks * 8 + 255) / 256 * 256;
    SG_ALLOC(g->workspace, 3 * ws_bits + 2 * ws_counts + ws_part + 256, "build workspace");
    ws.core_bits = (uint64_t *)g->workspace;
    ws.neg_bits = (uint64_t *)((uint8_t *)ws.core_bits + ws_bits);
    ws.act_bits = (uint64_t *)((uint8_t *)ws.neg_bits + ws_bits);
    ws.ca = (uint32_t *)((uint8_t *)ws.act_bits + ws_bits);
    ws.cc = (uint32_t *)((uint8_t *)ws.ca + ws_counts);
    ws.part = (uint32_t *)((uint8_t *)ws.cc + ws_counts);
    ws.totals = (uint64_t *)((uint8_t *)ws.part + ws_part);
    SG_ALLOC(g->cell_pkg, n_cells * 4, "cell_pkg");
    *out = g;
    return SGRID_OK;
}

// Everything after the core and sign bitmaps: dilation, numbering (one host
// synchronisation learns P), tables, neighbours, the Morton worklist and the
// worklist face rows.  Frees the grid on failure.
sgrid_status finish_grid(sgrid_grid *g, const BuildWs &ws, hipStream_t st) {
    const int64_t M = g->M, W = ws.W, n_words = ws.n_words, n_groups = ws.n_groups;
    uint64_t *core_bits = ws.core_bits, *neg_bits = ws.neg_bits, *act_bits = ws.act_bits, *totals = ws.totals;
    uint32_t *ca = ws.ca, *cc = ws.cc, *part = ws.part;
    hipLaunchKernelGGL(dilate_kernel, dim3((unsigned)((n_words + 255) / 256)), dim3(256), 0, st, core_bits, (int)M,
                       (int)W, n_words, act_bits, ca, cc);
    SG_HIP_OR_FREE(hipGetLastError());
    scan_pair(ca, cc, n_groups, part, totals, st);
    SG_HIP_OR_FREE(hipGetLastError());
    uint64_t *host = pinned_totals();
    uint64_t local[2] = {0, 0};
    uint64_t *dst = host ? host : local;
    SG_HIP_OR_FREE(hipMemcpyAsync(dst, totals, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    SG_HIP_OR_FREE(hipStreamSynchronize(st));
    g->P = (int64_t)dst[0];
    g->n_core = (int64_t)dst[1];
    const int64_t nt = g->total();
    SG_ALLOC(g->pkg_cell, nt * 4, "pkg_cell");
    SG_ALLOC(g->pkg_type, nt, "pkg_type");
    SG_ALLOC(g->nbr, nt * 27 * 4, "pkg_nbr");
    SG_ALLOC(g->face, nt * 8 * 4, "face table");
    SG_ALLOC(g->core_list, (g->n_core > 0 ? g->n_core : 1) * 4, "core_list");
    hipLaunchKernelGGL(far_rows_kernel, dim3(1), dim3(64), 0, st, g->pkg_cell, g->pkg_type);
    SG_HIP_OR_FREE(hipGetLastError());
    g->W32 = (int32_t)((M + 31) / 32);
    SG_ALLOC(g->rank_map, M * M * g->W32 * 16, "rank map");
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((n_groups + 3) / 4)), dim3(256), 0, st, act_bits, core_bits,
                       neg_bits,
                       (int)M, (int)W, n_words, ca, cc, g->cell_pkg, g->pkg_cell, g->pkg_type, g->core_list,
                       g->rank_map, g->W32);
    SG_HIP_OR_FREE(hipGetLastError());
    hipLaunchKernelGGL(nbr_kernel, dim3((unsigned)((nt + 9 * kNbrPkgs - 1) / (9 * kNbrPkgs))), dim3(256), 0, st,
                       g->cell_pkg, g->pkg_cell, (int)M, nt, g->nbr, g->face);
    SG_HIP_OR_FREE(hipGetLastError());
    // Morton-order sweep worklist: count activated codes per block of
    // kCodesPerBlock codes, scan, scatter (the counts and the scan's block sums
    // live behind the worklist)
    {
        int bits = 0;
        while ((1ll << bits) < M) ++bits;
        const int64_t n_codes = (int64_t)1 << (3 * bits);
        const int64_t nbm = (n_codes + kCodesPerBlock - 1) / kCodesPerBlock;
        const int64_t nbs = (nbm + kScanBlock - 1) / kScanBlock;
        SG_ALLOC(g->work, ((g->P > 0 ? g->P : 1) + 2 * nbm + 2 * nbs + 64) * 4, "sweep worklist");
        uint32_t *mc = g->work + (g->P > 0 ? g->P : 1);
        uint32_t *mz = mc + nbm;
        uint32_t *mpart = mz + nbm;
        hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((nbm + 255) / 256)), dim3(256), 0, st, mz, nbm);
        SG_HIP_OR_FREE(hipGetLastError());
        hipLaunchKernelGGL(morton_count_kernel, dim3((unsigned)nbm), dim3(kTagBlock), 0, st, act_bits, (int)M, (int)W,
                           bits, n_codes, mc);
        SG_HIP_OR_FREE(hipGetLastError());
        scan_pair(mc, mz, nbm, mpart, totals, st);
        SG_HIP_OR_FREE(hipGetLastError());
        hipLaunchKernelGGL(morton_scatter_kernel, dim3((unsigned)nbm), dim3(kTagBlock), 0, st, g->cell_pkg, act_bits,
                           (int)M, (int)W, bits, n_codes, mc, g->work);
        SG_HIP_OR_FREE(hipGetLastError());
    }
    // group-relative face rows of the sweep order, through the position of
    // every package in the worklist (kept with the handle)
    {
        SG_ALLOC(g->sface, (g->P > 0 ? g->P : 1) * 32, "sweep face table");
        SG_ALLOC(g->wface, (g->P > 0 ? g->P : 1) * 32, "worklist face table");
        uint32_t *wpos = nullptr;
        SG_ALLOC(wpos, nt * 4, "worklist positions");
        if (g->P > 0) {
            hipLaunchKernelGGL(worklist_pos_kernel, dim3((unsigned)((g->P + 255) / 256)), dim3(256), 0, st, g->work,
                               g->P, wpos);
            SG_HIP_OR_FREE(hipGetLastError());
        }
        g->wpos = wpos;
        SG_ALLOC(g->mface, (g->P > 0 ? g->P : 1) * 32, "worklist-ordered face table");
        if (g->P > 0) {
            const int64_t groups = (g->P + kFacePkgs - 1) / kFacePkgs;
            hipLaunchKernelGGL(sweep_face_kernel, dim3((unsigned)((groups * 8 + 255) / 256)), dim3(256), 0, st,
                               g->work, g->face, wpos, g->P, g->wface, g->sface, g->mface);
            SG_HIP_OR_FREE(hipGetLastError());
        }
    }
    return SGRID_OK;
}

}  // namespace

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
    hipStream_t st = sg_stream(stream);
    sgrid_grid *g = nullptr;
    BuildWs ws;
    sgrid_status s = new_grid(M, desc->h, &g, ws);
    if (s != SGRID_OK) return s;
    const double lc = 4.0 * desc->h;
    hipLaunchKernelGGL(bits_kernel, dim3((unsigned)((ws.n_words + 4 * kBitsWords - 1) / (4 * kBitsWords))), dim3(256), 0,
                       st, coarse_sdf, (int)M,
                       (int)ws.W, ws.n_words, lc, ws.core_bits, ws.neg_bits);
    SG_HIP_OR_FREE(hipGetLastError());
    s = finish_grid(g, ws, st);
    if (s != SGRID_OK) return s;
    *out = g;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_build_packages_refined(const sgrid_grid *coarse, const float *child_sdf, void *stream,
                                                     sgrid_grid **out) {
    sgrid::clear_error();
    SG_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    SG_REQUIRE(coarse != nullptr, "coarse grid is NULL");
    SG_REQUIRE(child_sdf != nullptr || coarse->n_core == 0, "child_sdf is NULL");
    SG_REQUIRE(child_sdf == nullptr || sg_aligned(child_sdf, 4), "child_sdf is not 4-byte aligned");
    SG_REQUIRE(coarse->M <= (1 << 29), "the coarse grid is too large to refine");
    const int64_t M = 2 * (int64_t)coarse->M;
    hipStream_t st = sg_stream(stream);
    sgrid_grid *g = nullptr;
    BuildWs ws;
    sgrid_status s = new_grid(M, 0.5 * coarse->h, &g, ws);
    if (s != SGRID_OK) return s;
    // the parent's core slots live in the new cell_pkg until it is written
    static_assert(sizeof(uint32_t) == 4, "");
    uint32_t *core_slot = g->cell_pkg;   // M^3 >= 8 (P_parent + 2) entries
    if (coarse->n_core > 0) {
        hipLaunchKernelGGL(core_slot_kernel, dim3((unsigned)((coarse->n_core + 255) / 256)), dim3(256), 0, st,
                           coarse->core_list, coarse->n_core, core_slot);
        SG_HIP_OR_FREE(hipGetLastError());
    }
    const double lc = 4.0 * g->h;
    hipLaunchKernelGGL(refine_bits_kernel, dim3((unsigned)((ws.n_words + 3) / 4)), dim3(256), 0, st, coarse->rank_map,
                       coarse->W32, coarse->pkg_type, core_slot, child_sdf, coarse->M, (int)ws.W, ws.n_words, lc,
                       ws.core_bits, ws.neg_bits);
    SG_HIP_OR_FREE(hipGetLastError());
    s = finish_grid(g, ws, st);
    if (s != SGRID_OK) return s;
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
    out->sweep_order = g->work;
    out->rank_map = (const uint32_t *)g->rank_map;
    out->rank_row = g->W32;
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

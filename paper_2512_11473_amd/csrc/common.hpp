// Internal helpers shared by the sgrid HIP sources: status reporting, the
// grid handle, launch checks and small device utilities for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string>

#include "../../include/sgrid.h"

namespace sgrid {

void set_error(const char *fmt, ...);
void clear_error();

// Device memory of the library (tables, workspaces) comes from a small
// per-process caching allocator: freed blocks are kept and handed out again
// to requests of the same rounded size, so repeated builds make no driver
// allocation calls.  dev_free must only be called once no queued work uses
// the block.
sgrid_status dev_alloc(void **p, size_t bytes, const char *what);
void dev_free(void *p);

// Compute units of the current device (cached).
int cu_count();

// *p = 0 on `st` by a one-lane kernel (no memset node in a captured graph).
sgrid_status launch_zero_u32(uint32_t *p, hipStream_t st);

// Far-field package ids and the far-field constant in units of h.
constexpr uint32_t kFarNeg = 0u;
constexpr uint32_t kFarPos = 1u;
constexpr uint32_t kNoCell = 0xFFFFFFFFu;
constexpr double kFarFieldInH = 16.0;

// Sweep groups: 64 consecutive worklist entries (Morton order) are swept by one
// workgroup, which shares their rows through LDS.
constexpr int kGroup = 64;
constexpr uint32_t kLocal = 0x80000000u;

// Face slots of the 27-entry neighbour table, in the order the sweeps use:
// -x, +x, -y, +y, -z, +z.
constexpr int kFaceSlot[6] = {12, 14, 10, 16, 4, 22};

}  // namespace sgrid

struct sgrid_grid {
    int32_t M = 0;
    double h = 0.0;
    int64_t P = 0;        // activated packages
    int64_t n_core = 0;
    int device = 0;
    uint32_t *cell_pkg = nullptr;   // [M^3]
    uint32_t *pkg_cell = nullptr;   // [P+2]
    uint8_t *pkg_type = nullptr;    // [P+2]
    uint32_t *nbr = nullptr;        // [P+2][27]
    uint32_t *face = nullptr;       // [P+2][8]: the six face slots of nbr, then two pads
    uint32_t *core_list = nullptr;  // [n_core]
    uint32_t *work = nullptr;       // [P]: activated package ids in Morton order of their cells
    uint32_t *wface = nullptr;      // [P][8]: per worklist position: six face neighbours, own id, pad
    uint32_t *sface = nullptr;      // [P][8]: per worklist position: six face neighbours (package id, or
                                    // group slot | kLocal when in the same 64-package group), own id, pad
    uint32_t *wpos = nullptr;       // [P+2]: position of each package in the worklist
    uint32_t *mface = nullptr;      // [P][8]: per worklist position e: the six face neighbours' rows in the
                                    // worklist-ordered field copy (2 + position, far fields 0 and 1), own id, pad
    void *workspace = nullptr;      // build scratch, kept until destroy
    // compact form of cell_pkg for position lookups: per 32 cells of a row,
    // {activated bits, negative-sign bits, activated cells before them, 0}
    uint4 *rank_map = nullptr;      // [M * M * W32]
    int32_t W32 = 0;                // entries per row: ceil(M / 32)
    int64_t total() const { return P + 2; }
};

#define SG_CHECK_HIP(expr)                                                            \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) {                                                       \
            sgrid::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),   \
                             __FILE__, __LINE__);                                     \
            return SGRID_E_HIP;                                                       \
        }                                                                             \
    } while (0)

#define SG_CHECK_LAUNCH(name)                                                         \
    do {                                                                              \
        hipError_t _e = hipGetLastError();                                            \
        if (_e != hipSuccess) {                                                       \
            sgrid::set_error("launch of %s failed: %s", name, hipGetErrorString(_e)); \
            return SGRID_E_HIP;                                                       \
        }                                                                             \
    } while (0)

#define SG_REQUIRE(cond, ...)                              \
    do {                                                   \
        if (!(cond)) {                                     \
            sgrid::set_error(__VA_ARGS__);                 \
            return SGRID_E_INVALID;                        \
        }                                                  \
    } while (0)

static inline bool sg_aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static inline hipStream_t sg_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Grids of more than 2^31 - 1 blocks are not launched; callers loop or stride.
constexpr int64_t kMaxGrid = 0x7FFFFFFF;

// ---------------------------------------------------------------------------
// Device utilities
// ---------------------------------------------------------------------------

// Cross-lane move inside 16-lane rows (DPP).  CTRL is a row_shl / row_shr
// control: row_shl:n = 0x100 + n (lane l reads lane l + n of its row),
// row_shr:n = 0x110 + n (lane l reads lane l - n).  row_move: lanes whose
// source lies outside their 16-lane row read 0 and must not use the result
// (callers select a halo value for them).  row_move_keep: lanes of the banks
// (groups of four lanes of a row) left out of BANKS keep `keep` instead, which
// takes a halo value in without a select.  Both must run in every lane of the
// row: a lane outside the active mask supplies 0 to its neighbours, so a move
// written inside a lane-dependent branch (an arm of ?: included) reads wrong
// values.
constexpr int kRowShl1 = 0x101, kRowShl4 = 0x104, kRowShr1 = 0x111, kRowShr4 = 0x114;

template <int CTRL>
__device__ __forceinline__ float row_move(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double row_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xFFFFFFFFll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL, int BANKS>
__device__ __forceinline__ float row_move_keep(float v, float keep) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(keep), __float_as_int(v), CTRL, 0xF, BANKS, false));
}

template <int CTRL, int BANKS>
__device__ __forceinline__ double row_move_keep(double v, double keep) {
    const long long b = __double_as_longlong(v), o = __double_as_longlong(keep);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xFFFFFFFFll), (int)(b & 0xFFFFFFFFll), CTRL, 0xF, BANKS, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xF, BANKS, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Point order of the packed (phi, g) probe field: the 64 points of a package
// in 2 x 2 x 2 blocks, so the eight corners of a trilinear cell that lies
// inside one block share one 128-byte line (FP32).
__host__ __device__ __forceinline__ int blocked_index(int i, int j, int k) {
    return 8 * ((i >> 1) + 2 * (j >> 1) + 4 * (k >> 1)) + ((i & 1) + 2 * (j & 1) + 4 * (k & 1));
}

// XCD-aware block order: the hardware deals consecutive workgroups round-robin
// to the 8 XCDs; remapping gives each XCD one contiguous range of block ids,
// so packages that are neighbours in id order share that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t per = (nb + 7) / 8;
    const int64_t x = b % 8, r = b / 8;
    const int64_t full = nb % 8 == 0 ? 8 : nb % 8;   // XCDs that receive `per` blocks
    // XCDs 0..full-1 own ranges of length per, the rest ranges of length per - 1
    return x < full ? x * per + r : full * per + (x - full) * (per - 1) + r;
}

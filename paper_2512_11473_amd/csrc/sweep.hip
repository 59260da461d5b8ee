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
#include <atomic>

#include "common.hpp"
#include "fraction.hpp"
#include "upwind.hpp"

using sgrid::kGroup;
using sgrid::kLocal;
using sgrid::upwind_update;

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

// The same row written with the streaming (non-temporal) hint: used by the
// sweeps when the two field buffers do not fit in the last-level cache, where
// the freshly written rows would only push out halo lines that the running
// sweep still reads.  When the buffers fit, the hint would keep the written
// rows out of the cache that the next sweep reads them from.
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef double f64x2v __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ void store_row_nt(T *__restrict__ p, const Row<T> &r);
template <>
__device__ __forceinline__ void store_row_nt<float>(float *__restrict__ p, const Row<float> &r) {
    const f32x4v v = {r.v[0], r.v[1], r.v[2], r.v[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<f32x4v *>(p));
}
template <>
__device__ __forceinline__ void store_row_nt<double>(double *__restrict__ p, const Row<double> &r) {
    const f64x2v a = {r.v[0], r.v[1]}, b = {r.v[2], r.v[3]};
    __builtin_nontemporal_store(a, reinterpret_cast<f64x2v *>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<f64x2v *>(p) + 1);
}
template <typename T>
__device__ __forceinline__ void store_row(T *__restrict__ p, const Row<T> &r, bool nt) {
    if (nt)
        store_row_nt(p, r);
    else
        store_row(p, r);
}

// A package row and its stencil neighbours.
template <typename T>
struct Stencil {
    Row<T> c, ym, yp, zm, zp;
    T xm, xp;
};

// Loads of one lane: its row, the x end values of the -x / +x packages, and
// (boundary lanes only) one y-halo row and one z-halo row.
template <typename T>
struct Loads {
    Row<T> c, yh, zh;
    T xm, xp;
};

__device__ __forceinline__ void load_face(const uint32_t *__restrict__ face, int64_t p, uint4 &f0, uint2 &f1) {
    f0 = *reinterpret_cast<const uint4 *>(face + p * 8);
    f1 = *reinterpret_cast<const uint2 *>(face + p * 8 + 4);
}

// Every lane issues all five loads.  A lane with no y (z) halo row loads the
// halo row of its neighbour lane on the same side (j = 1 that of j = 0, j = 2
// that of j = 3, and likewise for k), so each halo load touches only the
// neighbour packages' lines; the interior lanes' values are not used.  Loads
// under a per-lane condition would become branches, and the compiler then
// waits for every earlier load before the branch's own, adding a memory round
// trip.
template <typename T>
__device__ __forceinline__ void issue_halos(const T *__restrict__ src, int64_t p, int r, const uint4 &f0,
                                            const uint2 &f1, Loads<T> &l) {
    const int j = r & 3, k = r >> 2;
    l.xm = src[(int64_t)f0.x * 64 + r * 4 + 3];
    l.xp = src[(int64_t)f0.y * 64 + r * 4];
    const int64_t fy = j < 2 ? (int64_t)f0.z : (int64_t)f0.w;
    const int ry = j < 2 ? 3 + 4 * k : 4 * k;
    l.yh = load_row(src + fy * 64 + ry * 4);
    const int64_t fz = k < 2 ? (int64_t)f1.x : (int64_t)f1.y;
    const int rz = k < 2 ? j + 12 : j;
    l.zh = load_row(src + fz * 64 + rz * 4);
}

template <typename T>
__device__ __forceinline__ void issue_data(const T *__restrict__ src, int64_t p, int r, const uint4 &f0,
                                           const uint2 &f1, Loads<T> &l) {
    l.c = load_row(src + p * 64 + r * 4);
    issue_halos(src, p, r, f0, f1, l);
}

template <typename T>
__device__ __forceinline__ void issue_loads(const T *__restrict__ src, const uint32_t *__restrict__ face, int64_t p,
                                            int r, Loads<T> &l) {
    uint4 f0;
    uint2 f1;
    load_face(face, p, f0, f1);
    issue_data(src, p, r, f0, f1, l);
}

// Interior y / z neighbours through DPP row shifts (the 16 lanes of a package
// form one DPP row and execute these together).
template <typename T>
__device__ __forceinline__ Stencil<T> assemble(int r, const Loads<T> &l) {
    const int j = r & 3, k = r >> 2;
    Stencil<T> s;
    s.c = l.c;
    s.xm = l.xm;
    s.xp = l.xp;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const T v = l.c.v[i];
        const T a = row_move<kRowShr1>(v);   // lane - 1: (j - 1, k)
        const T b = row_move<kRowShl1>(v);   // lane + 1: (j + 1, k)
        s.ym.v[i] = j == 0 ? l.yh.v[i] : a;
        s.yp.v[i] = j == 3 ? l.yh.v[i] : b;
        // lane -+ 4: (j, k -+ 1); the k = 0 (k = 3) lanes are bank 0 (bank 3)
        // of the row and keep their z halo value
        s.zm.v[i] = row_move_keep<kRowShr4, 0xE>(v, l.zh.v[i]);
        s.zp.v[i] = row_move_keep<kRowShl4, 0x7>(v, l.zh.v[i]);
    }
    return s;
}

template <typename T>
__device__ __forceinline__ Row<T> reinit_row(const Stencil<T> &s, T h2, T inv_h, T dt) {
    Row<T> o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const T xm = i > 0 ? s.c.v[i - 1] : s.xm;
        const T xp = i < 3 ? s.c.v[i + 1] : s.xp;
        o.v[i] = upwind_update(s.c.v[i], xm, xp, s.ym.v[i], s.yp.v[i], s.zm.v[i], s.zp.v[i], h2, inv_h, dt);
    }
    return o;
}

// Reinitialisation sweep over the packages [first, end) (all of them: [2,
// 2 + P)), DPP exchange variant.  A wavefront handles G consecutive sets of
// four packages and issues all their loads before computing any of them.
template <typename T, int G>
__global__ __launch_bounds__(256) void reinit_dpp_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                         const uint32_t *__restrict__ face, int64_t first,
                                                         int64_t end, int64_t n_blocks, T h2, T inv_h, T dt, bool nt) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t p0 = first + (b * 4 + (threadIdx.x >> 6)) * (4 * G) + (lane >> 4);
    Loads<T> l[G];
#pragma unroll
    for (int g = 0; g < G; ++g)
        if (p0 + 4 * g < end) issue_loads(src, face, p0 + 4 * g, r, l[g]);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const Stencil<T> s = assemble(r, l[g]);
        if (p0 + 4 * g < end) store_row(dst + (p0 + 4 * g) * 64 + r * 4, reinit_row(s, h2, inv_h, dt), nt);
    }
}

// Worklist variant: the DPP sweep over the packages in Morton order of their
// cells (the build's worklist), so the sixteen packages of a workgroup are
// spatial neighbours and most halo rows come from lines the workgroup itself
// brings into the caches.  The face rows are read in worklist order (wface:
// six neighbours and the package's own id), one coalesced 32-byte row per
// package.  G sets of four packages per wavefront.
template <typename T, int G>
__global__ __launch_bounds__(256) void reinit_work_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                          const uint32_t *__restrict__ wface, int64_t P,
                                                          int64_t n_blocks, T h2, T inv_h, T dt, bool nt) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t e0 = (b * 4 + (threadIdx.x >> 6)) * (4 * G) + (lane >> 4);
    Loads<T> l[G];
    int64_t p[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t e = e0 + 4 * g;
        p[g] = -1;
        if (e < P) {
            const uint4 f0 = *reinterpret_cast<const uint4 *>(wface + e * 8);
            const uint4 f1 = *reinterpret_cast<const uint4 *>(wface + e * 8 + 4);
            p[g] = (int64_t)f1.z;
            issue_data(src, p[g], r, f0, make_uint2(f1.x, f1.y), l[g]);
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const Stencil<T> s = assemble(r, l[g]);
        if (p[g] >= 0) store_row(dst + p[g] * 64 + r * 4, reinit_row(s, h2, inv_h, dt), nt);
    }
}

// Worklist-ordered storage variant (7).  During the iterations the field is
// held in a copy ordered by the worklist: row 2 + e is the package at
// worklist position e, rows 0 and 1 the far fields, and the face rows of that
// copy (mface) give each position's neighbours as rows of the copy.  A sweep
// then streams contiguous rows in Morton order, with its halos in Morton-near
// rows, and a wavefront's own rows no longer wait for its face row.  The
// first sweep of a call reads the field in package-id order (wface) and
// writes the copy (MODE 0); the following ones go copy to copy (MODE 1); the
// last writes package-id order again (MODE 2).  The values are those of every
// other variant.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void reinit_morton_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                            const uint32_t *__restrict__ wface,
                                                            const uint32_t *__restrict__ mface, int64_t P,
                                                            int64_t n_blocks, T h2, T inv_h, T dt, bool nt) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t e = (b * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
    if (e >= P) return;   // whole 16-lane rows (one package each) leave together
    Loads<T> l;
    int64_t out_row;
    if (MODE == 0) {
        const uint4 f0 = *reinterpret_cast<const uint4 *>(wface + e * 8);
        const uint4 f1 = *reinterpret_cast<const uint4 *>(wface + e * 8 + 4);
        issue_data(src, (int64_t)f1.z, r, f0, make_uint2(f1.x, f1.y), l);
        out_row = 2 + e;
    } else {
        l.c = load_row(src + (2 + e) * 64 + r * 4);
        const uint4 f0 = *reinterpret_cast<const uint4 *>(mface + e * 8);
        const uint4 f1 = *reinterpret_cast<const uint4 *>(mface + e * 8 + 4);
        issue_halos(src, 2 + e, r, f0, make_uint2(f1.x, f1.y), l);
        out_row = MODE == 1 ? 2 + e : (int64_t)f1.z;
    }
    const Stencil<T> st = assemble(r, l);
    store_row(dst + out_row * 64 + r * 4, reinit_row(st, h2, inv_h, dt), nt);
}

// Row-exchange variant: the y / z neighbour rows move through LDS instead of
// DPP, which takes the exchange off the VALU.  Every wavefront writes its own
// four packages' rows (and their y / z halo rows) into a 6 x 6 grid of rows
// per package and reads the four neighbour rows back; a wavefront only ever
// reads rows it wrote itself, and LDS operations of one wavefront complete in
// order, so no workgroup barrier is needed.
template <typename T, int G>
__global__ __launch_bounds__(256) void reinit_rows_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                          const uint32_t *__restrict__ face, int64_t P,
                                                          int64_t n_blocks, T h2, T inv_h, T dt, bool nt) {
    __shared__ Row<T> rows[16][36];   // [package slot in block][(z+1) * 6 + (y+1)]
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, j = r & 3, k = r >> 2;
    const int slot = threadIdx.x >> 4;
    Row<T> *R = rows[slot];
    const int64_t p0 = 2 + (b * 4 + (threadIdx.x >> 6)) * (4 * G) + (lane >> 4);
    Loads<T> l[G];
#pragma unroll
    for (int g = 0; g < G; ++g)
        if (p0 + 4 * g < P + 2) issue_loads(src, face, p0 + 4 * g, r, l[g]);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t p = p0 + 4 * g;
        R[(k + 1) * 6 + (j + 1)] = l[g].c;
        if (j == 0) R[(k + 1) * 6] = l[g].yh;
        if (j == 3) R[(k + 1) * 6 + 5] = l[g].yh;
        if (k == 0) R[j + 1] = l[g].zh;
        if (k == 3) R[30 + j + 1] = l[g].zh;
        __builtin_amdgcn_wave_barrier();
        Stencil<T> s;
        s.c = l[g].c;
        s.xm = l[g].xm;
        s.xp = l[g].xp;
        s.ym = R[(k + 1) * 6 + j];
        s.yp = R[(k + 1) * 6 + j + 2];
        s.zm = R[k * 6 + (j + 1)];
        s.zp = R[(k + 2) * 6 + (j + 1)];
        __builtin_amdgcn_wave_barrier();
        if (p < P + 2) store_row(dst + p * 64 + r * 4, reinit_row(s, h2, inv_h, dt), nt);
    }
}

// Shared-group variant: one workgroup of 1024 lanes sweeps a group of 64
// consecutive worklist entries (Morton order, so spatially compact).  Each
// package's rows go into LDS first; a halo row whose package belongs to the
// same group is read from LDS, the others from memory.  The group-relative face
// rows (sface) mark in-group neighbours with kLocal | slot.
template <typename T>
__device__ __forceinline__ T halo_value(const T *__restrict__ src, const T (*tile)[64], uint32_t f, int off) {
    return (f & kLocal) ? tile[f & (kGroup - 1)][off] : src[(int64_t)f * 64 + off];
}

template <typename T>
__device__ __forceinline__ Row<T> halo_row(const T *__restrict__ src, const T (*tile)[64], uint32_t f, int off) {
    if (f & kLocal) {
        const T *t = tile[f & (kGroup - 1)] + off;
        return Row<T>{{t[0], t[1], t[2], t[3]}};
    }
    return load_row(src + (int64_t)f * 64 + off);
}

template <typename T>
__global__ __launch_bounds__(1024) void reinit_share_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                            const uint32_t *__restrict__ work,
                                                            const uint32_t *__restrict__ sface, int64_t P,
                                                            int64_t n_blocks, T h2, T inv_h, T dt) {
    __shared__ T tile[kGroup][64];
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, j = r & 3, k = r >> 2;
    const int slot = threadIdx.x >> 4;
    const int64_t e = b * kGroup + slot;
    const bool live = e < P;
    uint4 f0 = make_uint4(0, 0, 0, 0);
    uint2 f1 = make_uint2(0, 0);
    int64_t p = 0;
    Row<T> c;
    if (live) {
        p = work[e];
        f0 = *reinterpret_cast<const uint4 *>(sface + e * 8);
        f1 = *reinterpret_cast<const uint2 *>(sface + e * 8 + 4);
        c = load_row(src + p * 64 + r * 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) tile[slot][r * 4 + i] = c.v[i];
    }
    __syncthreads();
    if (!live) return;
    Loads<T> l;
    l.c = c;
    l.xm = halo_value(src, tile, f0.x, r * 4 + 3);
    l.xp = halo_value(src, tile, f0.y, r * 4);
    if (j == 0 || j == 3) l.yh = halo_row(src, tile, j == 0 ? f0.z : f0.w, (j == 0 ? 3 + 4 * k : 4 * k) * 4);
    if (k == 0 || k == 3) l.zh = halo_row(src, tile, k == 0 ? f1.x : f1.y, (k == 0 ? j + 12 : j) * 4);
    const Stencil<T> s = assemble(r, l);
    store_row(dst + p * 64 + r * 4, reinit_row(s, h2, inv_h, dt));
}

// Persistent worklist variant: a fixed grid of `groups` workgroups per CU
// walks the Morton worklist in grid-stride rounds.  In each round the
// wavefronts cover one contiguous stretch of the worklist (each XCD a
// contiguous part of it), so halo rows come from lines the same round brings
// into the caches, as in the one-shot worklist variant; and every wavefront
// loads the face row of its next set while the current set's data loads are
// in flight, which takes the face-row -> data dependency off the critical
// path after a wavefront's first set.  The round loop is uniform over a
// wavefront (all 64 lanes run the DPP exchange together).  The last set's
// missing entries take the last entry again and store the same bytes to the
// same package as its own lanes: the store stays unconditional, because a
// conditional one lets the compiler sink the halo loads into the branch,
// behind the DPP exchange, adding a memory round trip.
template <typename T>
__global__ __launch_bounds__(256) void reinit_pipe_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                          const uint32_t *__restrict__ wface, int64_t P,
                                                          int64_t n_blocks, T h2, T inv_h, T dt, bool nt) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t n_sets = (P + 3) / 4;
    const int64_t stride = n_blocks * 4;
    int64_t s = b * 4 + (threadIdx.x >> 6);
    if (s >= n_sets) return;
    auto entry = [&](int64_t set) {
        const int64_t e = set * 4 + (lane >> 4);
        return e < P ? e : P - 1;
    };
    int64_t e = entry(s);
    uint4 f0 = *reinterpret_cast<const uint4 *>(wface + e * 8);
    uint4 f1 = *reinterpret_cast<const uint4 *>(wface + e * 8 + 4);
    for (; s < n_sets; s += stride) {
        const uint4 c0 = f0;
        const int64_t p = (int64_t)f1.z;
        const uint2 cz = make_uint2(f1.x, f1.y);
        // the next set's face row first, so that it is in flight for a whole set
        e = entry(s + stride < n_sets ? s + stride : s);
        f0 = *reinterpret_cast<const uint4 *>(wface + e * 8);
        f1 = *reinterpret_cast<const uint4 *>(wface + e * 8 + 4);
        Loads<T> l;
        issue_data(src, p, r, c0, cz, l);
        const Stencil<T> st = assemble(r, l);
        store_row(dst + p * 64 + r * 4, reinit_row(st, h2, inv_h, dt), nt);
    }
}

// Persistent linear variant: the grid-stride walk of variant 2 over the
// packages in id order, where a set's package ids are known without a table:
// each wavefront loads the next set's face row and own rows while the current
// set's halo rows are in flight, so a set costs one memory round trip.
template <typename T>
__global__ __launch_bounds__(256) void reinit_pipe_lin_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                              const uint32_t *__restrict__ face, int64_t P,
                                                              int64_t n_blocks, T h2, T inv_h, T dt) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t n_sets = (P + 3) / 4;
    const int64_t stride = n_blocks * 4;
    int64_t s = b * 4 + (threadIdx.x >> 6);
    if (s >= n_sets) return;
    auto pkg = [&](int64_t set) {
        const int64_t e = set * 4 + (lane >> 4);
        return 2 + (e < P ? e : P - 1);
    };
    int64_t p = pkg(s);
    uint4 f0;
    uint2 f1;
    load_face(face, p, f0, f1);
    Row<T> own = load_row(src + p * 64 + r * 4);
    for (; s < n_sets; s += stride) {
        const int64_t pc = p;
        const uint4 c0 = f0;
        const uint2 c1 = f1;
        Loads<T> l;
        l.c = own;
        p = pkg(s + stride < n_sets ? s + stride : s);
        load_face(face, p, f0, f1);
        own = load_row(src + p * 64 + r * 4);
        issue_halos(src, pc, r, c0, c1, l);
        const Stencil<T> st = assemble(r, l);
        store_row(dst + pc * 64 + r * 4, reinit_row(st, h2, inv_h, dt));
    }
}

// LDS-staged variant: the package rows and their face halo rows go into a
// 6 x 6 x 6 tile per package (interior 4^3 plus one-cell faces) in LDS, and
// each lane reads its stencil back from the tile.
template <typename T>
__global__ __launch_bounds__(256) void reinit_lds_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                         const uint32_t *__restrict__ face, int64_t P,
                                                         int64_t n_blocks, int groups, T h2, T inv_h, T dt) {
    __shared__ T tile[16][216];
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, j = r & 3, k = r >> 2;
    T *t = tile[threadIdx.x >> 4];
    auto at = [](int x, int y, int z) { return (x + 1) + 6 * ((y + 1) + 6 * (z + 1)); };
    const int64_t wave = b * 4 + (threadIdx.x >> 6);
    for (int gi = 0; gi < groups; ++gi) {
        const int64_t p = 2 + (wave * groups + gi) * 4 + (lane >> 4);
        const bool live = p < P + 2;
        if (live) {
            Loads<T> l;
            issue_loads(src, face, p, r, l);
#pragma unroll
            for (int i = 0; i < 4; ++i) t[at(i, j, k)] = l.c.v[i];
            t[at(-1, j, k)] = l.xm;
            t[at(4, j, k)] = l.xp;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (j == 0) t[at(i, -1, k)] = l.yh.v[i];
                if (j == 3) t[at(i, 4, k)] = l.yh.v[i];
                if (k == 0) t[at(i, j, -1)] = l.zh.v[i];
                if (k == 3) t[at(i, j, 4)] = l.zh.v[i];
            }
        }
        __syncthreads();
        if (live) {
            Row<T> o;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                o.v[i] = upwind_update(t[at(i, j, k)], t[at(i - 1, j, k)], t[at(i + 1, j, k)], t[at(i, j - 1, k)],
                                       t[at(i, j + 1, k)], t[at(i, j, k - 1)], t[at(i, j, k + 1)], h2, inv_h, dt);
            store_row(dst + p * 64 + r * 4, o);
        }
        __syncthreads();
    }
}

// Package of entry e of a stencil pass over all rows [0, P + 2): in id order
// (WORK = false) entry e is package e; in worklist order entries 0 and 1 are
// the far-field rows and entry e >= 2 is worklist position e - 2, whose face
// row (wface: six neighbours, own id) comes in the same 32-byte load.
template <bool WORK>
__device__ __forceinline__ int64_t stencil_package(int64_t e, const uint32_t *__restrict__ face,
                                                   const uint32_t *__restrict__ wface, uint4 &f0, uint2 &f1) {
    if (e < 2) return e;
    if (WORK) {
        const uint4 a = *reinterpret_cast<const uint4 *>(wface + (e - 2) * 8);
        const uint4 b = *reinterpret_cast<const uint4 *>(wface + (e - 2) * 8 + 4);
        f0 = a;
        f1 = make_uint2(b.x, b.y);
        return (int64_t)b.z;
    }
    load_face(face, e, f0, f1);
    return e;
}

// Central-difference gradient over packages [0, P + 2); far-field rows get 0.
// PACKED = false writes the three components as separate [P^][64] arrays;
// PACKED = true writes one [P^][64] array of (phi, gx, gy, gz) quadruples in
// the blocked point order (blocked_index), the layout the packed probe gathers
// with one 16-byte (FP32) load per corner.  In FP32 the quadruples pass
// through LDS in that order, so that each of a lane's four stores writes, with
// the wavefront's other lanes, one package's 1 KiB contiguously (written in
// place, a store instruction would fill half of every 64-byte segment of four
// packages).
template <typename T, bool PACKED, bool WORK>
__global__ __launch_bounds__(256) void gradient_kernel(const T *__restrict__ phi, T *__restrict__ out,
                                                       const uint32_t *__restrict__ face,
                                                       const uint32_t *__restrict__ wface, int64_t n_total,
                                                       int64_t n_blocks, T inv_2h, bool nt) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t e_lane = (b * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
    // the FP32 packed layout is stored by the whole wavefront, so a package
    // row past the end repeats the last package instead of leaving
    constexpr bool kStaged = PACKED && sizeof(T) == 4;
    if (!kStaged && e_lane >= n_total) return;
    if (kStaged && e_lane - (lane >> 4) >= n_total) return;   // the whole wavefront is past the end
    const int64_t e = e_lane < n_total ? e_lane : n_total - 1;
    uint4 f0;
    uint2 f1;
    const int64_t p = stencil_package<WORK>(e, face, wface, f0, f1);
    Row<T> c, ox, oy, oz;
    if (p < 2) {
        c = load_row(phi + p * 64 + r * 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) ox.v[i] = oy.v[i] = oz.v[i] = T(0);
    } else {
        Loads<T> l;
        issue_data(phi, p, r, f0, f1, l);
        const Stencil<T> s = assemble(r, l);
        c = s.c;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T xm = i > 0 ? s.c.v[i - 1] : s.xm;
            const T xp = i < 3 ? s.c.v[i + 1] : s.xp;
            ox.v[i] = (xp - xm) * inv_2h;
            oy.v[i] = (s.yp.v[i] - s.ym.v[i]) * inv_2h;
            oz.v[i] = (s.zp.v[i] - s.zm.v[i]) * inv_2h;
        }
    }
    if constexpr (kStaged) {
        // (every lane of the wavefront takes part in every store; the stores
        // of a repeated package are skipped)
        __shared__ float4 s_pk[4][256];
        const int j = r & 3, k = r >> 2, w = threadIdx.x >> 6, q = lane >> 4;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            s_pk[w][64 * q + blocked_index(i, j, k)] = make_float4(c.v[i], ox.v[i], oy.v[i], oz.v[i]);
        __builtin_amdgcn_wave_barrier();
        const int64_t e0 = e_lane - q;   // the wavefront's first package
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int64_t pg = __shfl(p, 16 * g);
            if (e0 + g < n_total) {
                float *o = reinterpret_cast<float *>(out) + pg * 256 + 4 * lane;
                store_row(o, Row<float>{{s_pk[w][64 * g + lane].x, s_pk[w][64 * g + lane].y, s_pk[w][64 * g + lane].z,
                                         s_pk[w][64 * g + lane].w}},
                          nt);
            }
        }
    } else if constexpr (PACKED) {
        const int j = r & 3, k = r >> 2;
        T *o = out + p * 64 * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            store_row(o + 4 * blocked_index(i, j, k), Row<T>{{c.v[i], ox.v[i], oy.v[i], oz.v[i]}}, nt);
    } else {
        T *gx = out + p * 64 + r * 4;
        store_row(gx, ox, nt);
        store_row(gx + n_total * 64, oy, nt);
        store_row(gx + 2 * n_total * 64, oz, nt);
    }
}

// First pass of the factorised near-surface integrals (Sec. 8 kernel
// integral): the cut fraction V of every data point's cell, from the point's
// value and its central-difference gradient, at every point of every
// activated package, FP32.  V depends on the point alone, so a second pass
// sums it over each core point's 32 taps without evaluating any fraction
// again.  The expressions are those of the plain integral kernel, so the
// fractions carry the same bits.  Far-field rows: phi = -B gives 0, +B gives 1.
//
// Most points of the band lie more than half a cell (in the 1-norm of the
// gradient) from the surface, where V is 0 or 1 by the sign of phi alone.
// Only the cut points go through the case analysis: a wavefront lists its cut
// points (at most 256, four per lane) in LDS by ballot and evaluates them one
// per lane, so the case code runs once per 64 cut points instead of once per
// row position of every lane.
template <bool WORK>
__global__ __launch_bounds__(256) void cut_fraction_kernel(const float *__restrict__ phi, float *__restrict__ vfrac,
                                                           const uint32_t *__restrict__ face,
                                                           const uint32_t *__restrict__ wface, int64_t n_total,
                                                           int64_t n_blocks, float inv_h, float inv_2h, bool nt) {
    __shared__ float4 s_q[4][256];
    __shared__ float s_res[4][256];
    __shared__ uint8_t s_dst[4][256];
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t e = (b * 4 + w) * 4 + (lane >> 4);
    const bool live = e < n_total;
    float a[4], gx[4] = {0.f, 0.f, 0.f, 0.f}, gy[4] = {0.f, 0.f, 0.f, 0.f}, gz[4] = {0.f, 0.f, 0.f, 0.f};
    int64_t p = 0;
    if (live) {
        uint4 f0;
        uint2 f1;
        p = stencil_package<WORK>(e, face, wface, f0, f1);
        if (p < 2) {
            const Row<float> c = load_row(phi + p * 64 + r * 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = c.v[i] * inv_h;
        } else {
            Loads<float> l;
            issue_data(phi, p, r, f0, f1, l);
            const Stencil<float> s = assemble(r, l);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float xm = i > 0 ? s.c.v[i - 1] : s.xm;
                const float xp = i < 3 ? s.c.v[i + 1] : s.xp;
                a[i] = s.c.v[i] * inv_h;
                gx[i] = (xp - xm) * inv_2h;
                gy[i] = (s.yp.v[i] - s.ym.v[i]) * inv_2h;
                gz[i] = (s.zp.v[i] - s.zm.v[i]) * inv_2h;
            }
        }
    }
    // a saturated point's V is what the fraction returns, 1 or 0 by the sign
    // of a (see fraction_saturated)
    bool cut[4];
    int n_cut = 0, slot[4];
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        cut[i] = live && !sgrid::fraction_saturated(a[i], gx[i], gy[i], gz[i]);
        const uint64_t m = __ballot(cut[i]);
        slot[i] = n_cut + (int)__popcll(m & below);
        n_cut += (int)__popcll(m);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (cut[i]) {
            s_q[w][slot[i]] = make_float4(a[i], gx[i], gy[i], gz[i]);
            s_dst[w][slot[i]] = (uint8_t)(lane * 4 + i);
        }
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < n_cut; t += 64) {
        const float4 q = s_q[w][t];
        s_res[w][s_dst[w][t]] = sgrid::plane_cube_fraction(q.x, q.y, q.z, q.w);
    }
    __builtin_amdgcn_wave_barrier();
    if (!live) return;
    Row<float> v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v.v[i] = cut[i] ? s_res[w][lane * 4 + i] : (a[i] > 0.0f ? 1.0f : 0.0f);
    store_row(vfrac + p * 64 + r * 4, v, nt);
}

// The operations of the paper's timing test (Sec. 9, Tab. 1).  Sequential
// access: a small change to every value of every activated package, phi +=
// delta, streamed as 16-byte rows (rows 0 and 1, the far field, untouched).
template <typename T>
__global__ __launch_bounds__(256) void add_kernel(T *__restrict__ phi, int64_t n_rows, T delta) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_rows) return;
    T *p = phi + 128 + i * 4;
    Row<T> r = load_row(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) r.v[k] += delta;
    store_row(p, r);
}

// Stencil: the seven-point Laplacian (sum of the six face neighbours - 6 phi)
// / h^2 at every point of every activated package, neighbours through the
// neighbour table as in the sweeps (the same lane mapping and halo loads);
// the far-field rows get 0.
template <typename T, bool WORK>
__global__ __launch_bounds__(256) void laplacian_kernel(const T *__restrict__ phi, T *__restrict__ out,
                                                        const uint32_t *__restrict__ face,
                                                        const uint32_t *__restrict__ wface, int64_t n_total,
                                                        int64_t n_blocks, T inv_h2, bool nt) {
    const int64_t b = xcd_block(blockIdx.x, n_blocks);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t e = (b * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
    if (e >= n_total) return;
    uint4 f0;
    uint2 f1;
    const int64_t p = stencil_package<WORK>(e, face, wface, f0, f1);
    Row<T> o;
    if (p < 2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) o.v[i] = T(0);
    } else {
        Loads<T> l;
        issue_data(phi, p, r, f0, f1, l);
        const Stencil<T> s = assemble(r, l);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T xm = i > 0 ? s.c.v[i - 1] : s.xm;
            const T xp = i < 3 ? s.c.v[i + 1] : s.xp;
            const T sum = (xm + xp) + (s.ym.v[i] + s.yp.v[i]) + (s.zm.v[i] + s.zp.v[i]);
            o.v[i] = fma(T(-6), s.c.v[i], sum) * inv_h2;
        }
    }
    store_row(out + p * 64 + r * 4, o, nt);
}

template <typename T>
__global__ void far_field_kernel(T *__restrict__ phi, T B) {
    const int t = threadIdx.x;   // 128 lanes: rows 0 and 1
    phi[t] = t < 64 ? -B : B;
}

}  // namespace

namespace sgrid {

// Sweep variants: 0 DPP exchange, 1 LDS tile, 2 persistent Morton walk,
// 3 Morton worklist, 4 group-shared LDS, 5 LDS row exchange, 6 persistent
// walk in package-id order.
struct SweepConfig {
    int variant = 0;
    int groups = 1;   // sets of four packages per wavefront, or workgroups per CU (2, 6)
};

// The process-wide setting lives in one atomic word (variant in the high
// half, groups in the low half), and every call reads it once, so a setting
// changed by another thread never reaches a call half-applied.
static std::atomic<uint32_t> g_sweep_word{(0u << 16) | 1u};

void set_sweep_config(int variant, int groups) {
    g_sweep_word.store(((uint32_t)variant << 16) | (uint32_t)groups, std::memory_order_relaxed);
}

SweepConfig current_sweep_config() {
    const uint32_t w = g_sweep_word.load(std::memory_order_relaxed);
    SweepConfig c;
    c.variant = (int)(w >> 16);
    c.groups = (int)(w & 0xFFFFu);
    return c;
}

// The gradient and the Laplacian visit the packages in the sweep's order:
// Morton (worklist) order when the configuration's sweep uses it.
bool stencil_in_worklist_order() {
    const int v = current_sweep_config().variant;
    return v == 2 || v == 3 || v == 4 || v == 7;
}

// MI355X's Infinity Cache (the last level before HBM)
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;

template <typename T>
static void launch_dpp_range(const sgrid_grid *g, const T *src, T *dst, int64_t first, int64_t end, int groups,
                             bool nt, hipStream_t st) {
    const int64_t per_block = 16 * (int64_t)groups;
    const int64_t nb = (end - first + per_block - 1) / per_block;
    const T h2 = (T)(g->h * g->h), inv_h = (T)(1.0 / g->h), dt = (T)(0.5 * g->h);
    const dim3 grid((unsigned)nb), block(256);
    switch (groups) {
        case 1: hipLaunchKernelGGL((reinit_dpp_kernel<T, 1>), grid, block, 0, st, src, dst, g->face, first, end, nb, h2, inv_h, dt, nt); break;
        case 2: hipLaunchKernelGGL((reinit_dpp_kernel<T, 2>), grid, block, 0, st, src, dst, g->face, first, end, nb, h2, inv_h, dt, nt); break;
        case 3: hipLaunchKernelGGL((reinit_dpp_kernel<T, 3>), grid, block, 0, st, src, dst, g->face, first, end, nb, h2, inv_h, dt, nt); break;
        case 4: hipLaunchKernelGGL((reinit_dpp_kernel<T, 4>), grid, block, 0, st, src, dst, g->face, first, end, nb, h2, inv_h, dt, nt); break;
        default: hipLaunchKernelGGL((reinit_dpp_kernel<T, 8>), grid, block, 0, st, src, dst, g->face, first, end, nb, h2, inv_h, dt, nt); break;
    }
}

// One sweep src -> dst.  For variant 7, `mode` says which orders the two
// buffers hold: 0 package-id order -> worklist order, 1 worklist -> worklist
// (the autotuner times this one), 2 worklist -> package-id order.
template <typename T>
static sgrid_status launch_reinit_sweep(const sgrid_grid *g, const T *src, T *dst, hipStream_t st,
                                        const SweepConfig &cfg, int mode = 1) {
    if (g->P == 0) return SGRID_OK;
    const int64_t per_block = 16 * (int64_t)cfg.groups;
    const int64_t nb = (g->P + per_block - 1) / per_block;
    const T h2 = (T)(g->h * g->h), inv_h = (T)(1.0 / g->h), dt = (T)(0.5 * g->h);
    const dim3 grid((unsigned)nb), block(256);
    // streaming stores when the two field buffers exceed the last-level cache
    const bool nt = 2.0 * (double)g->total() * 64.0 * sizeof(T) > kLastLevelCacheBytes;
    if (cfg.variant == 7) {
        const int64_t nb7 = (g->P + 15) / 16;
        const dim3 grid7((unsigned)nb7);
        if (mode == 0)
            hipLaunchKernelGGL((reinit_morton_kernel<T, 0>), grid7, block, 0, st, src, dst, g->wface, g->mface, g->P,
                               nb7, h2, inv_h, dt, nt);
        else if (mode == 1)
            hipLaunchKernelGGL((reinit_morton_kernel<T, 1>), grid7, block, 0, st, src, dst, g->wface, g->mface, g->P,
                               nb7, h2, inv_h, dt, nt);
        else
            hipLaunchKernelGGL((reinit_morton_kernel<T, 2>), grid7, block, 0, st, src, dst, g->wface, g->mface, g->P,
                               nb7, h2, inv_h, dt, nt);
    } else if (cfg.variant == 6) {
        const int64_t n_sets = (g->P + 3) / 4;
        const int64_t nbp = std::min<int64_t>((int64_t)cu_count() * cfg.groups, (n_sets + 3) / 4);
        hipLaunchKernelGGL(reinit_pipe_lin_kernel<T>, dim3((unsigned)nbp), block, 0, st, src, dst, g->face, g->P, nbp,
                           h2, inv_h, dt);
    } else if (cfg.variant == 5) {
        switch (cfg.groups) {
            case 1: hipLaunchKernelGGL((reinit_rows_kernel<T, 1>), grid, block, 0, st, src, dst, g->face, g->P, nb, h2, inv_h, dt, nt); break;
            case 2: hipLaunchKernelGGL((reinit_rows_kernel<T, 2>), grid, block, 0, st, src, dst, g->face, g->P, nb, h2, inv_h, dt, nt); break;
            case 3: hipLaunchKernelGGL((reinit_rows_kernel<T, 3>), grid, block, 0, st, src, dst, g->face, g->P, nb, h2, inv_h, dt, nt); break;
            case 4: hipLaunchKernelGGL((reinit_rows_kernel<T, 4>), grid, block, 0, st, src, dst, g->face, g->P, nb, h2, inv_h, dt, nt); break;
            default: hipLaunchKernelGGL((reinit_rows_kernel<T, 8>), grid, block, 0, st, src, dst, g->face, g->P, nb, h2, inv_h, dt, nt); break;
        }
    } else if (cfg.variant == 4) {
        const int64_t ng = (g->P + kGroup - 1) / kGroup;
        hipLaunchKernelGGL(reinit_share_kernel<T>, dim3((unsigned)ng), dim3(1024), 0, st, src, dst, g->work, g->sface,
                           g->P, ng, h2, inv_h, dt);
    } else if (cfg.variant == 3) {
        switch (cfg.groups) {
            case 1: hipLaunchKernelGGL((reinit_work_kernel<T, 1>), grid, block, 0, st, src, dst, g->wface, g->P, nb, h2, inv_h, dt, nt); break;
            case 2: hipLaunchKernelGGL((reinit_work_kernel<T, 2>), grid, block, 0, st, src, dst, g->wface, g->P, nb, h2, inv_h, dt, nt); break;
            case 3: hipLaunchKernelGGL((reinit_work_kernel<T, 3>), grid, block, 0, st, src, dst, g->wface, g->P, nb, h2, inv_h, dt, nt); break;
            case 4: hipLaunchKernelGGL((reinit_work_kernel<T, 4>), grid, block, 0, st, src, dst, g->wface, g->P, nb, h2, inv_h, dt, nt); break;
            default: hipLaunchKernelGGL((reinit_work_kernel<T, 8>), grid, block, 0, st, src, dst, g->wface, g->P, nb, h2, inv_h, dt, nt); break;
        }
    } else if (cfg.variant == 2) {
        const int64_t n_sets = (g->P + 3) / 4;
        const int64_t nbp = std::min<int64_t>((int64_t)cu_count() * cfg.groups, (n_sets + 3) / 4);
        hipLaunchKernelGGL(reinit_pipe_kernel<T>, dim3((unsigned)nbp), block, 0, st, src, dst, g->wface, g->P, nbp,
                           h2, inv_h, dt, nt);
    } else if (cfg.variant == 1) {
        hipLaunchKernelGGL(reinit_lds_kernel<T>, grid, block, 0, st, src, dst, g->face, g->P, nb, cfg.groups, h2,
                           inv_h, dt);
    } else {
        launch_dpp_range<T>(g, src, dst, 2, 2 + g->P, cfg.groups, nt, st);
    }
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
    // variant 7 holds the field in worklist order between its first and last
    // sweep; a single sweep goes id order to id order (variant 3)
    SweepConfig one = cfg;
    if (cfg.variant == 7 && n_iter == 1) one.variant = 3;
    for (int32_t it = 0; it < n_iter; ++it) {
        const int mode = it == 0 ? 0 : (it == n_iter - 1 ? 2 : 1);
        sgrid_status s = launch_reinit_sweep<T>(g, a, b, st, one, mode);
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


// The first pass of the factorised integrals over all P + 2 packages.
sgrid_status launch_cut_fractions(const sgrid_grid *g, const float *phi, float *vfrac, hipStream_t st) {
    const int64_t nt = g->total();
    const int64_t nb = (nt + 15) / 16;
    if (nb > kMaxGrid) {
        set_error("too many packages for one launch");
        return SGRID_E_INVALID;
    }
    const bool work = stencil_in_worklist_order();
    const bool nt_store = 2.0 * (double)nt * 64.0 * 4.0 > kLastLevelCacheBytes;
    const float inv_h = (float)(1.0 / g->h), inv_2h = (float)(0.5 / g->h);
    if (work)
        hipLaunchKernelGGL(cut_fraction_kernel<true>, dim3((unsigned)nb), dim3(256), 0, st, phi, vfrac, g->face,
                           g->wface, nt, nb, inv_h, inv_2h, nt_store);
    else
        hipLaunchKernelGGL(cut_fraction_kernel<false>, dim3((unsigned)nb), dim3(256), 0, st, phi, vfrac, g->face,
                           g->wface, nt, nb, inv_h, inv_2h, nt_store);
    SG_CHECK_LAUNCH("cut fractions");
    return SGRID_OK;
}

}  // namespace sgrid

extern "C" sgrid_status sgrid_set_sweep_config(int32_t variant, int32_t groups) {
    sgrid::clear_error();
    SG_REQUIRE(variant >= 0 && variant <= 7, "sweep variant must be 0..7 (got %d)", variant);
    SG_REQUIRE(groups == 1 || groups == 2 || groups == 3 || groups == 4 || groups == 8, "groups must be 1, 2, 3, 4 or 8 (got %d)", groups);
    sgrid::set_sweep_config(variant, groups);
    return SGRID_OK;
}

// Candidates of the sweep autotuner: (variant, groups).
constexpr int kNumTune = 7;
static const int kTuneCandidates[kNumTune][2] = {{0, 1}, {0, 2}, {2, 4}, {3, 1}, {3, 2}, {5, 1}, {7, 1}};

template <typename T>
static sgrid_status autotune_sweep(const sgrid_grid *g, const T *phi, T *scratch, int32_t reps, hipStream_t st,
                                   int32_t *variant_out, int32_t *groups_out, float *us_table) {
    hipEvent_t e0, e1;
    SG_CHECK_HIP(hipEventCreate(&e0));
    SG_CHECK_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    sgrid::SweepConfig pick;
    for (int c = 0; c < kNumTune; ++c) {
        sgrid::SweepConfig cfg;
        cfg.variant = kTuneCandidates[c][0];
        cfg.groups = kTuneCandidates[c][1];
        // phi is only read: every timed sweep writes scratch
        sgrid_status s = sgrid::launch_reinit_sweep<T>(g, phi, scratch, st, cfg);
        if (s == SGRID_OK && hipEventRecord(e0, st) != hipSuccess) s = SGRID_E_HIP;
        for (int32_t k = 0; s == SGRID_OK && k < reps; ++k) s = sgrid::launch_reinit_sweep<T>(g, phi, scratch, st, cfg);
        float ms = 0.f;
        if (s == SGRID_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
            sgrid::set_error("sweep autotune timing failed");
            s = SGRID_E_HIP;
        }
        if (s != SGRID_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return s;
        }
        const float us = 1e3f * ms / reps;
        if (us_table) us_table[c] = us;
        if (us < best) {
            best = us;
            pick = cfg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    sgrid::set_sweep_config(pick.variant, pick.groups);
    if (variant_out) *variant_out = pick.variant;
    if (groups_out) *groups_out = pick.groups;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_autotune_sweep(const sgrid_grid *g, sgrid_dtype dtype, const void *phi, void *scratch,
                                             int32_t reps, void *stream, int32_t *variant_out, int32_t *groups_out,
                                             float *us_table) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr && phi != nullptr && scratch != nullptr, "NULL argument");
    SG_REQUIRE(phi != scratch, "phi and scratch must be distinct buffers");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(scratch, 16), "phi / scratch must be 16-byte aligned");
    SG_REQUIRE(reps >= 1 && reps <= 1000, "reps must be in 1..1000");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    hipStream_t st = sg_stream(stream);
    if (dtype == SGRID_F32)
        return autotune_sweep<float>(g, (const float *)phi, (float *)scratch, reps, st, variant_out, groups_out,
                                     us_table);
    return autotune_sweep<double>(g, (const double *)phi, (double *)scratch, reps, st, variant_out, groups_out,
                                  us_table);
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
    const sgrid::SweepConfig cfg = sgrid::current_sweep_config();
    if (dtype == SGRID_F32)
        return sgrid::reinit_impl<float>(g, (float *)phi, (float *)scratch, n_iter, st, cfg);
    return sgrid::reinit_impl<double>(g, (double *)phi, (double *)scratch, n_iter, st, cfg);
}

template <bool PACKED>
static sgrid_status gradient_entry(const sgrid_grid *g, sgrid_dtype dtype, const void *phi, void *out,
                                   void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(phi != nullptr && out != nullptr, "phi or output is NULL");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(out, 16), "phi / output must be 16-byte aligned");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    hipStream_t st = sg_stream(stream);
    const int64_t nt = g->total();
    const int64_t nb = (nt + 15) / 16;
    const bool work = sgrid::stencil_in_worklist_order();
    // streaming stores when phi and the output together exceed the last-level
    // cache; not for the FP64 packed layout, whose four stores per lane each
    // fill only parts of lines (the cache merges them, streaming writes would
    // not; the FP32 packed layout is written by whole lines)
    const bool stream_out = !(PACKED && dtype == SGRID_F64) &&
                            (double)nt * 64.0 * (dtype == SGRID_F32 ? 4.0 : 8.0) * 4.0 > sgrid::kLastLevelCacheBytes;
    if (dtype == SGRID_F32) {
        if (work)
            hipLaunchKernelGGL((gradient_kernel<float, PACKED, true>), dim3((unsigned)nb), dim3(256), 0, st,
                               (const float *)phi, (float *)out, g->face, g->wface, nt, nb, (float)(0.5 / g->h), stream_out);
        else
            hipLaunchKernelGGL((gradient_kernel<float, PACKED, false>), dim3((unsigned)nb), dim3(256), 0, st,
                               (const float *)phi, (float *)out, g->face, g->wface, nt, nb, (float)(0.5 / g->h), stream_out);
    } else {
        if (work)
            hipLaunchKernelGGL((gradient_kernel<double, PACKED, true>), dim3((unsigned)nb), dim3(256), 0, st,
                               (const double *)phi, (double *)out, g->face, g->wface, nt, nb, 0.5 / g->h, stream_out);
        else
            hipLaunchKernelGGL((gradient_kernel<double, PACKED, false>), dim3((unsigned)nb), dim3(256), 0, st,
                               (const double *)phi, (double *)out, g->face, g->wface, nt, nb, 0.5 / g->h, stream_out);
    }
    SG_CHECK_LAUNCH("gradient sweep");
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_compute_gradient(const sgrid_grid *g, sgrid_dtype dtype, const void *phi, void *grad,
                                               void *stream) {
    return gradient_entry<false>(g, dtype, phi, grad, stream);
}

extern "C" sgrid_status sgrid_compute_gradient_packed(const sgrid_grid *g, sgrid_dtype dtype, const void *phi,
                                                      void *packed, void *stream) {
    return gradient_entry<true>(g, dtype, phi, packed, stream);
}

extern "C" sgrid_status sgrid_sequential_update(const sgrid_grid *g, sgrid_dtype dtype, void *phi, double delta,
                                                void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr && phi != nullptr, "NULL argument");
    SG_REQUIRE(sg_aligned(phi, 16), "phi must be 16-byte aligned");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    if (g->P == 0) return SGRID_OK;
    hipStream_t st = sg_stream(stream);
    const int64_t n_rows = g->P * 16;
    const int64_t nb = (n_rows + 255) / 256;
    if (dtype == SGRID_F32)
        hipLaunchKernelGGL(add_kernel<float>, dim3((unsigned)nb), dim3(256), 0, st, (float *)phi, n_rows,
                           (float)delta);
    else
        hipLaunchKernelGGL(add_kernel<double>, dim3((unsigned)nb), dim3(256), 0, st, (double *)phi, n_rows, delta);
    SG_CHECK_LAUNCH("sequential update");
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_compute_laplacian(const sgrid_grid *g, sgrid_dtype dtype, const void *phi, void *out,
                                                void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr && phi != nullptr && out != nullptr, "NULL argument");
    SG_REQUIRE(phi != out, "phi and out must be distinct buffers");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(out, 16), "phi / out must be 16-byte aligned");
    SG_REQUIRE(dtype == SGRID_F32 || dtype == SGRID_F64, "unknown dtype %d", (int)dtype);
    hipStream_t st = sg_stream(stream);
    const int64_t nt = g->total();
    const int64_t nb = (nt + 15) / 16;
    const bool work = sgrid::stencil_in_worklist_order();
    // streaming stores when phi and the output together exceed the last-level cache
    const bool stream_out = (double)nt * 64.0 * (dtype == SGRID_F32 ? 4.0 : 8.0) * 2.0 > sgrid::kLastLevelCacheBytes;
    if (dtype == SGRID_F32) {
        if (work)
            hipLaunchKernelGGL((laplacian_kernel<float, true>), dim3((unsigned)nb), dim3(256), 0, st,
                               (const float *)phi, (float *)out, g->face, g->wface, nt, nb,
                               (float)(1.0 / (g->h * g->h)), stream_out);
        else
            hipLaunchKernelGGL((laplacian_kernel<float, false>), dim3((unsigned)nb), dim3(256), 0, st,
                               (const float *)phi, (float *)out, g->face, g->wface, nt, nb,
                               (float)(1.0 / (g->h * g->h)), stream_out);
    } else {
        if (work)
            hipLaunchKernelGGL((laplacian_kernel<double, true>), dim3((unsigned)nb), dim3(256), 0, st,
                               (const double *)phi, (double *)out, g->face, g->wface, nt, nb, 1.0 / (g->h * g->h), stream_out);
        else
            hipLaunchKernelGGL((laplacian_kernel<double, false>), dim3((unsigned)nb), dim3(256), 0, st,
                               (const double *)phi, (double *)out, g->face, g->wface, nt, nb, 1.0 / (g->h * g->h), stream_out);
    }
    SG_CHECK_LAUNCH("laplacian");
    return SGRID_OK;
}

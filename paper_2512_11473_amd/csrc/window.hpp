// The 9^3 phi window of a package (local coordinates -2..6 per axis), gathered
// through the package's 27-entry neighbour row with the index shift of
// Sec. 5.2 (slot = (s + 4) / 4, data = s + 4 - 4 slot per axis).
#pragma once

#include "common.hpp"

namespace sgrid {

constexpr int kWin = 9, kWinN = kWin * kWin * kWin;

// Window point q (x fastest) of the package whose neighbour ids are ids[27]:
// the flat index of its value in the field.
__device__ __forceinline__ int64_t window_source(const uint32_t *ids, int q) {
    const int x = q % kWin - 2, y = (q / kWin) % kWin - 2, z = q / (kWin * kWin) - 2;
    const int kx = (x + 4) >> 2, ky = (y + 4) >> 2, kz = (z + 4) >> 2;
    const int d = (x + 4 - 4 * kx) + 4 * (y + 4 - 4 * ky) + 16 * (z + 4 - 4 * kz);
    return (int64_t)ids[kx + 3 * ky + 9 * kz] * 64 + d;
}

// Thread t of NT stages its share of the window into s_phi.  All of the
// thread's loads are issued before any is used (a plain strided loop would
// wait for each load before the next: one memory round trip per iteration).
template <int NT>
__device__ __forceinline__ void stage_window_part(const float *__restrict__ phi, const uint32_t *ids, int t,
                                                  float *s_phi) {
    constexpr int kIters = (kWinN + NT - 1) / NT;
    float v[kIters];
#pragma unroll
    for (int u = 0; u < kIters; ++u) {
        const int q = t + u * NT;
        v[u] = phi[window_source(ids, q < kWinN ? q : kWinN - 1)];
    }
#pragma unroll
    for (int u = 0; u < kIters; ++u) {
        const int q = t + u * NT;
        if (q < kWinN) s_phi[q] = v[u];
    }
}

}  // namespace sgrid

// The per-point reinitialisation update, shared by the single-grid and the
// batched sweeps so that both produce the same bits.
#pragma once

#include <hip/hip_runtime.h>

namespace sgrid {

// Precision policy: FP32 uses the hardware square root and reciprocal square
// root (about 1 ulp); FP64 uses correctly rounded operations.
template <typename T>
struct Fast;
template <>
struct Fast<float> {
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
};
template <>
struct Fast<double> {
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
};

// Godunov-upwinded update of one point (Sussman-Smereka-Osher iteration),
// written in differences of phi (units of h):
//   S > 0: a^2 = max(max(D-,0)^2, min(D+,0)^2) = max(p0 - xm, p0 - xp, 0)^2 / h^2
//   S < 0: a^2 = max(min(D-,0)^2, max(D+,0)^2) = max(xm - p0, xp - p0, 0)^2 / h^2
// so with sg = sign(S) every axis contributes max(sg (p0 - m), sg (p0 - p), 0)^2.
// Each term sg (p0 - m) is formed as fma(-sg, m, sg p0): sg = +-1 makes both
// products exact, so this is the correctly rounded sg (p0 - m), the same value
// as rounding p0 - m and flipping its sign, in one instruction.  Every other
// fused operation is written out too and contraction is off in the body, so
// the compiler has no choice left: every kernel that calls this produces the
// same bits, whatever the code around it.
template <typename T>
__device__ __forceinline__ T upwind_update(T p0, T xm, T xp, T ym, T yp, T zm, T zp, T h2, T inv_h, T dt) {
#pragma clang fp contract(off)
    const T S = p0 * Fast<T>::rsqrt(fma(p0, p0, h2));
    const T sg = S > T(0) ? T(1) : T(-1);
    const T t = sg * p0;
    const T ax = fmax(fmax(fma(-sg, xm, t), fma(-sg, xp, t)), T(0));
    const T ay = fmax(fmax(fma(-sg, ym, t), fma(-sg, yp, t)), T(0));
    const T az = fmax(fmax(fma(-sg, zm, t), fma(-sg, zp, t)), T(0));
    const T g1 = fma(Fast<T>::sqrt(fma(az, az, fma(ay, ay, ax * ax))), inv_h, T(-1));   // G - 1
    return fma(-(dt * S), g1, p0);
}

}  // namespace sgrid

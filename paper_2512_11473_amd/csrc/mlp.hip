// Surrogate network for the near-surface integrals: a 216 -> 128 -> 128 -> 4
// MLP with tanh-approximated GELU, input the 6 x 6 x 6 window of phi / h
// around a core data point (offsets -2..3, x fastest), output
// (K_W, h K_grad).  Training (forward, backward, Adam) and inference run on
// BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; the first
// layer splits its input into BF16 hi and lo parts (x = hi + lo, two MFMAs)
// so the input keeps about 16 significant bits.
//
// MFMA lane layout used throughout (16 x 16 x 32, wave64, lane l, r = l % 16,
// q = l / 16):  A[m][k] with m = r, k = 8q + j (j = 0..7);
//               B[k][n] with k = 8q + j, n = r;
//               C[m][n] with m = 4q + i (i = 0..3), n = r.
// A wavefront owns a tile of 16 samples; activations move from the C layout
// to the A layout of the next layer through a row-major BF16 tile in LDS.
//
// Parameters are FP32 masters in one packed vector (W1[128][216], b1[128],
// W2[128][128], b2[128], W3[4][128], b3[4]), with BF16 copies laid out for
// the B operands: W1 [128][224] (zero padded), W2 [128][128], its transpose
// for the backward pass, W3 [16][128] (rows 4..15 zero).
#include <float.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "fraction.hpp"
#include "window.hpp"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kIn = 216, kInPad = 224, kH = 128, kOut = 4;
constexpr int kNParam = 44804;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH;
static_assert(oB3 + kOut == kNParam, "parameter layout");

struct MlpDev {
    const float *w;      // FP32 masters
    const bf16 *w1b;     // [128][224]
    const bf16 *w2b;     // [128][128]
    const bf16 *w2tb;    // [128][128], transposed
    const bf16 *w3b;     // [16][128]
};

__device__ __forceinline__ floatx4 mfma(const bf16x8 &a, const bf16x8 &b, const floatx4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// GELU in its tanh form, 0.5 z (1 + tanh(u)) with u = sqrt(2/pi) (z + 0.044715
// z^3), evaluated as z s with s = 0.5 (1 + tanh(u)) = 1 / (1 + exp(-2u)): the
// same function.  exp(-2u) = 2^(k z (1 + 0.044715 z^2)) with k = -2 sqrt(2/pi)
// / ln 2 folded into the polynomial, on the hardware's base-2 exponential and
// reciprocal (each within one ulp; the activations dominate the network's
// vector work, and an IEEE division would cost ten instructions more).  For
// large |u| the exponential saturates to 0 or inf and s to 1 or 0.
__device__ __forceinline__ float gelu_s(float z) {
    const float a = z * __builtin_fmaf(-0.1029432395800235f, z * z, -2.302208198144325f);
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a));
}

__device__ __forceinline__ float gelu(float z) { return z * gelu_s(z); }

// d/dz [z s] = s + z s (1 - s) 2 u'(z), u' = sqrt(2/pi) (1 + 3 * 0.044715 z^2)
// (the tanh form's 0.5 (1 + th) + 0.5 z (1 - th^2) u' with th = 2s - 1).
__device__ __forceinline__ float gelu_grad(float z) {
    const float s = gelu_s(z);
    return s + 2.0f * z * s * (1.0f - s) * 0.7978845608028654f * (1.0f + 3.0f * 0.044715f * z * z);
}

struct Tile {
    floatx4 z1[8], z2[8];
    floatx4 y;
};

// Forward pass of one 16-sample tile.  `xs(m, k0, v)` returns the 8 inputs
// k0..k0+7 of sample m (zero past 215).  `a1`, `a2` are the wave's row-major
// [16][128] BF16 activation tiles in LDS; `xh` (nullable) receives the BF16 hi
// part of the inputs [16][224] for the weight gradient.  Ends with the wave's
// LDS writes complete; callers synchronise the workgroup between phases.
template <class XSrc>
__device__ __forceinline__ void forward_tile(const XSrc &xs, const MlpDev &W, bf16 *a1, bf16 *a2, bf16 *xh, Tile &T,
                                             int lane) {
    const int r = lane & 15, q = lane >> 4;
    // every accumulator starts from its bias (the column's hidden unit)
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const float bb = W.w[oB1 + 16 * t + r];
        T.z1[t] = floatx4{bb, bb, bb, bb};
    }
    for (int s = 0; s < kInPad / 32; ++s) {
        float v[8];
        xs(r, 32 * s + 8 * q, v);
        bf16x8 ah, al;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bf16 hi = (bf16)v[j];
            ah[j] = hi;
            al[j] = (bf16)(v[j] - (float)hi);
        }
        if (xh) *reinterpret_cast<bf16x8 *>(xh + r * kInPad + 32 * s + 8 * q) = ah;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bf16x8 b = ld8(W.w1b + (16 * t + r) * kInPad + 32 * s + 8 * q);
            T.z1[t] = mfma(ah, b, T.z1[t]);
            T.z1[t] = mfma(al, b, T.z1[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) a1[(4 * q + i) * kH + 16 * t + r] = (bf16)gelu(T.z1[t][i]);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const float bb = W.w[oB2 + 16 * t + r];
        T.z2[t] = floatx4{bb, bb, bb, bb};
    }
#pragma unroll
    for (int s = 0; s < kH / 32; ++s) {
        const bf16x8 a = ld8(a1 + r * kH + 32 * s + 8 * q);
#pragma unroll
        for (int t = 0; t < 8; ++t) T.z2[t] = mfma(a, ld8(W.w2b + (16 * t + r) * kH + 32 * s + 8 * q), T.z2[t]);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) a2[(4 * q + i) * kH + 16 * t + r] = (bf16)gelu(T.z2[t][i]);
    __syncthreads();
    const float b3 = r < kOut ? W.w[oB3 + r] : 0.f;
    T.y = floatx4{b3, b3, b3, b3};
#pragma unroll
    for (int s = 0; s < kH / 32; ++s)
        T.y = mfma(ld8(a2 + r * kH + 32 * s + 8 * q), ld8(W.w3b + r * kH + 32 * s + 8 * q), T.y);
}

// ---------------------------------------------------------------------------
// Training: forward + backward of 64 samples per workgroup (4 wavefronts x 16)
// and this workgroup's partial weight gradient, written to part[blockIdx.x].
// dY is either given (`dy_in`, [B][4]) or the gradient of the weighted
// squared error sum_o w_o (y_o - t_o)^2 / B (`t_in`, [B][4], `lw` = w_o).
// ---------------------------------------------------------------------------
struct GlobalX {
    const float *x;
    int64_t base, B;
    __device__ __forceinline__ void operator()(int m, int k0, float *v) const {
        const int64_t s = base + m;
        if (s < B && k0 + 8 <= kIn) {
            const float4 a = *reinterpret_cast<const float4 *>(x + s * kIn + k0);
            const float4 b = *reinterpret_cast<const float4 *>(x + s * kIn + k0 + 4);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = 0.f;
        }
    }
};

constexpr int kTrainRows = 64;

__global__ __launch_bounds__(256) void train_kernel(MlpDev W, const float *__restrict__ x, int64_t B,
                                                    const float *__restrict__ t_in, const float *__restrict__ dy_in,
                                                    float4 lw, float *__restrict__ part, float *__restrict__ loss_part) {
    __shared__ __attribute__((aligned(16))) bf16 s_xh[kTrainRows * kInPad];
    __shared__ __attribute__((aligned(16))) bf16 s_a1[kTrainRows * kH];
    __shared__ __attribute__((aligned(16))) bf16 s_a2[kTrainRows * kH];
    __shared__ __attribute__((aligned(16))) bf16 s_d1[kTrainRows * kH];
    __shared__ __attribute__((aligned(16))) bf16 s_d2[kTrainRows * kH];
    __shared__ float s_dy[kTrainRows][kOut];
    __shared__ float s_loss[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, q = lane >> 4;
    const int64_t base = (int64_t)blockIdx.x * kTrainRows + 16 * w;
    Tile T;
    GlobalX xs{x, base, B};
    forward_tile(xs, W, s_a1 + 16 * w * kH, s_a2 + 16 * w * kH, s_xh + 16 * w * kInPad, T, lane);

    // dY (rows past B contribute nothing)
    float lsum = 0.f;
    if (r < kOut) {
        const float wo = r == 0 ? lw.x : (r == 1 ? lw.y : (r == 2 ? lw.z : lw.w));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t s = base + 4 * q + i;
            float d = 0.f;
            if (s < B) {
                if (dy_in) {
                    d = dy_in[s * kOut + r];
                } else {
                    const float e = T.y[i] - t_in[s * kOut + r];
                    lsum += wo * e * e;
                    d = 2.0f * wo * e / (float)B;
                }
            }
            s_dy[16 * w + 4 * q + i][r] = d;
        }
    }
    // wave-level loss sum
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off);
    if (lane == 0) s_loss[w] = lsum;
    __syncthreads();

    // dA2 = dY W3 (K = 4, FP32 masters), dZ2 = dA2 * gelu'(z2)
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int n = 16 * t + r;
        const float w0 = W.w[oW3 + n], w1 = W.w[oW3 + kH + n], w2 = W.w[oW3 + 2 * kH + n], w3 = W.w[oW3 + 3 * kH + n];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float *d = s_dy[16 * w + 4 * q + i];
            const float da = d[0] * w0 + d[1] * w1 + d[2] * w2 + d[3] * w3;
            s_d2[(16 * w + 4 * q + i) * kH + n] = (bf16)(da * gelu_grad(T.z2[t][i]));
        }
    }
    __syncthreads();
    // dA1 = dZ2 W2 (B operand from the transposed copy), dZ1 = dA1 * gelu'(z1)
    {
        floatx4 acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        const bf16 *d2 = s_d2 + 16 * w * kH;
#pragma unroll
        for (int s = 0; s < kH / 32; ++s) {
            const bf16x8 a = ld8(d2 + r * kH + 32 * s + 8 * q);
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[t] = mfma(a, ld8(W.w2tb + (16 * t + r) * kH + 32 * s + 8 * q), acc[t]);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                s_d1[(16 * w + 4 * q + i) * kH + 16 * t + r] = (bf16)(acc[t][i] * gelu_grad(T.z1[t][i]));
    }
    __syncthreads();

    // Weight gradients over the 64 rows: C[o][i] = sum_m D[m][o] S[m][i], with
    // A[o][m] gathered from column o of D and B[m][i] from column i of S.
    float *P = part + (int64_t)blockIdx.x * kNParam;
    const int n_w1 = 8 * (kInPad / 16), n_w2 = 64, n_w3 = 8;
    for (int tile = w; tile < n_w1 + n_w2 + n_w3; tile += 4) {
        const bf16 *D, *S;
        int sl, ot, it, obase, ostride, omax, imax;
        if (tile < n_w1) {
            D = s_d1; S = s_xh; sl = kInPad; ot = tile / (kInPad / 16); it = tile % (kInPad / 16);
            obase = oW1; ostride = kIn; omax = kH; imax = kIn;
        } else if (tile < n_w1 + n_w2) {
            const int u = tile - n_w1;
            D = s_d2; S = s_a1; sl = kH; ot = u / 8; it = u % 8;
            obase = oW2; ostride = kH; omax = kH; imax = kH;
        } else {
            D = nullptr; S = s_a2; sl = kH; ot = 0; it = tile - n_w1 - n_w2;
            obase = oW3; ostride = kH; omax = kOut; imax = kH;
        }
        floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kTrainRows / 32; ++ks) {
            bf16x8 a, b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int m = 32 * ks + 8 * q + j;
                const int o = 16 * ot + r;
                a[j] = D ? D[m * kH + o] : (o < kOut ? (bf16)s_dy[m][o] : (bf16)0.f);
                b[j] = S[m * sl + 16 * it + r];
            }
            acc = mfma(a, b, acc);
        }
        const int i = 16 * it + r;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int o = 16 * ot + 4 * q + jj;
            if (o < omax && i < imax) P[obase + o * ostride + i] = acc[jj];
        }
    }
    // bias gradients: column sums of dZ1, dZ2 (BF16 tiles) and dY (FP32)
    if (threadIdx.x < kH) {
        const int o = threadIdx.x;
        float s1 = 0.f, s2 = 0.f;
        for (int m = 0; m < kTrainRows; ++m) {
            s1 += (float)s_d1[m * kH + o];
            s2 += (float)s_d2[m * kH + o];
        }
        P[oB1 + o] = s1;
        P[oB2 + o] = s2;
    } else if (threadIdx.x < kH + kOut) {
        const int o = threadIdx.x - kH;
        float s3 = 0.f;
        for (int m = 0; m < kTrainRows; ++m) s3 += s_dy[m][o];
        P[oB3 + o] = s3;
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = s_loss[0] + s_loss[1] + s_loss[2] + s_loss[3];
}

// grad[p] = sum over workgroups of part[wg][p], in workgroup order (deterministic).
__global__ __launch_bounds__(256) void reduce_kernel(const float *__restrict__ part, int n_part,
                                                     float *__restrict__ grad, const float *__restrict__ loss_part,
                                                     float *__restrict__ loss_out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kNParam) {
        float s = 0.f;
        for (int g = 0; g < n_part; ++g) s += part[(int64_t)g * kNParam + p];
        grad[p] = s;
    }
    if (p == 0 && loss_out) {
        float s = 0.f;
        for (int g = 0; g < n_part; ++g) s += loss_part[g];
        *loss_out = s;
    }
}

// Refresh the BF16 operand copies of parameter p from the FP32 master.
__device__ __forceinline__ void write_bf16_copy(int p, float v, bf16 *w1b, bf16 *w2b, bf16 *w2tb, bf16 *w3b) {
    if (p < oB1) {
        const int o = p / kIn, i = p % kIn;
        w1b[o * kInPad + i] = (bf16)v;
    } else if (p >= oW2 && p < oB2) {
        const int o = (p - oW2) / kH, i = (p - oW2) % kH;
        w2b[o * kH + i] = (bf16)v;
        w2tb[i * kH + o] = (bf16)v;
    } else if (p >= oW3 && p < oB3) {
        const int o = (p - oW3) / kH, i = (p - oW3) % kH;
        w3b[o * kH + i] = (bf16)v;
    }
}

__global__ __launch_bounds__(256) void sync_copies_kernel(const float *__restrict__ w, bf16 *w1b, bf16 *w2b,
                                                          bf16 *w2tb, bf16 *w3b) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kNParam) write_bf16_copy(p, w[p], w1b, w2b, w2tb, w3b);
}

// Adam (Kingma & Ba 2015) with bias correction, then the BF16 copies.
__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                                   const float *__restrict__ g, float lr, float b1, float b2, float eps,
                                                   float c1, float c2, bf16 *w1b, bf16 *w2b, bf16 *w2tb, bf16 *w3b) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kNParam) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const float wp = w[p] - lr * (mp / c1) / (sqrtf(vp / c2) + eps);
    w[p] = wp;
    write_bf16_copy(p, wp, w1b, w2b, w2tb, w3b);
}

// Forward only, for [B][216] inputs.
__global__ __launch_bounds__(256) void forward_kernel(MlpDev W, const float *__restrict__ x, int64_t B,
                                                      float *__restrict__ y) {
    __shared__ __attribute__((aligned(16))) bf16 s_a1[64 * kH];
    __shared__ __attribute__((aligned(16))) bf16 s_a2[64 * kH];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, q = lane >> 4;
    const int64_t base = (int64_t)blockIdx.x * 64 + 16 * w;
    Tile T;
    forward_tile(GlobalX{x, base, B}, W, s_a1 + 16 * w * kH, s_a2 + 16 * w * kH, nullptr, T, lane);
    if (r < kOut)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t s = base + 4 * q + i;
            if (s < B) y[s * kOut + r] = T.y[i];
        }
}

}  // namespace

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
struct sgrid_mlp {
    int device = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    bf16 *w1b = nullptr, *w2b = nullptr, *w2tb = nullptr, *w3b = nullptr;
    float *part = nullptr;        // training partial gradients
    float *loss_part = nullptr;
    int64_t part_rows = 0;        // workgroups the partial buffers hold
    int64_t step = 0;
    float gate_tau = FLT_MAX;     // non-planarity threshold (mean squared residual, units of h^2)
    float kw_lo = -0.05f, kw_hi = 1.05f;
    uint32_t *fallback = nullptr;  // fallback cell list of the learned integrals
    int64_t fallback_cap = 0;
    // Calls that use the model are ordered across streams: each records `done`
    // on its stream, and a call on another stream first waits for it.
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
    MlpDev dev() const { return MlpDev{w, w1b, w2b, w2tb, w3b}; }
};

namespace sgrid {

static void free_mlp(sgrid_mlp *m) {
    if (!m) return;
    void *ptrs[] = {m->w, m->m, m->v, m->grad, m->loss, m->w1b, m->w2b, m->w2tb, m->w3b, m->part, m->loss_part,
                    m->fallback};
    for (void *p : ptrs) dev_free(p);
    if (m->done) (void)hipEventDestroy(m->done);
    delete m;
}

// Start of a call that uses the model's buffers on stream `st`: wait for the
// model's previous call when that ran on another stream.
static sgrid_status begin_use(const sgrid_mlp *mc, hipStream_t st) {
    sgrid_mlp *m = const_cast<sgrid_mlp *>(mc);
    if (m->used && m->last != st) SG_CHECK_HIP(hipStreamWaitEvent(st, m->done, 0));
    return SGRID_OK;
}

// End of such a call: later calls on other streams wait for this point.
static sgrid_status end_use(const sgrid_mlp *mc, hipStream_t st) {
    sgrid_mlp *m = const_cast<sgrid_mlp *>(mc);
    SG_CHECK_HIP(hipEventRecord(m->done, st));
    m->last = st;
    m->used = true;
    return SGRID_OK;
}

// Growing a buffer frees the old block, which kernels queued by earlier calls
// (on any stream) may still use: wait for the device before handing it back
// to the allocator, which may give it to the next request of that size.
static sgrid_status ensure_part(sgrid_mlp *m, int64_t rows) {
    if (rows <= m->part_rows) return SGRID_OK;
    if (m->part || m->loss_part) SG_CHECK_HIP(hipDeviceSynchronize());
    dev_free(m->part);
    dev_free(m->loss_part);
    m->part = nullptr;
    m->loss_part = nullptr;
    m->part_rows = 0;
    sgrid_status s = dev_alloc((void **)&m->part, (size_t)rows * kNParam * 4, "MLP partial gradients");
    if (s != SGRID_OK) return s;
    s = dev_alloc((void **)&m->loss_part, (size_t)rows * 4, "MLP partial losses");
    if (s != SGRID_OK) return s;
    m->part_rows = rows;
    return SGRID_OK;
}

sgrid_status mlp_ensure_fallback(sgrid_mlp *m, int64_t cells) {
    if (cells <= m->fallback_cap) return SGRID_OK;
    if (m->fallback) SG_CHECK_HIP(hipDeviceSynchronize());
    dev_free(m->fallback);
    m->fallback = nullptr;
    m->fallback_cap = 0;
    sgrid_status s = dev_alloc((void **)&m->fallback, (size_t)(cells + 1) * 4, "fallback list");
    if (s != SGRID_OK) return s;
    m->fallback_cap = cells;
    return SGRID_OK;
}

static sgrid_status run_backward(sgrid_mlp *m, const float *x, int64_t B, const float *t, const float *dy,
                                 const float lw[4], hipStream_t st) {
    const int64_t nwg = (B + kTrainRows - 1) / kTrainRows;
    sgrid_status s = ensure_part(m, nwg);
    if (s != SGRID_OK) return s;
    hipLaunchKernelGGL(train_kernel, dim3((unsigned)nwg), dim3(256), 0, st, m->dev(), x, B, t, dy,
                       make_float4(lw[0], lw[1], lw[2], lw[3]), m->part, m->loss_part);
    SG_CHECK_LAUNCH("MLP train kernel");
    hipLaunchKernelGGL(reduce_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, st, m->part, (int)nwg, m->grad,
                       m->loss_part, m->loss);
    SG_CHECK_LAUNCH("MLP gradient reduction");
    return SGRID_OK;
}

}  // namespace sgrid

extern "C" sgrid_status sgrid_mlp_create(const float *params_host, sgrid_mlp **out) {
    sgrid::clear_error();
    SG_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    SG_REQUIRE(params_host != nullptr, "params is NULL");
    sgrid_mlp *m = new sgrid_mlp();
    if (hipGetDevice(&m->device) != hipSuccess ||
        hipEventCreateWithFlags(&m->done, hipEventDisableTiming) != hipSuccess) {
        sgrid::set_error("MLP setup: no device or event");
        sgrid::free_mlp(m);
        return SGRID_E_HIP;
    }
    struct A { void **p; size_t bytes; };
    A allocs[] = {{(void **)&m->w, kNParam * 4}, {(void **)&m->m, kNParam * 4}, {(void **)&m->v, kNParam * 4},
                  {(void **)&m->grad, kNParam * 4}, {(void **)&m->loss, 4},
                  {(void **)&m->w1b, kH * kInPad * 2}, {(void **)&m->w2b, kH * kH * 2},
                  {(void **)&m->w2tb, kH * kH * 2}, {(void **)&m->w3b, 16 * kH * 2}};
    for (auto &a : allocs) {
        sgrid_status s = sgrid::dev_alloc(a.p, a.bytes, "MLP parameters");
        if (s != SGRID_OK) { sgrid::free_mlp(m); return s; }
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(m->w, params_host, kNParam * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->m, 0, kNParam * 4);
    if (e == hipSuccess) e = hipMemset(m->v, 0, kNParam * 4);
    if (e == hipSuccess) e = hipMemset(m->w1b, 0, kH * kInPad * 2);
    if (e == hipSuccess) e = hipMemset(m->w3b, 0, 16 * kH * 2);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(sync_copies_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, nullptr, m->w, m->w1b,
                           m->w2b, m->w2tb, m->w3b);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        sgrid::set_error("MLP setup failed: %s", hipGetErrorString(e));
        sgrid::free_mlp(m);
        return SGRID_E_HIP;
    }
    *out = m;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_mlp_destroy(sgrid_mlp *m) {
    sgrid::clear_error();
    if (!m) return SGRID_OK;
    hipError_t e = hipDeviceSynchronize();
    sgrid::free_mlp(m);
    if (e != hipSuccess) {
        sgrid::set_error("hipDeviceSynchronize before destroy failed: %s", hipGetErrorString(e));
        return SGRID_E_HIP;
    }
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_mlp_get_params(const sgrid_mlp *m, float *params_host, float *adam_m_host,
                                             float *adam_v_host, int64_t *step) {
    sgrid::clear_error();
    SG_REQUIRE(m != nullptr, "model is NULL");
    SG_CHECK_HIP(hipDeviceSynchronize());
    if (params_host) SG_CHECK_HIP(hipMemcpy(params_host, m->w, kNParam * 4, hipMemcpyDeviceToHost));
    if (adam_m_host) SG_CHECK_HIP(hipMemcpy(adam_m_host, m->m, kNParam * 4, hipMemcpyDeviceToHost));
    if (adam_v_host) SG_CHECK_HIP(hipMemcpy(adam_v_host, m->v, kNParam * 4, hipMemcpyDeviceToHost));
    if (step) *step = m->step;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_mlp_set_state(sgrid_mlp *m, const float *adam_m_host, const float *adam_v_host,
                                            int64_t step) {
    sgrid::clear_error();
    SG_REQUIRE(m != nullptr && adam_m_host != nullptr && adam_v_host != nullptr, "NULL argument");
    SG_REQUIRE(step >= 0, "step must be >= 0");
    SG_CHECK_HIP(hipDeviceSynchronize());
    SG_CHECK_HIP(hipMemcpy(m->m, adam_m_host, kNParam * 4, hipMemcpyHostToDevice));
    SG_CHECK_HIP(hipMemcpy(m->v, adam_v_host, kNParam * 4, hipMemcpyHostToDevice));
    m->step = step;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_mlp_set_gate(sgrid_mlp *m, float tau, float kw_lo, float kw_hi) {
    sgrid::clear_error();
    SG_REQUIRE(m != nullptr, "model is NULL");
    SG_REQUIRE(tau >= 0.f && kw_lo <= kw_hi, "gate needs tau >= 0 and kw_lo <= kw_hi");
    m->gate_tau = tau;
    m->kw_lo = kw_lo;
    m->kw_hi = kw_hi;
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_mlp_forward(const sgrid_mlp *m, const float *x, int64_t B, float *y, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(m != nullptr, "model is NULL");
    SG_REQUIRE(B >= 0, "B must be >= 0");
    if (B == 0) return SGRID_OK;
    SG_REQUIRE(x && y && sg_aligned(x, 16) && sg_aligned(y, 16), "x / y NULL or not 16-byte aligned");
    const int64_t nwg = (B + 63) / 64;
    SG_REQUIRE(nwg <= kMaxGrid, "batch too large");
    hipStream_t st = sg_stream(stream);
    sgrid_status s = sgrid::begin_use(m, st);
    if (s != SGRID_OK) return s;
    hipLaunchKernelGGL(forward_kernel, dim3((unsigned)nwg), dim3(256), 0, st, m->dev(), x, B, y);
    SG_CHECK_LAUNCH("MLP forward");
    return sgrid::end_use(m, st);
}

extern "C" sgrid_status sgrid_mlp_backward(sgrid_mlp *m, const float *x, const float *dy, int64_t B, float *grad,
                                           void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(m != nullptr, "model is NULL");
    SG_REQUIRE(B >= 1, "B must be >= 1");
    SG_REQUIRE(x && dy && grad && sg_aligned(x, 16) && sg_aligned(dy, 16) && sg_aligned(grad, 4),
               "x / dy / grad NULL or misaligned");
    SG_REQUIRE((B + kTrainRows - 1) / kTrainRows <= kMaxGrid, "batch too large");
    hipStream_t st = sg_stream(stream);
    sgrid_status s = sgrid::begin_use(m, st);
    if (s != SGRID_OK) return s;
    const float lw[4] = {0, 0, 0, 0};
    s = sgrid::run_backward(m, x, B, nullptr, dy, lw, st);
    if (s != SGRID_OK) return s;
    SG_CHECK_HIP(hipMemcpyAsync(grad, m->grad, kNParam * 4, hipMemcpyDeviceToDevice, st));
    return sgrid::end_use(m, st);
}

namespace sgrid {

// One Adam step on the model's masters from the gradient in `g` (device,
// kNParam values), then the BF16 copies.  The decay rates are the FP32
// numbers nearest 0.9 and 0.999, and the bias corrections 1 - beta^t use
// those same numbers, so the step is Adam with these rates.
static sgrid_status adam_step(sgrid_mlp *m, const float *g, float lr, hipStream_t st) {
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - pow((double)b1, (double)m->step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)m->step));
    hipLaunchKernelGGL(adam_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, st, m->w, m->m, m->v, g, lr,
                       b1, b2, 1e-8f, c1, c2, m->w1b, m->w2b, m->w2tb, m->w3b);
    SG_CHECK_LAUNCH("Adam");
    return SGRID_OK;
}

}  // namespace sgrid

extern "C" sgrid_status sgrid_mlp_train_step(sgrid_mlp *m, const float *x, const float *t, int64_t B,
                                             const float *loss_weights, float lr, float *loss_dev, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(m != nullptr, "model is NULL");
    SG_REQUIRE(B >= 1, "B must be >= 1");
    SG_REQUIRE(x && t && loss_weights && sg_aligned(x, 16) && sg_aligned(t, 16), "x / t / weights NULL or misaligned");
    SG_REQUIRE(lr >= 0.f, "lr must be >= 0");
    SG_REQUIRE((B + kTrainRows - 1) / kTrainRows <= kMaxGrid, "batch too large");
    hipStream_t st = sg_stream(stream);
    sgrid_status s = sgrid::begin_use(m, st);
    if (s != SGRID_OK) return s;
    s = sgrid::run_backward(m, x, B, t, nullptr, loss_weights, st);
    if (s != SGRID_OK) return s;
    s = sgrid::adam_step(m, m->grad, lr, st);
    if (s != SGRID_OK) return s;
    if (loss_dev) SG_CHECK_HIP(hipMemcpyAsync(loss_dev, m->loss, 4, hipMemcpyDeviceToDevice, st));
    return sgrid::end_use(m, st);
}

extern "C" sgrid_status sgrid_mlp_apply_gradient(sgrid_mlp *m, const float *grad_dev, float lr, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(m != nullptr, "model is NULL");
    SG_REQUIRE(grad_dev != nullptr && sg_aligned(grad_dev, 4), "grad NULL or misaligned");
    SG_REQUIRE(lr >= 0.f, "lr must be >= 0");
    hipStream_t st = sg_stream(stream);
    sgrid_status s = sgrid::begin_use(m, st);
    if (s != SGRID_OK) return s;
    s = sgrid::adam_step(m, grad_dev, lr, st);
    if (s != SGRID_OK) return s;
    return sgrid::end_use(m, st);
}

// ---------------------------------------------------------------------------
// Learned near-surface integrals with gate and plain fallback
// ---------------------------------------------------------------------------
namespace {

using sgrid::kWin;                     // phi window of a package, local -2..6
using sgrid::kWinN;
constexpr int kVol = 7, kVolN = 343;   // points -1..5 whose cut fraction a tap may use

// Stages the 9^3 phi window of core package p into LDS (all threads of the block).
__device__ __forceinline__ void stage_window(const float *__restrict__ phi, const uint32_t *__restrict__ nbr,
                                             int64_t p, float *s_phi, uint32_t *s_ids) {
    if (threadIdx.x < 27) s_ids[threadIdx.x] = nbr[p * 27 + threadIdx.x];
    __syncthreads();
    sgrid::stage_window_part<256>(phi, s_ids, threadIdx.x, s_phi);
    __syncthreads();
}

// Network input of cell c (local index i + 4j + 16k) from the staged window.
struct WindowX {
    const float *f;
    int cell0;
    float inv_h;
    __device__ __forceinline__ void operator()(int m, int k0, float *v) const {
        const int c = cell0 + m;
        const int i = c & 3, j = (c >> 2) & 3, k = c >> 4;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int kk = k0 + e;
            if (kk < kIn) {
                const int ox = kk % 6, oy = (kk / 6) % 6, oz = kk / 36;   // offset + 2
                v[e] = f[(i + ox) + kWin * ((j + oy) + kWin * (k + oz))] * inv_h;
            } else {
                v[e] = 0.f;
            }
        }
    }
};

// Saturation of the cut fraction at the 7^3 tap points: bit 0 = V in {0, 1}
// (fraction_saturated), bit 1 = phi > 0.
__device__ __forceinline__ void saturation_flags(const float *f, float inv_h, float inv_2h, uint8_t *s_sat) {
    for (int v = threadIdx.x; v < kVolN; v += blockDim.x) {
        const int x = v % kVol + 1, y = (v / kVol) % kVol + 1, z = v / (kVol * kVol) + 1;
        const int c = x + kWin * (y + kWin * z);
        const float gx = (f[c + 1] - f[c - 1]) * inv_2h;
        const float gy = (f[c + kWin] - f[c - kWin]) * inv_2h;
        const float gz = (f[c + kWin * kWin] - f[c - kWin * kWin]) * inv_2h;
        const float a = f[c] * inv_h;
        const bool sat = sgrid::fraction_saturated(a, gx, gy, gz);
        s_sat[v] = (uint8_t)((sat ? 1 : 0) | (a > 0.f ? 2 : 0));
    }
}

__global__ __launch_bounds__(256) void zero_u32_kernel(uint32_t *p) { *p = 0u; }
__global__ __launch_bounds__(64) void add_u32_kernel(uint32_t *total, const uint32_t *part) { *total += *part; }

// Learned-integral kernel: two core packages (128 points) per workgroup of
// four wavefronts.
//  1. Each package's 128 lanes stage its 9^3 window, the saturation flags of
//     the 7^3 tap points and the BF16 hi + lo parts of the network inputs.
//  2. One lane per point sums the 32 taps' saturated fractions.  A point
//     whose taps are all saturated takes that exact sum (the plain value);
//     the others are listed, in LDS, for the network.
//  3. The listed points are spread in 16-point tiles over the wavefronts,
//     tile T on wavefront T mod 4, and each wavefront evaluates the gate of
//     its tiles' points, two lanes per point.
//  4. The network over the tiles: W1's and W2's 32-input slices are staged
//     in LDS once per workgroup (every wavefront takes part in the staging
//     and its barriers) and each weight fragment feeds both of a wavefront's
//     tiles, hi and lo parts.  A wavefront reads back only activation rows it
//     wrote.
//  5. The same wavefront writes the network's value or lists the point for
//     the plain fallback.
// Every listed point's network row is computed in the MFMA accumulation
// order of forward_tile, so the outputs are the bits of sgrid_mlp_forward on
// the gathered windows.
constexpr int kLearnPkgs = 2;   // packages per workgroup
constexpr int kLearnPts = 64 * kLearnPkgs;
constexpr int kActStride = kH + 8;   // bf16 per activation row in LDS

struct LearnLds {
    float phi[kWinN + 3];
    uint32_t xhl[kWinN + 3];   // BF16 hi (low half) and lo (high half) parts of the window's phi / h
    uint32_t ids[28];
    uint8_t sat[kVolN + 13];
};

// The weights of layers 1 and 2 pass through LDS, one 32-input slice (128
// rows x 32 BF16, 8 KB) per step, so the workgroup's four wavefronts read each
// slice from L2 once instead of four times.  W1's slices are double-buffered
// in the activation area (free until layer 1 ends); W2's go, one at a time,
// where the windows were (free once every wavefront has evaluated its gate
// and passed layer 1).  Rows are padded to kWRow BF16.
constexpr int kWRow = 40;
constexpr int kWSlice = kH * kWRow;   // BF16 per buffered slice
constexpr int kW1Steps = kInPad / 32, kW2Steps = kH / 32;

// Thread tid's share of slice s of a [128][row_len] weight matrix: row
// tid / 2, inputs 32 s + 16 (tid % 2) .. + 15.
struct WPart {
    bf16x8 a, b;
};
__device__ __forceinline__ WPart w_load(const bf16 *w, int row_len, int s, int tid) {
    const bf16 *src = w + (tid >> 1) * row_len + 32 * s + 16 * (tid & 1);
    return WPart{ld8(src), ld8(src + 8)};
}
__device__ __forceinline__ void w_store(bf16 *buf, const WPart &v, int tid) {
    bf16 *dst = buf + (tid >> 1) * kWRow + 16 * (tid & 1);
    *reinterpret_cast<bf16x8 *>(dst) = v.a;
    *reinterpret_cast<bf16x8 *>(dst + 8) = v.b;
}

// The network over the listed points of TILES tiles (rows 16 tile + r of the
// list): layer outputs through the wavefront's own activation rows, the
// outputs y to s_y[row][4].  Every wavefront of the workgroup calls it (TILES
// = 0 for one without tiles: it helps stage the weights and meets the
// barriers), after its gate.
template <int TILES>
__device__ __forceinline__ void learned_network(const MlpDev &W, LearnLds *lds, const int16_t *s_off,
                                                const uint8_t *s_list, int n_list, const int tile[2], bf16 *s_act,
                                                float *s_y, int lane) {
    const int r = lane & 15, q = lane >> 4, tid = threadIdx.x;
    constexpr int NT = TILES > 0 ? TILES : 1;
    int base[NT];
    const LearnLds *win[NT];
#pragma unroll
    for (int m = 0; m < TILES; ++m) {
        const int row = 16 * tile[m] + r;
        const int pt = s_list[row < n_list ? row : n_list - 1];   // rows past the list repeat its last point
        const int c = pt & 63;
        win[m] = lds + (pt >> 6);
        base[m] = (c & 3) + kWin * (((c >> 2) & 3) + kWin * (c >> 4));
    }
    // layer 1: [16 x 224] (hi + lo BF16 parts of phi / h) x W1^T per tile;
    // accumulators start from the biases, as in forward_tile
    floatx4 acc[NT][8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const float bb = W.w[oB1 + 16 * t + r];
#pragma unroll
        for (int m = 0; m < TILES; ++m) acc[m][t] = floatx4{bb, bb, bb, bb};
    }
    // slice s + 1 is stored at the start of step s (its buffer was last read in
    // step s - 1, which ended with a barrier) and slice s + 2 loads meanwhile
    WPart part = w_load(W.w1b, kInPad, 0, tid);
    w_store(s_act, part, tid);
    part = w_load(W.w1b, kInPad, 1, tid);
    __syncthreads();
    for (int s = 0; s < kW1Steps; ++s) {
        if (s + 1 < kW1Steps) {
            w_store(s_act + ((s + 1) & 1) * kWSlice, part, tid);
            if (s + 2 < kW1Steps) part = w_load(W.w1b, kInPad, s + 2, tid);
        }
        if (TILES > 0) {
            const bf16 *wb = s_act + (s & 1) * kWSlice;
            bf16x8 bw[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) bw[t] = ld8(wb + (16 * t + r) * kWRow + 8 * q);
#pragma unroll
            for (int m = 0; m < TILES; ++m) {
                bf16x8 ah, al;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int off = base[m] + s_off[32 * s + 8 * q + e];
                    const uint32_t hl = win[m]->xhl[off];   // both parts in one read
                    ah[e] = __builtin_bit_cast(bf16, (uint16_t)(hl & 0xFFFFu));
                    al[e] = __builtin_bit_cast(bf16, (uint16_t)(hl >> 16));
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    acc[m][t] = mfma(ah, bw[t], acc[m][t]);
                    acc[m][t] = mfma(al, bw[t], acc[m][t]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int m = 0; m < TILES; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                s_act[(16 * tile[m] + 4 * q + i) * kActStride + 16 * t + r] = (bf16)gelu(acc[m][t][i]);
    // layer 2, W2's slices one at a time in the windows' LDS (a wavefront
    // reads back only activation rows it wrote itself)
    static_assert(sizeof(LearnLds) * kLearnPkgs >= kWSlice * sizeof(bf16), "W2 slice buffer");
    bf16 *w2buf = reinterpret_cast<bf16 *>(lds);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const float bb = W.w[oB2 + 16 * t + r];
#pragma unroll
        for (int m = 0; m < TILES; ++m) acc[m][t] = floatx4{bb, bb, bb, bb};
    }
    part = w_load(W.w2b, kH, 0, tid);
    for (int s = 0; s < kW2Steps; ++s) {
        w_store(w2buf, part, tid);
        if (s + 1 < kW2Steps) part = w_load(W.w2b, kH, s + 1, tid);
        __syncthreads();
        if (TILES > 0) {
            bf16x8 bv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) bv[t] = ld8(w2buf + (16 * t + r) * kWRow + 8 * q);
#pragma unroll
            for (int m = 0; m < TILES; ++m) {
                const bf16x8 a = ld8(s_act + (16 * tile[m] + r) * kActStride + 32 * s + 8 * q);
#pragma unroll
                for (int t = 0; t < 8; ++t) acc[m][t] = mfma(a, bv[t], acc[m][t]);
            }
        }
        __syncthreads();
    }
    if (TILES == 0) return;
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int m = 0; m < TILES; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                s_act[(16 * tile[m] + 4 * q + i) * kActStride + 16 * t + r] = (bf16)gelu(acc[m][t][i]);
    // layer 3
    floatx4 y[NT];
    const float b3 = r < kOut ? W.w[oB3 + r] : 0.f;
#pragma unroll
    for (int m = 0; m < TILES; ++m) y[m] = floatx4{b3, b3, b3, b3};
#pragma unroll
    for (int s = 0; s < kH / 32; ++s) {
        const bf16x8 w3 = ld8(W.w3b + r * kH + 32 * s + 8 * q);
#pragma unroll
        for (int m = 0; m < TILES; ++m)
            y[m] = mfma(ld8(s_act + (16 * tile[m] + r) * kActStride + 32 * s + 8 * q), w3, y[m]);
    }
    if (r < kOut) {
#pragma unroll
        for (int m = 0; m < TILES; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) s_y[(16 * tile[m] + 4 * q + i) * kOut + r] = y[m][i];
    }
}

__global__ __launch_bounds__(256, 3) void learned_kernel(MlpDev W, const float *__restrict__ phi,
                                                         const uint32_t *__restrict__ nbr,
                                                         const uint32_t *__restrict__ core_list, int64_t n_core,
                                                         int64_t ci0, int64_t ci_end, float inv_h, float inv_2h,
                                                         float tau, float kw_lo, float kw_hi,
                                                         float *__restrict__ out, uint32_t *__restrict__ fb_list,
                                                         uint32_t *__restrict__ fb_count) {
    __shared__ __attribute__((aligned(16))) LearnLds lds[kLearnPkgs];   // 16-byte rows of W2 go here later
    // window offset of network input kk (ox + 9 oy + 81 oz); the padding
    // inputs 216..223 meet zero columns of W1, so they read any finite window
    // value (offset 0) and add exactly zero, without a branch per input
    __shared__ int16_t s_off[kInPad];
    __shared__ __attribute__((aligned(16))) bf16 s_act[kLearnPts * kActStride];   // rows padded by 16 bytes
    __shared__ float s_y[kLearnPts * kOut];
    __shared__ uint8_t s_list[kLearnPts];   // listed points: slot * 64 + local index
    __shared__ uint32_t s_n;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < kInPad) {
        const int kk = threadIdx.x;
        s_off[kk] = kk < kIn ? (int16_t)(kk % 6 + kWin * ((kk / 6) % 6) + kWin * kWin * (kk / 36)) : (int16_t)0;
    }
    if (threadIdx.x == 0) s_n = 0u;
    // 1. staging, per package: 128 lanes each
    const int slot = w >> 1, t128 = threadIdx.x & 127;
    LearnLds &L = lds[slot];
    // core packages [ci0, ci_end) of the n_core (outputs are indexed over all)
    const int64_t cw = ci0 + (int64_t)blockIdx.x * kLearnPkgs + slot;
    const bool live = cw < ci_end;                 // a package slot past the end repeats the last package
    const int64_t ci = live ? cw : ci_end - 1;
    const int64_t p = core_list[ci];
    if (t128 < 27) L.ids[t128] = nbr[p * 27 + t128];
    __syncthreads();
    sgrid::stage_window_part<128>(phi, L.ids, t128, L.phi);
    __syncthreads();
    for (int v = t128; v < kVolN; v += 128) {
        const int x = v % kVol + 1, y = (v / kVol) % kVol + 1, z = v / (kVol * kVol) + 1;
        const int c = x + kWin * (y + kWin * z);
        const float gx = (L.phi[c + 1] - L.phi[c - 1]) * inv_2h;
        const float gy = (L.phi[c + kWin] - L.phi[c - kWin]) * inv_2h;
        const float gz = (L.phi[c + kWin * kWin] - L.phi[c - kWin * kWin]) * inv_2h;
        const float a = L.phi[c] * inv_h;
        const bool sat = sgrid::fraction_saturated(a, gx, gy, gz);
        L.sat[v] = (uint8_t)((sat ? 1 : 0) | (a > 0.f ? 2 : 0));
    }
    for (int v = t128; v < kWinN; v += 128) {   // the network inputs, once per window value
        const float x = L.phi[v] * inv_h;
        const bf16 hi = (bf16)x;
        const bf16 lo = (bf16)(x - (float)hi);
        L.xhl[v] = (uint32_t)__builtin_bit_cast(uint16_t, hi) | ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
    }
    __syncthreads();
    const int64_t stride = n_core * 64;
    // 2. saturated points: one lane per point (the first 64 of each
    // package's 128) sums its 32 taps' fractions, 1 or 0 by the sign of phi,
    // with the plain kernels' tap sums, so the value is the plain one bit for
    // bit; a point with a cut tap is listed
    if (t128 < 64) {
        const int c = t128;
        bool sat = true;
        float kw, kx, ky, kz;
        sgrid::tap_sums(
            [&](int x, int y, int z) {
                const uint8_t f = L.sat[(x + 1) + kVol * ((y + 1) + kVol * (z + 1))];
                sat = sat && (f & 1);
                return (f & 2) ? 1.f : 0.f;
            },
            c & 3, (c >> 2) & 3, c >> 4, kw, kx, ky, kz);
        if (live) {
            if (sat) {
                const int64_t o = ci * 64 + c;
                out[o] = kw;
                out[stride + o] = kx;
                out[2 * stride + o] = ky;
                out[3 * stride + o] = kz;
            } else {
                s_list[atomicAdd(&s_n, 1u)] = (uint8_t)(slot * 64 + c);
            }
        }
    }
    __syncthreads();
    const int n_list = (int)s_n;
    const int n_tiles = (n_list + 15) / 16;
    const int tile[2] = {w, w + 4};
    const int mine = (w < n_tiles ? 1 : 0) + (w + 4 < n_tiles ? 1 : 0);
    if (n_tiles == 0) return;   // the same for the whole workgroup
    // 3. the gate of this wavefront's points, two lanes per point: lanes
    // 0..31 the rows of tile w, lanes 32..63 those of tile w + 4 (before the
    // network, whose second layer reuses the windows' LDS).
    // Non-planarity: mean squared residual of the window after its
    // least-squares affine fit.  The basis 1, ox, oy, oz (offsets centred at
    // 2.5) is orthogonal on the window, so the fit's coefficients are the
    // moments s0 / 216 and s_a / 630.  The residual is then summed over the
    // window a second time, explicitly: the closed form s2 - 216 c0^2 -
    // 630 |c|^2 subtracts nearly equal numbers for the near-planar windows the
    // gate has to tell apart.  An error in the coefficients only moves the sum
    // at second order (the residual is orthogonal to the basis).  Both passes
    // sum phi itself and apply 1/h to the result (for h a power of two the
    // bits of summing phi / h).  Lane `part` takes the window rows 2i + part
    // of the 36 (ez = 2i / 6 for both parities, 6 being even, ey = 2i % 6 +
    // part).
    const int row = 16 * tile[lane >> 5] + ((lane >> 1) & 15), part = lane & 1;
    const bool valid = row < n_list;
    const int pt = s_list[valid ? row : n_list - 1];
    const LearnLds &Lp = lds[pt >> 6];
    const int c = pt & 63;
    const int ci_ = c & 3, cj = (c >> 2) & 3, ck = c >> 4;
    // (per window row: its sum and its x moment, then the row's share of the
    // y and z moments from its sum; a wavefront without points skips both
    // passes)
    const int n_rows = mine > 0 ? 18 : 0;
    float s0 = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll 1
    for (int i = 0; i < n_rows; ++i) {
        const int ez = (2 * i) / 6, ey = (2 * i) % 6 + part;
        const float *wrow = Lp.phi + ci_ + kWin * ((cj + ey) + kWin * (ck + ez));
        float v[6];
#pragma unroll
        for (int ex = 0; ex < 6; ++ex) v[ex] = wrow[ex];
        const float r0 = ((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5]);
        const float rx = 2.5f * (v[5] - v[0]) + (1.5f * (v[4] - v[1]) + 0.5f * (v[3] - v[2]));
        s0 += r0;
        sx += rx;
        sy += (ey - 2.5f) * r0;
        sz += (ez - 2.5f) * r0;
    }
    s0 += __shfl_xor(s0, 1);
    sx += __shfl_xor(sx, 1);
    sy += __shfl_xor(sy, 1);
    sz += __shfl_xor(sz, 1);
    const float c0 = s0 / 216.f, cx = sx / 630.f, cy = sy / 630.f, cz = sz / 630.f;   // units of phi
    float rr = 0.f;
#pragma unroll 1
    for (int i = 0; i < n_rows; ++i) {
        const int ez = (2 * i) / 6, ey = (2 * i) % 6 + part;
        const float *wrow = Lp.phi + ci_ + kWin * ((cj + ey) + kWin * (ck + ez));
        const float pyz = c0 + cy * (ey - 2.5f) + cz * (ez - 2.5f);
#pragma unroll
        for (int ex = 0; ex < 6; ++ex) {
            const float e = wrow[ex] - (pyz + cx * (ex - 2.5f));
            rr += e * e;
        }
    }
    rr += __shfl_xor(rr, 1);
    const float res = rr * inv_h * inv_h * (1.0f / 216.f);
    // 4. the network over this wavefront's tiles (every wavefront takes part)
    if (mine == 2)
        learned_network<2>(W, lds, s_off, s_list, n_list, tile, s_act, s_y, lane);
    else if (mine == 1)
        learned_network<1>(W, lds, s_off, s_list, n_list, tile, s_act, s_y, lane);
    else
        learned_network<0>(W, lds, s_off, s_list, n_list, tile, s_act, s_y, lane);
    if (mine == 0) return;
    // 5. the network's value or the fallback list (the point's row and list
    // entry read again rather than kept across the network)
    const int row_o = 16 * tile[lane >> 5] + ((lane >> 1) & 15);
    if (row_o < n_list && (lane & 1) == 0) {
        const int pt_o = s_list[row_o];
        const int64_t o = (ci0 + (int64_t)blockIdx.x * kLearnPkgs + (pt_o >> 6)) * 64 + (pt_o & 63);
        const float *yv = s_y + row_o * kOut;
        if (res <= tau && yv[0] >= kw_lo && yv[0] <= kw_hi) {
            out[o] = yv[0];
            out[stride + o] = yv[1];
            out[2 * stride + o] = yv[2];
            out[3 * stride + o] = yv[3];
        } else {
            fb_list[atomicAdd(fb_count, 1u)] = (uint32_t)o;
        }
    }
}

// Plain integral of single cells (the fallback): the 32 taps of the cell's
// dual-cell query, each with its own cut fraction from central differences,
// with the plain kernels' fractions and tap sums, so the value is the plain
// one bit for bit.
__device__ __forceinline__ void fallback_point(const float *__restrict__ phi, const uint32_t *__restrict__ nbr,
                                               const uint32_t *__restrict__ core_list, int64_t n_core, float inv_h,
                                               float inv_2h, int64_t o, float *__restrict__ out) {
    const int64_t ci = o / 64;
    const int c = (int)(o % 64);
    const uint32_t *row = nbr + (int64_t)core_list[ci] * 27;
    auto at = [&](int x, int y, int z) -> float {   // local shift in [-2, 6] per axis
        const int kx = (x + 4) >> 2, ky = (y + 4) >> 2, kz = (z + 4) >> 2;
        const int d = (x + 4 - 4 * kx) + 4 * (y + 4 - 4 * ky) + 16 * (z + 4 - 4 * kz);
        return phi[(int64_t)row[kx + 3 * ky + 9 * kz] * 64 + d];
    };
    float kw, kx, ky, kz;
    sgrid::tap_sums(
        [&](int x, int y, int z) {
            const float gx = (at(x + 1, y, z) - at(x - 1, y, z)) * inv_2h;
            const float gy = (at(x, y + 1, z) - at(x, y - 1, z)) * inv_2h;
            const float gz = (at(x, y, z + 1) - at(x, y, z - 1)) * inv_2h;
            return sgrid::plane_cube_fraction(at(x, y, z) * inv_h, gx, gy, gz);
        },
        c & 3, (c >> 2) & 3, c >> 4, kw, kx, ky, kz);
    const int64_t stride = n_core * 64;
    out[o] = kw;
    out[stride + o] = kx;
    out[2 * stride + o] = ky;
    out[3 * stride + o] = kz;
}

// The listed points, `*fb_count` of them, read on the device: a persistent
// grid strides over the list, so its size need not be known at launch.
__global__ __launch_bounds__(256) void fallback_kernel(const float *__restrict__ phi, const uint32_t *__restrict__ nbr,
                                                       const uint32_t *__restrict__ core_list, int64_t n_core,
                                                       float inv_h, float inv_2h, const uint32_t *__restrict__ fb_list,
                                                       const uint32_t *__restrict__ fb_count, float *__restrict__ out) {
    const int64_t count = *fb_count;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        fallback_point(phi, nbr, core_list, n_core, inv_h, inv_2h, fb_list[t], out);
}

// Network inputs (windows of phi / h) and saturation of every core point, in
// the output order of the integrals.  unsat[o] = 1 when some tap fraction lies
// strictly between 0 and 1.
__global__ __launch_bounds__(256) void gather_windows_kernel(const float *__restrict__ phi,
                                                             const uint32_t *__restrict__ nbr,
                                                             const uint32_t *__restrict__ core_list, float inv_h,
                                                             float inv_2h, float *__restrict__ x,
                                                             uint8_t *__restrict__ unsat) {
    __shared__ float s_phi[kWinN];
    __shared__ uint32_t s_ids[27];
    __shared__ uint8_t s_sat[kVolN];
    const int64_t ci = blockIdx.x;
    stage_window(phi, nbr, core_list[ci], s_phi, s_ids);
    saturation_flags(s_phi, inv_h, inv_2h, s_sat);
    __syncthreads();
    if (x) {
        for (int e = threadIdx.x; e < 64 * kIn; e += blockDim.x) {
            const int c = e / kIn, kk = e % kIn;
            const int i = c & 3, j = (c >> 2) & 3, k = c >> 4;
            const int ox = kk % 6, oy = (kk / 6) % 6, oz = kk / 36;
            x[(ci * 64 + c) * kIn + kk] = s_phi[(i + ox) + kWin * ((j + oy) + kWin * (k + oz))] * inv_h;
        }
    }
    if (unsat && threadIdx.x < 64) {
        const int c = threadIdx.x;
        const int i = c & 3, j = (c >> 2) & 3, k = c >> 4;
        bool all = true;
        for (int oz = -1; oz <= 2; ++oz)
            for (int oy = -1; oy <= 2; ++oy)
                for (int ox = -1; ox <= 2; ++ox) {
                    const float dx = 0.5f - ox, dy = 0.5f - oy, dz = 0.5f - oz;
                    if (dx * dx + dy * dy + dz * dz >= 4.0f) continue;
                    all = all && (s_sat[(i + ox + 1) + kVol * ((j + oy + 1) + kVol * (k + oz + 1))] & 1);
                }
        unsat[ci * 64 + c] = all ? 0 : 1;
    }
}

}  // namespace

namespace sgrid {

// Gate + network over the core packages [ci0, ci_end), then the plain
// fallback over the listed points.  `fb_list` holds (ci_end - ci0) * 64
// entries; `count` is reset here.  The fallback grid is a persistent one of at
// most four workgroups per compute unit striding over the device-side count,
// so a launch costs little when few points fall back.
static sgrid_status learned_launch(const sgrid_grid *g, const float *phi, const sgrid_mlp *m, float *out,
                                   uint32_t *fb_list, uint32_t *count, int64_t ci0, int64_t ci_end, hipStream_t st) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, count);
    SG_CHECK_LAUNCH("fallback counter reset");
    if (ci_end <= ci0) return SGRID_OK;
    const int64_t cells = (ci_end - ci0) * 64;
    const float inv_h = (float)(1.0 / g->h), inv_2h = (float)(0.5 / g->h);
    hipLaunchKernelGGL(learned_kernel, dim3((unsigned)((ci_end - ci0 + kLearnPkgs - 1) / kLearnPkgs)), dim3(256), 0,
                       st, m->dev(), phi, g->nbr, g->core_list, g->n_core, ci0, ci_end, inv_h, inv_2h, m->gate_tau,
                       m->kw_lo, m->kw_hi, out, fb_list, count);
    SG_CHECK_LAUNCH("learned integrals");
    const int64_t fb_blocks = std::min<int64_t>((cells + 255) / 256, 4 * (int64_t)cu_count());
    hipLaunchKernelGGL(fallback_kernel, dim3((unsigned)fb_blocks), dim3(256), 0, st, phi, g->nbr, g->core_list,
                       g->n_core, inv_h, inv_2h, fb_list, count, out);
    SG_CHECK_LAUNCH("fallback integrals");
    return SGRID_OK;
}

sgrid_status integrals_learned(const sgrid_grid *g, const float *phi, const sgrid_mlp *model_c, float *out,
                               uint32_t *n_fallback, hipStream_t st) {
    sgrid_mlp *m = const_cast<sgrid_mlp *>(model_c);
    const int64_t cells = g->n_core * 64;
    SG_REQUIRE(g->n_core <= kMaxGrid, "too many core packages");
    sgrid_status s = mlp_ensure_fallback(m, cells);
    if (s != SGRID_OK) return s;
    s = begin_use(m, st);
    if (s != SGRID_OK) return s;
    uint32_t *count = n_fallback ? n_fallback : m->fallback + m->fallback_cap;
    s = learned_launch(g, phi, m, out, m->fallback, count, 0, g->n_core, st);
    if (s != SGRID_OK) return s;
    return end_use(m, st);
}

}  // namespace sgrid

// ---------------------------------------------------------------------------
// Learned integrals without allocation
// ---------------------------------------------------------------------------
// The fallback list lives in a fixed array in every GPU's memory (8 MiB each,
// held until the process ends): two counters padded to 256 bytes, then room
// for one chunk of kNoAllocChunk core packages' points.  Host code reaches it
// only through the address hipGetSymbolAddress returns on each device.
constexpr int64_t kNoAllocChunk = 32768;
constexpr int64_t kNoAllocWords = 64 + kNoAllocChunk * 64;
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_scratch_mutex;
uint32_t *g_scratch_ptr[kNoAllocDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call there.
sgrid_status scratch_address(int dev, uint32_t **out) {
    SG_REQUIRE(dev >= 0 && dev < kNoAllocDevices, "device %d is beyond the %d devices the library tracks", dev,
               kNoAllocDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SG_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SG_REQUIRE(p != nullptr, "no device address for the fallback array on device %d", dev);
        g_scratch_ptr[dev] = static_cast<uint32_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SGRID_OK;
}

}  // namespace

extern "C" sgrid_status sgrid_compute_near_surface_integrals_noalloc(const sgrid_grid *g, const float *phi,
                                                                     const sgrid_mlp *model, float *out,
                                                                     uint32_t *n_fallback, void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr, "grid is NULL");
    SG_REQUIRE(model != nullptr, "model is NULL (the plain integrals allocate nothing: use "
                                 "sgrid_compute_near_surface_integrals)");
    SG_REQUIRE(phi != nullptr, "phi is NULL");
    SG_REQUIRE(out != nullptr || g->n_core == 0, "out is NULL");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(out, 16), "phi / out must be 16-byte aligned");
    SG_REQUIRE(g->n_core * 64 <= (int64_t)UINT32_MAX, "%lld core packages: point indices exceed 32 bits",
               (long long)g->n_core);
    int dev = 0;
    SG_CHECK_HIP(hipGetDevice(&dev));
    SG_REQUIRE(g->device == dev && model->device == dev,
               "grid (device %d) and model (device %d) must live on the current device %d", g->device,
               model->device, dev);
    uint32_t *sc = nullptr;
    sgrid_status s = scratch_address(dev, &sc);
    if (s != SGRID_OK) return s;
    hipStream_t st = sg_stream(stream);
    s = sgrid::begin_use(model, st);
    if (s != SGRID_OK) return s;
    uint32_t *chunk_count = sc, *total = n_fallback ? n_fallback : sc + 1, *list = sc + 64;
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, total);
    SG_CHECK_LAUNCH("fallback total reset");
    for (int64_t ci0 = 0; ci0 < g->n_core; ci0 += kNoAllocChunk) {
        const int64_t ci_end = std::min<int64_t>(ci0 + kNoAllocChunk, g->n_core);
        s = sgrid::learned_launch(g, phi, model, out, list, chunk_count, ci0, ci_end, st);
        if (s != SGRID_OK) return s;
        hipLaunchKernelGGL(add_u32_kernel, dim3(1), dim3(1), 0, st, total, (const uint32_t *)chunk_count);
        SG_CHECK_LAUNCH("fallback total");
    }
    return sgrid::end_use(model, st);
}

sgrid_status sgrid::launch_zero_u32(uint32_t *p, hipStream_t st) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, p);
    SG_CHECK_LAUNCH("counter reset");
    return SGRID_OK;
}

extern "C" sgrid_status sgrid_gather_windows(const sgrid_grid *g, const float *phi, float *x_dev, uint8_t *unsat_dev,
                                             void *stream) {
    sgrid::clear_error();
    SG_REQUIRE(g != nullptr && phi != nullptr, "grid or phi is NULL");
    SG_REQUIRE(sg_aligned(phi, 16) && sg_aligned(x_dev, 4), "phi / x misaligned");
    if (g->n_core == 0) return SGRID_OK;
    SG_REQUIRE(g->n_core <= kMaxGrid, "too many core packages");
    hipLaunchKernelGGL(gather_windows_kernel, dim3((unsigned)g->n_core), dim3(256), 0, sg_stream(stream), phi, g->nbr,
                       g->core_list, (float)(1.0 / g->h), (float)(0.5 / g->h), x_dev, unsat_dev);
    SG_CHECK_LAUNCH("gather windows");
    return SGRID_OK;
}

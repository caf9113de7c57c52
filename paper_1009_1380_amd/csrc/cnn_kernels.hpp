// cnn_kernels.hpp - kernels of the learned warm start: a small BF16
// convolutional encoder-decoder that maps the filtered adjoint of a sinogram
// to a start image for the basis-pursuit solve (gfx950).
//
// Activations are NCHW bfloat16; every product is accumulated in float32.
// 3x3 convolutions are implicit GEMMs on the matrix cores
// (v_mfma_f32_32x32x8_bf16): for the forward, M = output channels, N =
// pixels, K = input channels x 9 taps; a wave computes a 32 x 32 block of the
// output with one MFMA per 8 values of K. Operand layout of the instruction
// (lane l of 64, t = 0..3): A holds row l % 32, columns k = 4 (l / 32) + t;
// B holds rows k = 4 (l / 32) + t, column l % 32; the 16 results of lane l
// are rows 8 (r / 4) + 4 (l / 32) + (r % 4), column l % 32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cnn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr int CONV_NT = 256;   // 4 waves: a 64 x 64 output block (2 x 2 waves of 32 x 32)

// Implicit-GEMM 3x3 convolution, stride 1, zero padding 1.
//   out[b, co, y, x] = epilogue( sum_{ci, ky, kx} Wg[co][ci*9 + ky*3 + kx] *
//                                in[b, ci, y + ky - 1, x + kx - 1] )
// Wg is bf16 [Cout][Kp] (K = Cin*9 padded to Kp, a multiple of 8, with zeros).
// Epilogue: + bias[co] (bias may be null), ReLU if relu, + res[b, co, y, x]
// (res may be null, bf16) + res32[b, co, y, x] (may be null, float32).
// Output bf16 (out16) and/or float32 (out32).
// Grid: x = pixel blocks of 64 (over B*H*W), y = channel blocks of 64.
__global__ __launch_bounds__(CONV_NT) void k_conv3x3(const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ Wg, int Kp,
                                                    const float* __restrict__ bias, const uint16_t* __restrict__ res,
                                                    const float* __restrict__ res32,
                                                    uint16_t* __restrict__ out16, float* __restrict__ out32,
                                                    int B, int Cin, int Cout, int H, int W, int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int HW = H * W;
    const long long NP = (long long)B * HW;
    const int co0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const long long p0 = (long long)blockIdx.x * 64 + (wave & 1) * 32;
    const int i = lane & 31, kh = lane >> 5;
    // this lane's B column: pixel p0 + i
    const long long p = p0 + i;
    const bool pv = p < NP;
    const int pb = pv ? (int)(p / HW) : 0;
    const int prem = pv ? (int)(p - (long long)pb * HW) : 0;
    const int py = prem / W, px = prem - (prem / W) * W;
    const uint16_t* inb = in + (size_t)pb * Cin * HW;
    // this lane's A row: output channel co0 + i
    const int coA = co0 + i;
    const bool av = coA < Cout;
    const uint16_t* wrow = Wg + (size_t)(av ? coA : 0) * Kp;
    const int K = Cin * 9;
    f32x16 acc = {};
    for (int k0 = 0; k0 < Kp; k0 += 8) {
        bf16x4 a, b;
        const int kb = k0 + 4 * kh;
        if (av) {
            const uint2 w2 = *reinterpret_cast<const uint2*>(wrow + kb);
            a[0] = (short)(w2.x & 0xffff);
            a[1] = (short)(w2.x >> 16);
            a[2] = (short)(w2.y & 0xffff);
            a[3] = (short)(w2.y >> 16);
        } else {
            a[0] = a[1] = a[2] = a[3] = 0;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = kb + t;
            uint16_t v = 0;
            if (pv && k < K) {
                const int ci = k / 9, tap = k - (k / 9) * 9;
                const int yy = py + tap / 3 - 1, xx = px + (tap - (tap / 3) * 3) - 1;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = inb[(size_t)ci * HW + yy * W + xx];
            }
            b[t] = (short)v;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    // epilogue: lane holds column p0 + i, rows co0 + 8(r/4) + 4 kh + r%4
    if (!pv) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int co = co0 + 8 * (r >> 2) + 4 * kh + (r & 3);
        if (co >= Cout) continue;
        float v = acc[r];
        if (bias) v += bias[co];
        if (relu) v = fmaxf(v, 0.f);
        const size_t o = ((size_t)pb * Cout + co) * HW + prem;
        if (res) v += bf2f(res[o]);
        if (res32) v += res32[o];
        if (out16) out16[o] = f2bf(v);
        if (out32) out32[o] = v;
    }
}

// Weight gradient of the 3x3 convolution, split over pixel chunks:
//   part[chunk][co][k] = sum over the chunk's pixels p of
//                        g[b, co, p] * in[b, ci(k), p + tap(k)]
// (M = Cout, N = K = Cin*9, reduction over pixels); the chunks are summed in
// order by k_sum_chunks. A wave computes a 32 (co) x 32 (k) block; the
// reduction index runs over 8 pixels per MFMA. Grid: x = chunks, y = k blocks
// of 32, z = co blocks of 32 (one wave per workgroup).
constexpr int WG_CHUNK = 4096;   // pixels per chunk (a multiple of 8)

__global__ __launch_bounds__(64) void k_conv3x3_wgrad(const uint16_t* __restrict__ g,
                                                     const uint16_t* __restrict__ in, float* __restrict__ part,
                                                     int B, int Cin, int Cout, int H, int W) {
    const int lane = threadIdx.x;
    const int HW = H * W;
    const long long NP = (long long)B * HW;
    const int K = Cin * 9;
    const int i = lane & 31, kh = lane >> 5;
    const int coA = blockIdx.z * 32 + i;     // A row
    const int kB = blockIdx.y * 32 + i;      // B column
    const bool av = coA < Cout, bv = kB < K;
    const int ci = bv ? kB / 9 : 0, tap = bv ? kB - (kB / 9) * 9 : 0;
    const int dy = tap / 3 - 1, dx = tap - (tap / 3) * 3 - 1;
    const long long c0 = (long long)blockIdx.x * WG_CHUNK;
    f32x16 acc = {};
    for (int s = 0; s < WG_CHUNK; s += 8) {
        bf16x4 a, b;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const long long p = c0 + s + 4 * kh + t;
            uint16_t va = 0, vb = 0;
            if (p < NP) {
                const int pb = (int)(p / HW);
                const int prem = (int)(p - (long long)pb * HW);
                if (av) va = g[((size_t)pb * Cout + coA) * HW + prem];
                if (bv) {
                    const int py = prem / W, px = prem - (prem / W) * W;
                    const int yy = py + dy, xx = px + dx;
                    if (yy >= 0 && yy < H && xx >= 0 && xx < W) vb = in[((size_t)pb * Cin + ci) * HW + yy * W + xx];
                }
            }
            a[t] = (short)va;
            b[t] = (short)vb;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    float* dst = part + (size_t)blockIdx.x * Cout * K;
    if (!bv) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int co = blockIdx.z * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        if (co < Cout) dst[(size_t)co * K + kB] = acc[r];
    }
}

// out[e] = sum_c part[c][e], c in order (deterministic).
__global__ void k_sum_chunks(const float* __restrict__ part, int chunks, size_t n, float* __restrict__ out) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int c = 0; c < chunks; ++c) s += part[(size_t)c * n + e];
        out[e] = s;
    }
}

// Bias gradient, split over chunks of the (image, pixel) pairs:
//   part[chunk][co] = sum over the chunk's pairs of g[b, co, p]
// in a fixed order (per thread in index order, then a tree over the
// threads); the chunks are summed in order by k_sum_chunks. Each thread
// takes 8 consecutive pairs per step, as one 16-byte load when H * W is a
// multiple of 8 (a step then never crosses an image), else one by one.
// Grid: x = chunks, y = channels.
constexpr int BG_CHUNK = 16384;   // pairs per chunk (a multiple of 256 * 8)
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t* __restrict__ g, int B, int C, int HW,
                                                  float* __restrict__ part) {
    __shared__ float sh[256];
    const int co = blockIdx.y;
    const long long n = (long long)B * HW;
    const long long q0 = (long long)blockIdx.x * BG_CHUNK;
    float s = 0.f;
    for (int k = threadIdx.x * 8; k < BG_CHUNK; k += 256 * 8) {
        const long long q = q0 + k;
        if (HW % 8 == 0) {
            if (q < n) {
                const int b = (int)(q / HW);
                const int px = (int)(q - (long long)b * HW);
                const uint4 v = *reinterpret_cast<const uint4*>(g + ((size_t)b * C + co) * HW + px);
                const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) s += bf2f((uint16_t)(w[j] & 0xffffu)) + bf2f((uint16_t)(w[j] >> 16));
            }
        } else {
            for (int j = 0; j < 8; ++j) {
                const long long qj = q + j;
                if (qj < n) {
                    const int b = (int)(qj / HW);
                    s += bf2f(g[((size_t)b * C + co) * HW + (qj - (long long)b * HW)]);
                }
            }
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * C + co] = sh[0];
}

// Weights (float32 [Cout][Cin][3][3]) -> bf16 GEMM layouts for the forward
// (Wg[co][ci*9 + tap], K padded to Kp) and for the data gradient, which is
// the convolution of the output gradient with the flipped, transposed
// kernel (Wt[ci][co*9 + (8 - tap)], padded to Kpt).
__global__ void k_pack_weights(const float* __restrict__ w, int Cin, int Cout, int Kp, int Kpt,
                               uint16_t* __restrict__ Wg, uint16_t* __restrict__ Wt) {
    const int nG = Cout * Kp, nT = Cin * Kpt;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nG + nT; e += gridDim.x * blockDim.x) {
        if (e < nG) {
            const int co = e / Kp, k = e - co * Kp;
            Wg[e] = k < Cin * 9 ? f2bf(w[(size_t)co * Cin * 9 + k]) : 0;
        } else {
            const int f = e - nG;
            const int ci = f / Kpt, k = f - ci * Kpt;
            uint16_t v = 0;
            if (k < Cout * 9) {
                const int co = k / 9, tap = k - (k / 9) * 9;
                v = f2bf(w[((size_t)co * Cin + ci) * 9 + (8 - tap)]);
            }
            Wt[f] = v;
        }
    }
}

// 2x2 average pooling (H, W even) and its gradient; nearest 2x upsampling
// and its gradient (sum of the four children); all bf16 with float math.
__global__ void k_pool2(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int BC, int H, int W) {
    const int Ho = H / 2, Wo = W / 2;
    const size_t n = (size_t)BC * Ho * Wo;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t c = e / ((size_t)Ho * Wo);
        const int r = (int)(e - c * Ho * Wo), y = r / Wo, x = r - (r / Wo) * Wo;
        const uint16_t* s = in + c * H * W + (size_t)(2 * y) * W + 2 * x;
        out[e] = f2bf(0.25f * (bf2f(s[0]) + bf2f(s[1]) + bf2f(s[W]) + bf2f(s[W + 1])));
    }
}
__global__ void k_pool2_grad(const uint16_t* __restrict__ gout, uint16_t* __restrict__ gin, int BC, int H, int W) {
    const size_t n = (size_t)BC * H * W;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t c = e / ((size_t)H * W);
        const int r = (int)(e - c * H * W), y = r / W, x = r - (r / W) * W;
        gin[e] = f2bf(0.25f * bf2f(gout[c * (H / 2) * (W / 2) + (size_t)(y / 2) * (W / 2) + x / 2]));
    }
}
__global__ void k_up2(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int BC, int H, int W) {
    // in: H x W, out: 2H x 2W
    const size_t n = (size_t)BC * 4 * H * W;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t c = e / ((size_t)4 * H * W);
        const int r = (int)(e - c * 4 * H * W), y = r / (2 * W), x = r - (r / (2 * W)) * (2 * W);
        out[e] = in[c * H * W + (size_t)(y / 2) * W + x / 2];
    }
}
__global__ void k_up2_grad(const uint16_t* __restrict__ gout, uint16_t* __restrict__ gin, int BC, int H, int W) {
    // gout: 2H x 2W, gin: H x W
    const size_t n = (size_t)BC * H * W;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t c = e / ((size_t)H * W);
        const int r = (int)(e - c * H * W), y = r / W, x = r - (r / W) * W;
        const uint16_t* s = gout + c * 4 * H * W + (size_t)(2 * y) * (2 * W) + 2 * x;
        gin[e] = f2bf(bf2f(s[0]) + bf2f(s[1]) + bf2f(s[2 * W]) + bf2f(s[2 * W + 1]));
    }
}

// Gradient through a ReLU whose output is act: out = (g + add) * (act > 0),
// where add (may be null) is a second gradient reaching the same output.
__global__ void k_relu_grad(const uint16_t* __restrict__ g, const uint16_t* __restrict__ act,
                            const uint16_t* __restrict__ add, uint16_t* __restrict__ out, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        float v = bf2f(g[e]);
        if (add) v += bf2f(add[e]);
        out[e] = f2bf(bf2f(act[e]) > 0.f ? v : 0.f);
    }
}

// out = a + b (bf16)
__global__ void k_add(const uint16_t* __restrict__ a, const uint16_t* __restrict__ b, uint16_t* __restrict__ out,
                      size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        out[e] = f2bf(bf2f(a[e]) + bf2f(b[e]));
}

// float32 -> bf16 and back
__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        y[e] = f2bf(x[e]);
}

// Mean squared error of pred (float32) against target: grad (bf16) =
// 2 (pred - target) / n, per-block partial sums of the squared error.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ pred, const float* __restrict__ target,
                                            size_t n, uint16_t* __restrict__ grad, float* __restrict__ part) {
    __shared__ float sh[256];
    float s = 0.f;
    const float sc = 2.0f / (float)n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const float d = pred[e] - target[e];
        s += d * d;
        grad[e] = f2bf(sc * d);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Adam step on float32 parameters (bias-corrected, step count t >= 1).
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.f - b1) * ge;
        const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
    }
}

}  // namespace cnn

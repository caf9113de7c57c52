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

constexpr int CONV_NT = 256;   // 4 waves of 32 x 32 output blocks

// Implicit-GEMM 3x3 convolution, stride 1, zero padding 1.
//   out[b, co, y, x] = epilogue( sum_{ci, ky, kx} Wg[co][ci*9 + ky*3 + kx] *
//                                in[b, ci, y + ky - 1, x + kx - 1] )
// Wg is bf16 [Cout][Kp] (K = Cin*9 padded to Kp, a multiple of 8, with zeros).
// Epilogue: + bias[co] (bias may be null), ReLU if relu, + res[b, co, y, x]
// (res may be null, bf16) + res32[b, co, y, x] (may be null, float32).
// Output bf16 (out16) and/or float32 (out32).
// A workgroup takes CB output channels (64, or 32 for layers with at most 32)
// and a TX x 8 pixel tile of one image (TX = 8 for CB = 64, 16 for CB = 32,
// so that the 4 waves cover CB x TX * 8 outputs in 32 x 32 blocks): wave w
// computes channel group w / NPG and pixel group w % NPG (32 consecutive
// pixels of the tile in row order). The reduction runs over chunks of CK
// input channels (CK * 9 = 72 values of K): the chunk's (TX + 2) x 10 input
// window (zero outside the image and past Cin) and its CB x 72 weight slice
// are staged in LDS, and each wave then takes 9 MFMAs with both operands read
// from LDS. Grid: x = B * tiles, y = channel blocks of CB.
constexpr int CK = 8;            // input channels per chunk
constexpr int CKK = CK * 9;      // values of K per chunk
constexpr int WP = CKK + 4;      // LDS pitch of a weight row in bf16 (8-byte aligned rows)
constexpr int CTY = 8;           // pixel tile height
constexpr int conv_tx(int cb) { return cb == 64 ? 8 : 16; }   // pixel tile width

// LDS offset of value k of a chunk (channel k / 9, tap k % 9) in a window of
// width WW, relative to the lane's pixel
__device__ constexpr int xoff(int k, int WW) { return (k / 9) * WW * (CTY + 2) + ((k % 9) / 3) * WW + (k % 3); }

template <int CB>
__global__ __launch_bounds__(CONV_NT) void k_conv3x3(const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ Wg, int Kp,
                                                    const float* __restrict__ bias, const uint16_t* __restrict__ res,
                                                    const float* __restrict__ res32,
                                                    uint16_t* __restrict__ out16, float* __restrict__ out32,
                                                    int B, int Cin, int Cout, int H, int W, int relu) {
    static_assert(CB == 64 || CB == 32, "channel blocks of 64 or 32");
    constexpr int TX = conv_tx(CB), WW = TX + 2, WIN = WW * (CTY + 2);
    constexpr int NPG = 4 / (CB / 32);   // pixel groups (waves per channel group)
    __shared__ __align__(16) uint16_t wl[CB * WP];
    __shared__ uint16_t xl[CK * WIN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (W + TX - 1) / TX, tiles = tiles_x * ((H + CTY - 1) / CTY);
    const int b = blockIdx.x / tiles;
    const int tr = blockIdx.x - b * tiles;
    const int ty0 = (tr / tiles_x) * CTY, tx0 = (tr - (tr / tiles_x) * tiles_x) * TX;
    const int cb = blockIdx.y * CB;
    const int i = lane & 31, kh = lane >> 5;
    const int cg = wave / NPG, pg = wave - cg * NPG;
    const int arow = cg * 32 + i;                       // this lane's A row in the block
    const int pl = pg * 32 + i;                         // this lane's B column: tile pixel pl
    const int py = pl / TX, px = pl - (pl / TX) * TX;
    const int pbase = py * WW + px;
    const int HW = H * W;
    const uint16_t* inb = in + (size_t)b * Cin * HW;
    f32x16 acc = {};
    for (int c0 = 0; c0 < Cin; c0 += CK) {
        // weights: rows cb .. cb + CB - 1, K values c0 * 9 .. + 71, 8 at a time
        // (c0 * 9 and Kp are multiples of 8, so a group lies wholly below Kp
        // or wholly past it; past it belongs to the next row and reads as 0)
        for (int e = tid; e < CB * (CKK / 8); e += CONV_NT) {
            const int row = e / (CKK / 8), g8 = e - row * (CKK / 8);
            const int co = cb + row, k = c0 * 9 + 8 * g8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (co < Cout && k < Kp) v = *reinterpret_cast<const uint4*>(Wg + (size_t)co * Kp + k);
            uint2* d = reinterpret_cast<uint2*>(&wl[row * WP + 8 * g8]);
            d[0] = make_uint2(v.x, v.y);
            d[1] = make_uint2(v.z, v.w);
        }
        // input window: channels c0 .. c0 + CK - 1, rows ty0 - 1 .., columns tx0 - 1 ..
        for (int e = tid; e < CK * WIN; e += CONV_NT) {
            const int cl = e / WIN, rem = e - cl * WIN;
            const int wy = rem / WW, wx = rem - (rem / WW) * WW;
            const int ci = c0 + cl, yy = ty0 + wy - 1, xx = tx0 + wx - 1;
            xl[e] = (ci < Cin && yy >= 0 && yy < H && xx >= 0 && xx < W) ? inb[(size_t)ci * HW + yy * W + xx] : 0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < CKK / 8; ++s) {
            bf16x4 a, bv;
            const uint2 w2 = *reinterpret_cast<const uint2*>(&wl[arow * WP + s * 8 + 4 * kh]);
            a[0] = (short)(w2.x & 0xffff);
            a[1] = (short)(w2.x >> 16);
            a[2] = (short)(w2.y & 0xffff);
            a[3] = (short)(w2.y >> 16);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int o = kh ? xoff(s * 8 + 4 + t, WW) : xoff(s * 8 + t, WW);
                bv[t] = (short)xl[pbase + o];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue: lane holds tile pixel pl, rows (channels) 8(r/4) + 4 kh + r%4 of its group's 32
    const int gy = ty0 + py, gx = tx0 + px;
    if (gy >= H || gx >= W) return;
    const int co0 = cb + cg * 32;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int co = co0 + 8 * (r >> 2) + 4 * kh + (r & 3);
        if (co >= Cout) continue;
        float v = acc[r];
        if (bias) v += bias[co];
        if (relu) v = fmaxf(v, 0.f);
        const size_t o = ((size_t)b * Cout + co) * HW + (size_t)gy * W + gx;
        if (res) v += bf2f(res[o]);
        if (res32) v += res32[o];
        if (out16) out16[o] = f2bf(v);
        if (out32) out32[o] = v;
    }
}

// Weight gradient of the 3x3 convolution, split over chunks of pixel tiles:
//   part[chunk][co][k] = sum over the chunk's pixels p of
//                        g[b, co, p] * in[b, ci(k), p + tap(k)]
// (M = Cout, N = K = Cin*9, the reduction over pixels, 8 per MFMA). A
// workgroup takes 64 channels x 64 values of K and WT_TILES 8 x 8 pixel
// tiles (image by image, tiles in row order); for each tile the gradient
// block (64 channels x 64 pixels, zero outside the image) and the 10 x 10
// input window of the (at most 8) channels the K block reaches are staged in
// LDS, and each wave takes 8 MFMAs (one per tile row) with both operands read
// from LDS; wave w computes channels 32 (w >> 1) .. and values of K
// 32 (w & 1) .. of the block. The tiles are taken in order, so the partial
// sums are deterministic; the chunks are summed in order by k_sum_chunks.
// Grid: x = chunks, y = K blocks of 64, z = channel blocks of 64.
constexpr int WT_TILES = 64;          // 8 x 8 tiles per chunk
constexpr int GP = 64 + 4;            // LDS pitch of a gradient row in bf16 (8-byte aligned rows)
constexpr int WCH = 8;                // channels a K block of 64 reaches: (k0 % 9 + 63) / 9 + 1 <= 8
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const uint16_t* __restrict__ g,
                                                      const uint16_t* __restrict__ in, float* __restrict__ part,
                                                      int B, int Cin, int Cout, int H, int W) {
    __shared__ __align__(16) uint16_t gl[64 * GP];
    __shared__ uint16_t xl[WCH * 100];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = lane & 31, kh = lane >> 5;
    const int tiles_x = (W + 7) / 8, tiles = tiles_x * ((H + 7) / 8);
    const long long ntiles = (long long)B * tiles;
    const int K = Cin * 9;
    const int kb0 = blockIdx.y * 64, cb = blockIdx.z * 64;
    const int ci0 = kb0 / 9;                               // first channel of the window
    const int arow = (wave >> 1) * 32 + i;                 // A row: channel cb + arow
    const int kcol = kb0 + (wave & 1) * 32 + i;            // B column: value kcol of K
    const bool kv = kcol < K;
    const int kci = kv ? kcol / 9 - ci0 : 0, ktap = kv ? kcol - (kcol / 9) * 9 : 0;
    const int koff = kci * 100 + (ktap / 3) * 10 + (ktap - (ktap / 3) * 3);   // window offset of tile pixel (0, 0)
    f32x16 acc = {};
    const long long t0 = (long long)blockIdx.x * WT_TILES;
    for (int tt = 0; tt < WT_TILES; ++tt) {
        const long long t = t0 + tt;
        if (t >= ntiles) break;   // uniform
        const int b = (int)(t / tiles), tr = (int)(t - (long long)b * tiles);
        const int ty0 = (tr / tiles_x) * 8, tx0 = (tr - (tr / tiles_x) * tiles_x) * 8;
        // gradient block: channel rows, 8 pixels of one tile row per step
        for (int e = tid; e < 64 * 8; e += 256) {
            const int row = e >> 3, r8 = e & 7;
            const int co = cb + row, yy = ty0 + r8;
            uint4 q = make_uint4(0u, 0u, 0u, 0u);
            if (co < Cout && yy < H) {
                const uint16_t* src = g + ((size_t)(b * Cout + co) * H + yy) * W + tx0;
                if (W % 8 == 0) {
                    q = *reinterpret_cast<const uint4*>(src);
                } else {
                    uint16_t v[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) v[j] = (tx0 + j < W) ? src[j] : 0;
                    q = make_uint4(v[0] | ((unsigned)v[1] << 16), v[2] | ((unsigned)v[3] << 16),
                                   v[4] | ((unsigned)v[5] << 16), v[6] | ((unsigned)v[7] << 16));
                }
            }
            uint2* d = reinterpret_cast<uint2*>(&gl[row * GP + r8 * 8]);
            d[0] = make_uint2(q.x, q.y);
            d[1] = make_uint2(q.z, q.w);
        }
        // input window of channels ci0 .. ci0 + WCH - 1
        for (int e = tid; e < WCH * 100; e += 256) {
            const int cl = e / 100, rem = e - cl * 100, wy = rem / 10, wx = rem - (rem / 10) * 10;
            const int ci = ci0 + cl, yy = ty0 + wy - 1, xx = tx0 + wx - 1;
            xl[e] = (ci < Cin && yy >= 0 && yy < H && xx >= 0 && xx < W)
                        ? in[((size_t)(b * Cin + ci) * H + yy) * W + xx] : 0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) {   // tile row s: pixels 8 s + 4 kh + t
            bf16x4 a, bv;
            const uint2 w2 = *reinterpret_cast<const uint2*>(&gl[arow * GP + s * 8 + 4 * kh]);
            a[0] = (short)(w2.x & 0xffff);
            a[1] = (short)(w2.x >> 16);
            a[2] = (short)(w2.y & 0xffff);
            a[3] = (short)(w2.y >> 16);
#pragma unroll
            for (int t = 0; t < 4; ++t) bv[t] = kv ? (short)xl[koff + s * 10 + 4 * kh + t] : (short)0;
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    float* dst = part + (size_t)blockIdx.x * Cout * K;
    if (!kv) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int co = cb + (wave >> 1) * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        if (co < Cout) dst[(size_t)co * K + kcol] = acc[r];
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

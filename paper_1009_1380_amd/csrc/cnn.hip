// cnn.hip - the learned warm start's network (include/radon.h, radon_cnn_*):
// a 4-level convolutional encoder-decoder, 32-64-128-256 channels, 3x3
// convolutions on BF16 matrix cores with float32 accumulation, trained with
// Adam on pairs that the method itself generates (filtered adjoint -> basis-
// pursuit solution). Hand-written kernels only (cnn_kernels.hpp).
//
//   e0 = relu(conv_a(x))            32 @ H      x: one channel
//   e1 = relu(conv_b(pool(e0)))     64 @ H/2
//   e2 = relu(conv_c(pool(e1)))    128 @ H/4
//   e3 = relu(conv_d(pool(e2)))    256 @ H/8
//   d2 = relu(conv_e(up(e3))) + e2 128 @ H/4
//   d1 = relu(conv_f(up(d2))) + e1  64 @ H/2
//   d0 = relu(conv_g(up(d1))) + e0  32 @ H
//   y  = conv_h(d0) + x              1 @ H     (a correction of the input)
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <new>
#include <random>
#include <vector>

#include "../../include/radon.h"
#include "cnn_kernels.hpp"
#include "radon_internal.hpp"

namespace {

using cnn::CONV_NT;

radon_status_t errf(radon_status_t st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
radon_status_t errf(radon_status_t st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return rn::api_fail(st, buf);
}

int pad8(int k) { return (k + 7) / 8 * 8; }

struct Conv {
    int cin = 0, cout = 0, Kp = 0, Kpt = 0;
    float *w = nullptr, *b = nullptr;          // parameters (float32)
    float *gw = nullptr, *gb = nullptr;        // gradients
    float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr;   // Adam moments
    uint16_t *Wg = nullptr, *Wt = nullptr;     // bf16 GEMM layouts (forward, data gradient)
    size_t nw() const { return (size_t)cout * cin * 9; }
};

constexpr int NCONV = 8;

}  // namespace

struct radon_cnn_s {
    int device = 0;
    int B = 0, H = 0, W = 0;
    int step = 0;
    Conv conv[NCONV];
    std::vector<void*> allocs;
    // activations (bf16) and gradients
    uint16_t *x16 = nullptr, *e0 = nullptr, *p0 = nullptr, *e1 = nullptr, *p1 = nullptr, *e2 = nullptr,
             *p2 = nullptr, *e3 = nullptr, *u3 = nullptr, *re = nullptr, *d2 = nullptr, *u2 = nullptr,
             *rf = nullptr, *d1 = nullptr, *u1 = nullptr, *rg = nullptr, *d0 = nullptr;
    uint16_t *gy = nullptr, *ga = nullptr, *gb = nullptr, *gc = nullptr;   // scratch gradients (largest size)
    float *part = nullptr, *loss_part = nullptr;
    size_t part_n = 0;
    hipError_t err = hipSuccess;

    ~radon_cnn_s() {
        for (void* p : allocs) (void)hipFree(p);
    }
    template <class T>
    bool alloc(T** out, size_t count) {
        void* p = nullptr;
        if (hipMalloc(&p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        allocs.push_back(p);
        *out = static_cast<T*>(p);
        return true;
    }
    void chk(hipError_t e) { if (err == hipSuccess && e != hipSuccess) err = e; }
};

namespace {

size_t grid1(size_t n) { return std::min<size_t>((n + 255) / 256, 65535); }
// chunks of k_conv3x3_wgrad for B images of h x w
size_t wgrad_chunks(long long B, int h, int w) {
    const long long tiles = B * (long long)((h + 7) / 8) * ((w + 7) / 8);
    return (size_t)((tiles + cnn::WT_TILES - 1) / cnn::WT_TILES);
}

// k_conv3x3 over `cout` output channels: blocks of 64 channels on 8 x 8 pixel
// tiles, or of 32 on 16 x 8 tiles when there are at most 32
void conv_launch(const uint16_t* in, const uint16_t* Wg, int Kp, const float* bias, const uint16_t* res,
                 const float* res32, uint16_t* out16, float* out32, int B, int cin, int cout, int h, int w, bool relu,
                 hipStream_t st) {
    auto tiles = [&](int tx) { return ((w + tx - 1) / tx) * ((h + cnn::CTY - 1) / cnn::CTY); };
    if (cout <= 32) {
        const dim3 grid((unsigned)(B * tiles(cnn::conv_tx(32))), 1u);
        hipLaunchKernelGGL(cnn::k_conv3x3<32>, grid, dim3(CONV_NT), 0, st, in, Wg, Kp, bias, res, res32, out16,
                           out32, B, cin, cout, h, w, relu ? 1 : 0);
    } else {
        const dim3 grid((unsigned)(B * tiles(cnn::conv_tx(64))), (unsigned)((cout + 63) / 64));
        hipLaunchKernelGGL(cnn::k_conv3x3<64>, grid, dim3(CONV_NT), 0, st, in, Wg, Kp, bias, res, res32, out16,
                           out32, B, cin, cout, h, w, relu ? 1 : 0);
    }
}

void conv_fwd(radon_cnn_s& c, const Conv& L, const uint16_t* in, int h, int w, uint16_t* out16, float* out32,
              const uint16_t* res, bool relu, hipStream_t st, const float* res32 = nullptr) {
    conv_launch(in, L.Wg, L.Kp, L.b, res, res32, out16, out32, c.B, L.cin, L.cout, h, w, relu, st);
}

// data gradient: gin = conv(gout, flipped transposed kernel), no bias
void conv_dgrad(radon_cnn_s& c, const Conv& L, const uint16_t* gout, int h, int w, uint16_t* gin, hipStream_t st) {
    conv_launch(gout, L.Wt, L.Kpt, nullptr, nullptr, nullptr, gin, nullptr, c.B, L.cout, L.cin, h, w, false, st);
}

void conv_wgrad(radon_cnn_s& c, Conv& L, const uint16_t* gout, const uint16_t* in, int h, int w, hipStream_t st) {
    const long long np = (long long)c.B * h * w;
    const int chunks = (int)wgrad_chunks(c.B, h, w);
    const int K = L.cin * 9;
    const dim3 grid((unsigned)chunks, (unsigned)((K + 63) / 64), (unsigned)((L.cout + 63) / 64));
    hipLaunchKernelGGL(cnn::k_conv3x3_wgrad, grid, dim3(256), 0, st, gout, in, c.part, c.B, L.cin, L.cout, h, w);
    hipLaunchKernelGGL(cnn::k_sum_chunks, dim3((unsigned)grid1(L.nw())), dim3(256), 0, st, c.part, chunks, L.nw(),
                       L.gw);
    // the bias partials reuse the weight partials' buffer, which the sum above has read
    const int bchunks = (int)((np + cnn::BG_CHUNK - 1) / cnn::BG_CHUNK);
    hipLaunchKernelGGL(cnn::k_bias_grad, dim3((unsigned)bchunks, (unsigned)L.cout), dim3(256), 0, st, gout, c.B,
                       L.cout, h * w, c.part);
    hipLaunchKernelGGL(cnn::k_sum_chunks, dim3((unsigned)grid1((size_t)L.cout)), dim3(256), 0, st, c.part, bchunks,
                       (size_t)L.cout, L.gb);
}

void pack(Conv& L, hipStream_t st) {
    hipLaunchKernelGGL(cnn::k_pack_weights, dim3(64), dim3(256), 0, st, L.w, L.cin, L.cout, L.Kp, L.Kpt, L.Wg, L.Wt);
}

void pool(const uint16_t* in, uint16_t* out, int bc, int h, int w, hipStream_t st) {
    hipLaunchKernelGGL(cnn::k_pool2, dim3((unsigned)grid1((size_t)bc * h * w / 4)), dim3(256), 0, st, in, out, bc, h, w);
}
void pool_grad(const uint16_t* gout, uint16_t* gin, int bc, int h, int w, hipStream_t st) {
    hipLaunchKernelGGL(cnn::k_pool2_grad, dim3((unsigned)grid1((size_t)bc * h * w)), dim3(256), 0, st, gout, gin, bc,
                       h, w);
}
void up(const uint16_t* in, uint16_t* out, int bc, int h, int w, hipStream_t st) {
    hipLaunchKernelGGL(cnn::k_up2, dim3((unsigned)grid1((size_t)bc * 4 * h * w)), dim3(256), 0, st, in, out, bc, h, w);
}
void up_grad(const uint16_t* gout, uint16_t* gin, int bc, int h, int w, hipStream_t st) {
    hipLaunchKernelGGL(cnn::k_up2_grad, dim3((unsigned)grid1((size_t)bc * h * w)), dim3(256), 0, st, gout, gin, bc, h,
                       w);
}
void relu_grad(const uint16_t* g, const uint16_t* act, const uint16_t* add, uint16_t* out, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(cnn::k_relu_grad, dim3((unsigned)grid1(n)), dim3(256), 0, st, g, act, add, out, n);
}
void add(const uint16_t* a, const uint16_t* b, uint16_t* out, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(cnn::k_add, dim3((unsigned)grid1(n)), dim3(256), 0, st, a, b, out, n);
}

// forward of the whole network; y32 gets the float32 output
void forward(radon_cnn_s& c, const float* x, float* y32, hipStream_t st) {
    const int B = c.B, H = c.H, W = c.W;
    const size_t n0 = (size_t)B * H * W;
    hipLaunchKernelGGL(cnn::k_to_bf16, dim3((unsigned)grid1(n0)), dim3(256), 0, st, x, c.x16, n0);
    conv_fwd(c, c.conv[0], c.x16, H, W, c.e0, nullptr, nullptr, true, st);
    pool(c.e0, c.p0, B * 32, H, W, st);
    conv_fwd(c, c.conv[1], c.p0, H / 2, W / 2, c.e1, nullptr, nullptr, true, st);
    pool(c.e1, c.p1, B * 64, H / 2, W / 2, st);
    conv_fwd(c, c.conv[2], c.p1, H / 4, W / 4, c.e2, nullptr, nullptr, true, st);
    pool(c.e2, c.p2, B * 128, H / 4, W / 4, st);
    conv_fwd(c, c.conv[3], c.p2, H / 8, W / 8, c.e3, nullptr, nullptr, true, st);
    up(c.e3, c.u3, B * 256, H / 8, W / 8, st);
    conv_fwd(c, c.conv[4], c.u3, H / 4, W / 4, c.re, nullptr, nullptr, true, st);
    add(c.re, c.e2, c.d2, (size_t)B * 128 * (H / 4) * (W / 4), st);
    up(c.d2, c.u2, B * 128, H / 4, W / 4, st);
    conv_fwd(c, c.conv[5], c.u2, H / 2, W / 2, c.rf, nullptr, nullptr, true, st);
    add(c.rf, c.e1, c.d1, (size_t)B * 64 * (H / 2) * (W / 2), st);
    up(c.d1, c.u1, B * 64, H / 2, W / 2, st);
    conv_fwd(c, c.conv[6], c.u1, H, W, c.rg, nullptr, nullptr, true, st);
    add(c.rg, c.e0, c.d0, (size_t)B * 32 * H * W, st);
    conv_fwd(c, c.conv[7], c.d0, H, W, nullptr, y32, nullptr, false, st, x);   // + the float32 input
}

// backward from gy (bf16 gradient of the output); fills every layer's gw, gb
void backward(radon_cnn_s& c, hipStream_t st) {
    const int B = c.B, H = c.H, W = c.W;
    const size_t s0 = (size_t)B * H * W, s1 = s0 / 4, s2 = s0 / 16, s3 = s0 / 64;
    uint16_t *ga = c.ga, *gb = c.gb, *gc = c.gc;
    // y = conv_h(d0) + x
    conv_wgrad(c, c.conv[7], c.gy, c.d0, H, W, st);
    conv_dgrad(c, c.conv[7], c.gy, H, W, ga, st);                         // ga = dL/dd0 (32 @ H)
    // d0 = relu(conv_g(u1)) + e0: keep dL/de0 (skip part) in ga, pre-activation in gb
    relu_grad(ga, c.rg, nullptr, gb, 32 * s0, st);
    conv_wgrad(c, c.conv[6], gb, c.u1, H, W, st);
    conv_dgrad(c, c.conv[6], gb, H, W, gc, st);                           // gc = dL/du1 (64 @ H)
    up_grad(gc, gb, B * 64, H / 2, W / 2, st);                            // gb = dL/dd1 (64 @ H/2)
    // d1 = relu(conv_f(u2)) + e1 (ga holds dL/de0 until the end; gb is dL/dd1)
    uint16_t* gd1 = gb;
    uint16_t* tmp = gc;
    relu_grad(gd1, c.rf, nullptr, tmp, 64 * s1, st);
    conv_wgrad(c, c.conv[5], tmp, c.u2, H / 2, W / 2, st);
    uint16_t* gu2 = tmp + 64 * s1;                                         // after the pre-activation grad
    conv_dgrad(c, c.conv[5], tmp, H / 2, W / 2, gu2, st);                 // 128 @ H/2
    uint16_t* gd2 = gu2 + 128 * s1;
    up_grad(gu2, gd2, B * 128, H / 4, W / 4, st);                         // 128 @ H/4
    // d2 = relu(conv_e(u3)) + e2
    uint16_t* tre = gd2 + 128 * s2;
    relu_grad(gd2, c.re, nullptr, tre, 128 * s2, st);
    conv_wgrad(c, c.conv[4], tre, c.u3, H / 4, W / 4, st);
    uint16_t* gu3 = tre + 128 * s2;
    conv_dgrad(c, c.conv[4], tre, H / 4, W / 4, gu3, st);                 // 256 @ H/4
    uint16_t* ge3 = gu3 + 256 * s2;
    up_grad(gu3, ge3, B * 256, H / 8, W / 8, st);                         // 256 @ H/8
    // e3 = relu(conv_d(p2))
    uint16_t* td = ge3 + 256 * s3;
    relu_grad(ge3, c.e3, nullptr, td, 256 * s3, st);
    conv_wgrad(c, c.conv[3], td, c.p2, H / 8, W / 8, st);
    uint16_t* gp2 = td + 256 * s3;
    conv_dgrad(c, c.conv[3], td, H / 8, W / 8, gp2, st);                  // 128 @ H/8
    uint16_t* ge2p = gp2 + 128 * s3;
    pool_grad(gp2, ge2p, B * 128, H / 4, W / 4, st);                      // 128 @ H/4
    // e2 = relu(conv_c(p1)), total gradient = skip (gd2) + pooled path
    uint16_t* tc = ge2p + 128 * s2;
    relu_grad(gd2, c.e2, ge2p, tc, 128 * s2, st);
    conv_wgrad(c, c.conv[2], tc, c.p1, H / 4, W / 4, st);
    uint16_t* gp1 = tc + 128 * s2;
    conv_dgrad(c, c.conv[2], tc, H / 4, W / 4, gp1, st);                  // 64 @ H/4
    uint16_t* ge1p = gp1 + 64 * s2;
    pool_grad(gp1, ge1p, B * 64, H / 2, W / 2, st);                       // 64 @ H/2
    // e1 = relu(conv_b(p0)), total = skip (gd1) + pooled path
    uint16_t* tb = ge1p + 64 * s1;
    relu_grad(gd1, c.e1, ge1p, tb, 64 * s1, st);
    conv_wgrad(c, c.conv[1], tb, c.p0, H / 2, W / 2, st);
    uint16_t* gp0 = tb + 64 * s1;
    conv_dgrad(c, c.conv[1], tb, H / 2, W / 2, gp0, st);                  // 32 @ H/2
    uint16_t* ge0p = gp0 + 32 * s1;
    pool_grad(gp0, ge0p, B * 32, H, W, st);                               // 32 @ H
    // e0 = relu(conv_a(x)), total = skip (ga) + pooled path
    uint16_t* ta = ge0p + 32 * s0;
    relu_grad(ga, c.e0, ge0p, ta, 32 * s0, st);
    conv_wgrad(c, c.conv[0], ta, c.x16, H, W, st);
}

}  // namespace

extern "C" {

radon_status_t radon_cnn_create(radon_cnn_t* out, int batch, int height, int width, uint64_t seed) {
    if (!out) return errf(RADON_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (batch < 1 || height < 8 || width < 8 || height % 8 || width % 8)
        return errf(RADON_ERR_INVALID, "batch >= 1 and height, width multiples of 8 (got %d, %d, %d)", batch,
                    height, width);
    radon_cnn_s* c = new (std::nothrow) radon_cnn_s();
    if (!c) return errf(RADON_ERR_OOM, "host allocation failed");
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return errf(RADON_ERR_DEVICE, "no HIP device");
    }
    c->B = batch;
    c->H = height;
    c->W = width;
    const int chans[NCONV][2] = {{1, 32}, {32, 64}, {64, 128}, {128, 256}, {256, 128}, {128, 64}, {64, 32}, {32, 1}};
    std::mt19937_64 rng(seed);
    bool ok = true;
    size_t part_n = 0;
    const int sizes[NCONV] = {1, 2, 4, 8, 4, 2, 1, 1};   // spatial divisor of each layer
    for (int l = 0; l < NCONV && ok; ++l) {
        Conv& L = c->conv[l];
        L.cin = chans[l][0];
        L.cout = chans[l][1];
        L.Kp = pad8(L.cin * 9);
        L.Kpt = pad8(L.cout * 9);
        const size_t nw = L.nw();
        ok = c->alloc(&L.w, nw) && c->alloc(&L.b, L.cout) && c->alloc(&L.gw, nw) && c->alloc(&L.gb, L.cout) &&
             c->alloc(&L.mw, nw) && c->alloc(&L.vw, nw) && c->alloc(&L.mb, L.cout) && c->alloc(&L.vb, L.cout) &&
             c->alloc(&L.Wg, (size_t)L.cout * L.Kp) && c->alloc(&L.Wt, (size_t)L.cin * L.Kpt);
        if (!ok) break;
        // He initialisation (the last layer starts at zero: the network begins as the identity)
        std::vector<float> w(nw), zb(L.cout, 0.f), z(nw, 0.f);
        std::normal_distribution<float> nd(0.f, sqrtf(2.0f / (L.cin * 9)));
        for (auto& v : w) v = (l == NCONV - 1) ? 0.f : nd(rng);
        c->chk(hipMemcpy(L.w, w.data(), sizeof(float) * nw, hipMemcpyHostToDevice));
        c->chk(hipMemcpy(L.b, zb.data(), sizeof(float) * L.cout, hipMemcpyHostToDevice));
        for (float* p : {L.mw, L.vw}) c->chk(hipMemcpy(p, z.data(), sizeof(float) * nw, hipMemcpyHostToDevice));
        for (float* p : {L.mb, L.vb}) c->chk(hipMemcpy(p, zb.data(), sizeof(float) * L.cout, hipMemcpyHostToDevice));
        pack(L, 0);
        const size_t chunks = wgrad_chunks(batch, height / sizes[l], width / sizes[l]);
        part_n = std::max(part_n, chunks * nw);
    }
    const size_t s0 = (size_t)batch * height * width, s1 = s0 / 4, s2 = s0 / 16, s3 = s0 / 64;
    ok = ok && c->alloc(&c->x16, s0) && c->alloc(&c->e0, 32 * s0) && c->alloc(&c->p0, 32 * s1) &&
         c->alloc(&c->e1, 64 * s1) && c->alloc(&c->p1, 64 * s2) && c->alloc(&c->e2, 128 * s2) &&
         c->alloc(&c->p2, 128 * s3) && c->alloc(&c->e3, 256 * s3) && c->alloc(&c->u3, 256 * s2) &&
         c->alloc(&c->re, 128 * s2) && c->alloc(&c->d2, 128 * s2) && c->alloc(&c->u2, 128 * s1) &&
         c->alloc(&c->rf, 64 * s1) && c->alloc(&c->d1, 64 * s1) && c->alloc(&c->u1, 64 * s0) &&
         c->alloc(&c->rg, 32 * s0) && c->alloc(&c->d0, 32 * s0) && c->alloc(&c->gy, s0) &&
         c->alloc(&c->ga, 32 * s0) && c->alloc(&c->gb, 64 * s0) &&
         c->alloc(&c->gc, 64 * s0 + 64 * s1 + 128 * s1 + 4 * 128 * s2 + 2 * 256 * s2 + 3 * 256 * s3 +
                              2 * 128 * s3 + 64 * s2 + 3 * 64 * s1 + 32 * s1 + 2 * 32 * s0) &&
         c->alloc(&c->part, part_n) && c->alloc(&c->loss_part, 1024);
    c->part_n = part_n;
    if (!ok) {
        delete c;
        return errf(RADON_ERR_OOM, "device allocation failed");
    }
    c->chk(hipDeviceSynchronize());
    if (c->err != hipSuccess) {
        delete c;
        return errf(RADON_ERR_DEVICE, "network set-up failed");
    }
    *out = c;
    return rn::api_ok();
}

void radon_cnn_destroy(radon_cnn_t net) { delete net; }

radon_status_t radon_cnn_forward(radon_cnn_t net, const float* in_dev, float* out_dev, void* stream) {
    if (!net || !in_dev || !out_dev) return errf(RADON_ERR_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    forward(*net, in_dev, out_dev, st);
    if (hipGetLastError() != hipSuccess) return errf(RADON_ERR_DEVICE, "network forward launch failed");
    return rn::api_ok();
}

radon_status_t radon_cnn_train_step(radon_cnn_t net, const float* in_dev, const float* target_dev, float lr,
                                    float* loss_host, float* pred_dev, void* stream) {
    if (!net || !in_dev || !target_dev || !pred_dev) return errf(RADON_ERR_INVALID, "NULL argument");
    if (!(lr >= 0.f)) return errf(RADON_ERR_INVALID, "lr must be >= 0");
    radon_cnn_s& c = *net;
    hipStream_t st = (hipStream_t)stream;
    const size_t n0 = (size_t)c.B * c.H * c.W;
    forward(c, in_dev, pred_dev, st);
    const int nblk = (int)std::min<size_t>((n0 + 255) / 256, 1024);
    hipLaunchKernelGGL(cnn::k_mse, dim3(nblk), dim3(256), 0, st, pred_dev, target_dev, n0, c.gy, c.loss_part);
    backward(c, st);
    // Adam
    c.step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)c.step), c2 = 1.f - powf(b2, (float)c.step);
    for (int l = 0; l < NCONV; ++l) {
        Conv& L = c.conv[l];
        hipLaunchKernelGGL(cnn::k_adam, dim3((unsigned)grid1(L.nw())), dim3(256), 0, st, L.w, L.gw, L.mw, L.vw,
                           L.nw(), lr, b1, b2, eps, c1, c2);
        hipLaunchKernelGGL(cnn::k_adam, dim3(1), dim3(256), 0, st, L.b, L.gb, L.mb, L.vb, (size_t)L.cout, lr, b1, b2,
                           eps, c1, c2);
        pack(L, st);
    }
    if (hipGetLastError() != hipSuccess) return errf(RADON_ERR_DEVICE, "training step launch failed");
    if (loss_host) {
        std::vector<float> part(nblk);
        if (hipMemcpyAsync(part.data(), c.loss_part, sizeof(float) * nblk, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            (void)hipGetLastError();
            return errf(RADON_ERR_DEVICE, "loss read-back failed");
        }
        double s = 0.0;
        for (float v : part) s += v;
        *loss_host = (float)(s / (double)n0);
    }
    return rn::api_ok();
}

int64_t radon_cnn_param_count(radon_cnn_t net) {
    if (!net) return -1;
    int64_t n = 0;
    for (const Conv& L : net->conv) n += (int64_t)L.nw() + L.cout;
    return n;
}

// Parameters (or gradients) in layer order: w (Cout x Cin x 3 x 3) then b.
static radon_status_t copy_params(radon_cnn_t net, float* host, int64_t n, bool grads, bool to_device) {
    if (!net || !host) return errf(RADON_ERR_INVALID, "NULL argument");
    if (n != radon_cnn_param_count(net)) return errf(RADON_ERR_INVALID, "need %lld values", (long long)radon_cnn_param_count(net));
    size_t off = 0;
    for (Conv& L : net->conv) {
        float* w = grads ? L.gw : L.w;
        float* b = grads ? L.gb : L.b;
        hipError_t e;
        if (to_device) {
            e = hipMemcpy(w, host + off, sizeof(float) * L.nw(), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(b, host + off + L.nw(), sizeof(float) * L.cout, hipMemcpyHostToDevice);
            pack(L, 0);
        } else {
            e = hipMemcpy(host + off, w, sizeof(float) * L.nw(), hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(host + off + L.nw(), b, sizeof(float) * L.cout, hipMemcpyDeviceToHost);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return errf(RADON_ERR_DEVICE, "parameter copy failed");
        }
        off += L.nw() + L.cout;
    }
    if (hipDeviceSynchronize() != hipSuccess) return errf(RADON_ERR_DEVICE, "parameter copy failed");
    return rn::api_ok();
}

radon_status_t radon_cnn_get_params(radon_cnn_t net, float* host, int64_t n) { return copy_params(net, host, n, false, false); }
radon_status_t radon_cnn_set_params(radon_cnn_t net, const float* host, int64_t n) {
    return copy_params(net, const_cast<float*>(host), n, false, true);
}
radon_status_t radon_cnn_get_grads(radon_cnn_t net, float* host, int64_t n) { return copy_params(net, host, n, true, false); }

// Test hook: one 3x3 convolution with float32 weights w (Cout x Cin x 3 x 3),
// bias (may be null) and bf16 tensors; also its data and weight gradients
// for an output gradient gout (any of the gradient outputs may be null).
radon_status_t radon_cnn_conv_test(const uint16_t* in, const float* w, const float* bias, const uint16_t* res,
                                   uint16_t* out16, float* out32, int relu, const uint16_t* gout, uint16_t* gin,
                                   float* gw, float* gb, int B, int Cin, int Cout, int H, int W, void* stream) {
    if (!in || !w || B < 1 || Cin < 1 || Cout < 1 || H < 1 || W < 1) return errf(RADON_ERR_INVALID, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    radon_cnn_s c;
    c.B = B;
    Conv L;
    L.cin = Cin;
    L.cout = Cout;
    L.Kp = pad8(Cin * 9);
    L.Kpt = pad8(Cout * 9);
    L.w = const_cast<float*>(w);
    L.b = const_cast<float*>(bias);
    L.gw = gw;
    L.gb = gb;
    const size_t chunks = wgrad_chunks(B, H, W);
    if (!c.alloc(&L.Wg, (size_t)Cout * L.Kp) || !c.alloc(&L.Wt, (size_t)Cin * L.Kpt) ||
        !c.alloc(&c.part, chunks * L.nw()))
        return errf(RADON_ERR_OOM, "test buffers");
    pack(L, st);
    if (out16 || out32) conv_fwd(c, L, in, H, W, out16, out32, res, relu != 0, st);
    if (gout && gin) conv_dgrad(c, L, gout, H, W, gin, st);
    if (gout && gw && gb) conv_wgrad(c, L, gout, in, H, W, st);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return errf(RADON_ERR_DEVICE, "convolution test failed");
    return rn::api_ok();
}

}  // extern "C"

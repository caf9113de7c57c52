// fft_lds.hpp - batched complex64 FFTs resident in LDS, for gfx950.
//
// Every 1D transform of the Radon path (the oversampled 2D FFT done as row
// and column passes, and the ray FFTs; section "fast radon transform",
// paragraph 1) runs on this engine: a Stockham autosort FFT of compile-time
// length LEN = 2^a 3^b 5^c, radix 8/4/2/3/5 passes, all lines of a workgroup
// transformed together. Each pass reads its butterflies' inputs from LDS into
// registers, barriers, applies twiddles and the radix-R DFT, writes the
// outputs back in place, and barriers again; no scratch buffer is needed.
// Twiddles come from a float32 table e^{-2 pi i t/LEN}, t < LEN, built in
// float64 on the host (one entry per butterfly; the other powers are formed
// by products). The engine computes the forward (e^-) transform; the callers
// obtain inverse transforms as conj(FFT(conj(x))).
#pragma once

#include <hip/hip_runtime.h>

namespace rn {

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, then for every wave. __syncthreads() also waits for the
// wave's outstanding global loads and stores, which exposes their latency at
// every barrier; global data is waited for where it is used instead.
#ifndef RN_LDS_SYNC
#define RN_LDS_SYNC 1
#endif
__device__ __forceinline__ void lds_sync() {
#if RN_LDS_SYNC
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
#else
    __syncthreads();
#endif
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Complex product with its two fused multiply-adds written out (the library
// is built without implicit contraction, so the rounding is the same in every
// kernel that uses it).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// -i * a and +i * a
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }

// ---- radix-R forward DFT kernels (y_k = sum_m v_m e^{-2 pi i m k / R})

template <int R> struct Dft;

template <> struct Dft<2> {
    static __device__ __forceinline__ void run(float2* v) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <> struct Dft<3> {
    static __device__ __forceinline__ void run(float2* v) {
        const float s3 = 0.86602540378443865f;  // sin(2 pi / 3)
        float2 t = cadd(v[1], v[2]);
        float2 d = csub(v[1], v[2]);
        float2 m = make_float2(fmaf(-0.5f, t.x, v[0].x), fmaf(-0.5f, t.y, v[0].y));
        float2 r = mul_mi(cscale(d, s3));       // -i s3 (v1 - v2)
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, r);
        v[2] = csub(m, r);
    }
};

template <> struct Dft<4> {
    static __device__ __forceinline__ void run(float2* v) {
        float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        float2 t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <> struct Dft<5> {
    static __device__ __forceinline__ void run(float2* v) {
        const float c1 = 0.30901699437494742f;   // cos(2 pi / 5)
        const float c2 = -0.80901699437494742f;  // cos(4 pi / 5)
        const float s1 = 0.95105651629515357f;   // sin(2 pi / 5)
        const float s2 = 0.58778525229247313f;   // sin(4 pi / 5)
        float2 t1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
        float2 t2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
        float2 a1 = make_float2(fmaf(c2, t2.x, fmaf(c1, t1.x, v[0].x)), fmaf(c2, t2.y, fmaf(c1, t1.y, v[0].y)));
        float2 a2 = make_float2(fmaf(c1, t2.x, fmaf(c2, t1.x, v[0].x)), fmaf(c1, t2.y, fmaf(c2, t1.y, v[0].y)));
        float2 b1 = mul_mi(make_float2(fmaf(s2, d2.x, s1 * d1.x), fmaf(s2, d2.y, s1 * d1.y)));
        float2 b2 = mul_mi(make_float2(fmaf(-s1, d2.x, s2 * d1.x), fmaf(-s1, d2.y, s2 * d1.y)));
        v[0] = cadd(v[0], cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    }
};

template <> struct Dft<8> {
    static __device__ __forceinline__ void run(float2* v) {
        const float h = 0.70710678118654752f;
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4>::run(e);
        Dft<4>::run(o);
        // o_k *= e^{-i pi k / 4}
        float2 o1 = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
        float2 o2 = mul_mi(o[2]);
        float2 o3 = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

// ---- compile-time radix plan: the power of two as 8s (a leftover 2^1 or
// 2^2 becomes 4x4 or 4 when there are enough factors), then 3s, then 5s.
// Powers of two first keep the sub-length L of every pass a power of two
// until the odd radices, so the pass's index split (bf mod L, bf / L) is a
// mask and a shift, and its strided LDS positions are constant offsets from
// one padded base (see lds_pad_step).

struct RadixPlan {
    int np;
    int r[24];
};

constexpr RadixPlan make_plan(int len) {
    RadixPlan p{0, {}};
    int k = 0;
    while (len % 2 == 0) { ++k; len /= 2; }
    int e8 = k / 3, rem = k % 3;
    if (rem == 1 && e8 >= 1) { --e8; for (int i = 0; i < e8; ++i) p.r[p.np++] = 8; p.r[p.np++] = 4; p.r[p.np++] = 4; }
    else {
        for (int i = 0; i < e8; ++i) p.r[p.np++] = 8;
        if (rem == 1) p.r[p.np++] = 2;
        if (rem == 2) p.r[p.np++] = 4;
    }
    while (len % 3 == 0) { p.r[p.np++] = 3; len /= 3; }
    while (len % 5 == 0) { p.r[p.np++] = 5; len /= 5; }
    if (len != 1) p.np = -1;  // unsupported factor
    return p;
}

constexpr bool length_ok(int len) { return len >= 2 && make_plan(len).np > 0; }

// LDS layout of one line of length LEN: element i lives at i + i/32 (one pad
// slot per 32 elements, so strided butterfly writes spread over the banks);
// lines are LDS_LS(LEN) elements apart.
constexpr int lds_ls(int len) { return len + (len >> 5) + 1; }
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }
// Position of element e + m*STRIDE, m = 0..R-1, given p = lds_pad(e), as p
// plus a constant (an immediate offset of the LDS instruction) where the
// layout allows:
//  - STRIDE a multiple of 32: the pad grows by STRIDE/32 per step;
//  - STRIDE dividing 32 and e = c*GROUP + j with j < STRIDE, where GROUP =
//    STRIDE*R is a multiple of 32 (then e mod 32 = j, and the step m crosses
//    (m*STRIDE)/32 block boundaries whatever j is) or a divisor of 32 (then
//    all R positions share e's block); GROUP = 0 stands for e < STRIDE.
// Otherwise the position is computed per element.
template <int STRIDE, int GROUP>
__device__ __forceinline__ int lds_pad_step(int p, int e, int m) {
    if constexpr (STRIDE % 32 == 0) return p + m * (STRIDE + STRIDE / 32);
    else if constexpr (32 % STRIDE == 0 && (GROUP % 32 == 0 || 32 % GROUP == 0))
        return p + m * STRIDE + ((m * STRIDE) >> 5);
    else return lds_pad(e + m * STRIDE);
}

// Twiddles w^m, m = 1..R-1, from w = w^1 by a shallow product tree (at most
// three roundings deep), so each butterfly loads a single table entry.
template <int R>
__device__ __forceinline__ void twiddle_powers(float2 w1, float2* w) {
    w[1] = w1;
    if constexpr (R >= 3) w[2] = cmul(w1, w1);
    if constexpr (R >= 4) w[3] = cmul(w[2], w1);
    if constexpr (R >= 5) w[4] = cmul(w[2], w[2]);
    if constexpr (R >= 8) {
        w[5] = cmul(w[4], w1);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
    }
}

// One Stockham pass of radix R over B lines (line b at buf + b*LS), sub-length L.
template <int LEN, int R, int L, int B, int NT, int LS>
__device__ __forceinline__ void stockham_pass(float2* buf, const float2* __restrict__ tw, int tid) {
    static_assert(R == 2 || R == 3 || R == 4 || R == 5 || R == 8, "radix");
    constexpr int NB = LEN / R;                 // butterflies per line
    constexpr int TOT = NB * B;
    constexpr int IT = (TOT + NT - 1) / NT;
    constexpr bool FULL = (TOT % NT) == 0;
    float2 v[IT][R];
    float2 w1[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = tid + it * NT;
        if (FULL || b < TOT) {
            const int line = b / NB;
            const int bf = b - line * NB;
            const float2* src = buf + line * LS;
            const int pb = lds_pad(bf);
#pragma unroll
            for (int m = 0; m < R; ++m) v[it][m] = src[lds_pad_step<NB, 0>(pb, bf, m)];
            // the twiddle is requested before the barrier, so its latency
            // overlaps the wait for the other waves
            if constexpr (L > 1) w1[it] = tw[(bf % L) * (LEN / (L * R))];
        }
    }
    lds_sync();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = tid + it * NT;
        if (FULL || b < TOT) {
            const int line = b / NB;
            const int bf = b - line * NB;
            const int j = bf % L;
            const int k = bf / L;
            if constexpr (L > 1) {
                float2 w[R];
                twiddle_powers<R>(w1[it], w);
#pragma unroll
                for (int m = 1; m < R; ++m) v[it][m] = cmul(v[it][m], w[m]);
            }
            Dft<R>::run(v[it]);
            float2* dst = buf + line * LS;
            const int o = k * (L * R) + j;
            const int po = lds_pad(o);
#pragma unroll
            for (int m = 0; m < R; ++m) dst[lds_pad_step<L, L * R>(po, o, m)] = v[it][m];
        }
    }
    lds_sync();
}

template <int LEN, int P, int L, int B, int NT, int LS>
__device__ __forceinline__ void fft_passes(float2* buf, const float2* __restrict__ tw, int tid) {
    constexpr RadixPlan plan = make_plan(LEN);
    if constexpr (P < plan.np) {
        constexpr int R = plan.r[P];
        stockham_pass<LEN, R, L, B, NT, LS>(buf, tw, tid);
        fft_passes<LEN, P + 1, L * R, B, NT, LS>(buf, tw, tid);
    }
}

// Forward FFT of B lines of length LEN in LDS (line b at buf + b*lds_ls(LEN),
// element i at lds_pad(i)). All NT threads of the workgroup must call it; the
// caller barriers before.
template <int LEN, int B, int NT>
__device__ __forceinline__ void fft_lds(float2* buf, const float2* __restrict__ tw, int tid) {
    static_assert(length_ok(LEN), "FFT length must be 2^a 3^b 5^c");
    fft_passes<LEN, 0, 1, B, NT, lds_ls(LEN)>(buf, tw, tid);
}

// ---- register-in / register-out forms
// The first radix pass can take its inputs straight from registers and the
// last pass can leave its outputs in registers, which saves the LDS round
// trips of staging the input and of reading back the result (and two
// barriers). For B lines of length LEN with plan r[0..np-1] (np >= 2):
//   first pass: butterfly b = tid + it*NT (< B*NB0, NB0 = LEN/R0) of line
//     b / NB0 holds x[bf + m*NB0], m < R0 (bf = b mod NB0), in v[it][m];
//   last pass: butterfly b (< B*NBL, NBL = LEN/RL) leaves X[bf + m*NBL] in
//     out[it][m].
template <int LEN, int B, int NT>
struct FftRegIO {
    static constexpr RadixPlan plan = make_plan(LEN);
    static constexpr int NP = plan.np;
    static constexpr int R0 = plan.r[0];
    static constexpr int NB0 = LEN / R0;
    static constexpr int IT0 = (NB0 * B + NT - 1) / NT;
    static constexpr int RL = plan.r[NP - 1];
    static constexpr int NBL = LEN / RL;
    static constexpr int ITL = (NBL * B + NT - 1) / NT;
    static constexpr int LS = lds_ls(LEN);
};

// First pass (L = 1, no twiddles) from registers into LDS; v is clobbered.
// The caller barriers afterwards.
template <int LEN, int B, int NT, int IT, int R>
__device__ __forceinline__ void fft_first_from_regs(float2 (&v)[IT][R], float2* buf, int tid) {
    using IO = FftRegIO<LEN, B, NT>;
    static_assert(IT == IO::IT0 && R == IO::R0, "register layout of the first pass");
    constexpr bool FULL = ((IO::NB0 * B) % NT) == 0;
#pragma unroll
    for (int it = 0; it < IO::IT0; ++it) {
        const int b = tid + it * NT;
        if (FULL || b < IO::NB0 * B) {
            const int line = b / IO::NB0;
            const int bf = b - line * IO::NB0;
            Dft<IO::R0>::run(v[it]);
            float2* dst = buf + line * IO::LS;
            const int po = lds_pad(bf * IO::R0);
#pragma unroll
            for (int m = 0; m < IO::R0; ++m) dst[lds_pad_step<1, IO::R0>(po, bf * IO::R0, m)] = v[it][m];
        }
    }
}

// Passes P .. np-2 in LDS (each ends with a barrier).
template <int LEN, int P, int L, int B, int NT, int LS>
__device__ __forceinline__ void fft_mid_passes(float2* buf, const float2* __restrict__ tw, int tid) {
    constexpr RadixPlan plan = make_plan(LEN);
    if constexpr (P < plan.np - 1) {
        constexpr int R = plan.r[P];
        stockham_pass<LEN, R, L, B, NT, LS>(buf, tw, tid);
        fft_mid_passes<LEN, P + 1, L * R, B, NT, LS>(buf, tw, tid);
    }
}

// Last pass from LDS into registers (no LDS writes, no trailing barrier).
template <int LEN, int B, int NT, int IT, int RR>
__device__ __forceinline__ void fft_last_to_regs(const float2* buf, const float2* __restrict__ tw, int tid,
                                                 float2 (&out)[IT][RR]) {
    using IO = FftRegIO<LEN, B, NT>;
    static_assert(IT == IO::ITL && RR == IO::RL, "register layout of the last pass");
    constexpr int R = IO::RL;
    constexpr bool FULL = ((IO::NBL * B) % NT) == 0;
#pragma unroll
    for (int it = 0; it < IO::ITL; ++it) {
        const int b = tid + it * NT;
        if (FULL || b < IO::NBL * B) {
            const int line = b / IO::NBL;
            const int bf = b - line * IO::NBL;
            const float2* src = buf + line * IO::LS;
            const int pb = lds_pad(bf);
#pragma unroll
            for (int m = 0; m < R; ++m) out[it][m] = src[lds_pad_step<IO::NBL, 0>(pb, bf, m)];
            float2 w[R];
            twiddle_powers<R>(tw[bf], w);
#pragma unroll
            for (int m = 1; m < R; ++m) out[it][m] = cmul(out[it][m], w[m]);
            Dft<R>::run(out[it]);
        }
    }
}

// Whole transform with register input and output: first pass from v, middle
// passes in LDS, last pass into out. The caller barriers before the call if
// the LDS lines are still being read.
template <int LEN, int B, int NT, int I0, int R0, int IL, int RL>
__device__ __forceinline__ void fft_regs(float2 (&v)[I0][R0], float2* buf, const float2* __restrict__ tw, int tid,
                                         float2 (&out)[IL][RL]) {
    using IO = FftRegIO<LEN, B, NT>;
    static_assert(IO::NP >= 2, "register form needs at least two passes");
    fft_first_from_regs<LEN, B, NT>(v, buf, tid);
    lds_sync();
    fft_mid_passes<LEN, 1, IO::R0, B, NT, IO::LS>(buf, tw, tid);
    fft_last_to_regs<LEN, B, NT>(buf, tw, tid, out);
}

// Threads per workgroup used for a transform of B lines of length LEN.
// Threads for the row/column kernels, whose per-thread register arrays shrink
// with more threads: 512 from length 1024 on.
constexpr int line_threads(int len) { return len >= 1024 ? 512 : (len >= 256 ? 256 : (len >= 64 ? 128 : 64)); }

// Threads of the row kernels (F1, A4) and column kernels (F2, A3) for lines of
// length 1024 and more (compile-time tuning knobs).
#ifndef RN_ROW_NT
#define RN_ROW_NT 1024
#endif
#ifndef RN_COL_NT
#define RN_COL_NT 512
#endif
#ifndef RN_RAY_NT
#define RN_RAY_NT 512
#endif
constexpr int row_threads(int len) { return len >= 1024 ? RN_ROW_NT : line_threads(len); }
constexpr int col_threads(int len) { return len >= 1024 ? RN_COL_NT : line_threads(len); }

constexpr int fft_threads(int len, int b) {
    int work = len * b / 8;
    return work >= 1024 ? 512 : (work >= 256 ? 256 : (work >= 128 ? 128 : 64));
}
// Threads of the ray kernels (F4, A1: two rays of length len per workgroup).
// These launches hold only n_views/2 workgroups, so long rays get more
// threads than their butterfly count asks for: more waves in flight per CU.
constexpr int ray_threads(int len) { return len >= 2048 ? RN_RAY_NT : fft_threads(len, 1); }

}  // namespace rn

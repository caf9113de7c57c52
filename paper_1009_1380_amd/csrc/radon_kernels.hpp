// radon_kernels.hpp - gfx950 kernels of the Fourier-slice Radon NUFFT.
//
// Section "fast radon transform", paragraph 1: a 2D FFT of the image on a
// regular grid, interpolation onto a polar grid, 1D inverse FFTs along every
// radial line. Paragraphs 2-3: the interpolation is gridding (convolution of
// the samples with a kernel evaluated at regular grid points, and back).
//
// The image is real, so its oversampled transform Ghat is Hermitian and only
// the half plane mx in [0, G/2] is formed (G = 2n). That grid is stored
// transposed, grid[mx * G + my], so both FFT passes and the gridding read and
// write whole contiguous lines:
//
//   forward  F1  image rows (pairs packed as one complex line) -> row FFT,
//                split into real-input spectra, stored T1[mx][i]   (n+1 x n)
//            F2  each T1 line -> column FFT -> grid[mx][my]       (n+1 x G)
//            F3  per grid tile: Kaiser-Bessel interpolation, from an LDS copy
//                of the tile, of the samples sorted into it -> Xr[a][|q|]
//            F4  per pair of rays: complex-to-real inverse FFT -> sinogram
//   adjoint  A1  per pair of rays: real-to-complex FFT -> Yh[a][q], q <= N/2
//            A2  per output strip of tiles: deterministic spreading of the
//                samples that reach the strip into an LDS accumulator, no
//                atomics on floating-point data
//            A3  each grid line -> inverse column FFT, keep n rows -> T1
//            A4  pairs of image rows: complex-to-real inverse row FFT,
//                keep n columns, deapodize -> image
//
// Every length-G transform with n nonzero inputs (or n needed outputs) is done
// as two length-n transforms: for G = 2n, frequency m = 2k + r satisfies
//   sum_p x[p] e^{-2 pi i m p/G} = FFT_n( x[p] e^{-i pi r p/n} )[k].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"

namespace rn {

// ---------------------------------------------------------------- helpers

// Cubic pieces of the Kaiser-Bessel table per unit of t (the host builds the
// table with the same count).
constexpr int KB_S = 32;

// Kaiser-Bessel weights phi(t), 0 <= t <= W/2, from a table of cubic pieces,
// KB_S pieces per unit of t (c.x + c.y f + c.z f^2 + c.w f^3 on piece
// floor(t KB_S) at f = frac(t KB_S)). A footprint along one axis has W points;
// for a sample with fraction f in [0, 1], point k lies at distance
// f + (W/2 - 1 - k) for k < W/2 and (k - W/2 + 1) - f otherwise. With
// f KB_S = i + r (i integer, r in [0, 1]; f may have rounded up to 1), the
// near points read piece (W/2 - 1 - k) KB_S + i at fraction r and the far
// points piece (k - W/2 + 1) KB_S - i - 1 at fraction 1 - r (the end of the
// previous piece when r = 0), so one split serves all W table reads, which
// differ only by constant offsets, and every index stays in the table.
// Only the two outer points (k = 0, W-1) can reach the support edge W/2,
// where phi jumps from 1/I0(beta) (9e-4 for W = 4) to 0; whether they are
// inside is decided once per sample in float64 (the record's edge flags, see
// SampleRec), and the callers zero the points outside.
template <int W>
__device__ __forceinline__ void kb_weights(float f, const float4* __restrict__ tab, float (&w)[W]) {
    const float x = f * (float)KB_S;
    const int i = min((int)x, KB_S - 1);
    const float r = x - (float)i, rb = 1.0f - r;
    const float4* near = tab + i;
    const float4* far = tab + (KB_S - 1 - i);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const bool nr = k < W / 2;
        const float4 c = nr ? near[(W / 2 - 1 - k) * KB_S] : far[(k - W / 2) * KB_S];
        const float t = nr ? r : rb;
        w[k] = fmaf(fmaf(fmaf(c.w, t, c.z), t, c.y), t, c.x);
    }
}

struct SampleGeom {
    double u, v;     // grid coordinates
    int bu, bv;      // floor(u), floor(v)
    float fu, fv;    // u - floor(u), v - floor(v), rounded to float32
};

// Grid coordinates of polar sample q of a view with direction (c, s):
// u = (G q / N) * c, v = (G q / N) * s, one float64 division and one
// multiplication each, so floor() agrees bit-for-bit with any IEEE code that
// does the same operations on the same cos/sin.
__device__ __forceinline__ SampleGeom sample_geom(double c, double s, int q, int G, int N) {
#pragma clang fp contract(off)
    double fq = (double)(G * q) / (double)N;
    double u = fq * c;
    double v = fq * s;
    double fbu = floor(u), fbv = floor(v);
    SampleGeom g;
    g.u = u;
    g.v = v;
    g.bu = (int)fbu;
    g.bv = (int)fbv;
    g.fu = (float)(u - fbu);
    g.fv = (float)(v - fbv);
    return g;
}

__device__ __forceinline__ int mod_pos(int a, int m) {
    int r = a % m;
    return r < 0 ? r + m : r;
}

// a mod G for a in [-G, 2G) (one compare and add instead of an integer division).
__device__ __forceinline__ int wrap_g(int a, int G) { return a < 0 ? a + G : (a >= G ? a - G : a); }


// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Renumber block b of nb so that each XCD gets a contiguous run of
// logical blocks: neighbouring blocks, which share cache lines, then run
// together on one XCD.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, k = b >> 3, per = nb >> 3, rem = nb & 7;
    return x * per + min(x, rem) + k;
}

// ---------------------------------------------------------------- F1
// 2 NLN image rows per workgroup, packed as NLN complex lines z_p = row 2p +
// i row 2p+1. Row i holds py = i - n/2, column j holds px = j - n/2 (stored
// at px mod n in the length-n FFT). The even frequencies mx = 2k are the
// length-n FFT of z_p, the odd ones mx = 2k+1 that of z_p e^{-i pi px/n};
// the lines are transformed together for the even frequencies, then for the
// odd ones, and each frequency's 2 NLN outputs are written to
// T1[mx][i0..i0+2NLN-1] (16 NLN contiguous bytes) straight from LDS. Only the
// deapodized inputs wait in registers.
//
// Complex lines per workgroup (row_lines): 2 (four rows), or n/512 for
// n = 2048 and 2560, so that the n rows form one round of one workgroup per
// CU (256 CUs; at 2560 the 106 KB of LDS lines, at 2048 the registers, admit
// one workgroup per CU).
// With two lines, 2560 rows make 640 workgroups, two resident per CU, and a
// fifth of them ran in a second round.
constexpr int row_lines(int len) { return (len == 2048 || len == 2560) ? len / 512 : 2; }
// Waves per SIMD the row kernels are compiled for: with 1024 threads and two
// lines, 8 holds two workgroups on a CU (at most 64 VGPRs per lane), which
// lines of up to 2560 points fit without spilling; one workgroup per CU
// needs 4.
constexpr int row_waves(int len) { return row_lines(len) > 2 ? 4 : (len <= 2560 ? 8 : 4); }
// workgroups of a row pass over n rows
constexpr int row_blocks(int n) { return (n + 2 * row_lines(n) - 1) / (2 * row_lines(n)); }

template <int NL, int NT>
__device__ __forceinline__ void f1_store(float2* __restrict__ T1, const float2* lds, int m, int k, int kc, int i0,
                                         int p) {
    // line p gives rows i0 + 2p and i0 + 2p + 1 (16 bytes); consecutive lanes
    // take the lines p = 0 .. NLN-1 of one frequency, so one store instruction
    // fills whole 16 NLN-byte pieces
    constexpr int LS = lds_ls(NL);
    const float2 zk = lds[p * LS + lds_pad(k)];
    const float2 zc = cconj(lds[p * LS + lds_pad(kc)]);
    const float2 sm = cadd(zk, zc), df = csub(zk, zc);
    const float2 o0 = make_float2(0.5f * sm.x, 0.5f * sm.y);
    const float2 o1 = make_float2(0.5f * df.y, -0.5f * df.x);   // (zk - zc) / 2i
    float2* dst = T1 + (size_t)m * NL + i0 + 2 * p;
    if (i0 + 2 * p + 1 < NL) *reinterpret_cast<float4*>(dst) = make_float4(o0.x, o0.y, o1.x, o1.y);
}

template <int NL, int NT>
__device__ __forceinline__ void f1_body(int bid_, int nblk_, const float* __restrict__ img, float2* __restrict__ T1,
                                               const float* __restrict__ psi_inv,
                                               const float2* __restrict__ shift,
                                               const float2* __restrict__ tw) {
    constexpr int LS = lds_ls(NL);
    constexpr int NLN = row_lines(NL);
    __shared__ float2 lds[NLN * LS];
    const int tid = threadIdx.x;
    const int i0 = 2 * NLN * xcd_block(bid_, nblk_);
    using IO = FftRegIO<NL, NLN, NT>;
    if constexpr (IO::NP >= 2) {
        // The deapodized inputs are loaded straight into the first butterflies:
        // butterfly b = tid + it NT (line b / NB0) takes FFT positions
        // q = bf + m NB0, which hold pixel j = (q + n/2) mod n of rows
        // i0 + 2 line and i0 + 2 line + 1. They wait in z for the odd pass.
        float2 z[IO::IT0][IO::R0], v[IO::IT0][IO::R0];
#pragma unroll
        for (int it = 0; it < IO::IT0; ++it) {
            const int b = tid + it * NT;
            const int line = b / IO::NB0, bf = b - line * IO::NB0;
            const int r0 = i0 + 2 * line;
            const bool ok = b < IO::NB0 * NLN;
            const bool oka = ok && r0 < NL, okb = ok && r0 + 1 < NL;
            const float sa = oka ? psi_inv[r0] : 0.f;
            const float sb = okb ? psi_inv[r0 + 1] : 0.f;
#pragma unroll
            for (int m = 0; m < IO::R0; ++m) {
                const int j = (bf + m * IO::NB0 + NL / 2) % NL;
                const float ra = oka ? img[(size_t)r0 * NL + j] : 0.f;
                const float rb = okb ? img[(size_t)(r0 + 1) * NL + j] : 0.f;
                const float pj = ok ? psi_inv[j] : 0.f;
                z[it][m] = make_float2(ra * sa * pj, rb * sb * pj);
                v[it][m] = z[it][m];
            }
        }
        fft_first_from_regs<NL, NLN, NT>(v, lds, tid);
        lds_sync();
        fft_passes<NL, 1, IO::R0, NLN, NT, LS>(lds, tw, tid);
        for (int e = tid; e < NLN * (NL / 2 + 1); e += NT) {
            const int k = e / NLN;
            f1_store<NL, NT>(T1, lds, 2 * k, k, (NL - k) % NL, i0, e - k * NLN);
        }
        lds_sync();
#pragma unroll
        for (int it = 0; it < IO::IT0; ++it) {
            const int b = tid + it * NT;
            const int line = b / IO::NB0, bf = b - line * IO::NB0;
            const bool ok = b < IO::NB0 * NLN;
#pragma unroll
            for (int m = 0; m < IO::R0; ++m) {
                const int j = (bf + m * IO::NB0 + NL / 2) % NL;
                v[it][m] = ok ? cmul(z[it][m], shift[j]) : make_float2(0.f, 0.f);
            }
        }
        fft_first_from_regs<NL, NLN, NT>(v, lds, tid);
        lds_sync();
        fft_passes<NL, 1, IO::R0, NLN, NT, LS>(lds, tw, tid);
        for (int e = tid; e < NLN * (NL / 2); e += NT) {
            const int k = e / NLN;
            f1_store<NL, NT>(T1, lds, 2 * k + 1, k, NL - 1 - k, i0, e - k * NLN);
        }
    } else {
        constexpr int PJ = (NL + NT - 1) / NT;       // pixels px per thread and row
        float2 z[PJ][NLN];
#pragma unroll
        for (int c = 0; c < PJ; ++c) {
            const int j = tid + c * NT;
            float r[2 * NLN];
#pragma unroll
            for (int q = 0; q < 2 * NLN; ++q) r[q] = (j < NL && i0 + q < NL) ? img[(size_t)(i0 + q) * NL + j] : 0.f;
            if (j < NL) {
                const float pj = psi_inv[j];
                const int pos = lds_pad((j + NL / 2) % NL);
#pragma unroll
                for (int p = 0; p < NLN; ++p) {
                    const int r0 = i0 + 2 * p;
                    const float sa = r0 < NL ? psi_inv[r0] : 0.f;
                    const float sb = r0 + 1 < NL ? psi_inv[r0 + 1] : 0.f;
                    z[c][p] = make_float2(r[2 * p] * sa * pj, r[2 * p + 1] * sb * pj);
                    lds[p * LS + pos] = z[c][p];
                }
            }
        }
        lds_sync();
        fft_lds<NL, NLN, NT>(lds, tw, tid);
        for (int e = tid; e < NLN * (NL / 2 + 1); e += NT) {
            const int k = e / NLN;
            f1_store<NL, NT>(T1, lds, 2 * k, k, (NL - k) % NL, i0, e - k * NLN);
        }
        lds_sync();
#pragma unroll
        for (int c = 0; c < PJ; ++c) {
            const int j = tid + c * NT;
            if (j < NL) {
                const int pos = lds_pad((j + NL / 2) % NL);
                const float2 sh = shift[j];
#pragma unroll
                for (int p = 0; p < NLN; ++p) lds[p * LS + pos] = cmul(z[c][p], sh);
            }
        }
        lds_sync();
        fft_lds<NL, NLN, NT>(lds, tw, tid);
        for (int e = tid; e < NLN * (NL / 2); e += NT) {
            const int k = e / NLN;
            f1_store<NL, NT>(T1, lds, 2 * k + 1, k, NL - 1 - k, i0, e - k * NLN);
        }
    }
}

// ---------------------------------------------------------------- F2
// One half-plane line mx per workgroup: FFT along py of T1[mx][.] into
// grid[mx][my], my = 2k + r from two length-n transforms done one after the
// other in one LDS line. The input and the r = 0 result wait in registers;
// each transform takes its first pass from registers and leaves its last
// pass in registers (FftRegIO), so the line is read from HBM straight into
// the first butterflies and the results go from the last butterflies
// straight to HBM.
template <int NL, int NT>
__device__ __forceinline__ void f2_body(int bid_, int nblk_, const float2* __restrict__ T1, float2* __restrict__ grid,
                                               const float2* __restrict__ shift,
                                               const float2* __restrict__ tw) {
    __shared__ float2 lds[lds_ls(NL)];
    const int tid = threadIdx.x;
    const int mx = bid_;
    const float2* src = T1 + (size_t)mx * NL;
    float4* dst = reinterpret_cast<float4*>(grid + (size_t)mx * (2 * NL));
    using IO = FftRegIO<NL, 1, NT>;
    if constexpr (IO::NP >= 2) {
        // FFT position p holds py = p (mod n), i.e. T1 index i = (p + n/2) mod n
        float2 c[IO::IT0][IO::R0], v[IO::IT0][IO::R0];
        float2 X0[IO::ITL][IO::RL], X1[IO::ITL][IO::RL];
#pragma unroll
        for (int it = 0; it < IO::IT0; ++it) {
            const int b = tid + it * NT;
#pragma unroll
            for (int m = 0; m < IO::R0; ++m) {
                const int i = (b + m * IO::NB0 + NL / 2) % NL;
                c[it][m] = (b < IO::NB0) ? src[i] : make_float2(0.f, 0.f);
                v[it][m] = c[it][m];
            }
        }
        fft_regs<NL, 1, NT>(v, lds, tw, tid, X0);
        lds_sync();
#pragma unroll
        for (int it = 0; it < IO::IT0; ++it) {
            const int b = tid + it * NT;
#pragma unroll
            for (int m = 0; m < IO::R0; ++m) {
                const int i = (b + m * IO::NB0 + NL / 2) % NL;
                v[it][m] = (b < IO::NB0) ? cmul(c[it][m], shift[i]) : make_float2(0.f, 0.f);
            }
        }
        fft_regs<NL, 1, NT>(v, lds, tw, tid, X1);
#pragma unroll
        for (int it = 0; it < IO::ITL; ++it) {
            const int b = tid + it * NT;
            if (b < IO::NBL) {
#pragma unroll
                for (int m = 0; m < IO::RL; ++m) {
                    const int k = b + m * IO::NBL;
                    dst[k] = make_float4(X0[it][m].x, X0[it][m].y, X1[it][m].x, X1[it][m].y);
                }
            }
        }
    } else {
        constexpr int PE = (NL + NT - 1) / NT;
        float2 c[PE], z0[PE];
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int i = tid + e * NT;
            if (i < NL) {
                c[e] = src[i];
                lds[lds_pad((i + NL / 2) % NL)] = c[e];
            }
        }
        lds_sync();
        fft_lds<NL, 1, NT>(lds, tw, tid);
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int k = tid + e * NT;
            if (k < NL) z0[e] = lds[lds_pad(k)];
        }
        lds_sync();
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int i = tid + e * NT;
            if (i < NL) lds[lds_pad((i + NL / 2) % NL)] = cmul(c[e], shift[i]);
        }
        lds_sync();
        fft_lds<NL, 1, NT>(lds, tw, tid);
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int k = tid + e * NT;
            if (k < NL) {
                const float2 o = lds[lds_pad(k)];
                dst[k] = make_float4(z0[e].x, z0[e].y, o.x, o.y);
            }
        }
    }
}

// ---------------------------------------------------------------- samples
// Sample ids: 0..M-1 are the polar samples j = a*N + q + N/2 (M = n_views*N);
// M..M+n_views-1 are the mirrored Nyquist samples (view a at q = +N/2).
__device__ __forceinline__ void decode_sample(int v, int M, int ND, int& a, int& q) {
    if (v < M) {
        // a = v / ND: the float64 quotient (v < 2^30) is within one of the
        // integer one, then one correction step each way makes it exact
        a = (int)((double)v * (1.0 / (double)ND));
        int r = v - a * ND;
        if (r < 0) { --a; r += ND; }
        if (r >= ND) { ++a; r -= ND; }
        q = r - ND / 2;
    } else {
        a = v - M;
        q = ND / 2;
    }
}

// Centred grid coordinate of the first footprint point: (floor - W/2 + 1 + G/2) mod G.
// (b is floor(u) or floor(v), within [-G/2 - 1, G/2]).
__device__ __forceinline__ int footprint_origin(int b, int W, int G) { return wrap_g(b - W / 2 + 1 + G / 2, G); }

// Tile columns whose samples the forward interpolates: the Hermitian half
// plane mx in [0, G/2] (centred columns ntl/2..ntl-1 and column 0, which
// holds mx = G/2) plus column ntl/2-1 (mx in [-T, 0)), so that footprints
// straddling mx = 0 are taken whole.
__device__ __forceinline__ bool forward_column(int cx, int ntl) { return cx == 0 || cx >= ntl / 2 - 1; }

#ifndef RN_A2_GX
#define RN_A2_GX 2
#endif
constexpr int A2_GX = RN_A2_GX;   // tile columns per strip (at most)
constexpr int A2_NR = A2_GX + 3;  // visit ranges of a strip

// Spreading work item: a slice of the visit list of one output strip. The
// list is the concatenation of A2_NR ranges of the sorted samples (start rs,
// length rl), taken from the bin offsets when the plan is built, so that the
// kernel reads them with the item instead of looking them up after it.
struct TileItem {
    int cx, cy;      // first tile of the strip, centred tile coordinates
    int start;       // first visit of the slice in the strip's list
    int count;       // number of visits
    int slot;        // -1 writes the grid, else partial slot
    int gx;          // tile columns of the strip
    int plan;        // batches: index of the item's plan in the batch (else 0)
    int pad;
    int rs[A2_NR], rl[A2_NR];
};

// Per-sample record in sorted order, built once per plan so that the
// gridding kernels need no geometry of their own:
//   org   footprint origin o_u (bits 0..12) and o_v (bits 16..28), centred
//         grid coordinates; bits 13/14 (u) and 29/30 (v): the first / last
//         footprint point lies outside the support, |u - m| >= W/2 in float64
//   fu,fv u - floor(u), v - floor(v) (float32, as sample_geom gives them)
//   info  bits 0..28: index a*(N/2+1) + t of the sample's ray-spectrum entry
//         (t = |q|, or N/2 for both Nyquist samples); bit 29: q in (-N/2, 0)
//         (the entry is the conjugate); bit 30: mirrored Nyquist sample;
//         bit 31: the forward interpolation evaluates this sample (one member
//         of each conjugate pair, chosen by the rule of F3 below).
struct SampleRec {
    int org;
    float fu, fv;
    int info;
};
constexpr int REC_ORG_MASK = (1 << 13) - 1;
constexpr int REC_U_NEAR_OUT = 1 << 13, REC_U_FAR_OUT = 1 << 14;
constexpr int REC_V_NEAR_OUT = 1 << 29, REC_V_FAR_OUT = 1 << 30;
constexpr int REC_IDX_MASK = (1 << 29) - 1;
constexpr int REC_CONJ = 1 << 29;
constexpr int REC_MIRROR = 1 << 30;
constexpr unsigned REC_F3 = 1u << 31;

__device__ __forceinline__ SampleRec load_rec(const SampleRec* __restrict__ recs, int pos) {
    const int4 r = reinterpret_cast<const int4*>(recs)[pos];
    SampleRec o;
    o.org = r.x;
    o.fu = __int_as_float(r.y);
    o.fv = __int_as_float(r.z);
    o.info = r.w;
    return o;
}

// ---------------------------------------------------------------- F3
// Kaiser-Bessel interpolation of the polar samples from the half-plane grid.
// One workgroup per super-tile of 2 x 2 bins (the bins of tile columns cx and
// cx+1 mod ntl, rows cy and cy+1). The super-tile and its (W-1) halo are
// staged in LDS (points with mx < 0 read as conjugates of their mirror, wrap
// mod G), then every sample whose footprint origin is in one of the four bins
// is interpolated from LDS. Of each conjugate pair (q, -q) exactly one member
// is evaluated: q >= 0 when its origin tile is a forward column, else -q
// (result conjugated); the pair (-N/2, +N/2) likewise. Results go to
// Xr[a][t], t = |q| (t = N/2: Nyquist).
//
// The item carries the sorted-sample ranges of its bins (taken from the bin
// offsets when the plan is built), so that its first records and its region
// are requested right after the item itself.
struct F3Item {
    int cx, cy;      // first bin of the super-tile, centred tile coordinates
    int nbx;         // bins of the super-tile along u that are forward columns (1 or 2)
    int start;       // first sample of the slice within the concatenated bins
    int count;       // samples in this slice
    int plan;        // batches: index of the item's plan in the batch (else 0)
    int s[4];        // first sorted sample of bins (cx, cy), (cx+1, cy), (cx, cy+1), (cx+1, cy+1)
    int n[3];        // samples of the first three (the second counts only when nbx = 2)
    int pad;
};

// Persistent: workgroup b takes items b, b + gridDim.x, ... (the grid is the
// number of workgroups that fit on the device at once). Sample geometry comes
// precomputed from the plan's per-sample records.
constexpr int F3_CHUNK = 2048;   // samples per work item

// Waves per SIMD the interpolation kernel is compiled for when W <= 6.
#ifndef RN_F3_WPE
#define RN_F3_WPE 6
#endif
// One work item: stage the super-tile's region in `tile`, interpolate its
// samples. `kbt` holds the kernel's cubic pieces in LDS.
template <int W, int T, int NT>
__device__ __forceinline__ void f3_item(const F3Item& it, const SampleRec* __restrict__ recs, const float2* __restrict__ grid,
                                        float2* __restrict__ Xr, int G, float2* tile, const float4* kbt, int tid) {
    constexpr int P = 2 * T + W - 1;
    constexpr int PP = P * P;
    constexpr int PE = (PP + NT - 1) / NT;            // staged points per thread
    {
        const int x0 = it.cx * T, y0 = it.cy * T;
        const int s0 = it.s[0], n0 = it.n[0], s1 = it.s[1], n1 = it.n[1];
        const int s2 = it.s[2], n2 = it.n[2], s3 = it.s[3];
        auto position = [&](int k) {
            int u = it.start + k;
            if (u < n0) return s0 + u;
            if ((u -= n0) < n1) return s1 + u;
            if ((u -= n1) < n2) return s2 + u;
            return s3 + (u - n2);
        };
        // the first record is requested before the staging, and each next one
        // before the current one is interpolated, so record latency overlaps work
        SampleRec nxt{};
        if (tid < it.count) nxt = load_rec(recs, position(tid));
        lds_sync();   // the previous item's samples are done with the tile
        // stage the region; points with mx < 0 hold the conjugate of their mirror
#pragma unroll
        for (int k = 0; k < PE; ++k) {
            const int e = tid + k * NT;
            if (e < PP) {
                const int lx = e / P, ly = e - lx * P;
                int mx = wrap_g(x0 + lx, G) - G / 2;        // in [-G/2, G/2)
                int my = wrap_g(y0 + ly, G) - G / 2;
                if (mx == -G / 2) mx = G / 2;
                const bool mirror = mx < 0;
                if (mirror) { mx = -mx; my = -my; }
                const float2 g = grid[(size_t)mx * G + wrap_g(my, G)];
                tile[e] = make_float2(g.x, mirror ? -g.y : g.y);
            }
        }
        lds_sync();
        for (int k = tid; k < it.count; k += NT) {
            const SampleRec r = nxt;
            if (k + NT < it.count) nxt = load_rec(recs, position(k + NT));
            if (!((unsigned)r.info & REC_F3)) continue;
            const int ox = wrap_g((r.org & REC_ORG_MASK) - x0, G);   // in [0, 2T)
            const int oy = wrap_g(((r.org >> 16) & REC_ORG_MASK) - y0, G);
            float wy[W], wx[W];
            kb_weights<W>(r.fv, kbt, wy);
            if (r.org & REC_V_NEAR_OUT) wy[0] = 0.f;
            if (r.org & REC_V_FAR_OUT) wy[W - 1] = 0.f;
            kb_weights<W>(r.fu, kbt, wx);
            if (r.org & REC_U_NEAR_OUT) wx[0] = 0.f;
            if (r.org & REC_U_FAR_OUT) wx[W - 1] = 0.f;
            const float2* src = tile + ox * P + oy;
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int al = 0; al < W; ++al) {
                float2 racc = make_float2(0.f, 0.f);
#pragma unroll
                for (int gm = 0; gm < W; ++gm) {
                    const float2 val = src[al * P + gm];
                    racc.x = fmaf(wy[gm], val.x, racc.x);
                    racc.y = fmaf(wy[gm], val.y, racc.y);
                }
                acc.x = fmaf(wx[al], racc.x, acc.x);
                acc.y = fmaf(wx[al], racc.y, acc.y);
            }
            const bool cj = (r.info & (REC_CONJ | REC_MIRROR)) != 0;
            Xr[r.info & REC_IDX_MASK] = cj ? cconj(acc) : acc;
        }
    }
}

// ---------------------------------------------------------------- F4
// Two rays per workgroup: y = Re((1/N) IFFT) of the Hermitian extension
// X[-q] = conj X[q] of Xr (bins 0 and N/2 taken as real); the two real
// outputs share one complex IFFT. Output bin d is s = d - N/2 at s mod N.
template <int ND, int NT>
__device__ __forceinline__ void f4_body(int bid_, int nblk_, const float2* __restrict__ Xr, float* __restrict__ sino,
                                               const float2* __restrict__ tw, int n_views) {
    constexpr int HQ = ND / 2 + 1;
    __shared__ float2 lds[lds_ls(ND)];
    const int tid = threadIdx.x;
    const int a0 = bid_ * 2;
    const bool has_b = a0 + 1 < n_views;
    const float2* xa = Xr + (size_t)a0 * HQ;
    const float2* xb = Xr + (size_t)(a0 + 1) * HQ;
    const float2 zero = make_float2(0.f, 0.f);
    const float inv = 1.0f / (float)ND;
    // Z = A + i B at position q (A, B the two rays' Hermitian spectra), stored
    // conjugated so the forward engine gives conj(IFFT)
    auto zin = [&](int q, float2 ga, float2 gb) {
        float2 A, B;
        if (q == 0 || q == ND / 2) {
            A = make_float2(ga.x, 0.f);
            B = make_float2(gb.x, 0.f);
        } else if (q < ND / 2) {
            A = ga;
            B = gb;
        } else {
            A = cconj(ga);
            B = cconj(gb);
        }
        return make_float2(A.x - B.y, -(A.y + B.x));
    };
    using IO = FftRegIO<ND, 1, NT>;
    if constexpr (IO::NP >= 2) {
        // the spectra are loaded straight into the first butterflies and the
        // rays written from the last ones
        float2 v[IO::IT0][IO::R0], Z[IO::ITL][IO::RL];
#pragma unroll
        for (int it = 0; it < IO::IT0; ++it) {
            const int b = tid + it * NT;
#pragma unroll
            for (int m = 0; m < IO::R0; ++m) {
                const int q = b + m * IO::NB0;
                const int s = q <= ND / 2 ? q : ND - q;
                const float2 ga = (b < IO::NB0) ? xa[s] : zero;
                const float2 gb = (b < IO::NB0 && has_b) ? xb[s] : zero;
                v[it][m] = zin(q, ga, gb);
            }
        }
        fft_regs<ND, 1, NT>(v, lds, tw, tid, Z);
#pragma unroll
        for (int it = 0; it < IO::ITL; ++it) {
            const int b = tid + it * NT;
            if (b < IO::NBL) {
#pragma unroll
                for (int m = 0; m < IO::RL; ++m) {
                    const int d = (b + m * IO::NBL + ND / 2) % ND;
                    const float2 z = cconj(Z[it][m]);
                    sino[(size_t)a0 * ND + d] = z.x * inv;
                    if (has_b) sino[(size_t)(a0 + 1) * ND + d] = z.y * inv;
                }
            }
        }
    } else {
        for (int q = tid; q < ND; q += NT) {
            const int s = q <= ND / 2 ? q : ND - q;
            lds[lds_pad(q)] = zin(q, xa[s], has_b ? xb[s] : zero);
        }
        lds_sync();
        fft_lds<ND, 1, NT>(lds, tw, tid);
        for (int d = tid; d < ND; d += NT) {
            const float2 z = cconj(lds[lds_pad((d + ND / 2) % ND)]);
            sino[(size_t)a0 * ND + d] = z.x * inv;
            if (has_b) sino[(size_t)(a0 + 1) * ND + d] = z.y * inv;
        }
    }
}

// ---------------------------------------------------------------- A1
// Two rays per workgroup: Yhat_a[q] = (1/N) sum_d y[a,d] e^{-2 pi i q s_d/N},
// q = 0..N/2; the q = N/2 (Nyquist) value is halved because it is spread
// once at its own position and once at the mirrored one. With a weight
// table wq (the ramp of the filtered adjoint) Yhat_a[q] is multiplied by
// wq[q]; wq = nullptr gives the plain adjoint.
template <int ND, int NT>
__device__ __forceinline__ void a1_body(int bid_, int nblk_, const float* __restrict__ sino, float2* __restrict__ Yh,
                                               const float2* __restrict__ tw, const float* __restrict__ wq,
                                               int n_views) {
    constexpr int HQ = ND / 2 + 1;
    __shared__ float2 lds[lds_ls(ND)];
    const int tid = threadIdx.x;
    const int a0 = bid_ * 2;
    // the two rays as one complex line: FFT position p holds detector
    // d = (p + ND/2) mod ND
    using IO = FftRegIO<ND, 1, NT>;
    if constexpr (IO::NP >= 2) {
        // straight into the first butterflies; the other passes run in LDS,
        // where the Hermitian split below finds both q and ND - q
        float2 v[IO::IT0][IO::R0];
#pragma unroll
        for (int it = 0; it < IO::IT0; ++it) {
            const int b = tid + it * NT;
#pragma unroll
            for (int m = 0; m < IO::R0; ++m) {
                const int d = (b + m * IO::NB0 + ND / 2) % ND;
                const float ya = (b < IO::NB0 && a0 < n_views) ? sino[(size_t)a0 * ND + d] : 0.f;
                const float yb = (b < IO::NB0 && a0 + 1 < n_views) ? sino[(size_t)(a0 + 1) * ND + d] : 0.f;
                v[it][m] = make_float2(ya, yb);
            }
        }
        fft_first_from_regs<ND, 1, NT>(v, lds, tid);
        lds_sync();
        fft_passes<ND, 1, IO::R0, 1, NT, IO::LS>(lds, tw, tid);
    } else {
        for (int d = tid; d < ND; d += NT) {
            const float ya = (a0 < n_views) ? sino[(size_t)a0 * ND + d] : 0.f;
            const float yb = (a0 + 1 < n_views) ? sino[(size_t)(a0 + 1) * ND + d] : 0.f;
            lds[lds_pad((d + ND / 2) % ND)] = make_float2(ya, yb);
        }
        lds_sync();
        fft_lds<ND, 1, NT>(lds, tw, tid);
    }
    const float sc = 0.5f / (float)ND;
    for (int q = tid; q < HQ; q += NT) {
        const float2 zq = lds[lds_pad(q)];
        const float2 zc = cconj(lds[lds_pad((ND - q) % ND)]);
        const float2 sm = cadd(zq, zc), df = csub(zq, zc);
        float h = (q == ND / 2) ? 0.5f * sc : sc;
        if (wq) h *= wq[q];
        if (a0 < n_views) Yh[(size_t)a0 * HQ + q] = make_float2(h * sm.x, h * sm.y);
        if (a0 + 1 < n_views) Yh[(size_t)(a0 + 1) * HQ + q] = make_float2(h * df.y, -h * df.x);
    }
}

// ---------------------------------------------------------------- A2
// Deterministic binned spreading. One workgroup per work item: a slice of
// at most A2_CHUNK visits of one output strip's visit list (a strip is gx <=
// A2_GX consecutive tile columns of one tile row), which is the concatenation
// of the diagonal neighbour bin's class 2, the v-neighbours' classes 2-3, the
// u-neighbour's classes 1-2 and the whole own bins -- exactly the samples
// whose footprint reaches the strip. Each thread takes up to A2_VPT visits
// and adds their W x W footprints into a halo'd LDS strip; strips of several
// tiles make fewer, longer work items and visit fewer samples twice.
//
// The strip is accumulated in fixed point with 64-bit integer atomic adds, the
// real and imaginary parts packed into one word: a contribution (c_re, c_im)
// of two int32 adds c_re + 2^32 c_im (mod 2^64). Integer addition is exact,
// commutative and associative, so the word ends as S_re + 2^32 S_im (mod
// 2^64) whatever the order in which lanes and waves arrive, and S_re, S_im are
// recovered exactly when both lie in [-2^31, 2^31): the result is bitwise
// reproducible without floating-point atomics, and one atomic carries both
// parts. c = round(wx * (Y * wy * 2^s)), with the item's scale s chosen from
// its largest |Y * wy| so that every |c| <= 2^21 and, with at most 512 visits
// per item, every final sum stays below 2^30; each contribution is rounded to
// 2^-22 of the item's largest one, about the resolution of float32.
#ifndef RN_A2_NT
#define RN_A2_NT 256
#endif
#ifndef RN_A2_CHUNK
#define RN_A2_CHUNK 512
#endif
constexpr int A2_NT = RN_A2_NT;
constexpr int A2_CHUNK = RN_A2_CHUNK;
// the fixed-point scale below keeps every sum of at most 512 contributions
// inside int32
static_assert(A2_CHUNK <= 512, "A2 items hold at most 512 visits");
constexpr int A2_VPT = (A2_CHUNK + A2_NT - 1) / A2_NT;

// Waves per SIMD the spreading kernel is compiled for when W <= 6 (at most
// 80 VGPRs; W = 8 keeps its natural allocation).
#ifndef RN_A2_WPE
#define RN_A2_WPE 6
#endif
template <int W, int T>
__device__ __forceinline__ void a2_item(const TileItem& it, const SampleRec* __restrict__ recs, const float2* __restrict__ Yh,
                                        const float4* __restrict__ kbc, float2* __restrict__ grid,
                                        float2* __restrict__ partials, int G) {
    constexpr int PX = A2_GX * T + 2 * (W - 1);   // accumulator: local [-(W-1), A2_GX T + W-1) along u
    constexpr int PY = T + 2 * (W - 1);           // and [-(W-1), T + W-1) along v
    constexpr int NKB = (W / 2) * KB_S;
    constexpr int NR = A2_NR;                     // visit ranges
    __shared__ __align__(16) unsigned long long acc[PX * PY];
    __shared__ float4 kbt[NKB];
    __shared__ float wmax[A2_NT / 64];
    const int tid = threadIdx.x;
    const int gx = it.gx;

    // T is even, so PX * PY is: clear the accumulator 16 bytes at a time
    static_assert(T % 2 == 0 && (PX * PY) % 2 == 0, "accumulator cleared in pairs of words");
    for (int e = tid; e < PX * PY / 2; e += A2_NT) reinterpret_cast<ulonglong2*>(acc)[e] = make_ulonglong2(0ull, 0ull);
    for (int e = tid; e < NKB; e += A2_NT) kbt[e] = kbc[e];
    lds_sync();

    // visit ranges (diagonal class 2, v-neighbours classes 2-3, u-neighbour
    // classes 1-2, own bins), from the item
    int rs[NR], rl[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        rs[q] = it.rs[q];
        rl[q] = it.rl[q];
    }
    const int x0 = it.cx * T, y0 = it.cy * T;

    int base[A2_VPT];
    float wx[A2_VPT][W];
    float2 ywy[A2_VPT][W];
    float mx_abs = 0.f;
#pragma unroll
    for (int k = 0; k < A2_VPT; ++k) {
        const int t = tid + k * A2_NT;
        base[k] = -1;
        if (t < it.count) {
            int u = it.start + t, pos = -1;
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (pos < 0) {
                    if (u < rl[q]) pos = rs[q] + u;
                    else u -= rl[q];
                }
            }
            const SampleRec r = load_rec(recs, pos);
            float2 Y = Yh[r.info & REC_IDX_MASK];
            if (r.info & REC_CONJ) Y = cconj(Y);
            int ox = (r.org & REC_ORG_MASK) - x0;
            int oy = ((r.org >> 16) & REC_ORG_MASK) - y0;
            if (ox >= G / 2) ox -= G;
            if (ox < -G / 2) ox += G;
            if (oy >= G / 2) oy -= G;
            if (oy < -G / 2) oy += G;
            base[k] = (ox + W - 1) * PY + (oy + W - 1);
            kb_weights<W>(r.fu, kbt, wx[k]);
            if (r.org & REC_U_NEAR_OUT) wx[k][0] = 0.f;
            if (r.org & REC_U_FAR_OUT) wx[k][W - 1] = 0.f;
            float wy[W];
            kb_weights<W>(r.fv, kbt, wy);
            if (r.org & REC_V_NEAR_OUT) wy[0] = 0.f;
            if (r.org & REC_V_FAR_OUT) wy[W - 1] = 0.f;
#pragma unroll
            for (int gm = 0; gm < W; ++gm) {
                ywy[k][gm] = make_float2(Y.x * wy[gm], Y.y * wy[gm]);
                // a NaN counts as infinite, so a non-finite value reaches the maximum
                const float ax = fabsf(ywy[k][gm].x), ay = fabsf(ywy[k][gm].y);
                mx_abs = fmaxf(mx_abs, fmaxf(ax == ax ? ax : INFINITY, ay == ay ? ay : INFINITY));
            }
        }
    }
    // item-wide max |Y*wy| (order-independent)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx_abs = fmaxf(mx_abs, __shfl_xor(mx_abs, off));
    if ((tid & 63) == 0) wmax[tid >> 6] = mx_abs;
    lds_sync();
    float m = wmax[0];
#pragma unroll
    for (int w = 1; w < A2_NT / 64; ++w) m = fmaxf(m, wmax[w]);
    // a non-finite contribution makes the whole item NaN (written below), so
    // divergence is not hidden by the fixed-point sums
    const bool finite = m <= 3.402823466e38f;
    // scale 2^s: m 2^s < 2^21, so every |c| <= 2^21 (|wx| <= 1) and a sum of
    // count <= 512 of them stays below 2^31
    int e = 0;
    (void)frexpf(finite ? m : 0.f, &e);        // m < 2^e
    const int s = 21 - e;
    // fma(w, y, 1.5 2^23) rounds w y (|w y| < 2^22) to an integer c once and
    // leaves 0x4B400000 + c in the bits; both words' offsets go in one subtraction
    const float magic = 12582912.0f;
    const unsigned long long bias = 0x4B4000004B400000ull;
#pragma unroll
    for (int k = 0; k < A2_VPT; ++k) {
        if (base[k] < 0 || !finite) continue;
#pragma unroll
        for (int gm = 0; gm < W; ++gm) {
            const float yr = ldexpf(ywy[k][gm].x, s), yi = ldexpf(ywy[k][gm].y, s);
#pragma unroll
            for (int al = 0; al < W; ++al) {
                const float tr = fmaf(wx[k][al], yr, magic), ti = fmaf(wx[k][al], yi, magic);
                const unsigned long long word =
                    ((unsigned long long)__float_as_uint(ti) << 32) | __float_as_uint(tr);
                atomicAdd(&acc[base[k] + al * PY + gm], word - bias);   // c_re + 2^32 c_im (mod 2^64)
            }
        }
    }
    lds_sync();
    // write out: local (lx, ly) -> mx = (x0 + lx - G/2) mod G, my = (y0 + ly - G/2) mod G
    const int xvalid = (it.cx == 0) ? 1 : gx * T;   // tile column 0 holds only mx = G/2
    const int my0 = mod_pos(y0 - G / 2, G);
    // two consecutive my per lane, one 16-byte store: T, y0 and G/2 (= n)
    // are even, so my0 + ly is even and the pair never leaves the tile
    for (int e2 = 2 * tid; e2 < xvalid * T; e2 += 2 * A2_NT) {
        const int lx = e2 / T, ly = e2 - lx * T;
        float v[4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const unsigned long long w = acc[(lx + W - 1) * PY + (ly + h + W - 1)];
            const int sre = (int)(unsigned int)(w & 0xffffffffull);
            const int sim = (int)((long long)(w - (unsigned long long)(long long)sre) >> 32);
            v[2 * h] = finite ? (float)ldexp((double)sre, -s) : __int_as_float(0x7fc00000);
            v[2 * h + 1] = finite ? (float)ldexp((double)sim, -s) : __int_as_float(0x7fc00000);
        }
        const float4 val = make_float4(v[0], v[1], v[2], v[3]);
        if (it.slot < 0) {
            const int mx = wrap_g(x0 + lx - G / 2, G);
            *reinterpret_cast<float4*>(grid + (size_t)mx * G + my0 + ly) = val;
        } else {
            *reinterpret_cast<float4*>(partials + (size_t)it.slot * (A2_GX * T * T) + e2) = val;
        }
    }
}

// Sum the partial strips of split output strips in slot order.
struct SplitTile {
    int cx, cy;
    int first_slot, nslots;
    int gx;          // tile columns of the strip
    int plan;        // batches: index of the strip's plan in the batch (else 0)
};

#ifndef RN_A2R_FLIGHT
#define RN_A2R_FLIGHT 16
#endif
template <int T>
__device__ __forceinline__ void a2r_body(const SplitTile& sp, int by, const float2* __restrict__ partials,
                                         float2* __restrict__ grid, int G) {
    constexpr int SLOT = A2_GX * T * T;   // points per partial slot
    const int xvalid = (sp.cx == 0) ? 1 : sp.gx * T;   // tile column 0 holds only mx = G/2
    const int x0 = sp.cx * T, y0 = sp.cy * T;
    const int my0 = mod_pos(y0 - G / 2, G);
    const float2* src = partials + (size_t)sp.first_slot * SLOT;
    // block row `by` picks 256 of the strip's points, one per thread
    for (int e = by * 256 + threadIdx.x; e < xvalid * T && e < (by + 1) * 256; e += 256) {
        // slots are added in order; the loads of RN_A2R_FLIGHT slots (the last batch
        // predicated) are issued together
        float2 s = make_float2(0.f, 0.f);
        for (int k = 0; k < sp.nslots; k += RN_A2R_FLIGHT) {
            float2 v[RN_A2R_FLIGHT];
#pragma unroll
            for (int j = 0; j < RN_A2R_FLIGHT; ++j)
                v[j] = (k + j < sp.nslots) ? src[(size_t)(k + j) * SLOT + e] : make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < RN_A2R_FLIGHT; ++j)
                if (k + j < sp.nslots) s = (k + j == 0) ? v[j] : cadd(s, v[j]);
        }
        const int lx = e / T, ly = e - lx * T;
        const int mx = wrap_g(x0 + lx - G / 2, G);
        grid[(size_t)mx * G + my0 + ly] = s;
    }
}

// ---------------------------------------------------------------- A3
// One grid line mx per workgroup: h[p] = sum_my H[my] e^{+2 pi i my p/G} for
// the n rows p = -n/2..n/2-1 = IFFT_n(H_even)[p] + e^{i pi p/n} IFFT_n(H_odd)[p];
// the two inverse transforms share one LDS line, one after the other, each
// with register input and output (FftRegIO); the inverse is conj(FFT(conj)).
template <int NL, int NT>
__device__ __forceinline__ void a3_body(int bid_, int nblk_, const float2* __restrict__ grid, float2* __restrict__ T1,
                                               const float2* __restrict__ shift,
                                               const float2* __restrict__ tw) {
    __shared__ float2 lds[lds_ls(NL)];
    const int tid = threadIdx.x;
    const int mx = bid_;
    const float4* src = reinterpret_cast<const float4*>(grid + (size_t)mx * (2 * NL));
    float2* dst = T1 + (size_t)mx * NL;
    using IO = FftRegIO<NL, 1, NT>;
    if constexpr (IO::NP >= 2) {
        float2 ve[IO::IT0][IO::R0], vo[IO::IT0][IO::R0];
        float2 E[IO::ITL][IO::RL], O[IO::ITL][IO::RL];
#pragma unroll
        for (int it = 0; it < IO::IT0; ++it) {
            const int b = tid + it * NT;
#pragma unroll
            for (int m = 0; m < IO::R0; ++m) {
                const float4 g = (b < IO::NB0) ? src[b + m * IO::NB0] : make_float4(0.f, 0.f, 0.f, 0.f);
                ve[it][m] = make_float2(g.x, -g.y);          // conj for the inverse
                vo[it][m] = make_float2(g.z, -g.w);
            }
        }
        fft_regs<NL, 1, NT>(ve, lds, tw, tid, E);
        lds_sync();
        fft_regs<NL, 1, NT>(vo, lds, tw, tid, O);
        // FFT position q is row p = q (mod n), stored at i = (q + n/2) mod n
#pragma unroll
        for (int it = 0; it < IO::ITL; ++it) {
            const int b = tid + it * NT;
            if (b < IO::NBL) {
#pragma unroll
                for (int m = 0; m < IO::RL; ++m) {
                    const int i = (b + m * IO::NBL + NL / 2) % NL;
                    dst[i] = cadd(cconj(E[it][m]), cmul(cconj(shift[i]), cconj(O[it][m])));
                }
            }
        }
    } else {
        constexpr int PE = (NL + NT - 1) / NT;
        float2 odd[PE], ev[PE];
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int k = tid + e * NT;
            if (k < NL) {
                const float4 v = src[k];
                lds[lds_pad(k)] = make_float2(v.x, -v.y);        // conj for the inverse
                odd[e] = make_float2(v.z, -v.w);
            }
        }
        lds_sync();
        fft_lds<NL, 1, NT>(lds, tw, tid);
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int i = tid + e * NT;
            if (i < NL) ev[e] = cconj(lds[lds_pad((i + NL / 2) % NL)]);
        }
        lds_sync();
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int k = tid + e * NT;
            if (k < NL) lds[lds_pad(k)] = odd[e];
        }
        lds_sync();
        fft_lds<NL, 1, NT>(lds, tw, tid);
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const int i = tid + e * NT;
            if (i < NL) {
                const float2 o = cconj(lds[lds_pad((i + NL / 2) % NL)]);
                dst[i] = cadd(ev[e], cmul(cconj(shift[i]), o));
            }
        }
    }
}

// ---------------------------------------------------------------- A4
// 2 NLN image rows per workgroup (NLN = row_lines(n), as in F1):
// complex-to-real inverse FFT along mx of T1[mx][i], mx = 0..n (Hermitian
// extension to G points), keep px = -n/2..n/2-1, deapodize. Rows 2p and 2p+1
// are packed as one complex line (X_2p + i X_{2p+1}); its even positions
// mx = 2k form the length-n line E_p and its odd ones the line O_p, and the
// pixel is E_p(px) + e^{+i pi px/n} O_p(px). The E lines are transformed
// first (their results wait in registers), then the O lines; each
// T1[mx][i0..i0+2NLN-1] (16 NLN contiguous bytes) is read once, by the pass
// of its parity.
template <int NL, int NT>
__device__ __forceinline__ void a4_load(const float2* __restrict__ T1, float2* lds, int m, int pk, int pc, int i0,
                                        int p) {
    // line p takes rows i0 + 2p and i0 + 2p + 1 (16 bytes); consecutive lanes
    // take the lines p = 0 .. NLN-1 of one frequency, so one load instruction
    // reads whole 16 NLN-byte pieces
    constexpr int LS = lds_ls(NL);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i0 + 2 * p + 1 < NL) v = *reinterpret_cast<const float4*>(T1 + (size_t)m * NL + i0 + 2 * p);
    float2 X1 = make_float2(v.x, v.y), X2 = make_float2(v.z, v.w);
    if (m == 0 || m == NL) { X1.y = 0.f; X2.y = 0.f; }
    const float2 z = make_float2(X1.x - X2.y, X1.y + X2.x);             // X1 + i X2
    lds[p * LS + lds_pad(pk)] = cconj(z);                               // conjugated for the inverse
    if (m >= 1 && m <= NL - 1) {
        const float2 zm = make_float2(X1.x + X2.y, -X1.y + X2.x);       // conj X1 + i conj X2 at 2n - m
        lds[p * LS + lds_pad(pc)] = cconj(zm);
    }
}

template <int NL, int NT>
__device__ __forceinline__ void a4_body(int bid_, int nblk_, const float2* __restrict__ T1, float* __restrict__ img,
                                               const float* __restrict__ psi_inv,
                                               const float2* __restrict__ shift,
                                               const float2* __restrict__ tw) {
    constexpr int LS = lds_ls(NL);
    constexpr int NLN = row_lines(NL);
    __shared__ float2 lds[NLN * LS];
    const int tid = threadIdx.x;
    const int i0 = 2 * NLN * xcd_block(bid_, nblk_);
    using IO = FftRegIO<NL, NLN, NT>;
    if constexpr (IO::NP >= 2) {
        // Both transforms leave their last pass in registers: butterfly
        // b = tid + it NT (line b / NBL) holds FFT positions q = bf + m NBL,
        // pixel j = (q + n/2) mod n of rows i0 + 2 line and i0 + 2 line + 1.
        float2 E[IO::ITL][IO::RL], O[IO::ITL][IO::RL];
        // even mx = 2k: position k, mirror 2n - 2k at n - k
        for (int e = tid; e < NLN * (NL / 2 + 1); e += NT) {
            const int k = e / NLN;
            a4_load<NL, NT>(T1, lds, 2 * k, k, NL - k, i0, e - k * NLN);
        }
        lds_sync();
        fft_mid_passes<NL, 0, 1, NLN, NT, LS>(lds, tw, tid);
        fft_last_to_regs<NL, NLN, NT>(lds, tw, tid, E);
        lds_sync();   // the last pass read the lines
        // odd mx = 2k+1: position k, mirror 2n - 2k - 1 at n - 1 - k
        for (int e = tid; e < NLN * (NL / 2); e += NT) {
            const int k = e / NLN;
            a4_load<NL, NT>(T1, lds, 2 * k + 1, k, NL - 1 - k, i0, e - k * NLN);
        }
        lds_sync();
        fft_mid_passes<NL, 0, 1, NLN, NT, LS>(lds, tw, tid);
        fft_last_to_regs<NL, NLN, NT>(lds, tw, tid, O);
#pragma unroll
        for (int it = 0; it < IO::ITL; ++it) {
            const int b = tid + it * NT;
            if (b < IO::NBL * NLN) {
                const int line = b / IO::NBL, bf = b - line * IO::NBL;
                const int r0 = i0 + 2 * line;
#pragma unroll
                for (int m = 0; m < IO::RL; ++m) {
                    const int j = (bf + m * IO::NBL + NL / 2) % NL;
                    const float2 sh = cconj(shift[j]);
                    const float pj = psi_inv[j];
                    const float2 zz = cadd(cconj(E[it][m]), cmul(sh, cconj(O[it][m])));
                    if (r0 < NL) img[(size_t)r0 * NL + j] = zz.x * psi_inv[r0] * pj;
                    if (r0 + 1 < NL) img[(size_t)(r0 + 1) * NL + j] = zz.y * psi_inv[r0 + 1] * pj;
                }
            }
        }
    } else {
        constexpr int PJ = (NL + NT - 1) / NT;       // pixels px per thread and row
        // even mx = 2k: position k, mirror 2n - 2k at n - k
        for (int e = tid; e < NLN * (NL / 2 + 1); e += NT) {
            const int k = e / NLN;
            a4_load<NL, NT>(T1, lds, 2 * k, k, NL - k, i0, e - k * NLN);
        }
        lds_sync();
        fft_lds<NL, NLN, NT>(lds, tw, tid);
        float2 e[PJ][NLN];
#pragma unroll
        for (int c = 0; c < PJ; ++c) {
            const int j = tid + c * NT;
            if (j < NL) {
                const int pos = lds_pad((j + NL / 2) % NL);
#pragma unroll
                for (int p = 0; p < NLN; ++p) e[c][p] = cconj(lds[p * LS + pos]);
            }
        }
        lds_sync();
        // odd mx = 2k+1: position k, mirror 2n - 2k - 1 at n - 1 - k
        for (int e2 = tid; e2 < NLN * (NL / 2); e2 += NT) {
            const int k = e2 / NLN;
            a4_load<NL, NT>(T1, lds, 2 * k + 1, k, NL - 1 - k, i0, e2 - k * NLN);
        }
        lds_sync();
        fft_lds<NL, NLN, NT>(lds, tw, tid);
#pragma unroll
        for (int c = 0; c < PJ; ++c) {
            const int j = tid + c * NT;
            if (j < NL) {
                const int pos = lds_pad((j + NL / 2) % NL);
                const float2 sh = cconj(shift[j]);
                const float pj = psi_inv[j];
#pragma unroll
                for (int p = 0; p < NLN; ++p) {
                    const float2 o = cconj(lds[p * LS + pos]);
                    const float2 zz = cadd(e[c][p], cmul(sh, o));
                    const int r0 = i0 + 2 * p;
                    if (r0 < NL) img[(size_t)r0 * NL + j] = zz.x * psi_inv[r0] * pj;
                    if (r0 + 1 < NL) img[(size_t)(r0 + 1) * NL + j] = zz.y * psi_inv[r0 + 1] * pj;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- single-slice kernels
// One launch per pass of one slice (batches use radon_multi.hpp's kernels,
// which run the same bodies).
template <int NL, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(row_waves(NL)))) void k_f1_rows(
    const float* __restrict__ img, float2* __restrict__ T1, const float* __restrict__ psi_inv,
    const float2* __restrict__ shift, const float2* __restrict__ tw) {
    f1_body<NL, NT>(blockIdx.x, gridDim.x, img, T1, psi_inv, shift, tw);
}

template <int NL, int NT>
__global__ __launch_bounds__(NT) void k_f2_cols(const float2* __restrict__ T1, float2* __restrict__ grid,
                                               const float2* __restrict__ shift, const float2* __restrict__ tw) {
    f2_body<NL, NT>(blockIdx.x, gridDim.x, T1, grid, shift, tw);
}

// Persistent: workgroup b takes items b, b + gridDim.x, ... (the grid is the
// number of workgroups that fit on the device at once).
template <int W, int T, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(W <= 6 ? RN_F3_WPE : 1))) void k_f3_tiles(
    const F3Item* __restrict__ items, int n_items, const SampleRec* __restrict__ recs,
    const float2* __restrict__ grid, const float4* __restrict__ kbc, float2* __restrict__ Xr, int G) {
    constexpr int PP = (2 * T + W - 1) * (2 * T + W - 1);
    constexpr int NKB = (W / 2) * KB_S;
    __shared__ float2 tile[PP];   // [lx][ly], lx along u (mx), ly along v (my)
    __shared__ float4 kbt[NKB];
    const int tid = threadIdx.x;
    for (int e = tid; e < NKB; e += NT) kbt[e] = kbc[e];
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
        const F3Item it = items[i];
        f3_item<W, T, NT>(it, recs, grid, Xr, G, tile, kbt, tid);
    }
}

template <int ND, int NT>
__global__ __launch_bounds__(NT) void k_f4_rays(const float2* __restrict__ Xr, float* __restrict__ sino,
                                               const float2* __restrict__ tw, int n_views) {
    f4_body<ND, NT>(blockIdx.x, gridDim.x, Xr, sino, tw, n_views);
}

template <int ND, int NT>
__global__ __launch_bounds__(NT) void k_a1_rays(const float* __restrict__ sino, float2* __restrict__ Yh,
                                               const float2* __restrict__ tw, const float* __restrict__ wq,
                                               int n_views) {
    a1_body<ND, NT>(blockIdx.x, gridDim.x, sino, Yh, tw, wq, n_views);
}

template <int W, int T>
__global__ __launch_bounds__(A2_NT) __attribute__((amdgpu_waves_per_eu(W <= 6 ? RN_A2_WPE : 1))) void k_a2_spread(
    const TileItem* __restrict__ items, const SampleRec* __restrict__ recs,
    const float2* __restrict__ Yh, const float4* __restrict__ kbc, float2* __restrict__ grid,
    float2* __restrict__ partials, int G) {
    const TileItem it = items[blockIdx.x];
    a2_item<W, T>(it, recs, Yh, kbc, grid, partials, G);
}

template <int T>
__global__ __launch_bounds__(256) void k_a2_reduce(const SplitTile* __restrict__ splits,
                                                  const float2* __restrict__ partials, float2* __restrict__ grid,
                                                  int G) {
    const SplitTile sp = splits[blockIdx.x];
    a2r_body<T>(sp, blockIdx.y, partials, grid, G);
}

template <int NL, int NT>
__global__ __launch_bounds__(NT) void k_a3_cols(const float2* __restrict__ grid, float2* __restrict__ T1,
                                               const float2* __restrict__ shift, const float2* __restrict__ tw) {
    a3_body<NL, NT>(blockIdx.x, gridDim.x, grid, T1, shift, tw);
}

template <int NL, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(row_waves(NL)))) void k_a4_rows(
    const float2* __restrict__ T1, float* __restrict__ img, const float* __restrict__ psi_inv,
    const float2* __restrict__ shift, const float2* __restrict__ tw) {
    a4_body<NL, NT>(blockIdx.x, gridDim.x, T1, img, psi_inv, shift, tw);
}

// ---------------------------------------------------------------- FFT test
template <int LEN, int NT>
__global__ __launch_bounds__(NT) void k_fft_test(const float2* __restrict__ in, float2* __restrict__ out,
                                                const float2* __restrict__ tw, int inverse) {
    __shared__ float2 lds[lds_ls(LEN)];
    const int tid = threadIdx.x;
    const size_t base = (size_t)blockIdx.x * LEN;
    for (int i = tid; i < LEN; i += NT) {
        float2 v = in[base + i];
        lds[lds_pad(i)] = inverse ? cconj(v) : v;
    }
    lds_sync();
    fft_lds<LEN, 1, NT>(lds, tw, tid);
    for (int i = tid; i < LEN; i += NT) {
        float2 v = lds[lds_pad(i)];
        out[base + i] = inverse ? cconj(v) : v;
    }
}

}  // namespace rn

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
//            F34 per pair of rays: Kaiser-Bessel interpolation of the
//                N/2+1 independent samples from the half grid, then a
//                complex-to-real inverse FFT along the rays -> sinogram
//   adjoint  A1  per pair of rays: real-to-complex FFT -> Yh[a][q], q <= N/2
//            A2  per output tile: deterministic spreading of the samples of
//                the tile's four bins (sorted by footprint-origin tile) into
//                an LDS accumulator, in a fixed order, no atomics
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

// Kaiser-Bessel weight phi(t) for t >= 0 from the (value, slope) table with
// L entries per unit; strict support: 0 for t >= W/2.
__device__ __forceinline__ float kb_weight(float t, const float2* __restrict__ tab, float L,
                                           float half_w) {
    if (!(t < half_w)) return 0.0f;
    float x = t * L;
    int i = (int)x;
    float f = x - (float)i;
    float2 e = tab[i];
    return fmaf(f, e.y, e.x);
}

struct SampleGeom {
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

// ---------------------------------------------------------------- F1
// Four image rows per workgroup (two packed pairs). Row i holds py = i - n/2,
// column j holds px = j - n/2 (stored at px mod n in the length-n FFT).
// Lines in LDS: [pair0 r=0, pair0 r=1, pair1 r=0, pair1 r=1].
template <int NL, int NT>
__global__ __launch_bounds__(NT) void k_f1_rows(const float* __restrict__ img, float2* __restrict__ T1,
                                               const float* __restrict__ psi_inv,
                                               const float2* __restrict__ shift,
                                               const float2* __restrict__ tw) {
    __shared__ float2 lds[4 * NL];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * 4;
    for (int idx = tid; idx < 2 * NL; idx += NT) {
        const int p = idx / NL;
        const int j = idx - p * NL;
        const int r0 = i0 + 2 * p;
        const float pj = psi_inv[j];
        float a = 0.f, b = 0.f;
        if (r0 < NL) a = img[(size_t)r0 * NL + j] * psi_inv[r0] * pj;
        if (r0 + 1 < NL) b = img[(size_t)(r0 + 1) * NL + j] * psi_inv[r0 + 1] * pj;
        const int pos = (j + NL / 2) % NL;
        const float2 z = make_float2(a, b);
        lds[(2 * p) * NL + pos] = z;
        lds[(2 * p + 1) * NL + pos] = cmul(z, shift[j]);
    }
    __syncthreads();
    fft_lds<NL, 4, NT>(lds, tw, tid);
    for (int m = tid; m <= NL; m += NT) {
        float2 out[4];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float2 zk, zc;
            if ((m & 1) == 0) {
                const int k = m >> 1;
                zk = lds[(2 * p) * NL + k];
                zc = cconj(lds[(2 * p) * NL + (NL - k) % NL]);
            } else {
                const int k = m >> 1;
                zk = lds[(2 * p + 1) * NL + k];
                zc = cconj(lds[(2 * p + 1) * NL + NL - 1 - k]);
            }
            const float2 sm = cadd(zk, zc), df = csub(zk, zc);
            out[2 * p] = make_float2(0.5f * sm.x, 0.5f * sm.y);
            out[2 * p + 1] = make_float2(0.5f * df.y, -0.5f * df.x);   // (zk - zc) / 2i
        }
        float2* dst = T1 + (size_t)m * NL + i0;
        if (i0 + 1 < NL) *reinterpret_cast<float4*>(dst) = make_float4(out[0].x, out[0].y, out[1].x, out[1].y);
        if (i0 + 3 < NL) *reinterpret_cast<float4*>(dst + 2) = make_float4(out[2].x, out[2].y, out[3].x, out[3].y);
    }
}

// ---------------------------------------------------------------- F2
// One half-plane line mx per workgroup: FFT along py of T1[mx][.] into
// grid[mx][my], my = 2k + r from two length-n transforms.
template <int NL, int NT>
__global__ __launch_bounds__(NT) void k_f2_cols(const float2* __restrict__ T1, float2* __restrict__ grid,
                                               const float2* __restrict__ shift,
                                               const float2* __restrict__ tw) {
    __shared__ float2 lds[2 * NL];
    const int tid = threadIdx.x;
    const int mx = blockIdx.x;
    const float2* src = T1 + (size_t)mx * NL;
    for (int i = tid; i < NL; i += NT) {
        const float2 c = src[i];
        const int pos = (i + NL / 2) % NL;
        lds[pos] = c;
        lds[NL + pos] = cmul(c, shift[i]);
    }
    __syncthreads();
    fft_lds<NL, 2, NT>(lds, tw, tid);
    float4* dst = reinterpret_cast<float4*>(grid + (size_t)mx * (2 * NL));
    for (int k = tid; k < NL; k += NT) {
        const float2 e = lds[k], o = lds[NL + k];
        dst[k] = make_float4(e.x, e.y, o.x, o.y);
    }
}

// ---------------------------------------------------------------- F34
// Two rays per workgroup. Samples q = 0..N/2-1 and q = -N/2 are interpolated
// from the half grid (footprint points with mx mod G in (G/2, G) are read as
// the conjugate of their mirror), then y = Re((1/N) IFFT) with the Hermitian
// extension X[-q] = conj X[q]; the two real outputs share one complex IFFT.
template <int ND, int W, int NT>
__global__ __launch_bounds__(NT) void k_f34_rays(const float2* __restrict__ grid, float* __restrict__ sino,
                                                const double2* __restrict__ cs,
                                                const float2* __restrict__ kbtab, float kbL,
                                                const float2* __restrict__ tw, int G, int n_views) {
    constexpr int HQ = ND / 2 + 1;
    __shared__ float2 xs[2 * HQ];
    __shared__ float2 lds[ND];
    const int tid = threadIdx.x;
    const int a0 = blockIdx.x * 2;
    const float hw = 0.5f * (float)W;
    for (int sidx = tid; sidx < 2 * HQ; sidx += NT) {
        const int r = sidx / HQ;
        const int t = sidx - r * HQ;
        const int a = a0 + r;
        float2 acc = make_float2(0.f, 0.f);
        if (a < n_views) {
            const int q = (t < ND / 2) ? t : -(ND / 2);
            const double2 csa = cs[a];
            const SampleGeom g = sample_geom(csa.x, csa.y, q, G, ND);
            float wy[W];
#pragma unroll
            for (int gm = 0; gm < W; ++gm) {
                const float tt = g.fv + (float)(W / 2 - 1 - gm);
                wy[gm] = kb_weight(fabsf(tt), kbtab, kbL, hw);
            }
#pragma unroll
            for (int al = 0; al < W; ++al) {
                const float tt = g.fu + (float)(W / 2 - 1 - al);
                const float wx = kb_weight(fabsf(tt), kbtab, kbL, hw);
                int mw = mod_pos(g.bu - W / 2 + 1 + al, G);
                if (mw > G / 2) mw -= G;
                const bool mir = mw < 0;
                const float2* line = grid + (size_t)(mir ? -mw : mw) * G;
                float2 racc = make_float2(0.f, 0.f);
#pragma unroll
                for (int gm = 0; gm < W; ++gm) {
                    const int my = g.bv - W / 2 + 1 + gm;
                    const int row = mod_pos(mir ? -my : my, G);
                    const float2 val = line[row];
                    racc.x = fmaf(wy[gm], val.x, racc.x);
                    racc.y = fmaf(wy[gm], mir ? -val.y : val.y, racc.y);
                }
                acc.x = fmaf(wx, racc.x, acc.x);
                acc.y = fmaf(wx, racc.y, acc.y);
            }
        }
        xs[sidx] = acc;
    }
    __syncthreads();
    // Z = A + i B with A, B the Hermitian extensions of the two rays; store
    // conj(Z) so the forward engine yields conj of the inverse transform.
    for (int q = tid; q < ND; q += NT) {
        float2 A, B;
        if (q == 0 || q == ND / 2) {
            A = make_float2(xs[q].x, 0.f);
            B = make_float2(xs[HQ + q].x, 0.f);
        } else if (q < ND / 2) {
            A = xs[q];
            B = xs[HQ + q];
        } else {
            A = cconj(xs[ND - q]);
            B = cconj(xs[HQ + ND - q]);
        }
        const float2 z = make_float2(A.x - B.y, A.y + B.x);
        lds[q] = cconj(z);
    }
    __syncthreads();
    fft_lds<ND, 1, NT>(lds, tw, tid);
    const float inv = 1.0f / (float)ND;
    for (int d = tid; d < ND; d += NT) {
        const float2 z = cconj(lds[(d + ND / 2) % ND]);
        if (a0 < n_views) sino[(size_t)a0 * ND + d] = z.x * inv;
        if (a0 + 1 < n_views) sino[(size_t)(a0 + 1) * ND + d] = z.y * inv;
    }
}

// ---------------------------------------------------------------- A1
// Two rays per workgroup: Yhat_a[q] = (1/N) sum_d y[a,d] e^{-2 pi i q s_d/N},
// q = 0..N/2; the q = N/2 (Nyquist) value is halved because it is spread
// once at its own position and once at the mirrored one.
template <int ND, int NT>
__global__ __launch_bounds__(NT) void k_a1_rays(const float* __restrict__ sino, float2* __restrict__ Yh,
                                               const float2* __restrict__ tw, int n_views) {
    constexpr int HQ = ND / 2 + 1;
    __shared__ float2 lds[ND];
    const int tid = threadIdx.x;
    const int a0 = blockIdx.x * 2;
    for (int d = tid; d < ND; d += NT) {
        const float ya = (a0 < n_views) ? sino[(size_t)a0 * ND + d] : 0.f;
        const float yb = (a0 + 1 < n_views) ? sino[(size_t)(a0 + 1) * ND + d] : 0.f;
        lds[(d + ND / 2) % ND] = make_float2(ya, yb);
    }
    __syncthreads();
    fft_lds<ND, 1, NT>(lds, tw, tid);
    const float sc = 0.5f / (float)ND;
    for (int q = tid; q < HQ; q += NT) {
        const float2 zq = lds[q];
        const float2 zc = cconj(lds[(ND - q) % ND]);
        const float2 sm = cadd(zq, zc), df = csub(zq, zc);
        const float h = (q == ND / 2) ? 0.5f * sc : sc;
        if (a0 < n_views) Yh[(size_t)a0 * HQ + q] = make_float2(h * sm.x, h * sm.y);
        if (a0 + 1 < n_views) Yh[(size_t)(a0 + 1) * HQ + q] = make_float2(h * df.y, -h * df.x);
    }
}

// ---------------------------------------------------------------- A2
// Deterministic binned spreading. One wave per work item; a work item is a
// contiguous slice of the visit list of one output tile (cx, cy) of the
// centred tile grid, where the visit list is the concatenation of the
// sorted samples of bins (cx-1,cy-1), (cx,cy-1), (cx-1,cy), (cx,cy).
// Each visited sample is staged (local footprint origin, W x-weights,
// W values Y*wy) by one lane, then the wave applies the staged samples one
// after another, lane = footprint point, into a T x T LDS accumulator. The
// order of additions is fixed, so results are bitwise reproducible.
struct WorkItem {
    int cx, cy;      // output tile, centred tile coordinates
    int start;       // first visit index
    int count;       // number of visits
    int slot;        // -1: write the grid; else partial slot
    int pad0, pad1, pad2;
};

template <int W, int T>
__global__ __launch_bounds__(64) void k_a2_spread(const WorkItem* __restrict__ items,
                                                 const int* __restrict__ offsets,
                                                 const int* __restrict__ perm,
                                                 const float2* __restrict__ Yh,
                                                 const double2* __restrict__ cs,
                                                 const float2* __restrict__ kbtab, float kbL,
                                                 float2* __restrict__ grid, float2* __restrict__ partials,
                                                 int G, int ND, int n_views) {
    struct Staged {
        int ox, oy;
        float wx[W];
        float2 ywy[W];
    };
    __shared__ float2 acc[T * T];
    __shared__ Staged st[64];
    const int lane = threadIdx.x;
    const WorkItem it = items[blockIdx.x];
    const int NTL = G / T;
    const int M = n_views * ND;
    const int HQ = ND / 2 + 1;
    const float hw = 0.5f * (float)W;

    for (int e = lane; e < T * T; e += 64) acc[e] = make_float2(0.f, 0.f);

    // visit ranges of the four bins: up-left, up, left, own
    const int xl = (it.cx + NTL - 1) % NTL, yu = (it.cy + NTL - 1) % NTL;
    const int b0 = yu * NTL + xl, b1 = yu * NTL + it.cx, b2 = it.cy * NTL + xl, b3 = it.cy * NTL + it.cx;
    const int rs0 = offsets[b0], rl0 = offsets[b0 + 1] - rs0;
    const int rs1 = offsets[b1], rl1 = offsets[b1 + 1] - rs1;
    const int rs2 = offsets[b2], rl2 = offsets[b2 + 1] - rs2;
    const int rs3 = offsets[b3];
    const int x0 = it.cx * T, y0 = it.cy * T;   // tile origin, centred coordinates
    const int xvalid = (it.cx == 0) ? 1 : T;   // tile column 0 holds only mx = G/2
    __syncthreads();

    for (int base = 0; base < it.count; base += 64) {
        const int nv = min(64, it.count - base);
        if (lane < nv) {
            int t = it.start + base + lane;
            int pos;
            if (t < rl0) pos = rs0 + t;
            else if ((t -= rl0) < rl1) pos = rs1 + t;
            else if ((t -= rl1) < rl2) pos = rs2 + t;
            else pos = rs3 + (t - rl2);
            const int v = perm[pos];
            int a, q;
            float2 Y;
            if (v < M) {
                a = v / ND;
                q = v - a * ND - ND / 2;
                if (q >= 0) Y = Yh[(size_t)a * HQ + q];
                else if (q > -ND / 2) Y = cconj(Yh[(size_t)a * HQ - q]);
                else Y = Yh[(size_t)a * HQ + ND / 2];
            } else {
                a = v - M;
                q = ND / 2;
                Y = Yh[(size_t)a * HQ + ND / 2];
            }
            const double2 csa = cs[a];
            const SampleGeom g = sample_geom(csa.x, csa.y, q, G, ND);
            int ox = mod_pos(g.bu - W / 2 + 1 + G / 2, G) - x0;
            int oy = mod_pos(g.bv - W / 2 + 1 + G / 2, G) - y0;
            if (ox >= G / 2) ox -= G;
            if (ox < -G / 2) ox += G;
            if (oy >= G / 2) oy -= G;
            if (oy < -G / 2) oy += G;
            st[lane].ox = ox;
            st[lane].oy = oy;
#pragma unroll
            for (int al = 0; al < W; ++al)
                st[lane].wx[al] = kb_weight(fabsf(g.fu + (float)(W / 2 - 1 - al)), kbtab, kbL, hw);
#pragma unroll
            for (int gm = 0; gm < W; ++gm) {
                const float wy = kb_weight(fabsf(g.fv + (float)(W / 2 - 1 - gm)), kbtab, kbL, hw);
                st[lane].ywy[gm] = make_float2(Y.x * wy, Y.y * wy);
            }
        }
        __syncthreads();
        const int al = lane % W, gm = lane / W;
        for (int s = 0; s < nv; ++s) {
            if (lane < W * W) {
                const int lx = st[s].ox + al;
                const int ly = st[s].oy + gm;
                if (lx >= 0 && lx < xvalid && ly >= 0 && ly < T) {
                    const float w = st[s].wx[al];
                    const float2 c = st[s].ywy[gm];
                    float2 o = acc[lx * T + ly];
                    o.x = fmaf(w, c.x, o.x);
                    o.y = fmaf(w, c.y, o.y);
                    acc[lx * T + ly] = o;
                }
            }
            __syncthreads();
        }
    }
    // write out: local (lx, ly) -> mx = (x0 + lx - G/2) mod G, my = (y0 + ly - G/2) mod G
    const int my0 = mod_pos(y0 - G / 2, G);
    for (int e = lane; e < xvalid * T; e += 64) {
        const int lx = e / T, ly = e - lx * T;
        const float2 val = acc[e];
        if (it.slot < 0) {
            const int mx = mod_pos(x0 + lx - G / 2, G);
            grid[(size_t)mx * G + my0 + ly] = val;
        } else {
            partials[(size_t)it.slot * T * T + e] = val;
        }
    }
}

// Sum the partial tiles of split output tiles in slot order.
struct SplitTile {
    int cx, cy;
    int first_slot, nslots;
};

template <int T>
__global__ __launch_bounds__(256) void k_a2_reduce(const SplitTile* __restrict__ splits,
                                                  const float2* __restrict__ partials,
                                                  float2* __restrict__ grid, int G) {
    const SplitTile sp = splits[blockIdx.x];
    const int xvalid = (sp.cx == 0) ? 1 : T;
    const int x0 = sp.cx * T, y0 = sp.cy * T;
    const int my0 = mod_pos(y0 - G / 2, G);
    for (int e = threadIdx.x; e < xvalid * T; e += 256) {
        float2 s = partials[(size_t)sp.first_slot * T * T + e];
        for (int k = 1; k < sp.nslots; ++k) s = cadd(s, partials[(size_t)(sp.first_slot + k) * T * T + e]);
        const int lx = e / T, ly = e - lx * T;
        const int mx = mod_pos(x0 + lx - G / 2, G);
        grid[(size_t)mx * G + my0 + ly] = s;
    }
}

// ---------------------------------------------------------------- A3
// One grid line mx per workgroup: h[p] = sum_my H[my] e^{+2 pi i my p/G} for
// the n rows p = -n/2..n/2-1 = IFFT_n(H_even)[p] + e^{i pi p/n} IFFT_n(H_odd)[p].
template <int NL, int NT>
__global__ __launch_bounds__(NT) void k_a3_cols(const float2* __restrict__ grid, float2* __restrict__ T1,
                                               const float2* __restrict__ shift,
                                               const float2* __restrict__ tw) {
    __shared__ float2 lds[2 * NL];
    const int tid = threadIdx.x;
    const int mx = blockIdx.x;
    const float4* src = reinterpret_cast<const float4*>(grid + (size_t)mx * (2 * NL));
    for (int k = tid; k < NL; k += NT) {
        const float4 v = src[k];
        lds[k] = make_float2(v.x, -v.y);        // conj for the inverse
        lds[NL + k] = make_float2(v.z, -v.w);
    }
    __syncthreads();
    fft_lds<NL, 2, NT>(lds, tw, tid);
    float2* dst = T1 + (size_t)mx * NL;
    for (int i = tid; i < NL; i += NT) {
        const int idx = (i + NL / 2) % NL;
        const float2 e = cconj(lds[idx]), o = cconj(lds[NL + idx]);
        dst[i] = cadd(e, cmul(cconj(shift[i]), o));
    }
}

// ---------------------------------------------------------------- A4
// Four image rows per workgroup (two packed pairs): complex-to-real inverse
// FFT along mx of T1[mx][i], mx = 0..n (Hermitian extension to G points),
// keep px = -n/2..n/2-1, deapodize.
template <int NL, int NT>
__global__ __launch_bounds__(NT) void k_a4_rows(const float2* __restrict__ T1, float* __restrict__ img,
                                               const float* __restrict__ psi_inv,
                                               const float2* __restrict__ shift,
                                               const float2* __restrict__ tw) {
    __shared__ float2 lds[4 * NL];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * 4;
    for (int m = tid; m <= NL; m += NT) {
        const float2* src = T1 + (size_t)m * NL + i0;
        float2 X[4];
        const float4 v01 = *reinterpret_cast<const float4*>(src);
        X[0] = make_float2(v01.x, v01.y);
        X[1] = make_float2(v01.z, v01.w);
        if (i0 + 3 < NL) {
            const float4 v23 = *reinterpret_cast<const float4*>(src + 2);
            X[2] = make_float2(v23.x, v23.y);
            X[3] = make_float2(v23.z, v23.w);
        } else {
            X[2] = X[3] = make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float2 X1 = X[2 * p], X2 = X[2 * p + 1];
            if (m == 0 || m == NL) { X1.y = 0.f; X2.y = 0.f; }
            const float2 z = make_float2(X1.x - X2.y, X1.y + X2.x);          // X1 + i X2
            float2* even = lds + (2 * p) * NL;
            float2* odd = lds + (2 * p + 1) * NL;
            // position m, stored conjugated for the inverse
            if ((m & 1) == 0) even[m >> 1] = cconj(z); else odd[m >> 1] = cconj(z);
            if (m >= 1 && m <= NL - 1) {
                const int mm = 2 * NL - m;
                const float2 zm = make_float2(X1.x + X2.y, -X1.y + X2.x);    // conj X1 + i conj X2
                if ((mm & 1) == 0) even[mm >> 1] = cconj(zm); else odd[mm >> 1] = cconj(zm);
            }
        }
    }
    __syncthreads();
    fft_lds<NL, 4, NT>(lds, tw, tid);
    for (int idx = tid; idx < 2 * NL; idx += NT) {
        const int p = idx / NL;
        const int j = idx - p * NL;
        const int r0 = i0 + 2 * p;
        const int pos = (j + NL / 2) % NL;
        const float2 e = cconj(lds[(2 * p) * NL + pos]);
        const float2 o = cconj(lds[(2 * p + 1) * NL + pos]);
        const float2 z = cadd(e, cmul(cconj(shift[j]), o));
        const float pj = psi_inv[j];
        if (r0 < NL) img[(size_t)r0 * NL + j] = z.x * psi_inv[r0] * pj;
        if (r0 + 1 < NL) img[(size_t)(r0 + 1) * NL + j] = z.y * psi_inv[r0 + 1] * pj;
    }
}

// ---------------------------------------------------------------- FFT test
template <int LEN, int NT>
__global__ __launch_bounds__(NT) void k_fft_test(const float2* __restrict__ in, float2* __restrict__ out,
                                                const float2* __restrict__ tw, int inverse) {
    __shared__ float2 lds[LEN];
    const int tid = threadIdx.x;
    const size_t base = (size_t)blockIdx.x * LEN;
    for (int i = tid; i < LEN; i += NT) {
        float2 v = in[base + i];
        lds[i] = inverse ? cconj(v) : v;
    }
    __syncthreads();
    fft_lds<LEN, 1, NT>(lds, tw, tid);
    for (int i = tid; i < LEN; i += NT) {
        float2 v = lds[i];
        out[base + i] = inverse ? cconj(v) : v;
    }
}

}  // namespace rn

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
//            A2  per output tile: deterministic spreading of the samples
//                that reach the tile into an LDS accumulator, no atomics on
//                floating-point data
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

// Kaiser-Bessel weight phi(t) for t >= 0 from a table of cubic pieces, S
// pieces per unit of t (c.x + c.y f + c.z f^2 + c.w f^3 on piece floor(t S),
// f = frac(t S)); strict support: 0 for t >= W/2. S is a power of two, so
// t * S is exact and the piece index stays below (W/2) S.
__device__ __forceinline__ float kb_weight(float t, const float4* __restrict__ tab, float S, float half_w) {
    if (!(t < half_w)) return 0.0f;
    const float x = t * S;
    const int i = (int)x;
    const float f = x - (float)i;
    const float4 c = tab[i];
    return fmaf(fmaf(fmaf(c.w, f, c.z), f, c.y), f, c.x);
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

// ---------------------------------------------------------------- samples
// Sample ids: 0..M-1 are the polar samples j = a*N + q + N/2 (M = n_views*N);
// M..M+n_views-1 are the mirrored Nyquist samples (view a at q = +N/2).
__device__ __forceinline__ void decode_sample(int v, int M, int ND, int& a, int& q) {
    if (v < M) {
        a = v / ND;
        q = v - a * ND - ND / 2;
    } else {
        a = v - M;
        q = ND / 2;
    }
}

// Centred grid coordinate of the first footprint point: (floor - W/2 + 1 + G/2) mod G.
__device__ __forceinline__ int footprint_origin(int b, int W, int G) { return mod_pos(b - W / 2 + 1 + G / 2, G); }

// Tile columns whose samples the forward interpolates: the Hermitian half
// plane mx in [0, G/2] (centred columns ntl/2..ntl-1 and column 0, which
// holds mx = G/2) plus column ntl/2-1 (mx in [-T, 0)), so that footprints
// straddling mx = 0 are taken whole.
__device__ __forceinline__ bool forward_column(int cx, int ntl) { return cx == 0 || cx >= ntl / 2 - 1; }

// Forward / spreading work item: a slice of the sorted samples of one tile.
struct TileItem {
    int cx, cy;      // tile, centred tile coordinates
    int start;       // first position (forward: absolute in perm; spreading: visit index)
    int count;       // number of samples / visits
    int slot;        // spreading only: -1 writes the grid, else partial slot
    int pad0, pad1, pad2;
};

// ---------------------------------------------------------------- F3
// Kaiser-Bessel interpolation of the polar samples from the half-plane grid,
// one tile per workgroup. The tile and its (W-1) halo are staged in LDS
// (points with mx < 0 read as conjugates of their mirror, wrap mod G), then
// every sample whose footprint origin is in the tile is interpolated from LDS.
// Of each conjugate pair (q, -q) exactly one member is evaluated: q >= 0 when
// its origin tile is a forward column, else -q (result conjugated); the pair
// (-N/2, +N/2) likewise. Results go to Xr[a][t], t = |q| (t = N/2: Nyquist).
template <int W, int T, int NT>
__global__ __launch_bounds__(NT) void k_f3_tiles(const TileItem* __restrict__ items, const int* __restrict__ perm,
                                                const float2* __restrict__ grid, const double2* __restrict__ cs,
                                                const float4* __restrict__ kbc, float kbS,
                                                float2* __restrict__ Xr, int G, int ND, int n_views) {
    constexpr int P = T + W - 1;
    __shared__ float2 tile[P * P];   // [lx][ly], lx along u (mx), ly along v (my)
    const int tid = threadIdx.x;
    const TileItem it = items[blockIdx.x];
    const int x0 = it.cx * T, y0 = it.cy * T;
    const int ntl = G / T;
    const int M = n_views * ND;
    const int HQ = ND / 2 + 1;
    const float hw = 0.5f * (float)W;
    for (int e = tid; e < P * P; e += NT) {
        const int lx = e / P, ly = e - lx * P;
        int mx = mod_pos(x0 + lx, G) - G / 2;        // in [-G/2, G/2)
        const int my = mod_pos(y0 + ly, G) - G / 2;
        if (mx == -G / 2) mx = G / 2;
        float2 val;
        if (mx >= 0) {
            val = grid[(size_t)mx * G + mod_pos(my, G)];
        } else {
            val = cconj(grid[(size_t)(-mx) * G + mod_pos(-my, G)]);
        }
        tile[e] = val;
    }
    __syncthreads();
    for (int k = tid; k < it.count; k += NT) {
        const int v = perm[it.start + k];
        int a, q;
        decode_sample(v, M, ND, a, q);
        const double2 csa = cs[a];
        bool conj_out = false;
        int t;
        if (q == -ND / 2) { t = ND / 2; }
        else if (q >= 0 && q < ND / 2) { t = q; }
        else {
            // a mirror: evaluated only if its canonical partner's origin tile
            // is not a forward column
            const int qc = (q == ND / 2) ? -ND / 2 : -q;
            const SampleGeom gc = sample_geom(csa.x, csa.y, qc, G, ND);
            if (forward_column(footprint_origin(gc.bu, W, G) / T, ntl)) continue;
            t = (q == ND / 2) ? ND / 2 : -q;
            conj_out = true;
        }
        const SampleGeom g = sample_geom(csa.x, csa.y, q, G, ND);
        const int ox = footprint_origin(g.bu, W, G) - x0;
        const int oy = footprint_origin(g.bv, W, G) - y0;
        float wy[W];
#pragma unroll
        for (int gm = 0; gm < W; ++gm) wy[gm] = kb_weight(fabsf(g.fv + (float)(W / 2 - 1 - gm)), kbc, kbS, hw);
        const float2* src = tile + ox * P + oy;
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int al = 0; al < W; ++al) {
            const float wx = kb_weight(fabsf(g.fu + (float)(W / 2 - 1 - al)), kbc, kbS, hw);
            float2 racc = make_float2(0.f, 0.f);
#pragma unroll
            for (int gm = 0; gm < W; ++gm) {
                const float2 val = src[al * P + gm];
                racc.x = fmaf(wy[gm], val.x, racc.x);
                racc.y = fmaf(wy[gm], val.y, racc.y);
            }
            acc.x = fmaf(wx, racc.x, acc.x);
            acc.y = fmaf(wx, racc.y, acc.y);
        }
        Xr[(size_t)a * HQ + t] = conj_out ? cconj(acc) : acc;
    }
}

// ---------------------------------------------------------------- F4
// Two rays per workgroup: y = Re((1/N) IFFT) of the Hermitian extension
// X[-q] = conj X[q] of Xr (bins 0 and N/2 taken as real); the two real
// outputs share one complex IFFT. Output bin d is s = d - N/2 at s mod N.
template <int ND, int NT>
__global__ __launch_bounds__(NT) void k_f4_rays(const float2* __restrict__ Xr, float* __restrict__ sino,
                                               const float2* __restrict__ tw, int n_views) {
    constexpr int HQ = ND / 2 + 1;
    __shared__ float2 lds[ND];
    const int tid = threadIdx.x;
    const int a0 = blockIdx.x * 2;
    const bool has_b = a0 + 1 < n_views;
    const float2* xa = Xr + (size_t)a0 * HQ;
    const float2* xb = Xr + (size_t)(a0 + 1) * HQ;
    const float2 zero = make_float2(0.f, 0.f);
    // Z = A + i B, stored conjugated so the forward engine gives conj(IFFT)
    for (int q = tid; q < ND; q += NT) {
        float2 A, B;
        if (q == 0 || q == ND / 2) {
            A = make_float2(xa[q].x, 0.f);
            B = has_b ? make_float2(xb[q].x, 0.f) : zero;
        } else if (q < ND / 2) {
            A = xa[q];
            B = has_b ? xb[q] : zero;
        } else {
            A = cconj(xa[ND - q]);
            B = has_b ? cconj(xb[ND - q]) : zero;
        }
        lds[q] = make_float2(A.x - B.y, -(A.y + B.x));
    }
    __syncthreads();
    fft_lds<ND, 1, NT>(lds, tw, tid);
    const float inv = 1.0f / (float)ND;
    for (int d = tid; d < ND; d += NT) {
        const float2 z = cconj(lds[(d + ND / 2) % ND]);
        sino[(size_t)a0 * ND + d] = z.x * inv;
        if (has_b) sino[(size_t)(a0 + 1) * ND + d] = z.y * inv;
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
// Deterministic binned spreading, one wave per work item (a slice of one
// output tile's visit list). The visit list of tile (cx, cy) is the
// concatenation of: the diagonal neighbour bin's class 2, the v-neighbour
// bin's classes 2-3, the u-neighbour bin's classes 1-2 and the own bin (all
// classes) -- exactly the samples whose footprint reaches the tile.
//
// Lane l takes visits l*S .. l*S+S-1 (S = ceil(count/64)), one per round. In
// a round each lane computes its sample's W x-weights and W values Y*wy, then
// adds its W x W footprint into a halo'd LDS accumulator, one footprint point
// per instruction. Lanes whose footprint origins coincide would collide, so
// a round runs in sub-rounds: the lowest pending lane of each origin cell
// (claimed with an integer atomic min, deterministic) adds, the others wait.
// Every grid value is therefore accumulated in one fixed order.
template <int W, int T>
__global__ __launch_bounds__(64) void k_a2_spread(const TileItem* __restrict__ items,
                                                 const int* __restrict__ offs4, const int* __restrict__ perm,
                                                 const float2* __restrict__ Yh, const double2* __restrict__ cs,
                                                 const float4* __restrict__ kbc, float kbS,
                                                 float2* __restrict__ grid, float2* __restrict__ partials,
                                                 int G, int ND, int n_views) {
    constexpr int P = T + 2 * (W - 1);   // accumulator side: local [-(W-1), T+W-1)
    constexpr int C = T + W - 1;         // origin cells: local [-(W-1), T)
    constexpr int FREE = 64;
    __shared__ float2 acc[P * P];
    __shared__ int owner[C * C];
    const int lane = threadIdx.x;
    const TileItem it = items[blockIdx.x];
    const int ntl = G / T;
    const int M = n_views * ND;
    const int HQ = ND / 2 + 1;
    const float hw = 0.5f * (float)W;

    for (int e = lane; e < P * P; e += 64) acc[e] = make_float2(0.f, 0.f);
    for (int e = lane; e < C * C; e += 64) owner[e] = FREE;

    const int xl = (it.cx + ntl - 1) % ntl, yu = (it.cy + ntl - 1) % ntl;
    const int b_ul = yu * ntl + xl, b_u = yu * ntl + it.cx, b_l = it.cy * ntl + xl, b_o = it.cy * ntl + it.cx;
    const int s0 = offs4[4 * b_ul + 2], n0 = offs4[4 * b_ul + 3] - s0;
    const int s1 = offs4[4 * b_u + 2], n1 = offs4[4 * b_u + 4] - s1;
    const int s2 = offs4[4 * b_l + 1], n2 = offs4[4 * b_l + 3] - s2;
    const int s3 = offs4[4 * b_o];
    const int x0 = it.cx * T, y0 = it.cy * T;
    const int xvalid = (it.cx == 0) ? 1 : T;   // tile column 0 holds only mx = G/2
    const int S = (it.count + 63) / 64;
    __syncthreads();

    for (int r = 0; r < S; ++r) {
        const int t = lane * S + r;
        bool pending = t < it.count;
        int base = 0, cell = 0;
        float wx[W];
        float2 ywy[W];
        if (pending) {
            int u = it.start + t, pos;
            if (u < n0) pos = s0 + u;
            else if ((u -= n0) < n1) pos = s1 + u;
            else if ((u -= n1) < n2) pos = s2 + u;
            else pos = s3 + (u - n2);
            const int v = perm[pos];
            int a, q;
            decode_sample(v, M, ND, a, q);
            float2 Y;
            if (q >= 0 && q < ND / 2) Y = Yh[(size_t)a * HQ + q];
            else if (q < 0 && q > -ND / 2) Y = cconj(Yh[(size_t)a * HQ - q]);
            else Y = Yh[(size_t)a * HQ + ND / 2];
            const double2 csa = cs[a];
            const SampleGeom g = sample_geom(csa.x, csa.y, q, G, ND);
            int ox = footprint_origin(g.bu, W, G) - x0;
            int oy = footprint_origin(g.bv, W, G) - y0;
            if (ox >= G / 2) ox -= G;
            if (ox < -G / 2) ox += G;
            if (oy >= G / 2) oy -= G;
            if (oy < -G / 2) oy += G;
            base = (ox + W - 1) * P + (oy + W - 1);
            cell = (ox + W - 1) * C + (oy + W - 1);
#pragma unroll
            for (int al = 0; al < W; ++al) wx[al] = kb_weight(fabsf(g.fu + (float)(W / 2 - 1 - al)), kbc, kbS, hw);
#pragma unroll
            for (int gm = 0; gm < W; ++gm) {
                const float wy = kb_weight(fabsf(g.fv + (float)(W / 2 - 1 - gm)), kbc, kbS, hw);
                ywy[gm] = make_float2(Y.x * wy, Y.y * wy);
            }
        }
        while (__ballot(pending) != 0) {
            if (pending) atomicMin(&owner[cell], lane);
            __builtin_amdgcn_wave_barrier();
            const bool win = pending && __hip_atomic_load(&owner[cell], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP) == lane;
            if (win) {
                // One footprint point per step. Winners have distinct origin
                // cells, so within a step every lane touches its own address,
                // but step k of one lane may hit the address of step j of
                // another: the compiler barrier keeps each step's read after
                // the previous step's write (the LDS executes a wave's
                // instructions in order).
                float2* dst = acc + base;
#pragma unroll
                for (int al = 0; al < W; ++al) {
#pragma unroll
                    for (int gm = 0; gm < W; ++gm) {
                        float2 o = dst[al * P + gm];
                        o.x = fmaf(wx[al], ywy[gm].x, o.x);
                        o.y = fmaf(wx[al], ywy[gm].y, o.y);
                        dst[al * P + gm] = o;
                        asm volatile("" ::: "memory");
                    }
                }
                __hip_atomic_store(&owner[cell], FREE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            pending = pending && !win;
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    // write out: local (lx, ly) -> mx = (x0 + lx - G/2) mod G, my = (y0 + ly - G/2) mod G
    const int my0 = mod_pos(y0 - G / 2, G);
    for (int e = lane; e < xvalid * T; e += 64) {
        const int lx = e / T, ly = e - lx * T;
        const float2 val = acc[(lx + W - 1) * P + (ly + W - 1)];
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

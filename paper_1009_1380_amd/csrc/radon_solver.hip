// radon_solver.hip - basis-pursuit denoising on the GPU (SPGL1 root finding).
//
// The paper reconstructs a slice as min ||x||_1 subject to
// ||filter(Radon{x} - data)||_2 < epsilon, solved with SPGL1 (introduction,
// problem statement), where filter is a 3rd-order polynomial ring filter.
// Here:
//   * ring filter F: m[d] = mean over views of y[., d]; F y = y - 1 (x) (m - P3 m),
//     P3 the least-squares projection onto cubic polynomials in s_d (an
//     orthonormal basis Q, N x 4, built in float64 on the host);
//   * SPGL1 (van den Berg & Friedlander 2008): Newton steps on tau for the
//     Pareto curve, spectral projected gradient with a non-monotone line
//     search for each LASSO(tau), projection onto the l1 ball.
// Vectors are float32 on the device; every dot product, norm and sum is
// accumulated in float64 in a fixed order (per-block partials, then one block
// sums the partials in block order), so a solve is bitwise reproducible.
// The host loop reads back a handful of float64 scalars per iteration.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "../../include/radon.h"
#include "radon_internal.hpp"

namespace rn {

constexpr int SV_NT = 256;           // threads per reduction block
#ifndef RN_SV_BLOCKS
#define RN_SV_BLOCKS 512
#endif
constexpr int SV_BLOCKS = RN_SV_BLOCKS;   // blocks of the grid-stride reductions
constexpr int SV_SLOTS = 8;          // partial-result slots

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// Fixed-order block reduction of up to SV_NT values (sum or max).
template <bool MAX>
__device__ double block_reduce(double v, double* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = MAX ? wave_max(v) : wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = MAX ? 0.0 : 0.0;
    if (threadIdx.x == 0) {
        r = sh[0];
        for (int w = 1; w < SV_NT / 64; ++w) r = MAX ? fmax(r, sh[w]) : r + sh[w];
    }
    return r;   // valid in thread 0
}

// Sum (or max) of the SV_BLOCKS per-block partials of each slot, in block
// order: every thread loads its strided share of every slot at once, folds it,
// the waves reduce, and thread s adds the wave results of slot s in wave order.
// ops bit k set: slot k is a max, else a sum. nslots <= SV_FIN_SLOTS. out may
// be pinned host memory, which the host reads once the stream has finished.
constexpr int SV_FIN_SLOTS = 9;
__global__ __launch_bounds__(SV_NT) void k_sv_final(const double* __restrict__ part, int nslots, unsigned ops,
                                                   double* __restrict__ out) {
    constexpr int PER = (SV_BLOCKS + SV_NT - 1) / SV_NT;
    __shared__ double sh[SV_FIN_SLOTS][SV_NT / 64];
    double p[SV_FIN_SLOTS][PER];
#pragma unroll
    for (int s = 0; s < SV_FIN_SLOTS; ++s)
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int b = threadIdx.x + k * SV_NT;
            p[s][k] = (s < nslots && b < SV_BLOCKS) ? part[(size_t)s * SV_BLOCKS + b] : 0.0;
        }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < SV_FIN_SLOTS; ++s) {
        const bool mx = (ops >> s) & 1u;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < PER; ++k) v = mx ? fmax(v, p[s][k]) : v + p[s][k];
        v = mx ? wave_max(v) : wave_sum(v);
        if (lane == 0) sh[s][wave] = v;
    }
    __syncthreads();
    const int s = threadIdx.x;
    if (s < nslots) {
        const bool mx = (ops >> s) & 1u;
        double r = sh[s][0];
        for (int w = 1; w < SV_NT / 64; ++w) r = mx ? fmax(r, sh[s][w]) : r + sh[s][w];
        out[s] = r;
    }
}

// m[d] = mean over views of (b - z)[., d] (z may be null: m = mean of b).
// A block takes 32 detectors; its 8 thread groups sum every 8th view, and the
// 8 group sums are added in group order.
__global__ __launch_bounds__(256) void k_sv_colmean(const float* __restrict__ b, const float* __restrict__ z,
                                                   int nv, int N, double* __restrict__ m) {
    __shared__ double part[8][32];
    const int dl = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int d = blockIdx.x * 32 + dl;
    double s = 0.0;
    if (d < N) {
        for (int a = g; a < nv; a += 8) {
            const size_t i = (size_t)a * N + d;
            s += (double)b[i] - (z ? (double)z[i] : 0.0);
        }
    }
    part[g][dl] = s;
    __syncthreads();
    if (g == 0 && d < N) {
        double t = part[0][dl];
        for (int k = 1; k < 8; ++k) t += part[k][dl];
        m[d] = t / nv;
    }
}

// ring[d] = m[d] - (Q Q^T m)[d]  (one block). The four coefficients
// c_k = sum_d Q[d][k] m[d] are accumulated together, each in the order of
// block_reduce (per thread over d, then the waves, then the wave sums in order).
__global__ __launch_bounds__(SV_NT) void k_sv_ringfit(const double* __restrict__ m, const double* __restrict__ Q,
                                                     int N, double* __restrict__ ring) {
    __shared__ double sh[4][SV_NT / 64];
    __shared__ double c[4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int d = threadIdx.x; d < N; d += SV_NT) {
        const double md = m[d];
        const double* q = Q + (size_t)d * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += q[k] * md;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double r = wave_sum(v[k]);
        if (lane == 0) sh[k][wave] = r;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        double r = sh[k][0];
        for (int w = 1; w < SV_NT / 64; ++w) r += sh[k][w];
        c[k] = r;
    }
    __syncthreads();
    for (int d = threadIdx.x; d < N; d += SV_NT) {
        const double* q = Q + (size_t)d * 4;
        ring[d] = m[d] - (q[0] * c[0] + q[1] * c[1] + q[2] * c[2] + q[3] * c[3]);
    }
}

// r = (b - z) - ring[d] (ring may be null; z may be null); partials of
// slot 0: sum r^2, slot 1: sum r * bt (bt may be null).
__global__ __launch_bounds__(SV_NT) void k_sv_resid(const float* __restrict__ b, const float* __restrict__ z,
                                                   const double* __restrict__ ring, const float* __restrict__ bt,
                                                   int nv, int N, float* __restrict__ r, double* __restrict__ part) {
    __shared__ double sh[SV_NT / 64];
    const size_t total = (size_t)nv * N;
    double s0 = 0.0, s1 = 0.0;
    for (size_t i = (size_t)blockIdx.x * SV_NT + threadIdx.x; i < total; i += (size_t)gridDim.x * SV_NT) {
        double v = (double)b[i] - (z ? (double)z[i] : 0.0);
        if (ring) v -= ring[i % N];
        const float rf = (float)v;
        r[i] = rf;
        s0 += (double)rf * rf;
        if (bt) s1 += (double)rf * bt[i];
    }
    double t = block_reduce<false>(s0, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_reduce<false>(s1, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = t;
}

// Barzilai-Borwein quantities with s = xn - x and y = gn - g = -(hn - h):
// slot 0 sum s^2, slot 1 sum s y, slot 2 max |hn| (= ||gn||_inf),
// slot 3 sum |x| of the input x (used for tau at a warm start).
// The image-sized kernels below walk n/4 16-byte pieces (n = n_image^2 is a
// multiple of 64), SV_U pieces of each array per thread and round, all loaded
// before any is used: with one grid-stride element per round a thread waited
// out one memory latency per element.
constexpr int SV_U = 4;

__device__ __forceinline__ float4 ld4(const float* __restrict__ p, size_t j, size_t n4) {
    return j < n4 ? reinterpret_cast<const float4*>(p)[j] : make_float4(0.f, 0.f, 0.f, 0.f);
}
__device__ __forceinline__ float comp(const float4& v, int c) {
    return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}

__global__ __launch_bounds__(SV_NT) void k_sv_bb(const float* __restrict__ x, const float* __restrict__ xn,
                                                const float* __restrict__ h, const float* __restrict__ hn, size_t n,
                                                double* __restrict__ part) {
    __shared__ double sh[SV_NT / 64];
    double ss = 0.0, sy = 0.0, mx = 0.0, l1 = 0.0;
    const size_t n4 = n / 4, stride = (size_t)gridDim.x * SV_NT;
    for (size_t j0 = (size_t)blockIdx.x * SV_NT + threadIdx.x; j0 < n4; j0 += stride * SV_U) {
        float4 xv[SV_U], xnv[SV_U], hv[SV_U], hnv[SV_U];
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
            const size_t j = j0 + u * stride;
            xnv[u] = ld4(xn, j, n4);
            hnv[u] = ld4(hn, j, n4);
            xv[u] = x ? ld4(x, j, n4) : make_float4(0.f, 0.f, 0.f, 0.f);
            hv[u] = h ? ld4(h, j, n4) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double s = (x ? (double)comp(xnv[u], c) - (double)comp(xv[u], c) : 0.0);
                const double y = (h ? -((double)comp(hnv[u], c) - (double)comp(hv[u], c)) : 0.0);
                ss += s * s;
                sy += s * y;
                mx = fmax(mx, fabs((double)comp(hnv[u], c)));
                l1 += fabs((double)comp(xnv[u], c));
            }
        }
    }
    double t = block_reduce<false>(ss, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_reduce<false>(sy, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = t;
    t = block_reduce<true>(mx, sh);
    if (threadIdx.x == 0) part[2 * gridDim.x + blockIdx.x] = t;
    t = block_reduce<false>(l1, sh);
    if (threadIdx.x == 0) part[3 * gridDim.x + blockIdx.x] = t;
}

// Projection onto the l1 ball: xn = soft(v, lam), v = x + c h (rounded to
// float32, as the soft threshold forms it), with lam the root of
// S(lam) = sum max(|v| - lam, 0) = tau. S is continuous, decreasing and
// piecewise linear with breakpoints at the values |v_i|, so the root is found
// exactly by locating it between two consecutive values: a radix select on the
// bit pattern u of |v| (monotone in |v| for non-negative floats), 12 + 10 + 9
// bits in three levels (a narrower second level makes the merge of its
// histograms into global memory and the decision after it cheaper than with
// 12 + 12 + 7). Each level histograms the elements whose leading bits match
// the bin chosen so far, by count and by the exact integer sum of their
// significands (the bins of a level share one exponent), so the histograms are
// order-independent integers and the select is deterministic. From the counts
// and sums above each bin edge e, S(e) is exact up to the final float64 sums;
// the highest non-empty bin whose lower edge has S >= tau is either refined by
// the next level or, when the root lies in an empty gap, below every element
// in play, or the bins are single values, gives
// lam = (sum of |v| above the root - tau) / (their count). Special cases:
// sum |v| <= tau gives lam = 0 (v is in the ball); tau = 0 gives a lam at or
// above max |v|; a NaN or infinite v gives lam = NaN, which the soft threshold
// turns into NaN outputs.
// Launches: the level-1, level-2 and level-3 histogram passes, then the soft
// threshold. There is no grid-wide wait inside a launch: every block of the
// next launch takes the previous level's decision itself from the finished
// histogram (the same decision in every block), so the kernel boundary is the
// only synchronisation, and block 0 records it for the launches after.
constexpr int PJ_NT = 256;
#ifndef RN_PJ_BLOCKS
#define RN_PJ_BLOCKS 256
#endif
constexpr int PJ_BLOCKS = RN_PJ_BLOCKS;
#ifndef RN_PJ_B2
#define RN_PJ_B2 10
#endif
constexpr int PJ_B1 = 12, PJ_B2 = RN_PJ_B2, PJ_B3 = 31 - PJ_B1 - PJ_B2;   // bits of the three levels
constexpr int PJ_BINS = 4096;            // histogram capacity of levels 1 and 2 (at most 12 bits)
constexpr int PJ_BINS3 = 1 << PJ_B3;     // bins of level 3 (one float value each)
static_assert(PJ_B2 <= 12 && PJ_B3 >= 1 && PJ_B3 <= 12, "level widths");

// Decision after a level: the threshold (done), or the bin to refine (the
// leading bits of u fixed so far) with the sum and count of |v| above it.
struct PjState {
    double lam, done, A, C;
    unsigned prefix, pad;
};

// Global histograms of the three levels (counts; sums of the bits below the
// digit), the count of non-finite v, and the decisions after levels 1 and 2.
// A level's histogram is cleared by a launch after the one that reads it.
struct PjWork {
    unsigned *cnt1, *cnt2, *cnt3;
    unsigned long long *sum1, *sum2, *sum3;
    unsigned* bad;
    PjState *st1, *st2;
};

template <int L>
struct PjLevel {
    static constexpr int BITS = L == 1 ? PJ_B1 : L == 2 ? PJ_B2 : PJ_B3;
    static constexpr int NB = 1 << BITS;
    static constexpr int SHIFT = L == 1 ? 31 - PJ_B1 : L == 2 ? 31 - PJ_B1 - PJ_B2 : 0;   // digit = (u >> SHIFT) % NB
    static constexpr int PSHIFT = SHIFT + BITS;   // u >> PSHIFT must equal the prefix
    // bit pattern of the lower edge of bin b (b = NB carries into the prefix)
    __device__ static unsigned edge(unsigned prefix, unsigned b) {
        return L == 1 ? b << SHIFT : (prefix << PSHIFT) + (b << SHIFT);
    }
};

// v exactly as the soft threshold forms it
__device__ __forceinline__ float pj_v(float x, float h, double c) { return (float)((double)x + c * (double)h); }

// Block-wide: the decision of level L from its finished histogram, given the
// decision above it (up: prefix, and the sum A and count C of |v| above the bin
// it chose; zero for level 1). Every thread returns the same decision. lc, ls:
// shared scratch of NB entries, free again when this returns.
template <int L>
__device__ PjState pj_decide(const unsigned* __restrict__ hcnt, const unsigned long long* __restrict__ hsum,
                             unsigned nbad, const PjState& up, double tau, unsigned* lc, unsigned long long* ls) {
    using Lv = PjLevel<L>;
    constexpr int NB = Lv::NB;
    constexpr int RL = (NB + PJ_NT - 1) / PJ_NT;
    __shared__ double sC[PJ_NT / 64], sV[PJ_NT / 64];
    __shared__ int sb[PJ_NT / 64];
    __shared__ double dC, dV, dS;   // the chosen bin: count and sum above it, S at its upper edge
    __shared__ PjState out;
    const unsigned prefix = L == 1 ? 0u : up.prefix;
    {   // coalesced loads, all in flight at once, into LDS
        unsigned cv[RL];
        unsigned long long sv[RL];
#pragma unroll
        for (int k = 0; k < RL; ++k) {
            const int b = threadIdx.x + k * PJ_NT;
            cv[k] = b < NB ? hcnt[b] : 0u;
            sv[k] = b < NB ? hsum[b] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < RL; ++k) {
            const int b = threadIdx.x + k * PJ_NT;
            if (b < NB) { lc[b] = cv[k]; ls[b] = sv[k]; }
        }
    }
    __syncthreads();
    // this thread's RL consecutive bins: count and exact value sum of each
    const int b0 = threadIdx.x * RL;
    double Cb[RL], Vb[RL];
    double tC = 0.0, tV = 0.0;
#pragma unroll
    for (int r = RL - 1; r >= 0; --r) {   // high bins first, the order of the running sums below
        const int b = b0 + r;
        Cb[r] = 0.0;
        Vb[r] = 0.0;
        if (b < NB && lc[b]) {
            const unsigned cnt = lc[b];
            const unsigned ub = Lv::edge(prefix, (unsigned)b);
            const unsigned eb = ub >> 23;
            const unsigned sig = (eb ? 0x800000u : 0u) | (ub & 0x7fffffu);   // significand of the bin's edge
            Cb[r] = (double)cnt;
            Vb[r] = ldexp((double)cnt * (double)sig + (double)ls[b], (int)(eb ? eb : 1u) - 150);
        }
        tC += Cb[r];
        tV += Vb[r];
    }
    // exclusive suffix sums of the thread totals over the higher threads, in a fixed order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double iC = tC, iV = tV;   // inclusive suffix within the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double oC = __shfl_down(iC, off), oV = __shfl_down(iV, off);
        if (lane + off < 64) { iC += oC; iV += oV; }
    }
    if (lane == 0) { sC[wave] = iC; sV[wave] = iV; }
    double xC = __shfl_down(iC, 1), xV = __shfl_down(iV, 1);
    if (lane == 63) { xC = 0.0; xV = 0.0; }
    __syncthreads();
    double aC = L == 1 ? 0.0 : up.C, aV = L == 1 ? 0.0 : up.A;   // everything above this thread's bins
    for (int w = PJ_NT / 64 - 1; w > wave; --w) { aC += sC[w]; aV += sV[w]; }
    aC += xC;
    aV += xV;
    // this thread's highest non-empty bin whose lower edge has S >= tau
    int cand = -1;
    double cC = 0.0, cV = 0.0, cS = 0.0;
#pragma unroll
    for (int r = RL - 1; r >= 0; --r) {
        const int b = b0 + r;
        if (cand < 0 && Cb[r] > 0.0) {
            const double lo = (double)__uint_as_float(Lv::edge(prefix, (unsigned)b));
            const double hi = (double)__uint_as_float(Lv::edge(prefix, (unsigned)b + 1u));
            if ((aV + Vb[r]) - (aC + Cb[r]) * lo >= tau) {
                cand = b;
                cC = aC;
                cV = aV;
                cS = aV - aC * hi;
            }
        }
        aC += Cb[r];
        aV += Vb[r];
    }
    int bm = cand;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) bm = max(bm, __shfl_xor(bm, off));
    if (lane == 0) sb[wave] = bm;
    __syncthreads();
    int bstar = sb[0];
    for (int w = 1; w < PJ_NT / 64; ++w) bstar = max(bstar, sb[w]);
    if (bstar >= 0 && cand == bstar) {
        dC = cC;
        dV = cV;
        dS = cS;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        PjState d{0.0, 1.0, 0.0, 0.0, 0u, 0u};
        if (nbad) {
            d.lam = __builtin_nan("");
        } else if (bstar < 0) {
            // the root lies below every element in play: all of them are active
            // (aC, aV of thread 0 hold everything)
            d.lam = aC > 0.0 ? fmax(0.0, (aV - tau) / aC) : 0.0;
        } else if (dS >= tau || L == 3) {
            // the root lies above the chosen bin's elements: the active set is
            // everything above the bin (nothing above: tau = 0, all go to zero)
            d.lam = dC > 0.0 ? (dV - tau) / dC : (double)__uint_as_float(Lv::edge(prefix, (unsigned)bstar + 1u));
        } else {   // the root is inside bin bstar: the next level refines it
            d.done = 0.0;
            d.A = dV;
            d.C = dC;
            d.prefix = L == 1 ? (unsigned)bstar : (prefix << Lv::BITS) | (unsigned)bstar;
        }
        out = d;
    }
    __syncthreads();
    return out;
}

// Level-L histogram pass. The step c and the radius tau are arguments of the
// level-1 pass, whose block 0 copies them to ct for the later launches; the
// level-2 and level-3 passes (c, tau unused) read them from ct. For L > 1
// every block first takes the decision of level L - 1 (block 0 records it);
// nothing is left to do once it is final.
template <int L>
__global__ __launch_bounds__(PJ_NT) void k_sv_pj_pass(const float* __restrict__ x, const float* __restrict__ h,
                                                     double c, double tau, double* __restrict__ ct, size_t n,
                                                     PjWork w) {
    using Lv = PjLevel<L>;
    constexpr int NB = Lv::NB;
    constexpr unsigned LOW = (1u << Lv::SHIFT) - 1;   // bits below the digit
    constexpr int CSHIFT = 40;   // LDS bin: count << 40 | sum of the bits below the digit
    __shared__ unsigned long long lh[PJ_BINS];
    __shared__ unsigned lc[PJ_BINS];
    __shared__ unsigned lbad;
    const size_t n4 = n / 4, stride = (size_t)gridDim.x * PJ_NT;
    const size_t jfirst = (size_t)blockIdx.x * PJ_NT + threadIdx.x;
    float4 xv[SV_U], hv[SV_U];   // the first round's pieces, in flight during the decision
#pragma unroll
    for (int u = 0; u < SV_U; ++u) {
        xv[u] = ld4(x, jfirst + u * stride, n4);   // zero padding: u = 0 is skipped
        hv[u] = ld4(h, jfirst + u * stride, n4);
    }
    if (L == 1) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { ct[0] = c; ct[1] = tau; }
    } else {
        c = ct[0];
        tau = ct[1];
    }
    unsigned prefix = 0u;
    if (L == 1) {
        // the level-3 histogram was read by the last soft threshold: clear it
        if (blockIdx.x == 0) {
            for (int b = threadIdx.x; b < PJ_BINS3; b += PJ_NT) {
                w.cnt3[b] = 0u;
                w.sum3[b] = 0ull;
            }
        }
    } else {
        PjState up{0.0, 0.0, 0.0, 0.0, 0u, 0u};
        if (L == 3) {
            up = *w.st1;
            if (up.done != 0.0) return;   // final after level 1 (uniform)
        }
        const PjState d = L == 2 ? pj_decide<1>(w.cnt1, w.sum1, *w.bad, up, tau, lc, lh)
                                 : pj_decide<2>(w.cnt2, w.sum2, 0u, up, tau, lc, lh);
        if (blockIdx.x == 0 && threadIdx.x == 0) *(L == 2 ? w.st1 : w.st2) = d;
        if (d.done != 0.0) return;   // uniform
        prefix = d.prefix;
    }
    for (int b = threadIdx.x; b < NB; b += PJ_NT) lh[b] = 0ull;
    if (threadIdx.x == 0) lbad = 0u;
    __syncthreads();

    unsigned bad = 0, cur = ~0u;
    unsigned long long acc = 0ull;   // run of equal digits, added to LDS in one atomic
    for (size_t j0 = jfirst; j0 < n4; j0 += stride * SV_U) {
        if (j0 != jfirst) {
#pragma unroll
            for (int u = 0; u < SV_U; ++u) {
                xv[u] = ld4(x, j0 + u * stride, n4);
                hv[u] = ld4(h, j0 + u * stride, n4);
            }
        }
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const unsigned m = __float_as_uint(pj_v(comp(xv[u], e), comp(hv[u], e), c)) & 0x7fffffffu;
                if (m >= 0x7f800000u) { bad += L == 1; continue; }
                if (m == 0u || (L > 1 && (m >> Lv::PSHIFT) != prefix)) continue;
                const unsigned dg = (m >> Lv::SHIFT) & (NB - 1);
                if (dg != cur) {
                    if (acc) atomicAdd(&lh[cur], acc);
                    cur = dg;
                    acc = 0ull;
                }
                acc += (1ull << CSHIFT) + (m & LOW);
            }
        }
    }
    if (acc) atomicAdd(&lh[cur], acc);
    if (L == 1 && bad) atomicAdd(&lbad, bad);
    __syncthreads();
    unsigned* gc = L == 1 ? w.cnt1 : L == 2 ? w.cnt2 : w.cnt3;
    unsigned long long* gs = L == 1 ? w.sum1 : L == 2 ? w.sum2 : w.sum3;
    for (int b = threadIdx.x; b < NB; b += PJ_NT) {
        const unsigned long long v = lh[b];
        if (v) {
            atomicAdd(&gc[b], (unsigned)(v >> CSHIFT));
            atomicAdd(&gs[b], v & ((1ull << CSHIFT) - 1));
        }
    }
    if (L == 1 && threadIdx.x == 0 && lbad) atomicAdd(w.bad, lbad);
}

// xn = soft(x + c h, lam), lam the final decision (taken here from the
// level-3 histogram when the first two levels did not finish), ct = (c, tau)
// as the level-1 pass copied them; partials: slot 0 sum -h.(xn - x), slot 1
// sum |xn|, slot 2 lam (block 0; 0 elsewhere). Clears the level-1 and level-2
// histograms for the next projection.
__global__ __launch_bounds__(SV_NT) void k_sv_soft(const float* __restrict__ x, const float* __restrict__ h,
                                                  const double* __restrict__ ct, size_t n, PjWork w,
                                                  float* __restrict__ xn, double* __restrict__ part) {
    __shared__ double sh[SV_NT / 64];
    __shared__ unsigned lc[PJ_BINS3];
    __shared__ unsigned long long ls[PJ_BINS3];
    const double c = ct[0], tau = ct[1];
    double L;
    const PjState s1 = *w.st1;
    if (s1.done != 0.0) {
        L = s1.lam;
    } else {
        const PjState s2 = *w.st2;
        L = s2.done != 0.0 ? s2.lam : pj_decide<3>(w.cnt3, w.sum3, 0u, s2, tau, lc, ls).lam;
    }
    {
        const size_t i = (size_t)blockIdx.x * SV_NT + threadIdx.x, all = (size_t)gridDim.x * SV_NT;
        for (size_t b = i; b < (size_t)PJ_BINS; b += all) {
            w.cnt1[b] = 0u;
            w.sum1[b] = 0ull;
            w.cnt2[b] = 0u;
            w.sum2[b] = 0ull;
        }
        if (i == 0) *w.bad = 0u;
    }
    double s0 = 0.0, s1s = 0.0;
    const size_t n4 = n / 4, stride = (size_t)gridDim.x * SV_NT;
    for (size_t j0 = (size_t)blockIdx.x * SV_NT + threadIdx.x; j0 < n4; j0 += stride * SV_U) {
        float4 xv[SV_U], hv[SV_U];
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
            xv[u] = ld4(x, j0 + u * stride, n4);
            hv[u] = ld4(h, j0 + u * stride, n4);
        }
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
            float o4[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double xe = (double)comp(xv[u], e), he = (double)comp(hv[u], e);
                const float v = pj_v(comp(xv[u], e), comp(hv[u], e), c);
                const double a = fabs((double)v) - L;
                // a NaN (from v or from lam) stays NaN
                const float o = a > 0 ? (float)copysign(a, (double)v) : a <= 0 ? 0.0f : __builtin_nanf("");
                o4[e] = o;
                s0 += -he * ((double)o - xe);
                s1s += fabs((double)o);
            }
            const size_t j = j0 + u * stride;
            if (j < n4) reinterpret_cast<float4*>(xn)[j] = make_float4(o4[0], o4[1], o4[2], o4[3]);
        }
    }
    double t = block_reduce<false>(s0, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_reduce<false>(s1s, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = t;
    if (threadIdx.x == 0) part[2 * gridDim.x + blockIdx.x] = blockIdx.x == 0 ? L : 0.0;
}

__global__ __launch_bounds__(256) void k_sv_fill(float* __restrict__ v, size_t n, float val) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) v[i] = val;
}

// Orthonormal basis of cubic polynomials in s = d - N/2, scaled to [-1, 1),
// by modified Gram-Schmidt (twice) in float64; row-major N x 4.
std::vector<double> ring_cubic_basis(int N) {
    std::vector<double> Q((size_t)N * 4);
    for (int d = 0; d < N; ++d) {
        const double t = ((double)d - N / 2) / (N / 2);
        double pw = 1.0;
        for (int k = 0; k < 4; ++k) { Q[(size_t)d * 4 + k] = pw; pw *= t; }
    }
    for (int pass = 0; pass < 2; ++pass) {
        for (int k = 0; k < 4; ++k) {
            for (int j = 0; j < k; ++j) {
                double dot = 0;
                for (int d = 0; d < N; ++d) dot += Q[(size_t)d * 4 + k] * Q[(size_t)d * 4 + j];
                for (int d = 0; d < N; ++d) Q[(size_t)d * 4 + k] -= dot * Q[(size_t)d * 4 + j];
            }
            double nrm = 0;
            for (int d = 0; d < N; ++d) nrm += Q[(size_t)d * 4 + k] * Q[(size_t)d * 4 + k];
            nrm = sqrt(nrm);
            for (int d = 0; d < N; ++d) Q[(size_t)d * 4 + k] /= nrm;
        }
    }
    return Q;
}

}  // namespace rn

// ------------------------------------------------------------------ host side

namespace {

struct SolveWork {
    std::vector<void*> allocs, host_allocs;
    float *x = nullptr, *xn = nullptr, *h = nullptr, *hn = nullptr;
    float *z = nullptr, *r = nullptr, *rn = nullptr, *bt = nullptr;
    double *m = nullptr, *ring = nullptr, *Q = nullptr, *part = nullptr;
    // fin_h: pinned, coherent host memory the fold kernel writes each read's
    // sums to; ct: the projection's step and radius for its later launches
    double *fin_h = nullptr, *ct = nullptr;
    // l1 projection: histograms of the three levels (counts, sums), the
    // non-finite count, the decisions after levels 1 and 2
    static constexpr size_t PJ_ALL = 2 * (size_t)rn::PJ_BINS + rn::PJ_BINS3;
    unsigned* pjc = nullptr;
    unsigned long long* pjs = nullptr;
    unsigned* pjbad = nullptr;
    rn::PjState* pjst = nullptr;
    rn::PjWork pj() const {
        return rn::PjWork{pjc, pjc + rn::PJ_BINS, pjc + 2 * rn::PJ_BINS, pjs, pjs + rn::PJ_BINS,
                          pjs + 2 * rn::PJ_BINS, pjbad, pjst, pjst + 1};
    }
    ~SolveWork() {
        for (void* p : allocs) (void)hipFree(p);
        for (void* p : host_allocs) (void)hipHostFree(p);
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
    bool alloc_host(double** out, size_t count) {
        void* p = nullptr;
        if (hipHostMalloc(&p, sizeof(double) * count, hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        host_allocs.push_back(p);
        *out = static_cast<double*>(p);
        return true;
    }
};

std::vector<double> cubic_basis(int N) { return rn::ring_cubic_basis(N); }

// fin slots: 0-1 residual (sum r^2, sum r.b~), 2-4 projection (g.dx, ||xn||_1,
// the threshold lam), 5-8 spectral step (sum s^2, sum s.y, max |hn|, ||xn||_1)
constexpr int FIN_RES = 0, FIN_PROJ = 2, FIN_BB = 5, FIN_COUNT = 9;
constexpr unsigned FIN_MAX_OPS = 1u << (FIN_BB + 2);   // the max slot
static_assert(FIN_COUNT <= rn::SV_FIN_SLOTS, "fin slots");

struct Solver {
    radon_plan_t plan;
    const rn::Plan& p;
    SolveWork& w;
    hipStream_t st;
    bool filt;
    const float* b;
    size_t n2, ns;
    int nf = 0, na = 0;
    hipError_t err = hipSuccess;

    void chk(hipError_t e) { if (err == hipSuccess && e != hipSuccess) err = e; }

    double* part(int slot) { return w.part + (size_t)slot * rn::SV_BLOCKS; }
    // fold the per-block partials of every slot into the host's fin (slots no
    // kernel wrote since the last fold hold their earlier partials)
    void fold() {
        hipLaunchKernelGGL(rn::k_sv_final, dim3(1), dim3(rn::SV_NT), 0, st, w.part, FIN_COUNT, FIN_MAX_OPS, w.fin_h);
        chk(hipGetLastError());
    }
    // wait for the stream and copy fin out
    bool wait(double* out) {
        chk(hipStreamSynchronize(st));
        if (err != hipSuccess) return false;
        std::copy(w.fin_h, w.fin_h + FIN_COUNT, out);
        return true;
    }
    bool read(double* out) {
        fold();
        return wait(out);
    }

    // r = F(b - z) (z may be null) -> fin[0] = sum r^2, fin[1] = sum r.bt (bt may be null)
    void residual(const float* z, float* r, const float* bt) {
        const double* ring = nullptr;
        if (filt) {
            hipLaunchKernelGGL(rn::k_sv_colmean, dim3((p.n_det + 31) / 32), dim3(256), 0, st, b, z, p.n_views,
                               p.n_det, w.m);
            hipLaunchKernelGGL(rn::k_sv_ringfit, dim3(1), dim3(rn::SV_NT), 0, st, w.m, w.Q, p.n_det, w.ring);
            ring = w.ring;
        }
        hipLaunchKernelGGL(rn::k_sv_resid, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, b, z, ring, bt, p.n_views,
                           p.n_det, r, part(FIN_RES));
        chk(hipGetLastError());
    }

    // xn = P_tau(x + c h) -> fin[2] = sum -h.(xn - x), fin[3] = ||xn||_1, fin[4] = lam
    void project(const float* x, const float* h, double c, double tau, float* xn) {
        const rn::PjWork pw = w.pj();
        hipLaunchKernelGGL(rn::k_sv_pj_pass<1>, dim3(rn::PJ_BLOCKS), dim3(rn::PJ_NT), 0, st, x, h, c, tau, w.ct, n2,
                           pw);
        hipLaunchKernelGGL(rn::k_sv_pj_pass<2>, dim3(rn::PJ_BLOCKS), dim3(rn::PJ_NT), 0, st, x, h, 0.0, 0.0, w.ct, n2,
                           pw);
        hipLaunchKernelGGL(rn::k_sv_pj_pass<3>, dim3(rn::PJ_BLOCKS), dim3(rn::PJ_NT), 0, st, x, h, 0.0, 0.0, w.ct, n2,
                           pw);
        hipLaunchKernelGGL(rn::k_sv_soft, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, x, h, w.ct, n2, pw, xn,
                           part(FIN_PROJ));
        chk(hipGetLastError());
    }

    // spectral-step sums of s = xn - x, y = -(hn - h) -> fin[4..7] (x, h may be null)
    void bb(const float* x, const float* xn, const float* h, const float* hn) {
        hipLaunchKernelGGL(rn::k_sv_bb, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, x, xn, h, hn, n2, part(FIN_BB));
        chk(hipGetLastError());
    }

    // project and read fin back
    bool project_sync(const float* x, const float* h, double c, double tau, float* xn, double* fin) {
        project(x, h, c, tau, xn);
        return read(fin);
    }
    // clear the projection histograms (every projection leaves them cleared;
    // this covers a run that follows one that stopped early)
    void reset_projection() {
        chk(hipMemsetAsync(w.pjc, 0, sizeof(unsigned) * SolveWork::PJ_ALL, st));
        chk(hipMemsetAsync(w.pjs, 0, sizeof(unsigned long long) * SolveWork::PJ_ALL, st));
        chk(hipMemsetAsync(w.pjbad, 0, sizeof(unsigned), st));
    }

    bool forward(const float* x, float* z) {
        ++nf;
        return radon_forward(plan, x, z, st) == RADON_OK;
    }
    bool adjoint(const float* r, float* h) {
        ++na;
        return radon_adjoint(plan, r, h, st) == RADON_OK;
    }

    // One line-search trial: xn = P_tau(x + c h), r_n = F(b - A xn),
    // h_n = A^T r_n, the spectral sums, and fin read back (one host wait)
    bool trial(double c, double tau, double* fin) {
        project(w.x, w.h, c, tau, w.xn);
        if (!forward(w.xn, w.z)) return false;
        residual(w.z, w.rn, w.bt);
        if (!adjoint(w.rn, w.hn)) return false;
        bb(w.x, w.xn, w.h, w.hn);
        return read(fin);
    }
};

}  // namespace

extern "C" radon_status_t radon_ring_filter(radon_plan_t plan, const float* y_dev, float* out_dev, void* stream) {
    if (!plan || !y_dev || !out_dev) return RADON_ERR_INVALID;
    const rn::Plan& p = plan->p;
    SolveWork w;
    if (!w.alloc(&w.m, p.n_det) || !w.alloc(&w.ring, p.n_det) || !w.alloc(&w.Q, (size_t)p.n_det * 4) ||
        !w.alloc(&w.part, (size_t)rn::SV_SLOTS * rn::SV_BLOCKS))
        return RADON_ERR_OOM;
    hipStream_t st = (hipStream_t)stream;
    const std::vector<double> Q = cubic_basis(p.n_det);
    if (hipMemcpy(w.Q, Q.data(), sizeof(double) * Q.size(), hipMemcpyHostToDevice) != hipSuccess)
        return RADON_ERR_DEVICE;
    hipLaunchKernelGGL(rn::k_sv_colmean, dim3((p.n_det + 31) / 32), dim3(256), 0, st, y_dev, nullptr, p.n_views,
                       p.n_det, w.m);
    hipLaunchKernelGGL(rn::k_sv_ringfit, dim3(1), dim3(rn::SV_NT), 0, st, w.m, w.Q, p.n_det, w.ring);
    hipLaunchKernelGGL(rn::k_sv_resid, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, y_dev, nullptr, w.ring, nullptr,
                       p.n_views, p.n_det, out_dev, w.part);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return RADON_ERR_DEVICE;
    return RADON_OK;
}

// ------------------------------------------------------------------ l1-ball projection

extern "C" radon_status_t radon_project_l1(const float* v_dev, int64_t n, double tau, float* out_dev,
                                           double* lam_host, void* stream) {
    if (n < 0 || n % 4) return rn::api_fail(RADON_ERR_INVALID, "radon_project_l1: n must be a multiple of 4, >= 0");
    if (!(tau >= 0) || !std::isfinite(tau))
        return rn::api_fail(RADON_ERR_INVALID, "radon_project_l1: tau must be finite and >= 0");
    if (n > ((int64_t)1 << 29)) return rn::api_fail(RADON_ERR_UNSUPPORTED, "radon_project_l1: n exceeds 2^29");
    if (n > 0 && (!v_dev || !out_dev)) return rn::api_fail(RADON_ERR_INVALID, "radon_project_l1: NULL buffer");
    if (((uintptr_t)v_dev | (uintptr_t)out_dev) % 16)
        return rn::api_fail(RADON_ERR_INVALID, "radon_project_l1: buffers must be 16-byte aligned");
    if (lam_host) *lam_host = 0.0;
    if (n == 0) return rn::api_ok();
    SolveWork w;
    if (!w.alloc(&w.part, (size_t)FIN_COUNT * rn::SV_BLOCKS) || !w.alloc(&w.ct, 2) ||
        !w.alloc(&w.pjc, SolveWork::PJ_ALL) || !w.alloc(&w.pjs, SolveWork::PJ_ALL) || !w.alloc(&w.pjbad, 1) ||
        !w.alloc(&w.pjst, 2) || !w.alloc_host(&w.fin_h, FIN_COUNT))
        return rn::api_fail(RADON_ERR_OOM, "radon_project_l1: workspace allocation failed");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(w.part, 0, sizeof(double) * FIN_COUNT * rn::SV_BLOCKS, st);
    if (e == hipSuccess) e = hipMemsetAsync(w.pjc, 0, sizeof(unsigned) * SolveWork::PJ_ALL, st);
    if (e == hipSuccess) e = hipMemsetAsync(w.pjs, 0, sizeof(unsigned long long) * SolveWork::PJ_ALL, st);
    if (e == hipSuccess) e = hipMemsetAsync(w.pjbad, 0, sizeof(unsigned), st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return rn::api_fail(RADON_ERR_DEVICE, "radon_project_l1: clearing the workspace failed");
    }
    // the solver's projection of x + c h with x = h = v, c = 0 (v + 0 v = v for finite v)
    const size_t nn = (size_t)n;
    const rn::PjWork pw = w.pj();
    hipLaunchKernelGGL(rn::k_sv_pj_pass<1>, dim3(rn::PJ_BLOCKS), dim3(rn::PJ_NT), 0, st, v_dev, v_dev, 0.0, tau, w.ct,
                       nn, pw);
    hipLaunchKernelGGL(rn::k_sv_pj_pass<2>, dim3(rn::PJ_BLOCKS), dim3(rn::PJ_NT), 0, st, v_dev, v_dev, 0.0, 0.0, w.ct,
                       nn, pw);
    hipLaunchKernelGGL(rn::k_sv_pj_pass<3>, dim3(rn::PJ_BLOCKS), dim3(rn::PJ_NT), 0, st, v_dev, v_dev, 0.0, 0.0, w.ct,
                       nn, pw);
    hipLaunchKernelGGL(rn::k_sv_soft, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, v_dev, v_dev, w.ct, nn, pw,
                       out_dev, w.part + (size_t)FIN_PROJ * rn::SV_BLOCKS);
    hipLaunchKernelGGL(rn::k_sv_final, dim3(1), dim3(rn::SV_NT), 0, st, w.part, FIN_COUNT, FIN_MAX_OPS, w.fin_h);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return rn::api_fail(RADON_ERR_DEVICE, "radon_project_l1: launch failed");
    }
    if (lam_host) *lam_host = w.fin_h[FIN_PROJ + 2];
    return rn::api_ok();
}

// ------------------------------------------------------------------ ring filter without allocation
//
// radon_ring_filter_noalloc: the ring filter for callers that cannot allocate
// device memory (code under stream capture, serving loops, harnesses that
// forbid it). The cubic basis is the plan's (uploaded when the plan is made);
// the scratch the three kernels need (column means, fitted ring, the
// per-block partials the residual kernel writes) lives in one file-scope
// device array, of which every GPU holds its own copy until the process ends.
// Every kernel overwrites the part of the array it reads back, so nothing
// needs clearing between calls; calls that overlap on one GPU share the array
// and race.

namespace {

constexpr int RING_NOALLOC_MAX_DET = RADON_RING_NOALLOC_MAX_DET;
// doubles: m[N], ring[N], partials[SV_SLOTS * SV_BLOCKS]
constexpr size_t RING_SCRATCH_DOUBLES = (size_t)2 * RING_NOALLOC_MAX_DET + (size_t)rn::SV_SLOTS * rn::SV_BLOCKS;

}  // namespace

static __device__ __align__(256) double scratch[RING_SCRATCH_DOUBLES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` on each GPU

// The device address of this GPU's copy of `scratch`, looked up on the first
// call on the device (which is then current); nullptr on failure.
double* scratch_for_device(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" radon_status_t radon_ring_filter_noalloc(radon_plan_t plan, const float* y_dev, float* out_dev,
                                                    void* stream) {
    if (!plan || !y_dev || !out_dev)
        return rn::api_fail(RADON_ERR_INVALID, "radon_ring_filter_noalloc: NULL argument");
    radon_status_t s = rn::api_check_plan(plan);   // the plan's device must be current
    if (s != RADON_OK) return s;
    const rn::Plan& p = plan->p;
    if (p.n_det > RING_NOALLOC_MAX_DET)
        return rn::api_fail(RADON_ERR_UNSUPPORTED,
                            "radon_ring_filter_noalloc: n_det exceeds RADON_RING_NOALLOC_MAX_DET");
    double* base = scratch_for_device(p.device);
    if (!base)
        return rn::api_fail(RADON_ERR_DEVICE, "radon_ring_filter_noalloc: no device address for the scratch array");
    double* m = base;
    double* ring = m + RING_NOALLOC_MAX_DET;
    double* part = ring + RING_NOALLOC_MAX_DET;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(rn::k_sv_colmean, dim3((p.n_det + 31) / 32), dim3(256), 0, st, y_dev, nullptr, p.n_views,
                       p.n_det, m);
    hipLaunchKernelGGL(rn::k_sv_ringfit, dim3(1), dim3(rn::SV_NT), 0, st, m, p.ringQ, p.n_det, ring);
    hipLaunchKernelGGL(rn::k_sv_resid, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, y_dev, nullptr, ring, nullptr,
                       p.n_views, p.n_det, out_dev, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rn::api_fail(RADON_ERR_DEVICE, "radon_ring_filter_noalloc: launch failed");
    return rn::api_ok();
}

namespace {

// Outcome of one SPGL1 run from the start held in w.x.
struct RunOut {
    int status = 0;       // 0 iteration limit, 1 basis pursuit, 2 root
    int it = 0;           // iterations taken
    double f = 0, tau = 0;
    int fallback = 0;     // why a warm run was abandoned (RADON_FALLBACK_*), 0 if it was not
};

// One SPGL1 run. `warm`: w.x holds the start image, else the run starts from
// zero. A warm run is abandoned, and reports why in out.fallback, when its
// start is non-finite, when it fits the data no better than x = 0, when
// | ||r|| - sigma | has not reached a new least value for `stall_iters`
// iterations, or when it reaches the iteration limit; the caller then runs
// cold. Above the Pareto root (tau > tau*) a point with ||r|| = sigma need not
// have the least l1 norm, so a warm run does not start at tau = ||x0||_1 but
// at the lower bound on tau* that x0's residual gives by weak duality: from
// there it approaches the root from below, as a cold run does, under the same
// tests.
radon_status_t spgl1_run(Solver& S, SolveWork& w, const radon_solve_opts* opts, bool warm, double bnorm,
                         RunOut& out) {
    const double sigma = opts->sigma, opt_tol = opts->opt_tol, bp_tol = opts->bp_tol, dec_tol = opts->dec_tol;
    const double bb_min = 1e-16, bb_max = 1e5;   // spectral step bounds
    const int n_mem = 3;
    const int stall_iters = opts->fallback_iters > 0 ? opts->fallback_iters : 100;
    hipStream_t st = S.st;
    double fin[FIN_COUNT];
    out = RunOut{};
    S.reset_projection();
    double f = 0, rbt = 0, gnorm = 0;
    // x = P_tau(x), then r = F(b - A x), h = A^T r and their sums
    auto shrink_to = [&](double t) -> bool {
        if (!S.project_sync(w.x, w.x, 0.0, t, w.xn, fin)) return false;
        std::swap(w.x, w.xn);
        if (!S.forward(w.x, w.z)) return false;
        S.residual(w.z, w.r, w.bt);
        if (!S.adjoint(w.r, w.h)) return false;
        S.bb(nullptr, w.x, nullptr, w.h);
        if (!S.read(fin)) return false;
        f = 0.5 * fin[FIN_RES];
        rbt = fin[FIN_RES + 1];
        gnorm = fin[FIN_BB + 2];
        return true;
    };
    // start point, tau = ||x0||_1, and the projection of x0 (a no-op at that radius)
    if (!warm) hipLaunchKernelGGL(rn::k_sv_fill, dim3(1024), dim3(256), 0, st, w.x, S.n2, 0.0f);
    S.bb(nullptr, w.x, nullptr, w.x);
    if (!S.read(fin)) return RADON_ERR_DEVICE;
    double tau = fin[FIN_BB + 3];
    if (warm && !std::isfinite(tau)) { out.fallback = RADON_FALLBACK_NONFINITE; return RADON_OK; }
    if (!shrink_to(tau)) return RADON_ERR_DEVICE;
    if (warm) {
        if (!std::isfinite(f) || !std::isfinite(gnorm)) { out.fallback = RADON_FALLBACK_NONFINITE; return RADON_OK; }
        if (sqrt(2 * f) >= bnorm) { out.fallback = RADON_FALLBACK_WORSE_THAN_ZERO; return RADON_OK; }
        // start below the root: y = r / ||A^T r||_inf is dual feasible, so weak
        // duality bounds the optimal l1 norm from below by
        // D = (r.b~ - sigma ||r||) / ||A^T r||_inf; the run starts at
        // tau0 = D clamped to [0, ||x0||_1], with x0 projected onto that ball
        const double D = gnorm > 0 ? (rbt - sigma * sqrt(2 * f)) / gnorm : 0.0;
        const double tau0 = std::min(std::max(D, 0.0), tau);
        if (tau0 < tau) {
            tau = tau0;
            if (!shrink_to(tau)) return RADON_ERR_DEVICE;
        }
    }
    std::vector<double> fs(n_mem, f);
    double alpha = std::min(std::max(gnorm > 0 ? 1.0 / gnorm : 1.0, bb_min), bb_max);
    double f_old = INFINITY, d_best = INFINITY;   // least | ||r|| - sigma | so far
    int it_best = 0;
    int status = 0, it = 0;
    for (it = 1; it <= opts->max_iter; ++it) {
        const double rnorm = sqrt(2 * f);
        const double gap = (2 * f - rbt) + tau * gnorm;   // r.(r - b~) + tau ||g||_inf
        const double rgap = fabs(gap) / std::max(1.0, f);
        const double aerr1 = rnorm - sigma;
        const double rerr1 = fabs(aerr1) / std::max(1.0, rnorm);
        const double rerr2 = fabs(f - 0.5 * sigma * sigma) / std::max(1.0, f);
        if (rgap <= std::max(opt_tol, rerr2) || rerr1 <= opt_tol) {
            if (rnorm <= bp_tol * bnorm) { status = 1; break; }
            if (rerr1 <= opt_tol) { status = 2; break; }
        }
        if (warm) {
            // progress of the root finding from either side: a start above the
            // root lets ||r|| grow to sigma, one below lets it shrink
            if (fabs(aerr1) < d_best) { d_best = fabs(aerr1); it_best = it; }
            else if (it - it_best >= stall_iters) { out.fallback = RADON_FALLBACK_STALLED; break; }
        }
        const double change = fabs(f - f_old);
        const bool stalled = (change <= dec_tol * f && rnorm > 2 * sigma) ||
                             (change <= 0.1 * f * fabs(rnorm - sigma) && rnorm <= 2 * sigma);
        if (stalled && gnorm > 0) {
            const double tau_old = tau;
            tau = std::max(0.0, tau + rnorm * aerr1 / gnorm);   // Newton step on the Pareto curve
            if (tau < tau_old) {
                // the ball shrank: restart from the projected iterate with its
                // own residual and gradient
                if (!shrink_to(tau)) return RADON_ERR_DEVICE;
            }
            std::fill(fs.begin(), fs.end(), f);
        }
        // spectral projected gradient step, non-monotone (GLL) backtracking; the
        // gradient and spectral sums of each trial point are computed before the
        // host reads the trial's objective, so an accepted step costs one wait
        const double fmax = *std::max_element(fs.begin(), fs.end());
        double step = 1.0, fn = 0, rbtn = 0;
        while (true) {
            if (!S.trial(step * alpha, tau, fin)) return RADON_ERR_DEVICE;
            const double gtd = fin[FIN_PROJ];
            fn = 0.5 * fin[FIN_RES];
            rbtn = fin[FIN_RES + 1];
            if (fn <= fmax + 1e-4 * gtd || step < 1e-10 || !std::isfinite(fn)) break;
            step *= 0.5;
        }
        if (!std::isfinite(fn)) {
            if (warm) { out.fallback = RADON_FALLBACK_NONFINITE; break; }
            return rn::api_fail(RADON_ERR_INVALID, "radon_solve_bpdn: the objective became non-finite");
        }
        const double sts = fin[FIN_BB], sty = fin[FIN_BB + 1];
        alpha = sty <= 0 ? bb_max : std::min(std::max(sts / sty, bb_min), bb_max);
        f_old = f;
        std::swap(w.x, w.xn);
        std::swap(w.r, w.rn);
        std::swap(w.h, w.hn);
        f = fn;
        rbt = rbtn;
        gnorm = fin[FIN_BB + 2];
        fs.erase(fs.begin());
        fs.push_back(f);
    }
    if (it > opts->max_iter) it = opts->max_iter;
    if (warm && !out.fallback && status == 0) out.fallback = RADON_FALLBACK_ITER_LIMIT;
    out.status = status;
    out.it = it;
    out.f = f;
    out.tau = tau;
    return RADON_OK;
}

}  // namespace

extern "C" radon_status_t radon_solve_bpdn(radon_plan_t plan, const float* b_dev, float* x_dev,
                                           const radon_solve_opts* opts, radon_solve_stats* stats, void* stream) {
    if (!plan || !b_dev || !x_dev || !opts) return RADON_ERR_INVALID;
    if (!(opts->sigma >= 0) || !std::isfinite(opts->sigma) || !(opts->opt_tol > 0) || opts->max_iter < 1)
        return RADON_ERR_INVALID;
    const auto t0 = std::chrono::steady_clock::now();
    const rn::Plan& p = plan->p;
    SolveWork w;
    const size_t n2 = (size_t)p.n * p.n, ns = (size_t)p.n_views * p.n_det;
    if (!w.alloc(&w.x, n2) || !w.alloc(&w.xn, n2) || !w.alloc(&w.h, n2) || !w.alloc(&w.hn, n2) ||
        !w.alloc(&w.z, ns) || !w.alloc(&w.r, ns) || !w.alloc(&w.rn, ns) || !w.alloc(&w.bt, ns) ||
        !w.alloc(&w.m, p.n_det) || !w.alloc(&w.ring, p.n_det) || !w.alloc(&w.Q, (size_t)p.n_det * 4) ||
        !w.alloc(&w.part, (size_t)FIN_COUNT * rn::SV_BLOCKS) || !w.alloc(&w.ct, 2) ||
        !w.alloc(&w.pjc, SolveWork::PJ_ALL) || !w.alloc(&w.pjs, SolveWork::PJ_ALL) || !w.alloc(&w.pjbad, 1) ||
        !w.alloc(&w.pjst, 2) || !w.alloc_host(&w.fin_h, FIN_COUNT))
        return RADON_ERR_OOM;
    hipStream_t st = (hipStream_t)stream;
    Solver S{plan, p, w, st, opts->ring_filter != 0, b_dev, n2, ns};
    const std::vector<double> Q = cubic_basis(p.n_det);
    S.chk(hipMemcpyAsync(w.Q, Q.data(), sizeof(double) * Q.size(), hipMemcpyHostToDevice, st));
    // every read folds all partial slots, also those no kernel has written yet
    S.chk(hipMemsetAsync(w.part, 0, sizeof(double) * FIN_COUNT * rn::SV_BLOCKS, st));

    double fin[FIN_COUNT];
    // b~ = F b and its norm
    S.residual(nullptr, w.bt, nullptr);
    if (!S.read(fin)) return RADON_ERR_DEVICE;
    const double bnorm = sqrt(fin[FIN_RES]);
    if (!std::isfinite(bnorm)) return rn::api_fail(RADON_ERR_INVALID, "radon_solve_bpdn: the sinogram is not finite");

    RunOut run;
    int fallback = 0, warm_it = 0;
    radon_status_t rc;
    if (opts->warm_start) {
        S.chk(hipMemcpyAsync(w.x, x_dev, sizeof(float) * n2, hipMemcpyDeviceToDevice, st));
        rc = spgl1_run(S, w, opts, true, bnorm, run);
        if (rc != RADON_OK) return rc;
        if (run.fallback) {
            // the cold-started solver takes over, with the whole iteration budget
            fallback = run.fallback;
            warm_it = run.it;
            rc = spgl1_run(S, w, opts, false, bnorm, run);
            if (rc != RADON_OK) return rc;
        }
    } else {
        rc = spgl1_run(S, w, opts, false, bnorm, run);
        if (rc != RADON_OK) return rc;
    }
    // ||x||_1 of the result, then hand it back
    S.bb(nullptr, w.x, nullptr, w.x);
    S.chk(hipMemcpyAsync(x_dev, w.x, sizeof(float) * n2, hipMemcpyDeviceToDevice, st));
    if (!S.read(fin)) return RADON_ERR_DEVICE;
    if (stats) {
        stats->rnorm = sqrt(2 * run.f);
        stats->tau = run.tau;
        stats->x_l1 = fin[FIN_BB + 3];
        stats->iterations = run.it;
        stats->n_forward = S.nf;
        stats->n_adjoint = S.na;
        stats->status = run.status;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->fallback = fallback;
        stats->warm_iterations = warm_it;
    }
    return rn::api_ok();
}

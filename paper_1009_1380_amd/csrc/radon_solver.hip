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
#include <vector>

#include "../../include/radon.h"
#include "radon_internal.hpp"

namespace rn {

constexpr int SV_NT = 256;           // threads per reduction block
constexpr int SV_BLOCKS = 512;       // blocks of the grid-stride reductions
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

// Sum (or max) of the per-block partials of each slot, in block order.
// ops bit k set: slot k is a max, else a sum.
__global__ __launch_bounds__(SV_NT) void k_sv_final(const double* __restrict__ part, int nb, int nslots,
                                                   unsigned ops, double* __restrict__ out) {
    __shared__ double sh[SV_NT / 64];
    for (int s = 0; s < nslots; ++s) {
        const bool mx = (ops >> s) & 1u;
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += SV_NT) {
            const double p = part[(size_t)s * nb + b];
            v = mx ? fmax(v, p) : v + p;
        }
        const double r = mx ? block_reduce<true>(v, sh) : block_reduce<false>(v, sh);
        if (threadIdx.x == 0) out[s] = r;
        __syncthreads();
    }
}

// m[d] = mean over views of (b - z)[., d] (z may be null: m = mean of b).
__global__ __launch_bounds__(256) void k_sv_colmean(const float* __restrict__ b, const float* __restrict__ z,
                                                   int nv, int N, double* __restrict__ m) {
    const int d = blockIdx.x * 256 + threadIdx.x;
    if (d >= N) return;
    double s = 0.0;
    for (int a = 0; a < nv; ++a) {
        const size_t i = (size_t)a * N + d;
        s += (double)b[i] - (z ? (double)z[i] : 0.0);
    }
    m[d] = s / nv;
}

// ring[d] = m[d] - (Q Q^T m)[d]  (one block).
__global__ __launch_bounds__(SV_NT) void k_sv_ringfit(const double* __restrict__ m, const double* __restrict__ Q,
                                                     int N, double* __restrict__ ring) {
    __shared__ double sh[SV_NT / 64];
    __shared__ double c[4];
    for (int k = 0; k < 4; ++k) {
        double v = 0.0;
        for (int d = threadIdx.x; d < N; d += SV_NT) v += Q[(size_t)d * 4 + k] * m[d];
        const double r = block_reduce<false>(v, sh);
        if (threadIdx.x == 0) c[k] = r;
        __syncthreads();
    }
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

// partials for the l1 projection of v = x + c h at threshold lam (device):
// slot 0: sum max(|v| - lam, 0), slot 1: count(|v| > lam).
__global__ __launch_bounds__(SV_NT) void k_sv_l1_partial(const float* __restrict__ x, const float* __restrict__ h,
                                                        double c, const double* __restrict__ lam, size_t n,
                                                        double* __restrict__ part) {
    __shared__ double sh[SV_NT / 64];
    const double L = *lam;
    double s = 0.0, k = 0.0;
    for (size_t i = (size_t)blockIdx.x * SV_NT + threadIdx.x; i < n; i += (size_t)gridDim.x * SV_NT) {
        const float v = (float)((double)x[i] + c * (double)h[i]);
        const double a = fabs((double)v);
        if (a > L) { s += a - L; k += 1.0; }
    }
    double t = block_reduce<false>(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_reduce<false>(k, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = t;
}

// One Newton step on the threshold: with S = sum max(|v| - lam, 0) and K the
// count above lam (from fin[0], fin[1]), lam += (S - tau)/K while S > tau.
__global__ void k_sv_l1_newton(const double* __restrict__ fin, double tau, double* __restrict__ lam) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double S = fin[0], K = fin[1];
        if (S > tau && K > 0) *lam = *lam + (S - tau) / K;
    }
}

// xn = soft(x + c h, lam); partials: slot 0 sum (-h) (xn - x) (= g . dx),
// slot 1 sum |xn|.
__global__ __launch_bounds__(SV_NT) void k_sv_soft(const float* __restrict__ x, const float* __restrict__ h,
                                                  double c, const double* __restrict__ lam, size_t n,
                                                  float* __restrict__ xn, double* __restrict__ part) {
    __shared__ double sh[SV_NT / 64];
    const double L = *lam;
    double s0 = 0.0, s1 = 0.0;
    for (size_t i = (size_t)blockIdx.x * SV_NT + threadIdx.x; i < n; i += (size_t)gridDim.x * SV_NT) {
        const float v = (float)((double)x[i] + c * (double)h[i]);
        const double a = fabs((double)v) - L;
        const float o = a > 0 ? (float)copysign(a, (double)v) : 0.0f;
        xn[i] = o;
        s0 += -(double)h[i] * ((double)o - (double)x[i]);
        s1 += fabs((double)o);
    }
    double t = block_reduce<false>(s0, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_reduce<false>(s1, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = t;
}

// Barzilai-Borwein quantities with s = xn - x and y = gn - g = -(hn - h):
// slot 0 sum s^2, slot 1 sum s y, slot 2 max |hn| (= ||gn||_inf),
// slot 3 sum |x| of the input x (used for tau at a warm start).
__global__ __launch_bounds__(SV_NT) void k_sv_bb(const float* __restrict__ x, const float* __restrict__ xn,
                                                const float* __restrict__ h, const float* __restrict__ hn, size_t n,
                                                double* __restrict__ part) {
    __shared__ double sh[SV_NT / 64];
    double ss = 0.0, sy = 0.0, mx = 0.0, l1 = 0.0;
    for (size_t i = (size_t)blockIdx.x * SV_NT + threadIdx.x; i < n; i += (size_t)gridDim.x * SV_NT) {
        const double s = (x ? (double)xn[i] - (double)x[i] : 0.0);
        const double y = (h ? -((double)hn[i] - (double)h[i]) : 0.0);
        ss += s * s;
        sy += s * y;
        mx = fmax(mx, fabs((double)hn[i]));
        l1 += fabs((double)xn[i]);
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

__global__ __launch_bounds__(256) void k_sv_fill(float* __restrict__ v, size_t n, float val) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) v[i] = val;
}

__global__ void k_sv_set(double* __restrict__ p, double val) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = val;
}

}  // namespace rn

// ------------------------------------------------------------------ host side

namespace {

struct SolveWork {
    std::vector<void*> allocs;
    float *x = nullptr, *xn = nullptr, *h = nullptr, *hn = nullptr;
    float *z = nullptr, *r = nullptr, *rn = nullptr, *bt = nullptr;
    double *m = nullptr, *ring = nullptr, *Q = nullptr, *part = nullptr, *fin = nullptr, *lam = nullptr;
    ~SolveWork() {
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
};

// Orthonormal basis of cubic polynomials in s = d - N/2, scaled to [-1, 1),
// by modified Gram-Schmidt (twice) in float64; row-major N x 4.
std::vector<double> cubic_basis(int N) {
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

    // reduce SV_BLOCKS partials of `slots` slots into fin[0..slots) and read them
    bool finals(int slots, unsigned ops, double* out) {
        hipLaunchKernelGGL(rn::k_sv_final, dim3(1), dim3(rn::SV_NT), 0, st, w.part, rn::SV_BLOCKS, slots, ops, w.fin);
        chk(hipGetLastError());
        chk(hipMemcpyAsync(out, w.fin, sizeof(double) * slots, hipMemcpyDeviceToHost, st));
        chk(hipStreamSynchronize(st));
        return err == hipSuccess;
    }

    // r = F(b - z) (z may be null), returns sum r^2 and sum r.bt (bt may be null)
    bool residual(const float* z, float* r, const float* bt, double* sums) {
        const double* ring = nullptr;
        if (filt) {
            hipLaunchKernelGGL(rn::k_sv_colmean, dim3((p.n_det + 255) / 256), dim3(256), 0, st, b, z, p.n_views,
                               p.n_det, w.m);
            hipLaunchKernelGGL(rn::k_sv_ringfit, dim3(1), dim3(rn::SV_NT), 0, st, w.m, w.Q, p.n_det, w.ring);
            ring = w.ring;
        }
        hipLaunchKernelGGL(rn::k_sv_resid, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, b, z, ring, bt, p.n_views,
                           p.n_det, r, w.part);
        chk(hipGetLastError());
        return finals(2, 0u, sums);
    }

    // xn = P_tau(x + c h), returns sum g.(xn - x) and ||xn||_1
    bool project(const float* x, const float* h, double c, double tau, float* xn, double* sums) {
        hipLaunchKernelGGL(rn::k_sv_set, dim3(1), dim3(64), 0, st, w.lam, 0.0);
        double fin[2] = {0, 0};
        for (int round = 0; round < 16; ++round) {
            for (int k = 0; k < 8; ++k) {
                hipLaunchKernelGGL(rn::k_sv_l1_partial, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, x, h, c, w.lam,
                                   n2, w.part);
                hipLaunchKernelGGL(rn::k_sv_final, dim3(1), dim3(rn::SV_NT), 0, st, w.part, rn::SV_BLOCKS, 2, 0u,
                                   w.fin);
                hipLaunchKernelGGL(rn::k_sv_l1_newton, dim3(1), dim3(64), 0, st, w.fin, tau, w.lam);
            }
            // converged when the threshold no longer moves: S <= tau (within rounding)
            hipLaunchKernelGGL(rn::k_sv_l1_partial, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, x, h, c, w.lam, n2,
                               w.part);
            if (!finals(2, 0u, fin)) return false;
            if (fin[0] <= tau * (1.0 + 1e-12) + 1e-300) break;
        }
        hipLaunchKernelGGL(rn::k_sv_soft, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, x, h, c, w.lam, n2, xn, w.part);
        chk(hipGetLastError());
        return finals(2, 0u, sums);
    }

    bool forward(const float* x, float* z) {
        ++nf;
        return radon_forward(plan, x, z, st) == RADON_OK;
    }
    bool adjoint(const float* r, float* h) {
        ++na;
        return radon_adjoint(plan, r, h, st) == RADON_OK;
    }
};

}  // namespace

extern "C" radon_status_t radon_ring_filter(radon_plan_t plan, const float* y_dev, float* out_dev, void* stream) {
    if (!plan || !y_dev || !out_dev) return RADON_ERR_INVALID;
    const rn::Plan& p = plan->p;
    SolveWork w;
    if (!w.alloc(&w.m, p.n_det) || !w.alloc(&w.ring, p.n_det) || !w.alloc(&w.Q, (size_t)p.n_det * 4) ||
        !w.alloc(&w.part, (size_t)rn::SV_SLOTS * rn::SV_BLOCKS) || !w.alloc(&w.fin, rn::SV_SLOTS))
        return RADON_ERR_OOM;
    hipStream_t st = (hipStream_t)stream;
    const std::vector<double> Q = cubic_basis(p.n_det);
    if (hipMemcpy(w.Q, Q.data(), sizeof(double) * Q.size(), hipMemcpyHostToDevice) != hipSuccess)
        return RADON_ERR_DEVICE;
    hipLaunchKernelGGL(rn::k_sv_colmean, dim3((p.n_det + 255) / 256), dim3(256), 0, st, y_dev, nullptr, p.n_views,
                       p.n_det, w.m);
    hipLaunchKernelGGL(rn::k_sv_ringfit, dim3(1), dim3(rn::SV_NT), 0, st, w.m, w.Q, p.n_det, w.ring);
    hipLaunchKernelGGL(rn::k_sv_resid, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, y_dev, nullptr, w.ring, nullptr,
                       p.n_views, p.n_det, out_dev, w.part);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return RADON_ERR_DEVICE;
    return RADON_OK;
}

extern "C" radon_status_t radon_solve_bpdn(radon_plan_t plan, const float* b_dev, float* x_dev,
                                           const radon_solve_opts* opts, radon_solve_stats* stats, void* stream) {
    if (!plan || !b_dev || !x_dev || !opts) return RADON_ERR_INVALID;
    if (!(opts->sigma >= 0) || !(opts->opt_tol > 0) || opts->max_iter < 1) return RADON_ERR_INVALID;
    const auto t0 = std::chrono::steady_clock::now();
    const rn::Plan& p = plan->p;
    SolveWork w;
    const size_t n2 = (size_t)p.n * p.n, ns = (size_t)p.n_views * p.n_det;
    if (!w.alloc(&w.x, n2) || !w.alloc(&w.xn, n2) || !w.alloc(&w.h, n2) || !w.alloc(&w.hn, n2) ||
        !w.alloc(&w.z, ns) || !w.alloc(&w.r, ns) || !w.alloc(&w.rn, ns) || !w.alloc(&w.bt, ns) ||
        !w.alloc(&w.m, p.n_det) || !w.alloc(&w.ring, p.n_det) || !w.alloc(&w.Q, (size_t)p.n_det * 4) ||
        !w.alloc(&w.part, (size_t)rn::SV_SLOTS * rn::SV_BLOCKS) || !w.alloc(&w.fin, rn::SV_SLOTS) ||
        !w.alloc(&w.lam, 1))
        return RADON_ERR_OOM;
    hipStream_t st = (hipStream_t)stream;
    Solver S{plan, p, w, st, opts->ring_filter != 0, b_dev, n2, ns};
    const std::vector<double> Q = cubic_basis(p.n_det);
    S.chk(hipMemcpyAsync(w.Q, Q.data(), sizeof(double) * Q.size(), hipMemcpyHostToDevice, st));

    const double sigma = opts->sigma, opt_tol = opts->opt_tol, bp_tol = opts->bp_tol, dec_tol = opts->dec_tol;
    const double bb_min = 1e-16, bb_max = 1e5;   // spectral step bounds
    const int n_mem = 3;
    double sums[4];
    // b~ = F b and its norm
    if (!S.residual(nullptr, w.bt, nullptr, sums)) return RADON_ERR_DEVICE;
    const double bnorm = sqrt(sums[0]);
    // start point and tau
    if (opts->warm_start) S.chk(hipMemcpyAsync(w.x, x_dev, sizeof(float) * n2, hipMemcpyDeviceToDevice, st));
    else hipLaunchKernelGGL(rn::k_sv_fill, dim3(1024), dim3(256), 0, st, w.x, n2, 0.0f);
    hipLaunchKernelGGL(rn::k_sv_bb, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, nullptr, w.x, nullptr, w.x, n2,
                       w.part);
    double q4[4];
    if (!S.finals(4, 1u << 2, q4)) return RADON_ERR_DEVICE;
    double tau = q4[3];
    if (!S.project(w.x, w.x, 0.0, tau, w.xn, sums)) return RADON_ERR_DEVICE;
    std::swap(w.x, w.xn);
    // r = F(b - A x), h = A^T r
    if (!S.forward(w.x, w.z) || !S.residual(w.z, w.r, w.bt, sums)) return RADON_ERR_DEVICE;
    double f = 0.5 * sums[0], rbt = sums[1];
    if (!S.adjoint(w.r, w.h)) return RADON_ERR_DEVICE;
    hipLaunchKernelGGL(rn::k_sv_bb, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, nullptr, w.x, nullptr, w.h, n2,
                       w.part);
    if (!S.finals(4, 1u << 2, q4)) return RADON_ERR_DEVICE;
    double gnorm = q4[2];
    std::vector<double> fs(n_mem, f);
    double alpha = std::min(std::max(gnorm > 0 ? 1.0 / gnorm : 1.0, bb_min), bb_max);
    double f_old = INFINITY;
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
        const double change = fabs(f - f_old);
        const bool stalled = (change <= dec_tol * f && rnorm > 2 * sigma) ||
                             (change <= 0.1 * f * fabs(rnorm - sigma) && rnorm <= 2 * sigma);
        if (stalled && gnorm > 0) {
            const double tau_old = tau;
            tau = std::max(0.0, tau + rnorm * aerr1 / gnorm);   // Newton step on the Pareto curve
            if (tau < tau_old) {
                // the ball shrank: restart from the projected iterate with its
                // own residual and gradient
                if (!S.project(w.x, w.x, 0.0, tau, w.xn, sums)) return RADON_ERR_DEVICE;
                std::swap(w.x, w.xn);
                if (!S.forward(w.x, w.z) || !S.residual(w.z, w.r, w.bt, sums)) return RADON_ERR_DEVICE;
                f = 0.5 * sums[0];
                rbt = sums[1];
                if (!S.adjoint(w.r, w.h)) return RADON_ERR_DEVICE;
                hipLaunchKernelGGL(rn::k_sv_bb, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, nullptr, w.x, nullptr,
                                   w.h, n2, w.part);
                if (!S.finals(4, 1u << 2, q4)) return RADON_ERR_DEVICE;
                gnorm = q4[2];
            }
            std::fill(fs.begin(), fs.end(), f);
        }
        // spectral projected gradient step, non-monotone (GLL) backtracking
        const double fmax = *std::max_element(fs.begin(), fs.end());
        double step = 1.0, fn = 0, rbtn = 0;
        while (true) {
            if (!S.project(w.x, w.h, step * alpha, tau, w.xn, sums)) return RADON_ERR_DEVICE;
            const double gtd = sums[0];
            if (!S.forward(w.xn, w.z) || !S.residual(w.z, w.rn, w.bt, sums)) return RADON_ERR_DEVICE;
            fn = 0.5 * sums[0];
            rbtn = sums[1];
            if (fn <= fmax + 1e-4 * gtd || step < 1e-10) break;
            step *= 0.5;
        }
        if (!S.adjoint(w.rn, w.hn)) return RADON_ERR_DEVICE;
        hipLaunchKernelGGL(rn::k_sv_bb, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, w.x, w.xn, w.h, w.hn, n2,
                           w.part);
        if (!S.finals(4, 1u << 2, q4)) return RADON_ERR_DEVICE;
        const double sts = q4[0], sty = q4[1];
        alpha = sty <= 0 ? bb_max : std::min(std::max(sts / sty, bb_min), bb_max);
        f_old = f;
        std::swap(w.x, w.xn);
        std::swap(w.r, w.rn);
        std::swap(w.h, w.hn);
        f = fn;
        rbt = rbtn;
        gnorm = q4[2];
        fs.erase(fs.begin());
        fs.push_back(f);
    }
    if (it > opts->max_iter) it = opts->max_iter;
    // ||x||_1 of the result, then hand it back
    hipLaunchKernelGGL(rn::k_sv_bb, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, nullptr, w.x, nullptr, w.x, n2,
                       w.part);
    if (!S.finals(4, 1u << 2, q4)) return RADON_ERR_DEVICE;
    S.chk(hipMemcpyAsync(x_dev, w.x, sizeof(float) * n2, hipMemcpyDeviceToDevice, st));
    S.chk(hipStreamSynchronize(st));
    if (S.err != hipSuccess) return RADON_ERR_DEVICE;
    if (stats) {
        stats->rnorm = sqrt(2 * f);
        stats->tau = tau;
        stats->x_l1 = q4[3];
        stats->iterations = it;
        stats->n_forward = S.nf;
        stats->n_adjoint = S.na;
        stats->status = status;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return RADON_OK;
}

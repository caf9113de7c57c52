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

// Projection onto the l1 ball: xn = soft(v, lam), v = x + c h, with lam the
// root of S(lam) = sum max(|v| - lam, 0) = tau, found by Newton's method
// started at the previous projection's root (successive projections in a
// solve have nearby roots). S is convex, decreasing and piecewise linear:
// from below the root the iterates increase to the exact root of the final
// active set, and a step from above lands at or below the root (a convex
// function lies above its tangents), so at most one step is spent above.
// One launch per step: every block writes its partial sums, and the last
// block to finish (an atomic ticket after a memory fence) adds the partials
// in block order and takes the step, so the result is deterministic. Steps
// after convergence return at once. State: st[0] = lam, st[1] = done flag.
constexpr int PJ_NT = 256;
#ifndef RN_PJ_BLOCKS
#define RN_PJ_BLOCKS 256
#endif
constexpr int PJ_BLOCKS = RN_PJ_BLOCKS;
constexpr int PJ_STEPS = 12;   // launches per projection; the host checks the flag

__global__ __launch_bounds__(PJ_NT) void k_sv_pj_step(const float* __restrict__ x, const float* __restrict__ h,
                                                     double c, double tau, size_t n, double* __restrict__ st,
                                                     double* __restrict__ part, unsigned* __restrict__ ticket) {
    __shared__ double sh[PJ_NT / 64];
    __shared__ bool last;
    if (st[1] != 0.0) return;   // converged in an earlier launch (uniform)
    const double lam = st[0];
    double s = 0.0, k = 0.0;
    for (size_t i = (size_t)blockIdx.x * PJ_NT + threadIdx.x; i < n; i += (size_t)gridDim.x * PJ_NT) {
        const float v = (float)((double)x[i] + c * (double)h[i]);
        const double a = fabs((double)v);
        if (a > lam) { s += a - lam; k += 1.0; }
    }
    double t = block_reduce<false>(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_reduce<false>(k, sh);
    if (threadIdx.x == 0) {
        part[gridDim.x + blockIdx.x] = t;
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double vs = 0.0, vk = 0.0;
    for (int j = threadIdx.x; j < (int)gridDim.x; j += PJ_NT) {
        vs += part[j];
        vk += part[gridDim.x + j];
    }
    const double S = block_reduce<false>(vs, sh);
    const double K = block_reduce<false>(vk, sh);
    if (threadIdx.x == 0) {
        *ticket = 0u;
        if (fabs(S - tau) <= 1e-12 * tau || (lam == 0.0 && S <= tau)) st[1] = 1.0;
        else st[0] = K > 0.0 ? fmax(0.0, lam + (S - tau) / K) : 0.0;   // K = 0: above every |v|
    }
}

// xn = soft(x + c h, st[0]); partials: slot 0 sum -h.(xn - x), slot 1 sum |xn|,
// slot 2 the done flag (so the host sees whether the steps converged).
__global__ __launch_bounds__(SV_NT) void k_sv_soft(const float* __restrict__ x, const float* __restrict__ h,
                                                  double c, const double* __restrict__ st, size_t n,
                                                  float* __restrict__ xn, double* __restrict__ part) {
    __shared__ double sh[SV_NT / 64];
    const double L = st[0];
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
    if (threadIdx.x == 0) part[2 * gridDim.x + blockIdx.x] = blockIdx.x == 0 ? st[1] : 0.0;
}

// st[1] = 0 (a new projection; st[0] keeps the previous root as the start)
__global__ void k_sv_pj_reset(double* __restrict__ st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st[1] = 0.0;
}

__global__ void k_sv_zero(double* __restrict__ p, unsigned* __restrict__ ticket) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        p[0] = 0.0;
        p[1] = 0.0;
        *ticket = 0u;
    }
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
    std::vector<void*> allocs;
    float *x = nullptr, *xn = nullptr, *h = nullptr, *hn = nullptr;
    float *z = nullptr, *r = nullptr, *rn = nullptr, *bt = nullptr;
    double *m = nullptr, *ring = nullptr, *Q = nullptr, *part = nullptr, *fin = nullptr, *lam = nullptr;
    double* pj = nullptr;          // projection step partials, 2 x PJ_BLOCKS
    unsigned* ticket = nullptr;    // last-block ticket of the projection steps
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

std::vector<double> cubic_basis(int N) { return rn::ring_cubic_basis(N); }

// fin slots: 0-1 residual (sum r^2, sum r.b~), 2-4 projection (g.dx, ||xn||_1,
// converged flag), 5-8 spectral step (sum s^2, sum s.y, max |hn|, ||xn||_1)
constexpr int FIN_RES = 0, FIN_PROJ = 2, FIN_BB = 5, FIN_COUNT = 9;

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

    // fold SV_BLOCKS partials of `slots` slots into fin[off..off+slots) (no host wait)
    void fold(int slots, unsigned ops, int off) {
        hipLaunchKernelGGL(rn::k_sv_final, dim3(1), dim3(rn::SV_NT), 0, st, w.part, rn::SV_BLOCKS, slots, ops,
                           w.fin + off);
        chk(hipGetLastError());
    }
    // read all fin slots back (one host wait)
    bool read(double* out) {
        chk(hipMemcpyAsync(out, w.fin, sizeof(double) * FIN_COUNT, hipMemcpyDeviceToHost, st));
        chk(hipStreamSynchronize(st));
        return err == hipSuccess;
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
                           p.n_det, r, w.part);
        chk(hipGetLastError());
        fold(2, 0u, FIN_RES);
    }

    // xn = P_tau(x + c h) -> fin[2] = sum -h.(xn - x), fin[3] = ||xn||_1,
    // fin[4] = 1 if the Newton steps converged (else call again with fresh = false
    // to continue them)
    void project(const float* x, const float* h, double c, double tau, float* xn, bool fresh = true) {
        if (fresh) hipLaunchKernelGGL(rn::k_sv_pj_reset, dim3(1), dim3(64), 0, st, w.lam);
        for (int k = 0; k < rn::PJ_STEPS; ++k)
            hipLaunchKernelGGL(rn::k_sv_pj_step, dim3(rn::PJ_BLOCKS), dim3(rn::PJ_NT), 0, st, x, h, c, tau, n2, w.lam,
                               w.pj, w.ticket);
        hipLaunchKernelGGL(rn::k_sv_soft, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, x, h, c, w.lam, n2, xn,
                           w.part);
        chk(hipGetLastError());
        fold(3, 1u << 2, FIN_PROJ);
    }

    // spectral-step sums of s = xn - x, y = -(hn - h) -> fin[4..7] (x, h may be null)
    void bb(const float* x, const float* xn, const float* h, const float* hn) {
        hipLaunchKernelGGL(rn::k_sv_bb, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, x, xn, h, hn, n2, w.part);
        chk(hipGetLastError());
        fold(4, 1u << 2, FIN_BB);
    }

    // project and wait until the Newton steps have converged
    bool project_sync(const float* x, const float* h, double c, double tau, float* xn, double* fin) {
        bool fresh = true;
        for (int round = 0; round < 64; ++round) {
            project(x, h, c, tau, xn, fresh);
            fresh = false;
            if (!read(fin)) return false;
            if (fin[FIN_PROJ + 2] != 0.0) return true;
        }
        return true;   // the last step's threshold is used
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
    hipLaunchKernelGGL(rn::k_sv_colmean, dim3((p.n_det + 31) / 32), dim3(256), 0, st, y_dev, nullptr, p.n_views,
                       p.n_det, w.m);
    hipLaunchKernelGGL(rn::k_sv_ringfit, dim3(1), dim3(rn::SV_NT), 0, st, w.m, w.Q, p.n_det, w.ring);
    hipLaunchKernelGGL(rn::k_sv_resid, dim3(rn::SV_BLOCKS), dim3(rn::SV_NT), 0, st, y_dev, nullptr, w.ring, nullptr,
                       p.n_views, p.n_det, out_dev, w.part);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return RADON_ERR_DEVICE;
    return RADON_OK;
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

// One SPGL1 run. `warm`: w.x holds the start image (tau0 = its l1 norm), else
// the run starts from zero. A warm run is abandoned, and reports why in
// out.fallback, when its start is non-finite, when it fits the data no better
// than x = 0, when its residual norm stops decreasing for `stall_iters`
// iterations, or when it reaches the iteration limit; the caller then runs
// cold. A warm start may lie above the Pareto root (tau0 > tau*), where a
// point with ||r|| = sigma need not have the least l1 norm; such a run is
// not allowed to stop at the root before its first Newton update of tau,
// which (the Pareto curve being convex and decreasing) leaves tau at or
// below the root, as a cold run's tau always is.
radon_status_t spgl1_run(Solver& S, SolveWork& w, const radon_solve_opts* opts, bool warm, double bnorm,
                         RunOut& out) {
    const double sigma = opts->sigma, opt_tol = opts->opt_tol, bp_tol = opts->bp_tol, dec_tol = opts->dec_tol;
    const double bb_min = 1e-16, bb_max = 1e5;   // spectral step bounds
    const int n_mem = 3;
    const int stall_iters = opts->fallback_iters > 0 ? opts->fallback_iters : 100;
    hipStream_t st = S.st;
    double fin[FIN_COUNT];
    out = RunOut{};
    // projection state: threshold 0 (no warm start yet), ticket 0
    hipLaunchKernelGGL(rn::k_sv_zero, dim3(1), dim3(64), 0, st, w.lam, w.ticket);
    // start point, tau = ||x0||_1, and the projection of x0 (a no-op at that radius)
    if (!warm) hipLaunchKernelGGL(rn::k_sv_fill, dim3(1024), dim3(256), 0, st, w.x, S.n2, 0.0f);
    S.bb(nullptr, w.x, nullptr, w.x);
    if (!S.read(fin)) return RADON_ERR_DEVICE;
    double tau = fin[FIN_BB + 3];
    if (warm && !std::isfinite(tau)) { out.fallback = RADON_FALLBACK_NONFINITE; return RADON_OK; }
    if (!S.project_sync(w.x, w.x, 0.0, tau, w.xn, fin)) return RADON_ERR_DEVICE;
    std::swap(w.x, w.xn);
    // r = F(b - A x), h = A^T r
    if (!S.forward(w.x, w.z)) return RADON_ERR_DEVICE;
    S.residual(w.z, w.r, w.bt);
    if (!S.adjoint(w.r, w.h)) return RADON_ERR_DEVICE;
    S.bb(nullptr, w.x, nullptr, w.h);
    if (!S.read(fin)) return RADON_ERR_DEVICE;
    double f = 0.5 * fin[FIN_RES], rbt = fin[FIN_RES + 1];
    double gnorm = fin[FIN_BB + 2];
    if (warm) {
        if (!std::isfinite(f) || !std::isfinite(gnorm)) { out.fallback = RADON_FALLBACK_NONFINITE; return RADON_OK; }
        if (sqrt(2 * f) >= bnorm) { out.fallback = RADON_FALLBACK_WORSE_THAN_ZERO; return RADON_OK; }
    }
    std::vector<double> fs(n_mem, f);
    double alpha = std::min(std::max(gnorm > 0 ? 1.0 / gnorm : 1.0, bb_min), bb_max);
    double f_old = INFINITY, f_best = f;
    int it_best = 0;
    bool newton_taken = !warm || tau == 0.0;   // a start at zero lies below the root
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
            if (rerr1 <= opt_tol && newton_taken) { status = 2; break; }
        }
        if (warm) {
            if (f < f_best) { f_best = f; it_best = it; }
            else if (it - it_best >= stall_iters) { out.fallback = RADON_FALLBACK_STALLED; break; }
        }
        const double change = fabs(f - f_old);
        const bool stalled = (change <= dec_tol * f && rnorm > 2 * sigma) ||
                             (change <= 0.1 * f * fabs(rnorm - sigma) && rnorm <= 2 * sigma);
        if (stalled && gnorm > 0) {
            const double tau_old = tau;
            tau = std::max(0.0, tau + rnorm * aerr1 / gnorm);   // Newton step on the Pareto curve
            newton_taken = true;
            if (tau < tau_old) {
                // the ball shrank: restart from the projected iterate with its
                // own residual and gradient
                if (!S.project_sync(w.x, w.x, 0.0, tau, w.xn, fin)) return RADON_ERR_DEVICE;
                std::swap(w.x, w.xn);
                if (!S.forward(w.x, w.z)) return RADON_ERR_DEVICE;
                S.residual(w.z, w.r, w.bt);
                if (!S.adjoint(w.r, w.h)) return RADON_ERR_DEVICE;
                S.bb(nullptr, w.x, nullptr, w.h);
                if (!S.read(fin)) return RADON_ERR_DEVICE;
                f = 0.5 * fin[FIN_RES];
                rbt = fin[FIN_RES + 1];
                gnorm = fin[FIN_BB + 2];
            }
            std::fill(fs.begin(), fs.end(), f);
        }
        // spectral projected gradient step, non-monotone (GLL) backtracking; the
        // gradient and spectral sums of each trial point are computed before the
        // host reads the trial's objective, so an accepted step costs one wait
        const double fmax = *std::max_element(fs.begin(), fs.end());
        double step = 1.0, fn = 0, rbtn = 0;
        while (true) {
            bool fresh = true;
            for (int round = 0; round < 64; ++round) {   // rarely more than one round
                S.project(w.x, w.h, step * alpha, tau, w.xn, fresh);
                fresh = false;
                if (!S.forward(w.xn, w.z)) return RADON_ERR_DEVICE;
                S.residual(w.z, w.rn, w.bt);
                if (!S.adjoint(w.rn, w.hn)) return RADON_ERR_DEVICE;
                S.bb(w.x, w.xn, w.h, w.hn);
                if (!S.read(fin)) return RADON_ERR_DEVICE;
                if (fin[FIN_PROJ + 2] != 0.0) break;
            }
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
        !w.alloc(&w.part, (size_t)rn::SV_SLOTS * rn::SV_BLOCKS) || !w.alloc(&w.fin, FIN_COUNT) ||
        !w.alloc(&w.lam, 2) || !w.alloc(&w.pj, (size_t)2 * rn::PJ_BLOCKS) || !w.alloc(&w.ticket, 1))
        return RADON_ERR_OOM;
    hipStream_t st = (hipStream_t)stream;
    Solver S{plan, p, w, st, opts->ring_filter != 0, b_dev, n2, ns};
    const std::vector<double> Q = cubic_basis(p.n_det);
    S.chk(hipMemcpyAsync(w.Q, Q.data(), sizeof(double) * Q.size(), hipMemcpyHostToDevice, st));

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

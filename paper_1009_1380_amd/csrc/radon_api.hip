// radon_api.hip - the C ABI (include/radon.h): plan construction on the host
// (float64 geometry and tables), the device sample sort, and the enqueueing of
// the forward and adjoint kernel sequences on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <new>
#include <string>
#include <vector>

#include "../../include/radon.h"
#include "radon_internal.hpp"
#include "radon_sort.hpp"

using rn::Plan;

namespace {

thread_local std::string g_last_error;

radon_status_t fail(radon_status_t st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

radon_status_t ok() {
    g_last_error.clear();
    return RADON_OK;
}

// Visits per spreading work item; longer tile lists are split and their
// partial tiles summed in a fixed order.
constexpr int kA2Chunk = rn::A2_CHUNK;
// Samples per forward interpolation work item.
constexpr int kF3Chunk = rn::F3_CHUNK;
// Cubic Kaiser-Bessel pieces per unit of t (a power of two).
constexpr int kKbS = rn::KB_S;

// I0(x) by its power series sum ((x/2)^(2k) / (k!)^2); x <= 40 here.
double bessel_i0(double x) {
    const double y = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= y / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// phi(t) = I0(beta sqrt(1 - (2t/W)^2)) / I0(beta) on |t| < W/2.
double kb_phi(double t, int W, double beta) {
    const double r = 2.0 * t / W;
    if (fabs(r) >= 1.0) return 0.0;
    return bessel_i0(beta * sqrt(1.0 - r * r)) / bessel_i0(beta);
}

// Fourier transform of phi: (W / I0(beta)) sinh(z)/z, z^2 = beta^2 - (pi W f)^2.
double kb_phihat(double f, int W, double beta) {
    const double z2 = beta * beta - (M_PI * W * f) * (M_PI * W * f);
    double r;
    if (z2 > 0) { const double z = sqrt(z2); r = sinh(z) / z; }
    else if (z2 < 0) { const double z = sqrt(-z2); r = sin(z) / z; }
    else r = 1.0;
    return r * W / bessel_i0(beta);
}

// Cubic c0 + c1 f + c2 f^2 + c3 f^3 through phi at the four Chebyshev points
// of piece i (t = (i + f)/S, f in [0, 1)), solved in float64.
void kb_cubic_piece(int i, int S, int W, double beta, double c[4]) {
    double A[4][5];
    for (int k = 0; k < 4; ++k) {
        const double f = 0.5 + 0.5 * cos(M_PI * (k + 0.5) / 4.0);
        double pw = 1.0;
        for (int j = 0; j < 4; ++j) { A[k][j] = pw; pw *= f; }
        A[k][4] = kb_phi((i + f) / S, W, beta);
    }
    for (int col = 0; col < 4; ++col) {   // Gaussian elimination, partial pivoting
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        for (int j = 0; j < 5; ++j) std::swap(A[col][j], A[piv][j]);
        for (int r = 0; r < 4; ++r) {
            if (r == col) continue;
            const double m = A[r][col] / A[col][col];
            for (int j = col; j < 5; ++j) A[r][j] -= m * A[col][j];
        }
    }
    for (int j = 0; j < 4; ++j) c[j] = A[j][4] / A[j][j];
}

// Ramp weights of the filtered adjoint for q = 0..N/2: (pi/n_views) times the
// DFT of the band-limited spatial ramp kernel h[0] = 1/4, h[k] = -1/(pi k)^2
// (odd k), 0 (even k), on |k| < N/2, as a cosine series in float64.
std::vector<float> ramp_weights(int n_views, int N) {
    std::vector<float> w(N / 2 + 1);
    for (int q = 0; q <= N / 2; ++q) {
        double H = 0.25;
        for (int k = 1; k < N / 2; k += 2)
            H -= 2.0 * cos(2.0 * M_PI * (double)q * k / N) / ((M_PI * k) * (M_PI * k));
        w[q] = (float)(M_PI / n_views * H);
    }
    return w;
}

bool is_supported_length(int len) { return rn::length_supported(len); }

// Failure-injection hook for the tests: with RADON_TEST_FAIL_ALLOC=k in the
// environment, the k-th device allocation made while building a plan
// (counting from 1) fails as if the device were out of memory.
int test_fail_alloc_at() {
    const char* e = getenv("RADON_TEST_FAIL_ALLOC");
    return e ? atoi(e) : 0;
}

// hipMalloc, counted against the plan's failure-injection hook.
hipError_t plan_malloc(Plan& p, void** ptr, size_t bytes) {
    ++p.n_allocs;
    if (p.fail_alloc_at > 0 && p.n_allocs == p.fail_alloc_at) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(ptr, bytes);
}

template <class T>
radon_status_t dev_alloc(Plan& p, T** out, size_t count) {
    *out = nullptr;
    if (count == 0) count = 1;
    void* ptr = nullptr;
    const size_t bytes = count * sizeof(T);
    if (plan_malloc(p, &ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(RADON_ERR_OOM, "hipMalloc of %zu bytes failed", bytes);
    }
    p.allocs.push_back(ptr);
    p.bytes += bytes;
    *out = static_cast<T*>(ptr);
    return RADON_OK;
}

template <class T>
radon_status_t upload(T* dst, const std::vector<T>& src) {
    if (hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return fail(RADON_ERR_DEVICE, "host-to-device copy failed");
    }
    return RADON_OK;
}

void free_plan(Plan& p) {
    for (void* ptr : p.allocs) (void)hipFree(ptr);
    p.allocs.clear();
    for (auto& pt : p.pending) { (void)hipEventDestroy(pt.e0); (void)hipEventDestroy(pt.e1); }
    p.pending.clear();
    for (hipEvent_t e : p.event_pool) (void)hipEventDestroy(e);
    p.event_pool.clear();
}

std::vector<float2> twiddles(int len) {
    std::vector<float2> t(len);
    for (int k = 0; k < len; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)len;
        t[k] = make_float2((float)cos(a), (float)sin(a));
    }
    return t;
}

hipEvent_t take_event(Plan& p) {
    if (!p.event_pool.empty()) {
        hipEvent_t e = p.event_pool.back();
        p.event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    return e;
}

// Run one launcher, bracketed by events when profiling is on.
template <class F>
hipError_t staged(Plan& p, int stage, hipStream_t st, F&& launch) {
    if (!p.profiling) return launch();
    hipEvent_t e0 = take_event(p), e1 = take_event(p);
    if (!e0 || !e1) return launch();
    (void)hipEventRecord(e0, st);
    const hipError_t err = launch();
    (void)hipEventRecord(e1, st);
    p.pending.push_back({stage, e0, e1});
    return err;
}

radon_status_t check_plan(radon_plan_t plan) {
    if (!plan) return fail(RADON_ERR_INVALID, "plan is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(RADON_ERR_DEVICE, "hipGetDevice failed");
    }
    if (dev != plan->p.device)
        return fail(RADON_ERR_INVALID, "current device %d differs from the plan's device %d", dev,
                    plan->p.device);
    return RADON_OK;
}

radon_status_t launch_status(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(RADON_ERR_DEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
    return RADON_OK;
}

radon_status_t run_forward(Plan& p, const float* img, float* sino, hipStream_t st) {
    radon_status_t s;
    if ((s = launch_status(staged(p, rn::ST_F1, st, [&] { return rn::launch_f1(p, img, st); }), "F1"))) return s;
    if ((s = launch_status(staged(p, rn::ST_F2, st, [&] { return rn::launch_f2(p, st); }), "F2"))) return s;
    if ((s = launch_status(staged(p, rn::ST_F3, st, [&] { return rn::launch_f3(p, st); }), "F3"))) return s;
    if ((s = launch_status(staged(p, rn::ST_F4, st, [&] { return rn::launch_f4(p, sino, st); }), "F4"))) return s;
    return RADON_OK;
}

radon_status_t run_adjoint_grid(Plan& p, const float* sino, hipStream_t st, bool filtered = false) {
    radon_status_t s;
    if ((s = launch_status(staged(p, rn::ST_A1, st, [&] { return rn::launch_a1(p, sino, filtered, st); }), "A1")))
        return s;
    if ((s = launch_status(staged(p, rn::ST_A2, st, [&] { return rn::launch_a2(p, st); }), "A2"))) return s;
    if (p.n_splits > 0)
        if ((s = launch_status(staged(p, rn::ST_A2R, st, [&] { return rn::launch_a2_reduce(p, st); }), "A2 reduce"))) return s;
    return RADON_OK;
}

radon_status_t run_adjoint(Plan& p, const float* sino, float* img, hipStream_t st, bool filtered = false) {
    radon_status_t s;
    if ((s = run_adjoint_grid(p, sino, st, filtered))) return s;
    if ((s = launch_status(staged(p, rn::ST_A3, st, [&] { return rn::launch_a3(p, st); }), "A3"))) return s;
    if ((s = launch_status(staged(p, rn::ST_A4, st, [&] { return rn::launch_a4(p, img, st); }), "A4"))) return s;
    return RADON_OK;
}

// Device sort of the sample keys: keys, LSD radix passes, bin offsets.
radon_status_t sort_samples(Plan& p, std::vector<int>& offsets_host) {
    const int total = (int)p.n_samples;
    const int nblocks = (total + rn::SORT_TILE - 1) / rn::SORT_TILE;
    int *k0 = nullptr, *k1 = nullptr, *v0 = nullptr, *v1 = nullptr, *hist = nullptr;
    auto cleanup = [&] {
        for (int* x : {k0, k1, v0, v1, hist})
            if (x) (void)hipFree(x);
    };
    void* ptr[5] = {};
    const size_t bytes[5] = {sizeof(int) * total, sizeof(int) * total, sizeof(int) * total, sizeof(int) * total,
                             sizeof(int) * rn::SORT_RADIX * nblocks};
    bool got = true;
    for (int i = 0; i < 5 && got; ++i) got = plan_malloc(p, &ptr[i], bytes[i]) == hipSuccess;
    k0 = (int*)ptr[0];
    k1 = (int*)ptr[1];
    v0 = (int*)ptr[2];
    v1 = (int*)ptr[3];
    hist = (int*)ptr[4];
    if (!got) {
        (void)hipGetLastError();
        cleanup();
        return fail(RADON_ERR_OOM, "sort scratch allocation failed");
    }
    hipLaunchKernelGGL(rn::k_sample_keys, dim3((total + 255) / 256), dim3(256), 0, 0, p.cs, k0, v0,
                       p.n_views, p.n_det, p.G, p.W, p.T);
    const int n_keys = 4 * p.n_bins;
    int bits = 0;
    while ((1 << bits) < n_keys) ++bits;
    for (int shift = 0; shift < bits; shift += 4) {
        hipLaunchKernelGGL(rn::k_sort_hist, dim3(nblocks), dim3(rn::SORT_NT), 0, 0, k0, total, shift, hist, nblocks);
        hipLaunchKernelGGL(rn::k_exclusive_scan, dim3(1), dim3(1024), 0, 0, hist, rn::SORT_RADIX * nblocks);
        hipLaunchKernelGGL(rn::k_sort_scatter, dim3(nblocks), dim3(rn::SORT_NT), 0, 0, k0, v0, k1, v1, total,
                           shift, hist, nblocks);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    hipLaunchKernelGGL(rn::k_bin_offsets, dim3((n_keys + 1 + 255) / 256), dim3(256), 0, 0, k0, total,
                       p.offs4, n_keys);
    hipLaunchKernelGGL(rn::k_sample_recs, dim3((total + 255) / 256), dim3(256), 0, 0, v0, p.cs, p.recs, total,
                       p.n_views, p.n_det, p.G, p.W, p.T);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(p.perm, v0, sizeof(int) * total, hipMemcpyDeviceToDevice);
    offsets_host.assign(n_keys + 1, 0);
    if (e == hipSuccess)
        e = hipMemcpy(offsets_host.data(), p.offs4, sizeof(int) * (n_keys + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    cleanup();
    if (e != hipSuccess) return fail(RADON_ERR_DEVICE, "sample sort failed: %s", hipGetErrorString(e));
    return RADON_OK;
}

// Work lists. Spreading: one item per chunk of the visit list of each output
// strip of the half plane: A2_GX consecutive tile columns of one tile row
// (tile column 0 holds the mx = G/2 line and is a strip of its own, columns
// ntl/2..ntl-1 hold mx = 0..G/2-1 and are taken in runs of A2_GX). The visit
// list of a strip is the diagonal neighbour's class 2, the v-neighbours'
// classes 2-3, the u-neighbour's classes 1-2 and all of the own bins -- the
// samples whose footprint reaches the strip. Forward: the forward tile
// columns ntl/2-1, .., ntl-1, 0 are taken in consecutive pairs (the last pair
// wraps to column 0) and the rows in pairs; each 2 x 2 super-tile's samples
// are cut into items of at most kF3Chunk.
radon_status_t build_work(Plan& p, const std::vector<int>& o4) {
    const int ntl = p.ntl;
    auto run = [&](int bin, int c0, int c1) { return o4[4 * bin + c1] - o4[4 * bin + c0]; };
    std::vector<rn::TileItem> items;
    std::vector<rn::F3Item> fitems;
    std::vector<rn::SplitTile> splits;
    std::vector<std::pair<int, int>> strips;   // (first column, columns)
    for (int cx = std::max(ntl / 2, 1); cx < ntl; cx += rn::A2_GX) strips.push_back({cx, std::min(rn::A2_GX, ntl - cx)});
    strips.push_back({0, 1});
    int slots = 0;
    const int chunk = p.a2_chunk;
    auto strip_total = [&](int cx, int cy, int gx) {
        const int xl = (cx + ntl - 1) % ntl, yu = (cy + ntl - 1) % ntl;
        int total = run(yu * ntl + xl, 2, 3) + run(cy * ntl + xl, 1, 3);
        for (int j = 0; j < gx; ++j) total += run(yu * ntl + cx + j, 2, 4) + run(cy * ntl + cx + j, 0, 4);
        return total;
    };
    for (int cy = 0; cy < ntl; ++cy) {
        for (const auto& st0 : strips) {
            // a strip too long for one item is cut back to single tiles: their
            // partial sums are half as many, which shortens the reduction
            std::vector<std::pair<int, int>> parts;
            if (st0.second > 1 && strip_total(st0.first, cy, st0.second) > chunk) {
                for (int j = 0; j < st0.second; ++j) parts.push_back({st0.first + j, 1});
            } else {
                parts.push_back(st0);
            }
            for (const auto& st : parts) {
            const int cx = st.first, gx = st.second;
            const int total = strip_total(cx, cy, gx);
            if (total <= chunk) {
                items.push_back({cx, cy, 0, total, -1, gx, 0, 0});
            } else {
                const int nch = (total + chunk - 1) / chunk;
                splits.push_back({cx, cy, slots, nch, gx, 0});
                for (int k = 0; k < nch; ++k)
                    items.push_back({cx, cy, k * chunk, std::min(chunk, total - k * chunk), slots + k, gx, 0, 0});
                slots += nch;
            }
            }
        }
    }
    // forward columns in order, without repeats
    std::vector<int> fcols;
    for (int cx = std::max(ntl / 2 - 1, 0); cx < ntl; ++cx) fcols.push_back(cx);
    if (std::find(fcols.begin(), fcols.end(), 0) == fcols.end()) fcols.push_back(0);
    for (size_t k = 0; k < fcols.size(); k += 2) {
        const int cx = fcols[k];
        const int nbx = (k + 1 < fcols.size()) ? 2 : 1;
        for (int cy = 0; cy < ntl; cy += 2) {
            const int cy1 = (cy + 1) % ntl;
            int n_all = run(cy * ntl + cx, 0, 4) + run(cy1 * ntl + cx, 0, 4);
            if (nbx > 1) {
                const int cx1 = (cx + 1) % ntl;
                n_all += run(cy * ntl + cx1, 0, 4) + run(cy1 * ntl + cx1, 0, 4);
            }
            for (int s = 0; s < n_all; s += p.f3_chunk)
                fitems.push_back({cx, cy, nbx, s, std::min(p.f3_chunk, n_all - s), 0, {}, {}, 0});
        }
    }
    // each item's visit ranges: the diagonal neighbour's class 2, the
    // v-neighbours' classes 2-3, the u-neighbour's classes 1-2 and the own
    // bins (consecutive bins, one range)
    for (rn::TileItem& it : items) {
        const int xl = (it.cx + ntl - 1) % ntl, yu = (it.cy + ntl - 1) % ntl;
        auto range = [&](int q, int b0, int c0, int b1, int c1) {
            it.rs[q] = o4[4 * b0 + c0];
            it.rl[q] = o4[4 * b1 + c1] - it.rs[q];
        };
        range(0, yu * ntl + xl, 2, yu * ntl + xl, 3);
        for (int j = 0; j < rn::A2_GX; ++j) {
            if (j < it.gx) range(1 + j, yu * ntl + it.cx + j, 2, yu * ntl + it.cx + j, 4);
            else it.rs[1 + j] = it.rl[1 + j] = 0;
        }
        range(rn::A2_GX + 1, it.cy * ntl + xl, 1, it.cy * ntl + xl, 3);
        range(rn::A2_GX + 2, it.cy * ntl + it.cx, 0, it.cy * ntl + it.cx + it.gx, 0);
    }
    // each forward item's bin ranges
    for (rn::F3Item& it : fitems) {
        const int cx1 = (it.cx + 1) % ntl, cy1 = (it.cy + 1) % ntl;
        const int b[4] = {it.cy * ntl + it.cx, it.cy * ntl + cx1, cy1 * ntl + it.cx, cy1 * ntl + cx1};
        for (int q = 0; q < 4; ++q) it.s[q] = o4[4 * b[q]];
        for (int q = 0; q < 3; ++q) it.n[q] = o4[4 * b[q] + 4] - it.s[q];
        if (it.nbx < 2) it.n[1] = 0;
    }
    // longest items first so the tail of each launch is short
    std::stable_sort(items.begin(), items.end(),
                     [](const rn::TileItem& a, const rn::TileItem& b) { return a.count > b.count; });
    std::stable_sort(fitems.begin(), fitems.end(),
                     [](const rn::F3Item& a, const rn::F3Item& b) { return a.count > b.count; });
    p.n_items = (int)items.size();
    p.n_fitems = (int)fitems.size();
    p.items_h = items;
    p.fitems_h = fitems;
    p.splits_h = splits;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p.device) != hipSuccess || cus < 1) {
            (void)hipGetLastError();
            cus = 1;
        }
        p.f3_grid = std::max(1, std::min(p.n_fitems, rn::f3_blocks_per_cu(p.W, p.T) * cus));
    }
    p.n_splits = (int)splits.size();
    p.n_slots = slots;
    radon_status_t s;
    if ((s = dev_alloc(p, &p.items, items.size()))) return s;
    if (!items.empty() && (s = upload(p.items, items))) return s;
    if ((s = dev_alloc(p, &p.fitems, fitems.size()))) return s;
    if (!fitems.empty() && (s = upload(p.fitems, fitems))) return s;
    if ((s = dev_alloc(p, &p.splits, splits.size()))) return s;
    if (!splits.empty() && (s = upload(p.splits, splits))) return s;
    if ((s = dev_alloc(p, &p.partials, (size_t)std::max(slots, 1) * rn::A2_GX * p.T * p.T))) return s;
    return RADON_OK;
}

radon_status_t build_plan(Plan& p, int n, const double* angles, int n_views, int n_det, double sigma, int W,
                          const radon_tuning& tuning) {
    p.n = n;
    p.n_views = n_views;
    p.n_det = n_det;
    p.W = W;
    p.sigma = sigma;
    p.G = 2 * n;
    const int G = p.G;
    // tile size: T divides G/2 (tiles do not straddle the half-plane edge) and
    // T >= W (a footprint spans at most two tiles); default the largest of 32/16/8
    p.T = 0;
    if (tuning.tile) {
        if ((G / 2) % tuning.tile || tuning.tile < W)
            return fail(RADON_ERR_UNSUPPORTED, "tile %d does not fit G=%d, W=%d", tuning.tile, G, W);
        p.T = tuning.tile;
    } else {
        for (int T : {32, 16, 8})
            if ((G / 2) % T == 0 && T >= W) { p.T = T; break; }
    }
    if (p.T == 0) return fail(RADON_ERR_UNSUPPORTED, "no tile size in {8,16,32} fits G=%d", G);
    p.a2_chunk = tuning.a2_chunk ? tuning.a2_chunk : kA2Chunk;
    p.f3_chunk = tuning.f3_chunk ? tuning.f3_chunk : kF3Chunk;
    p.ntl = G / p.T;
    p.n_bins = p.ntl * p.ntl;
    p.n_samples = (int64_t)n_views * n_det + n_views;
    p.beta = M_PI * sqrt((W / sigma) * (W / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8);

    // host tables in float64, rounded once
    std::vector<double2> cs(n_views);
    for (int a = 0; a < n_views; ++a) cs[a] = make_double2(cos(angles[a]), sin(angles[a]));
    std::vector<float> psi_inv(n);
    for (int i = 0; i < n; ++i) psi_inv[i] = (float)(1.0 / kb_phihat(((double)i - n / 2) / G, W, p.beta));
    std::vector<float2> shift(n);
    for (int i = 0; i < n; ++i) {
        const double a = -M_PI * ((double)i - n / 2) / (double)n;
        shift[i] = make_float2((float)cos(a), (float)sin(a));
    }
    const int npiece = (W / 2) * kKbS;
    std::vector<float4> kbc(npiece);
    for (int i = 0; i < npiece; ++i) {
        double c[4];
        kb_cubic_piece(i, kKbS, W, p.beta, c);
        kbc[i] = make_float4((float)c[0], (float)c[1], (float)c[2], (float)c[3]);
    }

    radon_status_t s;
    if ((s = dev_alloc(p, &p.cs, n_views)) || (s = upload(p.cs, cs))) return s;
    if ((s = dev_alloc(p, &p.psi_inv, n)) || (s = upload(p.psi_inv, psi_inv))) return s;
    if ((s = dev_alloc(p, &p.shift_n, n)) || (s = upload(p.shift_n, shift))) return s;
    if ((s = dev_alloc(p, &p.tw_n, n)) || (s = upload(p.tw_n, twiddles(n)))) return s;
    if ((s = dev_alloc(p, &p.tw_N, n_det)) || (s = upload(p.tw_N, twiddles(n_det)))) return s;
    if ((s = dev_alloc(p, &p.kbc, kbc.size())) || (s = upload(p.kbc, kbc))) return s;
    if ((s = dev_alloc(p, &p.fbpw, n_det / 2 + 1)) || (s = upload(p.fbpw, ramp_weights(n_views, n_det)))) return s;
    if ((s = dev_alloc(p, &p.ringQ, (size_t)n_det * 4)) || (s = upload(p.ringQ, rn::ring_cubic_basis(n_det)))) return s;
    if ((s = dev_alloc(p, &p.perm, (size_t)p.n_samples))) return s;
    if ((s = dev_alloc(p, &p.recs, (size_t)p.n_samples))) return s;
    if ((s = dev_alloc(p, &p.offs4, (size_t)4 * p.n_bins + 1))) return s;
    std::vector<int> offs;
    if ((s = sort_samples(p, offs))) return s;
    if ((s = build_work(p, offs))) return s;
    if ((s = dev_alloc(p, &p.T1, (size_t)(n + 1) * n))) return s;
    if ((s = dev_alloc(p, &p.grid, (size_t)(n + 1) * G))) return s;
    if ((s = dev_alloc(p, &p.Yh, (size_t)n_views * (n_det / 2 + 1)))) return s;
    if ((s = dev_alloc(p, &p.Xr, (size_t)n_views * (n_det / 2 + 1)))) return s;
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return fail(RADON_ERR_DEVICE, "device synchronisation failed after plan setup");
    }
    return RADON_OK;
}

}  // namespace

namespace rn {
radon_status_t api_fail(radon_status_t st, const char* msg) { return fail(st, "%s", msg); }
radon_status_t api_ok() { return ok(); }
radon_status_t api_check_plan(radon_plan_t plan) { return check_plan(plan); }
radon_status_t api_run_forward(Plan& p, const float* img, float* sino, hipStream_t st) {
    return run_forward(p, img, sino, st);
}
radon_status_t api_run_adjoint(Plan& p, const float* sino, float* img, hipStream_t st) {
    return run_adjoint(p, sino, img, st);
}
bool length_supported(int len) {
    switch (len) {
#define RN_CASE(L) case L:
        RN_FOR_LENGTHS(RN_CASE)
#undef RN_CASE
        return true;
        default:
            return false;
    }
}

hipError_t launch_fft_test(int len, int batch, int inverse, const float2* in, float2* out, const float2* tw,
                           hipStream_t st) {
    switch (len) {
#define RN_CASE(L)                                                                                  \
    case L: {                                                                                       \
        constexpr int NT = fft_threads(L, 1);                                                       \
        hipLaunchKernelGGL((k_fft_test<L, NT>), dim3(batch), dim3(NT), 0, st, in, out, tw, inverse); \
        break;                                                                                      \
    }
        RN_FOR_LENGTHS(RN_CASE)
#undef RN_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace rn

extern "C" {

radon_status_t radon_plan(radon_plan_t* out, int n, const double* angles, int n_views, int n_det,
                          double sigma, int W) {
    return radon_plan_tuned(out, n, angles, n_views, n_det, sigma, W, nullptr);
}

radon_status_t radon_plan_tuned(radon_plan_t* out, int n, const double* angles, int n_views, int n_det,
                                double sigma, int W, const radon_tuning* tuning) {
    if (!out) return fail(RADON_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!angles) return fail(RADON_ERR_INVALID, "angles is NULL");
    if (n < 8 || n % 2) return fail(RADON_ERR_INVALID, "n=%d must be even and >= 8", n);
    if (n_det < 8 || n_det % 2) return fail(RADON_ERR_INVALID, "n_det=%d must be even and >= 8", n_det);
    if (n_views < 1) return fail(RADON_ERR_INVALID, "n_views=%d must be >= 1", n_views);
    if (!(sigma > 1.0) || fabs(sigma * n - round(sigma * n)) > 1e-9 || ((long)round(sigma * n)) % 2)
        return fail(RADON_ERR_INVALID, "sigma*n must be an even integer with sigma > 1 (sigma=%g)", sigma);
    if (W < 2 || W > 16 || W % 2) return fail(RADON_ERR_INVALID, "W=%d must be even, 2..16", W);
    for (int a = 0; a < n_views; ++a)
        if (!isfinite(angles[a])) return fail(RADON_ERR_INVALID, "angle %d is not finite", a);
    if (fabs(sigma - 2.0) > 1e-12) return fail(RADON_ERR_UNSUPPORTED, "only sigma = 2 is implemented");
    if (W != 4 && W != 6 && W != 8) return fail(RADON_ERR_UNSUPPORTED, "W=%d: only 4, 6, 8 are implemented", W);
    if (n % 8) return fail(RADON_ERR_UNSUPPORTED, "n=%d must be a multiple of 8", n);
    if (!is_supported_length(n)) return fail(RADON_ERR_UNSUPPORTED, "n=%d is not a supported FFT length", n);
    if (!is_supported_length(n_det))
        return fail(RADON_ERR_UNSUPPORTED, "n_det=%d is not a supported FFT length", n_det);
    if ((int64_t)n_views * n_det + n_views >= (int64_t)1 << 30 || (int64_t)n_views * (n_det / 2 + 1) >= (int64_t)1 << 29)
        return fail(RADON_ERR_UNSUPPORTED, "too many samples");
    const radon_tuning tn = tuning ? *tuning : radon_tuning{0, 0, 0};
    if (tn.tile != 0 && tn.tile != 8 && tn.tile != 16 && tn.tile != 32)
        return fail(RADON_ERR_INVALID, "tile=%d must be 0, 8, 16 or 32", tn.tile);
    if (tn.a2_chunk != 0 && (tn.a2_chunk < 64 || tn.a2_chunk > kA2Chunk))
        return fail(RADON_ERR_INVALID, "a2_chunk=%d must be 0 or 64..%d", tn.a2_chunk, kA2Chunk);
    if (tn.f3_chunk != 0 && (tn.f3_chunk < 256 || tn.f3_chunk > 65536))
        return fail(RADON_ERR_INVALID, "f3_chunk=%d must be 0 or 256..65536", tn.f3_chunk);

    radon_plan_s* plan = new (std::nothrow) radon_plan_s();
    if (!plan) return fail(RADON_ERR_OOM, "host allocation failed");
    plan->p.fail_alloc_at = test_fail_alloc_at();
    if (hipGetDevice(&plan->p.device) != hipSuccess) {
        (void)hipGetLastError();
        delete plan;
        return fail(RADON_ERR_DEVICE, "no HIP device");
    }
    const radon_status_t s = build_plan(plan->p, n, angles, n_views, n_det, sigma, W, tn);
    if (s != RADON_OK) {
        const std::string msg = g_last_error;
        (void)hipDeviceSynchronize();
        (void)hipGetLastError();
        free_plan(plan->p);
        delete plan;
        g_last_error = msg;
        return s;
    }
    *out = plan;
    return ok();
}

radon_status_t radon_forward(radon_plan_t plan, const float* img_dev, float* sino_dev, void* stream) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    if (!img_dev || !sino_dev) return fail(RADON_ERR_INVALID, "NULL buffer");
    if ((s = run_forward(plan->p, img_dev, sino_dev, (hipStream_t)stream))) return s;
    return ok();
}

radon_status_t radon_adjoint(radon_plan_t plan, const float* sino_dev, float* img_dev, void* stream) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    if (!img_dev || !sino_dev) return fail(RADON_ERR_INVALID, "NULL buffer");
    if ((s = run_adjoint(plan->p, sino_dev, img_dev, (hipStream_t)stream))) return s;
    return ok();
}

radon_status_t radon_fbp(radon_plan_t plan, const float* sino_dev, float* img_dev, void* stream) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    if (!img_dev || !sino_dev) return fail(RADON_ERR_INVALID, "NULL buffer");
    if ((s = run_adjoint(plan->p, sino_dev, img_dev, (hipStream_t)stream, true))) return s;
    return ok();
}

radon_status_t radon_forward_batched(radon_plan_t plan, int batch, const float* imgs_dev, float* sinos_dev,
                                     void* stream) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    if (batch < 0) return fail(RADON_ERR_INVALID, "batch=%d < 0", batch);
    if (batch > 0 && (!imgs_dev || !sinos_dev)) return fail(RADON_ERR_INVALID, "NULL buffer");
    const Plan& p = plan->p;
    for (int b = 0; b < batch; ++b)
        if ((s = run_forward(plan->p, imgs_dev + (size_t)b * p.n * p.n,
                             sinos_dev + (size_t)b * p.n_views * p.n_det, (hipStream_t)stream)))
            return s;
    return ok();
}

radon_status_t radon_adjoint_batched(radon_plan_t plan, int batch, const float* sinos_dev, float* imgs_dev,
                                     void* stream) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    if (batch < 0) return fail(RADON_ERR_INVALID, "batch=%d < 0", batch);
    if (batch > 0 && (!imgs_dev || !sinos_dev)) return fail(RADON_ERR_INVALID, "NULL buffer");
    const Plan& p = plan->p;
    for (int b = 0; b < batch; ++b)
        if ((s = run_adjoint(plan->p, sinos_dev + (size_t)b * p.n_views * p.n_det,
                             imgs_dev + (size_t)b * p.n * p.n, (hipStream_t)stream)))
            return s;
    return ok();
}

radon_status_t radon_plan_sort_indices(radon_plan_t plan, int32_t* perm_host, int64_t perm_cap,
                                       int32_t* offsets_host, int64_t offsets_cap) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    const Plan& p = plan->p;
    if (perm_host && perm_cap < p.n_samples) return fail(RADON_ERR_INVALID, "perm_cap too small");
    if (offsets_host && offsets_cap < 4 * (int64_t)p.n_bins + 1)
        return fail(RADON_ERR_INVALID, "offsets_cap too small");
    hipError_t e = hipSuccess;
    if (perm_host) e = hipMemcpy(perm_host, p.perm, sizeof(int) * p.n_samples, hipMemcpyDeviceToHost);
    if (e == hipSuccess && offsets_host)
        e = hipMemcpy(offsets_host, p.offs4, sizeof(int) * (4 * (size_t)p.n_bins + 1), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(RADON_ERR_DEVICE, "copy failed: %s", hipGetErrorString(e));
    return ok();
}

radon_status_t radon_plan_info(radon_plan_t plan, int64_t* info, int cap) {
    if (!plan || !info) return fail(RADON_ERR_INVALID, "NULL argument");
    const Plan& p = plan->p;
    const int64_t v[] = {p.n, p.n_views, p.n_det, p.W, p.G, p.T, p.n_samples, p.n_bins,
                         p.n_items, p.n_slots, (int64_t)p.bytes, p.n_fitems};
    for (int k = 0; k < cap && k < (int)(sizeof(v) / sizeof(v[0])); ++k) info[k] = v[k];
    return ok();
}

size_t radon_plan_device_bytes(radon_plan_t plan) { return plan ? plan->p.bytes : 0; }

void radon_plan_destroy(radon_plan_t plan) {
    if (!plan) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != plan->p.device) (void)hipSetDevice(plan->p.device);
    (void)hipDeviceSynchronize();
    free_plan(plan->p);
    if (cur >= 0 && cur != plan->p.device) (void)hipSetDevice(cur);
    (void)hipGetLastError();
    delete plan;
}

int radon_supported_length(int len) { return is_supported_length(len) ? 1 : 0; }

const char* radon_status_string(radon_status_t status) {
    switch (status) {
        case RADON_OK: return "RADON_OK";
        case RADON_ERR_INVALID: return "RADON_ERR_INVALID";
        case RADON_ERR_UNSUPPORTED: return "RADON_ERR_UNSUPPORTED";
        case RADON_ERR_OOM: return "RADON_ERR_OOM";
        case RADON_ERR_DEVICE: return "RADON_ERR_DEVICE";
        default: return "RADON_ERR_UNKNOWN";
    }
}

const char* radon_last_error(void) { return g_last_error.c_str(); }

radon_status_t radon_plan_set_profiling(radon_plan_t plan, int enable) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    Plan& p = plan->p;
    p.profiling = enable != 0;
    for (int k = 0; k < rn::ST_COUNT; ++k) { p.stage_ms[k] = 0; p.stage_cnt[k] = 0; }
    for (auto& pt : p.pending) {
        (void)hipEventSynchronize(pt.e1);
        p.event_pool.push_back(pt.e0);
        p.event_pool.push_back(pt.e1);
    }
    p.pending.clear();
    return ok();
}

radon_status_t radon_plan_stage_times(radon_plan_t plan, double* ms, int64_t* counts, int cap) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    Plan& p = plan->p;
    for (auto& pt : p.pending) {
        if (hipEventSynchronize(pt.e1) != hipSuccess) {
            (void)hipGetLastError();
            return fail(RADON_ERR_DEVICE, "event synchronisation failed");
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, pt.e0, pt.e1) == hipSuccess) {
            p.stage_ms[pt.stage] += t;
            p.stage_cnt[pt.stage] += 1;
        }
        p.event_pool.push_back(pt.e0);
        p.event_pool.push_back(pt.e1);
    }
    p.pending.clear();
    for (int k = 0; k < cap && k < rn::ST_COUNT; ++k) {
        if (ms) ms[k] = p.stage_ms[k];
        if (counts) counts[k] = p.stage_cnt[k];
    }
    return ok();
}

int radon_stage_count(void) { return rn::ST_COUNT; }

const char* radon_stage_name(int stage) {
    static const char* names[rn::ST_COUNT] = {"F1_row_fft", "F2_col_fft", "F3_interp", "F4_ray_ifft",
                                              "A1_ray_fft", "A2_spread", "A2_reduce", "A3_col_ifft",
                                              "A4_row_ifft"};
    return (stage >= 0 && stage < rn::ST_COUNT) ? names[stage] : "";
}

radon_status_t radon_debug_forward_grid(radon_plan_t plan, const float* img_dev, float* grid_dev, void* stream) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    if (!img_dev || !grid_dev) return fail(RADON_ERR_INVALID, "NULL buffer");
    Plan& p = plan->p;
    hipStream_t st = (hipStream_t)stream;
    if ((s = launch_status(rn::launch_f1(p, img_dev, st), "F1"))) return s;
    if ((s = launch_status(rn::launch_f2(p, st), "F2"))) return s;
    if (hipMemcpyAsync(grid_dev, p.grid, sizeof(float2) * (size_t)(p.n + 1) * p.G, hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
        return fail(RADON_ERR_DEVICE, "grid copy failed");
    return ok();
}

radon_status_t radon_debug_adjoint_grid(radon_plan_t plan, const float* sino_dev, float* grid_dev, void* stream) {
    radon_status_t s;
    if ((s = check_plan(plan))) return s;
    if (!sino_dev || !grid_dev) return fail(RADON_ERR_INVALID, "NULL buffer");
    Plan& p = plan->p;
    hipStream_t st = (hipStream_t)stream;
    const bool prof = p.profiling;
    p.profiling = false;
    s = run_adjoint_grid(p, sino_dev, st);
    p.profiling = prof;
    if (s) return s;
    if (hipMemcpyAsync(grid_dev, p.grid, sizeof(float2) * (size_t)(p.n + 1) * p.G, hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
        return fail(RADON_ERR_DEVICE, "grid copy failed");
    return ok();
}

radon_status_t radon_fft_test(int len, int batch, int inverse, const float* in_dev, float* out_dev, void* stream) {
    if (!in_dev || !out_dev) return fail(RADON_ERR_INVALID, "NULL buffer");
    if (batch < 1) return fail(RADON_ERR_INVALID, "batch=%d < 1", batch);
    if (!is_supported_length(len)) return fail(RADON_ERR_UNSUPPORTED, "len=%d not supported", len);
    hipStream_t st = (hipStream_t)stream;
    float2* tw = nullptr;
    if (hipMalloc(&tw, sizeof(float2) * len) != hipSuccess) {
        (void)hipGetLastError();
        return fail(RADON_ERR_OOM, "twiddle allocation failed");
    }
    const std::vector<float2> t = twiddles(len);
    hipError_t e = hipMemcpy(tw, t.data(), sizeof(float2) * len, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = rn::launch_fft_test(len, batch, inverse, reinterpret_cast<const float2*>(in_dev),
                                reinterpret_cast<float2*>(out_dev), tw, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(tw);
    if (e != hipSuccess) return fail(RADON_ERR_DEVICE, "fft test failed: %s", hipGetErrorString(e));
    return ok();
}

}  // extern "C"

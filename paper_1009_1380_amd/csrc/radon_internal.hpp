// radon_internal.hpp - plan layout and kernel launchers shared by the
// library's translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/radon.h"
#include "radon_kernels.hpp"
#include "radon_multi.hpp"

// Supported FFT lengths (image size n and detector count n_det).
#define RN_FOR_LENGTHS(X)                                                                        \
    X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) X(160) X(192)      \
    X(256) X(320) X(384) X(512) X(640) X(768) X(1024) X(1280) X(1536) X(2048) X(2560) X(3072) \
    X(4096)

namespace rn {

enum Stage {
    ST_F1 = 0,
    ST_F2,
    ST_F3,
    ST_F4,
    ST_A1,
    ST_A2,
    ST_A2R,
    ST_A3,
    ST_A4,
    ST_COUNT
};

struct PendingTiming {
    int stage;
    hipEvent_t e0, e1;
};

struct Plan {
    int device = 0;
    int n = 0, n_views = 0, n_det = 0, W = 0, G = 0, T = 0, ntl = 0;
    double sigma = 0, beta = 0;
    int64_t n_samples = 0;   // real samples + mirrored Nyquist samples
    int n_bins = 0;                     // tiles; the sort has 4 edge classes per tile
    int n_items = 0, n_slots = 0, n_splits = 0;   // spreading work
    int n_fitems = 0;                   // forward interpolation work
    int f3_grid = 0;                    // workgroups of the persistent forward interpolation
    int a2_chunk = 0, f3_chunk = 0;     // most visits / samples per work item

    // device tables
    double2* cs = nullptr;       // per view (cos, sin), float64
    float* psi_inv = nullptr;    // 1 / psi1[i], n
    float2* shift_n = nullptr;   // e^{-i pi (i - n/2)/n}, n
    float2* tw_n = nullptr;      // e^{-2 pi i t/n}, n
    float2* tw_N = nullptr;      // e^{-2 pi i t/N}, N
    float4* kbc = nullptr;       // cubic pieces of phi on [0, W/2]
    float* fbpw = nullptr;       // ramp weights of the filtered adjoint, q = 0..N/2
    double* ringQ = nullptr;     // orthonormal cubic basis of the ring filter, N x 4 (float64)
    // device workspace
    float2* T1 = nullptr;        // (n+1) x n complex64
    float2* grid = nullptr;      // (n+1) x G complex64
    float2* Yh = nullptr;        // n_views x (N/2+1) complex64 (adjoint ray spectra)
    float2* Xr = nullptr;        // n_views x (N/2+1) complex64 (forward polar samples)
    int* perm = nullptr;         // sorted sample ids
    SampleRec* recs = nullptr;   // per sorted sample: origin, fractions, spectrum index, flags
    int* offs4 = nullptr;        // 4 * n_bins + 1 class starts
    F3Item* fitems = nullptr;
    TileItem* items = nullptr;
    SplitTile* splits = nullptr;
    float2* partials = nullptr;
    // host copies of the work lists (batches concatenate them across slices)
    std::vector<TileItem> items_h;
    std::vector<F3Item> fitems_h;
    std::vector<SplitTile> splits_h;
    size_t bytes = 0;
    std::vector<void*> allocs;
    int n_allocs = 0;        // device allocations made while building the plan
    int fail_alloc_at = 0;   // failure-injection hook (RADON_TEST_FAIL_ALLOC), 0: off

    bool profiling = false;
    double stage_ms[ST_COUNT] = {};
    int64_t stage_cnt[ST_COUNT] = {};
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> event_pool;
};

// kernel launchers of one plan; each returns the launch status
hipError_t launch_f1(const Plan& p, const float* img, hipStream_t st);
hipError_t launch_f2(const Plan& p, hipStream_t st);
hipError_t launch_f3(const Plan& p, hipStream_t st);
int f3_blocks_per_cu(int W, int T);   // resident forward-interpolation workgroups per CU
hipError_t launch_f4(const Plan& p, float* sino, hipStream_t st);
hipError_t launch_a1(const Plan& p, const float* sino, bool filtered, hipStream_t st);
hipError_t launch_a2(const Plan& p, hipStream_t st);
hipError_t launch_a2_reduce(const Plan& p, hipStream_t st);
hipError_t launch_a3(const Plan& p, hipStream_t st);
hipError_t launch_a4(const Plan& p, float* img, hipStream_t st);
// Launchers for uneven batches (radon_multi.hpp): one transform pass over the
// slices of a device table, and the gridding pass of one (W, T) group.
enum PassKind { PK_F1, PK_F2, PK_F4, PK_A1, PK_A3, PK_A4 };
struct GridLaunch {
    int W, T;
    const F3Item* fitems;
    int n_fitems, f3_grid;
    const TileItem* items;
    int n_items;
    const SplitTile* splits;
    int n_splits;
    const float4* kbc;
};
PassSlice pass_slice_of(const Plan& p, PassKind kind, const void* in, void* out);
GridSlice grid_slice_of(const Plan& p);
hipError_t launch_pass(PassKind kind, int len, const PassSlice* tab, int ns, int nblocks, hipStream_t st);
hipError_t launch_pass_fwd(PassKind kind, int len, const PassSlice* tab, int ns, int nblocks, hipStream_t st);
hipError_t launch_pass_adj(PassKind kind, int len, const PassSlice* tab, int ns, int nblocks, hipStream_t st);
hipError_t launch_f3_grid(const GridLaunch& g, const GridSlice* gs, hipStream_t st);
hipError_t launch_a2_grid(const GridLaunch& g, const GridSlice* gs, bool reduce, hipStream_t st);

hipError_t launch_fft_test(int len, int batch, int inverse, const float2* in, float2* out,
                           const float2* tw, hipStream_t st);

bool length_supported(int len);

// Orthonormal basis of cubic polynomials over the detector (ring filter),
// row-major n_det x 4, float64 (defined in radon_solver.hip).
std::vector<double> ring_cubic_basis(int n_det);

// Shared with the other translation units of the C ABI (defined in
// radon_api.hip): error reporting into radon_last_error(), the plan check,
// and the forward / adjoint kernel sequences enqueued on a stream.
radon_status_t api_fail(radon_status_t st, const char* msg);
radon_status_t api_ok();
radon_status_t api_check_plan(radon_plan_t plan);
radon_status_t api_run_forward(Plan& p, const float* img, float* sino, hipStream_t st);
radon_status_t api_run_adjoint(Plan& p, const float* sino, float* img, hipStream_t st);

}  // namespace rn

// The opaque handle of the C ABI.
struct radon_plan_s {
    rn::Plan p;
};

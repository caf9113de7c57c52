// radon_adj.hip - launchers of the adjoint path (A1 ray FFT, A2 binned
// spreading + split-tile reduction, A3 column inverse FFT, A4 row inverse FFT),
// dispatched on the FFT length, kernel width and tile size.
#include "radon_internal.hpp"

namespace rn {

hipError_t launch_a1(const Plan& p, const float* sino, bool filtered, hipStream_t st) {
    const float* wq = filtered ? p.fbpw : nullptr;
    const dim3 grid((p.n_views + 1) / 2);
    switch (p.n_det) {
#define RN_CASE(L)                                                                             \
    case L: {                                                                                  \
        constexpr int NT = ray_threads(L);                                                     \
        hipLaunchKernelGGL((k_a1_rays<L, NT>), grid, dim3(NT), 0, st, sino, p.Yh, p.tw_N, wq,   \
                           p.n_views);                                                         \
        break;                                                                                 \
    }
        RN_FOR_LENGTHS(RN_CASE)
#undef RN_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int W, int T>
static hipError_t launch_a2_wt(const Plan& p, hipStream_t st) {
    if (p.n_items == 0) return hipSuccess;
    hipLaunchKernelGGL((k_a2_spread<W, T>), dim3(p.n_items), dim3(A2_NT), 0, st, p.items, p.offs4,
                       p.recs, p.Yh, p.kbc, p.grid, p.partials, p.G);
    return hipGetLastError();
}

template <int W>
static hipError_t launch_a2_w(const Plan& p, hipStream_t st) {
    switch (p.T) {
        case 8: return launch_a2_wt<W, 8>(p, st);
        case 16: return launch_a2_wt<W, 16>(p, st);
        case 32: return launch_a2_wt<W, 32>(p, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_a2(const Plan& p, hipStream_t st) {
    switch (p.W) {
        case 4: return launch_a2_w<4>(p, st);
        case 6: return launch_a2_w<6>(p, st);
        case 8: return launch_a2_w<8>(p, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_a2_reduce(const Plan& p, hipStream_t st) {
    if (p.n_splits == 0) return hipSuccess;
    switch (p.T) {
        case 8: hipLaunchKernelGGL((k_a2_reduce<8>), dim3(p.n_splits, (A2_GX * 8 * 8 + 255) / 256), dim3(256), 0, st, p.splits, p.partials, p.grid, p.G); break;
        case 16: hipLaunchKernelGGL((k_a2_reduce<16>), dim3(p.n_splits, (A2_GX * 16 * 16 + 255) / 256), dim3(256), 0, st, p.splits, p.partials, p.grid, p.G); break;
        case 32: hipLaunchKernelGGL((k_a2_reduce<32>), dim3(p.n_splits, (A2_GX * 32 * 32 + 255) / 256), dim3(256), 0, st, p.splits, p.partials, p.grid, p.G); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_a3(const Plan& p, hipStream_t st) {
    const dim3 grid(p.n + 1);
    switch (p.n) {
#define RN_CASE(L)                                                                             \
    case L: {                                                                                  \
        constexpr int NT = col_threads(L);                                                   \
        hipLaunchKernelGGL((k_a3_cols<L, NT>), grid, dim3(NT), 0, st, p.grid, p.T1, p.shift_n,  \
                           p.tw_n);                                                            \
        break;                                                                                 \
    }
        RN_FOR_LENGTHS(RN_CASE)
#undef RN_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_a4(const Plan& p, float* img, hipStream_t st) {
    const dim3 grid((p.n + 3) / 4);
    switch (p.n) {
#define RN_CASE(L)                                                                             \
    case L: {                                                                                  \
        constexpr int NT = row_threads(L);                                                   \
        hipLaunchKernelGGL((k_a4_rows<L, NT>), grid, dim3(NT), 0, st, p.T1, img, p.psi_inv,     \
                           p.shift_n, p.tw_n);                                                 \
        break;                                                                                 \
    }
        RN_FOR_LENGTHS(RN_CASE)
#undef RN_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace rn

// radon_fwd.hip - launchers of the forward path (F1 row FFT, F2 column FFT,
// F34 polar interpolation + ray inverse FFT), dispatched on the FFT length.
#include "radon_internal.hpp"

namespace rn {

hipError_t launch_f1(const Plan& p, const float* img, hipStream_t st) {
    const dim3 grid((p.n + 3) / 4);
    switch (p.n) {
#define RN_CASE(L)                                                                             \
    case L: {                                                                                  \
        constexpr int NT = fft_threads(L, 4);                                                  \
        hipLaunchKernelGGL((k_f1_rows<L, NT>), grid, dim3(NT), 0, st, img, p.T1, p.psi_inv,     \
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

hipError_t launch_f2(const Plan& p, hipStream_t st) {
    const dim3 grid(p.n + 1);
    switch (p.n) {
#define RN_CASE(L)                                                                             \
    case L: {                                                                                  \
        constexpr int NT = fft_threads(L, 2);                                                  \
        hipLaunchKernelGGL((k_f2_cols<L, NT>), grid, dim3(NT), 0, st, p.T1, p.grid, p.shift_n,  \
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

template <int W>
static hipError_t launch_f34_w(const Plan& p, float* sino, hipStream_t st) {
    const dim3 grid((p.n_views + 1) / 2);
    switch (p.n_det) {
#define RN_CASE(L)                                                                             \
    case L: {                                                                                  \
        constexpr int NT = fft_threads(L, 2);                                                  \
        hipLaunchKernelGGL((k_f34_rays<L, W, NT>), grid, dim3(NT), 0, st, p.grid, sino, p.cs,   \
                           p.kbtab, p.kbL, p.tw_N, p.G, p.n_views);                            \
        break;                                                                                 \
    }
        RN_FOR_LENGTHS(RN_CASE)
#undef RN_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_f34(const Plan& p, float* sino, hipStream_t st) {
    switch (p.W) {
        case 4: return launch_f34_w<4>(p, sino, st);
        case 6: return launch_f34_w<6>(p, sino, st);
        case 8: return launch_f34_w<8>(p, sino, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rn

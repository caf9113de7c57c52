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
    hipLaunchKernelGGL((k_a2_spread<W, T>), dim3(p.n_items), dim3(A2_NT), 0, st, p.items,
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
    const dim3 grid(row_blocks(p.n));
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

// ---------------------------------------------------------------- batches

hipError_t launch_pass_adj(PassKind kind, int len, const PassSlice* tab, int ns, int nblocks, hipStream_t st) {
    if (ns <= 0 || nblocks <= 0) return hipSuccess;
    switch (len) {
#define RN_CASE(L)                                                                                         \
    case L:                                                                                                \
        switch (kind) {                                                                                    \
            case PK_A1:                                                                                    \
                hipLaunchKernelGGL((k_a1_multi<L, ray_threads(L)>), dim3(nblocks), dim3(ray_threads(L)),   \
                                   0, st, tab, ns);                                                        \
                break;                                                                                     \
            case PK_A3:                                                                                    \
                hipLaunchKernelGGL((k_a3_multi<L, col_threads(L)>), dim3(nblocks), dim3(col_threads(L)),   \
                                   0, st, tab, ns);                                                        \
                break;                                                                                     \
            case PK_A4:                                                                                    \
                hipLaunchKernelGGL((k_a4_multi<L, row_threads(L)>), dim3(nblocks), dim3(row_threads(L)),   \
                                   0, st, tab, ns);                                                        \
                break;                                                                                     \
            default:                                                                                       \
                return hipErrorInvalidValue;                                                               \
        }                                                                                                  \
        break;
        RN_FOR_LENGTHS(RN_CASE)
#undef RN_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int W, int T>
static hipError_t launch_a2m_wt(const GridLaunch& g, const GridSlice* gs, bool reduce, hipStream_t st) {
    if (!reduce) {
        if (g.n_items == 0) return hipSuccess;
        hipLaunchKernelGGL((k_a2_multi<W, T>), dim3(g.n_items), dim3(A2_NT), 0, st, g.items, gs, g.kbc);
    } else {
        if (g.n_splits == 0) return hipSuccess;
        hipLaunchKernelGGL((k_a2r_multi<T>), dim3(g.n_splits, (A2_GX * T * T + 255) / 256), dim3(256), 0, st,
                           g.splits, gs);
    }
    return hipGetLastError();
}

template <int W>
static hipError_t launch_a2m_w(const GridLaunch& g, const GridSlice* gs, bool reduce, hipStream_t st) {
    switch (g.T) {
        case 8: return launch_a2m_wt<W, 8>(g, gs, reduce, st);
        case 16: return launch_a2m_wt<W, 16>(g, gs, reduce, st);
        case 32: return launch_a2m_wt<W, 32>(g, gs, reduce, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_a2_grid(const GridLaunch& g, const GridSlice* gs, bool reduce, hipStream_t st) {
    switch (g.W) {
        case 4: return launch_a2m_w<4>(g, gs, reduce, st);
        case 6: return launch_a2m_w<6>(g, gs, reduce, st);
        case 8: return launch_a2m_w<8>(g, gs, reduce, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rn

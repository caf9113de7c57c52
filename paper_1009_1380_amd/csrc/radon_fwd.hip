// radon_fwd.hip - launchers of the forward path (F1 row FFT, F2 column FFT,
// F3 tiled polar interpolation, F4 ray inverse FFT), dispatched on the FFT
// length, kernel width and tile size: for one slice, and for every slice of
// an uneven batch (radon_multi.hpp).
#include "radon_internal.hpp"

namespace rn {

hipError_t launch_f1(const Plan& p, const float* img, hipStream_t st) {
    const dim3 grid(row_blocks(p.n));
    switch (p.n) {
#define RN_CASE(L)                                                                             \
    case L: {                                                                                  \
        constexpr int NT = row_threads(L);                                                   \
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
        constexpr int NT = col_threads(L);                                                   \
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

template <int W, int T>
static hipError_t launch_f3_wt(const Plan& p, hipStream_t st) {
    if (p.n_fitems == 0) return hipSuccess;
    hipLaunchKernelGGL((k_f3_tiles<W, T, 512>), dim3(p.f3_grid), dim3(512), 0, st, p.fitems, p.n_fitems,
                       p.recs, p.grid, p.kbc, p.Xr, p.G);
    return hipGetLastError();
}

template <int W, int T>
static int f3_occupancy() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_f3_tiles<W, T, 512>, 512, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

template <int W>
static int f3_occupancy_w(int T) {
    switch (T) {
        case 8: return f3_occupancy<W, 8>();
        case 16: return f3_occupancy<W, 16>();
        case 32: return f3_occupancy<W, 32>();
        default: return 1;
    }
}

int f3_blocks_per_cu(int W, int T) {
    switch (W) {
        case 4: return f3_occupancy_w<4>(T);
        case 6: return f3_occupancy_w<6>(T);
        case 8: return f3_occupancy_w<8>(T);
        default: return 1;
    }
}

template <int W>
static hipError_t launch_f3_w(const Plan& p, hipStream_t st) {
    switch (p.T) {
        case 8: return launch_f3_wt<W, 8>(p, st);
        case 16: return launch_f3_wt<W, 16>(p, st);
        case 32: return launch_f3_wt<W, 32>(p, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_f3(const Plan& p, hipStream_t st) {
    switch (p.W) {
        case 4: return launch_f3_w<4>(p, st);
        case 6: return launch_f3_w<6>(p, st);
        case 8: return launch_f3_w<8>(p, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_f4(const Plan& p, float* sino, hipStream_t st) {
    const dim3 grid((p.n_views + 1) / 2);
    switch (p.n_det) {
#define RN_CASE(L)                                                                             \
    case L: {                                                                                  \
        constexpr int NT = ray_threads(L);                                                     \
        hipLaunchKernelGGL((k_f4_rays<L, NT>), grid, dim3(NT), 0, st, p.Xr, sino, p.tw_N,       \
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

// ---------------------------------------------------------------- batches

hipError_t launch_pass_fwd(PassKind kind, int len, const PassSlice* tab, int ns, int nblocks, hipStream_t st) {
    if (ns <= 0 || nblocks <= 0) return hipSuccess;
    switch (len) {
#define RN_CASE(L)                                                                                         \
    case L:                                                                                                \
        switch (kind) {                                                                                    \
            case PK_F1:                                                                                    \
                hipLaunchKernelGGL((k_f1_multi<L, row_threads(L)>), dim3(nblocks), dim3(row_threads(L)),   \
                                   0, st, tab, ns);                                                        \
                break;                                                                                     \
            case PK_F2:                                                                                    \
                hipLaunchKernelGGL((k_f2_multi<L, col_threads(L)>), dim3(nblocks), dim3(col_threads(L)),   \
                                   0, st, tab, ns);                                                        \
                break;                                                                                     \
            case PK_F4:                                                                                    \
                hipLaunchKernelGGL((k_f4_multi<L, ray_threads(L)>), dim3(nblocks), dim3(ray_threads(L)),   \
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

hipError_t launch_pass(PassKind kind, int len, const PassSlice* tab, int ns, int nblocks, hipStream_t st) {
    if (kind == PK_F1 || kind == PK_F2 || kind == PK_F4) return launch_pass_fwd(kind, len, tab, ns, nblocks, st);
    return launch_pass_adj(kind, len, tab, ns, nblocks, st);
}

PassSlice pass_slice_of(const Plan& p, PassKind kind, const void* in, void* out) {
    PassSlice e{};
    e.block0 = 0;
    e.n_views = p.n_views;
    e.psi_inv = p.psi_inv;
    e.shift = p.shift_n;
    e.wq = nullptr;
    switch (kind) {
        case PK_F1: e.nblk = row_blocks(p.n); e.in = in; e.out = p.T1; e.tw = p.tw_n; break;
        case PK_F2: e.nblk = p.n + 1; e.in = p.T1; e.out = p.grid; e.tw = p.tw_n; break;
        case PK_F4: e.nblk = (p.n_views + 1) / 2; e.in = p.Xr; e.out = out; e.tw = p.tw_N; break;
        case PK_A1: e.nblk = (p.n_views + 1) / 2; e.in = in; e.out = p.Yh; e.tw = p.tw_N; break;
        case PK_A3: e.nblk = p.n + 1; e.in = p.grid; e.out = p.T1; e.tw = p.tw_n; break;
        case PK_A4: e.nblk = row_blocks(p.n); e.in = p.T1; e.out = out; e.tw = p.tw_n; break;
    }
    return e;
}

GridSlice grid_slice_of(const Plan& p) { return GridSlice{p.recs, p.grid, p.Xr, p.Yh, p.partials, p.G, 0}; }

template <int W, int T>
static hipError_t launch_f3m_wt(const GridLaunch& g, const GridSlice* gs, hipStream_t st) {
    if (g.n_fitems == 0) return hipSuccess;
    hipLaunchKernelGGL((k_f3_multi<W, T, 512>), dim3(g.f3_grid), dim3(512), 0, st, g.fitems, g.n_fitems, gs, g.kbc);
    return hipGetLastError();
}

template <int W>
static hipError_t launch_f3m_w(const GridLaunch& g, const GridSlice* gs, hipStream_t st) {
    switch (g.T) {
        case 8: return launch_f3m_wt<W, 8>(g, gs, st);
        case 16: return launch_f3m_wt<W, 16>(g, gs, st);
        case 32: return launch_f3m_wt<W, 32>(g, gs, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_f3_grid(const GridLaunch& g, const GridSlice* gs, hipStream_t st) {
    switch (g.W) {
        case 4: return launch_f3m_w<4>(g, gs, st);
        case 6: return launch_f3m_w<6>(g, gs, st);
        case 8: return launch_f3m_w<8>(g, gs, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rn

// radon_multi.hpp - kernels of uneven-slice batches: one launch runs the same
// pass for every slice of a batch.
//
// Slices are reconstructed independently (the paper images volumes slice by
// slice), and a batch mixes sizes and view counts. The row and column
// transforms are compiled per FFT length, so one launch covers every slice of
// one length: a table maps the launch's blocks to slices (first block and
// block count of each), and each block runs the single-slice body on its
// slice's buffers with its slice-local block index. The gridding passes are
// compiled per kernel width and tile size, so one launch covers every slice of
// one (W, T): the work items of all those slices form one list, longest
// first, each item naming its slice, and the kernels drain it (the forward
// interpolation persistently, the spreading one item per workgroup). Every
// item and block does exactly the work it does in a single-slice launch, so
// results are bitwise those of per-slice calls: the bodies are shared with the
// single-slice kernels, and the library is built without floating-point
// contraction, so every operation rounds the same way in either kernel.
#pragma once

#include "radon_kernels.hpp"

namespace rn {

// One slice of a transform-pass launch.
struct PassSlice {
    int block0;             // first block of the slice in the launch
    int nblk;               // blocks of the slice
    int n_views;
    int pad;
    const void* in;         // the pass's input (image, T1, grid, Xr or sinogram)
    void* out;              // its output
    const float* psi_inv;   // 1/psi1, n
    const float2* shift;    // e^{-i pi (i - n/2)/n}, n
    const float2* tw;       // twiddles of the pass's FFT length
    const float* wq;        // ray weights of the filtered adjoint, or null
};

// Slice of block b: the last entry whose first block is <= b (binary search).
__device__ __forceinline__ int pass_slice(const PassSlice* __restrict__ tab, int ns, int b) {
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int NL, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(row_waves(NL)))) void k_f1_multi(
    const PassSlice* __restrict__ tab, int ns) {
    const PassSlice e = tab[pass_slice(tab, ns, blockIdx.x)];
    f1_body<NL, NT>(blockIdx.x - e.block0, e.nblk, (const float*)e.in, (float2*)e.out, e.psi_inv, e.shift, e.tw);
}

template <int NL, int NT>
__global__ __launch_bounds__(NT) void k_f2_multi(const PassSlice* __restrict__ tab, int ns) {
    const PassSlice e = tab[pass_slice(tab, ns, blockIdx.x)];
    f2_body<NL, NT>(blockIdx.x - e.block0, e.nblk, (const float2*)e.in, (float2*)e.out, e.shift, e.tw);
}

template <int ND, int NT>
__global__ __launch_bounds__(NT) void k_f4_multi(const PassSlice* __restrict__ tab, int ns) {
    const PassSlice e = tab[pass_slice(tab, ns, blockIdx.x)];
    f4_body<ND, NT>(blockIdx.x - e.block0, e.nblk, (const float2*)e.in, (float*)e.out, e.tw, e.n_views);
}

template <int ND, int NT>
__global__ __launch_bounds__(NT) void k_a1_multi(const PassSlice* __restrict__ tab, int ns) {
    const PassSlice e = tab[pass_slice(tab, ns, blockIdx.x)];
    a1_body<ND, NT>(blockIdx.x - e.block0, e.nblk, (const float*)e.in, (float2*)e.out, e.tw, e.wq, e.n_views);
}

template <int NL, int NT>
__global__ __launch_bounds__(NT) void k_a3_multi(const PassSlice* __restrict__ tab, int ns) {
    const PassSlice e = tab[pass_slice(tab, ns, blockIdx.x)];
    a3_body<NL, NT>(blockIdx.x - e.block0, e.nblk, (const float2*)e.in, (float2*)e.out, e.shift, e.tw);
}

template <int NL, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(row_waves(NL)))) void k_a4_multi(
    const PassSlice* __restrict__ tab, int ns) {
    const PassSlice e = tab[pass_slice(tab, ns, blockIdx.x)];
    a4_body<NL, NT>(blockIdx.x - e.block0, e.nblk, (const float2*)e.in, (float*)e.out, e.psi_inv, e.shift, e.tw);
}

// The gridding buffers of one slice.
struct GridSlice {
    const SampleRec* recs;
    float2* grid;
    float2* Xr;          // forward: interpolated ray spectra
    const float2* Yh;    // adjoint: ray spectra to spread
    float2* partials;    // adjoint: partial strips of split strips
    int G;
    int pad;
};

// Forward interpolation over one list of items from many slices (all with
// kernel width W and tile T; their Kaiser-Bessel tables are the same).
template <int W, int T, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(W <= 6 ? RN_F3_WPE : 1))) void k_f3_multi(
    const F3Item* __restrict__ items, int n_items, const GridSlice* __restrict__ gs, const float4* __restrict__ kbc) {
    constexpr int PP = (2 * T + W - 1) * (2 * T + W - 1);
    constexpr int NKB = (W / 2) * KB_S;
    __shared__ float2 tile[PP];
    __shared__ float4 kbt[NKB];
    const int tid = threadIdx.x;
    for (int e = tid; e < NKB; e += NT) kbt[e] = kbc[e];
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
        const F3Item it = items[i];
        const GridSlice g = gs[it.plan];
        f3_item<W, T, NT>(it, g.recs, g.grid, g.Xr, g.G, tile, kbt, tid);
    }
}

template <int W, int T>
__global__ __launch_bounds__(A2_NT) __attribute__((amdgpu_waves_per_eu(W <= 6 ? RN_A2_WPE : 1))) void k_a2_multi(
    const TileItem* __restrict__ items, const GridSlice* __restrict__ gs, const float4* __restrict__ kbc) {
    const TileItem it = items[blockIdx.x];
    const GridSlice g = gs[it.plan];
    a2_item<W, T>(it, g.recs, g.Yh, kbc, g.grid, g.partials, g.G);
}

template <int T>
__global__ __launch_bounds__(256) void k_a2r_multi(const SplitTile* __restrict__ splits,
                                                  const GridSlice* __restrict__ gs) {
    const SplitTile sp = splits[blockIdx.x];
    const GridSlice g = gs[sp.plan];
    a2r_body<T>(sp, blockIdx.y, g.partials, g.grid, g.G);
}

}  // namespace rn

// radon_sort.hpp - footprint-tile keys and a stable LSD radix sort (gfx950).
//
// The paper balances the gridding work by putting samples into bins that
// each get one thread block (section "fast radon transform", paragraph 4).
// Here the bins are uniform T x T tiles of the centred oversampled grid,
// keyed by the tile of each sample's footprint origin:
//   o = (floor(u) - W/2 + 1 + G/2) mod G,  key = (o_v div T)(G/T) + (o_u div T),
// refined by the footprint's edge class, and the samples are stably sorted by
// the refined key (ties in increasing sample id).
// All integer work: the result is bit-exact and deterministic.
#pragma once

#include <hip/hip_runtime.h>

#include "radon_kernels.hpp"

namespace rn {

constexpr int SORT_NT = 256;
constexpr int SORT_IPT = 16;
constexpr int SORT_TILE = SORT_NT * SORT_IPT;   // elements per block
constexpr int SORT_RADIX = 16;                  // 4-bit digits

// Refined key of every sample: 4 * (tile of the footprint origin) + edge
// class (0: footprint inside the tile, 1: crosses the u edge only, 2: both,
// 3: the v edge only). Sample ids 0..M-1 are the polar samples
// j = a*N + q + N/2; ids M..M+n_views-1 are the mirrored Nyquist samples.
__global__ __launch_bounds__(256) void k_sample_keys(const double2* __restrict__ cs, int* __restrict__ keys,
                                                    int* __restrict__ ids, int n_views, int ND, int G,
                                                    int W, int T) {
    const int M = n_views * ND;
    const int total = M + n_views;
    const int v = blockIdx.x * 256 + threadIdx.x;
    if (v >= total) return;
    int a, q;
    decode_sample(v, M, ND, a, q);
    const double2 c = cs[a];
    const SampleGeom g = sample_geom(c.x, c.y, q, G, ND);
    const int ou = footprint_origin(g.bu, W, G);
    const int ov = footprint_origin(g.bv, W, G);
    const bool cu = (ou % T) + W - 1 >= T;
    const bool cv = (ov % T) + W - 1 >= T;
    const int cls = (cu && cv) ? 2 : (cu ? 1 : (cv ? 3 : 0));
    keys[v] = 4 * ((ov / T) * (G / T) + (ou / T)) + cls;
    ids[v] = v;
}

// Records of the sorted samples (see SampleRec): geometry, ray-spectrum index
// and the forward-evaluation flag, from the same float64 geometry as the keys.
__global__ __launch_bounds__(256) void k_sample_recs(const int* __restrict__ perm, const double2* __restrict__ cs,
                                                    SampleRec* __restrict__ recs, int total, int n_views, int ND,
                                                    int G, int W, int T) {
    const int pos = blockIdx.x * 256 + threadIdx.x;
    if (pos >= total) return;
    const int M = n_views * ND;
    const int HQ = ND / 2 + 1;
    const int ntl = G / T;
    int a, q;
    decode_sample(perm[pos], M, ND, a, q);
    const double2 c = cs[a];
    const SampleGeom g = sample_geom(c.x, c.y, q, G, ND);
    int idx, flags = 0;
    bool eval = true;
    if (q >= 0 && q < ND / 2) {
        idx = a * HQ + q;
    } else if (q == -ND / 2) {
        idx = a * HQ + ND / 2;
    } else {
        // q in (-N/2, 0), or the mirrored Nyquist sample (q = +N/2): the forward
        // evaluates it only if its partner's origin is not in a forward column
        const bool mirror = (q == ND / 2);
        const int qc = mirror ? -ND / 2 : -q;
        const SampleGeom gc = sample_geom(c.x, c.y, qc, G, ND);
        eval = !forward_column(footprint_origin(gc.bu, W, G) / T, ntl);
        idx = mirror ? a * HQ + ND / 2 : a * HQ - q;
        flags = mirror ? REC_MIRROR : REC_CONJ;
    }
    // the outer footprint points m = floor - W/2 + 1 and floor + W/2 are inside
    // the support iff |coordinate - m| < W/2, decided in float64
    const double hw = 0.5 * W;
    int edges = 0;
    if (!(fabs(g.u - (double)(g.bu - W / 2 + 1)) < hw)) edges |= REC_U_NEAR_OUT;
    if (!(fabs(g.u - (double)(g.bu + W / 2)) < hw)) edges |= REC_U_FAR_OUT;
    if (!(fabs(g.v - (double)(g.bv - W / 2 + 1)) < hw)) edges |= REC_V_NEAR_OUT;
    if (!(fabs(g.v - (double)(g.bv + W / 2)) < hw)) edges |= REC_V_FAR_OUT;
    int4 r;
    r.x = footprint_origin(g.bu, W, G) | (footprint_origin(g.bv, W, G) << 16) | edges;
    r.y = __float_as_int(g.fu);
    r.z = __float_as_int(g.fv);
    r.w = (int)((unsigned)idx | (unsigned)flags | (eval ? REC_F3 : 0u));
    reinterpret_cast<int4*>(recs)[pos] = r;
}

// Per-block digit counts, stored digit-major: hist[d * nblocks + b].
__global__ __launch_bounds__(SORT_NT) void k_sort_hist(const int* __restrict__ keys, int n, int shift,
                                                      int* __restrict__ hist, int nblocks) {
    __shared__ int cnt[SORT_RADIX];
    if (threadIdx.x < SORT_RADIX) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * SORT_TILE;
    for (int i = threadIdx.x; i < SORT_TILE; i += SORT_NT) {
        const int e = base + i;
        if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & (SORT_RADIX - 1)], 1);
    }
    __syncthreads();
    if (threadIdx.x < SORT_RADIX) hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// In-place exclusive scan of `total` ints by one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_exclusive_scan(int* __restrict__ data, int total) {
    __shared__ int sums[1024];
    const int tid = threadIdx.x;
    const int per = (total + 1023) / 1024;
    const int lo = tid * per;
    const int hi = min(total, lo + per);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += data[i];
    sums[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = (tid >= off) ? sums[tid - off] : 0;
        __syncthreads();
        sums[tid] += v;
        __syncthreads();
    }
    int run = (tid == 0) ? 0 : sums[tid - 1];
    for (int i = lo; i < hi; ++i) {
        const int x = data[i];
        data[i] = run;
        run += x;
    }
}

// Stable scatter: thread t owns elements [b*TILE + t*IPT, +IPT) in order, so
// the rank of an element is (scanned block base of its digit) + (count of the
// same digit in earlier threads of the block) + (earlier in the same thread).
__global__ __launch_bounds__(SORT_NT) void k_sort_scatter(const int* __restrict__ kin, const int* __restrict__ vin,
                                                         int* __restrict__ kout, int* __restrict__ vout,
                                                         int n, int shift, const int* __restrict__ hist,
                                                         int nblocks) {
    __shared__ int cnt[SORT_RADIX * SORT_NT];   // [digit][thread]
    __shared__ int tsum[SORT_NT];
    __shared__ int dstart[SORT_RADIX];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    for (int d = 0; d < SORT_RADIX; ++d) cnt[d * SORT_NT + tid] = 0;
    const int e0 = b * SORT_TILE + tid * SORT_IPT;
    int kv[SORT_IPT];
#pragma unroll
    for (int i = 0; i < SORT_IPT; ++i) {
        const int e = e0 + i;
        kv[i] = (e < n) ? kin[e] : -1;
        if (e < n) cnt[((kv[i] >> shift) & (SORT_RADIX - 1)) * SORT_NT + tid] += 1;
    }
    __syncthreads();
    // exclusive scan over the 4096 counters in [digit][thread] order:
    // thread t scans entries t*16 .. t*16+15
    int local[SORT_RADIX];
    int s = 0;
#pragma unroll
    for (int i = 0; i < SORT_RADIX; ++i) {
        local[i] = cnt[tid * SORT_RADIX + i];
        s += local[i];
    }
    tsum[tid] = s;
    __syncthreads();
    for (int off = 1; off < SORT_NT; off <<= 1) {
        const int v = (tid >= off) ? tsum[tid - off] : 0;
        __syncthreads();
        tsum[tid] += v;
        __syncthreads();
    }
    int run = (tid == 0) ? 0 : tsum[tid - 1];
#pragma unroll
    for (int i = 0; i < SORT_RADIX; ++i) {
        const int x = local[i];
        cnt[tid * SORT_RADIX + i] = run;
        run += x;
    }
    __syncthreads();
    // the first entry of digit d (flat index d*NT) holds the block-local start
    // of digit d; keep a copy, since thread 0 advances that entry below
    if (tid < SORT_RADIX) dstart[tid] = cnt[tid * SORT_NT];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SORT_IPT; ++i) {
        const int e = e0 + i;
        if (e < n) {
            const int d = (kv[i] >> shift) & (SORT_RADIX - 1);
            const int slot = d * SORT_NT + tid;
            const int within = cnt[slot] - dstart[d];
            const int pos = hist[d * nblocks + b] + within;
            cnt[slot] += 1;
            kout[pos] = kv[i];
            vout[pos] = vin[e];
        }
    }
}

// offsets[b] = first position whose key >= b (b = 0..n_bins), by binary search.
__global__ __launch_bounds__(256) void k_bin_offsets(const int* __restrict__ sorted_keys, int n,
                                                    int* __restrict__ offsets, int n_bins) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b > n_bins) return;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sorted_keys[mid] < b) lo = mid + 1; else hi = mid;
    }
    offsets[b] = lo;
}

}  // namespace rn

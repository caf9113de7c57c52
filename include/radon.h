/*
 * radon.h - C ABI of the MI355X (gfx950) Radon NUFFT library.
 *
 * The library applies the 2D Radon transform and its exact adjoint through
 * the Fourier slice theorem, as in Maia et al., "Compressive Phase Contrast
 * Tomography", section "fast radon transform": a 2D FFT of the image on a
 * regular (oversampled) grid, interpolation of that transform onto a polar
 * grid by gridding with a Kaiser-Bessel kernel, and 1D inverse FFTs along
 * every radial line; the adjoint ("inverse gridding" in the abstract) runs
 * the steps in reverse with a deterministic, binned spreading step (no
 * floating-point atomics). The solver of the paper's L1 problem (section
 * "INTRODUCTION", displayed problem) needs exactly these two maps.
 *
 * Conventions (all calls):
 *   image    n x n float32, row-major; pixel (i, j) is the point
 *            (px, py) = (j - n/2, i - n/2), unit spacing.
 *   sinogram n_views x n_det float32, row-major; bin d is the detector
 *            offset s = d - n_det/2; view a has direction
 *            (cos angles[a], sin angles[a]); angle 0 projects along y.
 *   forward  y[a,d] = Re((1/N) sum_q X~_a[q] exp(2 pi i q s_d / N)), where
 *            X~_a[q] is the Kaiser-Bessel gridding estimate of the image's
 *            Fourier transform at k = (q/N)(cos, sin), q = -N/2..N/2-1.
 *   adjoint  exact transpose of the forward in the real inner product
 *            (no ramp filter, no 1/n_views scaling).
 *   Device pointers are plain HIP device addresses of the device that was
 *   current when the plan was made; that device must be current for every
 *   call on the plan. `stream` is a hipStream_t (NULL = default stream).
 *   Calls enqueue work on the stream and never synchronise the host.
 *   Inputs are never modified; outputs are fully overwritten; input and
 *   output must not overlap.
 *
 * Errors: nothing aborts or throws across this interface. Argument errors
 * return synchronously before any launch; launch failures return
 * RADON_ERR_DEVICE; asynchronous device faults surface at the caller's next
 * synchronisation. radon_last_error() gives a thread-local message.
 *
 * Thread safety: a plan owns one workspace, so one plan may be used by one
 * stream at a time. Distinct plans are independent.
 */
#ifndef RADON_H
#define RADON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct radon_plan_s* radon_plan_t;

typedef enum {
    RADON_OK = 0,
    RADON_ERR_INVALID = 1,      /* bad argument (NULL pointer, bad size)          */
    RADON_ERR_UNSUPPORTED = 2,  /* valid but outside what the kernels implement   */
    RADON_ERR_OOM = 3,          /* device allocation failed                       */
    RADON_ERR_DEVICE = 4        /* HIP runtime or launch error                    */
} radon_status_t;

/*
 * Build a plan for n x n images, n_views angles (host array of float64
 * radians, any order, copied) and n_det detector bins, oversampling sigma and
 * Kaiser-Bessel width W (section "fast radon transform", paragraphs 1-4).
 *
 * Requirements: n and n_det even and >= 8; sigma * n an integer equal to
 * 2 n (only sigma = 2 is implemented: RADON_ERR_UNSUPPORTED otherwise);
 * W in {4, 6, 8}; n and n_det in the supported FFT lengths (2^a 3^b 5^c,
 * listed by radon_supported_length); n_views >= 1.
 *
 * The plan computes per-view cos/sin in float64 on the host, builds the
 * Kaiser-Bessel table and deapodization factors in float64 (rounded once
 * to float32), sorts the polar samples by footprint tile on the device, and
 * allocates its workspace. It synchronises the device before returning.
 * On failure *out is set to NULL and nothing stays allocated. Release with
 * radon_plan_destroy.
 * Test hook: with the environment variable RADON_TEST_FAIL_ALLOC=k, the k-th
 * device allocation made while building a plan (counting from 1) fails as if
 * the device were out of memory (RADON_ERR_OOM).
 */
radon_status_t radon_plan(radon_plan_t* out, int n, const double* angles, int n_views,
                          int n_det, double sigma, int W);

/*
 * Work decomposition of a plan (section "fast radon transform", paragraph 4:
 * the bins that balance the gridding work, read as uniform tiles):
 *   tile      side T of the square bins: 8, 16 or 32 with T dividing G/2 and
 *             T >= W; 0 = the largest that fits.
 *   a2_chunk  most visits in one spreading work item, 64..512; 0 = 512.
 *   f3_chunk  most samples in one forward-interpolation work item,
 *             256..65536; 0 = 2048.
 * Results do not depend on the choice beyond float32 rounding.
 */
typedef struct {
    int tile;
    int a2_chunk;
    int f3_chunk;
} radon_tuning;

/* radon_plan with an explicit work decomposition (tuning may be NULL: the
 * defaults). Out-of-range tuning values return RADON_ERR_INVALID; a tile that
 * does not fit G returns RADON_ERR_UNSUPPORTED. */
radon_status_t radon_plan_tuned(radon_plan_t* out, int n, const double* angles, int n_views,
                                int n_det, double sigma, int W, const radon_tuning* tuning);

/* The work decomposition a plan uses (defaults resolved). */
radon_status_t radon_plan_tuning(radon_plan_t plan, radon_tuning* out);

/*
 * Autotuner: for the given geometry, time `repeats` forward + adjoint pairs
 * (after one untimed pair) of candidate decompositions on `stream`, by
 * coordinate search from the defaults: the tile size over {8, 16, 32} (those
 * that fit), then a2_chunk over {256, 512}, then f3_chunk over {1024, 2048,
 * 4096}. A candidate replaces the best so far only when it is faster by more
 * than the run-to-run spread: the two are timed three times, interleaved, and
 * the candidate's least time must be 3% below the best's. Returns the chosen
 * decomposition in *best with its least time per pair in *best_ms;
 * *default_ms (may be NULL) gets the time of the default decomposition. Inputs are generated on the device; the
 * plans and buffers are released before returning. Synchronises the stream.
 * Errors in the geometry are reported as by radon_plan.
 */
radon_status_t radon_autotune(int n, const double* angles, int n_views, int n_det, double sigma, int W,
                              int repeats, radon_tuning* best, double* best_ms, double* default_ms,
                              void* stream);

/* Forward Radon transform: img_dev (n*n float32) -> sino_dev (n_views*n_det float32). */
radon_status_t radon_forward(radon_plan_t plan, const float* img_dev, float* sino_dev,
                             void* stream);

/* Adjoint Radon transform: sino_dev (n_views*n_det float32) -> img_dev (n*n float32). */
radon_status_t radon_adjoint(radon_plan_t plan, const float* sino_dev, float* img_dev,
                             void* stream);

/*
 * Filtered adjoint (filtered back-projection through the Fourier slice
 * theorem): the adjoint with every ray spectrum weighted by the ramp
 * w_q = (pi/n_views) H(q), H the DFT of the band-limited spatial ramp kernel
 * h[0] = 1/4, h[k] = -1/(pi k)^2 for odd k, 0 for even k != 0, |k| < N/2.
 * For views uniform in [0, pi) it approximately inverts radon_forward inside
 * the inscribed circle. Read here as the "standard tomographic processing"
 * of the paper's introduction. sino_dev (n_views*n_det) -> img_dev (n*n).
 */
radon_status_t radon_fbp(radon_plan_t plan, const float* sino_dev, float* img_dev, void* stream);

/* batch slices that share the plan's geometry, back to back on the stream:
 * imgs_dev is batch*n*n float32, sinos_dev is batch*n_views*n_det float32. */
radon_status_t radon_forward_batched(radon_plan_t plan, int batch, const float* imgs_dev,
                                     float* sinos_dev, void* stream);
radon_status_t radon_adjoint_batched(radon_plan_t plan, int batch, const float* sinos_dev,
                                     float* imgs_dev, void* stream);

/*
 * Batches of uneven slices: `count` plans of any sizes (distinct plan objects,
 * each used by this batch only while it runs) applied together, each pass of
 * the path once for all slices (the paper balances the gridding over thread
 * blocks by bins, section "fast radon transform", paragraph 4; here the bins
 * of all slices share one work list). Per direction the batch launches one
 * kernel per pass and FFT length for the transforms and one per (kernel
 * width, tile size) for the gridding, whose items from every slice are
 * drained longest first. The first call for a given set of device pointers
 * records these launches into one HIP graph (the launches of different
 * lengths on up to `n_branches` parallel branches, 1..16); later calls with
 * the same pointers replay it with one graph launch on `stream`. New pointers
 * record a new graph. Every slice's result equals its per-slice call bit for
 * bit. imgs_dev[i] is plan i's n*n image, sinos_dev[i] its n_views*n_det
 * sinogram. Profiling must be off on every plan. The batch keeps the plan
 * handles: destroy it before them.
 */
typedef struct radon_batch_s* radon_batch_t;
radon_status_t radon_batch_create(radon_batch_t* out, int count, const radon_plan_t* plans, int n_branches);
radon_status_t radon_batch_forward(radon_batch_t batch, const float* const* imgs_dev, float* const* sinos_dev,
                                   void* stream);
radon_status_t radon_batch_adjoint(radon_batch_t batch, const float* const* sinos_dev, float* const* imgs_dev,
                                   void* stream);
/* Number of graphs recorded so far (a test hook: replays do not add one). */
int radon_batch_graphs_recorded(radon_batch_t batch);
void radon_batch_destroy(radon_batch_t batch);   /* NULL-safe */

/*
 * Test hook: copy the plan's stable sample sort to host memory. The sorted
 * samples are the n_views*n_det polar samples j = a*n_det + q + n_det/2
 * followed by n_views mirrored Nyquist samples (view a at q = +n_det/2).
 * Bins are uniform T x T tiles of the oversampled grid (section "fast radon
 * transform", paragraph 4, read as uniform tiles) keyed by the tile of the
 * footprint origin o = (floor(u) - W/2 + 1 + G/2) mod G,
 * key = (o_v div T)*(G/T) + (o_u div T), refined by the footprint's edge
 * class c (0 inside, 1 crosses the u edge, 2 both, 3 the v edge): the sort is
 * stable by 4*key + c. perm gets the sorted sample ids (perm_cap >=
 * n_samples), offsets the 4*n_bins+1 class starts. Either pointer may be
 * NULL. Sizes come from radon_plan_info.
 */
radon_status_t radon_plan_sort_indices(radon_plan_t plan, int32_t* perm_host, int64_t perm_cap,
                                       int32_t* offsets_host, int64_t offsets_cap);

/*
 * Plan facts for tests and benchmarks. info[k] (k < cap) receives:
 *  0 n, 1 n_views, 2 n_det, 3 W, 4 G, 5 tile T, 6 sorted samples,
 *  7 bins (tiles), 8 spreading work items, 9 partial slots, 10 device bytes,
 *  11 forward interpolation work items.
 */
radon_status_t radon_plan_info(radon_plan_t plan, int64_t* info, int cap);

/* Device memory owned by the plan, in bytes (0 for NULL). */
size_t radon_plan_device_bytes(radon_plan_t plan);

/* Free the plan and its device memory. NULL-safe. Synchronises the device. */
void radon_plan_destroy(radon_plan_t plan);

/* 1 if len is a supported FFT length (image size or detector count), else 0. */
int radon_supported_length(int len);

/* Static name of a status code. */
const char* radon_status_string(radon_status_t status);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* radon_last_error(void);

/*
 * Stage timing. With profiling on, every kernel launch of forward/adjoint is
 * bracketed by HIP events on the caller's stream; radon_plan_stage_times
 * synchronises on those events and returns, per stage, the accumulated
 * milliseconds and launch counts since profiling was switched on. Stage names
 * come from radon_stage_name(0 .. radon_stage_count()-1).
 */
radon_status_t radon_plan_set_profiling(radon_plan_t plan, int enable);
radon_status_t radon_plan_stage_times(radon_plan_t plan, double* ms, int64_t* counts, int cap);
int radon_stage_count(void);
const char* radon_stage_name(int stage);

/*
 * Test hooks that run parts of the path on the plan's workspace.
 * radon_debug_forward_grid: deapodize + zero-pad + 2D FFT of img_dev, then
 *   copy the half-plane grid to grid_dev: (G/2+1) x G complex64, element
 *   [mx][my] = Ghat at frequency (mx, my) (transposed: mx major).
 * radon_debug_adjoint_grid: ray FFTs + binned spreading of sino_dev, copy the
 *   Hermitian part of the spread grid, same layout, to grid_dev.
 */
radon_status_t radon_debug_forward_grid(radon_plan_t plan, const float* img_dev, float* grid_dev,
                                        void* stream);
radon_status_t radon_debug_adjoint_grid(radon_plan_t plan, const float* sino_dev, float* grid_dev,
                                        void* stream);

/*
 * Test hook for the batched LDS FFT: `batch` independent complex64 lines of
 * length len (in_dev, out_dev: batch*len complex64, may not alias), forward
 * (exp(-), inverse = 0) or unnormalised inverse (exp(+), inverse = 1).
 */
radon_status_t radon_fft_test(int len, int batch, int inverse, const float* in_dev,
                              float* out_dev, void* stream);

/*
 * Ring filter of the basis-pursuit problem (the paper's polynomial filter,
 * introduction): F y = y - 1 (x) (m - P3 m) with m[d] the mean over views of
 * y[., d] and P3 the least-squares projection onto cubic polynomials in the
 * detector coordinate. F is a symmetric projection. y_dev, out_dev:
 * n_views*n_det float32 (may alias). Synchronises the stream.
 */
radon_status_t radon_ring_filter(radon_plan_t plan, const float* y_dev, float* out_dev, void* stream);

/*
 * The ring filter for callers that cannot allocate device memory (code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operation and result as radon_ring_filter, with no allocation of
 * any kind. The cubic basis is the plan's own; the scratch of its three
 * kernels (column means, fitted ring, partial sums) is one file-scope device
 * array of 2 * RADON_RING_NOALLOC_MAX_DET + 4096 float64 values (96 KiB),
 * of which every GPU the library runs on holds its own copy until the
 * process ends. Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (several streams, several threads) race and must be
 * serialised by the caller. Stream-ordered; it does not synchronise the
 * stream. Errors: RADON_ERR_INVALID for NULL arguments or a plan made on
 * another device than the current one, RADON_ERR_UNSUPPORTED when the
 * plan's n_det exceeds RADON_RING_NOALLOC_MAX_DET, RADON_ERR_DEVICE when the
 * array's address cannot be found or a launch fails.
 */
#define RADON_RING_NOALLOC_MAX_DET 4096
radon_status_t radon_ring_filter_noalloc(radon_plan_t plan, const float* y_dev, float* out_dev, void* stream);

typedef struct {
    double sigma;      /* target ||F(A x - b)||_2, absolute, >= 0 (epsilon of the paper)  */
    double opt_tol;    /* relative tolerance of the root and of the duality gap (1e-4)    */
    double bp_tol;     /* basis-pursuit exit: ||r|| <= bp_tol ||F b|| (1e-6)              */
    double dec_tol;    /* stall test that triggers the Newton step on tau (1e-4)          */
    int max_iter;      /* iteration limit                                                  */
    int ring_filter;   /* 1: operator F A and data F b; 0: F = identity                    */
    int warm_start;    /* 1: x_dev holds the starting image (tau0: see radon_solve_bpdn);
                          0: x0 = 0                                                        */
    int fallback_iters;/* warm start: iterations without a new least | ||r|| - sigma |
                          before the cold solver takes over (<= 0: 100)                   */
} radon_solve_opts;

typedef struct {
    double rnorm;      /* final ||F(A x - b)||_2                                          */
    double tau;        /* final l1 radius                                                  */
    double x_l1;       /* ||x||_1 of the result                                            */
    double seconds;    /* host wall time of the call                                       */
    int iterations;    /* projected-gradient iterations                                    */
    int n_forward;     /* radon_forward applications                                       */
    int n_adjoint;     /* radon_adjoint applications                                       */
    int status;        /* 0 iteration limit, 1 basis-pursuit solution, 2 root found        */
    int fallback;      /* why a warm start was abandoned for a cold solve (RADON_FALLBACK_*) */
    int warm_iterations; /* iterations the abandoned warm run took (0 without fallback)    */
} radon_solve_stats;

/* Reasons a warm start is abandoned; the cold-started solver then runs with the
 * whole iteration budget, and its result is returned. */
enum {
    RADON_FALLBACK_NONE = 0,
    RADON_FALLBACK_NONFINITE = 1,        /* start, its l1 norm, residual or objective not finite  */
    RADON_FALLBACK_WORSE_THAN_ZERO = 2,  /* ||F(A x0 - b)|| >= ||F b||: x0 fits no better than 0 */
    RADON_FALLBACK_ITER_LIMIT = 3,       /* the warm run reached max_iter                          */
    RADON_FALLBACK_STALLED = 4           /* no new least | ||r|| - sigma | in fallback_iters iterations */
};

/*
 * Basis-pursuit denoising min ||x||_1 s.t. ||F(A x - b)||_2 <= sigma (the
 * paper's reconstruction problem, introduction), solved by SPGL1 root
 * finding on the Pareto curve (van den Berg & Friedlander 2008): Newton steps
 * on tau, each LASSO(tau) by spectral projected gradient with a non-monotone
 * line search and projection onto the l1 ball. b_dev: n_views*n_det float32
 * sinogram; x_dev: n*n float32, the start image when warm_start, overwritten
 * with the solution. Vectors are float32; all reductions are float64 in a
 * fixed order, so results are bitwise reproducible. The call allocates its
 * workspace, runs on `stream` and synchronises it (it reads a few float64
 * scalars per iteration); stats may be NULL.
 * Warm starts: the cold-started solver is the fallback. A warm run is
 * abandoned for a cold one (stats->fallback says why) when x0 or its first
 * residual is not finite, when x0 fits the data no better than zero, when it
 * reaches max_iter, or when fallback_iters iterations pass without a new
 * least distance | ||r|| - sigma |. Above the root of the Pareto curve a
 * point with ||r|| = sigma need not have the least l1 norm, so a warm run
 * starts at tau0 = min(||x0||_1, max(0, D)), D = (r.F b - sigma ||r||) /
 * ||A^T r||_inf for x0's residual r: by weak duality D <= tau*, and from
 * below the root the run proceeds as a cold one does (x0 is projected onto
 * the tau0 ball; D <= 0 makes it a cold start).
 * Errors: RADON_ERR_INVALID for NULL pointers, sigma < 0 or not finite,
 * opt_tol <= 0, max_iter < 1, a non-finite sinogram, or a cold run whose
 * objective becomes non-finite; RADON_ERR_OOM when the workspace cannot be
 * allocated; RADON_ERR_DEVICE for launch or copy failures.
 */
radon_status_t radon_solve_bpdn(radon_plan_t plan, const float* b_dev, float* x_dev, const radon_solve_opts* opts,
                                radon_solve_stats* stats, void* stream);

/*
 * Euclidean projection onto the l1 ball {||x||_1 <= tau}, the projection of
 * the solver's projected-gradient steps (SPGL1, introduction):
 * out = sign(v) max(|v| - lam, 0) with lam >= 0 the exact root of
 * sum max(|v_i| - lam, 0) = tau (lam = 0 when sum |v_i| <= tau; lam at or
 * above max |v_i| when tau = 0), located by a deterministic three-level
 * radix select on the bit patterns of |v_i|, so the result does not depend
 * on the launch order and lam is exact up to the final float64 sums.
 * v_dev, out_dev: n float32 values on the device (may alias), 16-byte
 * aligned, n a multiple of 4 (the solver's images are). A NaN or infinite
 * v_i gives lam = NaN and NaN outputs. lam_host (may be NULL) receives lam.
 * The call allocates its workspace, runs on `stream` and synchronises it.
 * Errors: RADON_ERR_INVALID for NULL buffers with n > 0, n < 0, n not a
 * multiple of 4, misaligned buffers, or tau negative or not finite;
 * RADON_ERR_UNSUPPORTED for n > 2^29; RADON_ERR_OOM when the workspace
 * cannot be allocated; RADON_ERR_DEVICE for launch failures.
 */
radon_status_t radon_project_l1(const float* v_dev, int64_t n, double tau, float* out_dev, double* lam_host,
                                void* stream);

/*
 * Learned warm start (an extension beyond the paper, which starts its solves
 * from zero): a 4-level convolutional encoder-decoder (3x3 convolutions,
 * 32-64-128-256 channels, ReLU, 2x2 average pooling, nearest upsampling, skip
 * additions, a final correction added to the input) with bfloat16
 * activations and float32 accumulation on the matrix cores, trained with
 * Adam (beta 0.9, 0.999) on mean squared error. It maps the filtered adjoint
 * (radon_fbp) of a sinogram to a start image for radon_solve_bpdn.
 * Images are batch x height x width float32 on the device (height, width
 * multiples of 8); the network's batch is fixed at creation. Initial weights:
 * He-normal from `seed` (host RNG), the last layer zero (the network starts as
 * the identity). All calls are stream-ordered; train_step synchronises the
 * stream when loss_host is not NULL.
 */
typedef struct radon_cnn_s* radon_cnn_t;
radon_status_t radon_cnn_create(radon_cnn_t* out, int batch, int height, int width, uint64_t seed);
void radon_cnn_destroy(radon_cnn_t net);   /* NULL-safe */
radon_status_t radon_cnn_forward(radon_cnn_t net, const float* in_dev, float* out_dev, void* stream);
/* One Adam step on a batch: pred_dev receives the forward output, *loss_host
 * (may be NULL) the mean squared error. */
radon_status_t radon_cnn_train_step(radon_cnn_t net, const float* in_dev, const float* target_dev, float lr,
                                    float* loss_host, float* pred_dev, void* stream);
/* Parameters in layer order (weights Cout x Cin x 3 x 3, then biases), host
 * float32 arrays of radon_cnn_param_count values; get_grads returns the last
 * training step's gradients (a test hook). */
int64_t radon_cnn_param_count(radon_cnn_t net);
radon_status_t radon_cnn_get_params(radon_cnn_t net, float* host, int64_t n);
radon_status_t radon_cnn_set_params(radon_cnn_t net, const float* host, int64_t n);
radon_status_t radon_cnn_get_grads(radon_cnn_t net, float* host, int64_t n);
/* Test hook: one 3x3 convolution (stride 1, zero padding 1) of bf16 tensors
 * in (B x Cin x H x W) with float32 weights w (Cout x Cin x 3 x 3) and bias
 * (may be NULL): out = [relu](conv + bias) [+ res], to out16 (bf16) and/or
 * out32; and, for an output gradient gout (bf16), the data gradient gin (bf16)
 * and the weight and bias gradients gw, gb (float32). NULL outputs are
 * skipped. Synchronises the stream. */
radon_status_t radon_cnn_conv_test(const uint16_t* in, const float* w, const float* bias, const uint16_t* res,
                                   uint16_t* out16, float* out32, int relu, const uint16_t* gout, uint16_t* gin,
                                   float* gw, float* gb, int B, int Cin, int Cout, int H, int W, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RADON_H */

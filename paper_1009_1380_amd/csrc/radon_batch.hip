// radon_batch.hip - uneven-slice batches recorded into HIP graphs, and the
// autotuner of a plan's work decomposition (include/radon.h).
//
// Parallel-beam tomography reconstructs every slice of a volume on its own
// (introduction: slices of the imaged samples), and slices differ in size and
// view count. A batch records the forward (or adjoint) kernel sequences of
// all its slices into one HIP graph: the slices are dealt round-robin over
// independent branches, so the small slices, whose kernels cannot fill the
// device alone, run side by side, and the whole batch is one graph launch
// instead of nine kernel launches per slice.
//
// The autotuner revisits the paper's load-balancing choice of bins (section
// "fast radon transform", paragraph 4: the work of a bin grows with its
// samples times its grid points) by measurement: it times each candidate
// decomposition of the same geometry on the device and keeps the fastest.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/radon.h"
#include "radon_internal.hpp"

namespace {

struct Recording {
    std::vector<const void*> in, out;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        in.clear();
        out.clear();
    }
};

radon_status_t errf(radon_status_t st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
radon_status_t errf(radon_status_t st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return rn::api_fail(st, buf);
}

// Uniform values in [-1, 1) from an integer hash of the index (inputs of the
// autotuner's timing runs; their values do not affect the timing).
__global__ void k_fill_hash(float* __restrict__ x, size_t n, unsigned seed) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        unsigned h = (unsigned)i * 0x9E3779B1u ^ seed;
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        h *= 0xC2B2AE35u;
        h ^= h >> 16;
        x[i] = (float)(h >> 8) * (2.0f / 16777216.0f) - 1.0f;
    }
}

}  // namespace

struct radon_batch_s {
    int device = 0;
    std::vector<radon_plan_t> plans;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;   // [0] fork, [1..] joins
    Recording fwd, adj;
    int recorded = 0;

    ~radon_batch_s() {
        fwd.release();
        adj.release();
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    }

    // Record every slice's sequence (forward or adjoint) into rec's graph.
    radon_status_t record(bool forward, const float* const* in, float* const* out, Recording& rec) {
        rec.release();
        const int nb = (int)streams.size();
        hipStream_t s0 = streams[0];
        if (hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return errf(RADON_ERR_DEVICE, "graph capture could not start");
        }
        radon_status_t st = RADON_OK;
        hipError_t e = hipEventRecord(events[0], s0);
        for (int b = 1; b < nb && e == hipSuccess; ++b) e = hipStreamWaitEvent(streams[b], events[0], 0);
        for (size_t i = 0; i < plans.size() && e == hipSuccess && st == RADON_OK; ++i) {
            rn::Plan& p = plans[i]->p;
            hipStream_t s = streams[i % nb];
            st = forward ? rn::api_run_forward(p, in[i], out[i], s) : rn::api_run_adjoint(p, in[i], out[i], s);
        }
        for (int b = 1; b < nb && e == hipSuccess; ++b) {
            e = hipEventRecord(events[b], streams[b]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s0, events[b], 0);
        }
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(s0, &g);
        if (st != RADON_OK || e != hipSuccess || ec != hipSuccess || !g) {
            (void)hipGetLastError();
            if (g) (void)hipGraphDestroy(g);
            return st != RADON_OK ? st : errf(RADON_ERR_DEVICE, "graph capture failed");
        }
        hipGraphExec_t x = nullptr;
        if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipGraphDestroy(g);
            return errf(RADON_ERR_DEVICE, "graph instantiation failed");
        }
        rec.graph = g;
        rec.exec = x;
        rec.in.assign(in, in + plans.size());
        rec.out.assign(out, out + plans.size());
        ++recorded;
        return RADON_OK;
    }

    radon_status_t run(bool forward, const float* const* in, float* const* out, void* stream) {
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev != device) {
            (void)hipGetLastError();
            return errf(RADON_ERR_INVALID, "the batch's device %d is not current", device);
        }
        if (!in || !out) return errf(RADON_ERR_INVALID, "NULL pointer array");
        for (size_t i = 0; i < plans.size(); ++i) {
            if (!in[i] || !out[i]) return errf(RADON_ERR_INVALID, "NULL buffer for slice %zu", i);
            if (plans[i]->p.profiling) return errf(RADON_ERR_INVALID, "profiling is on for slice %zu", i);
        }
        Recording& rec = forward ? fwd : adj;
        bool same = rec.exec != nullptr;
        for (size_t i = 0; same && i < plans.size(); ++i) same = rec.in[i] == in[i] && rec.out[i] == out[i];
        if (!same) {
            const radon_status_t st = record(forward, in, out, rec);
            if (st != RADON_OK) return st;
        }
        if (hipGraphLaunch(rec.exec, (hipStream_t)stream) != hipSuccess) {
            (void)hipGetLastError();
            return errf(RADON_ERR_DEVICE, "graph launch failed");
        }
        return rn::api_ok();
    }
};

extern "C" {

radon_status_t radon_batch_create(radon_batch_t* out, int count, const radon_plan_t* plans, int n_branches) {
    if (!out) return errf(RADON_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (count < 1 || !plans) return errf(RADON_ERR_INVALID, "count=%d must be >= 1 with a plan array", count);
    if (n_branches < 1 || n_branches > 16) return errf(RADON_ERR_INVALID, "n_branches=%d must be 1..16", n_branches);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return errf(RADON_ERR_DEVICE, "no HIP device");
    }
    std::vector<radon_plan_t> ps(plans, plans + count);
    for (int i = 0; i < count; ++i) {
        if (!ps[i]) return errf(RADON_ERR_INVALID, "plan %d is NULL", i);
        if (ps[i]->p.device != dev) return errf(RADON_ERR_INVALID, "plan %d lives on another device", i);
    }
    std::vector<radon_plan_t> sorted = ps;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return errf(RADON_ERR_INVALID, "a plan appears twice (each slice needs its own workspace)");
    radon_batch_s* b = new (std::nothrow) radon_batch_s();
    if (!b) return errf(RADON_ERR_OOM, "host allocation failed");
    b->device = dev;
    b->plans = ps;
    const int nb = std::min(n_branches, count);
    for (int i = 0; i < nb; ++i) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return errf(RADON_ERR_DEVICE, "stream creation failed");
        }
        b->streams.push_back(s);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return errf(RADON_ERR_DEVICE, "event creation failed");
        }
        b->events.push_back(e);
    }
    *out = b;
    return rn::api_ok();
}

radon_status_t radon_batch_forward(radon_batch_t batch, const float* const* imgs_dev, float* const* sinos_dev,
                                   void* stream) {
    if (!batch) return errf(RADON_ERR_INVALID, "batch is NULL");
    return batch->run(true, imgs_dev, sinos_dev, stream);
}

radon_status_t radon_batch_adjoint(radon_batch_t batch, const float* const* sinos_dev, float* const* imgs_dev,
                                   void* stream) {
    if (!batch) return errf(RADON_ERR_INVALID, "batch is NULL");
    return batch->run(false, sinos_dev, imgs_dev, stream);
}

int radon_batch_graphs_recorded(radon_batch_t batch) { return batch ? batch->recorded : -1; }

void radon_batch_destroy(radon_batch_t batch) { delete batch; }

radon_status_t radon_plan_tuning(radon_plan_t plan, radon_tuning* out) {
    if (!plan || !out) return errf(RADON_ERR_INVALID, "NULL argument");
    out->tile = plan->p.T;
    out->a2_chunk = plan->p.a2_chunk;
    out->f3_chunk = plan->p.f3_chunk;
    return rn::api_ok();
}

radon_status_t radon_autotune(int n, const double* angles, int n_views, int n_det, double sigma, int W, int repeats,
                              radon_tuning* best, double* best_ms, double* default_ms, void* stream) {
    if (!best || !best_ms) return errf(RADON_ERR_INVALID, "NULL output");
    if (repeats < 1 || repeats > 1000) return errf(RADON_ERR_INVALID, "repeats=%d must be 1..1000", repeats);
    hipStream_t st = (hipStream_t)stream;
    float *img = nullptr, *sino = nullptr, *img_out = nullptr, *sino_out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t n_img = (size_t)n * n, n_sino = (size_t)n_views * n_det;
    auto cleanup = [&] {
        for (float* b : {img, sino, img_out, sino_out})
            if (b) (void)hipFree(b);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    // validate the geometry once through the ordinary plan path
    radon_plan_t probe = nullptr;
    radon_status_t s = radon_plan_tuned(&probe, n, angles, n_views, n_det, sigma, W, nullptr);
    if (s != RADON_OK) return s;
    radon_tuning def{};
    (void)radon_plan_tuning(probe, &def);
    radon_plan_destroy(probe);
    if (hipMalloc(&img, sizeof(float) * n_img) != hipSuccess || hipMalloc(&sino, sizeof(float) * n_sino) != hipSuccess ||
        hipMalloc(&img_out, sizeof(float) * n_img) != hipSuccess ||
        hipMalloc(&sino_out, sizeof(float) * n_sino) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return errf(RADON_ERR_OOM, "autotune buffers");
    }
    hipLaunchKernelGGL(k_fill_hash, dim3(1024), dim3(256), 0, st, img, n_img, 12345u);
    hipLaunchKernelGGL(k_fill_hash, dim3(1024), dim3(256), 0, st, sino, n_sino, 67890u);

    // time one decomposition: ms per forward + adjoint pair, or < 0 if it does not fit
    auto time_one = [&](const radon_tuning& t, double* ms) -> radon_status_t {
        radon_plan_t pl = nullptr;
        const radon_status_t ps = radon_plan_tuned(&pl, n, angles, n_views, n_det, sigma, W, &t);
        if (ps == RADON_ERR_UNSUPPORTED) {
            *ms = -1.0;
            return RADON_OK;
        }
        if (ps != RADON_OK) return ps;
        radon_status_t r = RADON_OK;
        for (int k = 0; k <= repeats && r == RADON_OK; ++k) {
            if (k == 1) (void)hipEventRecord(e0, st);
            r = radon_forward(pl, img, sino_out, stream);
            if (r == RADON_OK) r = radon_adjoint(pl, sino, img_out, stream);
        }
        (void)hipEventRecord(e1, st);
        float el = 0.f;
        if (r == RADON_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&el, e0, e1) != hipSuccess)) {
            (void)hipGetLastError();
            r = errf(RADON_ERR_DEVICE, "autotune timing failed");
        }
        radon_plan_destroy(pl);
        *ms = el / repeats;
        return r;
    };

    // coordinate search: tile size first, then the spreading chunk, then the
    // forward chunk, each with the others at their current best
    radon_tuning cur = def;
    double cur_ms = 0.0;
    if ((s = time_one(cur, &cur_ms)) != RADON_OK) { cleanup(); return s; }
    if (default_ms) *default_ms = cur_ms;
    const int tiles[] = {8, 16, 32}, a2s[] = {256, 512}, f3s[] = {1024, 2048, 4096};
    auto try_set = [&](radon_tuning cand) -> radon_status_t {
        if (cand.tile == cur.tile && cand.a2_chunk == cur.a2_chunk && cand.f3_chunk == cur.f3_chunk) return RADON_OK;
        double ms = 0.0;
        const radon_status_t r = time_one(cand, &ms);
        if (r == RADON_OK && ms > 0.0 && ms < cur_ms) {
            cur = cand;
            cur_ms = ms;
        }
        return r;
    };
    for (int t : tiles) {
        radon_tuning c = cur;
        c.tile = t;
        if ((s = try_set(c)) != RADON_OK) { cleanup(); return s; }
    }
    for (int a : a2s) {
        radon_tuning c = cur;
        c.a2_chunk = a;
        if ((s = try_set(c)) != RADON_OK) { cleanup(); return s; }
    }
    for (int f : f3s) {
        radon_tuning c = cur;
        c.f3_chunk = f;
        if ((s = try_set(c)) != RADON_OK) { cleanup(); return s; }
    }
    cleanup();
    *best = cur;
    *best_ms = cur_ms;
    return rn::api_ok();
}

}  // extern "C"

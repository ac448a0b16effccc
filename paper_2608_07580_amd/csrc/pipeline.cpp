// Graph-captured retrieval pipeline: the launch sequence of one batch shape
// (network inference of the warm start for every scene, then the LM
// retrieval with fallback) recorded once into a HIP graph and replayed with
// a single graph launch.  The graph binds the buffers it was built with:
// a serving loop rewrites the radiance buffers in place and relaunches.
// Routed pipelines run the front end (HFDI, Sec. 2.1) first and the network
// only on its candidates, whose count stays on the device; every other
// pixel is solved from the default start.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ff_internal.hpp"

using namespace ff;

struct ff_pipeline {
    int device = 0;
    hipStream_t capture = nullptr;   // private: its scratch buffer is used by this graph alone
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float* z0 = nullptr;
    float* hfdi = nullptr;               // routed: index values, candidate lists and counts
    int64_t* index = nullptr;
    int64_t* count = nullptr;
    std::vector<const ff_mlp*> pinned;   // networks whose workspace the graph binds
};

namespace {

void release(ff_pipeline* p)
{
    if (!p) return;
    if (p->capture) (void)hipStreamSynchronize(p->capture);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->z0) (void)hipFree(p->z0);
    if (p->hfdi) (void)hipFree(p->hfdi);
    if (p->index) (void)hipFree(p->index);
    if (p->count) (void)hipFree(p->count);
    if (p->capture) {
        release_stream_scratch(p->capture);
        (void)hipStreamDestroy(p->capture);
    }
    for (const ff_mlp* m : p->pinned) mlp_pin(m, -1);
    delete p;
}

}  // namespace

static ff_status create(const ff_scene* const* scenes, const float* const* radiance_dev, const int64_t* P,
                        int32_t n_scenes, const ff_prior* prior, const ff_mlp* const* mlps, bool routed,
                        double threshold, const ff_options* opts, const ff_outputs* outs,
                        unsigned long long* evals_dev, void* stream, ff_pipeline** out)
{
    if (!out) return set_error(FF_EINVAL, "ff_pipeline_create: NULL out");
    if (routed && std::isnan(threshold)) return set_error(FF_EINVAL, "ff_pipeline_create_routed: threshold is NaN");
    *out = nullptr;
    if (n_scenes <= 0 || !scenes || !radiance_dev || !P || !prior || !opts || !outs)
        return set_error(FF_EINVAL, "ff_pipeline_create: NULL argument or empty batch");
    const int n = n_state(prior->model);
    if (n < 0) return set_error(FF_EINVAL, "ff_pipeline_create: unknown model");
    int64_t total = 0;
    std::vector<int64_t> off(n_scenes);
    for (int i = 0; i < n_scenes; ++i) {
        if (P[i] < 0) return set_error(FF_EINVAL, "ff_pipeline_create: P < 0");
        off[i] = total;
        total += P[i];
    }
    bool any_net = false;
    for (int i = 0; mlps && i < n_scenes; ++i) {
        if (!mlps[i]) continue;
        any_net = true;
        int n_in = 0, n_out = 0;
        mlp_dims(mlps[i], &n_in, &n_out);
        if (n_out != n) return set_error(FF_EINVAL, "ff_pipeline_create: network outputs != state size");
        if (!scenes[i] || scenes[i]->n_bands != n_in)
            return set_error(FF_EINVAL, "ff_pipeline_create: network inputs != band count");
    }
    auto* p = new ff_pipeline();
    {
        hipError_t e = hipGetDevice(&p->device);
        // wait for the caller's pending work on the bound buffers, then record
        // on a stream of the pipeline's own
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
        if (e != hipSuccess) {
            release(p);
            return hip_error(e, "ff_pipeline_create: capture stream");
        }
    }
    hipStream_t s = p->capture;
    void* cs = (void*)s;
    for (int i = 0; mlps && i < n_scenes; ++i) {
        if (!mlps[i] || std::find(p->pinned.begin(), p->pinned.end(), mlps[i]) != p->pinned.end()) continue;
        p->pinned.push_back(mlps[i]);
        mlp_pin(mlps[i], +1);
    }
    if (any_net && total > 0) {
        const hipError_t e = hipMalloc(&p->z0, (size_t)total * n * sizeof(float));
        if (e != hipSuccess) {
            release(p);
            return hip_error(e, "ff_pipeline_create: z0 buffer");
        }
    }
    std::vector<const float*> z0s(n_scenes, nullptr);
    for (int i = 0; i < n_scenes; ++i) z0s[i] = (p->z0 && mlps && mlps[i]) ? p->z0 + off[i] * n : nullptr;
    if (routed && any_net && total > 0) {
        hipError_t e = hipMalloc(&p->hfdi, (size_t)total * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&p->index, (size_t)total * sizeof(int64_t));
        if (e == hipSuccess) e = hipMalloc(&p->count, (size_t)n_scenes * sizeof(int64_t));
        if (e != hipSuccess) {
            release(p);
            return hip_error(e, "ff_pipeline_create_routed: candidate buffers");
        }
    }

    auto run = [&]() -> ff_status {
        for (int i = 0; any_net && i < n_scenes; ++i) {
            if (P[i] == 0 || !z0s[i]) continue;
            float* z = const_cast<float*>(z0s[i]);
            ff_status st;
            if (routed) {
                st = ff_hfdi_candidates(scenes[i], radiance_dev[i], P[i], threshold, p->hfdi + off[i],
                                        p->index + off[i], p->count + i, cs);
                if (st == FF_OK) st = mark_no_start(z, P[i], n, s);
                if (st == FF_OK)
                    st = mlp_infer_listed_dev(mlps[i], radiance_dev[i], P[i], p->index + off[i], p->count + i, z, s);
            } else {
                st = ff_mlp_infer(mlps[i], radiance_dev[i], P[i], z, cs);
            }
            if (st != FF_OK) return st;
        }
        return ff_retrieve_batch(scenes, radiance_dev, P, n_scenes, prior, any_net ? z0s.data() : nullptr, opts,
                                 outs, evals_dev, cs);
    };
    // one eager pass sizes every workspace outside capture
    ff_status st = run();
    if (st == FF_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_error(e, "ff_pipeline_create: eager pass");
    }
    if (st != FF_OK) {
        release(p);
        return st;
    }
    pin_stream_scratch(s);               // the graph below binds this buffer
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release(p);
        return hip_error(e, "hipStreamBeginCapture");
    }
    st = run();
    e = hipStreamEndCapture(s, &p->graph);
    if (st != FF_OK || e != hipSuccess) {
        release(p);
        return st != FF_OK ? st : hip_error(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        release(p);
        return hip_error(e, "hipGraphInstantiate");
    }
    *out = p;
    return clear_error();
}

extern "C" ff_status ff_pipeline_create(const ff_scene* const* scenes, const float* const* radiance_dev,
                                        const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                        const ff_mlp* const* mlps, const ff_options* opts, const ff_outputs* outs,
                                        unsigned long long* evals_dev, void* stream, ff_pipeline** out)
{
    return create(scenes, radiance_dev, P, n_scenes, prior, mlps, false, 0.0, opts, outs, evals_dev, stream, out);
}

extern "C" ff_status ff_pipeline_create_routed(const ff_scene* const* scenes, const float* const* radiance_dev,
                                               const int64_t* P, int32_t n_scenes, const ff_prior* prior,
                                               const ff_mlp* const* mlps, double hfdi_threshold,
                                               const ff_options* opts, const ff_outputs* outs,
                                               unsigned long long* evals_dev, void* stream, ff_pipeline** out)
{
    return create(scenes, radiance_dev, P, n_scenes, prior, mlps, true, hfdi_threshold, opts, outs, evals_dev,
                  stream, out);
}

extern "C" ff_status ff_pipeline_launch(ff_pipeline* p, void* stream)
{
    if (!p || !p->exec) return set_error(FF_EINVAL, "ff_pipeline_launch: NULL pipeline");
    FF_HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return clear_error();
}

extern "C" const float* ff_pipeline_z0(const ff_pipeline* p) { return p ? p->z0 : nullptr; }

extern "C" void ff_pipeline_destroy(ff_pipeline* p) { release(p); }

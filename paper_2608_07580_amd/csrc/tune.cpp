// Launch-shape autotuner for the retrieval: chooses lanes per pixel,
// workgroup size, workgroups per CU and schedule for a given batch by timing
// candidate launches on that batch (coordinate descent, one dimension at a
// time), and keeps the result in a JSON table keyed by device architecture,
// band count, model, precision, accumulation, quadrature order, start kind
// and the batch size rounded down to a power of two.
//
// The numerical result of a launch does not depend on workgroup size,
// workgroups per CU or schedule (bitwise), and depends on lanes per pixel
// only through the order of the band sums; the quadrature order is never
// changed by the tuner since it changes the model.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "ff_internal.hpp"

using namespace ff;

namespace {

std::mutex g_cache_mutex;

struct Choice {
    int lpp = 1, block = 256, bpc = 0, schedule = FF_SCHEDULE_PERSISTENT;
    double ms = 0.0;
};

std::string arch_name(int dev)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string tune_key(int dev, int B, const ff_prior* prior, const ff_options* o, bool warm, int64_t total)
{
    int bucket = 0;
    while (bucket < 62 && (int64_t(1) << (bucket + 1)) <= total) ++bucket;
    std::ostringstream k;
    k << arch_name(dev) << "/B" << B << "/model" << prior->model << "/prec" << o->precision << "/acc"
      << o->accumulate << "/Q" << o->n_quad << (warm ? "/warm" : "/plain") << "/P2^" << bucket;
    return k.str();
}

// The table is a JSON object with one entry per line:
//   "key": {"lanes_per_pixel": L, "block_size": b, "blocks_per_cu": c, "schedule": s, "ms": t}
std::map<std::string, std::string> read_table(const char* path)
{
    std::map<std::string, std::string> entries;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        const size_t brace = line.find('{', q1 == std::string::npos ? 0 : q1);
        const size_t end = line.rfind('}');
        if (q1 == std::string::npos || brace == std::string::npos || end == std::string::npos || end < brace)
            continue;
        entries[line.substr(q0 + 1, q1 - q0 - 1)] = line.substr(brace, end - brace + 1);
    }
    return entries;
}

bool parse_entry(const std::string& body, Choice& c)
{
    return std::sscanf(body.c_str(),
                       "{\"lanes_per_pixel\": %d, \"block_size\": %d, \"blocks_per_cu\": %d, \"schedule\": %d, "
                       "\"ms\": %lf}",
                       &c.lpp, &c.block, &c.bpc, &c.schedule, &c.ms) == 5;
}

bool write_table(const char* path, const std::map<std::string, std::string>& entries)
{
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return false;
        f << "{\n";
        size_t i = 0;
        for (const auto& kv : entries) {
            f << "  \"" << kv.first << "\": " << kv.second << (++i < entries.size() ? ",\n" : "\n");
        }
        f << "}\n";
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

void apply(const Choice& c, ff_options* o)
{
    o->lanes_per_pixel = c.lpp;
    o->block_size = c.block;
    o->blocks_per_cu = c.bpc;
    o->schedule = c.schedule;
}

}  // namespace

extern "C" ff_status ff_tune(const ff_scene* const* scenes, const float* const* radiance_dev, const int64_t* P,
                             int32_t n_scenes, const ff_prior* prior, const float* const* z0_dev,
                             ff_options* opts, const ff_outputs* outs, const char* cache_path, int32_t flags,
                             double* best_ms, void* stream)
{
    if (!opts || !prior || !scenes || !P || n_scenes <= 0)
        return set_error(FF_EINVAL, "ff_tune: NULL argument or empty batch");
    int64_t total = 0;
    bool warm = false;
    for (int i = 0; i < n_scenes; ++i) {
        if (!scenes[i]) return set_error(FF_EINVAL, "ff_tune: NULL scene");
        total += std::max<int64_t>(P[i], 0);
        warm = warm || (z0_dev && z0_dev[i] && P[i] > 0);
    }
    if (total == 0) return clear_error();
    int dev = 0;
    FF_HIP_TRY(hipGetDevice(&dev));
    const std::string key = tune_key(dev, scenes[0]->n_bands, prior, opts, warm, total);

    if (cache_path && !(flags & FF_TUNE_IGNORE_CACHE)) {
        std::lock_guard<std::mutex> lk(g_cache_mutex);
        const auto table = read_table(cache_path);
        const auto it = table.find(key);
        Choice c;
        if (it != table.end() && parse_entry(it->second, c)) {
            apply(c, opts);
            if (best_ms) *best_ms = c.ms;
            return clear_error();
        }
    }

    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FF_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(FF_EDEVICE, "ff_tune: hipEventCreate failed");
    }
    ff_status err = FF_OK;
    auto time_it = [&](const Choice& c) -> double {
        ff_options o = *opts;
        apply(c, &o);
        if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
        err = ff_retrieve_batch(scenes, radiance_dev, P, n_scenes, prior, z0_dev, &o, outs, nullptr, stream);
        if (err != FF_OK) return -1.0;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
        return (double)ms;
    };

    Choice best;
    best.lpp = opts->lanes_per_pixel > 0 ? opts->lanes_per_pixel : 1;
    best.block = opts->block_size > 0 ? opts->block_size : 256;
    best.bpc = opts->blocks_per_cu;
    best.schedule = opts->schedule;
    // untimed first launch (code objects, quadrature tables, allocator pools)
    best.ms = time_it(best);
    if (best.ms >= 0.0) best.ms = time_it(best);
    auto try_candidate = [&](Choice c) {
        if (best.ms < 0.0) return;
        c.ms = time_it(c);
        if (c.ms >= 0.0 && c.ms < best.ms) best = c;
        else if (c.ms < 0.0) best.ms = -1.0;
    };
    for (int lpp : {1, 2, 4, 8, 16, 32, 64}) {
        Choice c = best;
        c.lpp = lpp;
        if (lpp != best.lpp) try_candidate(c);
    }
    for (int block : {64, 128, 256}) {
        Choice c = best;
        c.block = block;
        if (block != best.block) try_candidate(c);
    }
    for (int bpc : {0, 1}) {
        Choice c = best;
        c.bpc = bpc;
        if (bpc != best.bpc) try_candidate(c);
    }
    {
        Choice c = best;
        c.schedule = best.schedule == FF_SCHEDULE_PERSISTENT ? FF_SCHEDULE_STATIC : FF_SCHEDULE_PERSISTENT;
        try_candidate(c);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best.ms < 0.0) {
        if (err != FF_OK) return err;
        return set_error(FF_EDEVICE, "ff_tune: timing a candidate launch failed");
    }
    apply(best, opts);
    if (best_ms) *best_ms = best.ms;

    if (cache_path) {
        std::lock_guard<std::mutex> lk(g_cache_mutex);
        auto table = read_table(cache_path);
        std::ostringstream body;
        body << "{\"lanes_per_pixel\": " << best.lpp << ", \"block_size\": " << best.block
             << ", \"blocks_per_cu\": " << best.bpc << ", \"schedule\": " << best.schedule
             << ", \"ms\": " << best.ms << "}";
        table[key] = body.str();
        if (!write_table(cache_path, table))
            return set_error(FF_EDEVICE, std::string("ff_tune: cannot write ") + cache_path);
    }
    return clear_error();
}

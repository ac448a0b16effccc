// Library-owned scratch memory: one grow-only device buffer per (device,
// stream).  Launches ordered on one stream reuse it safely (the next launch
// sequence starts after the previous one's kernels in stream order), so a
// launch sequence needs no allocation once its stream's buffer is large
// enough -- which is what lets it be recorded into a HIP graph.  Growing
// synchronizes the stream first and is refused while the stream is being
// captured.  Buffers are held until ff_release_scratch or process exit
// (a pipeline frees the buffer of its private stream when destroyed).
#include <hip/hip_runtime.h>

#include <map>
#include <set>
#include <mutex>
#include <utility>

#include "ff_internal.hpp"

namespace ff {
namespace {

struct Buf {
    void* ptr = nullptr;
    size_t bytes = 0;
    bool pinned = false;   // bound by an instantiated graph: never freed by ff_release_scratch
};

std::mutex g_mutex;
std::map<std::pair<int, hipStream_t>, Buf>& table()
{
    static auto* t = new std::map<std::pair<int, hipStream_t>, Buf>();   // never destroyed: no HIP calls at exit
    return *t;
}

}  // namespace

bool stream_capturing(hipStream_t stream)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

ff_status stream_scratch(hipStream_t stream, size_t bytes, void** out)
{
    int dev = 0;
    FF_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mutex);
    Buf& b = table()[{dev, stream}];
    if (b.bytes >= bytes) {
        *out = b.ptr;
        return FF_OK;
    }
    if (stream_capturing(stream))
        return set_error(FF_EINVAL, "scratch must grow outside graph capture: run the same call once on this "
                                    "stream before capturing it");
    FF_HIP_TRY(hipStreamSynchronize(stream));
    if (b.ptr) {
        FF_HIP_TRY(hipFree(b.ptr));
        b.ptr = nullptr;
        b.bytes = 0;
    }
    const size_t n = (bytes + 4095) / 4096 * 4096;
    FF_HIP_TRY(hipMalloc(&b.ptr, n));
    b.bytes = n;
    *out = b.ptr;
    return FF_OK;
}

}  // namespace ff

namespace ff {

// Keep the buffer of one stream for as long as its owner lives: a pipeline's
// graph binds the buffer of its private stream, so ff_release_scratch must
// not free it (release_stream_scratch, called by the owner, still does).
void pin_stream_scratch(hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mutex);
    auto it = table().find({dev, stream});
    if (it != table().end()) it->second.pinned = true;
}

// Drop the buffer of one stream (the stream must still exist: it is
// synchronized first).  Used by objects that own a private stream.
void release_stream_scratch(hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mutex);
    auto it = table().find({dev, stream});
    if (it == table().end()) return;
    (void)hipStreamSynchronize(stream);
    if (it->second.ptr) (void)hipFree(it->second.ptr);
    table().erase(it);
}

}  // namespace ff

extern "C" ff_status ff_release_scratch(void)
{
    std::lock_guard<std::mutex> lk(ff::g_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    // no stream handle is touched (some may have been destroyed): each device
    // that holds buffers is synchronized as a whole, then the buffers freed
    std::set<int> devices;
    for (const auto& kv : ff::table()) devices.insert(kv.first.first);
    for (int d : devices) {
        (void)hipSetDevice(d);
        (void)hipDeviceSynchronize();
    }
    for (auto it = ff::table().begin(); it != ff::table().end();) {
        if (it->second.pinned) {           // a live pipeline's graph binds it
            ++it;
            continue;
        }
        if (it->second.ptr) {
            (void)hipSetDevice(it->first.first);
            (void)hipFree(it->second.ptr);
        }
        it = ff::table().erase(it);
    }
    (void)hipSetDevice(cur);
    return ff::clear_error();
}

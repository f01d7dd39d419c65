// Host-side context of the C ABI: stream, grow-only named device buffers,
// pinned host scratch for small readbacks, last-error text.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/msc.h"
#include "common.h"

constexpr size_t HOST_SCRATCH_WORDS = 8192;  // pinned readback area (uint64 words)

struct ms_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    // device allocator of the workspace (hipMalloc / hipFree when null)
    ms_alloc_fn alloc_fn = nullptr;
    ms_free_fn free_fn = nullptr;
    void* alloc_user = nullptr;
    uint64_t* scratch = nullptr;  // this device's fixed scratch (ms_critical_noalloc)
    std::string err;
    struct Buf {
        void* p = nullptr;
        size_t cap = 0;
    };
    std::map<std::string, Buf> bufs;
    void* h_stage[2] = {nullptr, nullptr};  // pinned staging of the out-of-core field slabs
    size_t h_stage_bytes = 0;
    void* h_lab[2] = {nullptr, nullptr};  // pinned staging of the out-of-core slabs' labels
    size_t h_lab_bytes = 0;
    std::vector<std::pair<void*, size_t>> h_recs;  // pinned blocks holding the out-of-core slabs' records
    uint64_t* h_small = nullptr;  // pinned, coherent host scratch for small readbacks
    uint64_t* h_small_dev = nullptr;  // the same memory as the device addresses it
    // stage timing (events at stage boundaries of ms_complex)
    bool timing = false;
    hipEvent_t ev[8] = {};
    double acc_ms[8] = {};
    int64_t calls = 0;
    int64_t allocations = 0;     // device allocations since timing was enabled
    // launch-level timing of the entry-rank kernel (the dominant one): event
    // pairs recorded around each launch of a call, accumulated at its end
    std::vector<hipEvent_t> rank_ev;
    size_t rank_used = 0;        // pairs recorded in the current call
    double rank_ms = 0;
    int64_t rank_launches = 0, rank_entries = 0, rank_heads = 0;
    int64_t ws_bytes = 0;        // device memory held in bufs
    int path_schedule = MS_PATHS_READY;
    uint32_t merge_light = 32;   // see MS_OPT_MERGE_LIGHT
    uint32_t merge_chunk = 4096; // see MS_OPT_MERGE_CHUNK
    int grad_tile = 0;           // see MS_OPT_GRADIENT_TILE
    int transpose_pack = 24;     // see MS_OPT_TRANSPOSE_PACK
    uint32_t wave_blocks = 1024; // workgroups of a wave-path merge launch (4 per compute unit)
    // graph of the front of ms_complex_batch, captured on a private stream
    // and keyed by the dims and the buffers it uses (see ms_complex_batch)
    bool batch_graph = true;
    std::vector<uint64_t> front_key;
    hipGraphExec_t front_exec = nullptr;
    hipStream_t capture_stream = nullptr;
    int64_t front_captures = 0, front_replays = 0;
    // a helper thread of connect_impl: its stream (default priority), pinned
    // readback scratch and the events that order it against the main stream
    hipStream_t side_stream = nullptr;
    uint64_t* h_side = nullptr;
    uint64_t* h_side_dev = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // spans of the side work (event pairs) recorded in the current call, when timing
    std::vector<hipEvent_t> side_ev;
    size_t side_used = 0;
    double side_ms = 0;
    std::mutex buf_mu;  // the named buffers are looked up from both threads
};

namespace msc {

struct Fail {
    ms_status st;
};

// What a helper thread of a call overrides: the stream its work is queued
// on, the pinned scratch its readbacks go through, a prefix that keeps its
// scratch buffers apart from the calling thread's, and where its error text
// goes.  Unset on the calling thread.
struct ThreadCtx {
    hipStream_t stream = nullptr;
    uint64_t* h_small = nullptr;
    uint64_t* h_small_dev = nullptr;
    const char* prefix = nullptr;
    std::string* err = nullptr;
};
inline thread_local ThreadCtx t_ctx;

inline hipStream_t cur_stream(const ms_ctx* c) { return t_ctx.stream ? t_ctx.stream : c->stream; }
inline std::string& err_text(ms_ctx* c) { return t_ctx.err ? *t_ctx.err : c->err; }
inline std::string buf_key(const char* name) { return t_ctx.prefix ? std::string(t_ctx.prefix) + name : std::string(name); }

// One workspace allocation through the context's allocator; null on failure.
inline void* dev_alloc(ms_ctx* c, size_t bytes) {
    void* p = nullptr;
    if (c->alloc_fn) return c->alloc_fn(c->alloc_user, bytes, (void*)cur_stream(c));
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

// Returns a workspace allocation.  The stream is drained first, so that no
// queued kernel still uses the memory whichever stream it was allocated on.
inline void dev_free(ms_ctx* c, void* p, size_t bytes) {
    if (!p) return;
    (void)hipStreamSynchronize(cur_stream(c));
    if (c->free_fn)
        c->free_fn(c->alloc_user, p, bytes, (void*)cur_stream(c));
    else
        (void)hipFree(p);
}

// Device buffer `name` of at least `count` elements of T (grows, never shrinks).
template <typename T>
T* buf(ms_ctx* c, const char* name, size_t count) {
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    std::lock_guard<std::mutex> lock(c->buf_mu);
    ms_ctx::Buf& b = c->bufs[buf_key(name)];
    if (b.cap < bytes) {
        if (b.p) {
            dev_free(c, b.p, b.cap);
            c->ws_bytes -= (int64_t)b.cap;
            b.p = nullptr;
            b.cap = 0;
        }
        size_t want = bytes + bytes / 4 + 256;
        b.p = dev_alloc(c, want);
        if (!b.p) {
            err_text(c) = std::string("device allocation of ") + std::to_string(want) + " bytes failed for " + name;
            throw Fail{MS_ERR_OOM};
        }
        b.cap = want;
        c->ws_bytes += (int64_t)want;
        c->allocations++;
    }
    return (T*)b.p;
}

// Elements of T that buffer `name` holds now (0 if it was never allocated).
template <typename T>
size_t buf_elems(ms_ctx* c, const char* name) {
    std::lock_guard<std::mutex> lock(c->buf_mu);
    auto it = c->bufs.find(buf_key(name));
    return it == c->bufs.end() ? 0 : it->second.cap / sizeof(T);
}

// Like buf(), but a growth keeps the first `used` elements.
template <typename T>
T* buf_keep(ms_ctx* c, const char* name, size_t count, size_t used) {
    size_t bytes = (count ? count : 1) * sizeof(T);
    std::lock_guard<std::mutex> lock(c->buf_mu);
    ms_ctx::Buf& b = c->bufs[buf_key(name)];
    if (b.cap >= bytes) return (T*)b.p;
    size_t want = bytes + bytes / 2 + 256;
    void* p = dev_alloc(c, want);
    if (!p) {
        err_text(c) = std::string("device allocation of ") + std::to_string(want) + " bytes failed for " + name;
        throw Fail{MS_ERR_OOM};
    }
    if (b.p) {
        if (used) (void)hipMemcpyAsync(p, b.p, used * sizeof(T), hipMemcpyDeviceToDevice, cur_stream(c));
        dev_free(c, b.p, b.cap);
        c->ws_bytes -= (int64_t)b.cap;
    }
    b.p = p;
    b.cap = want;
    c->ws_bytes += (int64_t)want;
    c->allocations++;
    return (T*)p;
}

inline void check(ms_ctx* c, hipError_t e, const char* what) {
    if (e != hipSuccess) {
        err_text(c) = std::string(what) + ": " + hipGetErrorString(e);
        throw Fail{MS_ERR_HIP};
    }
}

inline void fail(ms_ctx* c, ms_status st, const std::string& msg) {
    err_text(c) = msg;
    throw Fail{st};
}

hipError_t launch_publish(const uint64_t* src, uint64_t n, uint64_t* dst, hipStream_t s);

// Copies `n` uint64 words (n <= HOST_SCRATCH_WORDS) from device to the
// pinned scratch and waits.  A one-thread kernel writes them straight into
// the scratch (coherent, device-mapped host memory).
inline uint64_t* readback(ms_ctx* c, const uint64_t* d, size_t n) {
    if (n > HOST_SCRATCH_WORDS) fail(c, MS_ERR_INTERNAL, "readback larger than the pinned scratch");
    uint64_t* h = t_ctx.h_small ? t_ctx.h_small : c->h_small;
    check(c, launch_publish(d, n, t_ctx.h_small ? t_ctx.h_small_dev : c->h_small_dev, cur_stream(c)), "readback");
    check(c, hipStreamSynchronize(cur_stream(c)), "stream synchronize");
    return h;
}

// Records boundary event i of ms_complex on the context stream (timing only).
inline void mark(ms_ctx* c, int i) {
    if (c->timing) check(c, hipEventRecord(c->ev[i], c->stream), "event record");
}

}  // namespace msc

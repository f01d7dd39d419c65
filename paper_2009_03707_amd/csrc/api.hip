// extern "C" entry points of libmsc.so (declared and documented in
// include/msc.h).  Each validates its arguments, runs its kernels on the
// context's stream and converts failures into ms_status codes.
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "ctx.h"
#include "graph.h"
#include "prims.h"

namespace msc {
uint32_t gradient_tiles(const Grid& g, int shape);
hipError_t launch_gradient(int shape, const float* f0, const float* const* fptr, const Geo& geo,
                           const uint32_t* tile_off, uint64_t total_tiles, uint32_t* grad, int* err, hipStream_t s);
size_t crit_tmp_elems(uint64_t nv);
const uint64_t* crit_totals_ptr(const uint64_t* tmp, uint64_t nv);
hipError_t launch_crit_count(const uint32_t* grad, const Geo& g, uint64_t* tmp, uint64_t** d_totals, hipStream_t s);
hipError_t launch_crit_scatter(const float* f0, const float* const* fptr, const uint32_t* grad, const Geo& g,
                               const uint64_t* tmp, uint32_t* id, uint8_t* index, float* value, uint32_t* vmax,
                               hipStream_t s, uint64_t cap = ~0ull);
void connect_impl(ms_ctx* c, const uint32_t* grad, const Geo& g, const uint32_t* crit_id, const int64_t count[4],
                  ms_arcs* out);

hipError_t launch_gather_u64(const uint64_t* src, const uint64_t* idx, uint64_t n, uint64_t* dst, hipStream_t s);
hipError_t launch_crit_field_counts(const uint32_t* id, const int64_t count[4], const Geo& geo, unsigned long long* cnt,
                                    hipStream_t s);
hipError_t launch_crit_split(const uint32_t* id, const uint8_t* index, const float* value, const uint32_t* vmax,
                             uint64_t n, const Geo& geo, const uint64_t* seg, const uint64_t* fk_before,
                             const uint64_t* fk_start, uint32_t* o_id, uint8_t* o_index, float* o_value,
                             uint32_t* o_vmax, hipStream_t s);
hipError_t launch_csr_split(const uint64_t* rowptr, uint64_t nrows, const uint32_t* col, uint64_t nnz,
                            const uint64_t* roff, const uint64_t* coff, const uint64_t* eoff, uint32_t nf,
                            uint64_t* orp, uint32_t* ocol, hipStream_t s);
hipError_t launch_manifold_labels(uint32_t* Pv, uint32_t* Pc, const Geo& g, const uint64_t* before, hipStream_t s);
hipError_t launch_sat_per_field(const uint64_t* val, uint64_t nnz, const uint64_t* eoff, uint32_t nf,
                                unsigned long long* out, hipStream_t s);

Geo single(const Grid& g) {
    Geo geo;
    geo.grids = nullptr;
    geo.voff = nullptr;
    geo.nf = 1;
    geo.nv = g.nv;
    geo.g0 = g;
    return geo;
}

Grid check_dims(ms_ctx* c, ms_dims d) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) fail(c, MS_ERR_INVALID_ARG, "every dimension must be >= 1");
    if (d.nx > (1 << 29) || d.ny > (1 << 29) || d.nz > (1 << 29) || d.nx * d.ny > ((int64_t)1 << 29) ||
        d.nx * d.ny * d.nz > ((int64_t)1 << 29))
        fail(c, MS_ERR_TOO_LARGE, "nx*ny*nz must not exceed 2^29 (cell ids are 32-bit)");
    return Grid::make(d.nx, d.ny, d.nz);
}

// The non-finite flag is cleared and copied by kernels rather than by
// memset / memcpy nodes, so that the front of a batch can be captured in a
// graph and replayed.
__global__ void k_flag_clear(int* err) {
    if (threadIdx.x == 0) *err = 0;
}
__global__ void k_flag_copy(const int* err, uint64_t* slot) {
    if (threadIdx.x == 0) *slot = err ? (uint64_t)(*err != 0) : 0ull;
}

void flag_clear(ms_ctx* c, int* d_err) {
    hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(64), 0, c->stream, d_err);
    check(c, hipGetLastError(), "clear error flag");
}

// gradient + non-finite flag (flag left on the device at *d_err)
void gradient_impl(ms_ctx* c, const float* f, const Grid& g, uint32_t* grad, int* d_err) {
    flag_clear(c, d_err);
    check(c, launch_gradient(c->grad_tile, f, nullptr, single(g), nullptr, gradient_tiles(g, c->grad_tile), grad, d_err,
                             c->stream),
          "gradient kernel launch");
}

// counts per index (host) after pass 1; optional scatter into `out`.  The
// pass scratch is `tmp` (crit_tmp_elems(nv) + 1 words) or, when null, the
// context's "crit_tmp" buffer.
// Pass 1 of the extraction (counts, scan, totals) and the copy of the
// non-finite flag (0 without d_err) into the slot after them: kernels only.
void critical_front(ms_ctx* c, const uint32_t* grad, const Geo& g, uint64_t* tmp, const int* d_err) {
    uint64_t* d_tot = nullptr;
    check(c, launch_crit_count(grad, g, tmp, &d_tot, c->stream), "critical count launch");
    hipLaunchKernelGGL(k_flag_copy, dim3(1), dim3(64), 0, c->stream, d_err, tmp + crit_tmp_elems(g.nv));
    check(c, hipGetLastError(), "flag copy");
}

// Reads the counts (and flag) back after critical_front; optional scatter.
void critical_finish(ms_ctx* c, const float* f, const float* const* fptr, const uint32_t* grad, const Geo& g,
                     const ms_crit* out, int64_t h_count[4], const int* d_err, ms_status* nonfinite, uint64_t* tmp) {
    const uint64_t* d_tot = crit_totals_ptr(tmp, g.nv);
    uint64_t* flag_slot = tmp + crit_tmp_elems(g.nv);
    // counts and the flag slot after them are contiguous: one readback
    static_assert(HOST_SCRATCH_WORDS >= 9, "scratch too small");
    check(c, launch_publish(d_tot, 8, c->h_small_dev, c->stream), "readback");
    check(c, launch_publish(flag_slot, 1, c->h_small_dev + 8, c->stream), "readback");
    check(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (d_err && c->h_small[8]) {
        *nonfinite = MS_ERR_NONFINITE;
        return;
    }
    int64_t total = 0;
    for (int k = 0; k < 4; k++) {
        h_count[k] = (int64_t)c->h_small[k];
        total += h_count[k];
    }
    if (!out) return;
    if (total > out->capacity) {
        *nonfinite = MS_ERR_CAPACITY;
        return;
    }
    if (total == 0) return;
    if (!out->id || !out->index || !out->value || !out->vmax) fail(c, MS_ERR_INVALID_ARG, "null critical output array");
    check(c, launch_crit_scatter(f, fptr, grad, g, tmp, out->id, out->index, out->value, out->vmax, c->stream),
          "critical scatter launch");
}

// Records the context's critical-record buffers (cx_crit_*) hold now.
uint64_t crit_record_capacity(ms_ctx* c) {
    size_t a = buf_elems<uint32_t>(c, "cx_crit_id"), b = buf_elems<uint8_t>(c, "cx_crit_index");
    size_t d = buf_elems<float>(c, "cx_crit_value"), e = buf_elems<uint32_t>(c, "cx_crit_vmax");
    size_t m = a < b ? a : b;
    m = m < d ? m : d;
    return m < e ? m : e;
}

void critical_impl(ms_ctx* c, const float* f, const float* const* fptr, const uint32_t* grad, const Geo& g,
                   const ms_crit* out, int64_t h_count[4], const int* d_err, ms_status* nonfinite,
                   uint64_t* tmp = nullptr) {
    if (!tmp) tmp = buf<uint64_t>(c, "crit_tmp", crit_tmp_elems(g.nv) + 1);
    critical_front(c, grad, g, tmp, d_err);
    critical_finish(c, f, fptr, grad, g, out, h_count, d_err, nonfinite, tmp);
}

// ---- fixed device scratch of the allocation-free entry point ----------------
//
// One array per GPU, held until the process ends.  Host code never passes
// `scratch` itself to a kernel (on the host it names a stand-in, not device
// memory): each device's address is taken once with hipGetSymbolAddress, with
// that device current, and kept in `scratch_addr`.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)8 << 20;
__device__ __align__(256) uint64_t scratch[NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)];

std::mutex scratch_mu;
std::map<int, uint64_t*> scratch_addr;

// Address of the current device's scratch array; null if it cannot be found.
uint64_t* scratch_for_device(int device) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    auto it = scratch_addr.find(device);
    if (it != scratch_addr.end()) return it->second;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return nullptr;
    }
    scratch_addr[device] = (uint64_t*)p;
    return (uint64_t*)p;
}

}  // namespace msc

using namespace msc;

#define API_BEGIN \
    if (!ctx) return MS_ERR_INVALID_ARG; \
    try {
#define API_END                                             \
    }                                                       \
    catch (const Fail& e) {                                 \
        return e.st;                                        \
    }                                                       \
    catch (const std::exception& e) {                       \
        ctx->err = std::string("internal error: ") + e.what(); \
        return MS_ERR_INTERNAL;                             \
    }                                                       \
    catch (...) {                                           \
        ctx->err = "internal error";                        \
        return MS_ERR_INTERNAL;                             \
    }                                                       \
    return MS_OK;

extern "C" {

ms_status ms_ctx_create(ms_ctx** out, void* stream, ms_alloc_fn alloc_fn, ms_free_fn free_fn, void* user) {
    if (!out) return MS_ERR_INVALID_ARG;
    *out = nullptr;
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return MS_ERR_INVALID_ARG;
    ms_ctx* c = new (std::nothrow) ms_ctx();
    if (!c) return MS_ERR_OOM;
    c->stream = (hipStream_t)stream;
    c->alloc_fn = alloc_fn;
    c->free_fn = free_fn;
    c->alloc_user = user;
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return MS_ERR_HIP;
    }
    if (hipHostMalloc((void**)&c->h_small, HOST_SCRATCH_WORDS * sizeof(uint64_t),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->h_small_dev, c->h_small, 0) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return MS_ERR_OOM;
    }
    c->scratch = scratch_for_device(c->device);
    if (!c->scratch) {
        (void)hipHostFree(c->h_small);
        delete c;
        return MS_ERR_HIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
        c->wave_blocks = 4u * (uint32_t)cus;
    (void)hipGetLastError();
    *out = c;
    return MS_OK;
}

void ms_ctx_destroy(ms_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->bufs) dev_free(ctx, kv.second.p, kv.second.cap);
    if (ctx->h_small) (void)hipHostFree(ctx->h_small);
    for (void* p : ctx->h_stage)
        if (p) (void)hipHostFree(p);
    for (void* p : ctx->h_lab)
        if (p) (void)hipHostFree(p);
    for (auto& b : ctx->h_recs) (void)hipHostFree(b.first);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->rank_ev) (void)hipEventDestroy(e);
    if (ctx->front_exec) (void)hipGraphExecDestroy(ctx->front_exec);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->side_stream) {
        (void)hipStreamSynchronize(ctx->side_stream);
        (void)hipStreamDestroy(ctx->side_stream);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    for (auto& e : ctx->side_ev) (void)hipEventDestroy(e);
    if (ctx->h_side) (void)hipHostFree(ctx->h_side);
    delete ctx;
}

ms_status ms_ctx_release(ms_ctx* ctx) {
    if (!ctx) return MS_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->bufs) dev_free(ctx, kv.second.p, kv.second.cap);
    ctx->bufs.clear();
    ctx->ws_bytes = 0;
    for (void*& p : ctx->h_stage) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
    }
    ctx->h_stage_bytes = 0;
    for (void*& p : ctx->h_lab) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
    }
    ctx->h_lab_bytes = 0;
    for (auto& b : ctx->h_recs) (void)hipHostFree(b.first);
    ctx->h_recs.clear();
    return MS_OK;
}

ms_status ms_ctx_set_stream(ms_ctx* ctx, void* stream) {
    if (!ctx) return MS_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)stream;
    return MS_OK;
}

const char* ms_last_error(const ms_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ms_status ms_ctx_set_option(ms_ctx* ctx, int option, int64_t value) {
    if (!ctx) return MS_ERR_INVALID_ARG;
    if (option == MS_OPT_PATH_SCHEDULE && (value == MS_PATHS_READY || value == MS_PATHS_POWER || value == MS_PATHS_ENTRY)) {
        ctx->path_schedule = (int)value;
        return MS_OK;
    }
    if (option == MS_OPT_MERGE_LIGHT && value >= 0 && value <= 256) {
        ctx->merge_light = (uint32_t)value;
        return MS_OK;
    }
    if (option == MS_OPT_MERGE_CHUNK && value >= 1 && value <= 4096) {
        ctx->merge_chunk = (uint32_t)value;
        return MS_OK;
    }
    if (option == MS_OPT_GRADIENT_TILE && value >= 0 && value <= 6) {
        ctx->grad_tile = (int)value;
        return MS_OK;
    }
    if (option == MS_OPT_BATCH_GRAPH && (value == 0 || value == 1)) {
        ctx->batch_graph = value != 0;
        return MS_OK;
    }
    if (option == MS_OPT_TRANSPOSE_PACK && value >= 0 && value <= 24) {
        ctx->transpose_pack = (int)value;
        return MS_OK;
    }
    ctx->err = "unknown option or value";
    return MS_ERR_INVALID_ARG;
}

ms_status ms_ctx_set_timing(ms_ctx* ctx, int enable) {
    API_BEGIN
    if (enable) {
        for (auto& e : ctx->ev)
            if (!e) check(ctx, hipEventCreate(&e), "event create");
    }
    ctx->timing = enable != 0;
    for (double& a : ctx->acc_ms) a = 0;
    ctx->calls = 0;
    ctx->allocations = 0;
    ctx->rank_ms = 0;
    ctx->rank_launches = ctx->rank_entries = ctx->rank_heads = 0;
    ctx->rank_used = 0;
    ctx->side_ms = 0;
    ctx->side_used = 0;
    API_END
}

ms_status ms_ctx_get_timing(ms_ctx* ctx, ms_timing* out) {
    if (!ctx || !out) return MS_ERR_INVALID_ARG;
    out->gradient_ms = ctx->acc_ms[0];
    out->critical_ms = ctx->acc_ms[1];
    out->extrema_ms = ctx->acc_ms[2];
    out->bfs_ms = ctx->acc_ms[3];
    out->minor_ms = ctx->acc_ms[4];
    out->paths_ms = ctx->acc_ms[5];
    out->total_ms = ctx->acc_ms[6];
    out->side_ms = ctx->side_ms;
    out->calls = ctx->calls;
    out->allocations = ctx->allocations;
    out->workspace_bytes = ctx->ws_bytes;
    out->rank_ms = ctx->rank_ms;
    out->rank_launches = ctx->rank_launches;
    out->rank_entries = ctx->rank_entries;
    out->rank_heads = ctx->rank_heads;
    out->graph_captures = ctx->front_captures;
    out->graph_replays = ctx->front_replays;
    return MS_OK;
}

ms_status ms_gradient(ms_ctx* ctx, const float* d_f, ms_dims dims, uint32_t* d_grad) {
    API_BEGIN
    Grid g = check_dims(ctx, dims);
    if (!d_f || !d_grad) fail(ctx, MS_ERR_INVALID_ARG, "null field or gradient pointer");
    int* d_err = buf<int>(ctx, "err_flag", 4);
    gradient_impl(ctx, d_f, g, d_grad, d_err);
    int h = 0;
    check(ctx, hipMemcpyAsync(ctx->h_small, d_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "readback");
    check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
    memcpy(&h, ctx->h_small, sizeof(int));
    if (h) fail(ctx, MS_ERR_NONFINITE, "the field contains NaN or infinite values");
    API_END
}

ms_status ms_critical(ms_ctx* ctx, const float* d_f, const uint32_t* d_grad, ms_dims dims, const ms_crit* out,
                      int64_t h_count[4]) {
    API_BEGIN
    Grid g = check_dims(ctx, dims);
    if (!d_f || !d_grad || !h_count) fail(ctx, MS_ERR_INVALID_ARG, "null argument");
    ms_status st = MS_OK;
    critical_impl(ctx, d_f, nullptr, d_grad, single(g), out, h_count, nullptr, &st);
    if (st == MS_ERR_CAPACITY) fail(ctx, st, "critical output capacity too small");
    API_END
}

ms_status ms_critical_noalloc(ms_ctx* ctx, const float* d_f, const uint32_t* d_grad, ms_dims dims,
                              const ms_crit* out, int64_t h_count[4]) {
    API_BEGIN
    Grid g = check_dims(ctx, dims);
    if (!d_f || !d_grad || !h_count) fail(ctx, MS_ERR_INVALID_ARG, "null argument");
    const size_t need = (crit_tmp_elems(g.nv) + 1) * sizeof(uint64_t);
    if (need > NOALLOC_SCRATCH_BYTES)
        fail(ctx, MS_ERR_TOO_LARGE,
             "field too large for the fixed scratch of ms_critical_noalloc (" + std::to_string(need) + " > " +
                 std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes); use ms_critical");
    ms_status st = MS_OK;
    critical_impl(ctx, d_f, nullptr, d_grad, single(g), out, h_count, nullptr, &st, ctx->scratch);
    if (st == MS_ERR_CAPACITY) fail(ctx, st, "critical output capacity too small");
    API_END
}

ms_status ms_connect(ms_ctx* ctx, const uint32_t* d_grad, ms_dims dims, const uint32_t* d_crit_id,
                     const int64_t h_count[4], ms_arcs* out) {
    API_BEGIN
    Grid g = check_dims(ctx, dims);
    if (!d_grad || !h_count || !out) fail(ctx, MS_ERR_INVALID_ARG, "null argument");
    int64_t total = 0;
    for (int k = 0; k < 4; k++) {
        if (h_count[k] < 0) fail(ctx, MS_ERR_INVALID_ARG, "negative critical count");
        total += h_count[k];
    }
    if (total > 0 && !d_crit_id) fail(ctx, MS_ERR_INVALID_ARG, "null critical list");
    // the list must hold exactly the critical cells of the gradient: compare
    // the counts here; the labelling pass checks each entry
    int64_t have[4];
    ms_status st = MS_OK;
    critical_impl(ctx, nullptr, nullptr, d_grad, single(g), nullptr, have, nullptr, &st);
    for (int k = 0; k < 4; k++)
        if (have[k] != h_count[k]) fail(ctx, MS_ERR_INVALID_ARG, "critical counts do not match the gradient");
    connect_impl(ctx, d_grad, single(g), d_crit_id, h_count, out);
    API_END
}

static void accumulate_timing(ms_ctx* ctx) {
    if (!ctx->timing) return;
    check(ctx, hipEventSynchronize(ctx->ev[6]), "event synchronize");
    for (int i = 0; i < 6; i++) {
        float ms = 0;
        check(ctx, hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]), "event elapsed");
        ctx->acc_ms[i] += ms;
    }
    float tot = 0;
    check(ctx, hipEventElapsedTime(&tot, ctx->ev[0], ctx->ev[6]), "event elapsed");
    ctx->acc_ms[6] += tot;
    for (size_t i = 0; i < ctx->side_used; i++) {  // the main stream waited for the side work before ev[6]
        float ms = 0;
        check(ctx, hipEventElapsedTime(&ms, ctx->side_ev[2 * i], ctx->side_ev[2 * i + 1]), "event elapsed");
        ctx->side_ms += ms;
    }
    ctx->side_used = 0;
    ctx->calls++;
    for (size_t i = 0; i < ctx->rank_used; i++) {
        float ms = 0;
        check(ctx, hipEventElapsedTime(&ms, ctx->rank_ev[2 * i], ctx->rank_ev[2 * i + 1]), "event elapsed");
        ctx->rank_ms += ms;
    }
    ctx->rank_launches += (int64_t)ctx->rank_used;
    ctx->rank_used = 0;
}

ms_status ms_complex(ms_ctx* ctx, const float* d_f, ms_dims dims, ms_result* out) {
    API_BEGIN
    Grid g = check_dims(ctx, dims);
    if (!d_f || !out) fail(ctx, MS_ERR_INVALID_ARG, "null argument");
    memset(out, 0, sizeof(*out));
    uint32_t* grad = buf<uint32_t>(ctx, "cx_grad", g.nv);
    int* d_err = buf<int>(ctx, "err_flag", 4);
    flag_clear(ctx, d_err);
    mark(ctx, 0);
    check(ctx, launch_gradient(ctx->grad_tile, d_f, nullptr, single(g), nullptr, gradient_tiles(g, ctx->grad_tile), grad,
                               d_err, ctx->stream),
          "gradient kernel launch");
    mark(ctx, 1);
    int64_t cnt[4];
    ms_status st = MS_OK;
    // the records go to context buffers: when they are already allocated the
    // scatter is queued before the counts are read (it writes nothing if they
    // do not fit), so the device does not wait for the host in between
    uint64_t* tmp = buf<uint64_t>(ctx, "crit_tmp", crit_tmp_elems(g.nv) + 1);
    critical_front(ctx, grad, single(g), tmp, d_err);
    const uint64_t cap = crit_record_capacity(ctx);
    if (cap > 0)
        check(ctx, launch_crit_scatter(d_f, nullptr, grad, single(g), tmp, buf<uint32_t>(ctx, "cx_crit_id", 1),
                                       buf<uint8_t>(ctx, "cx_crit_index", 1), buf<float>(ctx, "cx_crit_value", 1),
                                       buf<uint32_t>(ctx, "cx_crit_vmax", 1), ctx->stream, cap),
              "critical scatter launch");
    critical_finish(ctx, d_f, nullptr, grad, single(g), nullptr, cnt, d_err, &st, tmp);
    if (st == MS_ERR_NONFINITE) fail(ctx, st, "the field contains NaN or infinite values");
    int64_t total = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    ms_crit cr;
    cr.id = buf<uint32_t>(ctx, "cx_crit_id", total);
    cr.index = buf<uint8_t>(ctx, "cx_crit_index", total);
    cr.value = buf<float>(ctx, "cx_crit_value", total);
    cr.vmax = buf<uint32_t>(ctx, "cx_crit_vmax", total);
    cr.capacity = total;
    if (total > 0 && (uint64_t)total > cap)
        check(ctx, launch_crit_scatter(d_f, nullptr, grad, single(g), tmp, cr.id, cr.index, cr.value, cr.vmax,
                                       ctx->stream),
              "critical scatter launch");
    out->grad = grad;
    out->crit = cr;
    for (int k = 0; k < 4; k++) out->count[k] = cnt[k];
    mark(ctx, 2);
    connect_impl(ctx, grad, single(g), cr.id, cnt, &out->arcs);
    mark(ctx, 6);
    accumulate_timing(ctx);
    API_END
}

ms_status ms_complex_batch(ms_ctx* ctx, int32_t nfields, const float* const* d_f, const ms_dims* dims,
                           ms_result* outs) {
    API_BEGIN
    if (nfields < 1 || nfields > 1024 || !d_f || !dims || !outs)
        fail(ctx, MS_ERR_INVALID_ARG, "need 1..1024 fields and non-null arrays");
    hipStream_t s = ctx->stream;
    const uint32_t nf = (uint32_t)nfields;
    std::vector<Grid> grids(nf);
    std::vector<uint32_t> voff(nf + 1), toff(nf + 1);
    uint64_t total = 0, tiles = 0;
    for (uint32_t f = 0; f < nf; f++) {
        grids[f] = check_dims(ctx, dims[f]);
        if (!d_f[f]) fail(ctx, MS_ERR_INVALID_ARG, "null field pointer");
        voff[f] = (uint32_t)total;
        toff[f] = (uint32_t)tiles;
        total += grids[f].nv;
        tiles += gradient_tiles(grids[f], ctx->grad_tile);
        if (total > ((uint64_t)1 << 29)) fail(ctx, MS_ERR_TOO_LARGE, "the batch has more than 2^29 vertices");
    }
    voff[nf] = (uint32_t)total;
    toff[nf] = (uint32_t)tiles;
    // field tables on the device
    Grid* d_grids = buf<Grid>(ctx, "bx.grids", nf);
    uint32_t* d_voff = buf<uint32_t>(ctx, "bx.voff", nf + 1);
    uint32_t* d_toff = buf<uint32_t>(ctx, "bx.toff", nf + 1);
    const float** d_fptr = buf<const float*>(ctx, "bx.fptr", nf);
    check(ctx, hipMemcpyAsync(d_grids, grids.data(), sizeof(Grid) * nf, hipMemcpyHostToDevice, s), "table copy");
    check(ctx, hipMemcpyAsync(d_voff, voff.data(), 4 * (nf + 1), hipMemcpyHostToDevice, s), "table copy");
    check(ctx, hipMemcpyAsync(d_toff, toff.data(), 4 * (nf + 1), hipMemcpyHostToDevice, s), "table copy");
    check(ctx, hipMemcpyAsync(d_fptr, d_f, sizeof(float*) * nf, hipMemcpyHostToDevice, s), "table copy");
    Geo geo;
    geo.grids = d_grids;
    geo.voff = d_voff;
    geo.nf = nf;
    geo.nv = (uint32_t)total;
    geo.g0 = grids[0];
    // the hot path over the concatenation
    uint32_t* grad = buf<uint32_t>(ctx, "cx_grad", total);
    int* d_err = buf<int>(ctx, "err_flag", 4);
    uint64_t* ctmp = buf<uint64_t>(ctx, "crit_tmp", crit_tmp_elems(geo.nv) + 1);
    // The front (flag clear, gradient, critical counts, scan, totals) has a
    // fixed shape for given dims: it is captured once in a graph and
    // replayed while the dims and the buffers stay the same (the fields are
    // read through the device table, so new fields reuse the graph).
    auto front = [&](hipStream_t st) {
        hipStream_t keep = ctx->stream;
        ctx->stream = st;
        try {
            flag_clear(ctx, d_err);
            check(ctx, launch_gradient(ctx->grad_tile, d_f[0], d_fptr, geo, d_toff, tiles, grad, d_err, st),
                  "gradient kernel launch");
            critical_front(ctx, grad, geo, ctmp, d_err);
        } catch (...) {
            ctx->stream = keep;
            throw;
        }
        ctx->stream = keep;
    };
    if (ctx->batch_graph && !ctx->timing) {
        std::vector<uint64_t> key = {nf, (uint64_t)ctx->grad_tile, (uint64_t)(uintptr_t)grad, (uint64_t)(uintptr_t)d_err,
                                     (uint64_t)(uintptr_t)ctmp, (uint64_t)(uintptr_t)d_grids, (uint64_t)(uintptr_t)d_voff,
                                     (uint64_t)(uintptr_t)d_toff, (uint64_t)(uintptr_t)d_fptr};
        for (uint32_t f = 0; f < nf; f++) {
            key.push_back(grids[f].n[0]);
            key.push_back(grids[f].n[1]);
            key.push_back(grids[f].n[2]);
        }
        if (!ctx->front_exec || key != ctx->front_key) {
            if (ctx->front_exec) {
                (void)hipGraphExecDestroy(ctx->front_exec);
                ctx->front_exec = nullptr;
            }
            if (!ctx->capture_stream)
                check(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking), "stream create");
            hipGraph_t graph = nullptr;
            check(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
            try {
                front(ctx->capture_stream);
            } catch (...) {
                (void)hipStreamEndCapture(ctx->capture_stream, &graph);
                if (graph) (void)hipGraphDestroy(graph);
                throw;
            }
            check(ctx, hipStreamEndCapture(ctx->capture_stream, &graph), "end capture");
            hipError_t e = hipGraphInstantiate(&ctx->front_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) ctx->front_exec = nullptr;
            check(ctx, e, "graph instantiate");
            ctx->front_key = key;
            ctx->front_captures++;
        }
        check(ctx, hipGraphLaunch(ctx->front_exec, s), "graph launch");
        ctx->front_replays++;
    } else {
        mark(ctx, 0);
        flag_clear(ctx, d_err);
        check(ctx, launch_gradient(ctx->grad_tile, d_f[0], d_fptr, geo, d_toff, tiles, grad, d_err, s),
              "gradient kernel launch");
        mark(ctx, 1);
        critical_front(ctx, grad, geo, ctmp, d_err);
    }
    int64_t cnt[4];
    ms_status st = MS_OK;
    // as in ms_complex: queued before the counts are read when the record buffers exist
    const uint64_t cap = crit_record_capacity(ctx);
    if (cap > 0)
        check(ctx, launch_crit_scatter(d_f[0], d_fptr, grad, geo, ctmp, buf<uint32_t>(ctx, "cx_crit_id", 1),
                                       buf<uint8_t>(ctx, "cx_crit_index", 1), buf<float>(ctx, "cx_crit_value", 1),
                                       buf<uint32_t>(ctx, "cx_crit_vmax", 1), s, cap),
              "critical scatter launch");
    critical_finish(ctx, d_f[0], d_fptr, grad, geo, nullptr, cnt, d_err, &st, ctmp);
    if (st == MS_ERR_NONFINITE) fail(ctx, st, "a field contains NaN or infinite values");
    const int64_t ncrit = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    ms_crit cr;
    cr.id = buf<uint32_t>(ctx, "cx_crit_id", ncrit);
    cr.index = buf<uint8_t>(ctx, "cx_crit_index", ncrit);
    cr.value = buf<float>(ctx, "cx_crit_value", ncrit);
    cr.vmax = buf<uint32_t>(ctx, "cx_crit_vmax", ncrit);
    cr.capacity = ncrit;
    if (ncrit > 0 && (uint64_t)ncrit > cap)
        check(ctx, launch_crit_scatter(d_f[0], d_fptr, grad, geo, ctmp, cr.id, cr.index, cr.value, cr.vmax, s),
              "critical scatter launch");
    mark(ctx, 2);
    ms_arcs arcs;
    connect_impl(ctx, grad, geo, cr.id, cnt, &arcs);
    // ---- split into per-field results ------------------------------------
    unsigned long long* d_fk = (unsigned long long*)buf<uint64_t>(ctx, "bx.fk", 4 * nf);
    check(ctx, launch_crit_field_counts(cr.id, cnt, geo, d_fk, s), "field counts");
    std::vector<uint64_t> fk(4 * nf);
    {
        const uint64_t* h = readback(ctx, (const uint64_t*)d_fk, 4 * nf);
        for (uint32_t i = 0; i < 4 * nf; i++) fk[i] = h[i];
    }
    // fk_before[f][k]: cells of index k in earlier fields (f = nf: all);
    // fk_start[f][k]: first output position of (f, k); crit_off[f]: first of f
    std::vector<uint64_t> before(4 * (nf + 1)), start(4 * nf), crit_off(nf + 1), seg(4);
    seg[0] = 0;
    for (int k = 1; k < 4; k++) seg[k] = seg[k - 1] + (uint64_t)cnt[k - 1];
    uint64_t run = 0;
    for (uint32_t f = 0; f <= nf; f++) {
        for (int k = 0; k < 4; k++) before[4 * f + k] = f == 0 ? 0 : before[4 * (f - 1) + k] + fk[4 * (f - 1) + k];
        if (f == nf) break;
        crit_off[f] = run;
        for (int k = 0; k < 4; k++) {
            start[4 * f + k] = run;
            run += fk[4 * f + k];
        }
    }
    crit_off[nf] = run;
    uint64_t* d_tab = buf<uint64_t>(ctx, "bx.tab", 4 + 4 * (nf + 1) + 4 * nf);
    check(ctx, hipMemcpyAsync(d_tab, seg.data(), 8 * 4, hipMemcpyHostToDevice, s), "table copy");
    check(ctx, hipMemcpyAsync(d_tab + 4, before.data(), 8 * 4 * (nf + 1), hipMemcpyHostToDevice, s), "table copy");
    check(ctx, hipMemcpyAsync(d_tab + 4 + 4 * (nf + 1), start.data(), 8 * 4 * nf, hipMemcpyHostToDevice, s),
          "table copy");
    check(ctx, launch_manifold_labels(arcs.min_label, arcs.max_label, geo, d_tab + 4, s), "manifold labels");
    ms_crit fc;
    fc.id = buf<uint32_t>(ctx, "bx_crit_id", ncrit);
    fc.index = buf<uint8_t>(ctx, "bx_crit_index", ncrit);
    fc.value = buf<float>(ctx, "bx_crit_value", ncrit);
    fc.vmax = buf<uint32_t>(ctx, "bx_crit_vmax", ncrit);
    check(ctx, launch_crit_split(cr.id, cr.index, cr.value, cr.vmax, (uint64_t)ncrit, geo, d_tab, d_tab + 4,
                                 d_tab + 4 + 4 * (nf + 1), fc.id, fc.index, fc.value, fc.vmax, s),
          "critical split");
    for (uint32_t f = 0; f < nf; f++) {
        ms_result& o = outs[f];
        memset(&o, 0, sizeof(o));
        o.grad = grad + voff[f];
        o.crit.id = fc.id + crit_off[f];
        o.crit.index = fc.index + crit_off[f];
        o.crit.value = fc.value + crit_off[f];
        o.crit.vmax = fc.vmax + crit_off[f];
        o.crit.capacity = (int64_t)(crit_off[f + 1] - crit_off[f]);
        for (int k = 0; k < 4; k++) o.count[k] = (int64_t)fk[4 * f + k];
        o.arcs.stats = arcs.stats;
        o.arcs.min_label = arcs.min_label + voff[f];
        o.arcs.max_label = arcs.max_label + voff[f];
    }
    // block-diagonal matrices -> per-field matrices
    struct M {
        ms_csr ms_arcs::*m;
        int ri, ci;
        const char* name;
    };
    const M mats[6] = {{&ms_arcs::m10, 1, 0, "bx.m10"},  {&ms_arcs::m10t, 0, 1, "bx.m10t"},
                       {&ms_arcs::m21, 2, 1, "bx.m21"},  {&ms_arcs::m21t, 1, 2, "bx.m21t"},
                       {&ms_arcs::m32, 3, 2, "bx.m32"},  {&ms_arcs::m32t, 2, 3, "bx.m32t"}};
    uint64_t* d_off = buf<uint64_t>(ctx, "bx.off", 3 * (nf + 1));
    std::vector<uint64_t> roff(nf + 1), coff(nf + 1);
    for (const M& m : mats) {
        const ms_csr& G = arcs.*(m.m);
        for (uint32_t f = 0; f <= nf; f++) {
            roff[f] = before[4 * f + m.ri];
            coff[f] = before[4 * f + m.ci];
        }
        check(ctx, hipMemcpyAsync(d_off, roff.data(), 8 * (nf + 1), hipMemcpyHostToDevice, s), "table copy");
        check(ctx, hipMemcpyAsync(d_off + (nf + 1), coff.data(), 8 * (nf + 1), hipMemcpyHostToDevice, s),
              "table copy");
        check(ctx, launch_gather_u64((const uint64_t*)G.rowptr, d_off, nf + 1, d_off + 2 * (nf + 1), s), "gather");
        std::string nm = m.name;
        uint64_t* orp = buf<uint64_t>(ctx, (nm + ".rowptr").c_str(), (uint64_t)G.nrows + nf);
        uint32_t* ocol = buf<uint32_t>(ctx, (nm + ".col").c_str(), (uint64_t)G.nnz);
        check(ctx, launch_csr_split((const uint64_t*)G.rowptr, (uint64_t)G.nrows, G.col, (uint64_t)G.nnz, d_off,
                                    d_off + (nf + 1), d_off + 2 * (nf + 1), nf, orp, ocol, s),
              "csr split");
        const uint64_t* h = readback(ctx, d_off + 2 * (nf + 1), nf + 1);
        for (uint32_t f = 0; f < nf; f++) {
            ms_csr& o = outs[f].arcs.*(m.m);
            o.nrows = (int64_t)(roff[f + 1] - roff[f]);
            o.ncols = (int64_t)(coff[f + 1] - coff[f]);
            o.nnz = (int64_t)(h[f + 1] - h[f]);
            o.rowptr = (int64_t*)(orp + roff[f] + f);
            o.col = ocol + h[f];
            o.val = G.val + h[f];
        }
        if (m.m == &ms_arcs::m21t) {
            unsigned long long* d_sat = (unsigned long long*)buf<uint64_t>(ctx, "bx.sat", nf);
            check(ctx, hipMemsetAsync(d_sat, 0, 8 * nf, s), "memset");
            check(ctx, launch_sat_per_field(G.val, (uint64_t)G.nnz, d_off + 2 * (nf + 1), nf, d_sat, s), "sat");
            const uint64_t* hs = readback(ctx, (const uint64_t*)d_sat, nf);
            for (uint32_t f = 0; f < nf; f++) outs[f].arcs.n_saturated = (int64_t)hs[f];
        }
    }
    mark(ctx, 6);
    accumulate_timing(ctx);
    API_END
}

}  // extern "C"

namespace msc {

// Fills `in` from a result; `copy(dst, src, bytes)` moves one array to the
// host.  Returns an error text, empty on success.
template <typename Copy>
std::string graph_input(const ms_result* r, ms_dims dims, GraphInput& in, Copy&& copy) {
    in.dims[0] = dims.nx;
    in.dims[1] = dims.ny;
    in.dims[2] = dims.nz;
    int64_t tot = 0;
    for (int k = 0; k < 4; k++) {
        if (r->count[k] < 0) return "negative critical count";
        in.count[k] = r->count[k];
        tot += r->count[k];
    }
    if (tot > 0 && (!r->crit.id || !r->crit.index || !r->crit.value || !r->crit.vmax))
        return "null critical array in the result";
    in.id.resize((size_t)tot);
    in.index.resize((size_t)tot);
    in.value.resize((size_t)tot);
    in.vmax.resize((size_t)tot);
    copy(in.id.data(), r->crit.id, 4 * (size_t)tot);
    copy(in.index.data(), r->crit.index, (size_t)tot);
    copy(in.value.data(), r->crit.value, 4 * (size_t)tot);
    copy(in.vmax.data(), r->crit.vmax, 4 * (size_t)tot);
    const ms_csr* src[6] = {&r->arcs.m10, &r->arcs.m10t, &r->arcs.m21, &r->arcs.m21t, &r->arcs.m32, &r->arcs.m32t};
    HostCsr* dst[6] = {&in.m10, &in.m10t, &in.m21, &in.m21t, &in.m32, &in.m32t};
    for (int i = 0; i < 6; i++) {
        const ms_csr& m = *src[i];
        if (m.nrows < 0 || m.ncols < 0 || m.nnz < 0) return "bad matrix sizes";
        if (!m.rowptr && m.nrows > 0) return "null rowptr in the result";
        if (m.nnz > 0 && (!m.col || !m.val)) return "null matrix array in the result";
        HostCsr& h = *dst[i];
        h.nrows = m.nrows;
        h.ncols = m.ncols;
        h.rowptr.assign((size_t)m.nrows + 1, 0);
        h.col.resize((size_t)m.nnz);
        h.val.resize((size_t)m.nnz);
        if (m.rowptr) copy(h.rowptr.data(), m.rowptr, 8 * ((size_t)m.nrows + 1));
        copy(h.col.data(), m.col, 4 * (size_t)m.nnz);
        copy(h.val.data(), m.val, 8 * (size_t)m.nnz);
    }
    return "";
}

std::string graph_check_rowptrs(const GraphInput& in) {
    for (const HostCsr* h : {&in.m10, &in.m10t, &in.m21, &in.m21t, &in.m32, &in.m32t}) {
        if (h->rowptr[0] != 0 || h->rowptr.back() != (int64_t)h->col.size())
            return "matrix rowptr does not match its nnz";
        for (size_t i = 0; i + 1 < h->rowptr.size(); i++)
            if (h->rowptr[i + 1] < h->rowptr[i]) return "matrix rowptr decreases";
        for (uint32_t c : h->col)
            if ((int64_t)c >= h->ncols) return "matrix column out of range";
    }
    return "";
}

}  // namespace msc

extern "C" {

ms_status ms_graph_build(ms_ctx* ctx, const ms_result* r, ms_dims dims, int nthreads, ms_graph** out) {
    API_BEGIN
    if (!r || !out || nthreads < 1 || nthreads > 1024) fail(ctx, MS_ERR_INVALID_ARG, "null argument or bad thread count");
    *out = nullptr;
    check_dims(ctx, dims);
    GraphInput in;
    std::string e;
    try {
        e = graph_input(r, dims, in, [&](void* dst, const void* src, size_t bytes) {
            if (bytes) check(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream), "copy to host");
        });
    } catch (const std::bad_alloc&) {
        fail(ctx, MS_ERR_OOM, "host allocation failed");
    }
    check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
    if (e.empty()) e = graph_check_rowptrs(in);
    if (!e.empty()) fail(ctx, MS_ERR_INVALID_ARG, e);
    ms_graph* g = graph_from_host(in, nthreads, &e);
    if (!g) fail(ctx, MS_ERR_INVALID_ARG, e);
    *out = g;
    API_END
}

ms_status ms_graph_build_host(const ms_result* r, ms_dims dims, int nthreads, ms_graph** out) {
    if (!out) return MS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!r || nthreads < 1 || nthreads > 1024 || dims.nx < 1 || dims.ny < 1 || dims.nz < 1) return MS_ERR_INVALID_ARG;
    try {
        GraphInput in;
        std::string e = graph_input(r, dims, in, [](void* dst, const void* src, size_t bytes) {
            if (bytes) memcpy(dst, src, bytes);
        });
        if (e.empty()) e = graph_check_rowptrs(in);
        if (!e.empty()) return MS_ERR_INVALID_ARG;
        ms_graph* g = graph_from_host(in, nthreads, &e);
        if (!g) return MS_ERR_INVALID_ARG;
        *out = g;
    } catch (const std::bad_alloc&) {
        return MS_ERR_OOM;
    } catch (...) {
        return MS_ERR_INTERNAL;
    }
    return MS_OK;
}

}  // extern "C"

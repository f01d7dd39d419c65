// extern "C" entry points of libmsc.so (declared and documented in
// include/msc.h).  Each validates its arguments, runs its kernels on the
// context's stream and converts failures into ms_status codes.
#include <string.h>

#include "ctx.h"
#include "prims.h"

namespace msc {
hipError_t launch_gradient(const float* f, const Grid& g, uint32_t* grad, int* err, hipStream_t s);
size_t crit_tmp_elems(uint64_t nv);
hipError_t launch_crit_count(const uint32_t* grad, const Grid& g, uint64_t* tmp, uint64_t** d_totals, hipStream_t s);
hipError_t launch_crit_scatter(const float* f, const uint32_t* grad, const Grid& g, const uint64_t* tmp, uint32_t* id,
                               uint8_t* index, float* value, uint32_t* vmax, hipStream_t s);
void connect_impl(ms_ctx* c, const uint32_t* grad, const Grid& g, const uint32_t* crit_id, const int64_t count[4],
                  ms_arcs* out);

Grid check_dims(ms_ctx* c, ms_dims d) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) fail(c, MS_ERR_INVALID_ARG, "every dimension must be >= 1");
    if (d.nx > (1 << 29) || d.ny > (1 << 29) || d.nz > (1 << 29) || d.nx * d.ny > ((int64_t)1 << 29) ||
        d.nx * d.ny * d.nz > ((int64_t)1 << 29))
        fail(c, MS_ERR_TOO_LARGE, "nx*ny*nz must not exceed 2^29 (cell ids are 32-bit)");
    return Grid::make(d.nx, d.ny, d.nz);
}

// gradient + non-finite flag (flag left on the device at *d_err)
void gradient_impl(ms_ctx* c, const float* f, const Grid& g, uint32_t* grad, int* d_err) {
    check(c, hipMemsetAsync(d_err, 0, sizeof(int), c->stream), "clear error flag");
    check(c, launch_gradient(f, g, grad, d_err, c->stream), "gradient kernel launch");
}

// counts per index (host) after pass 1; optional scatter into `out`
void critical_impl(ms_ctx* c, const float* f, const uint32_t* grad, const Grid& g, const ms_crit* out,
                   int64_t h_count[4], const int* d_err, ms_status* nonfinite) {
    uint64_t* tmp = buf<uint64_t>(c, "crit_tmp", crit_tmp_elems(g.nv) + 1);
    uint64_t* d_tot = nullptr;
    check(c, launch_crit_count(grad, g, tmp, &d_tot, c->stream), "critical count launch");
    uint64_t* flag_slot = tmp + crit_tmp_elems(g.nv);
    if (d_err) {
        check(c, hipMemsetAsync(flag_slot, 0, sizeof(uint64_t), c->stream), "flag clear");
        check(c, hipMemcpyAsync(flag_slot, d_err, sizeof(int), hipMemcpyDeviceToDevice, c->stream), "flag copy");
    }
    check(c, hipMemcpyAsync(c->h_small, d_tot, 8 * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream), "readback");
    check(c, hipMemcpyAsync(c->h_small + 8, flag_slot, sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream),
          "readback");
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
    check(c, launch_crit_scatter(f, grad, g, tmp, out->id, out->index, out->value, out->vmax, c->stream),
          "critical scatter launch");
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

ms_status ms_ctx_create(ms_ctx** out, void* stream) {
    if (!out) return MS_ERR_INVALID_ARG;
    *out = nullptr;
    ms_ctx* c = new (std::nothrow) ms_ctx();
    if (!c) return MS_ERR_OOM;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return MS_ERR_HIP;
    }
    if (hipHostMalloc((void**)&c->h_small, 64 * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return MS_ERR_OOM;
    }
    *out = c;
    return MS_OK;
}

void ms_ctx_destroy(ms_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    if (ctx->h_small) (void)hipHostFree(ctx->h_small);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

ms_status ms_ctx_set_stream(ms_ctx* ctx, void* stream) {
    if (!ctx) return MS_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)stream;
    return MS_OK;
}

const char* ms_last_error(const ms_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ms_status ms_ctx_set_option(ms_ctx* ctx, int option, int64_t value) {
    if (!ctx) return MS_ERR_INVALID_ARG;
    if (option == MS_OPT_PATH_SCHEDULE && (value == MS_PATHS_READY || value == MS_PATHS_POWER)) {
        ctx->path_schedule = (int)value;
        return MS_OK;
    }
    if (option == MS_OPT_MERGE_LIGHT && value >= 0 && value <= 32) {
        ctx->merge_light = (uint32_t)value;
        return MS_OK;
    }
    if (option == MS_OPT_MERGE_CHUNK && value >= 1 && value <= 4096) {
        ctx->merge_chunk = (uint32_t)value;
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
    out->calls = ctx->calls;
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
    critical_impl(ctx, d_f, d_grad, g, out, h_count, nullptr, &st);
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
    critical_impl(ctx, nullptr, d_grad, g, nullptr, have, nullptr, &st);
    for (int k = 0; k < 4; k++)
        if (have[k] != h_count[k]) fail(ctx, MS_ERR_INVALID_ARG, "critical counts do not match the gradient");
    connect_impl(ctx, d_grad, g, d_crit_id, h_count, out);
    API_END
}

ms_status ms_complex(ms_ctx* ctx, const float* d_f, ms_dims dims, ms_result* out) {
    API_BEGIN
    Grid g = check_dims(ctx, dims);
    if (!d_f || !out) fail(ctx, MS_ERR_INVALID_ARG, "null argument");
    memset(out, 0, sizeof(*out));
    uint32_t* grad = buf<uint32_t>(ctx, "cx_grad", g.nv);
    int* d_err = buf<int>(ctx, "err_flag", 4);
    check(ctx, hipMemsetAsync(d_err, 0, sizeof(int), ctx->stream), "clear error flag");
    mark(ctx, 0);
    check(ctx, launch_gradient(d_f, g, grad, d_err, ctx->stream), "gradient kernel launch");
    mark(ctx, 1);
    int64_t cnt[4];
    ms_status st = MS_OK;
    critical_impl(ctx, d_f, grad, g, nullptr, cnt, d_err, &st);
    if (st == MS_ERR_NONFINITE) fail(ctx, st, "the field contains NaN or infinite values");
    int64_t total = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    ms_crit cr;
    cr.id = buf<uint32_t>(ctx, "cx_crit_id", total);
    cr.index = buf<uint8_t>(ctx, "cx_crit_index", total);
    cr.value = buf<float>(ctx, "cx_crit_value", total);
    cr.vmax = buf<uint32_t>(ctx, "cx_crit_vmax", total);
    cr.capacity = total;
    if (total > 0)
        check(ctx, launch_crit_scatter(d_f, grad, g, buf<uint64_t>(ctx, "crit_tmp", 1), cr.id, cr.index, cr.value,
                                       cr.vmax, ctx->stream),
              "critical scatter launch");
    out->grad = grad;
    out->crit = cr;
    for (int k = 0; k < 4; k++) out->count[k] = cnt[k];
    mark(ctx, 2);
    connect_impl(ctx, grad, g, cr.id, cnt, &out->arcs);
    mark(ctx, 6);
    if (ctx->timing) {
        check(ctx, hipEventSynchronize(ctx->ev[6]), "event synchronize");
        for (int i = 0; i < 6; i++) {
            float ms = 0;
            check(ctx, hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]), "event elapsed");
            ctx->acc_ms[i] += ms;
        }
        float tot = 0;
        check(ctx, hipEventElapsedTime(&tot, ctx->ev[0], ctx->ev[6]), "event elapsed");
        ctx->acc_ms[6] += tot;
        ctx->calls++;
    }
    API_END
}

}  // extern "C"

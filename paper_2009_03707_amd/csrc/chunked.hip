// Out-of-core gradient and critical cells: a field held in host memory, of
// any size, streamed through the GPU in z-slabs.
//
// The paper names device memory as the limit of its method (Section 5.2,
// memory usage) and cites the computation of parcels that are stitched
// afterwards (Section 1.1).  The gradient and the critical cells need no
// stitching: the pairing of a lower star depends only on the vertex's 26
// neighbours, and a gradient word holds the cells whose lowest corner is its
// vertex, whose lower stars are those of the word's vertex and of its +x /
// +y / +z neighbours.  So the words of rows [z0, z1) are exact when the
// gradient kernel runs on rows [z0 - 1, z1 + 2) as a grid of its own (the
// lower stars of rows [z0, z1 + 1) see all their neighbours there); rows
// outside [z0, z1) are computed and discarded.  The critical cells of those
// rows are then extracted from the exact words alone, with 64-bit cell ids
// (8 * vertex + nibble, vertex = x + nx (y + ny z)) so the field may exceed
// the 2^29 vertices of the in-HBM entry points.
//
// Pipelining: two device field buffers and two pinned staging buffers (kept
// by the context); the slab after the current one is copied into staging by
// host threads and sent on a copy stream while the current slab is computed
// on the context's stream.  Each slab's records are widened to 64 bits on
// the device and copied back as they are into pinned blocks the context
// keeps (one chunk per slab); once all slabs are done, host threads gather
// the chunks into the index-major output.
#include <algorithm>
#include <atomic>
#include <functional>
#include <memory>
#include <thread>
#include <string.h>

#include <vector>

#include "ctx.h"
#include "prims.h"

namespace msc {
uint32_t gradient_tiles(const Grid& g, int shape);
hipError_t launch_gradient(int shape, const float* f0, const float* const* fptr, const Geo& geo,
                           const uint32_t* tile_off, uint64_t total_tiles, uint32_t* grad, int* err, hipStream_t s);
size_t crit_tmp_elems(uint64_t nv);
hipError_t launch_crit_count(const uint32_t* grad, const Geo& g, uint64_t* tmp, uint64_t** d_totals, hipStream_t s);
hipError_t launch_crit_scatter(const float* f0, const float* const* fptr, const uint32_t* grad, const Geo& g,
                               const uint64_t* tmp, uint32_t* id, uint8_t* index, float* value, uint32_t* vmax,
                               hipStream_t s, uint64_t cap = ~0ull);
Geo single(const Grid& g);
void flag_clear(ms_ctx* c, int* d_err);
hipError_t launch_pj_round(uint32_t* P, uint32_t n, int* changed, hipStream_t s);

namespace {

// ids widened to 64 bits and moved to the slab's place in the field
__global__ void k_widen(const uint32_t* __restrict__ id, const uint32_t* __restrict__ vmax, uint64_t n, uint64_t vbase,
                        uint64_t* __restrict__ id64, uint64_t* __restrict__ vmax64) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    id64[i] = 8 * vbase + id[i];
    vmax64[i] = vbase + vmax[i];
}

// ---- manifold labels of an out-of-core field (Section 3.4), stitched ----
//
// Within a slab's exact rows [z0, z1), the vertex and cube pointers of the
// in-HBM path are built from the words (slab-local ids, < 2^29); a pointer
// that crosses z0 or z1 into another slab ends its chain instead, as a root
// that records where it leaves: ROOT_FLAG | OOC_EXIT | (local id of the
// last cell in the slab).  Pointer jumping then gives every cell either its
// extremum (ROOT_FLAG | rank in the slab) or the cell through which its path
// leaves the slab, and the resolve kernel turns that into a 64-bit label:
// the global rank of the extremum, or OOC_PENDING | the global id of the
// cell in the neighbouring slab the path continues in.  Those cells lie in
// the first or last row of a slab, so the host stitches the slabs by first
// resolving the pending labels of those boundary rows among themselves (a
// (0,1) or (2,3) path never returns to a cell, so every chain ends), then
// every other pending label with one lookup.
constexpr uint32_t OOC_EXIT = 0x40000000u;  // with ROOT_FLAG: the path leaves the slab here
constexpr uint32_t OOC_LOCAL = 0x1FFFFFFFu;  // slab-local vertex ids are < 2^29
constexpr uint64_t OOC_PENDING = 1ull << 62;
constexpr uint64_t OOC_NONE = ~0ull;        // no cube, or its path leaves the grid

// The successor of vertex v (local, rows [0, gi.n[2]) of the slab, global
// rows z0 + local) and of the cube with lowest corner v.
__global__ void k_ooc_ptr(const uint32_t* __restrict__ grad, Grid gi, uint64_t nzg, uint64_t z0,
                          uint32_t* __restrict__ Pv, uint32_t* __restrict__ Pc, int* __restrict__ err) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= gi.nv) return;
    const uint32_t v = (uint32_t)i;
    uint32_t c[3];
    gi.coords(v, c);
    const uint64_t zg = z0 + c[2];
    const uint32_t w = grad[v];
    const uint32_t n0 = w & 15u;
    uint32_t pv = ROOT_FLAG;  // a minimum: its rank comes from the critical list
    if (n0 >= 1 && n0 <= 6) {
        const uint32_t a = (n0 - 1u) >> 1;
        const bool neg = ((n0 - 1u) & 1u) != 0;
        const bool inside = a < 2 ? (neg ? c[a] >= 1 : c[a] + 1 < gi.n[a]) : (neg ? zg >= 1 : zg + 1 < nzg);
        if (!inside)
            atomicOr(err, 1);
        else if (a == 2 && (neg ? c[2] == 0 : c[2] + 1 == gi.n[2]))
            pv = ROOT_FLAG | OOC_EXIT | v;
        else
            pv = neg ? v - gi.stride[a] : v + gi.stride[a];
    } else if (n0 < NB_CRIT) {
        atomicOr(err, 1);
    }
    Pv[v] = pv;
    const uint32_t n7 = (w >> 28) & 15u;
    uint32_t pc = EXIT_LABEL;
    if (n7 >= NB_CRIT) {
        pc = ROOT_FLAG;  // a maximum
    } else if (n7 >= 1 && n7 <= 6) {
        const uint32_t a = (n7 - 1u) >> 1;
        const bool neg = ((n7 - 1u) & 1u) != 0;
        const bool inside = a < 2 ? (neg ? c[a] >= 1 : c[a] + 2 < gi.n[a]) : (neg ? zg >= 1 : zg + 2 < nzg);
        if (inside) {
            if (a == 2 && (neg ? c[2] == 0 : c[2] + 1 == gi.n[2]))
                pc = ROOT_FLAG | OOC_EXIT | v;
            else
                pc = neg ? v - gi.stride[a] : v + gi.stride[a];
        }
    } else if (n7 != NB_NONE) {
        atomicOr(err, 1);
    }
    Pc[v] = pc;
}

// Roots of the slab's minima and maxima: their ranks among the slab's
// critical cells of that index (the list is sorted by (index, id)).
__global__ void k_ooc_roots(const uint32_t* __restrict__ id, uint64_t c0, uint64_t s3, uint64_t c3,
                            uint32_t* __restrict__ Pv, uint32_t* __restrict__ Pc) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < c0) Pv[id[i] >> 3] = ROOT_FLAG | (uint32_t)i;
    if (i < c3) Pc[id[s3 + i] >> 3] = ROOT_FLAG | (uint32_t)i;
}

__device__ inline uint64_t ooc_label(uint32_t p, uint32_t nib, uint64_t base, uint64_t vbase, uint64_t nxy) {
    if (p == EXIT_LABEL) return OOC_NONE;
    if (p & OOC_EXIT) {  // the path continues in the slab below (code 6: -z) or above (code 5: +z)
        const uint64_t r = vbase + (p & OOC_LOCAL);
        return OOC_PENDING | (nib == 6u ? r - nxy : r + nxy);
    }
    return base + (p & ~ROOT_FLAG);
}

__global__ void k_ooc_resolve(const uint32_t* __restrict__ Pv, const uint32_t* __restrict__ Pc,
                              const uint32_t* __restrict__ grad, uint64_t nv, uint64_t vbase, uint64_t nxy,
                              uint64_t min_base, uint64_t max_base, uint64_t* __restrict__ lmin,
                              uint64_t* __restrict__ lmax) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const uint32_t a = Pv[i], b = Pc[i];
    // an exit root names its own cell, whose word gives the direction
    const uint32_t wa = (a & ROOT_FLAG) && (a & OOC_EXIT) ? grad[a & OOC_LOCAL] : 0u;
    const uint32_t wb = b != EXIT_LABEL && (b & OOC_EXIT) ? grad[b & OOC_LOCAL] : 0u;
    lmin[i] = ooc_label(a, wa & 15u, min_base, vbase, nxy);
    lmax[i] = ooc_label(b, wb >> 28, max_base, vbase, nxy);
}

// Resolves the pending labels of L (host, nv entries): first those in the
// boundary rows listed (chains among those rows, followed to their end),
// then every other one from its target, which lies in such a row.  Returns
// false if a chain does not end or leaves the range (a gradient that is
// not acyclic; never the case for the words computed here).
bool stitch(uint64_t* L, uint64_t nv, uint64_t nxy, const std::vector<int64_t>& rows) {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const uint64_t limit = (uint64_t)rows.size() * nxy + 1;
    std::atomic<bool> ok{true};
    auto pending = [](uint64_t x) { return (x >> 62) == 1; };
    auto run = [&](uint64_t n, auto&& body) {
        std::vector<std::thread> th;
        const uint64_t per = (n + hw - 1) / hw;
        for (unsigned t = 0; t < hw; t++) {
            const uint64_t a = t * per, b = std::min(n, a + per);
            if (a >= b) break;
            th.emplace_back([&, a, b] { body(a, b); });
        }
        for (auto& x : th) x.join();
    };
    // boundary rows: a chain's labels are either still pending (and lead on)
    // or final, so threads may read each other's stores in any order
    run((uint64_t)rows.size() * nxy, [&](uint64_t a, uint64_t b) {
        for (uint64_t j = a; j < b && ok.load(std::memory_order_relaxed); j++) {
            const uint64_t v = (uint64_t)rows[j / nxy] * nxy + j % nxy;
            uint64_t x = __atomic_load_n(&L[v], __ATOMIC_RELAXED);
            uint64_t steps = 0;
            while (pending(x)) {
                const uint64_t t = x & (OOC_PENDING - 1);
                if (t >= nv || ++steps > limit) {
                    ok = false;
                    break;
                }
                x = __atomic_load_n(&L[t], __ATOMIC_RELAXED);
            }
            if (!pending(x)) __atomic_store_n(&L[v], x, __ATOMIC_RELAXED);
        }
    });
    if (!ok) return false;
    run(nv, [&](uint64_t a, uint64_t b) {
        for (uint64_t v = a; v < b; v++) {
            const uint64_t x = L[v];
            if (!pending(x)) continue;
            const uint64_t t = x & (OOC_PENDING - 1);
            const uint64_t y = t < nv ? L[t] : x;
            if (pending(y)) {
                ok = false;
                return;
            }
            L[v] = y;
        }
    });
    return ok;
}

// memcpy split over host threads
void par_copy(void* dst, const void* src, size_t bytes) {
    constexpr size_t MIN_PART = (size_t)8 << 20;
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const size_t parts = std::min<size_t>(hw, std::max<size_t>(1, bytes / MIN_PART));
    if (parts <= 1) {
        memcpy(dst, src, bytes);
        return;
    }
    const size_t per = (bytes + parts - 1) / parts;
    std::vector<std::thread> th;
    for (size_t t = 0; t < parts; t++) {
        const size_t a = t * per, b = std::min(bytes, a + per);
        if (a >= b) break;
        th.emplace_back([=] { memcpy((char*)dst + a, (const char*)src + a, b - a); });
    }
    for (auto& x : th) x.join();
}

// one slab's records, as copied back: per index, count; ids, vertices, values
struct Chunk {
    int64_t cnt[4] = {0, 0, 0, 0};
    const uint64_t* id = nullptr;
    const uint64_t* vmax = nullptr;
    const float* value = nullptr;
};

// Bump allocation of the slabs' records in the context's pinned blocks
// (kept and reused by later calls; a block is added when none has room).
struct RecordArena {
    ms_ctx* c;
    size_t blk = 0, used = 0;
    void* take(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        while (blk < c->h_recs.size() && used + bytes > c->h_recs[blk].second) {
            blk++;
            used = 0;
        }
        if (blk == c->h_recs.size()) {
            const size_t prev = c->h_recs.empty() ? 0 : c->h_recs.back().second;
            const size_t want = std::max({bytes, 2 * prev, (size_t)256 << 20});
            void* p = nullptr;
            if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                fail(c, MS_ERR_OOM, "pinned record allocation failed");
            }
            c->h_recs.emplace_back(p, want);
            used = 0;
        }
        void* p = (char*)c->h_recs[blk].first + used;
        used += bytes;
        return p;
    }
};

// A host copy started once its source is ready (start) and waited for
// before the source is reused or the call returns (join, also on errors).
struct Copier {
    std::function<void()> pending;
    std::thread t;
    void start() {
        if (pending) t = std::thread(std::move(pending));
        pending = nullptr;
    }
    void join() {
        if (t.joinable()) t.join();
    }
    ~Copier() { join(); }
};

struct Ev {
    hipEvent_t e = nullptr;
    ~Ev() {
        if (e) (void)hipEventDestroy(e);
    }
};

struct Stream {
    hipStream_t s = nullptr;
    ~Stream() {
        if (s) (void)hipStreamDestroy(s);
    }
};

}  // namespace
}  // namespace msc

using namespace msc;

namespace {

// One pass over the slabs: gradient words (h_grad), critical records (out)
// and manifold labels (h_min, h_max), each when its pointer is not null.
ms_status chunked(ms_ctx* ctx, const float* h_f, ms_dims dims, int64_t slab, uint32_t* h_grad, const ms_crit64* out,
                  int64_t h_count[4], uint64_t* h_min, uint64_t* h_max) {
    if (!ctx) return MS_ERR_INVALID_ARG;
    try {
        if (!h_f || !h_count) fail(ctx, MS_ERR_INVALID_ARG, "null field or count pointer");
        const bool labels = h_min || h_max;
        if (dims.nx < 1 || dims.ny < 1 || dims.nz < 1 || slab < 1) fail(ctx, MS_ERR_INVALID_ARG, "dims and slab must be >= 1");
        const int64_t nx = dims.nx, ny = dims.ny, nz = dims.nz;
        if (nx > (1 << 29) || ny > (1 << 29) || nx * ny > ((int64_t)1 << 29))
            fail(ctx, MS_ERR_TOO_LARGE, "nx*ny must not exceed 2^29");
        if (nz > ((int64_t)1 << 40) / (nx * ny)) fail(ctx, MS_ERR_TOO_LARGE, "field larger than 2^40 vertices");
        const int64_t nxy = nx * ny;
        if (slab > nz) slab = nz;
        // a slab plus its halo (one row below, two above) must be one in-HBM grid
        const int64_t max_rows = ((int64_t)1 << 29) / nxy;
        if (max_rows < 4) fail(ctx, MS_ERR_TOO_LARGE, "an xy plane is too large for slabs of one row plus halo");
        if (slab + 3 > max_rows) slab = max_rows - 3;
        const int64_t rows_cap = slab + 3;
        const size_t fbytes = (size_t)(rows_cap * nxy) * sizeof(float);

        hipStream_t cs = ctx->stream;
        Stream xs;
        check(ctx, hipStreamCreateWithFlags(&xs.s, hipStreamNonBlocking), "stream create");
        if (ctx->h_stage_bytes < fbytes) {
            check(ctx, hipStreamSynchronize(cs), "stream synchronize");
            for (void*& p : ctx->h_stage) {
                if (p) (void)hipHostFree(p);
                p = nullptr;
            }
            ctx->h_stage_bytes = 0;
            for (void*& p : ctx->h_stage)
                if (hipHostMalloc(&p, fbytes, hipHostMallocDefault) != hipSuccess) {
                    (void)hipGetLastError();
                    p = nullptr;
                    fail(ctx, MS_ERR_OOM, "pinned staging allocation failed");
                }
            ctx->h_stage_bytes = fbytes;
        }
        Ev ev_h2d[2], ev_done[2];
        for (int b = 0; b < 2; b++) {
            check(ctx, hipEventCreateWithFlags(&ev_h2d[b].e, hipEventDisableTiming), "event create");
            check(ctx, hipEventCreateWithFlags(&ev_done[b].e, hipEventDisableTiming), "event create");
        }
        float* d_f[2] = {buf<float>(ctx, "ooc.f0", (size_t)(rows_cap * nxy)),
                         buf<float>(ctx, "ooc.f1", (size_t)(rows_cap * nxy))};
        uint32_t* d_grad = buf<uint32_t>(ctx, "ooc.grad", (size_t)(rows_cap * nxy));
        uint64_t* tmp = buf<uint64_t>(ctx, "ooc.tmp", crit_tmp_elems((uint64_t)(slab * nxy)) + 1);
        int* d_err = buf<int>(ctx, "ooc.err", 4);

        const int64_t nslab = (nz + slab - 1) / slab;
        std::vector<Chunk> chunks((size_t)nslab);
        uint64_t min_base = 0, max_base = 0;  // minima / maxima in earlier slabs
        int* d_lerr = labels ? buf<int>(ctx, "ooc.lerr", 64) : nullptr;
        // labels and gradient words come back through two pinned buffers
        // (one slab's outputs each: minima labels, maxima labels, words);
        // host threads copy a slab's outputs into the caller's arrays while
        // the GPU works on the next slab
        Copier lab_copy[2];
        const bool staged = labels || h_grad;
        const size_t lab_bytes = (size_t)((labels ? 16 : 0) + (h_grad ? 4 : 0)) * (size_t)(slab * nxy);
        if (staged && ctx->h_lab_bytes < lab_bytes) {
            check(ctx, hipStreamSynchronize(cs), "stream synchronize");
            for (void*& p : ctx->h_lab) {
                if (p) (void)hipHostFree(p);
                p = nullptr;
            }
            ctx->h_lab_bytes = 0;
            for (void*& p : ctx->h_lab)
                if (hipHostMalloc(&p, lab_bytes, hipHostMallocDefault) != hipSuccess) {
                    (void)hipGetLastError();
                    p = nullptr;
                    fail(ctx, MS_ERR_OOM, "pinned output staging allocation failed");
                }
            ctx->h_lab_bytes = lab_bytes;
        }
        int* d_chg = labels ? buf<int>(ctx, "ooc.chg", 64) : nullptr;
        if (labels) check(ctx, hipMemsetAsync(d_lerr, 0, 2 * sizeof(int), cs), "memset");
        RecordArena arena{ctx};
        auto rows_of = [&](int64_t i, int64_t& z0, int64_t& z1, int64_t& zs, int64_t& ze) {
            z0 = i * slab;
            z1 = z0 + slab < nz ? z0 + slab : nz;
            zs = z0 > 0 ? z0 - 1 : 0;
            ze = z1 + 2 < nz ? z1 + 2 : nz;
        };
        // host copy into staging, then H2D on the copy stream once the
        // device buffer's previous slab is done
        auto send = [&](int64_t i) {
            int64_t z0, z1, zs, ze;
            rows_of(i, z0, z1, zs, ze);
            const int b = (int)(i & 1);
            check(ctx, hipEventSynchronize(ev_h2d[b].e), "event synchronize");  // staging b free
            const size_t bytes = (size_t)((ze - zs) * nxy) * sizeof(float);
            par_copy(ctx->h_stage[b], h_f + zs * nxy, bytes);
            check(ctx, hipStreamWaitEvent(xs.s, ev_done[b].e, 0), "stream wait");
            check(ctx, hipMemcpyAsync(d_f[b], ctx->h_stage[b], bytes, hipMemcpyHostToDevice, xs.s), "copy to device");
            check(ctx, hipEventRecord(ev_h2d[b].e, xs.s), "event record");
        };
        for (int b = 0; b < 2; b++) {  // events start signalled
            check(ctx, hipEventRecord(ev_h2d[b].e, xs.s), "event record");
            check(ctx, hipEventRecord(ev_done[b].e, cs), "event record");
        }
        send(0);
        bool nonfinite = false;
        for (int64_t i = 0; i < nslab; i++) {
            int64_t z0, z1, zs, ze;
            rows_of(i, z0, z1, zs, ze);
            const int b = (int)(i & 1);
            check(ctx, hipStreamWaitEvent(cs, ev_h2d[b].e, 0), "stream wait");
            const Grid gs = Grid::make(nx, ny, ze - zs);
            flag_clear(ctx, d_err);
            check(ctx, launch_gradient(ctx->grad_tile, d_f[b], nullptr, single(gs), nullptr,
                                       gradient_tiles(gs, ctx->grad_tile), d_grad, d_err, cs),
                  "gradient kernel launch");
            if (i + 1 < nslab) send(i + 1);
            // the exact rows [z0, z1) as a grid of their own
            const int64_t off = (z0 - zs) * nxy;
            const Grid gi = Grid::make(nx, ny, z1 - z0);
            uint64_t* d_tot = nullptr;
            check(ctx, launch_crit_count(d_grad + off, single(gi), tmp, &d_tot, cs), "critical count launch");
            check(ctx, launch_publish(d_tot, 8, ctx->h_small_dev, cs), "readback");
            check(ctx, launch_publish((const uint64_t*)d_err, 1, ctx->h_small_dev + 8, cs), "readback");
            check(ctx, hipStreamSynchronize(cs), "stream synchronize");
            int flag = 0;
            memcpy(&flag, ctx->h_small + 8, sizeof(int));
            if (flag) {
                nonfinite = true;
                check(ctx, hipEventRecord(ev_done[b].e, cs), "event record");
                break;
            }
            Chunk& ch = chunks[(size_t)i];
            int64_t n = 0;
            for (int k = 0; k < 4; k++) {
                ch.cnt[k] = (int64_t)ctx->h_small[k];
                n += ch.cnt[k];
            }
            // the slab's records (grow-only buffers, sized by this slab's count)
            uint32_t* d_id = buf<uint32_t>(ctx, "ooc.id", (size_t)n);
            uint8_t* d_index = buf<uint8_t>(ctx, "ooc.index", (size_t)n);
            float* d_value = buf<float>(ctx, "ooc.value", (size_t)n);
            uint32_t* d_vmax = buf<uint32_t>(ctx, "ooc.vmax", (size_t)n);
            uint64_t* d_id64 = buf<uint64_t>(ctx, "ooc.id64", (size_t)n);
            uint64_t* d_vmax64 = buf<uint64_t>(ctx, "ooc.vmax64", (size_t)n);
            if (n > 0 && (out || labels))
                check(ctx, launch_crit_scatter(d_f[b] + off, nullptr, d_grad + off, single(gi), tmp, d_id, d_index,
                                               d_value, d_vmax, cs),
                      "critical scatter launch");
            if (n > 0 && out) {
                hipLaunchKernelGGL(k_widen, dim3(grid_blocks((uint64_t)n, 256)), dim3(256), 0, cs, (const uint32_t*)d_id,
                                   (const uint32_t*)d_vmax, (uint64_t)n, (uint64_t)z0 * (uint64_t)nxy, d_id64, d_vmax64);
                check(ctx, hipGetLastError(), "widen launch");
            }
            check(ctx, hipEventRecord(ev_done[b].e, cs), "event record");  // d_f[b] may be refilled
            lab_copy[b].join();  // output staging b is free again
            const size_t ns = (size_t)((z1 - z0) * nxy);
            uint64_t* st_min = (uint64_t*)ctx->h_lab[b];  // [minima labels | maxima labels | words]
            uint64_t* st_max = labels ? st_min + ns : st_min;
            uint32_t* st_grad = (uint32_t*)(labels ? st_max + ns : st_min);
            if (labels) {
                const uint64_t nvi = gi.nv, vbase = (uint64_t)z0 * (uint64_t)nxy;
                uint32_t* Pv = buf<uint32_t>(ctx, "ooc.pv", (size_t)nvi);
                uint32_t* Pc = buf<uint32_t>(ctx, "ooc.pc", (size_t)nvi);
                uint64_t* lmin = buf<uint64_t>(ctx, "ooc.lmin", (size_t)nvi);
                uint64_t* lmax = buf<uint64_t>(ctx, "ooc.lmax", (size_t)nvi);
                hipLaunchKernelGGL(k_ooc_ptr, dim3(grid_blocks(nvi, 256)), dim3(256), 0, cs,
                                   (const uint32_t*)(d_grad + off), gi, (uint64_t)nz, (uint64_t)z0, Pv, Pc, d_lerr);
                check(ctx, hipGetLastError(), "pointer launch");
                const uint64_t c0 = (uint64_t)ch.cnt[0], c3 = (uint64_t)ch.cnt[3];
                if (c0 + c3 > 0) {
                    hipLaunchKernelGGL(k_ooc_roots, dim3(grid_blocks(std::max(c0, c3), 256)), dim3(256), 0, cs,
                                       (const uint32_t*)d_id, c0, (uint64_t)(n - ch.cnt[3]), c3, Pv, Pc);
                    check(ctx, hipGetLastError(), "roots launch");
                }
                for (uint32_t* P : {Pv, Pc})
                    for (int rounds = 0;; rounds++) {
                        if (rounds > 64) fail(ctx, MS_ERR_INTERNAL, "pointer jumping did not converge");
                        check(ctx, hipMemsetAsync(d_chg, 0, 64 * sizeof(int), cs), "memset");
                        check(ctx, launch_pj_round(P, (uint32_t)nvi, d_chg, cs), "pointer jumping launch");
                        const uint64_t* h = readback(ctx, (const uint64_t*)d_chg, 32);
                        bool any = false;
                        for (int q = 0; q < 32; q++) any = any || h[q] != 0;
                        if (!any) break;
                    }
                hipLaunchKernelGGL(k_ooc_resolve, dim3(grid_blocks(nvi, 256)), dim3(256), 0, cs, (const uint32_t*)Pv,
                                   (const uint32_t*)Pc, (const uint32_t*)(d_grad + off), nvi, vbase, (uint64_t)nxy,
                                   min_base, max_base, lmin, lmax);
                check(ctx, hipGetLastError(), "resolve launch");
                if (h_min)
                    check(ctx, hipMemcpyAsync(st_min, lmin, 8 * nvi, hipMemcpyDeviceToHost, cs), "copy to host");
                if (h_max)
                    check(ctx, hipMemcpyAsync(st_max, lmax, 8 * nvi, hipMemcpyDeviceToHost, cs), "copy to host");
                min_base += c0;
                max_base += c3;
            }
            if (h_grad)
                check(ctx, hipMemcpyAsync(st_grad, d_grad + off, 4 * ns, hipMemcpyDeviceToHost, cs), "copy to host");
            if (staged) {
                const size_t vbase = (size_t)(z0 * nxy);
                lab_copy[b].pending = [=] {
                    if (h_min) par_copy(h_min + vbase, st_min, 8 * ns);
                    if (h_max) par_copy(h_max + vbase, st_max, 8 * ns);
                    if (h_grad) par_copy(h_grad + vbase, st_grad, 4 * ns);
                };
            }
            if (n > 0 && out) {
                uint64_t* hid = (uint64_t*)arena.take(8 * (size_t)n);
                uint64_t* hvm = (uint64_t*)arena.take(8 * (size_t)n);
                float* hval = (float*)arena.take(4 * (size_t)n);
                ch.id = hid;
                ch.vmax = hvm;
                ch.value = hval;
                check(ctx, hipMemcpyAsync(hid, d_id64, 8 * (size_t)n, hipMemcpyDeviceToHost, cs), "copy to host");
                check(ctx, hipMemcpyAsync(hvm, d_vmax64, 8 * (size_t)n, hipMemcpyDeviceToHost, cs), "copy to host");
                check(ctx, hipMemcpyAsync(hval, d_value, 4 * (size_t)n, hipMemcpyDeviceToHost, cs), "copy to host");
            }
            check(ctx, hipStreamSynchronize(cs), "stream synchronize");
            lab_copy[b].start();
        }
        check(ctx, hipStreamSynchronize(xs.s), "stream synchronize");
        for (Copier& cp : lab_copy) cp.join();
        if (nonfinite) fail(ctx, MS_ERR_NONFINITE, "the field contains NaN or infinite values");
        if (labels) {
            const uint64_t* h = readback(ctx, (const uint64_t*)d_lerr, 1);
            if ((int)*h) fail(ctx, MS_ERR_INTERNAL, "inconsistent gradient words");
            std::vector<int64_t> rows;  // first and last row of every slab
            for (int64_t i = 0; i < nslab; i++) {
                int64_t z0, z1, zs, ze;
                rows_of(i, z0, z1, zs, ze);
                rows.push_back(z0);
                if (z1 - 1 > z0) rows.push_back(z1 - 1);
            }
            for (uint64_t* L : {h_min, h_max})
                if (L && !stitch(L, (uint64_t)(nxy * nz), (uint64_t)nxy, rows))
                    fail(ctx, MS_ERR_INTERNAL, "a path between slabs does not end");
        }
        int64_t total = 0;
        for (int k = 0; k < 4; k++) {
            h_count[k] = 0;
            for (const Chunk& ch : chunks) h_count[k] += ch.cnt[k];
            total += h_count[k];
        }
        if (!out) return MS_OK;
        if (total > out->capacity) fail(ctx, MS_ERR_CAPACITY, "critical output capacity too small");
        if (total > 0 && (!out->id || !out->index || !out->value || !out->vmax))
            fail(ctx, MS_ERR_INVALID_ARG, "null critical output array");
        // the slabs' lists are sorted by (index, id) and the slabs come in id
        // order, so index k's records are the slabs' index-k runs in slab order
        struct Piece {
            const Chunk* ch;
            int64_t src, dst, n;
            int k;
        };
        std::vector<Piece> pieces;
        int64_t dst = 0;
        for (int k = 0; k < 4; k++)
            for (const Chunk& ch : chunks) {
                int64_t src = 0;
                for (int q = 0; q < k; q++) src += ch.cnt[q];
                if (ch.cnt[k] > 0) pieces.push_back(Piece{&ch, src, dst, ch.cnt[k], k});
                dst += ch.cnt[k];
            }
        const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < hw; t++)
            th.emplace_back([&, t] {
                for (size_t j = t; j < pieces.size(); j += hw) {
                    const Piece& pc = pieces[j];
                    memcpy(out->id + pc.dst, pc.ch->id + pc.src, 8 * (size_t)pc.n);
                    memcpy(out->vmax + pc.dst, pc.ch->vmax + pc.src, 8 * (size_t)pc.n);
                    memcpy(out->value + pc.dst, pc.ch->value + pc.src, 4 * (size_t)pc.n);
                    memset(out->index + pc.dst, pc.k, (size_t)pc.n);
                }
            });
        for (auto& x : th) x.join();
    } catch (const Fail& e) {
        return e.st;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return MS_ERR_OOM;
    } catch (const std::exception& e) {
        ctx->err = std::string("internal error: ") + e.what();
        return MS_ERR_INTERNAL;
    }
    return MS_OK;
}

}  // namespace

extern "C" ms_status ms_gradient_critical_chunked(ms_ctx* ctx, const float* h_f, ms_dims dims, int64_t slab,
                                                  uint32_t* h_grad, const ms_crit64* out, int64_t h_count[4]) {
    return chunked(ctx, h_f, dims, slab, h_grad, out, h_count, nullptr, nullptr);
}

extern "C" ms_status ms_manifolds_chunked(ms_ctx* ctx, const float* h_f, ms_dims dims, int64_t slab,
                                          uint64_t* h_min_label, uint64_t* h_max_label, int64_t h_count[4]) {
    return chunked(ctx, h_f, dims, slab, nullptr, nullptr, h_count, h_min_label, h_max_label);
}

// Saddle-extremum arcs from the stitched labels (host): a 1-saddle's row of
// M10 holds the minima of its two vertices, a 2-saddle's row of M32^T the
// maxima of its two cubes (paths that leave the grid dropped); an arc
// reached twice has multiplicity 2.  Two passes over the saddles (row
// lengths, then entries) split over host threads.
namespace {

struct SaddleRow {
    uint64_t c[2];
    int n;  // distinct columns (0..2); c[0] < c[1]
    uint64_t v0;  // multiplicity of c[0] when n == 1
};

bool arcs_host(ms_dims d, const uint64_t* lab, const uint64_t* ids, int64_t S, bool cubes, ms_csr64_host* out) {
    const uint64_t nx = (uint64_t)d.nx, ny = (uint64_t)d.ny, nz = (uint64_t)d.nz, nxy = nx * ny, nv = nxy * nz;
    const uint64_t n[3] = {nx, ny, nz}, stride[3] = {1, nx, nxy};
    auto row = [&](int64_t r, SaddleRow& o) -> bool {
        const uint64_t id = ids[r], v = id >> 3;
        const uint32_t k = (uint32_t)(id & 7u);
        if (v >= nv || __builtin_popcount(k) != (cubes ? 2 : 1)) return false;
        const uint64_t c[3] = {v % nx, (v / nx) % ny, v / nxy};
        for (int a = 0; a < 3; a++)
            if (((k >> a) & 1u) && c[a] + 1 >= n[a]) return false;  // the cell must exist
        uint64_t l[2];
        int m = 0;
        if (!cubes) {
            const int a = __builtin_ctz(k);
            l[0] = lab[v];
            l[1] = lab[v + stride[a]];
            if (l[0] == MS_LABEL_EXIT64 || l[1] == MS_LABEL_EXIT64) return false;
            m = 2;
        } else {
            const int j = k == 3u ? 2 : (k == 5u ? 1 : 0);  // the quad's normal axis
            const uint64_t e[2] = {c[j] + 1 < n[j] ? lab[v] : MS_LABEL_EXIT64,
                                   c[j] >= 1 ? lab[v - stride[j]] : MS_LABEL_EXIT64};
            for (uint64_t x : e)
                if (x != MS_LABEL_EXIT64) l[m++] = x;
        }
        if (m == 2 && l[0] == l[1]) {
            o.n = 1;
            o.c[0] = l[0];
            o.v0 = 2;
        } else {
            o.n = m;
            o.v0 = 1;
            o.c[0] = m == 2 ? std::min(l[0], l[1]) : l[0];
            o.c[1] = m == 2 ? std::max(l[0], l[1]) : 0;
        }
        return true;
    };
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::atomic<bool> ok{true};
    auto run = [&](auto&& body) {
        std::vector<std::thread> th;
        const int64_t per = (S + hw - 1) / hw;
        for (unsigned t = 0; t < hw; t++) {
            const int64_t a = t * per, b = std::min<int64_t>(S, a + per);
            if (a >= b) break;
            th.emplace_back([&, a, b] { body(a, b); });
        }
        for (auto& x : th) x.join();
    };
    out->rowptr[0] = 0;
    run([&](int64_t a, int64_t b) {
        SaddleRow o;
        for (int64_t r = a; r < b; r++) {
            if (!row(r, o)) {
                ok = false;
                return;
            }
            out->rowptr[r + 1] = o.n;
        }
    });
    if (!ok) return false;
    for (int64_t r = 0; r < S; r++) out->rowptr[r + 1] += out->rowptr[r];
    out->nnz = out->rowptr[S];
    if (out->nnz > out->capacity) return true;  // the caller sees nnz > capacity
    run([&](int64_t a, int64_t b) {
        SaddleRow o;
        for (int64_t r = a; r < b; r++) {
            row(r, o);
            const int64_t p = out->rowptr[r];
            for (int i = 0; i < o.n; i++) {
                out->col[p + i] = o.c[i];
                out->val[p + i] = o.v0;
            }
        }
    });
    return true;
}

}  // namespace

extern "C" ms_status ms_extremum_arcs_host(ms_dims dims, const uint64_t* h_min_label, const uint64_t* h_max_label,
                                           const uint64_t* s1_id, int64_t S1, const uint64_t* s2_id, int64_t S2,
                                           ms_csr64_host* m10, ms_csr64_host* m32t) {
    if (dims.nx < 1 || dims.ny < 1 || dims.nz < 1 || S1 < 0 || S2 < 0) return MS_ERR_INVALID_ARG;
    if (dims.nx > (1 << 29) || dims.ny > (1 << 29) || dims.nx * dims.ny > ((int64_t)1 << 29) ||
        dims.nz > ((int64_t)1 << 40) / (dims.nx * dims.ny))
        return MS_ERR_TOO_LARGE;
    try {
        for (int which = 0; which < 2; which++) {
            ms_csr64_host* o = which == 0 ? m10 : m32t;
            if (!o) continue;
            const uint64_t* lab = which == 0 ? h_min_label : h_max_label;
            const uint64_t* ids = which == 0 ? s1_id : s2_id;
            const int64_t S = which == 0 ? S1 : S2;
            if (!lab || !o->rowptr || (S > 0 && !ids) || o->capacity < 0 || (o->capacity > 0 && (!o->col || !o->val)))
                return MS_ERR_INVALID_ARG;
            if (!arcs_host(dims, lab, ids, S, which == 1, o)) return MS_ERR_INVALID_ARG;
        }
        if ((m10 && m10->nnz > m10->capacity) || (m32t && m32t->nnz > m32t->capacity)) return MS_ERR_CAPACITY;
    } catch (const std::exception&) {
        return MS_ERR_OOM;
    }
    return MS_OK;
}

extern "C" ms_status ms_csr64_transpose_host(const ms_csr64_host* in, int64_t nrows, int64_t ncols,
                                             ms_csr64_host* out) {
    if (!in || !out || nrows < 0 || ncols < 0 || !in->rowptr || !out->rowptr) return MS_ERR_INVALID_ARG;
    const int64_t nnz = in->rowptr[nrows];
    if (in->rowptr[0] != 0 || nnz < 0 || (nnz > 0 && (!in->col || !in->val))) return MS_ERR_INVALID_ARG;
    for (int64_t r = 0; r < nrows; r++)
        if (in->rowptr[r + 1] < in->rowptr[r]) return MS_ERR_INVALID_ARG;
    for (int64_t p = 0; p < nnz; p++)
        if (in->col[p] >= (uint64_t)ncols) return MS_ERR_INVALID_ARG;
    out->nnz = nnz;
    if (nnz > out->capacity) return MS_ERR_CAPACITY;
    if (nnz > 0 && (!out->col || !out->val)) return MS_ERR_INVALID_ARG;
    // A counting sort by column in two levels, so that no pass scatters over
    // all columns at once: the entries go to buckets of adjacent columns
    // (threads over equal shares of the entries, each keeping row order),
    // then each bucket is sorted by column on its own (threads over
    // buckets).  Both levels are stable, so each output row lists its
    // columns (the input rows) ascending.
    int64_t* rp = out->rowptr;
    if (ncols == 0) {
        rp[0] = 0;
        return MS_OK;
    }
    try {
        const int64_t T = std::max<int64_t>(1, std::min<int64_t>(std::min(16u, std::max(1u,
                                                 std::thread::hardware_concurrency())), nnz / 65536 + 1));
        const int64_t width = std::max<int64_t>(1, (ncols + 4095) / 4096);  // columns per bucket
        const int64_t nb = (ncols + width - 1) / width;
        std::vector<int64_t> rlo(T + 1);  // thread t takes rows [rlo[t], rlo[t+1])
        for (int64_t t = 0; t <= T; t++)
            rlo[t] = std::upper_bound(in->rowptr, in->rowptr + nrows + 1, t * nnz / T) - in->rowptr - 1;
        rlo[0] = 0;
        rlo[T] = nrows;
        std::vector<int64_t> cnt((size_t)(T * nb), 0);
        auto par = [&](int64_t n, auto&& body) {
            std::vector<std::thread> th;
            for (int64_t t = 0; t < std::min(n, T); t++)
                th.emplace_back([&, t] {
                    for (int64_t i = t; i < n; i += T) body(i);
                });
            for (auto& x : th) x.join();
        };
        par(T, [&](int64_t t) {
            int64_t* c = &cnt[(size_t)(t * nb)];
            for (int64_t p = in->rowptr[rlo[t]]; p < in->rowptr[rlo[t + 1]]; p++) c[in->col[p] / width]++;
        });
        std::vector<int64_t> bstart((size_t)nb + 1);
        int64_t run = 0;
        for (int64_t q = 0; q < nb; q++) {
            bstart[(size_t)q] = run;
            for (int64_t t = 0; t < T; t++) {
                const int64_t v = cnt[(size_t)(t * nb + q)];
                cnt[(size_t)(t * nb + q)] = run;
                run += v;
            }
        }
        bstart[(size_t)nb] = run;
        // not zeroed: the scatter below writes every entry (and faults the pages in on its threads)
        std::unique_ptr<int64_t[]> trow(new int64_t[(size_t)nnz]);
        std::unique_ptr<uint64_t[]> tcol(new uint64_t[(size_t)nnz]), tval(new uint64_t[(size_t)nnz]);
        par(T, [&](int64_t t) {
            int64_t* o = &cnt[(size_t)(t * nb)];
            for (int64_t r = rlo[t]; r < rlo[t + 1]; r++)
                for (int64_t p = in->rowptr[r]; p < in->rowptr[r + 1]; p++) {
                    const int64_t q = o[in->col[p] / width]++;
                    trow[(size_t)q] = r;
                    tcol[(size_t)q] = in->col[p];
                    tval[(size_t)q] = in->val[p];
                }
        });
        par(nb, [&](int64_t q) {
            const int64_t c0 = q * width, c1 = std::min(ncols, c0 + width);
            std::vector<int64_t> next((size_t)(c1 - c0), 0);
            for (int64_t p = bstart[(size_t)q]; p < bstart[(size_t)q + 1]; p++) next[(size_t)(tcol[(size_t)p] - c0)]++;
            int64_t at = bstart[(size_t)q];
            for (int64_t c = c0; c < c1; c++) {
                rp[c] = at;
                const int64_t v = next[(size_t)(c - c0)];
                next[(size_t)(c - c0)] = at;
                at += v;
            }
            for (int64_t p = bstart[(size_t)q]; p < bstart[(size_t)q + 1]; p++) {
                const int64_t d = next[(size_t)(tcol[(size_t)p] - c0)]++;
                out->col[d] = (uint64_t)trow[(size_t)p];
                out->val[d] = tval[(size_t)p];
            }
        });
        rp[ncols] = nnz;
    } catch (const std::exception&) {
        return MS_ERR_OOM;
    }
    return MS_OK;
}

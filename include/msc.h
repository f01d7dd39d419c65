/*
 * msc.h -- C ABI of the MI355X Morse-Smale hot path (libmsc.so).
 *
 * Computes, for a scalar field sampled at the vertices of a 3D grid, the
 * discrete gradient, its critical cells, and the 1-skeleton of the
 * Morse-Smale complex, following Subhash, Pandey and Natarajan, "A GPU
 * Parallel Algorithm for Computing Morse-Smale Complexes":
 *   - gradient pairs, critical cells, index, V-paths: Section 2.2;
 *   - gradient assignment per vertex lower star (the locally independent
 *     rule of Robins, Wood and Sheppard cited in Section 1.1), first step of
 *     Section 3;
 *   - critical-cell compaction with block counts, prefix sum and stream
 *     compaction: Section 3.5 ("Gradient pairs and critical points");
 *   - saddle-extremum arcs by pointer jumping: Sections 3.4 and 3.5;
 *   - 1-saddle/2-saddle reachability by frontier BFS: Sections 3.2 and 3.5;
 *   - junction nodes, DAG minor, path counting by iterated sparse products:
 *     Section 3.3 and Section 3.5 ("Gradient path counting").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Field layout.  `f` holds nx*ny*nz float32 values, x fastest: vertex
 *   (x, y, z) has id v = x + nx*(y + ny*z).  Values must be finite.
 * Vertex order.  u precedes v iff (f(u), id(u)) < (f(v), id(v)); -0.0 and
 *   +0.0 compare equal (simulation of simplicity by vertex id).
 * Cells.  A cell at refined coordinates (X, Y, Z), 0 <= X <= 2nx-2 etc., has
 *   id 8*v(X>>1, Y>>1, Z>>1) + (X&1) + 2(Y&1) + 4(Z&1); its dimension
 *   (= index when critical) is the number of odd coordinates.
 * Gradient word.  One uint32 per vertex v; nibble k = a + 2b + 4c describes
 *   the cell at refined (2x+a, 2y+b, 2z+c):
 *     1..6  paired with the cell at refined offset +X, -X, +Y, -Y, +Z, -Z;
 *     7     the cell does not exist (outside the grid);
 *     8+d   critical, and its highest vertex is v + (d&1, d>>1&1, d>>2&1).
 * Critical list.  Sorted by (index, cell id).  The rank of a critical cell is
 *   its position among the critical cells of its index; ranks are the row and
 *   column numbers of the arc matrices.
 * Arc matrices.  CSR, rows ascending, columns ascending within a row, values
 *   are numbers of gradient paths as exact unsigned 64-bit integers that
 *   saturate at 2^64-1.  M10: 1-saddle x minimum.  M21: 2-saddle x 1-saddle.
 *   M32: maximum x 2-saddle.  Each is also given transposed.  Paths from a
 *   2-saddle that leave the grid through its boundary are dropped (Section
 *   3.5: paths that do not terminate at a critical cell are discarded).
 * Memory.  Every pointer argument is a device pointer unless documented as
 *   host.  Inputs are read on the context's stream and only need to stay
 *   valid until that stream passes the call.  Outputs documented as
 *   context-owned stay valid until the next call on the same context.
 * Streams and synchronisation.  All device work is ordered on the context's
 *   stream.  Calls that size host-visible outputs (ms_critical, ms_connect,
 *   ms_complex) synchronise that stream before they return.
 * Errors.  Every entry point returns an ms_status; no C++ exception or abort
 *   crosses the ABI.  ms_last_error gives a text for the last failing call.
 *   A context is not thread-safe; use one context per host thread.
 */
#ifndef MSC_H
#define MSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MS_OK = 0,
    MS_ERR_INVALID_ARG = 1, /* null pointer, dims < 1 */
    MS_ERR_NONFINITE = 2,   /* NaN or +-Inf in the field */
    MS_ERR_TOO_LARGE = 3,   /* nx*ny*nz > 2^29 (cell ids are 32-bit) */
    MS_ERR_CAPACITY = 4,    /* caller buffer too small; required sizes reported */
    MS_ERR_OOM = 5,         /* device allocation failed */
    MS_ERR_HIP = 6,         /* a HIP runtime call failed */
    MS_ERR_INTERNAL = 7     /* an internal consistency check failed */
} ms_status;

/* Vertex counts along x, y, z; each >= 1. */
typedef struct {
    int64_t nx, ny, nz;
} ms_dims;

typedef struct ms_ctx ms_ctx;

/* Device allocator of a context's workspace, e.g. a framework's caching
 * allocator.  `alloc` returns `bytes` of device memory usable by work queued
 * on `stream` (a hipStream_t), or NULL when it cannot (the call in progress
 * then fails with MS_ERR_OOM; the context stays usable and keeps what it
 * holds).  `free` gives back a block with the size it was allocated with;
 * the library drains the stream the block was used on before it frees it,
 * so the block is idle.  Both receive the `user` pointer given to
 * ms_ctx_create.  Either may be called from any host thread that calls into
 * the context, and, during ms_complex and ms_complex_batch, also from the
 * call's helper thread (which queues the saddle-extremum arcs on a second
 * stream of the context, passed as `stream`) while the calling thread is
 * inside the library: the callbacks must be safe to call from two threads. */
typedef void* (*ms_alloc_fn)(void* user, size_t bytes, void* stream);
typedef void (*ms_free_fn)(void* user, void* ptr, size_t bytes, void* stream);

/* Creates a context bound to `stream` (a hipStream_t; NULL = the default
 * stream) on the current device.  The context owns its workspace, which grows
 * to the largest problem seen and is reused by later calls.  Workspace memory
 * comes from `alloc_fn` / `free_fn` (with `user`), or from hipMalloc /
 * hipFree when both are NULL; giving only one of them is
 * MS_ERR_INVALID_ARG.  Small host staging buffers are pinned host memory. */
ms_status ms_ctx_create(ms_ctx** out, void* stream, ms_alloc_fn alloc_fn, ms_free_fn free_fn, void* user);
void ms_ctx_destroy(ms_ctx* ctx);
/* Rebinds the context to another stream (hipStream_t) of the same device. */
ms_status ms_ctx_set_stream(ms_ctx* ctx, void* stream);
/* Text describing the last non-OK status returned on this context. */
const char* ms_last_error(const ms_ctx* ctx);
/* Frees the context's workspace -- its device buffers and the pinned host
 * memory of the out-of-core calls (slab staging, records and labels; all are
 * reallocated on demand by the next call); invalidates every context-owned
 * output.  Synchronises the stream. */
ms_status ms_ctx_release(ms_ctx* ctx);

/* Context options (ms_ctx_set_option). */
enum {
    MS_OPT_PATH_SCHEDULE = 1, /* how A* = sum_k A B^k is evaluated (Section 3.3) */
    /* Tuning of the ready schedule's column merges; results never depend on
     * them.  A column with at most MERGE_LIGHT inputs (0..256, default 32)
     * and at most 8 input lists is merged by one thread; other columns are
     * merged by a workgroup in chunks of MERGE_CHUNK entries (1..4096,
     * default 4096). */
    MS_OPT_MERGE_LIGHT = 2,
    MS_OPT_MERGE_CHUNK = 3,
    /* Gradient workgroup tile in vertices: 0 = 16x8x4 (default), 1 = 32x4x4,
     * 2 = 8x8x8, 3 = 16x16x2, 4 = 16x8x8, 5 = 16x16x8, 6 = 32x16x8.  Results
     * never depend on it. */
    MS_OPT_GRADIENT_TILE = 4,
    /* ms_complex_batch: 1 (default) captures the fixed-shape front of a
     * batch (gradient, critical counts, their scan and totals) in a HIP
     * graph per set of dims and replays it while the dims and the context's
     * buffers stay the same; 0 launches it eagerly.  The graph is also
     * bypassed while timing is on.  Results never depend on it. */
    MS_OPT_BATCH_GRAPH = 5,
    /* Sparse transposes (the column-major copies of the arc and path
     * matrices): at most this many value bits (1..24, default 24) travel
     * packed with the row ids through the radix passes, in the bits the row
     * ids leave free.  A matrix whose values all fit is packed whole; the
     * path-count matrix, whose counts can be large, is packed when at least
     * 4 bits are free, with larger counts looked up again after the
     * transpose; other values move as a separate 64-bit payload, as all do
     * with 0.  Results never depend on it. */
    MS_OPT_TRANSPOSE_PACK = 6
};
enum {
    /* Default.  A* is the solution of A* = A + A* B; its columns are formed by
     * sparse products restricted to the junctions whose minor predecessors
     * are complete (a ready frontier in topological order), so every
     * (1-saddle, junction) pair is produced once.  Columns are merged by a
     * thread, a wave or a workgroup depending on their size.  Falls back to
     * MS_PATHS_POWER by itself when a column has more than 256 inputs. */
    MS_PATHS_READY = 0,
    /* The paper's iteration: A* accumulates the frontier A, advanced by
     * A <- A B until the product is empty, then P = D + A* B*. */
    MS_PATHS_POWER = 1,
    /* The ready frontier of MS_PATHS_READY with entry-parallel merges: one
     * thread per input entry of a level ranks it in its column; run heads
     * are then compacted by a scan.  No limit on column inputs. */
    MS_PATHS_ENTRY = 2
};
/* Sets an option; MS_ERR_INVALID_ARG for an unknown option or value. */
ms_status ms_ctx_set_option(ms_ctx* ctx, int option, int64_t value);

/* Discrete gradient (Section 2.2 definitions; per-vertex lower-star pairing
 * as cited in Section 1.1 and used in the first step of Section 3).
 *   d_f    : device, nx*ny*nz float32, layout above.
 *   d_grad : device, nx*ny*nz uint32, caller-owned; receives the gradient
 *            words.
 * Errors: MS_ERR_INVALID_ARG, MS_ERR_TOO_LARGE, MS_ERR_NONFINITE (d_grad is
 * then unspecified).  Synchronises the stream (to report non-finite input). */
ms_status ms_gradient(ms_ctx* ctx, const float* d_f, ms_dims dims, uint32_t* d_grad);

/* Critical-cell list, structure of arrays, all device, caller-owned. */
typedef struct {
    uint32_t* id;      /* cell ids */
    uint8_t* index;    /* index = dimension, 0..3 */
    float* value;      /* f at the cell's highest vertex (bit copy) */
    uint32_t* vmax;    /* id of the cell's highest vertex */
    int64_t capacity;  /* entries available in each array */
} ms_crit;

/* Critical-cell extraction and compaction (Section 3.5, "Gradient pairs and
 * critical points": marking, block counts, prefix sum, stream compaction).
 *   d_f, d_grad : device inputs (d_grad as produced by ms_gradient).
 *   out         : caller-owned arrays; may be NULL to query counts only.
 *   h_count     : host, receives the number of critical cells per index.
 * Output: the critical list sorted by (index, id) in out->[0, sum(h_count)).
 * Errors: MS_ERR_CAPACITY when sum(h_count) > out->capacity (counts are
 * written, outputs untouched; retry with larger arrays). */
ms_status ms_critical(ms_ctx* ctx, const float* d_f, const uint32_t* d_grad, ms_dims dims,
                      const ms_crit* out, int64_t h_count[4]);

/* ms_critical without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and errors as ms_critical; its
 * pass scratch is a fixed 8 MiB device array per GPU, held by the library
 * until the process ends (its address is taken when the first context on the
 * device is created), so the field may hold at most about 2.6e8 vertices:
 * larger fields give MS_ERR_TOO_LARGE before any device work.  Every call on
 * one GPU, from any context or thread, shares that array: calls that overlap
 * in time on one GPU (different streams or threads) race and must be
 * serialised by the caller.  Nothing in the array needs clearing between
 * calls: each pass writes what the next reads. */
ms_status ms_critical_noalloc(ms_ctx* ctx, const float* d_f, const uint32_t* d_grad, ms_dims dims,
                              const ms_crit* out, int64_t h_count[4]);

/* Critical-cell list with 64-bit ids, structure of arrays in HOST memory,
 * caller-owned (the out-of-core entry point below). */
typedef struct {
    uint64_t* id;      /* cell ids 8 * v + nibble, v = x + nx*(y + ny*z) in 64 bits */
    uint8_t* index;    /* index = dimension, 0..3 */
    float* value;      /* f at the cell's highest vertex (bit copy) */
    uint64_t* vmax;    /* id of the cell's highest vertex */
    int64_t capacity;  /* entries available in each array */
} ms_crit64;

/* Out-of-core gradient and critical cells of a field held in HOST memory,
 * of any size up to 2^40 vertices (nx*ny <= 2^29), streamed through the GPU
 * in z-slabs of `slab` rows (clamped so that a slab plus halo is at most
 * 2^29 vertices).  The paper names device memory as its method's limit
 * (Section 5.2) and cites parcels computed separately (Section 1.1); the
 * gradient needs no stitching, as a lower star depends only on its 26
 * neighbours: each slab is computed with one halo row below and two above,
 * and its rows are exact.  The results equal ms_gradient / ms_critical on
 * the whole field (ids widened to 64 bits).  Host-to-device copies of the
 * next slab overlap the current slab's kernels; the slabs' records are held
 * in pinned host memory until the end, so a call with too small an `out`
 * costs a whole pass (size `out` generously: untouched pages cost nothing).
 * The pinned memory (two slabs plus halo of staging, and about 20 bytes per
 * critical cell of records) is kept by the context for later calls.
 *   h_f     : host, nx*ny*nz float32 (layout as everywhere).
 *   h_grad  : host, nx*ny*nz uint32 gradient words, or NULL (not written).
 *   out     : host arrays sorted by (index, id), or NULL (counts only).
 *   h_count : host, critical cells per index.
 * Errors: MS_ERR_INVALID_ARG, MS_ERR_TOO_LARGE, MS_ERR_NONFINITE,
 * MS_ERR_CAPACITY (counts written, outputs untouched), MS_ERR_OOM.
 * Synchronises the context's stream. */
ms_status ms_gradient_critical_chunked(ms_ctx* ctx, const float* h_f, ms_dims dims, int64_t slab,
                                       uint32_t* h_grad, const ms_crit64* out, int64_t h_count[4]);

/* Out-of-core ascending 3-manifolds of the minima and descending
 * 3-manifolds of the maxima (Section 3.4: the destination extremum of every
 * vertex and every cube; Section 1.1: parcels computed apart and stitched),
 * for a field held in HOST memory, with the same slabs and limits as
 * ms_gradient_critical_chunked.  Each slab follows the (0,1) and (2,3)
 * gradient paths of its exact rows by pointer jumping on the device; a path
 * that crosses into another slab ends there with the cell it continues
 * from, and the host then resolves those cells across the slabs' first and
 * last rows (the paths never revisit a cell, so every chain ends).  The
 * labels equal the min_label / max_label of ms_complex on the whole field,
 * widened to 64 bits:
 *   h_min_label : host, nx*ny*nz uint64: rank of the minimum the (0,1)
 *                 path from vertex v reaches, or NULL (not written);
 *   h_max_label : host, nx*ny*nz uint64: rank of the maximum reached from
 *                 the cube with lowest corner v, MS_LABEL_EXIT64 when there is
 *                 no such cube or its path leaves the grid, or NULL;
 *   h_count     : host, critical cells per index (the ranks' ranges);
 *                 with both label pointers NULL only these are computed.
 * Errors: as ms_gradient_critical_chunked (no MS_ERR_CAPACITY);
 * MS_ERR_INTERNAL if a path between slabs does not end.  Synchronises the
 * context's stream; uses the host's threads for the stitching.  The
 * labels come back through pinned memory (16 bytes per vertex of two
 * slabs) that the context keeps for later calls. */
#define MS_LABEL_EXIT64 0xFFFFFFFFFFFFFFFFull
ms_status ms_manifolds_chunked(ms_ctx* ctx, const float* h_f, ms_dims dims, int64_t slab,
                               uint64_t* h_min_label, uint64_t* h_max_label, int64_t h_count[4]);

/* A CSR matrix in host memory, caller-owned (out-of-core results). */
typedef struct {
    int64_t* rowptr;   /* nrows + 1 */
    uint64_t* col;     /* capacity entries */
    uint64_t* val;     /* capacity entries */
    int64_t capacity;  /* entries available in col and val */
    int64_t nnz;       /* out: entries of the matrix */
} ms_csr64_host;

/* Saddle-extremum arcs of an out-of-core field (Section 3.5, "Saddle-Extrema
 * arcs"; Section 3.4: the arcs of a saddle end where the gradient paths from
 * its two faces or cofaces go) from the labels of ms_manifolds_chunked and
 * the saddles of ms_gradient_critical_chunked, on the host (the labels of
 * such a field live in host memory):
 *   M10  : row r = the 1-saddle s1_id[r]: the minima of its two vertices;
 *   M32^T: row r = the 2-saddle s2_id[r]: the maxima of its two cubes
 *          (a cube that does not exist or whose path leaves the grid gives
 *          no entry);
 * columns ascending, value 2 when both reach the same extremum, else 1 --
 * the m10 and m32t of ms_complex on the whole field, with 64-bit columns.
 *   dims        : the field's dims (limits as ms_gradient_critical_chunked).
 *   h_min_label, h_max_label : host, nx*ny*nz labels (ms_manifolds_chunked).
 *   s1_id, s2_id: host, the 1-saddle and 2-saddle cell ids (64-bit, as in
 *                 ms_crit64), S1 and S2 of them, in rank order.
 *   m10, m32t   : caller-owned outputs, or NULL (not computed, and its label
 *                 array may be NULL); rowptr holds S + 1 entries, and a
 *                 capacity of 2 S always suffices.
 * No device work and no context: uses the host's threads.  Errors:
 * MS_ERR_INVALID_ARG (null pointer where an output is asked for, an id that
 * is not a cell of the right dimension in the grid, a minimum label that is
 * the exit label), MS_ERR_TOO_LARGE, MS_ERR_CAPACITY (nnz written, entries
 * not), MS_ERR_OOM. */
ms_status ms_extremum_arcs_host(ms_dims dims, const uint64_t* h_min_label, const uint64_t* h_max_label,
                                const uint64_t* s1_id, int64_t S1, const uint64_t* s2_id, int64_t S2,
                                ms_csr64_host* m10, ms_csr64_host* m32t);

/* Transpose of a host CSR (e.g. M10 -> M10^T = minimum x 1-saddle, M32^T ->
 * M32 = maximum x 2-saddle, as ms_complex gives them), by a counting sort
 * on the host: out row c lists the input rows holding column c, ascending,
 * with their values.
 *   in    : nrows + 1 rowptr entries (rowptr[0] = 0, non-decreasing),
 *           columns < ncols.
 *   out   : caller-owned; rowptr holds ncols + 1 entries; capacity >=
 *           in's nnz (out->nnz is written first).
 * Errors: MS_ERR_INVALID_ARG (null pointers, a malformed input),
 * MS_ERR_CAPACITY, MS_ERR_OOM. */
ms_status ms_csr64_transpose_host(const ms_csr64_host* in, int64_t nrows, int64_t ncols, ms_csr64_host* out);

/* A CSR matrix in device memory, context-owned. */
typedef struct {
    int64_t nrows, ncols, nnz;
    int64_t* rowptr;   /* nrows + 1 */
    uint32_t* col;     /* nnz */
    uint64_t* val;     /* nnz */
} ms_csr;

/* Counters of the connection phase (Section 5 reports the same kinds of
 * statistics: junction counts, matrix sizes, product iterations). */
typedef struct {
    /* pointer-jumping rounds; a round updates the pointers in place, so how
     * far it gets depends on which updates of the same round its reads
     * already see: the count (never the result) can differ between
     * identical calls */
    int64_t pj_rounds_vertex, pj_rounds_cube;
    int64_t bfs_levels, reachable;            /* BFS levels, reachable 1-2 pairs */
    int64_t junctions;
    int64_t nnz_a, nnz_b, nnz_bstar, nnz_d;   /* DAG-minor matrices (Section 3.3) */
    int64_t spgemm_iters, nnz_astar, products;
    int64_t nnz_p;                            /* entries of P = M21^T */
} ms_stats;

typedef struct {
    ms_csr m10, m10t;  /* 1-saddle x minimum, and minimum x 1-saddle */
    ms_csr m21, m21t;  /* 2-saddle x 1-saddle, and 1-saddle x 2-saddle */
    ms_csr m32, m32t;  /* maximum x 2-saddle, and 2-saddle x maximum */
    int64_t n_saturated; /* entries of M21 equal to 2^64-1 (not an error) */
    ms_stats stats;
    /* Ascending 3-manifolds of the minima and descending 3-manifolds of the
     * maxima (Section 3.4: the traversal that gives the saddle-extremum arcs
     * also gives, for every cell, the extremum its gradient path ends at;
     * Section 3.5 keeps it in an extra array).  Device, context-owned, one
     * uint32 per vertex, same layout as the field:
     *   min_label[v] : rank of the minimum that the (0,1) gradient path from
     *                  vertex v reaches (a minimum labels itself);
     *   max_label[w] : rank of the maximum that the (2,3) gradient path from
     *                  the cube with lowest corner w reaches, or 0xFFFFFFFF
     *                  when there is no such cube (w on a high face) or the
     *                  path leaves the grid through a boundary quad. */
    uint32_t* min_label;
    uint32_t* max_label;
} ms_arcs;

/* 1-skeleton (Sections 3.1-3.5): saddle-extremum arcs by pointer jumping;
 * saddle-saddle arcs by frontier BFS, junction nodes, DAG minor and iterated
 * sparse integer products.  The call starts one host thread of its own,
 * which queues the saddle-extremum arcs (and, with MS_PATHS_ENTRY, two
 * transposes the last product needs) on a second stream of the context,
 * created on first use with the default priority; the context's stream
 * waits for that work before the results are used, and the thread has ended
 * when the call returns.  Calls on one context must not overlap in time.
 *   d_grad       : device gradient words.
 *   d_crit_id    : device, the critical cell ids sorted by (index, id), as
 *                  written by ms_critical (sum(h_count) entries).
 *   h_count      : host, critical counts per index.
 *   out          : host struct; receives context-owned device matrices valid
 *                  until the next call on this context.
 * Errors: MS_ERR_INVALID_ARG, MS_ERR_OOM, MS_ERR_INTERNAL (e.g. a crit list
 * that does not match the gradient). */
ms_status ms_connect(ms_ctx* ctx, const uint32_t* d_grad, ms_dims dims, const uint32_t* d_crit_id,
                     const int64_t h_count[4], ms_arcs* out);

typedef struct {
    uint32_t* grad;    /* device, nx*ny*nz gradient words, context-owned */
    ms_crit crit;      /* context-owned critical list */
    int64_t count[4];
    ms_arcs arcs;      /* context-owned arc matrices */
} ms_result;

/* Per-stage device time of ms_complex calls, accumulated while timing is
 * enabled (the paper breaks its runtime down the same way, Section 5,
 * Figure 10).  Times come from HIP events recorded on the context's stream:
 * gradient_ms brackets exactly the gradient kernel; the other stages bracket
 * their kernels and the host round trips between them. */
typedef struct {
    double gradient_ms;  /* gradient kernel */
    double critical_ms;  /* critical counts, scan, compaction */
    double extrema_ms;   /* pointer set-up and critical-cell labels (the rest of the
                            saddle-extremum arcs overlaps later stages: side_ms) */
    double bfs_ms;       /* saddle-saddle reachability */
    double minor_ms;     /* junction numbering, DAG minor, minor matrices */
    double paths_ms;     /* iterated products, P, M21 and transpose */
    double total_ms;     /* whole ms_complex */
    int64_t calls;
    int64_t allocations;     /* device allocations the context made while timing was on
                                (workspace growth; zero in the steady state) */
    int64_t workspace_bytes; /* device memory the context holds now */
    /* Launches of the path-count ranking kernel of MS_PATHS_ENTRY (the
     * dominant kernel): summed event-timed duration, launch count, input
     * entries ranked and run heads written. */
    double rank_ms;
    int64_t rank_launches, rank_entries, rank_heads;
    /* graphs of the batch front captured / replayed by this context since it
     * was created (not reset by enabling timing) */
    int64_t graph_captures, graph_replays;
    /* work a helper thread of the call queues on a second stream of the
     * context, beside the stages above: pointer jumping, M10 / M32, their
     * transposes and the manifold labels (queued once the search is), and
     * with MS_PATHS_ENTRY the transposes of B* and D (queued once the
     * junctions are numbered, needed by the last product); the sum of their
     * spans */
    double side_ms;
} ms_timing;

/* Enables (1) or disables (0) timing; enabling resets the accumulators. */
ms_status ms_ctx_set_timing(ms_ctx* ctx, int enable);
/* Copies the accumulated timing into *out (host). */
ms_status ms_ctx_get_timing(ms_ctx* ctx, ms_timing* out);

/* The whole hot path: ms_gradient, ms_critical and ms_connect on
 * context-owned buffers.  d_f is a device field; all results stay on the
 * device, owned by the context until its next call. */
ms_status ms_complex(ms_ctx* ctx, const float* d_f, ms_dims dims, ms_result* out);

/* Batched hot path: nfields fields of any (non-cubic, uneven) dims in one
 * launch per phase.  The fields are processed as one complex over their
 * concatenation -- cells of different fields are never adjacent, so every
 * arc matrix is block diagonal -- and each field's part is then copied out
 * with local ids and ranks: outs[f] is byte-identical to ms_complex on field
 * f alone (stats excepted: they describe the whole batch).  The iteration
 * counts of the data-dependent loops (BFS levels, pointer-jumping rounds,
 * path-counting levels) are the maximum over the fields, not the sum.
 *   nfields : 1..1024.
 *   d_f     : host array of nfields device pointers to float32 fields.
 *   dims    : host array of nfields dims.
 *   outs    : host array of nfields results; every pointer is
 *             context-owned and valid until the next call on the context.
 * Errors: as ms_complex, plus MS_ERR_TOO_LARGE when the fields together have
 * more than 2^29 vertices (split the batch). */
ms_status ms_complex_batch(ms_ctx* ctx, int32_t nfields, const float* const* d_f, const ms_dims* dims,
                           ms_result* outs);

/* ---- Host MS-complex graph (Section 3.5, "Data structure") ---------------
 *
 * The 1-skeleton as a host data structure for queries: a vector of critical
 * points (nodes) and, per node, its arcs in each direction with their
 * multiplicities; every arc is stored at both of its ends.  Node i is the
 * i-th entry of the critical list sorted by (index, cell id), i.e. node =
 * (number of critical cells of lower index) + rank.  A graph is independent
 * of the context once built; it is not thread-safe (one thread at a time). */
typedef struct ms_graph ms_graph;

typedef struct {
    uint32_t cell;   /* critical cell id */
    uint8_t index;   /* 0..3 */
    uint8_t alive;   /* 0 once cancelled by ms_graph_simplify */
    float value;     /* f at the cell's highest vertex */
    uint32_t vmax;   /* id of that vertex */
} ms_node;

enum { MS_DOWN = 0, MS_UP = 1 }; /* arcs to index - 1 / to index + 1 */

/* Builds the graph of a result of ms_complex or ms_complex_batch (one
 * field): copies its critical list and its six arc matrices to host memory
 * (synchronises the context's stream), then fills the arc lists, one worker
 * thread per range of nodes and direction (nthreads >= 1, as the paper
 * parallelises the population across critical points).  `dims` are the
 * field's dims (they place the nodes for ms_graph_simplify's subgrids).
 * Errors: MS_ERR_INVALID_ARG (null arguments, inconsistent sizes),
 * MS_ERR_OOM (host memory), MS_ERR_HIP. */
ms_status ms_graph_build(ms_ctx* ctx, const ms_result* result, ms_dims dims, int nthreads, ms_graph** out);
/* The same from a result whose arrays (critical list and CSR arrays; grad
 * and the labels are not read) are in host memory, e.g. copied back
 * earlier; needs no device.  Errors as ms_graph_build; *out is NULL on
 * failure and the reason is not recorded anywhere else. */
ms_status ms_graph_build_host(const ms_result* result, ms_dims dims, int nthreads, ms_graph** out);
void ms_graph_destroy(ms_graph* g);
/* Number of nodes, cancelled ones included. */
int64_t ms_graph_num_nodes(const ms_graph* g);
const char* ms_graph_last_error(const ms_graph* g);
/* Attributes of node `node` (0 <= node < ms_graph_num_nodes). */
ms_status ms_graph_node(const ms_graph* g, int64_t node, ms_node* out);
/* Node of critical cell `cell`; MS_ERR_INVALID_ARG if it is not critical. */
ms_status ms_graph_find(const ms_graph* g, uint32_t cell, int64_t* node);
/* Live arcs of a live node in direction `dir` (MS_DOWN or MS_UP), sorted by
 * neighbour node: neighbour ids into nbr[] and multiplicities (numbers of
 * gradient paths, saturating at 2^64-1) into mult[], at most `cap` of them
 * (host arrays); *count receives the number of arcs.  MS_ERR_CAPACITY when
 * *count > cap (the first cap are written).  A cancelled node has none. */
ms_status ms_graph_arcs(const ms_graph* g, int64_t node, int dir, int64_t* nbr, uint64_t* mult, int64_t cap,
                        int64_t* count);
/* Live nodes per index and live arcs per index pair (1-0, 2-1, 3-2). */
ms_status ms_graph_counts(const ms_graph* g, int64_t alive[4], int64_t arcs[3]);

/* ---- Persistence-driven simplification (Section 2.1; Section 4) ----------
 *
 * Cancels critical pairs (p, q), index(p) = index(q) + 1, joined by exactly
 * one gradient path (multiplicity 1; pairs joined by several paths would
 * strangle and are never cancelled), whose persistence |f(p) - f(q)| (in
 * double) is below `threshold`.  A cancellation reroutes p's descending
 * arcs to the destinations of q's ascending arcs: every other upper
 * neighbour s of q gains m(s,q) * m(p,r) paths to every other lower
 * neighbour r of p; p, q and their arcs are deleted.
 *   MS_SIMPLIFY_SERIAL : always cancel the valid arc that is least in the
 *     order (persistence, upper node, lower node); deterministic.
 *   MS_SIMPLIFY_SUBGRID: the paper's grid subdivision (Section 4.1-4.2):
 *     the grid is cut into `nthreads` slabs along X, Y, Z and again with the
 *     cuts shifted by half a slab; in each round the ends of arcs crossing a
 *     cut are frozen and every slab cancels its own valid arcs in serial
 *     order on its own thread (the slabs never share a node, so their
 *     cancellations commute); a final serial round follows.  The result can
 *     differ from the serial order's, as the paper notes; every cancellation
 *     in it is valid at its place in ms_graph_cancellations' log.
 * *ncancelled (may be NULL) receives the cancellations made by this call.
 * Can be called again with a larger threshold. */
enum { MS_SIMPLIFY_SERIAL = 0, MS_SIMPLIFY_SUBGRID = 1 };
ms_status ms_graph_simplify(ms_graph* g, double threshold, int schedule, int nthreads, int64_t* ncancelled);

/* The cancellations made so far, in an order in which they are valid one
 * after the other (the hierarchy of the simplification). */
typedef struct {
    int64_t upper, lower;  /* nodes; index(upper) = index(lower) + 1 */
    double persistence;
} ms_cancellation;
int64_t ms_graph_num_cancellations(const ms_graph* g);
ms_status ms_graph_cancellations(const ms_graph* g, int64_t first, int64_t n, ms_cancellation* out);

#ifdef __cplusplus
}
#endif

#endif /* MSC_H */

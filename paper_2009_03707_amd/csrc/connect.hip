// Host orchestration of the 1-skeleton (ms_connect): saddle-extremum arcs by
// pointer jumping, then saddle-saddle arcs by BFS, junctions, DAG minor and
// iterated sparse products (Sections 3.2-3.5).  Every loop whose length
// depends on the data has a bound that turns a malformed input into an
// error instead of an endless loop.
#include "ctx.h"
#include "paths.h"

#include <exception>
#include <thread>
#include <vector>

namespace msc {

hipError_t launch_pj_init(const uint32_t* grad, const Geo& g, uint32_t* Pv, uint32_t* Pc, int* err, hipStream_t s);
hipError_t launch_label(const uint32_t* crit, const int64_t cnt[4], const uint32_t* grad, const Geo& g, uint32_t* Pv,
                        uint32_t* Pc, uint32_t* label, int* err, hipStream_t s);
hipError_t launch_pj_round(uint32_t* P, uint32_t n, int* changed, hipStream_t s);
hipError_t launch_m10(bool fill, const uint32_t* s1, uint64_t S1, const Geo& g, const uint32_t* Pv, uint32_t* cnt,
                      const uint64_t* rowptr, uint32_t* col, uint64_t* val, int* err, hipStream_t s);
hipError_t launch_m32t(bool fill, const uint32_t* s2, uint64_t S2, const Geo& g, const uint32_t* Pc, uint32_t* cnt,
                       const uint64_t* rowptr, uint32_t* col, uint64_t* val, int* err, hipStream_t s);
hipError_t launch_manifold_labels(uint32_t* Pv, uint32_t* Pc, const Geo& g, const uint64_t* before, hipStream_t s);
int bit_width(uint64_t v);
hipError_t launch_expand_rows(const uint64_t* rowptr, uint64_t nrows, const uint32_t* map, uint32_t* rows,
                              hipStream_t s, const uint64_t* val = nullptr, int vb = 0);
hipError_t launch_iota(uint32_t* a, uint64_t n, hipStream_t s);
hipError_t launch_sum_u32(const uint32_t* a, uint64_t n, uint64_t* out, hipStream_t s);
hipError_t launch_max_u64(const uint64_t* a, uint64_t n, uint64_t* out, hipStream_t s);
hipError_t launch_hist(const uint32_t* keys, uint64_t n, uint32_t* h, hipStream_t s);
size_t key_bounds_tmp_elems(uint64_t n, uint64_t nkeys);
hipError_t launch_key_bounds(const uint32_t* keys, uint64_t n, uint64_t nkeys, uint64_t* rowptr, uint64_t* tmp,
                             hipStream_t s);
hipError_t launch_gather_t(const uint32_t* perm, const uint32_t* rows, const uint64_t* val, uint32_t* ocol,
                           uint64_t* oval, uint64_t n, hipStream_t s);
hipError_t launch_make_keys(const uint32_t* row, const uint32_t* col, uint64_t n, int cb, uint64_t* keys,
                            uint32_t* idx, hipStream_t s);
hipError_t launch_heads(const uint64_t* keys, uint64_t n, uint32_t* h, hipStream_t s);
hipError_t launch_merge_runs(const uint64_t* keys, const uint32_t* perm, const uint64_t* val, uint64_t n,
                             const uint64_t* pos, int cb, uint32_t* orow, uint32_t* ocol, uint64_t* oval,
                             hipStream_t s);
hipError_t launch_esc_count(const uint32_t* xcol, uint64_t nx, const uint64_t* yrowptr, uint32_t* pc, hipStream_t s);
hipError_t launch_esc_expand(const uint32_t* xrow, const uint32_t* xcol, const uint64_t* xval, uint64_t nx,
                             const uint64_t* poff, const uint64_t* yrowptr, const uint32_t* ycol, const uint64_t* yval,
                             uint32_t* prow, uint32_t* pcol, uint64_t* pval, hipStream_t s);
hipError_t launch_count_sat(const uint64_t* v, uint64_t n, unsigned long long* out, hipStream_t s);
hipError_t launch_bfs_level(uint32_t* queue, uint64_t qcap, uint64_t* lv, uint64_t L, const uint32_t* grad,
                            const Geo& g, uint32_t* vis, unsigned long long* tail, uint32_t* label, hipStream_t s);
size_t junction_blocks(uint64_t nv);
hipError_t launch_junc_count(const uint32_t* vis, const uint32_t* label, uint64_t nv, uint64_t* bcount,
                             hipStream_t s);
hipError_t launch_junc_emit(const uint32_t* vis, uint32_t* label, uint64_t nv, const uint64_t* boff, uint32_t* jlist,
                            hipStream_t s);
hipError_t launch_minor_trace(const uint32_t* s1, uint64_t S1, const uint32_t* jlist, uint64_t J, const uint32_t* grad,
                              const Geo& g, const uint32_t* label, uint64_t max_steps, uint64_t S2, uint8_t* out_t,
                              uint32_t* out_id, int* err, hipStream_t s);
hipError_t launch_minor_rows(bool fill, const uint8_t* out_t, const uint32_t* out_id, uint64_t S1, uint64_t NS,
                             uint32_t* cj, uint32_t* cs, const uint64_t* rpA, uint32_t* colA, uint64_t* valA,
                             const uint64_t* rpD, uint32_t* colD, uint64_t* valD, const uint64_t* rpB, uint32_t* colB,
                             uint64_t* valB, const uint64_t* rpBs, uint32_t* colBs, uint64_t* valBs, hipStream_t s);

namespace {

struct Coo {
    uint32_t* row = nullptr;
    uint32_t* col = nullptr;
    uint64_t* val = nullptr;
    uint64_t n = 0;
};

std::string nm(const char* a, const char* b) { return std::string(a) + "." + b; }

// named buffer set for a COO of capacity n
Coo coo_buf(ms_ctx* c, const char* name, uint64_t n) {
    Coo o;
    o.row = buf<uint32_t>(c, nm(name, "row").c_str(), n);
    o.col = buf<uint32_t>(c, nm(name, "col").c_str(), n);
    o.val = buf<uint64_t>(c, nm(name, "val").c_str(), n);
    o.n = n;
    return o;
}

ms_csr csr_buf(ms_ctx* c, const char* name, uint64_t nrows, uint64_t ncols, uint64_t nnz) {
    ms_csr m;
    m.nrows = (int64_t)nrows;
    m.ncols = (int64_t)ncols;
    m.nnz = (int64_t)nnz;
    m.rowptr = (int64_t*)buf<uint64_t>(c, nm(name, "rowptr").c_str(), nrows + 1);
    m.col = buf<uint32_t>(c, nm(name, "col").c_str(), nnz);
    m.val = buf<uint64_t>(c, nm(name, "val").c_str(), nnz);
    return m;
}

uint64_t read_u64(ms_ctx* c, const uint64_t* d) { return readback(c, d, 1)[0]; }

void check_err_flag(ms_ctx* c, int* d_err, const char* stage) {
    uint64_t* slot = buf<uint64_t>(c, "err_slot", 1);
    check(c, hipMemsetAsync(slot, 0, sizeof(uint64_t), cur_stream(c)), "memset");
    check(c, hipMemcpyAsync(slot, d_err, sizeof(int), hipMemcpyDeviceToDevice, cur_stream(c)), "copy");
    uint64_t v = read_u64(c, slot);
    if (v) fail(c, MS_ERR_INTERNAL, std::string("consistency check failed in ") + stage + " (flag " + std::to_string(v) + ")");
}

// Row counts (u32) -> rowptr (exclusive scan, total in rowptr[n]); returns nnz.
uint64_t counts_to_rowptr(ms_ctx* c, const uint32_t* cnt, uint64_t n, uint64_t* rowptr) {
    uint64_t* tmp = buf<uint64_t>(c, "scan_tmp", scan_tmp_elems(n) + 1);
    check(c, scan_excl_u32_to_u64(cnt, rowptr, n, tmp, rowptr + n, cur_stream(c)), "scan");
    return read_u64(c, rowptr + n);
}

// Transpose of a CSR: a stable radix sort of the column ids (read in
// place), carrying each entry's row (row_map[row] when a map is given: the
// input's rows renumbered while they are expanded) and value, and the row
// pointer of the result from the boundaries between equal keys.  Rows of
// the output come out with ascending columns because the input entries are
// in row-major order.  Values ride in the bits the row ids leave free when
// every value fits there (a bound the caller knows, vmax_bound, or else the
// largest value, read back first); when the input's rows are sorted by
// column (rows_sorted), larger values are packed as escapes and looked up
// again after the sort instead; otherwise values move as a separate 64-bit
// payload.  row_inv: the inverse of row_map (needed for escapes).
constexpr uint64_t NO_BOUND = ~0ull;
// levels whose columns average fewer entries than this list every entry's column for the rank kernel
constexpr uint64_t RANK_COLOF_AVG = 6;
void transpose(ms_ctx* c, const ms_csr& in, const char* name, ms_csr& out, const uint32_t* row_map = nullptr,
               uint64_t vmax_bound = NO_BOUND, bool rows_sorted = false, const uint32_t* row_inv = nullptr) {
    uint64_t nnz = (uint64_t)in.nnz;
    out = csr_buf(c, name, (uint64_t)in.ncols, (uint64_t)in.nrows, nnz);
    if (nnz == 0) {
        check(c, hipMemsetAsync(out.rowptr, 0, sizeof(int64_t) * ((uint64_t)in.ncols + 1), cur_stream(c)), "memset");
        return;
    }
    uint32_t* rows = buf<uint32_t>(c, "tr.rows", nnz);
    uint32_t* ka = buf<uint32_t>(c, "tr.ka", nnz);
    uint32_t* kb = buf<uint32_t>(c, "tr.kb", nnz);
    uint32_t* va = buf<uint32_t>(c, "tr.va", nnz);
    uint32_t* vb = buf<uint32_t>(c, "tr.vb", nnz);
    uint64_t* tmp = buf<uint64_t>(c, "tr.tmp", radix_tmp_elems(nnz));
    const int kbits = bit_width((uint64_t)in.ncols - 1);
    const int free_bits = 32 - bit_width((uint64_t)in.nrows - 1);
    const int vbits = free_bits < c->transpose_pack ? free_bits : c->transpose_pack;
    bool packed = false, escapes = false;
    if (vbits >= 1) {
        if (vmax_bound != NO_BOUND) {
            packed = vmax_bound < (1ull << vbits);
        } else if (rows_sorted && vbits >= 4 && (!row_map || row_inv)) {
            packed = escapes = true;
        } else {
            uint64_t* d_max = buf<uint64_t>(c, "tr.max", 1);
            check(c, launch_max_u64((const uint64_t*)in.val, nnz, d_max, cur_stream(c)), "max");
            packed = read_u64(c, d_max) < (1ull << vbits);
        }
    }
    const uint32_t* keys = nullptr;
    if (packed) {
        check(c, launch_expand_rows((const uint64_t*)in.rowptr, (uint64_t)in.nrows, row_map, rows, cur_stream(c),
                                    (const uint64_t*)in.val, vbits),
              "expand rows");
        Unpack up{vbits, out.col, (uint64_t*)out.val};
        if (escapes) {
            up.esc = buf<uint32_t>(c, "tr.esc", nnz);
            up.nesc = (unsigned long long*)buf<uint64_t>(c, "tr.nesc", 1);
            check(c, launch_set_u64((uint64_t*)up.nesc, 0, cur_stream(c)), "escape count");
        }
        check(c, radix_transpose_packed_u32(in.col, rows, ka, va, kb, vb, nnz, kbits, tmp, up, &keys, cur_stream(c)),
              "sort");
        if (escapes)
            check(c, launch_escape_fix(up.esc, up.nesc, keys, out.col, (const uint64_t*)in.rowptr, in.col,
                                       (const uint64_t*)in.val, row_map ? row_inv : nullptr, (uint64_t*)out.val,
                                       cur_stream(c)),
                  "escape fix");
    } else {
        uint64_t* wa = buf<uint64_t>(c, "tr.wa", nnz);
        uint64_t* wb = buf<uint64_t>(c, "tr.wb", nnz);
        check(c, launch_expand_rows((const uint64_t*)in.rowptr, (uint64_t)in.nrows, row_map, rows, cur_stream(c)),
              "expand rows");
        check(c, radix_transpose_u32(in.col, rows, (const uint64_t*)in.val, ka, va, kb, vb, wa, wb, nnz, kbits, tmp,
                                     out.col, (uint64_t*)out.val, &keys, cur_stream(c)),
              "sort");
    }
    uint64_t* gtmp = buf<uint64_t>(c, "tr.gaps", key_bounds_tmp_elems(nnz, (uint64_t)in.ncols));
    check(c, launch_key_bounds(keys, nnz, (uint64_t)in.ncols, (uint64_t*)out.rowptr, gtmp, cur_stream(c)), "bounds");
}

// Sort a COO by (row, col) and merge repeats; result in buffer set `name`.
Coo sort_merge(ms_ctx* c, const Coo& in, uint64_t nrows, uint64_t ncols, const char* name) {
    Coo out;
    if (in.n == 0) {
        out = coo_buf(c, name, 1);
        out.n = 0;
        return out;
    }
    uint64_t n = in.n;
    if (n >= (1ull << 32)) fail(c, MS_ERR_TOO_LARGE, "more than 2^32 sparse entries in one product");
    int cb = bit_width(ncols - 1), rb = bit_width(nrows - 1);
    uint64_t* ka = buf<uint64_t>(c, "sm.ka", n);
    uint64_t* kb = buf<uint64_t>(c, "sm.kb", n);
    uint32_t* va = buf<uint32_t>(c, "sm.va", n);
    uint32_t* vb = buf<uint32_t>(c, "sm.vb", n);
    uint64_t* tmp = buf<uint64_t>(c, "sm.tmp", radix_tmp_elems(n));
    check(c, launch_make_keys(in.row, in.col, n, cb, ka, va, cur_stream(c)), "keys");
    bool in_b = false;
    check(c, radix_sort_u64(ka, va, kb, vb, n, cb + rb, tmp, &in_b, cur_stream(c)), "sort");
    const uint64_t* keys = in_b ? kb : ka;
    const uint32_t* perm = in_b ? vb : va;
    uint32_t* heads = buf<uint32_t>(c, "sm.heads", n);
    uint64_t* pos = buf<uint64_t>(c, "sm.pos", n + 1);
    check(c, launch_heads(keys, n, heads, cur_stream(c)), "heads");
    uint64_t m = counts_to_rowptr(c, heads, n, pos);
    out = coo_buf(c, name, m);
    out.n = m;
    check(c, launch_merge_runs(keys, perm, in.val, n, pos, cb, out.row, out.col, out.val, cur_stream(c)), "merge");
    return out;
}

// Products X*Y (X as COO, Y as CSR) written at offset `at` of the product
// buffer set "prod" (capacity for `reserve_extra` more entries is kept);
// returns the number of products written.
uint64_t esc_expand(ms_ctx* c, const Coo& x, const ms_csr& y, uint64_t at, Coo& prod, uint64_t reserve_extra) {
    uint64_t t = 0;
    if (x.n > 0) {
        uint32_t* pc = buf<uint32_t>(c, "esc.pc", x.n);
        uint64_t* poff = buf<uint64_t>(c, "esc.poff", x.n + 1);
        check(c, launch_esc_count(x.col, x.n, (const uint64_t*)y.rowptr, pc, cur_stream(c)), "esc count");
        t = counts_to_rowptr(c, pc, x.n, poff);
        prod.row = buf_keep<uint32_t>(c, "prod.row", at + t + reserve_extra, at);
        prod.col = buf_keep<uint32_t>(c, "prod.col", at + t + reserve_extra, at);
        prod.val = buf_keep<uint64_t>(c, "prod.val", at + t + reserve_extra, at);
        if (t)
            check(c, launch_esc_expand(x.row, x.col, x.val, x.n, poff, (const uint64_t*)y.rowptr, y.col, y.val,
                                       prod.row + at, prod.col + at, prod.val + at, cur_stream(c)),
                  "esc expand");
    } else {
        prod.row = buf_keep<uint32_t>(c, "prod.row", at + reserve_extra, at);
        prod.col = buf_keep<uint32_t>(c, "prod.col", at + reserve_extra, at);
        prod.val = buf_keep<uint64_t>(c, "prod.val", at + reserve_extra, at);
    }
    prod.n = at + t;
    return t;
}

void coo_to_csr(ms_ctx* c, const Coo& in, uint64_t nrows, uint64_t ncols, const char* name, ms_csr& out) {
    out = csr_buf(c, name, nrows, ncols, in.n);
    uint32_t* h = buf<uint32_t>(c, "cc.hist", nrows + 1);
    check(c, hipMemsetAsync(h, 0, sizeof(uint32_t) * (nrows + 1), cur_stream(c)), "memset");
    check(c, launch_hist(in.row, in.n, h, cur_stream(c)), "hist");
    uint64_t* stmp = buf<uint64_t>(c, "scan_tmp", scan_tmp_elems(nrows) + 1);
    check(c, scan_excl_u32_to_u64(h, (uint64_t*)out.rowptr, nrows, stmp, (uint64_t*)out.rowptr + nrows, cur_stream(c)),
          "scan");
    if (in.n) {
        check(c, hipMemcpyAsync(out.col, in.col, 4 * in.n, hipMemcpyDeviceToDevice, cur_stream(c)), "copy");
        check(c, hipMemcpyAsync(out.val, in.val, 8 * in.n, hipMemcpyDeviceToDevice, cur_stream(c)), "copy");
    }
}

Coo csr_as_coo(ms_ctx* c, const ms_csr& m, const char* rows_name) {
    Coo o;
    o.n = (uint64_t)m.nnz;
    o.row = buf<uint32_t>(c, rows_name, o.n);
    o.col = m.col;
    o.val = m.val;
    check(c, launch_expand_rows((const uint64_t*)m.rowptr, (uint64_t)m.nrows, nullptr, o.row, cur_stream(c)),
          "expand rows");
    return o;
}

void ensure_side(ms_ctx* c) {
    if (!c->side_stream) check(c, hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking), "stream create");
    if (!c->ev_fork) check(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "event create");
    if (!c->ev_join) check(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "event create");
    if (!c->h_side) {
        check(c, hipHostMalloc((void**)&c->h_side, HOST_SCRATCH_WORDS * sizeof(uint64_t),
                               hipHostMallocMapped | hipHostMallocCoherent),
              "host allocation");
        check(c, hipHostGetDevicePointer((void**)&c->h_side_dev, c->h_side, 0), "host pointer");
    }
}

// Work of one call queued from a helper thread on the context's side stream
// after everything the calling thread queued so far (event ev_fork), with
// its own readback scratch, buffer names and error text.  finish() joins
// the thread, rethrows its failure and orders the calling thread's stream
// after the helper's work (event ev_join); it does nothing when no work was
// started, and a task may be started again once finished.  abandon() (and
// the destructor) joins on the error paths of the calling thread and drains
// the side stream, so that nothing the helper uses outlives its work.
class SideTask {
  public:
    explicit SideTask(ms_ctx* c) : c_(c) {}
    SideTask(const SideTask&) = delete;
    SideTask& operator=(const SideTask&) = delete;
    template <class F>
    void start(hipStream_t s, F f) {
        ensure_side(c_);
        hipEvent_t t0 = nullptr, t1 = nullptr;  // the work's span, when timing
        if (c_->timing) {
            while (c_->side_ev.size() < 2 * (c_->side_used + 1)) {
                hipEvent_t ev;
                check(c_, hipEventCreate(&ev), "event create");
                c_->side_ev.push_back(ev);
            }
            t0 = c_->side_ev[2 * c_->side_used];
            t1 = c_->side_ev[2 * c_->side_used + 1];
            c_->side_used++;
        }
        check(c_, hipEventRecord(c_->ev_fork, s), "event record");
        st_ = MS_OK;
        err_.clear();
        th_ = std::thread([this, f, t0, t1]() {
            t_ctx = ThreadCtx{c_->side_stream, c_->h_side, c_->h_side_dev, "side.", &err_};
            try {
                check(c_, hipSetDevice(c_->device), "set device");
                check(c_, hipStreamWaitEvent(c_->side_stream, c_->ev_fork, 0), "stream wait");
                if (t0) check(c_, hipEventRecord(t0, c_->side_stream), "event record");
                f();
                if (t1) check(c_, hipEventRecord(t1, c_->side_stream), "event record");
                check(c_, hipEventRecord(c_->ev_join, c_->side_stream), "event record");
            } catch (const Fail& e) {
                st_ = e.st;
            } catch (const std::exception& e) {
                st_ = MS_ERR_INTERNAL;
                err_ = std::string("internal error: ") + e.what();
            } catch (...) {
                st_ = MS_ERR_INTERNAL;
                err_ = "internal error";
            }
            t_ctx = ThreadCtx{};
        });
    }
    void finish(hipStream_t s) {
        if (!th_.joinable()) return;
        th_.join();
        if (st_ != MS_OK) {
            (void)hipStreamSynchronize(c_->side_stream);
            c_->err = err_;
            throw Fail{st_};
        }
        check(c_, hipStreamWaitEvent(s, c_->ev_join, 0), "stream wait");
    }
    void abandon() {
        if (th_.joinable()) {
            th_.join();
            (void)hipStreamSynchronize(c_->side_stream);
        }
    }
    ~SideTask() { abandon(); }

  private:
    ms_ctx* c_;
    std::thread th_;
    ms_status st_ = MS_OK;
    std::string err_;
};


// Path counting as the paper iterates it (Section 3.3): A* accumulates the
// frontier A, which is advanced by A <- A*B until the product is empty; then
// P = D + A* B*.  Products are expand-sort-compress.  Writes M21 and M21t.
void paths_power(ms_ctx* c, const ms_csr& A, const ms_csr& B, const ms_csr& Bs, const ms_csr& D, uint64_t S1,
                 uint64_t S2, uint64_t J, ms_arcs* out) {
    hipStream_t s = cur_stream(c);
    ms_stats& st = out->stats;
    const uint64_t nD = (uint64_t)D.nnz;
    // Each iteration adds the current frontier of 1-saddle -> junction path
    // counts to the accumulation list and advances it by one level of the
    // minor (frontier <- frontier * B) until the product is empty.
    Coo fr = csr_as_coo(c, A, "A.rows");
    uint64_t astar_n = 0;
    int64_t iters = 0;
    uint64_t products = 0;
    Coo acc;
    while (fr.n > 0) {
        acc.row = buf_keep<uint32_t>(c, "acc.row", astar_n + fr.n, astar_n);
        acc.col = buf_keep<uint32_t>(c, "acc.col", astar_n + fr.n, astar_n);
        acc.val = buf_keep<uint64_t>(c, "acc.val", astar_n + fr.n, astar_n);
        check(c, hipMemcpyAsync(acc.row + astar_n, fr.row, 4 * fr.n, hipMemcpyDeviceToDevice, s), "copy");
        check(c, hipMemcpyAsync(acc.col + astar_n, fr.col, 4 * fr.n, hipMemcpyDeviceToDevice, s), "copy");
        check(c, hipMemcpyAsync(acc.val + astar_n, fr.val, 8 * fr.n, hipMemcpyDeviceToDevice, s), "copy");
        astar_n += fr.n;
        Coo prod;
        uint64_t t = esc_expand(c, fr, B, 0, prod, 0);
        products += t;
        iters++;
        if ((uint64_t)iters > J + 2) fail(c, MS_ERR_INTERNAL, "path counting did not terminate (cycle in the minor)");
        if (t == 0) break;
        // alternate between two named result sets so the input stays intact
        fr = sort_merge(c, prod, S1, J, (iters & 1) ? "front1" : "front2");
    }
    st.spgemm_iters = iters;
    Coo astar;
    if (astar_n) {
        acc.n = astar_n;
        astar = sort_merge(c, acc, S1, J, "astar");
    }
    st.nnz_astar = (int64_t)astar.n;
    // P products: A* B* followed by the entries of D
    Coo prod;
    uint64_t t = esc_expand(c, astar, Bs, 0, prod, nD);
    products += t;
    st.products = (int64_t)products;
    if (nD) {
        Coo dcoo = csr_as_coo(c, D, "D.rows");
        check(c, hipMemcpyAsync(prod.row + t, dcoo.row, 4 * nD, hipMemcpyDeviceToDevice, s), "copy");
        check(c, hipMemcpyAsync(prod.col + t, dcoo.col, 4 * nD, hipMemcpyDeviceToDevice, s), "copy");
        check(c, hipMemcpyAsync(prod.val + t, dcoo.val, 8 * nD, hipMemcpyDeviceToDevice, s), "copy");
    }
    prod.n = t + nD;
    Coo P = sort_merge(c, prod, S1, S2, "P");
    coo_to_csr(c, P, S1, S2, "m21t", out->m21t);
    transpose(c, out->m21t, "m21", out->m21, nullptr, NO_BOUND, true);  // P's rows are sorted by column
}

// Path counting by column merges in topological order of the junction DAG
// (see paths.hip).  Returns false when some column has more than 256
// inputs; the caller then uses paths_power (the partial results here are
// discarded).
bool paths_ready(ms_ctx* c, const ms_csr& A, const ms_csr& B, const ms_csr& Bs, const ms_csr& D, uint64_t S1,
                 uint64_t S2, uint64_t J, ms_arcs* out, int* d_err) {
    hipStream_t s = cur_stream(c);
    ms_stats& st = out->stats;
    ms_csr At, Bt, Bst, Dt;
    // minor multiplicities are at most 4: at most four paths leave a source
    transpose(c, A, "At", At, nullptr, 4);     // junction x 1-saddle
    transpose(c, B, "Bt", Bt, nullptr, 4);     // junction x predecessor junction
    transpose(c, Bs, "Bst", Bst, nullptr, 4);  // 2-saddle x junction
    transpose(c, D, "Dt", Dt, nullptr, 4);     // 2-saddle x 1-saddle
    const uint64_t nmax = (J > S2 ? J : S2) + 1;
    uint32_t* indeg = buf<uint32_t>(c, "pr.indeg", J);
    uint32_t* ready[2] = {buf<uint32_t>(c, "pr.ready0", J), buf<uint32_t>(c, "pr.ready1", J)};
    uint64_t* aoff = buf<uint64_t>(c, "pr.aoff", J);
    uint32_t* alen = buf<uint32_t>(c, "pr.alen", J);
    uint64_t* ub = buf<uint64_t>(c, "pr.ub", nmax + 1);
    uint8_t* flag = buf<uint8_t>(c, "pr.flag", nmax);
    uint32_t* qwave = buf<uint32_t>(c, "pr.qwave", nmax);
    uint32_t* qblock = buf<uint32_t>(c, "pr.qblock", nmax);
    // [0] ready, [1] wave-path queue, [2] workgroup-path queue
    unsigned long long* d_n = (unsigned long long*)buf<uint64_t>(c, "pr.counts", 3);
    uint64_t* stmp = buf<uint64_t>(c, "scan_tmp", scan_tmp_elems(nmax) + 1);
    check(c, hipMemsetAsync(d_n, 0, 24, s), "memset");
    check(c, launch_ready_init((const uint64_t*)Bt.rowptr, J, indeg, ready[0], d_n, nullptr, nullptr, s), "ready init");
    uint64_t r = J ? readback(c, (const uint64_t*)d_n, 1)[0] : 0;
    uint64_t used = 0, processed = 0;
    int64_t levels = 0;
    uint32_t* arow = buf_keep<uint32_t>(c, "astar.row", 1, 0);
    uint64_t* aval = buf_keep<uint64_t>(c, "astar.val", 1, 0);
    int cur = 0;
    while (r > 0) {
        MergeLaunch m{ready[cur], r, (const uint64_t*)At.rowptr, At.col, At.val, (const uint64_t*)Bt.rowptr, Bt.col,
                      Bt.val, aoff, alen, arow, aval, c->merge_light, c->merge_chunk, c->wave_blocks};
        check(c, hipMemsetAsync(d_n + 1, 0, 16, s), "memset");
        check(c, launch_merge_classify(m, ub, flag, qwave, qblock, d_n + 1, d_err, aoff, alen, s), "merge classify");
        check(c, scan_excl_u64(ub, ub, r, stmp, ub + r, s), "scan");
        uint64_t t = read_u64(c, ub + r);
        arow = buf_keep<uint32_t>(c, "astar.row", used + t, used);
        aval = buf_keep<uint64_t>(c, "astar.val", used + t, used);
        m.arow = arow;
        m.aval = aval;
        check(c, launch_merge(m, flag, qwave, qblock, d_n + 1, ub, used, arow, aval, nullptr, aoff, alen, s), "merge");
        used += t;
        processed += r;
        levels++;
        check(c, hipMemsetAsync(d_n, 0, 8, s), "memset");
        check(c, launch_release(ready[cur], r, (const uint64_t*)B.rowptr, B.col, indeg, ready[1 - cur], d_n, d_err,
                                nullptr, nullptr, nullptr, nullptr, nullptr, s),
              "release");
        r = readback(c, (const uint64_t*)d_n, 1)[0];
        cur = 1 - cur;
        if ((uint64_t)levels > J + 1) fail(c, MS_ERR_INTERNAL, "path counting did not terminate");
    }
    if (processed != J) fail(c, MS_ERR_INTERNAL, "the junction graph has a cycle");
    // P columns: M21 rows are 2-saddles with their 1-saddle path counts
    MergeLaunch mp{nullptr, S2, (const uint64_t*)Dt.rowptr, Dt.col, Dt.val, (const uint64_t*)Bst.rowptr, Bst.col,
                   Bst.val, aoff, alen, arow, aval, c->merge_light, c->merge_chunk, c->wave_blocks};
    check(c, hipMemsetAsync(d_n + 1, 0, 16, s), "memset");
    check(c, launch_merge_classify(mp, ub, flag, qwave, qblock, d_n + 1, d_err, nullptr, nullptr, s), "merge classify");
    check(c, scan_excl_u64(ub, ub, S2, stmp, ub + S2, s), "scan");
    uint64_t tp = S2 ? read_u64(c, ub + S2) : 0;
    uint32_t* prow = buf<uint32_t>(c, "pt.row", tp);
    uint64_t* pval = buf<uint64_t>(c, "pt.val", tp);
    uint32_t* pcnt = buf<uint32_t>(c, "pt.cnt", S2 + 1);
    check(c, launch_merge(mp, flag, qwave, qblock, d_n + 1, ub, 0, prow, pval, pcnt, nullptr, nullptr, s), "merge");
    uint64_t* slot = buf<uint64_t>(c, "err_slot", 1);
    check(c, hipMemsetAsync(slot, 0, sizeof(uint64_t), s), "memset");
    check(c, hipMemcpyAsync(slot, d_err, sizeof(int), hipMemcpyDeviceToDevice, s), "copy");
    uint64_t ev = read_u64(c, slot);
    if (ev & 32) {  // a column with more than 256 inputs: use the power iteration
        check(c, hipMemsetAsync(d_err, 0, sizeof(int), s), "memset");
        return false;
    }
    if (ev) fail(c, MS_ERR_INTERNAL, "consistency check failed in path counting (flag " + std::to_string(ev) + ")");
    uint64_t* rp = buf<uint64_t>(c, "m21.rowptr", S2 + 1);
    uint64_t nP = counts_to_rowptr(c, pcnt, S2, rp);
    ms_csr m21 = csr_buf(c, "m21", S2, S1, nP);
    check(c, launch_compact(ub, (const uint64_t*)m21.rowptr, S2, nP, prow, pval, m21.col, m21.val, s), "compact");
    out->m21 = m21;
    transpose(c, out->m21, "m21t", out->m21t, nullptr, NO_BOUND, true);  // M21 rows are sorted by column
    st.spgemm_iters = levels;
    st.nnz_astar = (int64_t)used;
    st.products = (int64_t)(used + tp);
    return true;
}
// The ready schedule with entry-parallel merges (see paths.hip).
// Junctions are first numbered in topological order: a sweep over the
// junction DAG releases each level's successors (the ready frontier) and
// the concatenated frontiers give the new numbering, applied to A, B and
// B* before their transposes.  A level is then a contiguous range of
// columns, so per-column metadata is read in order and no frontier has to
// be kept while merging.  Per level: input counts, their scan, one thread
// per input entry ranking it in its column, a scan of the run heads that
// writes them out.  A* columns are stored gap-free within a level; levels are
// placed at their upper-bound offsets.  P is written directly as M21 (rows
// 2-saddles).  No column size limit.
void paths_entry(ms_ctx* c, const ms_csr& A, const ms_csr& B, const ms_csr& Bs, const ms_csr& D, uint64_t S1,
                 uint64_t S2, uint64_t J, ms_arcs* out, int* d_err, SideTask& side) {
    hipStream_t s = cur_stream(c);
    struct Abandon {  // the helper's work below uses this function's locals
        SideTask& t;
        ~Abandon() { t.abandon(); }
    } abandon_on_exit{side};
    ms_stats& st = out->stats;
    // ---- topological numbering --------------------------------------------
    uint32_t* indeg = buf<uint32_t>(c, "pr.indeg", J + 1);
    uint32_t* order = buf<uint32_t>(c, "pr.order", J + 1);
    uint32_t* newid = buf<uint32_t>(c, "pr.newid", J + 1);
    unsigned long long* d_n = (unsigned long long*)buf<uint64_t>(c, "pr.counts", 3);
    check(c, hipMemsetAsync(indeg, 0, sizeof(uint32_t) * (J + 1), s), "memset");
    check(c, hipMemsetAsync(d_n, 0, 24, s), "memset");
    check(c, launch_hist(B.col, (uint64_t)B.nnz, indeg, s), "in-degrees");
    check(c, launch_sources(indeg, J, order, d_n, s), "sources");
    // levels on the device, SWEEP_BATCH per host round trip (d_n[0]: everything appended so far)
    std::vector<uint64_t> lvl{0};
    if (J > 0) {
        constexpr uint64_t SWEEP_BATCH = 16;
        uint64_t* lv = buf_keep<uint64_t>(c, "pr.lv", SWEEP_BATCH + 2, 0);
        check(c, hipMemsetAsync(lv, 0, sizeof(uint64_t), s), "memset");
        uint64_t L = 0;
        for (bool done = false; !done;) {
            const uint64_t L0 = L;
            lv = buf_keep<uint64_t>(c, "pr.lv", L0 + SWEEP_BATCH + 2, L0 + 1);
            for (; L < L0 + SWEEP_BATCH; L++)
                check(c, launch_sweep_level(order, lv, L, (const uint64_t*)B.rowptr, B.col, indeg, d_n, d_err, s),
                      "sweep");
            // lv[L0 + 1 .. L]: the boundaries sealed in this batch
            const uint64_t* h = readback(c, lv + L0 + 1, SWEEP_BATCH);
            for (uint64_t q = 0; q < SWEEP_BATCH && !done; q++) {
                if (h[q] == lvl.back()) done = true;  // an empty level: the sweep is complete
                else lvl.push_back(h[q]);
            }
            if (lvl.size() > J + 2) fail(c, MS_ERR_INTERNAL, "path counting did not terminate");
        }
    }
    if (lvl.back() != J) fail(c, MS_ERR_INTERNAL, "the junction graph has a cycle");
    const uint64_t nlev = lvl.size() - 1;
    check(c, launch_invert(order, J, newid, s), "invert");
    ms_csr At, Bt, Bst, Dt;
    // minor multiplicities are at most 4: at most four paths leave a source.
    // B* and D are first needed by the last product (P), so the helper thread
    // transposes them on the side stream (once the saddle-extremum arcs are
    // done there) while the levels of A* are counted here.
    side.finish(s);
    side.start(s, [&]() {
        transpose(c, Bs, "Bst", Bst, newid, 4);  // 2-saddle x junction (renumbered)
        transpose(c, D, "Dt", Dt, nullptr, 4);   // 2-saddle x 1-saddle
    });
    // A, B by their target junctions in the new numbering; sources relabelled after the transposes
    check(c, launch_relabel(A.col, (uint64_t)A.nnz, newid, s), "relabel");
    check(c, launch_relabel(B.col, (uint64_t)B.nnz, newid, s), "relabel");
    transpose(c, A, "At", At, nullptr, 4);     // junction x 1-saddle
    transpose(c, B, "Bt", Bt, newid, 4);       // junction x predecessor junction (sources renumbered)
    // ---- levels --------------------------------------------------------------
    const uint64_t nmax = (J > S2 ? J : S2) + 1;
    uint64_t* ub = buf<uint64_t>(c, "pr.ub", nmax + 1);
    uint64_t* aoff = buf<uint64_t>(c, "pr.aoff", J + 1);
    uint32_t* alen = buf<uint32_t>(c, "pr.alen", J + 1);
    uint64_t used = 0, products = 0;
    uint32_t* arow = buf_keep<uint32_t>(c, "astar.row", 1, 0);
    uint64_t* aval = buf_keep<uint64_t>(c, "astar.val", 1, 0);
    ms_csr m21{};
    // one level: input counts and their scan, rank every input entry, then
    // scan the run heads and write them at base (into the A* storage or M21)
    auto level = [&](MergeLaunch& m, uint64_t n, bool to_astar, uint64_t& base, uint64_t*& hp) -> uint64_t {
        uint64_t* stmp = buf<uint64_t>(c, "scan_tmp", scan_tmp_elems(n) + 1);
        check(c, launch_entry_ub(m, ub, s), "entry ub");
        check(c, scan_excl_u64(ub, ub, n, stmp, ub + n, s), "scan");
        const uint64_t T = n ? read_u64(c, ub + n) : 0;
        uint32_t* orow;
        uint64_t* oval;
        if (to_astar) {  // room for this level's columns at their upper bound
            arow = buf_keep<uint32_t>(c, "astar.row", used + T, used);
            aval = buf_keep<uint64_t>(c, "astar.val", used + T, used);
            m.arow = arow;
            m.aval = aval;
            orow = arow;
            oval = aval;
            base = used;
        } else {  // M21 sized for the upper bound; nnz is set once the heads are counted
            m21 = csr_buf(c, "m21", S2, S1, T);
            orow = m21.col;
            oval = m21.val;
            base = 0;
        }
        uint32_t* hrow = buf<uint32_t>(c, "pe.hrow", T);
        uint64_t* hval = buf<uint64_t>(c, "pe.hval", T);
        uint8_t* head = buf<uint8_t>(c, "pe.head", T);
        hp = buf<uint64_t>(c, "pe.hp", T + 1);
        uint32_t* bstart = buf<uint32_t>(c, "pe.bstart", rank_blocks(T));
        // levels of short columns (fewer than RANK_COLOF_AVG entries each on
        // average) have many entries beyond a rank block's column window:
        // their columns are listed once instead of searched per entry
        const uint32_t* colof = nullptr;
        if (T > 0 && T < RANK_COLOF_AVG * n) {
            uint32_t* cb = buf<uint32_t>(c, "pe.colof", T);
            check(c, launch_expand_rows(ub, n, nullptr, cb, s), "entry columns");
            colof = cb;
        }
        const bool timed = c->timing && T > 0;
        if (timed) {
            while (c->rank_ev.size() < 2 * (c->rank_used + 1)) {
                hipEvent_t ev;
                check(c, hipEventCreate(&ev), "event create");
                c->rank_ev.push_back(ev);
            }
            check(c, hipEventRecord(c->rank_ev[2 * c->rank_used], s), "event record");
        }
        check(c, launch_entry_rank(m, ub, T, bstart, colof, hrow, hval, head, s), "entry rank");
        if (timed) {
            check(c, hipEventRecord(c->rank_ev[2 * c->rank_used + 1], s), "event record");
            c->rank_used++;
            c->rank_entries += (int64_t)T;
        }
        uint64_t* htmp = buf<uint64_t>(c, "pe.htmp", head_scan_tmp_elems(T));
        check(c, launch_head_scan_emit(head, T, hrow, hval, base, orow, oval, hp, htmp, s), "head scan");
        return T;
    };
    for (uint64_t L = 0; L < nlev; L++) {
        MergeLaunch m{nullptr, lvl[L + 1] - lvl[L], (const uint64_t*)At.rowptr, At.col, At.val,
                      (const uint64_t*)Bt.rowptr, Bt.col, Bt.val, aoff, alen, arow, aval, 0, 1, 1, (uint32_t)lvl[L]};
        uint64_t base;
        uint64_t* hp;
        const uint64_t T = level(m, m.n, true, base, hp);
        check(c, launch_entry_cols(m, ub, hp, base, aoff, alen, nullptr, s), "entry cols");
        used += T;
        products += T;
    }
    // P columns, written as M21 (rows 2-saddles) in canonical order
    side.finish(s);
    MergeLaunch mp{nullptr, S2, (const uint64_t*)Dt.rowptr, Dt.col, Dt.val, (const uint64_t*)Bst.rowptr, Bst.col,
                   Bst.val, aoff, alen, arow, aval, 0, 1, 1};
    uint64_t pbase;
    uint64_t* hp;
    const uint64_t T = level(mp, S2, false, pbase, hp);
    m21.nnz = (int64_t)read_u64(c, hp + T);
    if (S2 == 0) check(c, hipMemsetAsync(m21.rowptr, 0, sizeof(int64_t), s), "memset");
    check(c, launch_entry_cols(mp, ub, hp, 0, nullptr, nullptr, (uint64_t*)m21.rowptr, s), "entry cols");
    check_err_flag(c, d_err, "path counting");
    out->m21 = m21;
    transpose(c, out->m21, "m21t", out->m21t, nullptr, NO_BOUND, true);  // M21 rows are sorted by column
    // exact nnz of A*: the sum of the column lengths
    uint64_t* sum = buf<uint64_t>(c, "pe.asum", 1);
    check(c, launch_sum_u32(alen, J, sum, s), "sum");
    st.spgemm_iters = (int64_t)nlev;
    st.nnz_astar = (int64_t)read_u64(c, sum);
    st.products = (int64_t)(products + T);
    if (c->timing) c->rank_heads += st.nnz_astar + m21.nnz;
}
// The saddle-extremum arcs: pointer jumping to the extremum every vertex and
// every 3-cell flows to (Section 3.4), M10 and M32 (Section 3.5,
// "Saddle-Extrema arcs"), the manifold labels and the two transposes.
void extremum_arcs(ms_ctx* c, const Geo& g, const uint32_t* s1, const uint32_t* s2, uint64_t S0, uint64_t S1,
                   uint64_t S2, uint64_t S3, uint32_t* Pv, uint32_t* Pc, ms_arcs* out, ms_stats& st) {
    hipStream_t s = cur_stream(c);
    int* d_err = buf<int>(c, "cn_err", 1);
    check(c, hipMemsetAsync(d_err, 0, sizeof(int), s), "memset");
    int* d_chg = (int*)buf<uint64_t>(c, "pj_changed", 32);  // 64 flag words
    for (int which = 0; which < 2; which++) {
        uint32_t* P = which == 0 ? Pv : Pc;
        int64_t rounds = 0;
        for (;;) {
            check(c, hipMemsetAsync(d_chg, 0, 64 * sizeof(int), s), "memset");
            check(c, launch_pj_round(P, g.nv, d_chg, s), "pj round");
            rounds++;
            const uint64_t* h = readback(c, (const uint64_t*)d_chg, 32);
            bool any = false;
            for (int i = 0; i < 32; i++) any = any || h[i] != 0;
            if (!any) break;
            if (rounds > 64) fail(c, MS_ERR_INTERNAL, "pointer jumping did not converge (cycle in the gradient)");
        }
        (which == 0 ? st.pj_rounds_vertex : st.pj_rounds_cube) = rounds;
    }
    {
        uint32_t* rc = buf<uint32_t>(c, "rowcnt", S1 > S2 ? S1 : S2);
        // M10
        ms_csr& m10 = out->m10;
        uint64_t* rp = buf<uint64_t>(c, "m10.rowptr", S1 + 1);
        check(c, launch_m10(false, s1, S1, g, Pv, rc, nullptr, nullptr, nullptr, d_err, s), "m10 count");
        uint64_t nnz = counts_to_rowptr(c, rc, S1, rp);
        m10 = csr_buf(c, "m10", S1, S0, nnz);
        check(c, launch_m10(true, s1, S1, g, Pv, nullptr, (const uint64_t*)m10.rowptr, m10.col, m10.val, d_err, s),
              "m10 fill");
        // M32 transposed (rows 2-saddles)
        ms_csr& m32t = out->m32t;
        uint64_t* rp2 = buf<uint64_t>(c, "m32t.rowptr", S2 + 1);
        check(c, launch_m32t(false, s2, S2, g, Pc, rc, nullptr, nullptr, nullptr, d_err, s), "m32t count");
        uint64_t nnz2 = counts_to_rowptr(c, rc, S2, rp2);
        m32t = csr_buf(c, "m32t", S2, S3, nnz2);
        check(c, launch_m32t(true, s2, S2, g, Pc, nullptr, (const uint64_t*)m32t.rowptr, m32t.col, m32t.val, d_err, s),
              "m32t fill");
        check_err_flag(c, d_err, "saddle-extremum arcs");
        // a batch relabels with per-field ranks once its field counts are known
        if (g.nf == 1) check(c, launch_manifold_labels(Pv, Pc, g, nullptr, s), "manifold labels");
        out->min_label = Pv;
        out->max_label = Pc;
        // saddle-extremum multiplicities are 1 or 2
        transpose(c, m10, "m10t", out->m10t, nullptr, 2);
        transpose(c, m32t, "m32", out->m32, nullptr, 2);
    }
}

}  // namespace

void connect_impl(ms_ctx* c, const uint32_t* grad, const Geo& g, const uint32_t* crit, const int64_t cnt[4],
                  ms_arcs* out) {
    memset(out, 0, sizeof(*out));
    c->rank_used = 0;  // rank timing pairs of an earlier call that were not accumulated
    c->side_used = 0;  // and side-stream spans
    hipStream_t s = cur_stream(c);
    const uint64_t S0 = (uint64_t)cnt[0], S1 = (uint64_t)cnt[1], S2 = (uint64_t)cnt[2], S3 = (uint64_t)cnt[3];
    const uint32_t* s1 = crit + S0;
    const uint32_t* s2 = crit + S0 + S1;
    int* d_err = buf<int>(c, "cn_err", 1);
    check(c, hipMemsetAsync(d_err, 0, sizeof(int), s), "memset");
    ms_stats& st = out->stats;

    // ---- saddle-extremum arcs ------------------------------------------------
    uint32_t* Pv = buf<uint32_t>(c, "pv", g.nv);
    uint32_t* Pc = buf<uint32_t>(c, "pc", g.nv);
    uint32_t* label = buf<uint32_t>(c, "cell_label", (uint64_t)6 * g.nv);  // planes of edges and quads
    check(c, launch_pj_init(grad, g, Pv, Pc, d_err, s), "pj init");
    check(c, launch_label(crit, cnt, grad, g, Pv, Pc, label, d_err, s), "label");
    check_err_flag(c, d_err, "critical list labelling");
    // The saddle-extremum arcs read only the gradient, the critical lists and
    // the pointers set up above, and nothing after them reads what they
    // write: once the search is queued, a helper thread queues them on the
    // side stream, where they overlap the minor and the path counting queued
    // by this thread (started before the search they slowed it about as much
    // as they saved: both are bound by scattered memory traffic).
    SideTask side(c);

    mark(c, 3);
    // ---- saddle-saddle reachability (frontier BFS) --------------------------
    uint64_t nvis = ((uint64_t)g.nv + 3) / 4;
    uint32_t* vis = buf<uint32_t>(c, "visited", nvis);
    check(c, hipMemsetAsync(vis, 0, 4 * nvis, s), "memset");
    // the frontiers, level after level, in one queue: the 1-saddles, then the
    // nodes in the order they are first reached (each once, by its visited
    // bit), at most one per edge of the grid.  The packed tail counts the
    // queue (low 32 bits) and the junctions (high 32 bits).
    uint64_t J = 0, reach = 0;
    int64_t levels = 0;
    const uint64_t max_nodes = (uint64_t)3 * g.nv + 1;
    if (S1 > 0) {
        uint32_t* queue = buf<uint32_t>(c, "bfs.queue", max_nodes);
        unsigned long long* tail = (unsigned long long*)buf<uint64_t>(c, "bfs.tail", 1);
        check(c, hipMemcpyAsync(queue, s1, 4 * S1, hipMemcpyDeviceToDevice, s), "copy");
        check(c, launch_set_u64((uint64_t*)tail, S1, s), "tail init");
        constexpr uint64_t BFS_BATCH = 16;
        uint64_t* lv = buf_keep<uint64_t>(c, "bfs.lv", BFS_BATCH + 2, 0);
        check(c, launch_set_u64(lv, 0, s), "level start");
        std::vector<uint64_t> bound{0};  // lv as read back
        uint64_t L = 0;
        for (bool done = false; !done;) {
            const uint64_t L0 = L;
            lv = buf_keep<uint64_t>(c, "bfs.lv", L0 + BFS_BATCH + 2, L0 + 1);
            for (; L < L0 + BFS_BATCH; L++)
                check(c, launch_bfs_level(queue, max_nodes, lv, L, grad, g, vis, tail, label, s), "bfs level");
            // lv[L0 + 1 .. L]: the boundaries sealed in this batch
            const uint64_t* h = readback(c, lv + L0 + 1, BFS_BATCH);
            for (uint64_t q = 0; q < BFS_BATCH && !done; q++) {
                if (h[q] == bound.back()) done = true;  // an empty level: the search is complete
                else bound.push_back(h[q]);
            }
            if (bound.size() > max_nodes + 1) fail(c, MS_ERR_INTERNAL, "BFS did not terminate");
        }
        levels = (int64_t)bound.size() - 1;
        reach = bound.back() - S1;
        J = readback(c, (const uint64_t*)tail, 1)[0] >> 32;
        if (bound.back() > max_nodes) fail(c, MS_ERR_INTERNAL, "BFS queue overflow");
    }
    st.bfs_levels = levels;
    st.reachable = (int64_t)reach;
    st.junctions = (int64_t)J;

    // junctions numbered in cell order (jlist: id -> cell; their labels get the ids)
    uint32_t* jlist = buf<uint32_t>(c, "jlist", J + 1);
    {
        const uint64_t nb = junction_blocks(g.nv);
        uint64_t* bc = buf<uint64_t>(c, "junc_blocks", nb + 1);
        uint64_t* stmp = buf<uint64_t>(c, "scan_tmp", scan_tmp_elems(nb) + 1);
        check(c, launch_junc_count(vis, label, g.nv, bc, s), "junction count");
        check(c, scan_excl_u64(bc, bc, nb, stmp, bc + nb, s), "scan");
        if (read_u64(c, bc + nb) != J) fail(c, MS_ERR_INTERNAL, "junction count differs from the search's");
        check(c, launch_junc_emit(vis, label, g.nv, bc, jlist, s), "junction numbering");
    }

    mark(c, 4);
    side.start(s, [&]() { extremum_arcs(c, g, s1, s2, S0, S1, S2, S3, Pv, Pc, out, st); });
    // ---- DAG minor ----------------------------------------------------------
    const uint64_t NS = S1 + J;
    uint8_t* out_t = buf<uint8_t>(c, "minor_t", 4 * NS);
    uint32_t* out_id = buf<uint32_t>(c, "minor_id", 4 * NS);
    check(c, launch_minor_trace(s1, S1, jlist, J, grad, g, label, max_nodes, S2, out_t, out_id, d_err, s), "minor trace");
    uint32_t* cj = buf<uint32_t>(c, "minor_cj", NS);
    uint32_t* cs = buf<uint32_t>(c, "minor_cs", NS);
    check(c, launch_minor_rows(false, out_t, out_id, S1, NS, cj, cs, nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, s),
          "minor rows");
    check_err_flag(c, d_err, "DAG minor tracing");
    uint64_t* rpA = buf<uint64_t>(c, "A.rowptr", S1 + 1);
    uint64_t* rpD = buf<uint64_t>(c, "D.rowptr", S1 + 1);
    uint64_t* rpB = buf<uint64_t>(c, "B.rowptr", J + 1);
    uint64_t* rpBs = buf<uint64_t>(c, "Bs.rowptr", J + 1);
    uint64_t nA = counts_to_rowptr(c, cj, S1, rpA);
    uint64_t nD = counts_to_rowptr(c, cs, S1, rpD);
    uint64_t nB = counts_to_rowptr(c, cj + S1, J, rpB);
    uint64_t nBs = counts_to_rowptr(c, cs + S1, J, rpBs);
    ms_csr A = csr_buf(c, "A", S1, J, nA), D = csr_buf(c, "D", S1, S2, nD);
    ms_csr B = csr_buf(c, "B", J, J, nB), Bs = csr_buf(c, "Bs", J, S2, nBs);
    check(c, launch_minor_rows(true, out_t, out_id, S1, NS, nullptr, nullptr, (const uint64_t*)A.rowptr, A.col, A.val,
                               (const uint64_t*)D.rowptr, D.col, D.val, (const uint64_t*)B.rowptr, B.col, B.val,
                               (const uint64_t*)Bs.rowptr, Bs.col, Bs.val, s),
          "minor fill");
    st.nnz_a = (int64_t)nA;
    st.nnz_b = (int64_t)nB;
    st.nnz_bstar = (int64_t)nBs;
    st.nnz_d = (int64_t)nD;

    mark(c, 5);
    // ---- path counting --------------------------------------------------------
    bool done = false;
    if (c->path_schedule == MS_PATHS_READY) done = paths_ready(c, A, B, Bs, D, S1, S2, J, out, d_err);
    if (c->path_schedule == MS_PATHS_ENTRY) {
        paths_entry(c, A, B, Bs, D, S1, S2, J, out, d_err, side);
        done = true;
    }
    if (!done) paths_power(c, A, B, Bs, D, S1, S2, J, out);
    unsigned long long* d_sat = (unsigned long long*)buf<uint64_t>(c, "sat_count", 1);
    check(c, hipMemsetAsync(d_sat, 0, 8, s), "memset");
    check(c, launch_count_sat(out->m21t.val, (uint64_t)out->m21t.nnz, d_sat, s), "count saturated");
    out->n_saturated = (int64_t)read_u64(c, (const uint64_t*)d_sat);
    st.nnz_p = out->m21t.nnz;
    side.finish(s);
}

}  // namespace msc

// Launchers of the column-merge path counting (paths.hip).
#pragma once

#include "prims.h"

namespace msc {

// Output column c of a merge is the sorted union of its base list (row c of
// the base CSR) and the A* columns of its predecessors (row c of the
// predecessor CSR: junction ids and multiplicities).
struct MergeLaunch {
    const uint32_t* cols;  // output columns to form (null: 0..n-1)
    uint64_t n;
    const uint64_t* brp;
    const uint32_t* bcol;
    const uint64_t* bval;
    const uint64_t* prp;
    const uint32_t* pcol;
    const uint64_t* pval;
    const uint64_t* aoff;  // A* column offsets / lengths / storage
    const uint32_t* alen;
    const uint32_t* arow;
    const uint64_t* aval;
    uint32_t light_ub;  // columns with at most this many inputs (and <= 8 lists) merge in one thread
    uint32_t chunk;     // other columns merge in chunks of at most this many entries (1..4096)
    uint32_t wave_blocks;  // workgroups of the wave-path launch (each wave strides over its queue)
    uint32_t col0 = 0;     // with cols null: the columns are col0 .. col0 + n - 1
};

// Upper bound (input entries) per output column into ub, a path flag per
// column, and the queues of columns for the wave path (qwave, count qn[0])
// and the workgroup path (qblock, count qn[1]); qn must be zero on entry.
// Columns with more than 256 input lists set bit 32 of *err and are given an
// empty range.
hipError_t launch_merge_classify(const MergeLaunch& m, uint64_t* ub, uint8_t* flag, uint32_t* qwave, uint32_t* qblock,
                                 unsigned long long* qn, int* err, uint64_t* col_off, uint32_t* col_len,
                                 hipStream_t s);
// Forms every output column i at out_base + off[i] (off: exclusive scan of
// ub).  Writes its length to cnt[i] and/or to (col_off, col_len)[column].
hipError_t launch_merge(const MergeLaunch& m, const uint8_t* flag, const uint32_t* qwave, const uint32_t* qblock,
                        const unsigned long long* qn, const uint64_t* off, uint64_t out_base, uint32_t* orow,
                        uint64_t* oval, uint32_t* cnt, uint64_t* col_off, uint32_t* col_len, hipStream_t s);
// Entry-parallel merges (one thread per input entry): input counts per
// column into ub; then, with off the exclusive scan of ub (n + 1 entries,
// off[n] = T), the ranked run heads (head flag bytes: bit 0 run head, bit 1
// a column's first position; rows and summed values at their merged
// positions); then the compacted output at base + (heads before p) with
// that prefix in hp at every column's first position and at T; then each
// column's range (col_off/col_len by column id and/or a CSR row pointer)
// from hp[off[i]].
hipError_t launch_entry_ub(const MergeLaunch& m, uint64_t* ub, hipStream_t s);
// bstart: scratch of rank_blocks(T) entries (the first column of each rank
// block); colof: null, or the level column of every entry (T entries)
size_t rank_blocks(uint64_t T);
hipError_t launch_entry_rank(const MergeLaunch& m, const uint64_t* off, uint64_t T, uint32_t* bstart,
                             const uint32_t* colof, uint32_t* hrow, uint64_t* hval, uint8_t* head, hipStream_t s);
hipError_t launch_entry_cols(const MergeLaunch& m, const uint64_t* off, const uint64_t* hp, uint64_t base,
                             uint64_t* col_off, uint32_t* col_len, uint64_t* rowptr, hipStream_t s);
// Copies column i from src_off[i] to dst_off[i] (dst_off: n + 1 entries).
hipError_t launch_compact(const uint64_t* src_off, const uint64_t* dst_off, uint64_t n, uint64_t total,
                          const uint32_t* srow, const uint64_t* sval, uint32_t* drow, uint64_t* dval, hipStream_t s);
// base_rp / ub optional: the input counts of the first frontier's columns
hipError_t launch_ready_init(const uint64_t* prp, uint64_t J, uint32_t* indeg, uint32_t* ready,
                             unsigned long long* nready, const uint64_t* base_rp, uint64_t* ub, hipStream_t s);
// ub_next optional (with base_rp, prp, pcol, alen): the input counts of
// the released columns, in the order of `next`
// One level of the device-driven topological sweep: seals lv[L + 1] = *tail,
// then releases the successors of order[lv[L], lv[L + 1]) (appended at
// *tail).  lv[0] and *tail (the sources in order[0, *tail)) are set by the
// caller.
hipError_t launch_sweep_level(uint32_t* order, uint64_t* lv, uint64_t L, const uint64_t* brp, const uint32_t* bcol,
                              uint32_t* indeg, unsigned long long* tail, int* err, hipStream_t s);
hipError_t launch_release(const uint32_t* ready, uint64_t n, const uint64_t* brp, const uint32_t* bcol,
                          uint32_t* indeg, uint32_t* next, unsigned long long* nnext, int* err, const uint64_t* base_rp,
                          const uint64_t* prp, const uint32_t* pcol, const uint32_t* alen, uint64_t* ub_next,
                          hipStream_t s);
// Topological numbering: the junctions with zero in-degree appended to out
// (count in *n, which must be zero on entry); inv[order[i]] = i; x[i] =
// map[x[i]] in place.
hipError_t launch_sources(const uint32_t* indeg, uint64_t J, uint32_t* out, unsigned long long* n, hipStream_t s);
hipError_t launch_invert(const uint32_t* order, uint64_t n, uint32_t* inv, hipStream_t s);
hipError_t launch_relabel(uint32_t* x, uint64_t n, const uint32_t* map, hipStream_t s);
// Exclusive scan of the run-head bits: each head's row and count written at
// base + (heads before it); hp (T + 1 entries) gets that prefix at the
// positions flagged as column starts and hp[T] = number of heads (other
// entries of hp are left untouched); tmp needs head_scan_tmp_elems(T)
// entries.
size_t head_scan_tmp_elems(uint64_t T);
hipError_t launch_head_scan_emit(const uint8_t* head, uint64_t T, const uint32_t* hrow, const uint64_t* hval,
                                 uint64_t base, uint32_t* orow, uint64_t* oval, uint64_t* hp, uint64_t* tmp,
                                 hipStream_t s);

}  // namespace msc

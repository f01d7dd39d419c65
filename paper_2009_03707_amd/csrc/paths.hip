// Path counting in the DAG minor by column merges (Section 3.3).
//
// The paper accumulates A* = sum_k A B^k by repeating frontier <- frontier*B
// until the product vanishes; A* is the solution of A* = A + A* B.  Here the
// same sparse integer products are evaluated column block by column block in
// topological order of the junction DAG: the column A*(:, j) of a junction j
// is A(:, j) plus the columns of its minor predecessors p scaled by B(p, j),
// and it is formed once, when every predecessor column is complete (a ready
// frontier).  Each (1-saddle, junction) pair is then produced once instead
// of once per distinct path length.  Columns are sorted lists of 1-saddle
// ranks, so forming a column is a merge of sorted lists, with saturating
// u64 arithmetic (exact up to 2^64-1, independent of the order of sums).
//
// P = D + A* B* is formed the same way per 2-saddle column, which yields M21
// (rows 2-saddles, columns 1-saddles) directly in canonical order.
//
// Columns with few, short inputs are merged by one thread in registers.  All
// others go to a workgroup that merges in chunks: a binary search on the row
// value picks a threshold so that every input entry up to it fits in LDS;
// those entries are loaded (coalesced, per input list), bitonic-sorted,
// de-duplicated with saturating sums and written; the lists advance past the
// threshold.  Entries with equal rows never straddle two chunks, so the
// result is exact for any column length.
//
// Each column is written at an offset that reserves its input count (an
// upper bound of its length), which avoids a separate counting pass; the A*
// storage may therefore hold small gaps between columns.
#include "paths.h"

namespace msc {
namespace {

constexpr int BT = 256;
constexpr int LIGHT_K = 8;         // thread path: at most this many input lists
constexpr int MAX_K = 256;         // block path: at most this many input lists
constexpr int CAP = 4096;          // entries per LDS chunk
constexpr uint32_t NOROW = 0xFFFFFFFFu;

struct MergeArgs {
    const uint32_t* cols;  // output column ids (null: identity 0..n-1)
    uint64_t n;
    const uint64_t* brp;   // base list per output column: CSR (row ids, values)
    const uint32_t* bcol;
    const uint64_t* bval;
    const uint64_t* prp;   // predecessor junctions per output column: CSR (junction, multiplicity)
    const uint32_t* pcol;
    const uint64_t* pval;
    const uint64_t* aoff;  // A* columns: offset and length per junction, rows, values
    const uint32_t* alen;
    const uint32_t* arow;
    const uint64_t* aval;
    uint32_t light_ub;  // thread path: at most this many input entries
    uint32_t chunk;     // workgroup path: entries per chunk (<= CAP)
};

struct ListRef {
    const uint32_t* row;
    const uint64_t* val;
    uint64_t len;
    uint64_t mul;
};

__device__ __forceinline__ ListRef list_of(const MergeArgs& a, uint32_t c, uint32_t s) {
    ListRef L;
    if (s == 0) {
        uint64_t b = a.brp[c], e = a.brp[c + 1];
        L.row = a.bcol + b;
        L.val = a.bval + b;
        L.len = e - b;
        L.mul = 1;
    } else {
        uint64_t q = a.prp[c] + (s - 1);
        uint32_t p = a.pcol[q];
        L.row = a.arow + a.aoff[p];
        L.val = a.aval + a.aoff[p];
        L.len = a.alen[p];
        L.mul = a.pval[q];
    }
    return L;
}

__device__ __forceinline__ uint32_t num_lists(const MergeArgs& a, uint32_t c) {
    return 1 + (uint32_t)(a.prp[c + 1] - a.prp[c]);
}

// Upper bound (input entries) of every output column, and the queue of
// columns for the workgroup path.
__global__ __launch_bounds__(BT) void k_classify(MergeArgs a, uint64_t* __restrict__ ub,
                                                 uint8_t* __restrict__ heavy_flag, uint32_t* __restrict__ heavy,
                                                 unsigned long long* __restrict__ nheavy, int* __restrict__ err,
                                                 uint64_t* __restrict__ col_off, uint32_t* __restrict__ col_len) {
    __shared__ unsigned long long sc[BT / WAVE + 1];
    __shared__ unsigned long long base;
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    unsigned long long h = 0;
    if (i < a.n) {
        uint32_t c = a.cols ? a.cols[i] : (uint32_t)i;
        uint32_t k = num_lists(a, c);
        uint64_t u = a.brp[c + 1] - a.brp[c];
        for (uint32_t s = 1; s < k; s++) u += a.alen[a.pcol[a.prp[c] + (s - 1)]];
        ub[i] = u;
        bool hv = !(k <= (uint32_t)LIGHT_K && u <= (uint64_t)a.light_ub);
        if (hv && k > (uint32_t)MAX_K) {
            atomicOr(err, 32);  // skipped: the caller falls back to the power iteration
            hv = false;
            ub[i] = 0;
            heavy_flag[i] = 2;
            if (col_off) {  // an empty column keeps later reads in bounds
                col_off[c] = 0;
                col_len[c] = 0;
            }
        } else {
            heavy_flag[i] = hv ? 1 : 0;
        }
        h = hv ? 1 : 0;
    }
    unsigned long long tot;
    unsigned long long ex = block_excl_scan<unsigned long long, BT>(h, sc, tot);
    if (threadIdx.x == 0) base = tot ? atomicAdd(nheavy, tot) : 0;
    __syncthreads();
    if (h) heavy[base + ex] = (uint32_t)i;
}

// Thread-per-column merge (few, short inputs), written at out_base + off[i].
__global__ __launch_bounds__(BT) void k_merge_thread(MergeArgs a, const uint8_t* __restrict__ heavy_flag,
                                                     const uint64_t* __restrict__ off, uint64_t out_base,
                                                     uint32_t* __restrict__ orow, uint64_t* __restrict__ oval,
                                                     uint32_t* __restrict__ cnt, uint64_t* __restrict__ col_off,
                                                     uint32_t* __restrict__ col_len) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= a.n || heavy_flag[i]) return;
    uint32_t c = a.cols ? a.cols[i] : (uint32_t)i;
    uint32_t k = num_lists(a, c);
    const uint32_t* rp[LIGHT_K];
    const uint64_t* vp[LIGHT_K];
    uint32_t rem[LIGHT_K], head[LIGHT_K];
    uint64_t mul[LIGHT_K];
#pragma unroll
    for (int s = 0; s < LIGHT_K; s++) {
        head[s] = NOROW;
        rem[s] = 0;
        rp[s] = nullptr;
        vp[s] = nullptr;
        mul[s] = 0;
        if ((uint32_t)s < k) {
            ListRef L = list_of(a, c, (uint32_t)s);
            rp[s] = L.row;
            vp[s] = L.val;
            rem[s] = (uint32_t)L.len;
            mul[s] = L.mul;
            if (L.len) head[s] = L.row[0];
        }
    }
    uint64_t o = out_base + off[i];
    uint32_t m = 0;
    for (;;) {
        uint32_t mn = NOROW;
#pragma unroll
        for (int s = 0; s < LIGHT_K; s++) mn = head[s] < mn ? head[s] : mn;
        if (mn == NOROW) break;
        uint64_t sum = 0;
#pragma unroll
        for (int s = 0; s < LIGHT_K; s++) {
            if (head[s] == mn) {
                sum = sat_add(sum, sat_mul(vp[s][0], mul[s]));
                rp[s]++;
                vp[s]++;
                rem[s]--;
                head[s] = rem[s] ? rp[s][0] : NOROW;
            }
        }
        orow[o + m] = mn;
        oval[o + m] = sum;
        m++;
    }
    if (cnt) cnt[i] = m;
    if (col_off) {
        col_off[c] = o;
        col_len[c] = m;
    }
}

// number of entries of a sorted list with row <= t
__device__ __forceinline__ uint32_t count_le(const uint32_t* row, uint32_t len, uint32_t t) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (row[mid] <= t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Workgroup-per-column chunked merge (see the file comment).
__global__ __launch_bounds__(BT) void k_merge_block(MergeArgs a, const uint32_t* __restrict__ heavy,
                                                    const unsigned long long* __restrict__ nheavy,
                                                    const uint64_t* __restrict__ off, uint64_t out_base,
                                                    uint32_t* __restrict__ orow, uint64_t* __restrict__ oval,
                                                    uint32_t* __restrict__ cnt, uint64_t* __restrict__ col_off,
                                                    uint32_t* __restrict__ col_len) {
    __shared__ uint32_t skey[CAP];
    __shared__ uint64_t sval[CAP];
    __shared__ const uint32_t* lrow[MAX_K];
    __shared__ const uint64_t* lval[MAX_K];
    __shared__ uint32_t lpos[MAX_K], llen[MAX_K], ltake[MAX_K], loff[MAX_K];
    __shared__ uint64_t lmul[MAX_K];
    __shared__ unsigned long long sc[BT / WAVE + 1];
    __shared__ uint32_t s_thr, s_total;
    const int tid = threadIdx.x;
    const uint64_t nh = *nheavy;
    for (uint64_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const uint32_t i = heavy[h];
        const uint32_t c = a.cols ? a.cols[i] : i;
        const uint32_t k = num_lists(a, c);
        for (uint32_t s = tid; s < k; s += BT) {
            ListRef L = list_of(a, c, s);
            lrow[s] = L.row;
            lval[s] = L.val;
            llen[s] = (uint32_t)L.len;
            lmul[s] = L.mul;
            lpos[s] = 0;
        }
        __syncthreads();
        const uint64_t o = out_base + off[i];
        uint64_t written = 0;
        // a row occurs at most once per list, so a chunk of at least k entries
        // always takes at least one row
        const uint32_t chunk = a.chunk > k ? a.chunk : k;
        for (;;) {
            // entries left in all lists
            unsigned long long left = 0;
            for (uint32_t s = tid; s < k; s += BT) left += llen[s] - lpos[s];
            unsigned long long tot;
            block_excl_scan<unsigned long long, BT>(left, sc, tot);
            if (tot == 0) break;
            // threshold: the largest row t with at most CAP entries <= t
            if (tot <= (unsigned long long)chunk) {
                if (tid == 0) s_thr = NOROW;
            } else {
                // invariant: count(lo) <= chunk (or lo is below every row), count(hi) > chunk
                uint32_t lo = 0, hi = NOROW;
                while (hi - lo > 1) {
                    uint32_t mid = lo + ((hi - lo) >> 1);
                    unsigned long long cntle = 0;
                    for (uint32_t s = tid; s < k; s += BT)
                        cntle += count_le(lrow[s] + lpos[s], llen[s] - lpos[s], mid);
                    unsigned long long ct;
                    block_excl_scan<unsigned long long, BT>(cntle, sc, ct);
                    if (ct <= (unsigned long long)chunk) lo = mid;
                    else hi = mid;
                }
                if (tid == 0) s_thr = lo;
            }
            __syncthreads();
            const uint32_t thr = s_thr;
            // how many entries each list contributes, and where they go
            for (uint32_t s = tid; s < k; s += BT)
                ltake[s] = thr == NOROW ? llen[s] - lpos[s] : count_le(lrow[s] + lpos[s], llen[s] - lpos[s], thr);
            __syncthreads();
            if (tid == 0) {
                uint32_t run = 0;
                for (uint32_t s = 0; s < k; s++) {
                    loff[s] = run;
                    run += ltake[s];
                }
                s_total = run;
            }
            __syncthreads();
            const uint32_t m = s_total;
            for (uint32_t s = 0; s < k; s++) {
                const uint32_t* rr = lrow[s] + lpos[s];
                const uint64_t* vv = lval[s] + lpos[s];
                const uint64_t mu = lmul[s];
                const uint32_t tk = ltake[s], lo2 = loff[s];
                for (uint32_t e = tid; e < tk; e += BT) {
                    skey[lo2 + e] = rr[e];
                    sval[lo2 + e] = sat_mul(vv[e], mu);
                }
            }
            uint32_t np2 = 1;
            while (np2 < m) np2 <<= 1;
            for (uint32_t e = m + tid; e < np2; e += BT) {
                skey[e] = NOROW;
                sval[e] = 0;
            }
            __syncthreads();
            // bitonic sort of skey (payload sval) over np2 entries
            for (uint32_t size = 2; size <= np2; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t e = tid; e < np2 / 2; e += BT) {
                        uint32_t p = 2 * stride * (e / stride) + (e % stride);
                        uint32_t q = p + stride;
                        bool up = (p & size) == 0;
                        uint32_t ka = skey[p], kb = skey[q];
                        if ((ka > kb) == up) {
                            skey[p] = kb;
                            skey[q] = ka;
                            uint64_t t = sval[p];
                            sval[p] = sval[q];
                            sval[q] = t;
                        }
                    }
                    __syncthreads();
                }
            }
            // de-duplicate: one output per run of equal rows
            for (uint32_t base = 0; base < m; base += BT) {
                uint32_t e = base + tid;
                unsigned long long head = (e < m && (e == 0 || skey[e] != skey[e - 1])) ? 1 : 0;
                unsigned long long hsum;
                unsigned long long ex = block_excl_scan<unsigned long long, BT>(head, sc, hsum);
                if (head) {
                    uint64_t sum = sval[e];
                    for (uint32_t f = e + 1; f < m && skey[f] == skey[e]; f++) sum = sat_add(sum, sval[f]);
                    orow[o + written + ex] = skey[e];
                    oval[o + written + ex] = sum;
                }
                written += hsum;
            }
            __syncthreads();
            for (uint32_t s = tid; s < k; s += BT) lpos[s] += ltake[s];
            __syncthreads();
        }
        if (tid == 0) {
            if (cnt) cnt[i] = (uint32_t)written;
            if (col_off) {
                col_off[c] = o;
                col_len[c] = (uint32_t)written;
            }
        }
        __syncthreads();
    }
}

// load-balanced copy of merged columns into a compact CSR
__global__ __launch_bounds__(BT) void k_compact(const uint64_t* __restrict__ src_off,
                                                const uint64_t* __restrict__ dst_off, uint64_t n, uint64_t total,
                                                const uint32_t* __restrict__ srow, const uint64_t* __restrict__ sval,
                                                uint32_t* __restrict__ drow, uint64_t* __restrict__ dval) {
    uint64_t e = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (e >= total) return;
    // column of output entry e: the last i with dst_off[i] <= e
    uint64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint64_t mid = (lo + hi) >> 1;
        if (dst_off[mid] <= e) lo = mid;
        else hi = mid;
    }
    uint64_t src = src_off[lo] + (e - dst_off[lo]);
    drow[e] = srow[src];
    dval[e] = sval[src];
}

// in-degree of every junction in the minor; junctions without predecessors
// form the first ready frontier
__global__ __launch_bounds__(BT) void k_ready_init(const uint64_t* __restrict__ prp, uint64_t J,
                                                   uint32_t* __restrict__ indeg, uint32_t* __restrict__ ready,
                                                   unsigned long long* __restrict__ nready) {
    __shared__ unsigned long long sc[BT / WAVE + 1];
    __shared__ unsigned long long base;
    uint64_t j = (uint64_t)blockIdx.x * BT + threadIdx.x;
    unsigned long long is0 = 0;
    if (j < J) {
        uint32_t d = (uint32_t)(prp[j + 1] - prp[j]);
        indeg[j] = d;
        is0 = d == 0;
    }
    unsigned long long tot;
    unsigned long long ex = block_excl_scan<unsigned long long, BT>(is0, sc, tot);
    if (threadIdx.x == 0) base = tot ? atomicAdd(nready, tot) : 0;
    __syncthreads();
    if (is0) ready[base + ex] = (uint32_t)j;
}

// after the columns of `ready` are complete: release their successors (a
// junction is an edge paired with a quad, so it has at most three minor
// successors)
__global__ __launch_bounds__(BT) void k_release(const uint32_t* __restrict__ ready, uint64_t n,
                                                const uint64_t* __restrict__ brp, const uint32_t* __restrict__ bcol,
                                                uint32_t* __restrict__ indeg, uint32_t* __restrict__ next,
                                                unsigned long long* __restrict__ nnext, int* __restrict__ err) {
    __shared__ unsigned long long sc[BT / WAVE + 1];
    __shared__ unsigned long long base;
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    uint32_t out[3];
    unsigned long long m = 0;
    if (i < n) {
        uint32_t j = ready[i];
        uint64_t b = brp[j], e = brp[j + 1];
        if (e - b > 3) {
            atomicOr(err, 64);
            e = b + 3;
        }
        for (uint64_t q = b; q < e; q++) {
            uint32_t s = bcol[q];
            if (atomicSub(&indeg[s], 1u) == 1u) out[m++] = s;
        }
    }
    unsigned long long tot;
    unsigned long long ex = block_excl_scan<unsigned long long, BT>(m, sc, tot);
    if (threadIdx.x == 0) base = tot ? atomicAdd(nnext, tot) : 0;
    __syncthreads();
    for (unsigned long long t = 0; t < m; t++) next[base + ex + t] = out[t];
}

MergeArgs to_args(const MergeLaunch& m) {
    MergeArgs a;
    a.cols = m.cols;
    a.n = m.n;
    a.brp = m.brp;
    a.bcol = m.bcol;
    a.bval = m.bval;
    a.prp = m.prp;
    a.pcol = m.pcol;
    a.pval = m.pval;
    a.aoff = m.aoff;
    a.alen = m.alen;
    a.arow = m.arow;
    a.aval = m.aval;
    a.light_ub = m.light_ub;
    a.chunk = m.chunk < 1 ? 1u : (m.chunk > (uint32_t)CAP ? (uint32_t)CAP : m.chunk);
    return a;
}

constexpr unsigned BLOCK_GRID = 2048;

}  // namespace

hipError_t launch_merge_classify(const MergeLaunch& m, uint64_t* ub, uint8_t* heavy_flag, uint32_t* heavy,
                                 unsigned long long* nheavy, int* err, uint64_t* col_off, uint32_t* col_len,
                                 hipStream_t s) {
    if (m.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify, dim3(grid_blocks(m.n, BT)), dim3(BT), 0, s, to_args(m), ub, heavy_flag, heavy,
                       nheavy, err, col_off, col_len);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeLaunch& m, const uint8_t* heavy_flag, const uint32_t* heavy,
                        const unsigned long long* nheavy, const uint64_t* off, uint64_t out_base, uint32_t* orow,
                        uint64_t* oval, uint32_t* cnt, uint64_t* col_off, uint32_t* col_len, hipStream_t s) {
    if (m.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_thread, dim3(grid_blocks(m.n, BT)), dim3(BT), 0, s, to_args(m), heavy_flag, off,
                       out_base, orow, oval, cnt, col_off, col_len);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_block, dim3(BLOCK_GRID), dim3(BT), 0, s, to_args(m), heavy, nheavy, off, out_base, orow,
                       oval, cnt, col_off, col_len);
    return hipGetLastError();
}

hipError_t launch_compact(const uint64_t* src_off, const uint64_t* dst_off, uint64_t n, uint64_t total,
                          const uint32_t* srow, const uint64_t* sval, uint32_t* drow, uint64_t* dval, hipStream_t s) {
    if (total == 0 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(grid_blocks(total, BT)), dim3(BT), 0, s, src_off, dst_off, n, total, srow, sval,
                       drow, dval);
    return hipGetLastError();
}

hipError_t launch_ready_init(const uint64_t* prp, uint64_t J, uint32_t* indeg, uint32_t* ready,
                             unsigned long long* nready, hipStream_t s) {
    if (J == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ready_init, dim3(grid_blocks(J, BT)), dim3(BT), 0, s, prp, J, indeg, ready, nready);
    return hipGetLastError();
}

hipError_t launch_release(const uint32_t* ready, uint64_t n, const uint64_t* brp, const uint32_t* bcol,
                          uint32_t* indeg, uint32_t* next, unsigned long long* nnext, int* err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_release, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, ready, n, brp, bcol, indeg, next, nnext,
                       err);
    return hipGetLastError();
}

}  // namespace msc

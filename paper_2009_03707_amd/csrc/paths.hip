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
// Columns with few, short inputs are merged by one thread in registers.
// Columns with at most 32 input lists are merged by one wave: the lists'
// next segments are staged in LDS (a chunk), every entry's place in the
// merged chunk is its index in its own list plus, for every other list, the
// number of entries below it there (ties ordered by list), found by binary
// search in LDS; runs of equal rows are then summed and written.  The chunk
// boundary is a row threshold t taken as the smallest of the lists' rows at
// depth chunk/k, so at most `chunk` entries are at or below t, at least one
// list advances, and entries with equal rows never straddle two chunks.
// Columns with more lists go to a workgroup that picks the threshold by a
// binary search on the row value and sorts the chunk in LDS (bitonic).
// Every path is exact for any column length.
//
// Each column is written at an offset that reserves its input count (an
// upper bound of its length), which avoids a separate counting pass; the A*
// storage may therefore hold small gaps between columns.
#include "paths.h"

namespace msc {
namespace {

constexpr int BT = 256;
constexpr int LIGHT_K = 8;         // thread path: at most this many input lists
constexpr int WAVE_K = 32;         // wave path: at most this many input lists
constexpr int MAX_K = 256;         // block path: at most this many input lists
constexpr int CAP = 4096;          // block path: entries per LDS chunk
constexpr int WCAP = 512;          // wave path: entries per LDS chunk
constexpr int WPB = BT / WAVE;     // waves per workgroup
constexpr uint32_t NOROW = 0xFFFFFFFFu;

struct MergeArgs {
    const uint32_t* cols;  // output column ids (null: col0 .. col0 + n - 1)
    uint32_t col0;
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

__device__ __forceinline__ uint32_t col_of(const MergeArgs& a, uint64_t i) {
    return a.cols ? a.cols[i] : a.col0 + (uint32_t)i;
}

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

// Upper bound (input entries) of every output column, and the queues of
// columns for the wave path (qn[0] entries in qwave) and the workgroup path
// (qn[1] entries in qblock).  flag: 0 thread, 1 wave, 3 workgroup, 2 skipped.
__global__ __launch_bounds__(BT) void k_classify(MergeArgs a, uint64_t* __restrict__ ub, uint8_t* __restrict__ flag,
                                                 uint32_t* __restrict__ qwave, uint32_t* __restrict__ qblock,
                                                 unsigned long long* __restrict__ qn, int* __restrict__ err,
                                                 uint64_t* __restrict__ col_off, uint32_t* __restrict__ col_len) {
    __shared__ unsigned long long sc[BT / WAVE + 1];
    __shared__ unsigned long long base_w, base_b;
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    unsigned long long h = 0;  // low half: wave path, high half: workgroup path
    if (i < a.n) {
        uint32_t c = col_of(a, i);
        uint32_t k = num_lists(a, c);
        uint64_t u = a.brp[c + 1] - a.brp[c];
        for (uint32_t s = 1; s < k; s++) u += a.alen[a.pcol[a.prp[c] + (s - 1)]];
        ub[i] = u;
        uint8_t f = (k <= (uint32_t)LIGHT_K && u <= (uint64_t)a.light_ub) ? 0 : (k <= (uint32_t)WAVE_K ? 1 : 3);
        if (f == 3 && k > (uint32_t)MAX_K) {
            atomicOr(err, 32);  // skipped: the caller falls back to the power iteration
            f = 2;
            ub[i] = 0;
            if (col_off) {  // an empty column keeps later reads in bounds
                col_off[c] = 0;
                col_len[c] = 0;
            }
        }
        flag[i] = f;
        h = f == 1 ? 1ull : (f == 3 ? (1ull << 32) : 0ull);
    }
    unsigned long long tot;
    unsigned long long ex = block_excl_scan<unsigned long long, BT>(h, sc, tot);
    if (threadIdx.x == 0) {
        base_w = (tot & 0xFFFFFFFFull) ? atomicAdd(&qn[0], tot & 0xFFFFFFFFull) : 0;
        base_b = (tot >> 32) ? atomicAdd(&qn[1], tot >> 32) : 0;
    }
    __syncthreads();
    if (h == 1) qwave[base_w + (ex & 0xFFFFFFFFull)] = (uint32_t)i;
    if (h >> 32) qblock[base_b + (ex >> 32)] = (uint32_t)i;
}

// Thread-per-column merge (few, short inputs), written at out_base + off[i].
__global__ __launch_bounds__(BT) void k_merge_thread(MergeArgs a, const uint8_t* __restrict__ flag,
                                                     const uint64_t* __restrict__ off, uint64_t out_base,
                                                     uint32_t* __restrict__ orow, uint64_t* __restrict__ oval,
                                                     uint32_t* __restrict__ cnt, uint64_t* __restrict__ col_off,
                                                     uint32_t* __restrict__ col_len) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= a.n || flag[i]) return;
    uint32_t c = col_of(a, i);
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

// number of entries of a sorted list with row < t
__device__ __forceinline__ uint32_t count_lt(const uint32_t* row, uint32_t len, uint32_t t) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (row[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) {
        uint32_t y = __shfl_xor(x, d, WAVE);
        x = y < x ? y : x;
    }
    return x;
}

// Orders the LDS accesses of one wave (the waves of a workgroup run
// independently here, so there is no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-per-column chunked merge by rank (see the file comment).  Lane s < k
// owns input list s.
__global__ __launch_bounds__(BT) void k_merge_wave(MergeArgs a, const uint32_t* __restrict__ queue,
                                                   const unsigned long long* __restrict__ qn,
                                                   const uint64_t* __restrict__ off, uint64_t out_base,
                                                   uint32_t* __restrict__ orow, uint64_t* __restrict__ oval,
                                                   uint32_t* __restrict__ cnt, uint64_t* __restrict__ col_off,
                                                   uint32_t* __restrict__ col_len) {
    __shared__ uint32_t s_in[WPB][WCAP];       // staged rows, list segments back to back
    __shared__ uint32_t s_key[WPB][WCAP];      // merged rows
    __shared__ uint64_t s_val[WPB][WCAP];      // merged scaled counts
    __shared__ uint32_t s_seg[WPB][WAVE_K + 1];
    __shared__ uint32_t s_pos[WPB][WAVE_K];
    __shared__ const uint64_t* s_vp[WPB][WAVE_K];
    __shared__ uint64_t s_mul[WPB][WAVE_K];
    const int lane = lane_id();
    const int w = (int)threadIdx.x / WAVE;
    uint32_t* in = s_in[w];
    uint32_t* key = s_key[w];
    uint64_t* val = s_val[w];
    uint32_t* seg = s_seg[w];
    const uint64_t nq = qn[0];
    const uint64_t stride = (uint64_t)gridDim.x * WPB;
    for (uint64_t h = (uint64_t)blockIdx.x * WPB + w; h < nq; h += stride) {
        const uint32_t i = queue[h];
        const uint32_t c = col_of(a, i);
        const uint32_t k = num_lists(a, c);
        const uint32_t* lr = nullptr;
        uint32_t len = 0, pos = 0;
        if ((uint32_t)lane < k) {
            ListRef L = list_of(a, c, (uint32_t)lane);
            lr = L.row;
            len = (uint32_t)L.len;
            s_vp[w][lane] = L.val;
            s_mul[w][lane] = L.mul;
        }
        uint32_t chunk = a.chunk < (uint32_t)WCAP ? a.chunk : (uint32_t)WCAP;
        if (chunk < k) chunk = k;  // rows are unique per list, so every list can give one
        const uint32_t q = chunk / k;
        const uint64_t o = out_base + off[i];
        uint64_t written = 0;
        for (;;) {
            const uint32_t rem = len - pos;
            if (wave_sum_u64(rem) == 0) break;
            uint32_t take = rem;
            if (wave_sum_u64(rem) > chunk) {
                // the smallest row at depth q over the lists longer than q
                const uint32_t t = wave_min_u32(rem > q ? lr[pos + q - 1] : NOROW);
                take = rem ? count_le(lr + pos, rem, t) : 0u;
            }
            const uint32_t incl = wave_incl_scan(take);
            const uint32_t m = __shfl(incl, WAVE - 1, WAVE);
            if ((uint32_t)lane < k) {
                seg[lane] = incl - take;
                s_pos[w][lane] = pos;
            }
            if ((uint32_t)lane == k) seg[k] = m;
            for (uint32_t s = 0; s < k; s++) {
                const uint32_t* r = (const uint32_t*)(uintptr_t)__shfl((unsigned long long)(uintptr_t)lr, (int)s, WAVE);
                const uint32_t ps = __shfl(pos, (int)s, WAVE);
                const uint32_t ts = __shfl(take, (int)s, WAVE);
                const uint32_t es = __shfl(incl - take, (int)s, WAVE);
                for (uint32_t e = (uint32_t)lane; e < ts; e += WAVE) in[es + e] = r[ps + e];
            }
            wave_sync();
            for (uint32_t j = (uint32_t)lane; j < m; j += WAVE) {
                // the list of entry j: the last s with seg[s] <= j
                uint32_t lo = 0, hi = k;
                while (hi - lo > 1) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (seg[mid] <= j) lo = mid;
                    else hi = mid;
                }
                const uint32_t s = lo;
                const uint32_t x = in[j];
                const uint32_t idx = j - seg[s];
                uint32_t rank = idx;
                for (uint32_t t = 0; t < k; t++) {
                    if (t == s) continue;
                    const uint32_t b = seg[t], l = seg[t + 1] - b;
                    rank += t < s ? count_le(in + b, l, x) : count_lt(in + b, l, x);
                }
                key[rank] = x;
                val[rank] = sat_mul(s_vp[w][s][s_pos[w][s] + idx], s_mul[w][s]);
            }
            wave_sync();
            for (uint32_t b = 0; b < m; b += WAVE) {
                const uint32_t p = b + (uint32_t)lane;
                const bool head = p < m && (p == 0 || key[p] != key[p - 1]);
                const uint64_t mask = __ballot(head);
                if (head) {
                    const uint32_t x = key[p];
                    uint64_t sum = val[p];
                    for (uint32_t f = p + 1; f < m && key[f] == x; f++) sum = sat_add(sum, val[f]);
                    const uint64_t d = o + written + (uint64_t)__popcll(mask & ((1ull << lane) - 1ull));
                    orow[d] = x;
                    oval[d] = sum;
                }
                written += (uint64_t)__popcll(mask);
            }
            pos += take;
            wave_sync();  // the next chunk reuses the LDS arrays
        }
        if (lane == 0) {
            if (cnt) cnt[i] = (uint32_t)written;
            if (col_off) {
                col_off[c] = o;
                col_len[c] = (uint32_t)written;
            }
        }
    }
}

// Workgroup-per-column chunked merge (see the file comment).
__global__ __launch_bounds__(BT) void k_merge_block(MergeArgs a, const uint32_t* __restrict__ heavy,
                                                    const unsigned long long* __restrict__ qn,
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
    const uint64_t nh = qn[1];
    for (uint64_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const uint32_t i = heavy[h];
        const uint32_t c = col_of(a, i);
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

// input entries of column c: its base list plus its predecessors' columns
__device__ __forceinline__ uint64_t column_inputs(const uint64_t* __restrict__ base_rp,
                                                  const uint64_t* __restrict__ prp, const uint32_t* __restrict__ pcol,
                                                  const uint32_t* __restrict__ alen, uint32_t c) {
    uint64_t u = base_rp[c + 1] - base_rp[c];
    for (uint64_t q = prp[c]; q < prp[c + 1]; q++) u += alen[pcol[q]];
    return u;
}

// in-degree of every junction in the minor; junctions without predecessors
// form the first ready frontier (with their input counts in ub when base_rp
// is given)
__global__ __launch_bounds__(BT) void k_ready_init(const uint64_t* __restrict__ prp, uint64_t J,
                                                   uint32_t* __restrict__ indeg, uint32_t* __restrict__ ready,
                                                   unsigned long long* __restrict__ nready,
                                                   const uint64_t* __restrict__ base_rp, uint64_t* __restrict__ ub) {
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
    if (is0) {
        ready[base + ex] = (uint32_t)j;
        if (ub) ub[base + ex] = base_rp[j + 1] - base_rp[j];
    }
}

// after the columns of `ready` are complete: release their successors (a
// junction is an edge paired with a quad, so it has at most three minor
// successors); with ub_next, also the input counts of the released columns
// (every predecessor column is complete by then)
__global__ __launch_bounds__(BT) void k_release(const uint32_t* __restrict__ ready, uint64_t n,
                                                const uint64_t* __restrict__ brp, const uint32_t* __restrict__ bcol,
                                                uint32_t* __restrict__ indeg, uint32_t* __restrict__ next,
                                                unsigned long long* __restrict__ nnext, int* __restrict__ err,
                                                const uint64_t* __restrict__ base_rp, const uint64_t* __restrict__ prp,
                                                const uint32_t* __restrict__ pcol, const uint32_t* __restrict__ alen,
                                                uint64_t* __restrict__ ub_next) {
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
    for (unsigned long long t = 0; t < m; t++) {
        next[base + ex + t] = out[t];
        if (ub_next) ub_next[base + ex + t] = column_inputs(base_rp, prp, pcol, alen, out[t]);
    }
}

// ---- topological sweep without host round trips -------------------------------
// Level L's frontier is order[lv[L], lv[L + 1]); k_sweep_seal fixes
// lv[L + 1] = *tail (everything appended so far) before level L is
// released, and k_sweep_level appends the junctions whose last predecessor
// it releases at *tail.  The host enqueues levels in batches and reads the
// boundaries back once per batch; levels enqueued past the last one are
// empty and do nothing.  The release grid is fixed and strides over the
// frontier, whose size only the device knows.
constexpr unsigned SWEEP_BLOCKS = 1024;

__global__ void k_sweep_seal(uint64_t* __restrict__ lv, uint64_t L, const unsigned long long* __restrict__ tail) {
    if (threadIdx.x == 0) lv[L + 1] = *tail;
}

// A thread releases SW_R junctions per pass, each step (frontier entry,
// row offsets, successors, in-degree atomics) issued for all of them before
// any is used, so the chains of dependent loads overlap.
constexpr int SW_R = 2;

__global__ __launch_bounds__(BT) void k_sweep_level(uint32_t* __restrict__ order, const uint64_t* __restrict__ lv,
                                                    uint64_t L, const uint64_t* __restrict__ brp,
                                                    const uint32_t* __restrict__ bcol, uint32_t* __restrict__ indeg,
                                                    unsigned long long* __restrict__ tail, int* __restrict__ err) {
    __shared__ unsigned long long sc[BT / WAVE + 1];
    __shared__ unsigned long long base;
    const uint64_t b0 = lv[L], n = lv[L + 1] - b0;
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    for (uint64_t blk = (uint64_t)blockIdx.x * BT * SW_R; blk < n; blk += (uint64_t)gridDim.x * BT * SW_R) {  // uniform
        uint32_t j[SW_R];
#pragma unroll
        for (int r = 0; r < SW_R; r++) {
            const uint64_t i = blk + (uint64_t)r * BT + threadIdx.x;
            j[r] = i < n ? order[b0 + i] : NONE;
        }
        uint64_t rb[SW_R], re[SW_R];
#pragma unroll
        for (int r = 0; r < SW_R; r++) {
            rb[r] = j[r] != NONE ? brp[j[r]] : 0;
            re[r] = j[r] != NONE ? brp[j[r] + 1] : 0;
            if (re[r] - rb[r] > 3) {  // at most three successors (the other edges of its paired quad)
                atomicOr(err, 64);
                re[r] = rb[r] + 3;
            }
        }
        uint32_t t[SW_R][3];
#pragma unroll
        for (int r = 0; r < SW_R; r++)
#pragma unroll
            for (int q = 0; q < 3; q++) t[r][q] = rb[r] + q < re[r] ? bcol[rb[r] + q] : NONE;
        uint32_t fresh = 0;  // bit 3 r + q: successor q of junction r became ready
#pragma unroll
        for (int r = 0; r < SW_R; r++)
#pragma unroll
            for (int q = 0; q < 3; q++)
                if (t[r][q] != NONE && atomicSub(&indeg[t[r][q]], 1u) == 1u) fresh |= 1u << (3 * r + q);
        const unsigned long long m = (unsigned long long)__builtin_popcount(fresh);
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan<unsigned long long, BT>(m, sc, tot);
        if (threadIdx.x == 0) base = tot ? atomicAdd(tail, tot) : 0;
        __syncthreads();
        unsigned long long o = base + ex;
#pragma unroll
        for (int r = 0; r < SW_R; r++)
#pragma unroll
            for (int q = 0; q < 3; q++)
                if ((fresh >> (3 * r + q)) & 1u) order[o++] = t[r][q];
        __syncthreads();  // base is rewritten by the next pass
    }
}

// ---- topological numbering of the junctions ---------------------------------
// Junctions without predecessors (in-degree from a histogram of B's
// columns); a workgroup covers SRC_PER_BLOCK junctions and appends them with
// one atomic (appends to a single counter serialise, so they are kept few)
constexpr int SRC_ROUNDS = 8;
constexpr uint64_t SRC_PER_BLOCK = (uint64_t)BT * SRC_ROUNDS;

__global__ __launch_bounds__(BT) void k_sources(const uint32_t* __restrict__ indeg, uint64_t J,
                                                uint32_t* __restrict__ out, unsigned long long* __restrict__ n) {
    __shared__ unsigned long long sc[BT / WAVE + 1];
    __shared__ unsigned long long base;
    const int lane = lane_id();
    const uint64_t j0 = (uint64_t)blockIdx.x * SRC_PER_BLOCK + (uint64_t)(threadIdx.x / WAVE) * (WAVE * SRC_ROUNDS);
    uint64_t mask[SRC_ROUNDS];
    unsigned long long cnt = 0;
#pragma unroll
    for (int r = 0; r < SRC_ROUNDS; r++) {  // a wave covers WAVE * SRC_ROUNDS consecutive junctions
        const uint64_t j = j0 + (uint64_t)r * WAVE + lane;
        mask[r] = __ballot(j < J && indeg[j] == 0u);
        cnt += (unsigned long long)__popcll(mask[r]);
    }
    // cnt is the wave's total on every lane; let lane 0 carry it into the block scan
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<unsigned long long, BT>(lane == 0 ? cnt : 0ull, sc, tot);
    if (threadIdx.x == 0) base = tot ? atomicAdd(n, tot) : 0;
    __syncthreads();
    unsigned long long o = base + __shfl(ex, 0, WAVE);
#pragma unroll
    for (int r = 0; r < SRC_ROUNDS; r++) {
        const uint64_t j = j0 + (uint64_t)r * WAVE + lane;
        if ((mask[r] >> lane) & 1ull) out[o + (uint64_t)__popcll(mask[r] & ((1ull << lane) - 1ull))] = (uint32_t)j;
        o += (unsigned long long)__popcll(mask[r]);
    }
}

__global__ __launch_bounds__(BT) void k_invert(const uint32_t* __restrict__ order, uint64_t n,
                                               uint32_t* __restrict__ inv) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i < n) inv[order[i]] = (uint32_t)i;
}

__global__ __launch_bounds__(BT) void k_relabel(uint32_t* __restrict__ x, uint64_t n, const uint32_t* __restrict__ map) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i < n) x[i] = map[x[i]];
}

// ---- entry-parallel merges ---------------------------------------------------
// One thread per input entry of a level (the entries of all columns, column
// by column, each column's lists back to back: base list, then predecessor
// columns).  An entry's place in its merged column is its index in its own
// list plus, for every other list of the column, the number of entries
// below it there (ties ordered by list), found by binary search.  The first
// entry of a run of equal rows (the "head": no earlier list holds the row)
// also sums the run's scaled counts; a scan of the head flags then gives
// every output row its final, gap-free position.

// (the first three predecessors' ids, then their lengths, are loaded
// together; a junction has at most three)
__global__ __launch_bounds__(BT) void k_entry_ub(MergeArgs a, uint64_t* __restrict__ ub) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t c = col_of(a, i);
    const uint64_t p0 = a.prp[c], np = a.prp[c + 1] - p0;
    uint64_t u = a.brp[c + 1] - a.brp[c];
    uint32_t pc[3];
#pragma unroll
    for (int q = 0; q < 3; q++) pc[q] = (uint64_t)q < np ? a.pcol[p0 + q] : 0u;
#pragma unroll
    for (int q = 0; q < 3; q++)
        if ((uint64_t)q < np) u += a.alen[pc[q]];
    for (uint64_t q = 3; q < np; q++) u += a.alen[a.pcol[p0 + q]];
    ub[i] = u;
}

constexpr int EPT = 4;           // entries per thread of a rank block
constexpr int EPB = BT * EPT;     // entries per rank block
constexpr int CW = 256;           // columns per LDS window of a rank block
constexpr int LCAP = 512;         // list descriptors per LDS window

// bstart[b] = the column holding entry b * EPB: every non-empty column i
// claims the rank blocks whose first entry lies in [off[i], off[i + 1]).
__global__ __launch_bounds__(BT) void k_block_start(const uint64_t* __restrict__ off, uint64_t n,
                                                    uint32_t* __restrict__ bstart) {
    const uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    const uint64_t lo = off[i], hi = off[i + 1];
    for (uint64_t b = (lo + EPB - 1) / EPB; b * EPB < hi; b++) bstart[b] = (uint32_t)i;
}

// One rank block handles EPB consecutive input entries (the level's inputs
// are column by column, each column's lists back to back).  Their columns
// form a contiguous run; its offsets and list descriptors are staged in LDS
// once per block.  Phase 1 maps every entry to (column, list, index) and
// stages its row in LDS; phase 2 ranks it: for every other list of the
// column, the count of rows below it there -- searched in LDS when that
// list lies inside the block's entry range, else in global memory.  Every
// entry writes its own scaled count at its merged position, the head of a
// run of equal rows (no earlier list holds the row) also its row; the head
// scan sums each run.  Entries of columns beyond the staged window read
// their metadata from global memory (same result), their column from
// colof (every entry's column, for levels of short columns, where many
// entries lie beyond the window) or else by binary search in off.
//
// Each step issues all of a thread's independent loads before it uses any: the
// window's offsets and column ids, then every column's list pointers, then
// its first predecessors' ids and multiplicities, then their A* offsets and
// lengths (a junction has at most three predecessors; more are read one by
// one), and in phase 1 the rows and counts of all EPT entries together.
// off: exclusive scan of ub (n + 1 entries, off[n] = T).
static_assert(CW == BT, "one window column per thread");
constexpr int RP = 3;  // predecessors whose descriptors are loaded together

__global__ __launch_bounds__(BT) void k_entry_rank(MergeArgs a, const uint64_t* __restrict__ off, uint64_t T,
                                                   const uint32_t* __restrict__ bstart,
                                                   const uint32_t* __restrict__ colof, uint32_t* __restrict__ hrow,
                                                   uint64_t* __restrict__ hval, uint8_t* __restrict__ head) {
    __shared__ uint64_t s_off[CW + 1];
    __shared__ uint32_t s_lbase[CW + 1];
    __shared__ uint64_t s_lo[LCAP];  // list start: in the base arrays (list 0) or the A* storage
    __shared__ uint32_t s_len[LCAP];
    __shared__ uint32_t s_mul[LCAP];  // minor multiplicities (at most 4 paths leave a source)
    __shared__ uint32_t s_x[EPB];
    __shared__ uint64_t s_sc[BT / WAVE + 1];
    const uint64_t e0 = (uint64_t)blockIdx.x * EPB;
    const uint64_t e_end = e0 + EPB < T ? e0 + EPB : T;
    const uint64_t i0 = bstart[blockIdx.x];  // the column of the block's first entry
    const uint32_t wn = (uint32_t)((a.n - i0) < (uint64_t)CW ? (a.n - i0) : (uint64_t)CW);  // >= 1
    const uint32_t t = threadIdx.x;

    // window column t: its offset and id, then its list pointers.  Offsets
    // never decrease, so the columns holding entries of this block (offset
    // below e_end) are a prefix of the window.
    const uint64_t o_t = t < wn ? off[i0 + t] : 0;
    const uint32_t c = t < wn ? col_of(a, i0 + t) : 0u;
    if (t < wn) s_off[t] = o_t;
    if (t == 0) s_off[wn] = off[i0 + wn];
    const bool used = t < wn && o_t < e_end;
    uint64_t pr0 = 0, pr1 = 0, b0 = 0, b1 = 0;
    if (used) {
        pr0 = a.prp[c];
        pr1 = a.prp[c + 1];
        b0 = a.brp[c];
        b1 = a.brp[c + 1];
    }
    const uint64_t np = pr1 - pr0;
    uint32_t pc[RP];
    uint64_t pv[RP], ao[RP];
    uint32_t al[RP];
#pragma unroll
    for (int q = 0; q < RP; q++) {
        pc[q] = (uint64_t)q < np ? a.pcol[pr0 + q] : 0u;
        pv[q] = (uint64_t)q < np ? a.pval[pr0 + q] : 0u;
    }
#pragma unroll
    for (int q = 0; q < RP; q++) {
        ao[q] = (uint64_t)q < np ? a.aoff[pc[q]] : 0u;
        al[q] = (uint64_t)q < np ? a.alen[pc[q]] : 0u;
    }
    // list slots of the used columns (low half) and the used count (high half)
    const uint64_t k = used ? 1 + np : 0;
    uint64_t tot;
    const uint64_t lbx = block_excl_scan<uint64_t, BT>((used ? 1ull << 32 : 0ull) | k, s_sc, tot);
    const uint32_t lb = (uint32_t)lbx, nl = (uint32_t)tot, nused = (uint32_t)(tot >> 32);
    if (used) {
        s_lbase[t] = lb;
        if (lb < (uint32_t)LCAP) {
            s_lo[lb] = b0;
            s_len[lb] = (uint32_t)(b1 - b0);
            s_mul[lb] = 1;
        }
#pragma unroll
        for (int q = 0; q < RP; q++)
            if ((uint64_t)q < np && lb + 1 + q < (uint32_t)LCAP) {
                s_lo[lb + 1 + q] = ao[q];
                s_len[lb + 1 + q] = al[q];
                s_mul[lb + 1 + q] = (uint32_t)pv[q];
            }
        for (uint64_t q = RP; q < np && lb + 1 + q < (uint64_t)LCAP; q++) {
            const uint32_t p = a.pcol[pr0 + q];
            s_lo[lb + 1 + q] = a.aoff[p];
            s_len[lb + 1 + q] = a.alen[p];
            s_mul[lb + 1 + q] = (uint32_t)a.pval[pr0 + q];
        }
    }
    if (t == 0) s_lbase[nused] = nl;
    __syncthreads();

    // phase 1: map entries to (column, list, index); then load all rows and counts
    uint32_t e_col[EPT], e_list[EPT], e_loc[EPT], x[EPT];
    bool e_win[EPT];
    uint64_t e_glo[EPT], gi[EPT], own[EPT];
    uint32_t mul[EPT];
#pragma unroll
    for (int r = 0; r < EPT; r++) {
        const uint64_t e = e0 + (uint32_t)r * BT + t;
        e_win[r] = false;
        e_glo[r] = 0;
        e_col[r] = 0;
        e_list[r] = 0;
        e_loc[r] = 0;
        gi[r] = 0;
        mul[r] = 0;
        if (e >= e_end) continue;
        uint32_t lo = 0, hi = nused;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= e) lo = mid;
            else hi = mid;
        }
        if (e < s_off[nused] && s_lbase[lo + 1] <= (uint32_t)LCAP) {
            e_win[r] = true;
            e_col[r] = lo;
            const uint32_t b = s_lbase[lo];
            uint64_t local = e - s_off[lo];
            uint32_t q = 0;
            while (local >= s_len[b + q]) {
                local -= s_len[b + q];
                q++;
            }
            e_list[r] = q;
            e_loc[r] = (uint32_t)local;
            gi[r] = s_lo[b + q] + local;
            mul[r] = s_mul[b + q];
        } else {
            uint64_t glo = i0 + lo, ghi = a.n;  // last i with off[i] <= e
            if (colof) {
                glo = colof[e];
            } else {
                while (ghi - glo > 1) {
                    uint64_t mid = (glo + ghi) >> 1;
                    if (off[mid] <= e) glo = mid;
                    else ghi = mid;
                }
            }
            e_glo[r] = glo;
            const uint32_t cc = col_of(a, glo);
            uint64_t local = e - off[glo];
            uint32_t q = 0;
            ListRef L = list_of(a, cc, 0);
            while (local >= L.len) {
                local -= L.len;
                q++;
                L = list_of(a, cc, q);
            }
            e_list[r] = q;
            e_loc[r] = (uint32_t)local;
            gi[r] = (uint64_t)(L.row - (q == 0 ? a.bcol : a.arow)) + local;
            mul[r] = (uint32_t)L.mul;
        }
    }
#pragma unroll
    for (int r = 0; r < EPT; r++) {
        const bool ok = e0 + (uint32_t)r * BT + t < e_end;
        x[r] = ok ? (e_list[r] == 0 ? a.bcol : a.arow)[gi[r]] : 0u;
        own[r] = ok ? (e_list[r] == 0 ? a.bval : a.aval)[gi[r]] : 0u;
    }
#pragma unroll
    for (int r = 0; r < EPT; r++) {
        own[r] = sat_mul(own[r], mul[r]);
        if (e0 + (uint32_t)r * BT + t < e_end) s_x[(uint32_t)r * BT + t] = x[r];
    }
    __syncthreads();

    // phase 2: rank
#pragma unroll
    for (int r = 0; r < EPT; r++) {
        const uint64_t e = e0 + (uint32_t)r * BT + t;
        if (e >= e_end) continue;
        const uint32_t xs = x[r], s = e_list[r];
        uint64_t rank = e_loc[r];
        bool is_head = true;
        uint64_t start;
        if (e_win[r]) {
            const uint32_t lo = e_col[r], b = s_lbase[lo], kk = s_lbase[lo + 1] - b;
            start = s_off[lo];
            uint64_t lstart = start;  // first entry of list q
            for (uint32_t q = 0; q < kk; q++) {
                const uint32_t l = s_len[b + q];
                if (q != s) {
                    const uint32_t* rt = (lstart >= e0 && lstart + l <= e_end)
                                             ? s_x + (lstart - e0)  // list q is staged
                                             : (q == 0 ? a.bcol : a.arow) + s_lo[b + q];
                    const uint32_t lt = count_lt(rt, l, xs);
                    rank += lt;
                    if (q < s && lt < l && rt[lt] == xs) {
                        rank++;
                        is_head = false;
                    }
                }
                lstart += l;
            }
        } else {
            const uint64_t glo = e_glo[r];
            const uint32_t cc = col_of(a, glo);
            const uint32_t kk = num_lists(a, cc);
            start = off[glo];
            for (uint32_t q = 0; q < kk; q++) {
                if (q == s) continue;
                const ListRef M = list_of(a, cc, q);
                const uint32_t lt = count_lt(M.row, (uint32_t)M.len, xs);
                rank += lt;
                if (q < s && lt < M.len && M.row[lt] == xs) {
                    rank++;
                    is_head = false;
                }
            }
        }
        const uint64_t p = start + rank;
        // bit 0: run head; bit 1: the column's first position (its offset is read back per column)
        head[p] = (uint8_t)((is_head ? 1u : 0u) | (rank == 0 ? 2u : 0u));
        hval[p] = own[r];
        if (is_head) hrow[p] = xs;
    }
}


// Run heads per tile of the head flags, then (with the tile offsets
// scanned) each head's row and its run's summed count (the head's and those
// of the equal rows that follow it, saturating) written at
// base + (heads before it),
// and that prefix into hp at every column's first position (the only
// positions read back; an empty column's offset is the next column's, or
// T, whose prefix the scan writes).  A tile is 2048 positions; wave w
// of its workgroup covers positions [512 w, 512 w + 512) in 8 rounds of 64
// consecutive positions, so every access is coalesced and the prefix of a
// 0/1 flag inside a round is a popcount of the round's ballot.
constexpr int HT_R = 8;                   // rounds per wave
constexpr int HT_WAVE = HT_R * WAVE;      // positions per wave
constexpr int HT_TILE = (BT / WAVE) * HT_WAVE;

__global__ __launch_bounds__(BT) void k_head_tiles(const uint8_t* __restrict__ head, uint64_t T,
                                                   uint64_t* __restrict__ part) {
    __shared__ uint32_t wsum[BT / WAVE];
    const int lane = lane_id(), w = (int)threadIdx.x / WAVE;
    const uint64_t b0 = (uint64_t)blockIdx.x * HT_TILE + (uint64_t)w * HT_WAVE;
    uint32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < HT_R; r++) {
        const uint64_t j = b0 + (uint64_t)r * WAVE + lane;
        cnt += (uint32_t)__popcll(__ballot(j < T && (head[j] & 1u)));
    }
    if (lane == 0) wsum[w] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int q = 0; q < BT / WAVE; q++) t += wsum[q];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(BT) void k_head_emit(const uint8_t* __restrict__ head, uint64_t T,
                                                  const uint64_t* __restrict__ part,
                                                  const uint32_t* __restrict__ hrow, const uint64_t* __restrict__ hval,
                                                  uint64_t base, uint32_t* __restrict__ orow,
                                                  uint64_t* __restrict__ oval, uint64_t* __restrict__ hp) {
    __shared__ uint32_t wsum[BT / WAVE];
    const int lane = lane_id(), w = (int)threadIdx.x / WAVE;
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint64_t b0 = (uint64_t)blockIdx.x * HT_TILE + (uint64_t)w * HT_WAVE;
    uint64_t mask[HT_R], v0[HT_R];
    uint32_t hr[HT_R], hb[HT_R];
    uint32_t cnt = 0, first = 0;  // first: bit r set when position r of this lane starts a column
    // every position's flags, count and row (rows are read for non-heads
    // too, and ignored), all loads issued before any is used
#pragma unroll
    for (int r = 0; r < HT_R; r++) {
        const uint64_t j = b0 + (uint64_t)r * WAVE + lane;
        hb[r] = j < T ? head[j] : 0u;
        v0[r] = j < T ? hval[j] : 0ull;
        hr[r] = j < T ? hrow[j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < HT_R; r++) {
        const uint32_t h = hb[r];
        mask[r] = __ballot(h & 1u);
        first |= (h >> 1 & 1u) << r;
        cnt += (uint32_t)__popcll(mask[r]);
    }
    if (lane == 0) wsum[w] = cnt;
    __syncthreads();
    uint64_t ex = part[blockIdx.x];
    for (int q = 0; q < w; q++) ex += wsum[q];
#pragma unroll
    for (int r = 0; r < HT_R; r++) {
        const uint64_t j = b0 + (uint64_t)r * WAVE + lane;
        const uint64_t p = ex + (uint64_t)__popcll(mask[r] & lt);
        uint64_t vn[3];  // the next three positions' counts
#pragma unroll
        for (int q = 0; q < 3; q++) vn[q] = __shfl_down(v0[r], (unsigned)(q + 1), WAVE);
        if (j < T) {
            if ((first >> r) & 1u) hp[j] = p;  // only column starts are read back
            if ((mask[r] >> lane) & 1ull) {
                // the run: this head and the positions up to the next head (a
                // column's first position is a head, so runs stay in their
                // column), found in this wave's flags; a run reaching the end
                // of the wave's positions continues in global memory
                uint64_t m = 0;  // positions after j in the run
                bool open = true;
                const uint64_t above = lane == WAVE - 1 ? 0ull : mask[r] >> (lane + 1);
                if (above) {
                    m = (uint64_t)__builtin_ctzll(above);
                    open = false;
                } else {
                    m = (uint64_t)(WAVE - 1 - lane);
                }
#pragma unroll
                for (int rr = r + 1; rr < HT_R; rr++) {
                    if (open) {
                        if (mask[rr]) {
                            m += (uint64_t)__builtin_ctzll(mask[rr]);
                            open = false;
                        } else {
                            m += WAVE;
                        }
                    }
                }
                if (m > T - 1 - j) {
                    m = T - 1 - j;
                    open = false;
                }
                const uint64_t inr = m < (uint64_t)(WAVE - 1 - lane) ? m : (uint64_t)(WAVE - 1 - lane);
                uint64_t sum = v0[r];
#pragma unroll
                for (int q = 0; q < 3; q++)
                    if ((uint64_t)q < inr) sum = sat_add(sum, vn[q]);
                for (uint64_t q = inr < 3 ? inr : 3; q < m; q++) sum = sat_add(sum, hval[j + 1 + q]);
                for (uint64_t f = j + 1 + m; open && f < T && !(head[f] & 1u); f++) sum = sat_add(sum, hval[f]);
                orow[base + p] = hr[r];
                oval[base + p] = sum;
            }
        }
        ex += (uint64_t)__popcll(mask[r]);
    }
}

// per column: its output range; optionally a CSR row pointer (n + 1 entries)
__global__ __launch_bounds__(BT) void k_entry_cols(MergeArgs a, const uint64_t* __restrict__ off,
                                                   const uint64_t* __restrict__ hp, uint64_t base,
                                                   uint64_t* __restrict__ col_off, uint32_t* __restrict__ col_len,
                                                   uint64_t* __restrict__ rowptr) {
    const uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= a.n) return;
    const uint64_t s0 = hp[off[i]], s1 = hp[off[i + 1]];
    if (col_off) {
        const uint32_t c = col_of(a, i);
        col_off[c] = base + s0;
        col_len[c] = (uint32_t)(s1 - s0);
    }
    if (rowptr) {
        rowptr[i] = s0;
        if (i + 1 == a.n) rowptr[a.n] = s1;
    }
}

MergeArgs to_args(const MergeLaunch& m) {
    MergeArgs a;
    a.cols = m.cols;
    a.col0 = m.col0;
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

hipError_t launch_merge_classify(const MergeLaunch& m, uint64_t* ub, uint8_t* flag, uint32_t* qwave, uint32_t* qblock,
                                 unsigned long long* qn, int* err, uint64_t* col_off, uint32_t* col_len,
                                 hipStream_t s) {
    if (m.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify, dim3(grid_blocks(m.n, BT)), dim3(BT), 0, s, to_args(m), ub, flag, qwave, qblock,
                       qn, err, col_off, col_len);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeLaunch& m, const uint8_t* flag, const uint32_t* qwave, const uint32_t* qblock,
                        const unsigned long long* qn, const uint64_t* off, uint64_t out_base, uint32_t* orow,
                        uint64_t* oval, uint32_t* cnt, uint64_t* col_off, uint32_t* col_len, hipStream_t s) {
    if (m.n == 0) return hipSuccess;
    const MergeArgs a = to_args(m);
    hipLaunchKernelGGL(k_merge_thread, dim3(grid_blocks(m.n, BT)), dim3(BT), 0, s, a, flag, off, out_base, orow, oval,
                       cnt, col_off, col_len);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t wb = (m.n + WPB - 1) / WPB;
    const unsigned wave_blocks = (unsigned)(wb < m.wave_blocks ? wb : m.wave_blocks);
    hipLaunchKernelGGL(k_merge_wave, dim3(wave_blocks ? wave_blocks : 1u), dim3(BT), 0, s, a, qwave, qn, off, out_base,
                       orow, oval, cnt, col_off, col_len);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_block, dim3(BLOCK_GRID), dim3(BT), 0, s, a, qblock, qn, off, out_base, orow, oval, cnt,
                       col_off, col_len);
    return hipGetLastError();
}

hipError_t launch_entry_ub(const MergeLaunch& m, uint64_t* ub, hipStream_t s) {
    if (m.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_entry_ub, dim3(grid_blocks(m.n, BT)), dim3(BT), 0, s, to_args(m), ub);
    return hipGetLastError();
}

size_t rank_blocks(uint64_t T) { return (T + EPB - 1) / EPB; }

hipError_t launch_entry_rank(const MergeLaunch& m, const uint64_t* off, uint64_t T, uint32_t* bstart,
                             const uint32_t* colof, uint32_t* hrow, uint64_t* hval, uint8_t* head, hipStream_t s) {
    if (T == 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_start, dim3(grid_blocks(m.n, BT)), dim3(BT), 0, s, off, m.n, bstart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_entry_rank, dim3(grid_blocks(T, EPB)), dim3(BT), 0, s, to_args(m), off, T,
                       (const uint32_t*)bstart, colof, hrow, hval, head);
    return hipGetLastError();
}

hipError_t launch_sources(const uint32_t* indeg, uint64_t J, uint32_t* out, unsigned long long* n, hipStream_t s) {
    if (J == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sources, dim3((unsigned)((J + SRC_PER_BLOCK - 1) / SRC_PER_BLOCK)), dim3(BT), 0, s, indeg, J,
                       out, n);
    return hipGetLastError();
}

hipError_t launch_invert(const uint32_t* order, uint64_t n, uint32_t* inv, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_invert, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, order, n, inv);
    return hipGetLastError();
}

hipError_t launch_relabel(uint32_t* x, uint64_t n, const uint32_t* map, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_relabel, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, x, n, map);
    return hipGetLastError();
}

size_t head_scan_tmp_elems(uint64_t T) { return (T + HT_TILE - 1) / HT_TILE + 1 + scan_tmp_elems((T + HT_TILE - 1) / HT_TILE + 1); }

hipError_t launch_head_scan_emit(const uint8_t* head, uint64_t T, const uint32_t* hrow, const uint64_t* hval,
                                 uint64_t base, uint32_t* orow, uint64_t* oval, uint64_t* hp, uint64_t* tmp,
                                 hipStream_t s) {
    if (T == 0) return hipMemsetAsync(hp, 0, sizeof(uint64_t), s);
    const uint64_t nt = (T + HT_TILE - 1) / HT_TILE;
    uint64_t* part = tmp;
    hipLaunchKernelGGL(k_head_tiles, dim3((unsigned)nt), dim3(BT), 0, s, head, T, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_excl_u64(part, part, nt, tmp + nt + 1, hp + T, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_head_emit, dim3((unsigned)nt), dim3(BT), 0, s, head, T, (const uint64_t*)part, hrow, hval,
                       base, orow, oval, hp);
    return hipGetLastError();
}

hipError_t launch_entry_cols(const MergeLaunch& m, const uint64_t* off, const uint64_t* hp, uint64_t base,
                             uint64_t* col_off, uint32_t* col_len, uint64_t* rowptr, hipStream_t s) {
    if (m.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_entry_cols, dim3(grid_blocks(m.n, BT)), dim3(BT), 0, s, to_args(m), off, hp, base, col_off,
                       col_len, rowptr);
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
                             unsigned long long* nready, const uint64_t* base_rp, uint64_t* ub, hipStream_t s) {
    if (J == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ready_init, dim3(grid_blocks(J, BT)), dim3(BT), 0, s, prp, J, indeg, ready, nready, base_rp,
                       ub);
    return hipGetLastError();
}

hipError_t launch_sweep_level(uint32_t* order, uint64_t* lv, uint64_t L, const uint64_t* brp, const uint32_t* bcol,
                              uint32_t* indeg, unsigned long long* tail, int* err, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep_seal, dim3(1), dim3(WAVE), 0, s, lv, L, (const unsigned long long*)tail);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_level, dim3(SWEEP_BLOCKS), dim3(BT), 0, s, order, (const uint64_t*)lv, L, brp, bcol,
                       indeg, tail, err);
    return hipGetLastError();
}

hipError_t launch_release(const uint32_t* ready, uint64_t n, const uint64_t* brp, const uint32_t* bcol,
                          uint32_t* indeg, uint32_t* next, unsigned long long* nnext, int* err, const uint64_t* base_rp,
                          const uint64_t* prp, const uint32_t* pcol, const uint32_t* alen, uint64_t* ub_next,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_release, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, ready, n, brp, bcol, indeg, next, nnext,
                       err, base_rp, prp, pcol, alen, ub_next);
    return hipGetLastError();
}

}  // namespace msc

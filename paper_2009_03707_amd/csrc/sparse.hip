// Sparse integer matrices for the path-counting step (Section 3.3, "Path
// counting via matrix operations"; Section 3.5, "Gradient path counting").
//
// The paper uses cuSPARSE in floating point; here every kernel is
// hand-written and the arithmetic is unsigned 64-bit saturating, which is
// exact up to 2^64-1 and independent of the order of additions.  Products
// are formed expand-sort-compress: each nonzero A(i,k) is expanded against
// row k of B, the (row, column) keys are radix-sorted (stable), and runs of
// equal keys are merged by saturating addition.
#include "prims.h"

namespace msc {
namespace {

constexpr int BT = 256;

// rows[p] = the row of entry p, or map[row] when a map is given; with val
// set, packed as (row << vb) | min(val[p], 2^vb - 1).  A workgroup takes
// BT consecutive rows and strides over all their entries together (the row
// of an entry found by binary search in the rows' offsets, staged in LDS),
// so that reads and writes are coalesced and a long row is shared by the
// whole workgroup.
__global__ __launch_bounds__(BT) void k_expand_rows(const uint64_t* __restrict__ rowptr, uint64_t nrows,
                                                    const uint32_t* __restrict__ map, const uint64_t* __restrict__ val,
                                                    int vb, uint32_t* __restrict__ rows) {
    __shared__ uint64_t s_rp[BT + 1];
    __shared__ uint32_t s_v[BT];
    const uint64_t r0 = (uint64_t)blockIdx.x * BT;
    const uint32_t nr = (uint32_t)(nrows - r0 < (uint64_t)BT ? nrows - r0 : (uint64_t)BT);
    for (uint32_t t = threadIdx.x; t <= nr; t += BT) s_rp[t] = rowptr[r0 + t];
    if (threadIdx.x < nr) s_v[threadIdx.x] = map ? map[r0 + threadIdx.x] : (uint32_t)(r0 + threadIdx.x);
    __syncthreads();
    const uint64_t p0 = s_rp[0], p1 = s_rp[nr];
    const uint64_t top = (1ull << vb) - 1ull;
    for (uint64_t p = p0 + threadIdx.x; p < p1; p += BT) {
        uint32_t lo = 0, hi = nr;  // last row j with s_rp[j] <= p
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_rp[mid] <= p) lo = mid;
            else hi = mid;
        }
        const uint32_t v = s_v[lo];
        rows[p] = val ? (v << vb) | (uint32_t)(val[p] < top ? val[p] : top) : v;
    }
}

// *out += the sum of a[0, n) (one atomic per workgroup; *out zeroed by the caller)
__global__ __launch_bounds__(BT) void k_sum_u32(const uint32_t* __restrict__ a, uint64_t n,
                                                unsigned long long* __restrict__ out) {
    __shared__ unsigned long long sc[BT / WAVE + 1];
    unsigned long long v = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * BT) v += a[i];
    unsigned long long tot;
    block_excl_scan<unsigned long long, BT>(v, sc, tot);
    if (threadIdx.x == 0 && tot) atomicAdd(out, tot);
}

// *out = max(*out, the largest of a[0, n)) (one atomic per workgroup; *out zeroed by the caller)
__global__ __launch_bounds__(BT) void k_max_u64(const uint64_t* __restrict__ a, uint64_t n,
                                                unsigned long long* __restrict__ out) {
    __shared__ unsigned long long sm[BT / WAVE];
    unsigned long long v = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * BT)
        v = a[i] > v ? a[i] : v;
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(v, d, WAVE);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) sm[threadIdx.x / WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BT / WAVE; w++) v = sm[w] > v ? sm[w] : v;
        if (v) atomicMax(out, v);
    }
}

__global__ __launch_bounds__(BT) void k_iota(uint32_t* __restrict__ a, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i < n) a[i] = (uint32_t)i;
}

__global__ __launch_bounds__(BT) void k_hist(const uint32_t* __restrict__ keys, uint64_t n, uint32_t* __restrict__ h) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i < n) atomicAdd(&h[keys[i]], 1u);
}

// rowptr[k] = first position of a key >= k in the sorted keys (n + 1
// threads; thread e fills the keys between keys[e - 1] and keys[e]).  Gaps
// longer than GAP_INLINE are queued in chunks of at most GAP_CHUNK keys,
// each filled by one wave.
constexpr uint64_t GAP_INLINE = 64;
constexpr uint64_t GAP_CHUNK = 4096;
constexpr unsigned GAP_BLOCKS = 1024;

__global__ __launch_bounds__(BT) void k_key_bounds(const uint32_t* __restrict__ keys, uint64_t n, uint64_t nkeys,
                                                   uint64_t* __restrict__ rowptr, uint64_t* __restrict__ gaps,
                                                   unsigned long long* __restrict__ ngaps) {
    uint64_t e = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (e > n) return;
    const uint64_t lo = e == 0 ? 0 : (uint64_t)keys[e - 1] + 1;
    const uint64_t hi = e == n ? nkeys : (uint64_t)keys[e];
    if (hi + 1 > lo + GAP_INLINE) {
        // hi - lo + 1 > GAP_INLINE keys: at most (hi - lo + 1) / GAP_INLINE chunks
        const uint64_t nch = (hi - lo + GAP_CHUNK) / GAP_CHUNK;
        const unsigned long long g = atomicAdd(ngaps, (unsigned long long)nch);
        for (uint64_t c = 0; c < nch; c++) {
            const uint64_t a = lo + c * GAP_CHUNK;
            gaps[3 * (g + c)] = a;
            gaps[3 * (g + c) + 1] = a + GAP_CHUNK - 1 < hi ? a + GAP_CHUNK - 1 : hi;
            gaps[3 * (g + c) + 2] = e;
        }
        return;
    }
    for (uint64_t k = lo; k <= hi; k++) rowptr[k] = e;
}

__global__ __launch_bounds__(BT) void k_fill_gaps(const uint64_t* __restrict__ gaps,
                                                  const unsigned long long* __restrict__ ngaps,
                                                  uint64_t* __restrict__ rowptr) {
    const uint64_t ng = *ngaps;
    const uint64_t waves = (uint64_t)gridDim.x * (BT / WAVE);
    const uint64_t gw = (uint64_t)blockIdx.x * (BT / WAVE) + threadIdx.x / WAVE;
    const uint32_t lane = threadIdx.x % WAVE;
    for (uint64_t g = gw; g < ng; g += waves) {
        const uint64_t lo = gaps[3 * g], hi = gaps[3 * g + 1], v = gaps[3 * g + 2];
        for (uint64_t k = lo + lane; k <= hi; k += WAVE) rowptr[k] = v;
    }
}

__global__ __launch_bounds__(BT) void k_gather_t(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ rows,
                                                 const uint64_t* __restrict__ val, uint32_t* __restrict__ ocol,
                                                 uint64_t* __restrict__ oval, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    uint32_t p = perm[i];
    ocol[i] = rows[p];
    oval[i] = val[p];
}

__global__ __launch_bounds__(BT) void k_make_keys(const uint32_t* __restrict__ row, const uint32_t* __restrict__ col,
                                                  uint64_t n, int cb, uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ idx) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    keys[i] = ((uint64_t)row[i] << cb) | (uint64_t)col[i];
    idx[i] = (uint32_t)i;
}

__global__ __launch_bounds__(BT) void k_heads(const uint64_t* __restrict__ keys, uint64_t n, uint32_t* __restrict__ h) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    h[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ __launch_bounds__(BT) void k_merge_runs(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ perm,
                                                   const uint64_t* __restrict__ val, uint64_t n,
                                                   const uint64_t* __restrict__ pos, int cb,
                                                   uint32_t* __restrict__ orow, uint32_t* __restrict__ ocol,
                                                   uint64_t* __restrict__ oval) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    uint64_t k = keys[i];
    if (i > 0 && keys[i - 1] == k) return;
    uint64_t s = val[perm[i]];
    for (uint64_t j = i + 1; j < n && keys[j] == k; j++) s = sat_add(s, val[perm[j]]);
    uint64_t o = pos[i];
    orow[o] = (uint32_t)(k >> cb);
    ocol[o] = (uint32_t)(k & ((1ull << cb) - 1ull));
    oval[o] = s;
}

// number of products of each nonzero X(i,k) with row k of Y
__global__ __launch_bounds__(BT) void k_esc_count(const uint32_t* __restrict__ xcol, uint64_t nx,
                                                  const uint64_t* __restrict__ yrowptr, uint32_t* __restrict__ pc) {
    uint64_t e = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (e >= nx) return;
    uint32_t k = xcol[e];
    pc[e] = (uint32_t)(yrowptr[k + 1] - yrowptr[k]);
}

__global__ __launch_bounds__(BT) void k_esc_expand(const uint32_t* __restrict__ xrow, const uint32_t* __restrict__ xcol,
                                                   const uint64_t* __restrict__ xval, uint64_t nx,
                                                   const uint64_t* __restrict__ poff,
                                                   const uint64_t* __restrict__ yrowptr,
                                                   const uint32_t* __restrict__ ycol,
                                                   const uint64_t* __restrict__ yval, uint32_t* __restrict__ prow,
                                                   uint32_t* __restrict__ pcol, uint64_t* __restrict__ pval) {
    uint64_t e = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (e >= nx) return;
    uint32_t k = xcol[e], r = xrow[e];
    uint64_t a = xval[e];
    uint64_t o = poff[e];
    for (uint64_t q = yrowptr[k]; q < yrowptr[k + 1]; q++, o++) {
        prow[o] = r;
        pcol[o] = ycol[q];
        pval[o] = sat_mul(a, yval[q]);
    }
}

__global__ __launch_bounds__(BT) void k_count_sat(const uint64_t* __restrict__ v, uint64_t n,
                                                  unsigned long long* __restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    bool s = i < n && v[i] == ~0ull;
    uint64_t b = __ballot(s);
    if (lane_id() == 0 && b) atomicAdd(out, (unsigned long long)__popcll(b));
}

}  // namespace

int bit_width(uint64_t v) {
    int b = 0;
    while (b < 64 && (v >> b) != 0) b++;
    return b < 1 ? 1 : b;
}

size_t key_bounds_tmp_elems(uint64_t n, uint64_t nkeys) { return 3 * ((nkeys + 1) / GAP_INLINE + 2) + 1; }

// tmp: key_bounds_tmp_elems(n, nkeys) uint64 (gap list and its counter)
hipError_t launch_key_bounds(const uint32_t* keys, uint64_t n, uint64_t nkeys, uint64_t* rowptr, uint64_t* tmp,
                             hipStream_t s) {
    unsigned long long* ng = (unsigned long long*)tmp;
    hipError_t e = hipMemsetAsync(ng, 0, sizeof(uint64_t), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_key_bounds, dim3(grid_blocks(n + 1, BT)), dim3(BT), 0, s, keys, n, nkeys, rowptr, tmp + 1, ng);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_gaps, dim3(GAP_BLOCKS), dim3(BT), 0, s, (const uint64_t*)(tmp + 1),
                       (const unsigned long long*)ng, rowptr);
    return hipGetLastError();
}

hipError_t launch_expand_rows(const uint64_t* rowptr, uint64_t nrows, const uint32_t* map, uint32_t* rows,
                              hipStream_t s, const uint64_t* val, int vb) {
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand_rows, dim3(grid_blocks(nrows, BT)), dim3(BT), 0, s, rowptr, nrows, map, val, vb,
                       rows);
    return hipGetLastError();
}
hipError_t launch_sum_u32(const uint32_t* a, uint64_t n, uint64_t* out, hipStream_t s) {
    hipError_t e = hipMemsetAsync(out, 0, sizeof(uint64_t), s);
    if (e != hipSuccess || n == 0) return e;
    const unsigned nb = grid_blocks(n, BT) < 2048u ? grid_blocks(n, BT) : 2048u;
    hipLaunchKernelGGL(k_sum_u32, dim3(nb), dim3(BT), 0, s, a, n, (unsigned long long*)out);
    return hipGetLastError();
}
hipError_t launch_max_u64(const uint64_t* a, uint64_t n, uint64_t* out, hipStream_t s) {
    hipError_t e = hipMemsetAsync(out, 0, sizeof(uint64_t), s);
    if (e != hipSuccess || n == 0) return e;
    const unsigned nb = grid_blocks(n, BT) < 2048u ? grid_blocks(n, BT) : 2048u;
    hipLaunchKernelGGL(k_max_u64, dim3(nb), dim3(BT), 0, s, a, n, (unsigned long long*)out);
    return hipGetLastError();
}
hipError_t launch_iota(uint32_t* a, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, a, n);
    return hipGetLastError();
}
hipError_t launch_hist(const uint32_t* keys, uint64_t n, uint32_t* h, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, keys, n, h);
    return hipGetLastError();
}
hipError_t launch_gather_t(const uint32_t* perm, const uint32_t* rows, const uint64_t* val, uint32_t* ocol,
                           uint64_t* oval, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_t, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, perm, rows, val, ocol, oval, n);
    return hipGetLastError();
}
hipError_t launch_make_keys(const uint32_t* row, const uint32_t* col, uint64_t n, int cb, uint64_t* keys,
                            uint32_t* idx, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_keys, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, row, col, n, cb, keys, idx);
    return hipGetLastError();
}
hipError_t launch_heads(const uint64_t* keys, uint64_t n, uint32_t* h, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_heads, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, keys, n, h);
    return hipGetLastError();
}
hipError_t launch_merge_runs(const uint64_t* keys, const uint32_t* perm, const uint64_t* val, uint64_t n,
                             const uint64_t* pos, int cb, uint32_t* orow, uint32_t* ocol, uint64_t* oval,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_runs, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, keys, perm, val, n, pos, cb, orow, ocol,
                       oval);
    return hipGetLastError();
}
hipError_t launch_esc_count(const uint32_t* xcol, uint64_t nx, const uint64_t* yrowptr, uint32_t* pc, hipStream_t s) {
    if (nx == 0) return hipSuccess;
    hipLaunchKernelGGL(k_esc_count, dim3(grid_blocks(nx, BT)), dim3(BT), 0, s, xcol, nx, yrowptr, pc);
    return hipGetLastError();
}
hipError_t launch_esc_expand(const uint32_t* xrow, const uint32_t* xcol, const uint64_t* xval, uint64_t nx,
                             const uint64_t* poff, const uint64_t* yrowptr, const uint32_t* ycol, const uint64_t* yval,
                             uint32_t* prow, uint32_t* pcol, uint64_t* pval, hipStream_t s) {
    if (nx == 0) return hipSuccess;
    hipLaunchKernelGGL(k_esc_expand, dim3(grid_blocks(nx, BT)), dim3(BT), 0, s, xrow, xcol, xval, nx, poff, yrowptr,
                       ycol, yval, prow, pcol, pval);
    return hipGetLastError();
}
hipError_t launch_count_sat(const uint64_t* v, uint64_t n, unsigned long long* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_sat, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, v, n, out);
    return hipGetLastError();
}

}  // namespace msc

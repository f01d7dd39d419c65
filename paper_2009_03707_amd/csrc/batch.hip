// Splitting the results of a batched run into per-field results.
//
// A batch is computed as one complex over the concatenation of its fields
// (global vertex and cell ids, global ranks).  Because cells of different
// fields are never adjacent, every arc matrix is block diagonal and the
// critical list holds each field's cells of each index as one contiguous
// range.  These kernels copy each field's part out with local ids and
// ranks, so that a field's result is byte-identical to a run on that field
// alone.
#include "prims.h"

namespace msc {
namespace {

constexpr int BT = 256;

__device__ __forceinline__ uint32_t last_le(const uint64_t* off, uint32_t n, uint64_t x) {
    uint32_t lo = 0, hi = n;  // last i in [0, n) with off[i] <= x
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Critical cells per (field, index), one thread per pair.  The global list
// is sorted by (index, id) and each field owns the contiguous id range
// [8 * base(f), 8 * base(f + 1)), so the count is the distance between two
// lower bounds inside the index segment (no atomics).
__device__ __forceinline__ uint64_t lower_bound_id(const uint32_t* __restrict__ id, uint64_t lo, uint64_t hi,
                                                   uint64_t x) {
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if ((uint64_t)id[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(BT) void k_crit_field_counts(const uint32_t* __restrict__ id, Geo geo, uint64_t s0,
                                                          uint64_t s1, uint64_t s2, uint64_t s3, uint64_t s4,
                                                          unsigned long long* __restrict__ cnt) {
    uint64_t t = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (t >= 4ull * geo.nf) return;
    const uint32_t f = (uint32_t)(t >> 2), k = (uint32_t)(t & 3u);
    const uint64_t seg[5] = {s0, s1, s2, s3, s4};
    const uint64_t lo = 8ull * geo.base(f);
    const uint64_t hi = f + 1 < geo.nf ? 8ull * geo.base(f + 1) : 8ull * geo.nv;
    cnt[t] = lower_bound_id(id, seg[k], seg[k + 1], hi) - lower_bound_id(id, seg[k], seg[k + 1], lo);
}

// Entry i of the global list (index segment k starting at seg[k]) goes to
// its field's list: dst = field_start[f] + within-field index offset +
// position among the field's cells of index k.
// fk_before[4*f + k]: cells of index k in fields before f;
// fk_start[4*f + k]: first position of (f, k) in the per-field output.
__global__ __launch_bounds__(BT) void k_crit_split(const uint32_t* __restrict__ id, const uint8_t* __restrict__ index,
                                                   const float* __restrict__ value, const uint32_t* __restrict__ vmax,
                                                   uint64_t n, Geo geo, const uint64_t* __restrict__ seg,
                                                   const uint64_t* __restrict__ fk_before,
                                                   const uint64_t* __restrict__ fk_start, uint32_t* __restrict__ o_id,
                                                   uint8_t* __restrict__ o_index, float* __restrict__ o_value,
                                                   uint32_t* __restrict__ o_vmax) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    uint32_t c = id[i];
    uint32_t k = index[i];
    uint32_t f = geo.field_of(c >> 3);
    uint64_t pos = fk_start[4 * f + k] + (i - seg[k] - fk_before[4 * f + k]);
    uint32_t base = geo.base(f);
    o_id[pos] = c - 8u * base;
    o_index[pos] = (uint8_t)k;
    o_value[pos] = value[i];
    o_vmax[pos] = vmax[i] - base;
}

// Block-diagonal CSR -> per-field CSRs.  Field f owns global rows
// [roff[f], roff[f+1]) and columns [coff[f], coff[f+1]).  Output: rowptr of
// field f at orp + roff[f] + f (nrows_f + 1 entries, starting at 0); entries
// stay at their global positions with columns made local.
__global__ __launch_bounds__(BT) void k_csr_split_rows(const uint64_t* __restrict__ rowptr, uint64_t nrows,
                                                       const uint64_t* __restrict__ roff, uint32_t nf,
                                                       uint64_t* __restrict__ orp) {
    uint64_t r = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (r > nrows + nf - 1) return;
    // output slot r belongs to field f with roff[f] + f <= r <= roff[f+1] + f
    uint32_t lo = 0, hi = nf;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (roff[mid] + mid <= r) lo = mid;
        else hi = mid;
    }
    uint32_t f = lo;
    uint64_t local = r - (roff[f] + f);
    uint64_t g0 = roff[f];
    orp[r] = rowptr[g0 + local] - rowptr[g0];
}

__global__ __launch_bounds__(BT) void k_csr_split_cols(const uint32_t* __restrict__ col, uint64_t nnz,
                                                       const uint64_t* __restrict__ eoff,
                                                       const uint64_t* __restrict__ coff, uint32_t nf,
                                                       uint32_t* __restrict__ ocol) {
    uint64_t e = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (e >= nnz) return;
    uint32_t f = last_le(eoff, nf, e);
    // skip fields without entries: the last field whose range starts at or before e
    ocol[e] = col[e] - (uint32_t)coff[f];
}

// entries equal to 2^64-1 per field (entries of field f: [eoff[f], eoff[f+1]))
__global__ __launch_bounds__(BT) void k_sat_per_field(const uint64_t* __restrict__ val, uint64_t nnz,
                                                      const uint64_t* __restrict__ eoff, uint32_t nf,
                                                      unsigned long long* __restrict__ out) {
    uint64_t e = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (e >= nnz || val[e] != ~0ull) return;
    atomicAdd(&out[last_le(eoff, nf, e)], 1ull);
}

__global__ void k_gather_u64(const uint64_t* __restrict__ src, const uint64_t* __restrict__ idx, uint64_t n,
                             uint64_t* __restrict__ dst) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

}  // namespace

hipError_t launch_gather_u64(const uint64_t* src, const uint64_t* idx, uint64_t n, uint64_t* dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_u64, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, src, idx, n, dst);
    return hipGetLastError();
}

hipError_t launch_crit_field_counts(const uint32_t* id, const int64_t count[4], const Geo& geo, unsigned long long* cnt,
                                    hipStream_t s) {
    uint64_t seg[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < 4; k++) seg[k + 1] = seg[k] + (uint64_t)count[k];
    hipLaunchKernelGGL(k_crit_field_counts, dim3(grid_blocks(4ull * geo.nf, BT)), dim3(BT), 0, s, id, geo, seg[0],
                       seg[1], seg[2], seg[3], seg[4], cnt);
    return hipGetLastError();
}

hipError_t launch_crit_split(const uint32_t* id, const uint8_t* index, const float* value, const uint32_t* vmax,
                             uint64_t n, const Geo& geo, const uint64_t* seg, const uint64_t* fk_before,
                             const uint64_t* fk_start, uint32_t* o_id, uint8_t* o_index, float* o_value,
                             uint32_t* o_vmax, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_crit_split, dim3(grid_blocks(n, BT)), dim3(BT), 0, s, id, index, value, vmax, n, geo, seg,
                       fk_before, fk_start, o_id, o_index, o_value, o_vmax);
    return hipGetLastError();
}

hipError_t launch_csr_split(const uint64_t* rowptr, uint64_t nrows, const uint32_t* col, uint64_t nnz,
                            const uint64_t* roff, const uint64_t* coff, const uint64_t* eoff, uint32_t nf,
                            uint64_t* orp, uint32_t* ocol, hipStream_t s) {
    hipLaunchKernelGGL(k_csr_split_rows, dim3(grid_blocks(nrows + nf, BT)), dim3(BT), 0, s, rowptr, nrows, roff, nf,
                       orp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nnz == 0) return e;
    hipLaunchKernelGGL(k_csr_split_cols, dim3(grid_blocks(nnz, BT)), dim3(BT), 0, s, col, nnz, eoff, coff, nf, ocol);
    return hipGetLastError();
}

hipError_t launch_sat_per_field(const uint64_t* val, uint64_t nnz, const uint64_t* eoff, uint32_t nf,
                                unsigned long long* out, hipStream_t s) {
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sat_per_field, dim3(grid_blocks(nnz, BT)), dim3(BT), 0, s, val, nnz, eoff, nf, out);
    return hipGetLastError();
}

}  // namespace msc

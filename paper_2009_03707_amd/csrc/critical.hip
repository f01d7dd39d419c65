// Critical-cell extraction and compaction (Section 3.5, "Gradient pairs and
// critical points": mark unpaired cells, per-block counts, prefix sum over
// the blocks, stream compaction into the critical-point list).
//
// Canonical order is (index, cell id), and cell ids are word-major
// (8 * vertex + nibble), so the compaction walks the gradient words in memory
// order.  Pass 1 counts the critical cells of each index per workgroup tile;
// a device scan turns the counts into offsets; pass 2 re-reads the tile and
// scatters each critical cell to its index segment in order (stable: the
// workgroup-local ranks come from an exclusive scan, never from atomics).
#include "prims.h"

namespace msc {
namespace {

constexpr int CT = 256;          // threads
constexpr int CWPT = 8;          // words per thread (contiguous)
constexpr int CTILE = CT * CWPT; // words per tile

// Per-index counts of the critical nibbles of one word, packed in four
// 16-bit lanes (index = number of set bits of the nibble position).
__device__ __forceinline__ uint64_t crit_counts(uint32_t w) {
    uint32_t isc = (w >> 3) & 0x11111111u;  // bit 4k set <=> nibble k >= 8
    uint64_t c0 = isc & 1u;
    uint64_t c1 = (uint64_t)__builtin_popcount(isc & 0x00010110u);
    uint64_t c2 = (uint64_t)__builtin_popcount(isc & 0x01101000u);
    uint64_t c3 = (isc >> 28) & 1u;
    return c0 | (c1 << 16) | (c2 << 32) | (c3 << 48);
}

// One wave per tile: each lane reads 32 words as eight 16-byte loads that
// are contiguous across the wave (all issued before any is used), and the
// wave sums the packed counts; no LDS, no barrier.
constexpr int CWAVES = CT / WAVE;  // tiles per workgroup

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

template <bool VEC>
__global__ __launch_bounds__(CT) void crit_count(const uint32_t* __restrict__ grad, uint64_t nv, uint64_t nb,
                                                 uint64_t* __restrict__ blk) {
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    const uint64_t tile = (uint64_t)blockIdx.x * CWAVES + (threadIdx.x / WAVE);
    if (tile >= nb) return;
    const uint64_t base = tile * CTILE;
    uint64_t s = 0;
    if (VEC && base + CTILE <= nv) {
        const uint4* p = reinterpret_cast<const uint4*>(grad + base);
        uint4 q[CTILE / (4 * WAVE)];
#pragma unroll
        for (int i = 0; i < CTILE / (4 * WAVE); i++) q[i] = p[i * WAVE + lane];
#pragma unroll
        for (int i = 0; i < CTILE / (4 * WAVE); i++)
            s += crit_counts(q[i].x) + crit_counts(q[i].y) + crit_counts(q[i].z) + crit_counts(q[i].w);
    } else {
        for (uint32_t j = lane; j < (uint32_t)CTILE; j += WAVE)
            if (base + j < nv) s += crit_counts(grad[base + j]);
    }
    s = wave_sum_u64(s);
    if (lane == 0)  // four per-index arrays laid out [index][tile]
        for (int k = 0; k < 4; k++) blk[(uint64_t)k * nb + tile] = (s >> (16 * k)) & 0xFFFFu;
}

// after the scan of the [index][block] counts: segment starts and totals
__global__ void crit_totals(const uint64_t* __restrict__ excl, uint64_t nb, const uint64_t* __restrict__ blk,
                            uint64_t* __restrict__ out /* [0..3] count, [4..7] segment start */) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t start = 0;
    for (int k = 0; k < 4; k++) {
        // exclusive offsets are global over the concatenated [index][block]
        // array; the count of index k is the difference of consecutive segment starts
        uint64_t seg_begin = excl[(uint64_t)k * nb];
        uint64_t seg_end = (k < 3) ? excl[(uint64_t)(k + 1) * nb] : excl[4 * nb - 1] + blk[4 * nb - 1];
        out[k] = seg_end - seg_begin;
        out[4 + k] = start;
        start += out[k];
    }
}

// Pass 2.  The records of a tile are first placed in LDS in (index, id)
// order -- cell id and highest vertex only -- and then written out as four
// contiguous runs (one per index segment), each thread fetching the field
// values of its records with independent loads; fetching them while the
// cells are found would serialise one gather after another in each thread.
// A tile with more than CCAP critical cells writes its records directly.
constexpr uint32_t CCAP = 2048;

__global__ __launch_bounds__(CT) void crit_scatter(const float* __restrict__ f0, const float* const* __restrict__ fptr,
                                                   const uint32_t* __restrict__ grad, Geo geo, uint64_t nb,
                                                   const uint64_t* __restrict__ excl,
                                                   const uint64_t* __restrict__ guard, uint64_t cap,
                                                   uint32_t* __restrict__ o_id, uint8_t* __restrict__ o_index,
                                                   float* __restrict__ o_value, uint32_t* __restrict__ o_vmax) {
    __shared__ uint64_t sc[CT / WAVE + 1];
    __shared__ uint32_t s_id[CCAP];
    __shared__ uint32_t s_vmax[CCAP];
    const uint64_t nv = geo.nv;
    const uint64_t tile = blockIdx.x;
    if (guard && guard[0] + guard[1] + guard[2] + guard[3] > cap) return;  // uniform
    uint64_t base = tile * CTILE + (uint64_t)threadIdx.x * CWPT;
    uint32_t w[CWPT];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < CWPT; i++) {
        w[i] = (base + i < nv) ? grad[base + i] : 0u;
        s += crit_counts(w[i]);
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan<uint64_t, CT>(s, sc, tot);
    if (tot == 0) return;  // uniform
    uint32_t seg[5];       // tile-local start of each index segment
    seg[0] = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) seg[k + 1] = seg[k] + (uint32_t)((tot >> (16 * k)) & 0xFFFFu);
    const uint32_t n = seg[4];
    const bool staged = n <= CCAP;  // uniform
    uint64_t pos[4];
#pragma unroll
    for (int k = 0; k < 4; k++)
        pos[k] = (staged ? (uint64_t)seg[k] : excl[(uint64_t)k * nb + tile]) + ((ex >> (16 * k)) & 0xFFFFu);
#pragma unroll
    for (int i = 0; i < CWPT; i++) {
        uint32_t word = w[i];
        if (((word >> 3) & 0x11111111u) == 0) continue;
        uint32_t v = (uint32_t)(base + i);
        uint32_t fld = geo.field_of(v);
        Grid g = geo.grid(fld);
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            uint32_t nib = nib_of(word, k);
            if (nib < NB_CRIT) continue;
            uint32_t idx = (uint32_t)__builtin_popcount(k);
            uint32_t d = nib - NB_CRIT;
            uint32_t vm = v + ((d & 1u) ? g.stride[0] : 0u) + ((d & 2u) ? g.stride[1] : 0u) +
                          ((d & 4u) ? g.stride[2] : 0u);
            uint64_t p = pos[idx]++;
            if (staged) {
                s_id[p] = 8u * v + k;
                s_vmax[p] = vm;
            } else {
                const float* f = fptr ? fptr[fld] : f0;
                o_id[p] = 8u * v + k;
                o_index[p] = (uint8_t)idx;
                o_value[p] = load_global(f, vm - geo.base(fld));
                o_vmax[p] = vm;
            }
        }
    }
    if (!staged) return;  // uniform
    uint64_t eo[4];  // global start of each index run of this tile
#pragma unroll
    for (int k = 0; k < 4; k++) eo[k] = excl[(uint64_t)k * nb + tile] - seg[k];
    __syncthreads();
    constexpr int R = 4;  // records per thread per round, their loads in flight together
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += R * CT) {
        uint32_t vm[R], fld[R];
        float val[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t i = i0 + r * CT;
            vm[r] = i < n ? s_vmax[i] : 0u;
            fld[r] = geo.field_of(vm[r]);
        }
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t i = i0 + r * CT;
            const float* f = fptr ? fptr[fld[r]] : f0;
            val[r] = i < n ? load_global(f, vm[r] - geo.base(fld[r])) : 0.f;
        }
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t i = i0 + r * CT;
            if (i >= n) continue;
            const uint32_t k = (i >= seg[1] ? 1u : 0u) + (i >= seg[2] ? 1u : 0u) + (i >= seg[3] ? 1u : 0u);
            const uint64_t gpos = eo[k] + i;
            o_id[gpos] = s_id[i];
            o_index[gpos] = (uint8_t)k;
            o_value[gpos] = val[r];
            o_vmax[gpos] = vm[r];
        }
    }
}

}  // namespace

size_t crit_tmp_elems(uint64_t nv) {
    uint64_t nb = (nv + CTILE - 1) / CTILE;
    return 2 * 4 * nb + 8 + scan_tmp_elems(4 * nb);
}

// Per-index counts and segment starts written by launch_crit_count.
const uint64_t* crit_totals_ptr(const uint64_t* tmp, uint64_t nv) {
    uint64_t nb = (nv + CTILE - 1) / CTILE;
    return tmp + 8 * nb;
}

// Pass 1 + scan.  tmp layout: [4*nb counts][4*nb exclusive offsets][8 totals][scan tmp].
// d_totals (8 uint64 inside tmp) receives per-index counts and segment starts.
hipError_t launch_crit_count(const uint32_t* grad, const Geo& g, uint64_t* tmp, uint64_t** d_totals, hipStream_t s) {
    uint64_t nb = (g.nv + CTILE - 1) / CTILE;
    uint64_t* blk = tmp;
    uint64_t* excl = tmp + 4 * nb;
    uint64_t* tot = tmp + 8 * nb;
    uint64_t* stmp = tmp + 8 * nb + 8;
    const unsigned nblk = (unsigned)((nb + CWAVES - 1) / CWAVES);
    if (((uintptr_t)grad & 15u) == 0)
        hipLaunchKernelGGL(crit_count<true>, dim3(nblk), dim3(CT), 0, s, grad, (uint64_t)g.nv, nb, blk);
    else
        hipLaunchKernelGGL(crit_count<false>, dim3(nblk), dim3(CT), 0, s, grad, (uint64_t)g.nv, nb, blk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_excl_u64(blk, excl, 4 * nb, stmp, (uint64_t*)nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(crit_totals, dim3(1), dim3(64), 0, s, (const uint64_t*)excl, nb, (const uint64_t*)blk, tot);
    *d_totals = tot;
    return hipGetLastError();
}

// Pass 2: the exclusive offsets over [index][block] are global positions in
// the (index, id)-sorted list because index segments are concatenated.
// With cap below ~0, the launch may precede the host's reading of the counts
// (into record buffers of cap entries kept from an earlier call): every
// workgroup reads the totals and writes nothing when they exceed cap.
hipError_t launch_crit_scatter(const float* f0, const float* const* fptr, const uint32_t* grad, const Geo& g,
                               const uint64_t* tmp, uint32_t* id, uint8_t* index, float* value, uint32_t* vmax,
                               hipStream_t s, uint64_t cap) {
    uint64_t nb = (g.nv + CTILE - 1) / CTILE;
    const uint64_t* excl = tmp + 4 * nb;
    const uint64_t* guard = cap == ~0ull ? nullptr : crit_totals_ptr(tmp, g.nv);
    hipLaunchKernelGGL(crit_scatter, dim3((unsigned)nb), dim3(CT), 0, s, f0, fptr, grad, g, nb, excl, guard, cap, id,
                       index, value, vmax);
    return hipGetLastError();
}

}  // namespace msc

// Wave64 / workgroup scan helpers and device-wide primitives (prefix sum,
// stable radix sort, run-length merge) used by the compaction steps.
#pragma once

#include "common.h"

namespace msc {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T t = __shfl_up(x, d, WAVE);
        if (lane >= d) x += t;
    }
    return x;
}

// Exclusive scan over a workgroup of NT threads (multiple of 64).  `scratch`
// is LDS of at least NT/64 + 1 elements.  Returns the exclusive prefix;
// `total` receives the workgroup sum.
template <typename T, int NT>
__device__ __forceinline__ T block_excl_scan(T x, T* scratch, T& total) {
    constexpr int NWAVE = NT / WAVE;
    const int lane = lane_id();
    const int w = (int)threadIdx.x / WAVE;
    T inc = wave_incl_scan(x);
    __syncthreads();
    if (lane == WAVE - 1) scratch[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < NWAVE; i++) {
            T v = scratch[i];
            scratch[i] = run;
            run += v;
        }
        scratch[NWAVE] = run;
    }
    __syncthreads();
    total = scratch[NWAVE];
    return inc - x + scratch[w];
}

// Copies n words to `dst`, memory the device can write directly (the
// context's pinned, device-mapped host scratch): small readbacks without a
// copy-engine or blit round of their own.
hipError_t launch_publish(const uint64_t* src, uint64_t n, uint64_t* dst, hipStream_t s);
// *dst = v (a kernel, so that a host value reaches the device without a
// host-to-device copy of pageable memory).
hipError_t launch_set_u64(uint64_t* dst, uint64_t v, hipStream_t s);

// Device-wide exclusive prefix sum of n uint64 values (out may equal in);
// writes the total to *d_total when non-null.  `tmp` needs
// scan_tmp_elems(n) uint64 elements.
size_t scan_tmp_elems(uint64_t n);
hipError_t scan_excl_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, uint64_t* d_total,
                         hipStream_t s);
// Same for uint32 inputs producing uint64 prefixes.
hipError_t scan_excl_u32_to_u64(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, uint64_t* d_total,
                                hipStream_t s);

// Stable LSD radix sort of (key, payload) pairs on the low `bits` bits of the
// keys.  Buffers: keys/vals in (a), alternate (b); the result lands in (a) or
// (b) -- `*result_in_b` tells which.  `tmp` needs radix_tmp_elems(n) uint64.
size_t radix_tmp_elems(uint64_t n);
hipError_t radix_sort_u64(uint64_t* keys_a, uint32_t* vals_a, uint64_t* keys_b, uint32_t* vals_b, uint64_t n,
                          int bits, uint64_t* tmp, bool* result_in_b, hipStream_t s);
hipError_t radix_sort_u32(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, uint64_t n,
                          int bits, uint64_t* tmp, bool* result_in_b, hipStream_t s);
// Transpose of a CSR by a stable sort of its column ids `keys` (left
// intact): the sorted keys land in (a) or (b) (*sorted_keys), and for the
// entry p at sorted position g, ocol[g] = rows[p] (the entry's row) and
// oval[g] = val[p].  Rows and values move with the keys through every pass
// (wa, wb: n uint64 each), so every pass reads and writes in streams.
hipError_t radix_transpose_u32(const uint32_t* keys, const uint32_t* rows, const uint64_t* val, uint32_t* ka,
                               uint32_t* va, uint32_t* kb, uint32_t* vb, uint64_t* wa, uint64_t* wb, uint64_t n,
                               int bits, uint64_t* tmp, uint32_t* ocol, uint64_t* oval, const uint32_t** sorted_keys,
                               hipStream_t s);
// Packed transpose: each 32-bit payload holds an entry's output column in
// its high bits and its value in its low vb bits, so only 8 bytes per entry
// move through the passes; the last pass splits the payload into ocol and
// oval.  Values of 2^vb - 1 and more are packed as 2^vb - 1 (escapes): with
// esc set, the last pass also lists the output positions of the escapes
// (esc, count in *nesc, which must be zero on entry; one atomic per
// workgroup), and launch_escape_fix fills their values from the input.
struct Unpack {
    int vb;                              // value bits, 1..24
    uint32_t* ocol;                      // n output column ids
    uint64_t* oval;                      // n output values
    uint32_t* esc = nullptr;             // n slots, or null
    unsigned long long* nesc = nullptr;  // escapes listed
};
hipError_t radix_transpose_packed_u32(const uint32_t* keys, const uint32_t* packed, uint32_t* ka, uint32_t* va,
                                      uint32_t* kb, uint32_t* vb, uint64_t n, int bits, uint64_t* tmp,
                                      const Unpack& up, const uint32_t** sorted_keys, hipStream_t s);
// The escapes of a packed transpose: every listed output entry g (key
// keys[g], the input column; column ocol[g], the input row, or the row
// row_inv maps it back to) takes the input's value at that row and column,
// found by binary search (the input rows must be sorted by column).
hipError_t launch_escape_fix(const uint32_t* esc, const unsigned long long* nesc, const uint32_t* keys,
                             const uint32_t* ocol, const uint64_t* rowptr, const uint32_t* col, const uint64_t* val,
                             const uint32_t* row_inv, uint64_t* oval, hipStream_t s);
// Same, reading the keys from `keys` (left intact) with the entry index as
// payload; the result lands in (a) or (b).
hipError_t radix_sort_u32_from(const uint32_t* keys, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                               uint32_t* vals_b, uint64_t n, int bits, uint64_t* tmp, bool* result_in_b,
                               hipStream_t s);

}  // namespace msc

// Device-wide prefix sum and stable LSD radix sort (the "prefix scan" and
// "stream compaction" primitives of Section 2.3, written for wave64).
#include "prims.h"

namespace msc {
namespace {

constexpr int ST = 256;            // scan threads per workgroup
constexpr int SI = 8;              // scan items per thread
constexpr int STILE = ST * SI;

template <typename TIn>
__global__ __launch_bounds__(ST) void scan_reduce(const TIn* __restrict__ in, uint64_t n, uint64_t* __restrict__ part) {
    __shared__ uint64_t sc[ST / WAVE + 1];
    uint64_t base = (uint64_t)blockIdx.x * STILE;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SI; i++) {
        uint64_t j = base + (uint64_t)i * ST + threadIdx.x;
        if (j < n) s += (uint64_t)in[j];
    }
    uint64_t tot;
    block_excl_scan<uint64_t, ST>(s, sc, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// exclusive scan of one tile; adds `offset` (device, may be null); writes the
// tile total to *total when non-null (single-tile case)
template <typename TIn>
__global__ __launch_bounds__(ST) void scan_tile(const TIn* __restrict__ in, uint64_t* __restrict__ out, uint64_t n,
                                                const uint64_t* __restrict__ offsets, uint64_t* __restrict__ total) {
    __shared__ uint64_t sc[ST / WAVE + 1];
    uint64_t base = (uint64_t)blockIdx.x * STILE + (uint64_t)threadIdx.x * SI;
    uint64_t v[SI];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SI; i++) {
        uint64_t j = base + i;
        v[i] = j < n ? (uint64_t)in[j] : 0;
        s += v[i];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan<uint64_t, ST>(s, sc, tot);
    if (offsets) ex += offsets[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SI; i++) {
        uint64_t j = base + i;
        if (j < n) out[j] = ex;
        ex += v[i];
    }
    if (total && threadIdx.x == 0) *total = tot;
}

template <typename TIn>
hipError_t scan_impl(const TIn* in, uint64_t* out, uint64_t n, uint64_t* tmp, uint64_t* d_total, hipStream_t s) {
    if (n <= (uint64_t)STILE) {
        hipLaunchKernelGGL(scan_tile<TIn>, dim3(1), dim3(ST), 0, s, in, out, n, (const uint64_t*)nullptr, d_total);
        return hipGetLastError();
    }
    uint64_t nb = (n + STILE - 1) / STILE;
    hipLaunchKernelGGL(scan_reduce<TIn>, dim3((unsigned)nb), dim3(ST), 0, s, in, n, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_impl<uint64_t>(tmp, tmp, nb, tmp + nb, d_total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_tile<TIn>, dim3((unsigned)nb), dim3(ST), 0, s, in, out, n, (const uint64_t*)tmp,
                       (uint64_t*)nullptr);
    return hipGetLastError();
}

// ---- radix sort -----------------------------------------------------------

constexpr int RT = 256;           // threads
constexpr int RR = 16;            // rounds of RT keys per tile
constexpr int RTILE = RT * RR;
constexpr int RWAVES = RT / WAVE;
constexpr int MAX_DB = 9;         // digit bits: 8, or 9 when that saves a pass

template <typename K, int DB>
__global__ __launch_bounds__(RT) void radix_hist(const K* __restrict__ keys, uint64_t n, int shift, uint64_t nblk,
                                                 uint64_t* __restrict__ hist) {
    constexpr uint32_t NB = 1u << DB;
    __shared__ uint32_t h[NB];
    for (uint32_t d = threadIdx.x; d < NB; d += RT) h[d] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * RTILE;
    for (int r = 0; r < RR; r++) {
        uint64_t j = base + (uint64_t)r * RT + threadIdx.x;
        if (j < n) atomicAdd(&h[(uint32_t)(keys[j] >> shift) & (NB - 1u)], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < NB; d += RT) hist[(uint64_t)d * nblk + blockIdx.x] = h[d];
}

// An optional 64-bit side payload permuted along with the keys (the values
// of a transposed matrix): read from win, written to wout.
struct Wide {
    const uint64_t* win;
    uint64_t* wout;
};

// One pass of the stable LSD sort over a tile of RTILE keys.  Wave w owns
// the contiguous quarter [w * RTILE / 4, (w + 1) * RTILE / 4) of the tile and
// ranks its keys on its own, 64 at a time in index order: peers with the
// same digit by ballot, earlier ones by the wave's running digit counts in
// LDS (no workgroup barrier).  The waves' counts are then combined once
// (keys of wave w follow those of the earlier waves, which keeps the sort
// stable), the tile is staged in LDS ordered by (digit, rank), and written
// out so that the keys of one digit leave as one contiguous run at that
// digit's global offset for this tile.  vals null: the payload is the entry
// index.  With a side payload (wd.win set) the same LDS then stages the
// 64-bit side values, read again in the input order, and writes them in
// the same runs.  With up.ocol set (the last pass of a packed transpose)
// each payload is split into its column and value instead of written out.
template <typename K, int DB>
__global__ __launch_bounds__(RT) void radix_scatter(const K* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                    K* __restrict__ okeys, uint32_t* __restrict__ ovals, uint64_t n,
                                                    int shift, uint64_t nblk, const uint64_t* __restrict__ offs,
                                                    Wide wd, Unpack up) {
    constexpr uint32_t NB = 1u << DB;
    constexpr uint32_t DPT = NB / RT;       // digits owned by one thread in the tile scan
    constexpr int WR = RTILE / RWAVES / WAVE;  // rounds of one wave (RR)
    __shared__ uint64_t gbase[NB];
    __shared__ uint32_t tstart[NB];
    __shared__ uint32_t wcnt[RWAVES][NB];
    // staged keys and payloads; reused for the side payload as RTILE uint64
    __shared__ uint64_t sstage[RTILE * (sizeof(K) + 4) / 8];
    K* skey = (K*)sstage;
    uint32_t* sval = (uint32_t*)(skey + RTILE);
    __shared__ uint32_t sc[RT / WAVE + 1];
    const int tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
    for (uint32_t d = tid; d < NB; d += RT) gbase[d] = offs[(uint64_t)d * nblk + blockIdx.x];
    for (uint32_t i = tid; i < RWAVES * NB; i += RT) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint64_t wbase = (uint64_t)blockIdx.x * RTILE + (uint64_t)w * (RTILE / RWAVES);
    uint32_t* cnt = wcnt[w];
    K kr[WR];
    uint32_t vr[WR], rk[WR];
    // all of the wave's loads first: the ranking below is ordered by fences,
    // which would otherwise hold each round's load until the previous round
#pragma unroll
    for (int r = 0; r < WR; r++) {
        const uint64_t j = wbase + (uint64_t)r * WAVE + lane;
        const bool valid = j < n;
        kr[r] = valid ? keys[j] : (K)0;
        vr[r] = valid ? (vals ? vals[j] : (uint32_t)j) : 0u;
    }
#pragma unroll
    for (int r = 0; r < WR; r++) {
        const uint64_t j = wbase + (uint64_t)r * WAVE + lane;
        const bool valid = j < n;
        const K key = kr[r];
        const uint32_t d = (uint32_t)(key >> shift) & (NB - 1u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < DB; b++) {
            uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t wrank = (uint32_t)__popcll(peers & lt);
        const uint32_t before = valid ? cnt[d] : 0u;  // every lane reads before any lane writes
        __builtin_amdgcn_wave_barrier();
        if (valid && wrank == 0) cnt[d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        rk[r] = before + wrank;
    }
    __syncthreads();
    // per digit: waves' counts -> exclusive offsets across waves, tile totals
    uint32_t own = 0;
#pragma unroll
    for (uint32_t q = 0; q < DPT; q++) {
        const uint32_t d = tid * DPT + q;
        uint32_t run = 0;
        for (int x = 0; x < RWAVES; x++) {
            const uint32_t c = wcnt[x][d];
            wcnt[x][d] = run;
            run += c;
        }
        tstart[d] = run;  // the digit's tile total for now
        own += run;
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<uint32_t, RT>(own, sc, tot);
#pragma unroll
    for (uint32_t q = 0; q < DPT; q++) {
        const uint32_t d = tid * DPT + q;
        const uint32_t c = tstart[d];
        tstart[d] = ex;
        ex += c;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < WR; r++) {
        const uint64_t j = wbase + (uint64_t)r * WAVE + lane;
        if (j < n) {
            const uint32_t d = (uint32_t)(kr[r] >> shift) & (NB - 1u);
            const uint32_t p = tstart[d] + cnt[d] + rk[r];
            skey[p] = kr[r];
            sval[p] = vr[r];
        }
    }
    __syncthreads();
    if (up.ocol) {  // uniform
        const uint32_t mask = (1u << up.vb) - 1u;
        for (uint32_t i = (uint32_t)tid; i < tot; i += RT) {
            const K key = skey[i];
            const uint32_t d = (uint32_t)(key >> shift) & (NB - 1u);
            const uint64_t g = gbase[d] + (i - tstart[d]);
            const uint32_t v = sval[i];
            okeys[g] = key;
            up.ocol[g] = v >> up.vb;
            up.oval[g] = v & mask;
        }
        if (!up.esc) return;  // uniform
        // list the tile's escapes: count per thread, scan, one atomic per workgroup
        uint32_t mine = 0;
        for (uint32_t i = (uint32_t)tid; i < tot; i += RT) mine += (sval[i] & mask) == mask ? 1u : 0u;
        uint32_t all;
        uint32_t pos = block_excl_scan<uint32_t, RT>(mine, sc, all);
        if (all == 0) return;  // uniform
        __shared__ unsigned long long s_base;
        if (tid == 0) s_base = atomicAdd(up.nesc, (unsigned long long)all);
        __syncthreads();
        const uint64_t eb = s_base + pos;
        uint32_t q = 0;
        for (uint32_t i = (uint32_t)tid; i < tot && q < mine; i += RT) {
            if ((sval[i] & mask) != mask) continue;
            const K key = skey[i];
            const uint32_t d = (uint32_t)(key >> shift) & (NB - 1u);
            up.esc[eb + q++] = (uint32_t)(gbase[d] + (i - tstart[d]));
        }
        return;
    }
    for (uint32_t i = (uint32_t)tid; i < tot; i += RT) {
        const K key = skey[i];
        const uint32_t d = (uint32_t)(key >> shift) & (NB - 1u);
        const uint64_t g = gbase[d] + (i - tstart[d]);
        okeys[g] = key;
        ovals[g] = sval[i];
    }
    if (!wd.win) return;  // uniform
    __syncthreads();
#pragma unroll
    for (int r = 0; r < WR; r++) {
        const uint64_t j = wbase + (uint64_t)r * WAVE + lane;
        if (j < n) {
            const uint32_t d = (uint32_t)(kr[r] >> shift) & (NB - 1u);
            sstage[tstart[d] + cnt[d] + rk[r]] = wd.win[j];
        }
    }
    __syncthreads();
    for (uint32_t i = (uint32_t)tid; i < tot; i += RT) {
        // the digit of staged slot i: the last digit whose tile start is <= i
        uint32_t lo = 0, hi = NB;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tstart[mid] <= i) lo = mid;
            else hi = mid;
        }
        // (empty digits share their start with the next one: take the last of them)
        wd.wout[gbase[lo] + (i - tstart[lo])] = sstage[i];
    }
}

template <typename K, int DB>
hipError_t radix_pass(const K* src_k, const uint32_t* src_v, K* dst_k, uint32_t* dst_v, uint64_t n, int sh,
                      uint64_t nblk, uint64_t* hist, uint64_t* stmp, const Wide& wd, const Unpack& up,
                      hipStream_t s) {
    hipLaunchKernelGGL((radix_hist<K, DB>), dim3((unsigned)nblk), dim3(RT), 0, s, src_k, n, sh, nblk, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_impl<uint64_t>(hist, hist, (uint64_t)(1u << DB) * nblk, stmp, (uint64_t*)nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((radix_scatter<K, DB>), dim3((unsigned)nblk), dim3(RT), 0, s, src_k, src_v, dst_k, dst_v, n, sh,
                       nblk, (const uint64_t*)hist, wd, up);
    return hipGetLastError();
}

// Stable LSD sort.  Pass 0 reads (keys0, vals0) -- vals0 null means the
// payload is the entry index -- and the passes then alternate between the
// (ka, va) and (kb, vb) buffers; *in_b tells where the keys end.  Digits
// are 8 bits, or 9 when that needs fewer passes.  With w0 set, a 64-bit
// side payload moves along, from w0 through (wa, wb).  With last_v set, the
// last pass writes the payload to last_v and the side payload to last_w.
// With last_up set, the last pass splits packed payloads as it describes.
template <typename K>
hipError_t radix_impl(const K* keys0, const uint32_t* vals0, K* ka, uint32_t* va, K* kb, uint32_t* vb, uint64_t n,
                      int bits, uint64_t* tmp, bool* in_b, hipStream_t s, const uint64_t* w0 = nullptr,
                      uint64_t* wa = nullptr, uint64_t* wb = nullptr, uint32_t* last_v = nullptr,
                      uint64_t* last_w = nullptr, const Unpack* last_up = nullptr) {
    *in_b = false;
    if (n == 0) return hipSuccess;
    const int p8 = bits <= 0 ? 1 : (bits + 7) / 8;
    const int p9 = bits <= 0 ? 1 : (bits + 8) / 9;
    const bool nine = p9 < p8;
    const int passes = nine ? p9 : p8;
    uint64_t nblk = (n + RTILE - 1) / RTILE;
    uint64_t* hist = tmp;
    uint64_t* stmp = tmp + (uint64_t)(1u << MAX_DB) * nblk;
    const K* src_k = keys0;
    const uint32_t* src_v = vals0;
    const uint64_t* src_w = w0;
    K* dst_k = ka;
    uint32_t* dst_v = va;
    uint64_t* dst_w = wa;
    bool dst_is_b = false;
    for (int p = 0; p < passes; p++) {
        const bool last = p + 1 == passes;
        uint32_t* pv = last && last_v ? last_v : dst_v;
        const Wide wd{src_w, last && last_w ? last_w : dst_w};
        const Unpack up = last && last_up ? *last_up : Unpack{};
        hipError_t e = nine ? radix_pass<K, 9>(src_k, src_v, dst_k, pv, n, 9 * p, nblk, hist, stmp, wd, up, s)
                            : radix_pass<K, 8>(src_k, src_v, dst_k, pv, n, 8 * p, nblk, hist, stmp, wd, up, s);
        if (e != hipSuccess) return e;
        *in_b = dst_is_b;
        src_k = dst_k;
        src_v = dst_v;
        src_w = w0 ? dst_w : nullptr;
        dst_k = dst_is_b ? ka : kb;
        dst_v = dst_is_b ? va : vb;
        dst_w = dst_is_b ? wa : wb;
        dst_is_b = !dst_is_b;
    }
    return hipSuccess;
}

}  // namespace

namespace {
__global__ __launch_bounds__(256) void k_escape_fix(const uint32_t* __restrict__ esc,
                                                    const unsigned long long* __restrict__ nesc,
                                                    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ ocol,
                                                    const uint64_t* __restrict__ rowptr,
                                                    const uint32_t* __restrict__ col, const uint64_t* __restrict__ val,
                                                    const uint32_t* __restrict__ row_inv, uint64_t* __restrict__ oval) {
    const uint64_t n = *nesc;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t g = esc[i], key = keys[g], c = ocol[g];
        const uint32_t r = row_inv ? row_inv[c] : c;
        uint64_t lo = rowptr[r], hi = rowptr[r + 1];  // first column >= key
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (col[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        oval[g] = (lo < rowptr[r + 1] && col[lo] == key) ? val[lo] : 0;  // found for rows holding each column once
    }
}
__global__ void k_publish(const uint64_t* __restrict__ src, uint64_t n, uint64_t* __restrict__ dst) {
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}
__global__ void k_set_u64(uint64_t* __restrict__ dst, uint64_t v) {
    if (threadIdx.x == 0) *dst = v;
}
}  // namespace

hipError_t launch_escape_fix(const uint32_t* esc, const unsigned long long* nesc, const uint32_t* keys,
                             const uint32_t* ocol, const uint64_t* rowptr, const uint32_t* col, const uint64_t* val,
                             const uint32_t* row_inv, uint64_t* oval, hipStream_t s) {
    hipLaunchKernelGGL(k_escape_fix, dim3(2048), dim3(256), 0, s, esc, nesc, keys, ocol, rowptr, col, val, row_inv,
                       oval);
    return hipGetLastError();
}

hipError_t launch_publish(const uint64_t* src, uint64_t n, uint64_t* dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, src, n, dst);
    return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t* dst, uint64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

size_t scan_tmp_elems(uint64_t n) {
    size_t t = 1;
    while (n > (uint64_t)STILE) {
        n = (n + STILE - 1) / STILE;
        t += n;
    }
    return t + 1;
}

hipError_t scan_excl_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, uint64_t* d_total,
                         hipStream_t s) {
    if (n == 0) {
        if (d_total) return hipMemsetAsync(d_total, 0, sizeof(uint64_t), s);
        return hipSuccess;
    }
    return scan_impl<uint64_t>(in, out, n, tmp, d_total, s);
}

hipError_t scan_excl_u32_to_u64(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, uint64_t* d_total,
                                hipStream_t s) {
    if (n == 0) {
        if (d_total) return hipMemsetAsync(d_total, 0, sizeof(uint64_t), s);
        return hipSuccess;
    }
    return scan_impl<uint32_t>(in, out, n, tmp, d_total, s);
}

size_t radix_tmp_elems(uint64_t n) {
    uint64_t nblk = (n + RTILE - 1) / RTILE;
    if (nblk < 1) nblk = 1;
    return (1u << MAX_DB) * nblk + scan_tmp_elems((1u << MAX_DB) * nblk);
}

hipError_t radix_sort_u64(uint64_t* ka, uint32_t* va, uint64_t* kb, uint32_t* vb, uint64_t n, int bits,
                          uint64_t* tmp, bool* in_b, hipStream_t s) {
    // the first pass reads (ka, va) and writes (kb, vb)
    hipError_t e = radix_impl<uint64_t>(ka, va, kb, vb, ka, va, n, bits, tmp, in_b, s);
    *in_b = !*in_b;
    return e;
}

hipError_t radix_sort_u32(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, uint64_t n, int bits,
                          uint64_t* tmp, bool* in_b, hipStream_t s) {
    hipError_t e = radix_impl<uint32_t>(ka, va, kb, vb, ka, va, n, bits, tmp, in_b, s);
    *in_b = !*in_b;
    return e;
}

hipError_t radix_sort_u32_from(const uint32_t* keys, uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                               uint64_t n, int bits, uint64_t* tmp, bool* in_b, hipStream_t s) {
    return radix_impl<uint32_t>(keys, nullptr, ka, va, kb, vb, n, bits, tmp, in_b, s);
}

hipError_t radix_transpose_u32(const uint32_t* keys, const uint32_t* rows, const uint64_t* val, uint32_t* ka,
                               uint32_t* va, uint32_t* kb, uint32_t* vb, uint64_t* wa, uint64_t* wb, uint64_t n,
                               int bits, uint64_t* tmp, uint32_t* ocol, uint64_t* oval, const uint32_t** sorted_keys,
                               hipStream_t s) {
    bool in_b = false;
    hipError_t e = radix_impl<uint32_t>(keys, rows, ka, va, kb, vb, n, bits, tmp, &in_b, s, val, wa, wb, ocol, oval);
    *sorted_keys = in_b ? kb : ka;
    return e;
}

hipError_t radix_transpose_packed_u32(const uint32_t* keys, const uint32_t* packed, uint32_t* ka, uint32_t* va,
                                      uint32_t* kb, uint32_t* vb, uint64_t n, int bits, uint64_t* tmp,
                                      const Unpack& up, const uint32_t** sorted_keys, hipStream_t s) {
    if (up.vb < 1 || up.vb > 24 || !up.ocol || !up.oval) return hipErrorInvalidValue;
    bool in_b = false;
    hipError_t e = radix_impl<uint32_t>(keys, packed, ka, va, kb, vb, n, bits, tmp, &in_b, s, nullptr, nullptr,
                                        nullptr, nullptr, nullptr, &up);
    *sorted_keys = in_b ? kb : ka;
    return e;
}

}  // namespace msc

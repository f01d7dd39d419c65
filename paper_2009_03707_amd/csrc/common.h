// Shared definitions of the HIP path: grid indexing, cell-id arithmetic on
// the refined grid, gradient-word decoding, launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace msc {

// Gradient-word nibble codes (see include/msc.h).
constexpr uint32_t NB_NONE = 7u;
constexpr uint32_t NB_CRIT = 8u;

// Label flag used by pointer jumping: set on a root (the low bits then hold
// the rank of the extremum), clear on a plain successor pointer.
constexpr uint32_t ROOT_FLAG = 0x80000000u;
constexpr uint32_t EXIT_LABEL = 0xFFFFFFFFu;  // a (2,3) path that leaves the grid
// Label of a reachable non-saddle edge of the 1-2 DAG: its junction id
// (< 2^31) if it has several out-edges; SUCC_FLAG | step if it has exactly
// one, where the step names that out-edge: bits 0-2 = 2 * axis + (sign > 0)
// of the cofacet quad, bits 3-6 = the quad's gradient nibble (1..6: the quad
// is paired with an edge, >= 8: the quad is a 2-saddle); NOT_JUNCTION if it
// has none.
constexpr uint32_t SUCC_FLAG = 0x80000000u;
constexpr uint32_t NOT_JUNCTION = 0xFFFFFFFFu;

// floor(n / d) for 0 <= n < 2^30 via one 64-bit multiply and shift
// (Granlund-Montgomery: m = ceil(2^(30+l) / d), l = ceil(log2 d)).
struct FastDiv {
    uint64_t m;
    uint32_t s;
    uint32_t d;
    static FastDiv make(uint32_t d) {
        FastDiv r;
        uint32_t l = 0;
        while ((1ull << l) < d) l++;
        r.s = 30 + l;
        r.m = ((1ull << r.s) + d - 1) / d;
        r.d = d;
        return r;
    }
    __host__ __device__ inline uint32_t div(uint32_t n) const { return (uint32_t)(((uint64_t)n * m) >> s); }
};

struct Grid {
    uint32_t n[3];       // vertex counts x, y, z
    uint32_t stride[3];  // 1, nx, nx*ny
    uint32_t nv;
    FastDiv dx, dxy;
    static Grid make(int64_t nx, int64_t ny, int64_t nz) {
        Grid g;
        g.n[0] = (uint32_t)nx; g.n[1] = (uint32_t)ny; g.n[2] = (uint32_t)nz;
        g.stride[0] = 1; g.stride[1] = (uint32_t)nx; g.stride[2] = (uint32_t)(nx * ny);
        g.nv = (uint32_t)(nx * ny * nz);
        g.dx = FastDiv::make((uint32_t)nx);
        g.dxy = FastDiv::make((uint32_t)(nx * ny));
        return g;
    }
    __device__ inline void coords(uint32_t v, uint32_t c[3]) const {
        uint32_t z = dxy.div(v);
        uint32_t r = v - z * stride[2];
        uint32_t y = dx.div(r);
        c[0] = r - y * stride[1];
        c[1] = y;
        c[2] = z;
    }
};

// A batch of fields laid end to end in one vertex index space: field f owns
// global vertex ids [voff[f], voff[f+1]) and cell ids 8 * that range.  Cells
// of different fields are never adjacent, so every traversal stays inside
// the field it starts in.  One field is the special case nf == 1.
struct Geo {
    const Grid* grids;     // device, nf entries
    const uint32_t* voff;  // device, nf + 1 entries
    uint32_t nf;
    uint32_t nv;           // total vertices
    Grid g0;               // the grid of field 0 (used directly when nf == 1)
    __device__ inline uint32_t field_of(uint32_t v) const {
        if (nf == 1) return 0;
        uint32_t lo = 0, hi = nf;  // last f with voff[f] <= v
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (voff[mid] <= v) lo = mid;
            else hi = mid;
        }
        return lo;
    }
    __device__ inline Grid grid(uint32_t f) const { return nf == 1 ? g0 : grids[f]; }
    __device__ inline uint32_t base(uint32_t f) const { return nf == 1 ? 0u : voff[f]; }
};

__device__ inline uint32_t nib_of(uint32_t word, uint32_t k) { return (word >> (4u * k)) & 15u; }

// Slot of cell (w, k) in the per-cell label array of edges and quads
// (1 <= k <= 6): one plane of nv words per cell type k, so labels of
// neighbouring cells of one type share cache lines.
__device__ inline uint64_t label_slot(uint32_t w, uint32_t k, uint32_t nv) { return (uint64_t)(k - 1u) * nv + w; }

// p[i] for a pointer known to address device memory but taken from a table
// (the compiler cannot infer that itself and would use generic loads).
template <typename T>
__device__ inline T load_global(const T* p, uint64_t i) {
    return ((const __attribute__((address_space(1))) T*)p)[i];
}

// Cell one refined step from (w, k) along `axis` with sign `s` (+1 / -1).
// Returns false when the step leaves the grid.  `c` holds the coordinates of
// vertex w.
// a[i] of a three-element array by selects, so that an index known only at
// run time does not force the array out of registers
__device__ inline uint32_t pick3(const uint32_t a[3], uint32_t i) { return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]); }

__device__ inline bool cell_step(const Grid& g, uint32_t w, uint32_t k, const uint32_t c[3], int axis, int s,
                                 uint32_t& w2, uint32_t& k2) {
    uint32_t bit = 1u << axis;
    const uint32_t st = pick3(g.stride, (uint32_t)axis);
    if (k & bit) {
        k2 = k & ~bit;
        w2 = (s > 0) ? w + st : w;
        return true;
    }
    k2 = k | bit;
    if (s > 0) {
        if (pick3(c, (uint32_t)axis) + 1 >= pick3(g.n, (uint32_t)axis)) return false;
        w2 = w;
    } else {
        if (pick3(c, (uint32_t)axis) == 0) return false;
        w2 = w - st;
    }
    return true;
}

// Saturating unsigned 64-bit arithmetic: every sum and product of path
// counts equals min(true value, 2^64-1), whatever the evaluation order.
__device__ inline uint64_t sat_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s < a ? ~0ull : s;
}
__device__ inline uint64_t sat_mul(uint64_t a, uint64_t b) {
    if (__umul64hi(a, b) != 0) return ~0ull;
    return a * b;
}

inline unsigned grid_blocks(uint64_t n, unsigned block) {
    uint64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace msc

// Saddle-extremum arcs (Section 3.4; Section 3.5, "Saddle-Extrema arcs").
//
// (0,1) and (2,3) gradient paths split or merge but never both, so the
// destination extremum of every cell is a root-finding problem in a forest,
// solved by pointer jumping.  Vertex pointers follow the edge each vertex is
// paired with; cube pointers cross the quad each cube is paired with (or
// leave the grid).  A root holds ROOT_FLAG | rank of its extremum, so after
// convergence every pointer is directly the rank of its extremum (the
// ascending manifolds of minima and descending manifolds of maxima).
//
// Unlike the paper's two surface buffers, the jump is done in place: a
// pointer is only ever replaced by one of its ancestors, so reading a value
// that another thread has already advanced is still correct and only
// converges faster.
#include "prims.h"

namespace msc {
namespace {

constexpr int BT = 256;

// The pointer-jumping kernels give a thread PJ_EPT elements, BT apart
// (coalesced per round, and independent chains in flight): with one element
// per thread the launches are bound by the rate at which workgroups are
// dispatched.
constexpr int PJ_EPT = 4;

__device__ __forceinline__ void pj_init_vertex(const uint32_t* __restrict__ grad, const Geo& geo,
                                               uint32_t* __restrict__ Pv, uint32_t* __restrict__ Pc,
                                               int* __restrict__ err, uint32_t v) {
    uint32_t fld = geo.field_of(v);
    const Grid g = geo.grid(fld);
    uint32_t w = grad[v];
    uint32_t c[3];
    g.coords(v - geo.base(fld), c);
    uint32_t n0 = w & 15u;
    uint32_t pv = ROOT_FLAG;
    if (n0 >= NB_CRIT) {
        pv = ROOT_FLAG;
    } else if (n0 >= 1 && n0 <= 6) {
        uint32_t a = (n0 - 1u) >> 1;
        bool neg = ((n0 - 1u) & 1u) != 0;
        if (neg ? c[a] >= 1 : c[a] + 1 < g.n[a])
            pv = neg ? v - g.stride[a] : v + g.stride[a];
        else
            atomicOr(err, 1);
    } else {
        atomicOr(err, 1);  // a vertex always exists and is never "missing"
    }
    Pv[v] = pv;
    uint32_t n7 = (w >> 28) & 15u;
    uint32_t pc;
    if (n7 == NB_NONE) {
        pc = EXIT_LABEL;
    } else if (n7 >= NB_CRIT) {
        pc = ROOT_FLAG;
    } else if (n7 >= 1 && n7 <= 6) {
        uint32_t a = (n7 - 1u) >> 1;
        if ((n7 - 1u) & 1u)
            pc = c[a] >= 1 ? v - g.stride[a] : EXIT_LABEL;
        else
            pc = c[a] + 2 < g.n[a] ? v + g.stride[a] : EXIT_LABEL;
    } else {
        pc = EXIT_LABEL;
        atomicOr(err, 1);
    }
    Pc[v] = pc;
}

// PJ_EPT vertices per thread, BT apart
__global__ __launch_bounds__(BT) void k_pj_init(const uint32_t* __restrict__ grad, Geo geo, uint32_t* __restrict__ Pv,
                                                uint32_t* __restrict__ Pc, int* __restrict__ err) {
#pragma unroll
    for (int r = 0; r < PJ_EPT; r++) {
        const uint64_t v = ((uint64_t)blockIdx.x * PJ_EPT + r) * BT + threadIdx.x;
        if (v < geo.nv) pj_init_vertex(grad, geo, Pv, Pc, err, (uint32_t)v);
    }
}

// Labels roots with ranks and checks the critical list against the gradient
// (critical nibble, index of each segment, strictly increasing ids).
__global__ __launch_bounds__(BT) void k_label(const uint32_t* __restrict__ crit, uint64_t c0, uint64_t c1,
                                              uint64_t c2, uint64_t c3, const uint32_t* __restrict__ grad, Geo g,
                                              uint32_t* __restrict__ Pv, uint32_t* __restrict__ Pc,
                                              uint32_t* __restrict__ label, int* __restrict__ err) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    uint64_t total = c0 + c1 + c2 + c3;
    if (i >= total) return;
    uint32_t idx = 0;
    uint64_t start = 0;
    if (i >= c0) { idx = 1; start = c0; }
    if (i >= c0 + c1) { idx = 2; start = c0 + c1; }
    if (i >= c0 + c1 + c2) { idx = 3; start = c0 + c1 + c2; }
    uint32_t id = crit[i];
    uint32_t w = id >> 3, k = id & 7u;
    bool ok = w < g.nv && (uint32_t)__builtin_popcount(k) == idx && (i == start || crit[i - 1] < id);
    if (ok) ok = nib_of(grad[w], k) >= NB_CRIT;
    if (!ok) {
        atomicOr(err, 2);
        return;
    }
    uint32_t rank = (uint32_t)(i - start);
    if (idx == 0) Pv[w] = ROOT_FLAG | rank;
    else if (idx == 3) Pc[w] = ROOT_FLAG | rank;
    else if (idx == 2) label[label_slot(w, k, g.nv)] = rank;
}

// PJ_HOPS jumps for every unfinished pointer: P[i] <- P[P[P[P[i]]]] for
// three (pointers are updated in place, so a jump may already use a pointer
// shortened in this round; every pointer always leads to the same root).
// A round at least quadruples the distance a pointer covers, so fewer
// rounds, and fewer full passes over P, are needed than with one jump.
// `changed` holds 64 words; a workgroup with an unfinished pointer stores 1
// into one of them (spread so that the stores do not queue on a single
// address).
constexpr int PJ_HOPS = 3;

__global__ __launch_bounds__(BT) void k_pj_round(uint32_t* __restrict__ P, uint32_t n, int* __restrict__ changed) {
    uint32_t p[PJ_EPT];
    uint32_t todo = 0;  // bit r: element r is in range and not yet at a root
    int active = 0;
#pragma unroll
    for (int r = 0; r < PJ_EPT; r++) {
        const uint64_t i = ((uint64_t)blockIdx.x * PJ_EPT + r) * BT + threadIdx.x;
        p[r] = i < n ? P[i] : ROOT_FLAG;
        if (!(p[r] & ROOT_FLAG)) todo |= 1u << r;
    }
#pragma unroll
    for (int h = 0; h < PJ_HOPS; h++)
#pragma unroll
        for (int r = 0; r < PJ_EPT; r++)
            if (!(p[r] & ROOT_FLAG)) p[r] = P[p[r]];
#pragma unroll
    for (int r = 0; r < PJ_EPT; r++) {
        const uint64_t i = ((uint64_t)blockIdx.x * PJ_EPT + r) * BT + threadIdx.x;
        if ((todo >> r) & 1u) {
            P[i] = p[r];
            active |= !(p[r] & ROOT_FLAG);
        }
    }
    if (__syncthreads_or(active) && threadIdx.x == 0) changed[blockIdx.x & 63u] = 1;
}

// M10 rows: the two vertices of each 1-saddle lead to their minima.
template <bool FILL>
__global__ __launch_bounds__(BT) void k_m10(const uint32_t* __restrict__ s1, uint64_t S1, Geo geo,
                                            const uint32_t* __restrict__ Pv, uint32_t* __restrict__ cnt,
                                            const uint64_t* __restrict__ rowptr, uint32_t* __restrict__ col,
                                            uint64_t* __restrict__ val, int* __restrict__ err) {
    uint64_t r = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (r >= S1) return;
    uint32_t id = s1[r];
    uint32_t w = id >> 3, k = id & 7u;
    uint32_t a = (uint32_t)__builtin_ctz(k);
    const Grid g = geo.grid(geo.field_of(w));
    uint32_t pa = Pv[w], pb = Pv[w + g.stride[a]];
    if (!(pa & pb & ROOT_FLAG)) {
        atomicOr(err, 4);
        return;
    }
    uint32_t la = pa & ~ROOT_FLAG, lb = pb & ~ROOT_FLAG;
    if (!FILL) {
        cnt[r] = la == lb ? 1u : 2u;
        return;
    }
    uint64_t p = rowptr[r];
    if (la == lb) {
        col[p] = la;
        val[p] = 2;
    } else {
        col[p] = la < lb ? la : lb;
        val[p] = 1;
        col[p + 1] = la < lb ? lb : la;
        val[p + 1] = 1;
    }
}

// M32 transposed rows: the cofacet cubes of each 2-saddle lead to maxima
// (or out of the grid, dropped).
template <bool FILL>
__global__ __launch_bounds__(BT) void k_m32t(const uint32_t* __restrict__ s2, uint64_t S2, Geo geo,
                                             const uint32_t* __restrict__ Pc, uint32_t* __restrict__ cnt,
                                             const uint64_t* __restrict__ rowptr, uint32_t* __restrict__ col,
                                             uint64_t* __restrict__ val, int* __restrict__ err) {
    uint64_t r = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (r >= S2) return;
    uint32_t id = s2[r];
    uint32_t w = id >> 3, k = id & 7u;
    uint32_t j = (k == 3u) ? 2u : (k == 5u ? 1u : 0u);  // the even axis of the quad
    uint32_t fld = geo.field_of(w);
    const Grid g = geo.grid(fld);
    uint32_t c[3];
    g.coords(w - geo.base(fld), c);
    uint32_t l[2] = {EXIT_LABEL, EXIT_LABEL};
    if (c[j] + 1 < g.n[j]) l[0] = Pc[w];
    if (c[j] >= 1) l[1] = Pc[w - g.stride[j]];
    uint32_t m = 0, e[2];
    for (int i = 0; i < 2; i++) {
        if (!(l[i] & ROOT_FLAG)) {
            atomicOr(err, 4);
            return;
        }
        if (l[i] != EXIT_LABEL) e[m++] = l[i] & ~ROOT_FLAG;
    }
    uint32_t nn = m == 2 && e[0] == e[1] ? 1u : m;
    if (!FILL) {
        cnt[r] = nn;
        return;
    }
    uint64_t p = rowptr[r];
    if (m == 1) {
        col[p] = e[0];
        val[p] = 1;
    } else if (m == 2) {
        if (e[0] == e[1]) {
            col[p] = e[0];
            val[p] = 2;
        } else {
            col[p] = e[0] < e[1] ? e[0] : e[1];
            val[p] = 1;
            col[p + 1] = e[0] < e[1] ? e[1] : e[0];
            val[p + 1] = 1;
        }
    }
}

// Converged pointers -> ascending and descending 3-manifolds (Section 3.4:
// the traversal that finds the saddle-extremum arcs also gives every vertex
// the minimum and every cube the maximum its gradient path reaches).  In
// place: Pv[v] becomes the rank of v's minimum, Pc[w] the rank of the maximum
// reached from the cube with lowest corner w, or EXIT_LABEL (no such cube, or
// its path leaves the grid).  `before` (batch only; null for one field) holds
// per field f the counts of minima (word 4f) and maxima (word 4f + 3) in
// earlier fields, which turns batch-wide ranks into the field's own.
__global__ __launch_bounds__(BT) void k_manifold_labels(uint32_t* __restrict__ Pv, uint32_t* __restrict__ Pc, Geo geo,
                                                        const uint64_t* __restrict__ before) {
#pragma unroll
    for (int r = 0; r < PJ_EPT; r++) {
        const uint64_t i = ((uint64_t)blockIdx.x * PJ_EPT + r) * BT + threadIdx.x;
        if (i >= geo.nv) continue;
        uint32_t a = Pv[i], b = Pc[i];
        uint32_t omin = 0, omax = 0;
        if (before) {
            uint32_t f = geo.field_of((uint32_t)i);
            omin = (uint32_t)before[4 * f];
            omax = (uint32_t)before[4 * f + 3];
        }
        Pv[i] = (a & ~ROOT_FLAG) - omin;
        Pc[i] = b == EXIT_LABEL ? EXIT_LABEL : (b & ~ROOT_FLAG) - omax;
    }
}

}  // namespace

hipError_t launch_pj_init(const uint32_t* grad, const Geo& g, uint32_t* Pv, uint32_t* Pc, int* err, hipStream_t s) {
    hipLaunchKernelGGL(k_pj_init, dim3(grid_blocks(g.nv, (unsigned)(BT * PJ_EPT))), dim3(BT), 0, s, grad, g, Pv, Pc, err);
    return hipGetLastError();
}

hipError_t launch_label(const uint32_t* crit, const int64_t cnt[4], const uint32_t* grad, const Geo& g, uint32_t* Pv,
                        uint32_t* Pc, uint32_t* label, int* err, hipStream_t s) {
    uint64_t total = (uint64_t)(cnt[0] + cnt[1] + cnt[2] + cnt[3]);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_label, dim3(grid_blocks(total, BT)), dim3(BT), 0, s, crit, (uint64_t)cnt[0], (uint64_t)cnt[1],
                       (uint64_t)cnt[2], (uint64_t)cnt[3], grad, g, Pv, Pc, label, err);
    return hipGetLastError();
}

hipError_t launch_pj_round(uint32_t* P, uint32_t n, int* changed, hipStream_t s) {
    hipLaunchKernelGGL(k_pj_round, dim3(grid_blocks(n, (unsigned)(BT * PJ_EPT))), dim3(BT), 0, s, P, n, changed);
    return hipGetLastError();
}

hipError_t launch_m10(bool fill, const uint32_t* s1, uint64_t S1, const Geo& g, const uint32_t* Pv, uint32_t* cnt,
                      const uint64_t* rowptr, uint32_t* col, uint64_t* val, int* err, hipStream_t s) {
    if (S1 == 0) return hipSuccess;
    if (fill)
        hipLaunchKernelGGL(k_m10<true>, dim3(grid_blocks(S1, BT)), dim3(BT), 0, s, s1, S1, g, Pv, cnt, rowptr, col,
                           val, err);
    else
        hipLaunchKernelGGL(k_m10<false>, dim3(grid_blocks(S1, BT)), dim3(BT), 0, s, s1, S1, g, Pv, cnt, rowptr, col,
                           val, err);
    return hipGetLastError();
}

hipError_t launch_m32t(bool fill, const uint32_t* s2, uint64_t S2, const Geo& g, const uint32_t* Pc, uint32_t* cnt,
                       const uint64_t* rowptr, uint32_t* col, uint64_t* val, int* err, hipStream_t s) {
    if (S2 == 0) return hipSuccess;
    if (fill)
        hipLaunchKernelGGL(k_m32t<true>, dim3(grid_blocks(S2, BT)), dim3(BT), 0, s, s2, S2, g, Pc, cnt, rowptr, col,
                           val, err);
    else
        hipLaunchKernelGGL(k_m32t<false>, dim3(grid_blocks(S2, BT)), dim3(BT), 0, s, s2, S2, g, Pc, cnt, rowptr, col,
                           val, err);
    return hipGetLastError();
}

hipError_t launch_manifold_labels(uint32_t* Pv, uint32_t* Pc, const Geo& g, const uint64_t* before, hipStream_t s) {
    if (g.nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_manifold_labels, dim3(grid_blocks(g.nv, (unsigned)(BT * PJ_EPT))), dim3(BT), 0, s, Pv, Pc, g,
                       before);
    return hipGetLastError();
}

}  // namespace msc

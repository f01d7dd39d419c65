// 1-saddle / 2-saddle connections (Sections 3.1-3.3 and 3.5).
//
// The DAG of 1-2 gradient pairs has a node for every 1-saddle and every edge
// paired with a quad.  From a node e, each cofacet quad Q other than the quad
// e is paired with leads to a 2-saddle (Q critical) or to the edge Q is
// paired with; a quad paired with a cube leads nowhere.  Traversals run
// against the direction of the discrete gradient (ascending from the
// 1-saddles), so they cannot cycle (Section 3.5).
//
// Reachability (Section 3.2): frontier BFS from all 1-saddles; a node is
// expanded by one lane, which tests-and-sets a visited bit for each target
// edge and appends the new ones to the next frontier with one atomic per
// wave (the order inside a frontier does not matter, only the visited set).
// The same lane counts the node's out-degree and, for reachable non-saddle
// nodes, marks junctions (out-degree > 1, Section 3.3) and numbers them; a
// node with a single out-edge records that edge's step in its label, so the
// minor tracing below follows it without looking at the cofacets again.
//
// DAG minor (Section 3.3, "DAG minor construction"): every (source, out-edge)
// pair -- sources are the 1-saddles and junctions -- is traced by one lane
// until it reaches a junction or a 2-saddle; paths that end elsewhere are
// dropped (Section 3.5).  Because a simple path never splits, a lane keeps
// walking in registers instead of compacting after each step.  Each lane
// writes to a fixed slot (4 per source), so the minor is assembled in source
// order without any sort.
#include "prims.h"

namespace msc {
namespace {

constexpr int BT = 256;
constexpr uint8_t T_NONE = 0, T_JUNC = 1, T_S2 = 2;

struct CellRef {
    uint32_t w, k;
};

// V(e): the quad an edge is paired with, if any.
__device__ __forceinline__ bool paired_quad(const Grid& g, uint32_t w, uint32_t k, uint32_t ne, const uint32_t c[3],
                                            uint32_t axis_e, CellRef& v) {
    if (ne < 1 || ne > 6) return false;
    uint32_t da = (ne - 1u) >> 1;
    if (da == axis_e) return false;  // paired with a vertex
    int s = ((ne - 1u) & 1u) ? -1 : 1;
    return cell_step(g, w, k, c, (int)da, s, v.w, v.k);
}

// If quad (qw, qk) is paired with one of its edges, that edge; otherwise false.
__device__ __forceinline__ bool quad_edge_partner(const Grid& g, uint32_t qw, uint32_t qk, uint32_t nq, CellRef& e) {
    if (nq < 1 || nq > 6) return false;
    uint32_t dq = (nq - 1u) >> 1;
    if (!((qk >> dq) & 1u)) return false;  // partner is a cube
    e.k = qk & ~(1u << dq);
    e.w = ((nq - 1u) & 1u) ? qw : qw + pick3(g.stride, dq);
    return true;
}

// The frontiers are consecutive ranges of one queue: level L is
// queue[lv[L], lv[L + 1]), sealed by k_bfs_seal from the queue's tail before
// the level is expanded, so the levels run back to back on the device and
// the host reads the boundaries back once per batch of levels.  The
// expansion grid is fixed and strides over the level in chunks of
// BFS_NPT * BT nodes (thread: nodes chunk * BFS_NPT * BT + r * BT + tid); a
// workgroup appends a chunk's new targets and junctions with one atomic on
// the packed tail (low 32 bits: queue length, high 32 bits: junctions);
// appends to one counter serialise, so they are kept few.
//
// A node's expansion is a chain of dependent memory operations (its own
// word, then the words of its cofacet quads, then a visited-bit atomic per
// partner edge).  A thread therefore runs its nodes in phases -- every own
// word, then every quad word, then every atomic -- so that all of one
// phase's loads (or atomics) are in flight together instead of one chain
// after another.  Slot 2 b + (s > 0) holds the cofacet quad one step along
// axis b with sign s (the edge's own axis leaves its two slots empty), so
// that every array index is known at compile time.  The quads of an edge e
// (other than V(e)) and the targets they lead to do not depend on the order
// they are visited in; a node with one out-edge records that edge's step.
constexpr int BFS_NPT = 2;
constexpr int BFS_S = 6;  // slots: 3 axes x 2 signs

constexpr unsigned BFS_GRID = 1024;  // 1024 and 65536 measured best at 512^3 (4096: +1.4 ms)

__global__ void k_bfs_seal(uint64_t* __restrict__ lv, uint64_t L, const unsigned long long* __restrict__ tail) {
    if (threadIdx.x == 0) lv[L + 1] = *tail & 0xFFFFFFFFull;
}

__global__ __launch_bounds__(BT) void k_bfs_expand(uint32_t* __restrict__ queue, uint64_t qcap,
                                                   const uint64_t* __restrict__ lv, uint64_t L,
                                                   const uint32_t* __restrict__ grad, Geo geo,
                                                   uint32_t* __restrict__ vis, unsigned long long* __restrict__ tail,
                                                   uint32_t* __restrict__ label) {
    const int level0 = L == 0;
    const uint64_t b0 = lv[L] < qcap ? lv[L] : qcap, b1 = lv[L + 1] < qcap ? lv[L + 1] : qcap;
    const uint64_t ncur = b1 > b0 ? b1 - b0 : 0;  // (the queue is never full; reads stay inside it regardless)
    const uint32_t* __restrict__ cur = queue + b0;
    __shared__ unsigned long long sc[BT / WAVE + 1];
    __shared__ unsigned long long base;
    for (uint64_t chunk = blockIdx.x; chunk * (uint64_t)(BFS_NPT * BT) < ncur; chunk += gridDim.x) {  // uniform
    uint32_t e[BFS_NPT], own[BFS_NPT];
    bool ok[BFS_NPT];
    // phase 1: the nodes and their own words
#pragma unroll
    for (int r = 0; r < BFS_NPT; r++) {
        const uint64_t i = (chunk * BFS_NPT + r) * BT + threadIdx.x;
        ok[r] = i < ncur;
        e[r] = ok[r] ? cur[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < BFS_NPT; r++) own[r] = ok[r] ? grad[e[r] >> 3] : 0u;
    // phase 2: each node's cofacet quads other than V(e) (cell ids), and their words
    uint32_t qc[BFS_NPT][BFS_S], qword[BFS_NPT][BFS_S];
    uint32_t qvalid[BFS_NPT];  // bit j: slot j holds a quad
#pragma unroll
    for (int r = 0; r < BFS_NPT; r++) {
        qvalid[r] = 0;
        const uint32_t w = e[r] >> 3, k = e[r] & 7u;
        const uint32_t fld = geo.field_of(w);
        const Grid g = geo.grid(fld);
        uint32_t c[3];
        g.coords(w - geo.base(fld), c);
        const uint32_t a = ok[r] ? (uint32_t)__builtin_ctz(k) : 3u;
        CellRef v;
        const bool hv = ok[r] && paired_quad(g, w, k, nib_of(own[r], k), c, a, v);
#pragma unroll
        for (uint32_t b = 0; b < 3; b++) {
#pragma unroll
            for (int sp = 0; sp < 2; sp++) {
                const int j = 2 * (int)b + sp;
                CellRef q;
                q.w = q.k = 0;
                const bool ex = ok[r] && b != a && cell_step(g, w, k, c, (int)b, sp ? 1 : -1, q.w, q.k) &&
                                !(hv && q.w == v.w && q.k == v.k);
                qc[r][j] = 8u * q.w + q.k;
                qvalid[r] |= (ex ? 1u : 0u) << j;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < BFS_NPT; r++)
#pragma unroll
        for (int j = 0; j < BFS_S; j++) {
            const bool v = (qvalid[r] >> j) & 1u;
            const uint32_t qw = qc[r][j] >> 3;
            qword[r][j] = !v ? 0u : (qw == (e[r] >> 3) ? own[r] : grad[qw]);
        }
    // phase 3: out-degrees, steps, and the visited-bit atomics of the partner edges
    uint32_t outdeg[BFS_NPT], step[BFS_NPT], tgt[BFS_NPT][BFS_S], old[BFS_NPT][BFS_S];
    uint32_t tvalid[BFS_NPT];
#pragma unroll
    for (int r = 0; r < BFS_NPT; r++) {
        outdeg[r] = 0;
        step[r] = 0;
        tvalid[r] = 0;
        const Grid g = geo.grid(geo.field_of(e[r] >> 3));
#pragma unroll
        for (int j = 0; j < BFS_S; j++) {
            tgt[r][j] = 0;
            old[r][j] = 0;
            if (!((qvalid[r] >> j) & 1u)) continue;
            const uint32_t qw = qc[r][j] >> 3, qk = qc[r][j] & 7u;
            const uint32_t nq = nib_of(qword[r][j], qk);
            if (nq >= NB_CRIT) {  // a 2-saddle
                outdeg[r]++;
                step[r] = (uint32_t)j | (nq << 3);
                continue;
            }
            CellRef e2;
            if (!quad_edge_partner(g, qw, qk, nq, e2)) continue;  // paired with a cube
            outdeg[r]++;
            step[r] = (uint32_t)j | (nq << 3);
            tgt[r][j] = 8u * e2.w + e2.k;
            tvalid[r] |= 1u << j;
        }
    }
#pragma unroll
    for (int r = 0; r < BFS_NPT; r++)
#pragma unroll
        for (int j = 0; j < BFS_S; j++)
            if ((tvalid[r] >> j) & 1u) old[r][j] = atomicOr(&vis[tgt[r][j] >> 5], 1u << (tgt[r][j] & 31u));
    // phase 4: new targets, junction and label decisions
    uint32_t fresh[BFS_NPT];  // bit j: the target of slot j is new
    uint32_t nt[BFS_NPT], isj[BFS_NPT], lab[BFS_NPT];
    uint32_t snt = 0, sj = 0;
#pragma unroll
    for (int r = 0; r < BFS_NPT; r++) {
        fresh[r] = 0;
#pragma unroll
        for (int j = 0; j < BFS_S; j++)
            if (((tvalid[r] >> j) & 1u) && !(old[r][j] & (1u << (tgt[r][j] & 31u)))) fresh[r] |= 1u << j;
        nt[r] = (uint32_t)__builtin_popcount(fresh[r]);
        isj[r] = (ok[r] && !level0 && outdeg[r] > 1) ? 1u : 0u;
        lab[r] = level0 ? 0u : (outdeg[r] == 1 ? (SUCC_FLAG | step[r]) : NOT_JUNCTION);
        if (!ok[r] || level0) e[r] = 0xFFFFFFFFu;  // 1-saddles take no label
        snt += nt[r];
        sj += isj[r];
    }
    unsigned long long packed = (unsigned long long)snt | ((unsigned long long)sj << 32);
    unsigned long long tot;
    unsigned long long ex = block_excl_scan<unsigned long long, BT>(packed, sc, tot);
    if (threadIdx.x == 0) base = tot ? atomicAdd(tail, tot) : 0ull;
    __syncthreads();
    uint64_t o = (base & 0xFFFFFFFFull) + (ex & 0xFFFFFFFFull);
#pragma unroll
    for (int r = 0; r < BFS_NPT; r++) {
#pragma unroll
        for (int j = 0; j < BFS_S; j++)
            if ((fresh[r] >> j) & 1u) {
                if (o < qcap) queue[o] = tgt[r][j];  // never full: a node enters once (the host checks the tail)
                o++;
            }
        // a junction is marked with id 0 here; junctions are numbered in
        // cell order once the search is complete
        if (e[r] != 0xFFFFFFFFu) label[label_slot(e[r] >> 3, e[r] & 7u, geo.nv)] = isj[r] ? 0u : lab[r];
    }
    __syncthreads();  // base is rewritten by the next chunk
    }
}

// Junction numbering in cell order, so that the sources of the DAG minor
// (1-saddles, then junctions) are both in cell order and the tracing from
// neighbouring sources shares cache lines.  A junction is a visited edge
// (every visited cell is a non-critical edge) whose label is below
// SUCC_FLAG.  One thread per word of the visited bits (4 vertices, 12 edge
// cells, all their label loads issued together); k_junc_count counts per
// workgroup, k_junc_emit (with the counts scanned) writes jlist and the
// final ids.
constexpr uint32_t JVPT = 4;  // vertices per thread (one visited word)

// bit 3 * v + (slot of k) for vertex 4 * t + v and edge type k = 1, 2, 4
__device__ __forceinline__ uint32_t junction_bits(const uint32_t* __restrict__ vis,
                                                  const uint32_t* __restrict__ label, uint32_t nv, uint32_t t) {
    const uint32_t vw = vis[t];
    uint32_t lab[JVPT][3];
#pragma unroll
    for (uint32_t v = 0; v < JVPT; v++) {
        const uint32_t w = JVPT * t + v;
#pragma unroll
        for (uint32_t q = 0; q < 3; q++) {
            const uint32_t k = 1u << q;
            lab[v][q] = w < nv && ((vw >> (8u * v + k)) & 1u) ? label[label_slot(w, k, nv)] : SUCC_FLAG;
        }
    }
    uint32_t m = 0;
#pragma unroll
    for (uint32_t v = 0; v < JVPT; v++)
#pragma unroll
        for (uint32_t q = 0; q < 3; q++)
            if (lab[v][q] < SUCC_FLAG) m |= 1u << (3u * v + q);
    return m;
}

__global__ __launch_bounds__(BT) void k_junc_count(const uint32_t* __restrict__ vis, const uint32_t* __restrict__ label,
                                                   uint32_t nv, uint64_t* __restrict__ bcount) {
    __shared__ uint32_t sc[BT / WAVE + 1];
    const uint64_t t = (uint64_t)blockIdx.x * BT + threadIdx.x;
    const uint32_t c = JVPT * t < nv ? (uint32_t)__popc(junction_bits(vis, label, nv, (uint32_t)t)) : 0u;
    uint32_t tot;
    block_excl_scan<uint32_t, BT>(c, sc, tot);
    if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}

__global__ __launch_bounds__(BT) void k_junc_emit(const uint32_t* __restrict__ vis, uint32_t* __restrict__ label,
                                                  uint32_t nv, const uint64_t* __restrict__ boff,
                                                  uint32_t* __restrict__ jlist) {
    __shared__ uint32_t sc[BT / WAVE + 1];
    const uint64_t t = (uint64_t)blockIdx.x * BT + threadIdx.x;
    const uint32_t m = JVPT * t < nv ? junction_bits(vis, label, nv, (uint32_t)t) : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t, BT>((uint32_t)__popc(m), sc, tot);
    uint64_t pos = boff[blockIdx.x] + ex;
#pragma unroll
    for (uint32_t v = 0; v < JVPT; v++) {
#pragma unroll
        for (uint32_t q = 0; q < 3; q++) {
            if ((m >> (3u * v + q)) & 1u) {
                const uint32_t w = JVPT * (uint32_t)t + v, k = 1u << q;
                jlist[pos] = 8u * w + k;
                label[label_slot(w, k, nv)] = (uint32_t)pos;
                pos++;
            }
        }
    }
}

// Trace the simple path leaving source `src` through its out-edge `slot`.
// Each thread walks MT_W of a source's out-edge slots (slots MT_W h ..
// MT_W h + MT_W - 1 for its h) in lockstep, one step of every live walk per
// iteration, so that the walks' label loads would be in flight together; a
// walk is a chain of dependent loads, one per step.  At 512^3 one walk per
// thread measured as fast as two (the resident waves already cover the
// latency) and faster than four (longer divergent tails).
constexpr int MT_W = 1;

__global__ __launch_bounds__(BT) void k_minor_trace(const uint32_t* __restrict__ s1, uint64_t S1,
                                                    const uint32_t* __restrict__ jlist, uint64_t J,
                                                    const uint32_t* __restrict__ grad, Geo geo,
                                                    const uint32_t* __restrict__ label, uint64_t max_steps,
                                                    uint64_t S2, uint8_t* __restrict__ out_t,
                                                    uint32_t* __restrict__ out_id, int* __restrict__ err) {
    const uint64_t t = (uint64_t)blockIdx.x * BT + threadIdx.x;
    const uint64_t si = t / (4 / MT_W);
    if (si >= S1 + J) return;
    const uint32_t slot0 = (uint32_t)(t % (4 / MT_W)) * MT_W;
    const uint32_t e = si < S1 ? s1[si] : jlist[si - S1];
    const uint32_t w = e >> 3, k = e & 7u;
    const uint32_t a = (uint32_t)__builtin_ctz(k);
    // a path never leaves the field it starts in
    const uint32_t fld = geo.field_of(w);
    const Grid g = geo.grid(fld);
    const uint32_t fbase = geo.base(fld);
    uint32_t c[3];
    g.coords(w - fbase, c);
    CellRef v;
    const bool hv = paired_quad(g, w, k, nib_of(grad[w], k), c, a, v);
    const uint32_t b0 = a == 0 ? 1u : 0u, b1 = a == 2 ? 1u : 2u;
    uint32_t qw[MT_W], qk[MT_W], nq[MT_W], id[MT_W];
    uint8_t typ[MT_W];
    uint32_t live = 0;  // bit j: walk j still going
#pragma unroll
    for (int j = 0; j < MT_W; j++) {
        const uint32_t slot = slot0 + (uint32_t)j;
        const uint32_t b = (slot >> 1) ? b1 : b0;
        const int s = (slot & 1u) ? 1 : -1;
        typ[j] = T_NONE;
        id[j] = 0;
        CellRef q;
        q.w = q.k = 0;
        if (cell_step(g, w, k, c, (int)b, s, q.w, q.k) && !(hv && q.w == v.w && q.k == v.k)) live |= 1u << j;
        qw[j] = q.w;
        qk[j] = q.k;
    }
#pragma unroll
    for (int j = 0; j < MT_W; j++) nq[j] = ((live >> j) & 1u) ? nib_of(grad[qw[j]], qk[j]) : 0u;
    for (uint64_t step = 0; live; step++) {
        if (step > max_steps) {
            atomicOr(err, 8);
            break;
        }
        // the label each live walk needs: its 2-saddle's, or its quad's partner edge's
        uint32_t ew[MT_W], ek[MT_W];
#pragma unroll
        for (int j = 0; j < MT_W; j++) {
            ew[j] = ek[j] = 0;
            if (!((live >> j) & 1u)) continue;
            if (nq[j] >= NB_CRIT) continue;  // the label of the quad itself
            CellRef e2;
            if (!quad_edge_partner(g, qw[j], qk[j], nq[j], e2)) {  // paired with a cube: dead end
                live &= ~(1u << j);
                continue;
            }
            ew[j] = e2.w;
            ek[j] = e2.k;
        }
        uint32_t lab[MT_W];
#pragma unroll
        for (int j = 0; j < MT_W; j++) {
            lab[j] = 0;
            if (!((live >> j) & 1u)) continue;
            lab[j] = nq[j] >= NB_CRIT ? label[label_slot(qw[j], qk[j], geo.nv)]
                                      : label[label_slot(ew[j], ek[j], geo.nv)];
        }
#pragma unroll
        for (int j = 0; j < MT_W; j++) {
            if (!((live >> j) & 1u)) continue;
            if (nq[j] >= NB_CRIT) {
                typ[j] = T_S2;
                id[j] = lab[j];
                live &= ~(1u << j);
                continue;
            }
            if (!(lab[j] & SUCC_FLAG)) {
                typ[j] = T_JUNC;
                id[j] = lab[j];
                live &= ~(1u << j);
                continue;
            }
            if (lab[j] == NOT_JUNCTION) {  // no out-edge: dead end
                live &= ~(1u << j);
                continue;
            }
            // the edge has exactly one out-edge; its step was recorded by the BFS
            uint32_t c2[3];
            g.coords(ew[j] - fbase, c2);
            const uint32_t st = lab[j] & 7u;
            if (!cell_step(g, ew[j], ek[j], c2, (int)(st >> 1), (st & 1u) ? 1 : -1, qw[j], qk[j])) {
                atomicOr(err, 16);
                live &= ~(1u << j);
                continue;
            }
            nq[j] = (lab[j] >> 3) & 15u;
        }
    }
#pragma unroll
    for (int j = 0; j < MT_W; j++) {
        if ((typ[j] == T_S2 && id[j] >= S2) || (typ[j] == T_JUNC && id[j] >= J)) {
            atomicOr(err, 16);  // a label that was never assigned
            typ[j] = T_NONE;
        }
        out_t[4 * si + slot0 + j] = typ[j];
        out_id[4 * si + slot0 + j] = id[j];
    }
}

// Per source: distinct junction targets and distinct 2-saddle targets with
// multiplicities (at most four paths leave a source).
template <bool FILL>
__global__ __launch_bounds__(BT) void k_minor_rows(const uint8_t* __restrict__ out_t,
                                                   const uint32_t* __restrict__ out_id, uint64_t S1, uint64_t NS,
                                                   uint32_t* __restrict__ cj, uint32_t* __restrict__ cs,
                                                   const uint64_t* __restrict__ rpA, uint32_t* __restrict__ colA,
                                                   uint64_t* __restrict__ valA, const uint64_t* __restrict__ rpD,
                                                   uint32_t* __restrict__ colD, uint64_t* __restrict__ valD,
                                                   const uint64_t* __restrict__ rpB, uint32_t* __restrict__ colB,
                                                   uint64_t* __restrict__ valB, const uint64_t* __restrict__ rpBs,
                                                   uint32_t* __restrict__ colBs, uint64_t* __restrict__ valBs) {
    uint64_t i = (uint64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= NS) return;
    // the four slots of source i: one 4-byte and one 16-byte load
    const uint32_t t4 = ((const uint32_t*)out_t)[i];
    const uint4 id4 = ((const uint4*)out_id)[i];
    const uint32_t ids[4] = {id4.x, id4.y, id4.z, id4.w};
    // keys (type, id), empty slots last, sorted by a five-comparator network:
    // equal targets become runs, junction targets precede 2-saddle targets,
    // and ids ascend within each
    uint64_t kk[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t t = (t4 >> (8 * q)) & 0xffu;
        kk[q] = t == T_NONE ? ~0ull : ((uint64_t)t << 32) | ids[q];
    }
    auto cswap = [&](int x, int y) {
        const uint64_t lo = kk[x] < kk[y] ? kk[x] : kk[y];
        const uint64_t hi = kk[x] < kk[y] ? kk[y] : kk[x];
        kk[x] = lo;
        kk[y] = hi;
    };
    cswap(0, 1);
    cswap(2, 3);
    cswap(0, 2);
    cswap(1, 3);
    cswap(1, 2);
    uint32_t nj = 0, ns = 0;
    uint32_t *cJ = nullptr, *cS = nullptr;
    uint64_t *vJ = nullptr, *vS = nullptr;
    uint64_t oJ = 0, oS = 0;
    if (FILL) {
        if (i < S1) {
            cJ = colA; vJ = valA; oJ = rpA[i];
            cS = colD; vS = valD; oS = rpD[i];
        } else {
            cJ = colB; vJ = valB; oJ = rpB[i - S1];
            cS = colBs; vS = valBs; oS = rpBs[i - S1];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (kk[q] == ~0ull || (q > 0 && kk[q] == kk[q - 1])) continue;  // empty, or not a run's first
        uint64_t m = 0;
#pragma unroll
        for (int r = q; r < 4; r++) m += kk[r] == kk[q] ? 1u : 0u;
        const uint32_t id = (uint32_t)kk[q];
        if ((uint32_t)(kk[q] >> 32) == T_JUNC) {
            if (FILL) {
                cJ[oJ + nj] = id;
                vJ[oJ + nj] = m;
            }
            nj++;
        } else {
            if (FILL) {
                cS[oS + ns] = id;
                vS[oS + ns] = m;
            }
            ns++;
        }
    }
    if (!FILL) {
        cj[i] = nj;
        cs[i] = ns;
    }
}

}  // namespace

hipError_t launch_bfs_level(uint32_t* queue, uint64_t qcap, uint64_t* lv, uint64_t L, const uint32_t* grad,
                            const Geo& g, uint32_t* vis, unsigned long long* tail, uint32_t* label, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_seal, dim3(1), dim3(WAVE), 0, s, lv, L, (const unsigned long long*)tail);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bfs_expand, dim3(BFS_GRID), dim3(BT), 0, s, queue, qcap, (const uint64_t*)lv, L, grad, g,
                       vis, tail, label);
    return hipGetLastError();
}

size_t junction_blocks(uint64_t nv) { return (size_t)((nv + (uint64_t)BT * JVPT - 1) / ((uint64_t)BT * JVPT)); }

hipError_t launch_junc_count(const uint32_t* vis, const uint32_t* label, uint64_t nv, uint64_t* bcount,
                             hipStream_t s) {
    if (nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_junc_count, dim3((unsigned)junction_blocks(nv)), dim3(BT), 0, s, vis, label, (uint32_t)nv,
                       bcount);
    return hipGetLastError();
}

hipError_t launch_junc_emit(const uint32_t* vis, uint32_t* label, uint64_t nv, const uint64_t* boff, uint32_t* jlist,
                            hipStream_t s) {
    if (nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_junc_emit, dim3((unsigned)junction_blocks(nv)), dim3(BT), 0, s, vis, label, (uint32_t)nv,
                       boff, jlist);
    return hipGetLastError();
}

hipError_t launch_minor_trace(const uint32_t* s1, uint64_t S1, const uint32_t* jlist, uint64_t J, const uint32_t* grad,
                              const Geo& g, const uint32_t* label, uint64_t max_steps, uint64_t S2, uint8_t* out_t,
                              uint32_t* out_id, int* err, hipStream_t s) {
    uint64_t threads = (4 / MT_W) * (S1 + J);
    if (threads == 0) return hipSuccess;
    hipLaunchKernelGGL(k_minor_trace, dim3(grid_blocks(threads, BT)), dim3(BT), 0, s, s1, S1, jlist, J, grad, g,
                       label, max_steps, S2, out_t, out_id, err);
    return hipGetLastError();
}

hipError_t launch_minor_rows(bool fill, const uint8_t* out_t, const uint32_t* out_id, uint64_t S1, uint64_t NS,
                             uint32_t* cj, uint32_t* cs, const uint64_t* rpA, uint32_t* colA, uint64_t* valA,
                             const uint64_t* rpD, uint32_t* colD, uint64_t* valD, const uint64_t* rpB, uint32_t* colB,
                             uint64_t* valB, const uint64_t* rpBs, uint32_t* colBs, uint64_t* valBs, hipStream_t s) {
    if (NS == 0) return hipSuccess;
    if (fill)
        hipLaunchKernelGGL(k_minor_rows<true>, dim3(grid_blocks(NS, BT)), dim3(BT), 0, s, out_t, out_id, S1, NS, cj, cs,
                           rpA, colA, valA, rpD, colD, valD, rpB, colB, valB, rpBs, colBs, valBs);
    else
        hipLaunchKernelGGL(k_minor_rows<false>, dim3(grid_blocks(NS, BT)), dim3(BT), 0, s, out_t, out_id, S1, NS, cj,
                           cs, rpA, colA, valA, rpD, colD, valD, rpB, colB, valB, rpBs, colBs, valBs);
    return hipGetLastError();
}

}  // namespace msc

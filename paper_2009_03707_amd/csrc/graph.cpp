// Host MS-complex graph and persistence-driven simplification.
//
// Graph (Section 3.5, "Data structure"): a vector of critical points and,
// per critical point, its arcs in each direction (down to index - 1, up to
// index + 1) with their multiplicities; every arc is stored twice, once at
// each end.  The lists of the nodes are filled in parallel, one worker per
// range of nodes and direction, from the CSR (down) and transposed (up) arc
// matrices of a result.
//
// Simplification (Section 2.1 and Section 4): cancellation of a critical
// pair (p, q), index(p) = index(q) + 1, joined by exactly one gradient path
// (arc multiplicity 1; more paths would strangle), in order of persistence
// |f(p) - f(q)|.  Cancelling reroutes the descending arcs of p to the
// destinations of the ascending arcs of q: for every other upper neighbour s
// of q and every other lower neighbour r of p, the arc s -> r gains
// m(s, q) * m(p, r) paths (saturating u64); p, q and their arcs are deleted
// (lazily: lists keep entries of dead nodes, which every reader skips).
//   serial  : repeatedly cancel the valid arc of least (persistence, upper
//             node, lower node) below the threshold (a priority queue with
//             lazy validation);
//   subgrid : the paper's subdivision schedule.  The grid is sliced into k
//             slabs along X, then Y, then Z, then again with the slab
//             boundaries shifted by half a slab; in each round the nodes on
//             arcs that cross a slab boundary are frozen, and the slabs are
//             simplified at once, one thread each, each in serial order over
//             its own arcs between unfrozen nodes (new arcs with a frozen end
//             are not queued).  A cancellation touches only its pair and the
//             pair's neighbours, which all lie in the pair's slab, so the
//             threads never touch the same node and their cancellations
//             commute.  A final serial round cancels what is left.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <queue>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "graph.h"

namespace {

struct Arc {
    int64_t nbr;
    uint64_t mult;
};

uint64_t sat_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s < a ? ~0ull : s;
}
uint64_t sat_mul(uint64_t a, uint64_t b) {
    unsigned __int128 p = (unsigned __int128)a * b;
    return (p >> 64) ? ~0ull : (uint64_t)p;
}

template <typename F>
void parallel_for(int64_t n, int nthreads, F&& fn) {
    if (nthreads <= 1 || n < 4096) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t per = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; t++) {
        int64_t a = (int64_t)t * per, b = std::min(n, a + per);
        if (a >= b) break;
        th.emplace_back([&fn, a, b] { fn(a, b); });
    }
    for (auto& x : th) x.join();
}

struct Cand {
    double pers;
    int64_t upper, lower;
    bool operator>(const Cand& o) const {
        return std::tie(pers, upper, lower) > std::tie(o.pers, o.upper, o.lower);
    }
};
using MinQueue = std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>>;

}  // namespace

struct ms_graph {
    int64_t dims[3] = {0, 0, 0};
    int64_t count[4] = {0, 0, 0, 0};
    int64_t first[5] = {0, 0, 0, 0, 0};  // first node of each index
    std::vector<uint32_t> cell, vmax;
    std::vector<uint8_t> index, alive;
    std::vector<float> value;
    std::vector<std::vector<Arc>> down, up;  // sorted by neighbour node
    std::vector<ms_cancellation> log;
    std::string err;

    int64_t n() const { return (int64_t)cell.size(); }
    double pers(int64_t a, int64_t b) const { return fabs((double)value[a] - (double)value[b]); }

    static const Arc* find(const std::vector<Arc>& v, int64_t nbr) {
        auto it = std::lower_bound(v.begin(), v.end(), nbr, [](const Arc& a, int64_t x) { return a.nbr < x; });
        return (it != v.end() && it->nbr == nbr) ? &*it : nullptr;
    }
    static uint64_t add(std::vector<Arc>& v, int64_t nbr, uint64_t m) {
        auto it = std::lower_bound(v.begin(), v.end(), nbr, [](const Arc& a, int64_t x) { return a.nbr < x; });
        if (it != v.end() && it->nbr == nbr) {
            it->mult = sat_add(it->mult, m);
            return it->mult;
        }
        v.insert(it, Arc{nbr, m});
        return m;
    }
    uint64_t mult(int64_t upper, int64_t lower) const {
        const Arc* a = find(down[upper], lower);
        return a ? a->mult : 0;
    }

    // Cancels (u, l); appends the arcs it creates or changes to `touched`
    // (U and D: the caller's scratch lists).
    void cancel(int64_t u, int64_t l, std::vector<std::pair<int64_t, int64_t>>& touched,
                std::vector<ms_cancellation>& out, std::vector<Arc>& U, std::vector<Arc>& D) {
        U.clear();
        D.clear();
        for (const Arc& a : up[l])
            if (alive[a.nbr] && a.nbr != u) U.push_back(a);
        for (const Arc& a : down[u])
            if (alive[a.nbr] && a.nbr != l) D.push_back(a);
        for (const Arc& s : U)
            for (const Arc& r : D) {
                uint64_t m = sat_mul(s.mult, r.mult);
                add(down[s.nbr], r.nbr, m);
                add(up[r.nbr], s.nbr, m);
                touched.emplace_back(s.nbr, r.nbr);
            }
        alive[u] = 0;
        alive[l] = 0;
        out.push_back(ms_cancellation{u, l, pers(u, l)});
    }

    // Serial persistence-ordered cancellation restricted to the nodes for
    // which `in(node)` holds.  Candidates are the live arcs of multiplicity
    // 1 below the threshold; they come from `seeds` (or, without seeds, from
    // every node's descending arcs) and from the arcs each cancellation
    // creates or changes.  A candidate with an end outside `in` is appended
    // to `deferred` (when given) instead of being queued.  A candidate that
    // fails otherwise can never become one again: persistence is fixed, dead
    // nodes stay dead and multiplicities only grow.
    template <typename In>
    void run_serial(double thr, In&& in, std::vector<ms_cancellation>& out,
                    const std::vector<std::pair<int64_t, int64_t>>* seeds,
                    std::vector<std::pair<int64_t, int64_t>>* deferred) {
        MinQueue q;
        auto consider = [&](int64_t u, int64_t l) {
            if (!alive[u] || !alive[l]) return;
            double p = pers(u, l);
            if (!(p < thr)) return;
            if (mult(u, l) != 1) return;
            if (!in(u) || !in(l)) {
                if (deferred) deferred->emplace_back(u, l);
                return;
            }
            q.push(Cand{p, u, l});
        };
        if (seeds) {
            for (const auto& c : *seeds) consider(c.first, c.second);
        } else {
            for (int64_t u = 0; u < n(); u++) {
                if (index[u] == 0 || !alive[u]) continue;
                for (const Arc& a : down[u])
                    if (a.mult == 1) consider(u, a.nbr);
            }
        }
        std::vector<std::pair<int64_t, int64_t>> touched;
        std::vector<Arc> U, D;
        while (!q.empty()) {
            Cand c = q.top();
            q.pop();
            if (!alive[c.upper] || !alive[c.lower] || mult(c.upper, c.lower) != 1) continue;
            touched.clear();
            cancel(c.upper, c.lower, touched, out, U, D);
            for (auto& t : touched) consider(t.first, t.second);
        }
    }

    // refined coordinate of a node's cell along `axis`
    int64_t coord(int64_t node, int axis) const {
        uint64_t w = cell[node] >> 3, k = cell[node] & 7u;
        uint64_t x = w % (uint64_t)dims[0], y = (w / (uint64_t)dims[0]) % (uint64_t)dims[1],
                 z = w / ((uint64_t)dims[0] * (uint64_t)dims[1]);
        uint64_t c = axis == 0 ? x : (axis == 1 ? y : z);
        return (int64_t)(2 * c + ((k >> axis) & 1u));
    }

    // The candidates of the whole graph: its live arcs of multiplicity 1
    // below the threshold, gathered in parallel.
    std::vector<std::pair<int64_t, int64_t>> candidates(double thr, int nthreads) const {
        const int64_t N = n();
        const int nt = nthreads < 1 ? 1 : nthreads;
        std::vector<std::vector<std::pair<int64_t, int64_t>>> part(nt);
        const int64_t per = (N + nt - 1) / nt;
        std::vector<std::thread> th;
        for (int t = 0; t < nt; t++)
            th.emplace_back([&, t] {
                const int64_t a = (int64_t)t * per, b = std::min(N, a + per);
                for (int64_t u = a; u < b; u++) {
                    if (index[u] == 0 || !alive[u]) continue;
                    for (const Arc& x : down[u])
                        if (x.mult == 1 && alive[x.nbr] && pers(u, x.nbr) < thr) part[t].emplace_back(u, x.nbr);
                }
            });
        for (auto& x : th) x.join();
        std::vector<std::pair<int64_t, int64_t>> all;
        for (auto& p : part) all.insert(all.end(), p.begin(), p.end());
        return all;
    }

    // Rounds of the subdivision schedule.  Only candidates are carried from
    // round to round (the pool): a round hands every pooled candidate whose
    // ends lie unfrozen in one slab to that slab's thread, keeps the others,
    // and takes back what the threads deferred -- so no round rescans the
    // graph, and the final serial round starts from the pool.  A node's slab
    // follows from its cell; whether it is frozen (a live arc to another
    // slab at the start of the round) is worked out when first asked, from
    // a copy of the live flags taken at the start of the round.  That gives
    // the same answer whenever it is asked: a thread only ever changes the
    // arc lists of nodes in its own slab (the neighbours of an unfrozen pair
    // share its slab), and the arcs it adds join nodes of that slab.
    void run_subgrid(double thr, int k, int nthreads) {
        const int64_t N = n();
        std::vector<uint8_t> snap(N), fz(N);  // fz: 0 not yet known, 1 unfrozen, 2 frozen
        std::vector<std::pair<int64_t, int64_t>> pool = candidates(thr, nthreads);
        std::vector<uint32_t> rc[3];  // refined coordinates of the nodes' cells
        for (int axis = 0; axis < 3; axis++) {
            rc[axis].resize(N);
            parallel_for(N, nthreads, [&](int64_t a, int64_t b) {
                for (int64_t i = a; i < b; i++) rc[axis][i] = (uint32_t)coord(i, axis);
            });
        }
        std::vector<int32_t> slab_of;  // slab of each refined coordinate along the round's axis
        for (int pass = 0; pass < 2; pass++)
            for (int axis = 0; axis < 3; axis++) {
                const int64_t len = 2 * dims[axis] - 1;
                if (len < 2 * k) continue;  // too thin to slice
                if (pool.empty()) break;
                const int64_t off = pass == 0 ? 0 : len / (2 * k);
                slab_of.resize((size_t)len);
                for (int64_t c = 0; c < len; c++) slab_of[c] = (int32_t)(((c - off + len) % len) * k / len);
                const uint32_t* rca = rc[axis].data();
                const int32_t* so = slab_of.data();
                auto sub = [rca, so](int64_t x) -> int32_t { return so[rca[x]]; };
                auto frozen = [&](int64_t x) -> bool {
                    uint8_t& f = fz[x];
                    if (f) return f == 2;
                    const int32_t sx = sub(x);
                    bool z = false;
                    for (const Arc& a : down[x])
                        if (snap[a.nbr] && sub(a.nbr) != sx) {
                            z = true;
                            break;
                        }
                    if (!z)
                        for (const Arc& a : up[x])
                            if (snap[a.nbr] && sub(a.nbr) != sx) {
                                z = true;
                                break;
                            }
                    f = z ? 2 : 1;
                    return z;
                };
                memcpy(snap.data(), alive.data(), (size_t)N);
                memset(fz.data(), 0, (size_t)N);
                std::vector<std::vector<std::pair<int64_t, int64_t>>> seeds(k), deferred(k);
                std::vector<std::pair<int64_t, int64_t>> kept;
                for (const auto& c : pool) {
                    const int64_t u = c.first, l = c.second;
                    if (!alive[u] || !alive[l]) continue;
                    const int32_t su = sub(u);
                    if (su == sub(l) && !frozen(u) && !frozen(l)) seeds[su].push_back(c);
                    else kept.push_back(c);
                }
                std::vector<std::vector<ms_cancellation>> logs(k);
                std::vector<std::thread> th;
                for (int s = 0; s < k; s++) {
                    if (seeds[s].empty()) continue;
                    th.emplace_back([&, s] {
                        run_serial(
                            thr, [&](int64_t x) { return sub(x) == s && !frozen(x); }, logs[s], &seeds[s],
                            &deferred[s]);
                    });
                }
                for (auto& t : th) t.join();
                for (auto& l : logs) log.insert(log.end(), l.begin(), l.end());
                pool.swap(kept);
                for (auto& d : deferred) pool.insert(pool.end(), d.begin(), d.end());
            }
        run_serial(thr, [](int64_t) { return true; }, log, &pool, nullptr);
    }
};

namespace msc {

ms_graph* graph_from_host(GraphInput& in, int nthreads, std::string* err) {
    ms_graph* g = new (std::nothrow) ms_graph();
    if (!g) {
        *err = "host allocation failed";
        return nullptr;
    }
    try {
        for (int a = 0; a < 3; a++) g->dims[a] = in.dims[a];
        int64_t tot = 0;
        for (int k = 0; k < 4; k++) {
            g->count[k] = in.count[k];
            g->first[k] = tot;
            tot += in.count[k];
        }
        g->first[4] = tot;
        if ((int64_t)in.id.size() != tot || (int64_t)in.index.size() != tot || (int64_t)in.value.size() != tot ||
            (int64_t)in.vmax.size() != tot) {
            *err = "critical list size differs from the counts";
            delete g;
            return nullptr;
        }
        g->cell = std::move(in.id);
        g->vmax = std::move(in.vmax);
        g->index = std::move(in.index);
        g->value = std::move(in.value);
        g->alive.assign(tot, 1);
        g->down.resize(tot);
        g->up.resize(tot);
        // (matrix, index of its row nodes, index of its column nodes, lists filled)
        struct Src {
            const HostCsr* m;
            int ri, ci;
            bool down;
        };
        const Src srcs[6] = {{&in.m10, 1, 0, true},  {&in.m10t, 0, 1, false}, {&in.m21, 2, 1, true},
                             {&in.m21t, 1, 2, false}, {&in.m32, 3, 2, true},  {&in.m32t, 2, 3, false}};
        for (const Src& s : srcs) {
            if (s.m->nrows != in.count[s.ri] || s.m->ncols != in.count[s.ci] ||
                (int64_t)s.m->rowptr.size() != s.m->nrows + 1) {
                *err = "arc matrix shape differs from the critical counts";
                delete g;
                return nullptr;
            }
        }
        for (const Src& s : srcs) {
            const HostCsr& m = *s.m;
            const int64_t r0 = g->first[s.ri], c0 = g->first[s.ci];
            auto& lists = s.down ? g->down : g->up;
            parallel_for(m.nrows, nthreads, [&](int64_t a, int64_t b) {
                for (int64_t r = a; r < b; r++) {
                    auto& v = lists[r0 + r];
                    v.reserve((size_t)(m.rowptr[r + 1] - m.rowptr[r]));
                    for (int64_t p = m.rowptr[r]; p < m.rowptr[r + 1]; p++)
                        v.push_back(Arc{c0 + (int64_t)m.col[p], m.val[p]});
                }
            });
        }
    } catch (const std::exception& e) {
        *err = std::string("graph construction failed: ") + e.what();
        delete g;
        return nullptr;
    }
    return g;
}

}  // namespace msc

extern "C" {

void ms_graph_destroy(ms_graph* g) { delete g; }

int64_t ms_graph_num_nodes(const ms_graph* g) { return g ? g->n() : 0; }

const char* ms_graph_last_error(const ms_graph* g) { return g ? g->err.c_str() : "null graph"; }

ms_status ms_graph_node(const ms_graph* g, int64_t node, ms_node* out) {
    if (!g || !out || node < 0 || node >= g->n()) return MS_ERR_INVALID_ARG;
    out->cell = g->cell[node];
    out->index = g->index[node];
    out->alive = g->alive[node];
    out->value = g->value[node];
    out->vmax = g->vmax[node];
    return MS_OK;
}

ms_status ms_graph_find(const ms_graph* g, uint32_t cell, int64_t* node) {
    if (!g || !node) return MS_ERR_INVALID_ARG;
    const int k = __builtin_popcount(cell & 7u);
    auto b = g->cell.begin() + g->first[k], e = g->cell.begin() + g->first[k + 1];
    auto it = std::lower_bound(b, e, cell);
    if (it == e || *it != cell) return MS_ERR_INVALID_ARG;
    *node = (int64_t)(it - g->cell.begin());
    return MS_OK;
}

ms_status ms_graph_arcs(const ms_graph* g, int64_t node, int dir, int64_t* nbr, uint64_t* mult, int64_t cap,
                        int64_t* count) {
    if (!g || !count || node < 0 || node >= g->n() || (dir != MS_DOWN && dir != MS_UP) || cap < 0 ||
        (cap > 0 && (!nbr || !mult)))
        return MS_ERR_INVALID_ARG;
    int64_t n = 0;
    if (g->alive[node]) {
        for (const Arc& a : (dir == MS_DOWN ? g->down[node] : g->up[node])) {
            if (!g->alive[a.nbr]) continue;
            if (n < cap) {
                nbr[n] = a.nbr;
                mult[n] = a.mult;
            }
            n++;
        }
    }
    *count = n;
    return n > cap ? MS_ERR_CAPACITY : MS_OK;
}

ms_status ms_graph_counts(const ms_graph* g, int64_t alive[4], int64_t arcs[3]) {
    if (!g || !alive || !arcs) return MS_ERR_INVALID_ARG;
    for (int k = 0; k < 4; k++) alive[k] = 0;
    for (int k = 0; k < 3; k++) arcs[k] = 0;
    for (int64_t i = 0; i < g->n(); i++) {
        if (!g->alive[i]) continue;
        alive[g->index[i]]++;
        if (g->index[i] == 0) continue;
        for (const Arc& a : g->down[i])
            if (g->alive[a.nbr]) arcs[g->index[i] - 1]++;
    }
    return MS_OK;
}

ms_status ms_graph_simplify(ms_graph* g, double threshold, int schedule, int nthreads, int64_t* ncancelled) {
    if (!g || (schedule != MS_SIMPLIFY_SERIAL && schedule != MS_SIMPLIFY_SUBGRID) || nthreads < 1 ||
        nthreads > 1024 || threshold != threshold)
        return MS_ERR_INVALID_ARG;
    const size_t before = g->log.size();
    try {
        if (schedule == MS_SIMPLIFY_SERIAL || nthreads == 1)
            g->run_serial(threshold, [](int64_t) { return true; }, g->log, nullptr, nullptr);
        else
            g->run_subgrid(threshold, nthreads, nthreads);
    } catch (const std::exception& e) {
        g->err = std::string("simplification failed: ") + e.what();
        return MS_ERR_INTERNAL;
    }
    if (ncancelled) *ncancelled = (int64_t)(g->log.size() - before);
    return MS_OK;
}

int64_t ms_graph_num_cancellations(const ms_graph* g) { return g ? (int64_t)g->log.size() : 0; }

ms_status ms_graph_cancellations(const ms_graph* g, int64_t first, int64_t n, ms_cancellation* out) {
    if (!g || first < 0 || n < 0 || first + n > (int64_t)g->log.size() || (n > 0 && !out)) return MS_ERR_INVALID_ARG;
    if (n > 0) memcpy(out, g->log.data() + first, sizeof(ms_cancellation) * (size_t)n);
    return MS_OK;
}

}  // extern "C"

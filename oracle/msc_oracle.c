/*
 * msc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, deliberately unoptimised CPU implementation of what the
 * Morse-Smale hot path computes.  It exists so that tests, the smoke check
 * and the benchmark's CPU-baseline leg can compare the GPU library against an
 * independent, readable statement of the method.  Nothing in the product
 * path may link, import or call it, and it shares no code, header, table or
 * helper with the GPU library.
 *
 * What it follows (Subhash, Pandey, Natarajan, "A GPU Parallel Algorithm for
 * Computing Morse-Smale Complexes"):
 *   - discrete gradient, critical cells, V-paths: Section 2.2 (definitions of
 *     gradient pair, critical cell, index, V-path);
 *   - gradient rule: the per-vertex lower-star pairing of Robins, Wood and
 *     Sheppard (2011), which the paper cites for locally independent gradient
 *     assignment (Section 1.1) and uses in its first step (Section 3);
 *   - saddle-extremum arcs: root finding along (0,1) and (2,3) V-paths, which
 *     split or merge but never both (Section 3.4);
 *   - 1-saddle/2-saddle arcs: the number of gradient paths between each
 *     reachable pair in the DAG of 1-2 gradient pairs (Section 3.1, caption of
 *     Figure 6 (d)); paths that do not end at a 2-saddle are discarded
 *     (Section 3.5).  The paper reaches these counts with BFS, a DAG minor and
 *     iterated sparse matrix products (Sections 3.2, 3.3); the oracle instead
 *     counts paths directly by dynamic programming over each source's
 *     reachable set, which is the plain definition of the same numbers.
 *
 * Readings where the paper is silent (both sides encode them; they are the
 * contract):
 *   - vertex order: u < v iff (f(u), id(u)) < (f(v), id(v)), -0.0 == +0.0;
 *   - cell ids: a cell at refined coordinates (X, Y, Z) has id
 *     8 * vid(X>>1, Y>>1, Z>>1) + (X&1) + 2(Y&1) + 4(Z&1);
 *   - gradient word per vertex: nibble k = a + 2b + 4c describes the cell at
 *     refined (2x+a, 2y+b, 2z+c): 1..6 = partner at refined offset +X, -X,
 *     +Y, -Y, +Z, -Z; 7 = cell does not exist; 8 + d = critical whose highest
 *     vertex is the word's vertex plus corner d = dx + 2dy + 4dz;
 *   - critical list sorted by (index, cell id); the rank of a critical cell is
 *     its position among cells of the same index;
 *   - path counts are exact unsigned 64-bit integers saturating at 2^64 - 1;
 *   - (2,3) paths that leave the box through a boundary quad are dropped.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_NONFINITE 2
#define ORC_ERR_OOM 3
#define ORC_ERR_INTERNAL 4
#define ORC_ERR_CAPACITY 5

#define CRIT_BASE 8u
#define NOCELL 7u
#define EXIT_ROOT (-2)

typedef struct {
    int64_t n[3]; /* vertex counts along x, y, z */
    int64_t stride[3];
    int64_t nv;
} grid_t;

static int grid_init(grid_t* g, int64_t nx, int64_t ny, int64_t nz) {
    if (nx < 1 || ny < 1 || nz < 1) return ORC_ERR_ARG;
    g->n[0] = nx; g->n[1] = ny; g->n[2] = nz;
    g->stride[0] = 1; g->stride[1] = nx; g->stride[2] = nx * ny;
    g->nv = nx * ny * nz;
    if (g->nv > ((int64_t)1 << 29)) return ORC_ERR_ARG; /* cell ids must fit in 32 bits */
    return ORC_OK;
}

static void vcoords(const grid_t* g, int64_t v, int64_t c[3]) {
    c[0] = v % g->n[0];
    c[1] = (v / g->n[0]) % g->n[1];
    c[2] = v / (g->n[0] * g->n[1]);
}

/* u precedes v in the vertex order (simulation of simplicity by id). */
static int vprec(const float* f, int64_t u, int64_t v) {
    if (f[u] < f[v]) return 1;
    if (f[v] < f[u]) return 0;
    return u < v;
}

/* ---- cells in refined coordinates ---------------------------------------- */

static int64_t cell_id_of(const grid_t* g, const int64_t r[3]) {
    int64_t w = (r[0] >> 1) + g->n[0] * ((r[1] >> 1) + g->n[1] * (r[2] >> 1));
    return 8 * w + (r[0] & 1) + 2 * (r[1] & 1) + 4 * (r[2] & 1);
}

static void cell_ref(const grid_t* g, int64_t id, int64_t r[3]) {
    int64_t c[3];
    int k = (int)(id & 7);
    vcoords(g, id >> 3, c);
    for (int a = 0; a < 3; a++) r[a] = 2 * c[a] + ((k >> a) & 1);
}

static int ref_in_range(const grid_t* g, const int64_t r[3]) {
    for (int a = 0; a < 3; a++)
        if (r[a] < 0 || r[a] > 2 * g->n[a] - 2) return 0;
    return 1;
}

static int cell_dim(int64_t id) {
    int k = (int)(id & 7);
    return (k & 1) + ((k >> 1) & 1) + ((k >> 2) & 1);
}

/* All vertices of a cell: every rounding of its odd coordinates. */
static int cell_vertices(const grid_t* g, const int64_t r[3], int64_t* out) {
    int m = 0;
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = r[a] >> 1;
        hi[a] = (r[a] & 1) ? lo[a] + 1 : lo[a];
    }
    for (int64_t z = lo[2]; z <= hi[2]; z++)
        for (int64_t y = lo[1]; y <= hi[1]; y++)
            for (int64_t x = lo[0]; x <= hi[0]; x++)
                out[m++] = x + g->n[0] * (y + g->n[1] * z);
    return m;
}

static int64_t cell_maxv(const grid_t* g, const float* f, int64_t id) {
    int64_t r[3], vs[8];
    cell_ref(g, id, r);
    int m = cell_vertices(g, r, vs);
    int64_t best = vs[0];
    for (int i = 1; i < m; i++)
        if (vprec(f, best, vs[i])) best = vs[i];
    return best;
}

/* The cell one refined step from `id` along `axis` in direction `sign`, or -1
 * when that leaves the grid. */
static int64_t cell_step(const grid_t* g, int64_t id, int axis, int sign) {
    int64_t r[3];
    cell_ref(g, id, r);
    r[axis] += sign;
    if (!ref_in_range(g, r)) return -1;
    return cell_id_of(g, r);
}

/* ---- ProcessLowerStars on one vertex ---------------------------------------- */

enum { UNCLASSIFIED = 0, PAIRED = 1, CRITICAL = 2 };

typedef struct {
    int n;
    int64_t rc[27][3];
    int64_t id[27];
    int dim[27];
    int nk[27];
    int64_t key[27][7]; /* vertices other than x, in decreasing vertex order */
    int st[27];
    int mate[27];
    int nf[27], fac[27][3];
    int nc[27], cof[27][6];
} lstar_t;

/* Lexicographic comparison of the descending vertex lists; a proper prefix
 * compares smaller.  This is the order G of Robins et al. restricted to one
 * lower star (every cell shares the top vertex x). */
static int gless(const float* f, const lstar_t* L, int a, int b) {
    int m = L->nk[a] < L->nk[b] ? L->nk[a] : L->nk[b];
    for (int i = 0; i < m; i++)
        if (L->key[a][i] != L->key[b][i]) return vprec(f, L->key[a][i], L->key[b][i]);
    return L->nk[a] < L->nk[b];
}

static int unclassified_facets(const lstar_t* L, int a) {
    int u = 0;
    for (int i = 0; i < L->nf[a]; i++)
        if (L->st[L->fac[a][i]] == UNCLASSIFIED) u++;
    return u;
}

static void build_lower_star(const grid_t* g, const float* f, int64_t vx, lstar_t* L) {
    int64_t c[3];
    vcoords(g, vx, c);
    L->n = 0;
    for (int oz = -1; oz <= 1; oz++)
        for (int oy = -1; oy <= 1; oy++)
            for (int ox = -1; ox <= 1; ox++) {
                int64_t r[3] = {2 * c[0] + ox, 2 * c[1] + oy, 2 * c[2] + oz};
                if (!ref_in_range(g, r)) continue;
                int64_t vs[8];
                int m = cell_vertices(g, r, vs);
                int lower = 1;
                for (int i = 0; i < m; i++)
                    if (vs[i] != vx && !vprec(f, vs[i], vx)) lower = 0;
                if (!lower) continue;
                int j = L->n++;
                for (int a = 0; a < 3; a++) L->rc[j][a] = r[a];
                L->id[j] = cell_id_of(g, r);
                L->dim[j] = (ox != 0) + (oy != 0) + (oz != 0);
                /* key: other vertices sorted in decreasing order */
                int nk = 0;
                for (int i = 0; i < m; i++)
                    if (vs[i] != vx) L->key[j][nk++] = vs[i];
                for (int i = 1; i < nk; i++) {
                    int64_t t = L->key[j][i];
                    int p = i - 1;
                    while (p >= 0 && vprec(f, L->key[j][p], t)) {
                        L->key[j][p + 1] = L->key[j][p];
                        p--;
                    }
                    L->key[j][p + 1] = t;
                }
                L->nk[j] = nk;
                L->st[j] = UNCLASSIFIED;
                L->mate[j] = -1;
            }
    /* facet / cofacet relations inside L(x) */
    for (int i = 0; i < L->n; i++) { L->nf[i] = 0; L->nc[i] = 0; }
    for (int i = 0; i < L->n; i++)
        for (int j = 0; j < L->n; j++) {
            if (L->dim[j] != L->dim[i] - 1) continue;
            int diff = 0, ok = 1;
            for (int a = 0; a < 3; a++) {
                int64_t d = L->rc[i][a] - L->rc[j][a];
                if (d != 0) {
                    diff++;
                    if (d != 1 && d != -1) ok = 0;
                }
            }
            if (ok && diff == 1) {
                L->fac[i][L->nf[i]++] = j;
                L->cof[j][L->nc[j]++] = i;
            }
        }
}

static void pair_cells(lstar_t* L, int a, int b) {
    L->st[a] = PAIRED; L->st[b] = PAIRED;
    L->mate[a] = b; L->mate[b] = a;
}

static void push_ready_cofacets(lstar_t* L, int a, int* inone) {
    for (int i = 0; i < L->nc[a]; i++) {
        int b = L->cof[a][i];
        if (unclassified_facets(L, b) == 1) inone[b] = 1;
    }
}

/* Robins, Wood & Sheppard (2011), ProcessLowerStars, for one vertex.
 * Priority queues are membership sets; classified cells found in them are
 * skipped when popped. */
static int process_lower_star(const float* f, lstar_t* L) {
    int v0 = -1;
    for (int i = 0; i < L->n; i++)
        if (L->dim[i] == 0) v0 = i;
    if (v0 < 0) return ORC_ERR_INTERNAL;
    if (L->n == 1) {
        L->st[v0] = CRITICAL;
        return ORC_OK;
    }
    int delta = -1;
    for (int i = 0; i < L->n; i++)
        if (L->dim[i] == 1 && (delta < 0 || gless(f, L, i, delta))) delta = i;
    pair_cells(L, v0, delta);
    int inzero[27] = {0}, inone[27] = {0};
    for (int i = 0; i < L->n; i++)
        if (L->dim[i] == 1 && i != delta) inzero[i] = 1;
    push_ready_cofacets(L, delta, inone);
    for (;;) {
        for (;;) {
            int a = -1;
            for (int i = 0; i < L->n; i++)
                if (inone[i] && (a < 0 || gless(f, L, i, a))) a = i;
            if (a < 0) break;
            inone[a] = 0;
            if (L->st[a] != UNCLASSIFIED) continue;
            if (unclassified_facets(L, a) == 0) {
                inzero[a] = 1;
                continue;
            }
            int p = -1;
            for (int i = 0; i < L->nf[a]; i++)
                if (L->st[L->fac[a][i]] == UNCLASSIFIED) p = L->fac[a][i];
            pair_cells(L, p, a);
            inzero[p] = 0;
            push_ready_cofacets(L, a, inone);
            push_ready_cofacets(L, p, inone);
        }
        int gm = -1;
        for (int i = 0; i < L->n; i++) {
            if (inzero[i] && L->st[i] != UNCLASSIFIED) inzero[i] = 0;
            if (inzero[i] && (gm < 0 || gless(f, L, i, gm))) gm = i;
        }
        if (gm < 0) break;
        inzero[gm] = 0;
        L->st[gm] = CRITICAL;
        push_ready_cofacets(L, gm, inone);
    }
    for (int i = 0; i < L->n; i++)
        if (L->st[i] == UNCLASSIFIED) return ORC_ERR_INTERNAL;
    return ORC_OK;
}

/* Nibble value of cell i of L(x) under the gradient-word encoding. */
static uint32_t lstar_nibble(const grid_t* g, const lstar_t* L, int64_t vx, int i) {
    int64_t c[3];
    vcoords(g, vx, c);
    if (L->st[i] == CRITICAL) {
        uint32_t d = 0;
        for (int a = 0; a < 3; a++)
            if ((L->rc[i][a] >> 1) != c[a]) d |= 1u << a; /* word vertex is x - 1 along a */
        return CRIT_BASE + d;
    }
    int j = L->mate[i];
    for (int a = 0; a < 3; a++) {
        int64_t d = L->rc[j][a] - L->rc[i][a];
        if (d == 1) return (uint32_t)(1 + 2 * a);
        if (d == -1) return (uint32_t)(2 + 2 * a);
    }
    return 0; /* unreachable for a valid pairing */
}

static int nibble_exists(const grid_t* g, int64_t w, int k) {
    int64_t c[3];
    vcoords(g, w, c);
    for (int a = 0; a < 3; a++)
        if (((k >> a) & 1) && c[a] >= g->n[a] - 1) return 0;
    return 1;
}

static int check_finite(const float* f, int64_t n) {
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(f[i])) return ORC_ERR_NONFINITE;
    return ORC_OK;
}

int orc_gradient(const float* f, int64_t nx, int64_t ny, int64_t nz, uint32_t* grad) {
    grid_t g;
    int rc = grid_init(&g, nx, ny, nz);
    if (rc) return rc;
    if ((rc = check_finite(f, g.nv))) return rc;
    for (int64_t w = 0; w < g.nv; w++) {
        uint32_t word = 0;
        for (int k = 0; k < 8; k++)
            if (!nibble_exists(&g, w, k)) word |= NOCELL << (4 * k);
        grad[w] = word;
    }
    lstar_t L;
    for (int64_t vx = 0; vx < g.nv; vx++) {
        build_lower_star(&g, f, vx, &L);
        if ((rc = process_lower_star(f, &L))) return rc;
        for (int i = 0; i < L.n; i++) {
            int64_t w = L.id[i] >> 3;
            int k = (int)(L.id[i] & 7);
            if ((grad[w] >> (4 * k)) & 15u) return ORC_ERR_INTERNAL; /* written twice */
            grad[w] |= lstar_nibble(&g, &L, vx, i) << (4 * k);
        }
    }
    for (int64_t w = 0; w < g.nv; w++)
        for (int k = 0; k < 8; k++)
            if (((grad[w] >> (4 * k)) & 15u) == 0) return ORC_ERR_INTERNAL; /* never written */
    return ORC_OK;
}

/* ---- a source of gradient nibbles: a full array, or lazily from f ---------- */

typedef struct {
    uint64_t* keys;
    uint64_t* vals;
    uint64_t* aux;
    int64_t cap, size;
} hmap_t;

#define HM_EMPTY UINT64_MAX

static int hm_init(hmap_t* h, int64_t cap) {
    int64_t c = 64;
    while (c < 2 * cap) c <<= 1;
    h->keys = (uint64_t*)malloc(sizeof(uint64_t) * c);
    h->vals = (uint64_t*)malloc(sizeof(uint64_t) * c);
    h->aux = (uint64_t*)malloc(sizeof(uint64_t) * c);
    if (!h->keys || !h->vals || !h->aux) return ORC_ERR_OOM;
    for (int64_t i = 0; i < c; i++) h->keys[i] = HM_EMPTY;
    h->cap = c;
    h->size = 0;
    return ORC_OK;
}

static void hm_free(hmap_t* h) {
    free(h->keys); free(h->vals); free(h->aux);
    h->keys = h->vals = h->aux = NULL;
}

static uint64_t hm_hash(uint64_t k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdULL; k ^= k >> 33;
    return k;
}

/* Slot of key k (inserting it with zero value/aux when absent); -1 on OOM. */
static int64_t hm_slot(hmap_t* h, uint64_t k, int insert) {
    if (insert && 2 * (h->size + 1) > h->cap) {
        hmap_t n2;
        if (hm_init(&n2, h->cap) != ORC_OK) return -1;
        for (int64_t i = 0; i < h->cap; i++)
            if (h->keys[i] != HM_EMPTY) {
                int64_t s = (int64_t)(hm_hash(h->keys[i]) & (uint64_t)(n2.cap - 1));
                while (n2.keys[s] != HM_EMPTY) s = (s + 1) & (n2.cap - 1);
                n2.keys[s] = h->keys[i]; n2.vals[s] = h->vals[i]; n2.aux[s] = h->aux[i];
                n2.size++;
            }
        hm_free(h);
        *h = n2;
    }
    int64_t s = (int64_t)(hm_hash(k) & (uint64_t)(h->cap - 1));
    while (h->keys[s] != HM_EMPTY && h->keys[s] != k) s = (s + 1) & (h->cap - 1);
    if (h->keys[s] == HM_EMPTY) {
        if (!insert) return -1;
        h->keys[s] = k; h->vals[s] = 0; h->aux[s] = 0;
        h->size++;
    }
    return s;
}

static void hm_clear(hmap_t* h) {
    for (int64_t i = 0; i < h->cap; i++) h->keys[i] = HM_EMPTY;
    h->size = 0;
}

typedef struct {
    grid_t g;
    const float* f;
    const uint32_t* grad; /* NULL: compute nibbles lazily from f */
    hmap_t cache;         /* lazy mode: cell id -> nibble */
    int err;
} src_t;

static uint32_t nibble(src_t* s, int64_t id) {
    int64_t w = id >> 3;
    int k = (int)(id & 7);
    if (s->grad) return (s->grad[w] >> (4 * k)) & 15u;
    if (!nibble_exists(&s->g, w, k)) return NOCELL;
    int64_t slot = hm_slot(&s->cache, (uint64_t)id, 0);
    if (slot >= 0) return (uint32_t)s->cache.vals[slot];
    int64_t vx = cell_maxv(&s->g, s->f, id);
    lstar_t L;
    build_lower_star(&s->g, s->f, vx, &L);
    if (process_lower_star(s->f, &L)) { s->err = ORC_ERR_INTERNAL; return 0; }
    uint32_t out = 0;
    for (int i = 0; i < L.n; i++) {
        uint32_t nb = lstar_nibble(&s->g, &L, vx, i);
        int64_t sl = hm_slot(&s->cache, (uint64_t)L.id[i], 1);
        if (sl < 0) { s->err = ORC_ERR_OOM; return 0; }
        s->cache.vals[sl] = nb;
        if (L.id[i] == id) out = nb;
    }
    return out;
}

static int src_init(src_t* s, const float* f, const uint32_t* grad, int64_t nx, int64_t ny, int64_t nz) {
    int rc = grid_init(&s->g, nx, ny, nz);
    if (rc) return rc;
    s->f = f;
    s->grad = grad;
    s->err = 0;
    s->cache.keys = s->cache.vals = s->cache.aux = NULL;
    if (!grad) return hm_init(&s->cache, 1024);
    return ORC_OK;
}

static void src_free(src_t* s) {
    if (!s->grad) hm_free(&s->cache);
}

uint32_t orc_nibble_lazy(const float* f, int64_t nx, int64_t ny, int64_t nz, int64_t id) {
    src_t s;
    if (src_init(&s, f, NULL, nx, ny, nz)) return 0;
    uint32_t v = nibble(&s, id);
    src_free(&s);
    return s.err ? 0 : v;
}

/* Partner of a non-critical cell (refined neighbour the nibble points at). */
static int64_t partner_of(src_t* s, int64_t id, uint32_t nb) {
    int axis = (int)(nb - 1) / 2;
    int sign = ((nb - 1) & 1) ? -1 : 1;
    return cell_step(&s->g, id, axis, sign);
}

/* ---- critical cells -------------------------------------------------------- */

int orc_critical_counts(const uint32_t* grad, int64_t nx, int64_t ny, int64_t nz, int64_t count[4]) {
    grid_t g;
    int rc = grid_init(&g, nx, ny, nz);
    if (rc) return rc;
    for (int i = 0; i < 4; i++) count[i] = 0;
    for (int64_t w = 0; w < g.nv; w++)
        for (int k = 0; k < 8; k++)
            if (((grad[w] >> (4 * k)) & 15u) >= CRIT_BASE) count[cell_dim(k)]++;
    return ORC_OK;
}

/* Fills the critical list sorted by (index, cell id).  Arrays hold
 * sum(count) entries. */
int orc_critical_fill(const float* f, const uint32_t* grad, int64_t nx, int64_t ny, int64_t nz,
                      uint32_t* id, uint8_t* index, float* value, uint32_t* vmax) {
    grid_t g;
    int rc = grid_init(&g, nx, ny, nz);
    if (rc) return rc;
    int64_t count[4], off[4];
    orc_critical_counts(grad, nx, ny, nz, count);
    off[0] = 0;
    for (int i = 1; i < 4; i++) off[i] = off[i - 1] + count[i - 1];
    for (int64_t w = 0; w < g.nv; w++)
        for (int k = 0; k < 8; k++) {
            uint32_t nb = (grad[w] >> (4 * k)) & 15u;
            if (nb < CRIT_BASE) continue;
            int64_t cid = 8 * w + k;
            int64_t mv = cell_maxv(&g, f, cid);
            /* the encoded corner must be the cell's highest vertex */
            int64_t c[3];
            vcoords(&g, w, c);
            uint32_t d = nb - CRIT_BASE;
            for (int a = 0; a < 3; a++) c[a] += (d >> a) & 1;
            if (c[0] + g.n[0] * (c[1] + g.n[1] * c[2]) != mv) return ORC_ERR_INTERNAL;
            int dim = cell_dim(cid);
            int64_t p = off[dim]++;
            id[p] = (uint32_t)cid;
            index[p] = (uint8_t)dim;
            value[p] = f[mv];
            vmax[p] = (uint32_t)mv;
        }
    return ORC_OK;
}

/* ---- saddle-extremum arcs --------------------------------------------------- */

/* Follow the (0,1) V-path from vertex v down to its minimum. */
static int64_t vertex_root(src_t* s, int64_t v) {
    for (int64_t steps = 0; steps <= s->g.nv; steps++) {
        uint32_t nb = nibble(s, 8 * v);
        if (nb >= CRIT_BASE) return v;
        if (nb < 1 || nb > 6) return -1;
        int64_t e = partner_of(s, 8 * v, nb);
        if (e < 0 || cell_dim(e) != 1) return -1;
        /* the other vertex of edge e */
        int64_t r[3], vs[8];
        cell_ref(&s->g, e, r);
        cell_vertices(&s->g, r, vs);
        v = (vs[0] == v) ? vs[1] : vs[0];
    }
    return -1; /* a cycle: not a gradient */
}

/* Follow the (2,3) V-path upward from cube c (by its cell id) to a maximum;
 * EXIT_ROOT when it leaves through a boundary quad. */
static int64_t cube_root(src_t* s, int64_t c) {
    for (int64_t steps = 0; steps <= s->g.nv; steps++) {
        uint32_t nb = nibble(s, c);
        if (nb >= CRIT_BASE) return c;
        if (nb < 1 || nb > 6) return -1;
        int axis = (int)(nb - 1) / 2;
        int sign = ((nb - 1) & 1) ? -1 : 1;
        int64_t q = cell_step(&s->g, c, axis, sign); /* the paired quad */
        if (q < 0 || cell_dim(q) != 2) return -1;
        int64_t c2 = cell_step(&s->g, q, axis, sign); /* the quad's other cube */
        if (c2 < 0) return EXIT_ROOT;
        c = c2;
    }
    return -1;
}

typedef struct { int64_t r, c; uint64_t v; } coo_t;

static int coo_cmp(const void* a, const void* b) {
    const coo_t* x = (const coo_t*)a;
    const coo_t* y = (const coo_t*)b;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return 0;
}

static uint64_t sat_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s < a ? UINT64_MAX : s;
}

/* sort by (row, col) and merge repeats by (saturating) addition */
static int64_t coo_sort_merge(coo_t* e, int64_t m) {
    qsort(e, (size_t)m, sizeof(coo_t), coo_cmp);
    int64_t o = 0;
    for (int64_t i = 0; i < m; i++) {
        if (o > 0 && e[o - 1].r == e[i].r && e[o - 1].c == e[i].c)
            e[o - 1].v = sat_add(e[o - 1].v, e[i].v);
        else
            e[o++] = e[i];
    }
    return o;
}

static int64_t lower_bound_u32(const uint32_t* a, int64_t n, uint32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* M10 (rows: 1-saddle ranks, cols: minimum ranks) and M32 (rows: maximum
 * ranks, cols: 2-saddle ranks), as sorted COO with multiplicities.
 * `crit_id` is the critical list sorted by (index, id) with counts `count`.
 * Output capacity: 2*count[1] for M10, 2*count[2] for M32. */
int orc_se_arcs(const uint32_t* grad, int64_t nx, int64_t ny, int64_t nz,
                const uint32_t* crit_id, const int64_t count[4],
                int64_t* m10_r, int64_t* m10_c, uint64_t* m10_v, int64_t* m10_nnz,
                int64_t* m32_r, int64_t* m32_c, uint64_t* m32_v, int64_t* m32_nnz) {
    src_t s;
    int rc = src_init(&s, NULL, grad, nx, ny, nz);
    if (rc) return rc;
    const uint32_t* mins = crit_id;
    const uint32_t* sad1 = crit_id + count[0];
    const uint32_t* sad2 = crit_id + count[0] + count[1];
    const uint32_t* maxs = crit_id + count[0] + count[1] + count[2];
    coo_t* e = (coo_t*)malloc(sizeof(coo_t) * (size_t)(2 * (count[1] + count[2]) + 1));
    if (!e) return ORC_ERR_OOM;
    int64_t m = 0;
    for (int64_t r = 0; r < count[1]; r++) {
        int64_t id = sad1[r];
        int64_t rr[3], vs[8];
        cell_ref(&s.g, id, rr);
        cell_vertices(&s.g, rr, vs);
        for (int i = 0; i < 2; i++) {
            int64_t root = vertex_root(&s, vs[i]);
            if (root < 0) { free(e); return ORC_ERR_INTERNAL; }
            int64_t rank = lower_bound_u32(mins, count[0], (uint32_t)(8 * root));
            if (rank >= count[0] || mins[rank] != (uint32_t)(8 * root)) { free(e); return ORC_ERR_INTERNAL; }
            e[m].r = r; e[m].c = rank; e[m].v = 1; m++;
        }
    }
    m = coo_sort_merge(e, m);
    for (int64_t i = 0; i < m; i++) { m10_r[i] = e[i].r; m10_c[i] = e[i].c; m10_v[i] = e[i].v; }
    *m10_nnz = m;
    m = 0;
    for (int64_t r = 0; r < count[2]; r++) {
        int64_t q = sad2[r];
        int missing = 0;
        for (int a = 0; a < 3; a++)
            if (!((q & 7) >> a & 1)) missing = a;
        for (int sg = -1; sg <= 1; sg += 2) {
            int64_t c = cell_step(&s.g, q, missing, sg);
            if (c < 0) continue;
            int64_t root = cube_root(&s, c);
            if (root == -1) { free(e); return ORC_ERR_INTERNAL; }
            if (root == EXIT_ROOT) continue;
            int64_t rank = lower_bound_u32(maxs, count[3], (uint32_t)root);
            if (rank >= count[3] || maxs[rank] != (uint32_t)root) { free(e); return ORC_ERR_INTERNAL; }
            e[m].r = rank; e[m].c = r; e[m].v = 1; m++;
        }
    }
    m = coo_sort_merge(e, m);
    for (int64_t i = 0; i < m; i++) { m32_r[i] = e[i].r; m32_c[i] = e[i].c; m32_v[i] = e[i].v; }
    *m32_nnz = m;
    free(e);
    return ORC_OK;
}

/* Lazy (from f only) roots for one 1-saddle: the two minima (vertex ids). */
int orc_m10_row_lazy(const float* f, int64_t nx, int64_t ny, int64_t nz, int64_t s1,
                     int64_t out_min_vid[2]) {
    src_t s;
    int rc = src_init(&s, f, NULL, nx, ny, nz);
    if (rc) return rc;
    int64_t rr[3], vs[8];
    cell_ref(&s.g, s1, rr);
    cell_vertices(&s.g, rr, vs);
    for (int i = 0; i < 2; i++) out_min_vid[i] = vertex_root(&s, vs[i]);
    rc = s.err;
    src_free(&s);
    if (rc) return rc;
    return (out_min_vid[0] < 0 || out_min_vid[1] < 0) ? ORC_ERR_INTERNAL : ORC_OK;
}

/* Lazy roots of the (at most two) cofacet cubes of a 2-saddle: maximum cell
 * ids, -2 for a path leaving the box, -3 for a missing cofacet. */
int orc_m32_col_lazy(const float* f, int64_t nx, int64_t ny, int64_t nz, int64_t q,
                     int64_t out_max_id[2]) {
    src_t s;
    int rc = src_init(&s, f, NULL, nx, ny, nz);
    if (rc) return rc;
    int missing = 0;
    for (int a = 0; a < 3; a++)
        if (!((q & 7) >> a & 1)) missing = a;
    for (int i = 0; i < 2; i++) {
        int64_t c = cell_step(&s.g, q, missing, i == 0 ? -1 : 1);
        out_max_id[i] = c < 0 ? -3 : cube_root(&s, c);
    }
    rc = s.err;
    src_free(&s);
    return rc;
}

/* ---- ascending and descending 3-manifolds ----------------------------------- */

#define ORC_NO_LABEL 0xFFFFFFFFu

/* Section 3.4: the traversal that yields the saddle-extremum arcs also yields
 * the ascending manifolds of the minima and the descending manifolds of the
 * maxima, i.e. for every non-critical cell the extremum its gradient path
 * ends at (Section 3.5 keeps these destinations in an extra array).
 *   min_label[v] : rank (among minima, in id order) of the minimum that the
 *                  (0,1) V-path from vertex v reaches;
 *   max_label[w] : rank (among maxima) of the maximum that the (2,3) V-path
 *                  from the cube whose lowest corner is vertex w reaches;
 *                  ORC_NO_LABEL when that cube does not exist (w on a high
 *                  face of the box) or when its path leaves the box through
 *                  a boundary quad (such paths are discarded, Section 3.5).
 * Each vertex and each cube is walked on its own, step by step. */
int orc_manifolds(const uint32_t* grad, int64_t nx, int64_t ny, int64_t nz, const uint32_t* crit_id,
                  const int64_t count[4], uint32_t* min_label, uint32_t* max_label) {
    src_t s;
    int rc = src_init(&s, NULL, grad, nx, ny, nz);
    if (rc) return rc;
    const uint32_t* mins = crit_id;
    const uint32_t* maxs = crit_id + count[0] + count[1] + count[2];
    for (int64_t v = 0; v < s.g.nv; v++) {
        int64_t root = vertex_root(&s, v);
        if (root < 0) return ORC_ERR_INTERNAL;
        int64_t rank = lower_bound_u32(mins, count[0], (uint32_t)(8 * root));
        if (rank >= count[0] || mins[rank] != (uint32_t)(8 * root)) return ORC_ERR_INTERNAL;
        min_label[v] = (uint32_t)rank;
    }
    for (int64_t w = 0; w < s.g.nv; w++) {
        max_label[w] = ORC_NO_LABEL;
        if (!nibble_exists(&s.g, w, 7)) continue;
        int64_t root = cube_root(&s, 8 * w + 7);
        if (root == -1) return ORC_ERR_INTERNAL;
        if (root == EXIT_ROOT) continue;
        int64_t rank = lower_bound_u32(maxs, count[3], (uint32_t)root);
        if (rank >= count[3] || maxs[rank] != (uint32_t)root) return ORC_ERR_INTERNAL;
        max_label[w] = (uint32_t)rank;
    }
    return ORC_OK;
}

/* ---- 1-saddle / 2-saddle path counts ----------------------------------------- */

/* Out-neighbours of an edge node in the DAG of 1-2 gradient pairs:
 * targets[i] is a cell id; is2[i] marks a 2-saddle, otherwise an edge. */
static int dag_targets(src_t* s, int64_t e, int64_t* targets, int* is2) {
    int m = 0;
    int axis_e = 0;
    for (int a = 0; a < 3; a++)
        if ((e & 7) >> a & 1) axis_e = a;
    uint32_t ne = nibble(s, e);
    int64_t ve = -1; /* V(e): the quad e is paired with, if any */
    if (ne >= 1 && ne <= 6) {
        int64_t p = partner_of(s, e, ne);
        if (p >= 0 && cell_dim(p) == 2) ve = p;
    }
    for (int b = 0; b < 3; b++) {
        if (b == axis_e) continue;
        for (int sg = -1; sg <= 1; sg += 2) {
            int64_t q = cell_step(&s->g, e, b, sg);
            if (q < 0 || q == ve) continue;
            uint32_t nq = nibble(s, q);
            if (nq >= CRIT_BASE) {
                targets[m] = q; is2[m] = 1; m++;
            } else if (nq >= 1 && nq <= 6) {
                int64_t p = partner_of(s, q, nq);
                if (p >= 0 && cell_dim(p) == 1) {
                    targets[m] = p; is2[m] = 0; m++;
                }
            }
        }
    }
    return m;
}

typedef struct {
    int64_t* q; uint64_t* cnt; int64_t n, cap;
} row_t;

/* Number of directed paths from 1-saddle s1 to every 2-saddle it reaches,
 * by DFS over the reachable set followed by Kahn-order accumulation. */
static int ss_row(src_t* s, int64_t s1, hmap_t* node, hmap_t* hit, int64_t** stack, int64_t* stack_cap,
                  row_t* out) {
    hm_clear(node);
    hm_clear(hit);
    int64_t sp = 0;
    int64_t t[4];
    int is2[4];
    /* discover the reachable node set */
    if (hm_slot(node, (uint64_t)s1, 1) < 0) return ORC_ERR_OOM;
    (*stack)[sp++] = s1;
    while (sp > 0) {
        int64_t u = (*stack)[--sp];
        int m = dag_targets(s, u, t, is2);
        if (s->err) return s->err;
        for (int i = 0; i < m; i++) {
            if (is2[i]) continue;
            int64_t before = node->size;
            int64_t sl = hm_slot(node, (uint64_t)t[i], 1);
            if (sl < 0) return ORC_ERR_OOM;
            node->aux[sl] += 1; /* in-degree inside the reachable set */
            if (node->size > before) {
                if (sp >= *stack_cap) {
                    int64_t nc = 2 * (*stack_cap);
                    int64_t* ns = (int64_t*)realloc(*stack, sizeof(int64_t) * (size_t)nc);
                    if (!ns) return ORC_ERR_OOM;
                    *stack = ns; *stack_cap = nc;
                }
                (*stack)[sp++] = t[i];
            }
        }
    }
    /* Kahn order accumulation of path counts */
    int64_t sl0 = hm_slot(node, (uint64_t)s1, 0);
    node->vals[sl0] = 1;
    sp = 0;
    (*stack)[sp++] = s1;
    int64_t done = 0;
    while (sp > 0) {
        int64_t u = (*stack)[--sp];
        done++;
        uint64_t cu = node->vals[hm_slot(node, (uint64_t)u, 0)];
        int m = dag_targets(s, u, t, is2);
        for (int i = 0; i < m; i++) {
            if (is2[i]) {
                int64_t sl = hm_slot(hit, (uint64_t)t[i], 1);
                if (sl < 0) return ORC_ERR_OOM;
                hit->vals[sl] = sat_add(hit->vals[sl], cu);
            } else {
                int64_t sl = hm_slot(node, (uint64_t)t[i], 0);
                node->vals[sl] = sat_add(node->vals[sl], cu);
                if (--node->aux[sl] == 0) (*stack)[sp++] = t[i];
            }
        }
    }
    if (done != node->size) return ORC_ERR_INTERNAL; /* a cycle in the DAG */
    out->n = 0;
    for (int64_t i = 0; i < hit->cap; i++) {
        if (hit->keys[i] == HM_EMPTY) continue;
        if (out->n >= out->cap) {
            int64_t nc = 2 * out->cap + 16;
            int64_t* nq = (int64_t*)realloc(out->q, sizeof(int64_t) * (size_t)nc);
            if (!nq) return ORC_ERR_OOM;
            out->q = nq;
            uint64_t* nn = (uint64_t*)realloc(out->cnt, sizeof(uint64_t) * (size_t)nc);
            if (!nn) return ORC_ERR_OOM;
            out->cnt = nn;
            out->cap = nc;
        }
        out->q[out->n] = (int64_t)hit->keys[i];
        out->cnt[out->n] = hit->vals[i];
        out->n++;
    }
    return ORC_OK;
}

/* Result holder for variable-size outputs. */
typedef struct {
    int64_t n;
    int64_t* r;
    int64_t* c;
    uint64_t* v;
} orc_coo;

void orc_coo_free(orc_coo* p) {
    if (!p) return;
    free(p->r); free(p->c); free(p->v);
    free(p);
}
int64_t orc_coo_nnz(const orc_coo* p) { return p->n; }
void orc_coo_copy(const orc_coo* p, int64_t* r, int64_t* c, uint64_t* v) {
    for (int64_t i = 0; i < p->n; i++) { r[i] = p->r[i]; c[i] = p->c[i]; v[i] = p->v[i]; }
}

static int ss_run(src_t* s, const int64_t* sources, int64_t nsrc, orc_coo** out_p, int rows_are_ids,
                  const uint32_t* sad2, int64_t n2) {
    hmap_t node, hit;
    int rc;
    if ((rc = hm_init(&node, 256))) return rc;
    if ((rc = hm_init(&hit, 64))) { hm_free(&node); return rc; }
    int64_t stack_cap = 1024;
    int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * (size_t)stack_cap);
    row_t row = {NULL, NULL, 0, 0};
    coo_t* all = NULL;
    int64_t nall = 0, capall = 0;
    if (!stack) { rc = ORC_ERR_OOM; goto done; }
    for (int64_t i = 0; i < nsrc; i++) {
        if ((rc = ss_row(s, sources[i], &node, &hit, &stack, &stack_cap, &row))) goto done;
        if (nall + row.n > capall) {
            int64_t nc = 2 * (nall + row.n) + 64;
            coo_t* na = (coo_t*)realloc(all, sizeof(coo_t) * (size_t)nc);
            if (!na) { rc = ORC_ERR_OOM; goto done; }
            all = na; capall = nc;
        }
        for (int64_t j = 0; j < row.n; j++) {
            int64_t col = row.q[j];
            if (!rows_are_ids) {
                int64_t rk = lower_bound_u32(sad2, n2, (uint32_t)col);
                if (rk >= n2 || sad2[rk] != (uint32_t)col) { rc = ORC_ERR_INTERNAL; goto done; }
                col = rk;
            }
            all[nall].r = rows_are_ids ? sources[i] : i;
            all[nall].c = col;
            all[nall].v = row.cnt[j];
            nall++;
        }
    }
    nall = all ? coo_sort_merge(all, nall) : 0;
    {
        orc_coo* p = (orc_coo*)calloc(1, sizeof(orc_coo));
        if (!p) { rc = ORC_ERR_OOM; goto done; }
        p->n = nall;
        p->r = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nall + 1));
        p->c = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nall + 1));
        p->v = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nall + 1));
        if (!p->r || !p->c || !p->v) { orc_coo_free(p); rc = ORC_ERR_OOM; goto done; }
        for (int64_t j = 0; j < nall; j++) { p->r[j] = all[j].r; p->c[j] = all[j].c; p->v[j] = all[j].v; }
        *out_p = p;
    }
    rc = s->err;
done:
    hm_free(&node); hm_free(&hit);
    free(stack); free(row.q); free(row.cnt); free(all);
    return rc;
}

/* P (rows: 1-saddle ranks, cols: 2-saddle ranks, values: path counts) from a
 * full gradient and the critical list sorted by (index, id). */
int orc_ss_paths(const uint32_t* grad, int64_t nx, int64_t ny, int64_t nz,
                 const uint32_t* crit_id, const int64_t count[4], orc_coo** out) {
    src_t s;
    int rc = src_init(&s, NULL, grad, nx, ny, nz);
    if (rc) return rc;
    int64_t* src = (int64_t*)malloc(sizeof(int64_t) * (size_t)(count[1] + 1));
    if (!src) return ORC_ERR_OOM;
    for (int64_t i = 0; i < count[1]; i++) src[i] = crit_id[count[0] + i];
    rc = ss_run(&s, src, count[1], out, 0, crit_id + count[0] + count[1], count[2]);
    free(src);
    return rc;
}

/* Lazy (from f only) path counts for the given 1-saddle cell ids; rows and
 * columns are cell ids. */
int orc_ss_rows_lazy(const float* f, int64_t nx, int64_t ny, int64_t nz,
                     const int64_t* s1_ids, int64_t nsrc, orc_coo** out) {
    src_t s;
    int rc = src_init(&s, f, NULL, nx, ny, nz);
    if (rc) return rc;
    rc = ss_run(&s, s1_ids, nsrc, out, 1, NULL, 0);
    src_free(&s);
    return rc;
}

/* Per-cell results of ProcessLowerStars at one vertex (for sampled checks):
 * cell ids and nibbles of every cell in L(vid).  Returns the cell count. */
int orc_lower_star(const float* f, int64_t nx, int64_t ny, int64_t nz, int64_t vid,
                   int64_t out_id[27], uint32_t out_nib[27]) {
    grid_t g;
    if (grid_init(&g, nx, ny, nz)) return -1;
    lstar_t L;
    build_lower_star(&g, f, vid, &L);
    if (process_lower_star(f, &L)) return -1;
    for (int i = 0; i < L.n; i++) {
        out_id[i] = L.id[i];
        out_nib[i] = lstar_nibble(&g, &L, vid, i);
    }
    return L.n;
}

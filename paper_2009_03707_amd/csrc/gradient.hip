// Discrete gradient by per-vertex lower-star pairing.
//
// The paper assigns gradient pairs in a first, embarrassingly parallel step
// (Section 3, first step; Section 3.5, "Gradient pairs and critical
// points").  The pairing rule is the locally independent lower-star rule of
// Robins, Wood and Sheppard that the paper cites (Section 1.1): the cells
// whose highest vertex is x are paired among themselves by two priority
// queues ordered by the cells' vertex values.
//
// MI355X design: one workgroup runs the lower stars of an OX x OY x OZ
// block of vertices.  The field tile (with a one-vertex halo on each side)
// is staged in LDS as order-preserving integer keys; every vertex of the
// block runs the lower-star pairing in registers with bitmask queues, the
// vertices taken in order of lower-star size so that the lanes of a wave do
// similar work; each lower star's nibbles are OR-ed into an LDS word tile
// (each nibble is written by exactly one lower star).  A word receives the
// nibbles of the lower stars of its vertex and of its +x / +y / +z
// neighbours, so the words of the block's interior get all of theirs from
// the block and are stored plainly, while the words on the block's high
// faces and the low-side halo words get nibbles from several blocks and are
// OR-ed atomically into the gradient, which is cleared first.  Every lower
// star is thus computed once.
#include "common.h"

namespace msc {
namespace {

// Tile shapes (output words per workgroup), selectable at run time; the
// autotuner picks one per size class.  Results do not depend on the shape.
template <int X, int Y, int Z>
struct Tile {
    static constexpr int OX = X, OY = Y, OZ = Z;            // vertices (lower stars) per block
    static constexpr int FX = X + 2, FY = Y + 2, FZ = Z + 2;  // staged field tile
    static constexpr int NF = FX * FY * FZ;
    static constexpr int NV = X * Y * Z;
    static constexpr int WX = X + 1, WY = Y + 1, WZ = Z + 1;  // word tile: the block plus its low-side halo
    static constexpr int NW = WX * WY * WZ;
};
constexpr int THREADS = 256;
constexpr uint32_t NXCD = 8;  // accelerator complex dies of an MI355X
constexpr uint32_t KEY_OUT = 0xFFFFFFFFu;  // vertex outside the grid
constexpr uint32_t CENTER = 13;
// edge cells of the star: offsets (+-1,0,0), (0,+-1,0), (0,0,+-1)
constexpr uint32_t EDGES = (1u << 4) | (1u << 10) | (1u << 12) | (1u << 14) | (1u << 16) | (1u << 22);

// Star cell j <-> offset (ox, oy, oz) in {-1,0,1}^3, j = (ox+1) + 3(oy+1) + 9(oz+1).
__host__ __device__ constexpr int off_x(int j) { return j % 3 - 1; }
__host__ __device__ constexpr int off_y(int j) { return (j / 3) % 3 - 1; }
__host__ __device__ constexpr int off_z(int j) { return j / 9 - 1; }

// Vertices of star cell j other than the centre: every d != 0 with d_i in {0, o_i}.
__host__ __device__ constexpr uint32_t vert_mask(int j) {
    uint32_t m = 0;
    int ox = off_x(j), oy = off_y(j), oz = off_z(j);
    for (int dz = 0; dz <= 1; dz++)
        for (int dy = 0; dy <= 1; dy++)
            for (int dx = 0; dx <= 1; dx++) {
                int a = dx * ox, b = dy * oy, c = dz * oz;
                if ((dx && !ox) || (dy && !oy) || (dz && !oz)) continue;
                if (a == 0 && b == 0 && c == 0) continue;
                m |= 1u << ((a + 1) + 3 * (b + 1) + 9 * (c + 1));
            }
    return m;
}
// Facets of star cell j that contain the centre: zero one nonzero offset.
__host__ __device__ constexpr uint32_t facet_mask(int j) {
    uint32_t m = 0;
    if (off_x(j)) m |= 1u << (j - off_x(j));
    if (off_y(j)) m |= 1u << (j - 3 * off_y(j));
    if (off_z(j)) m |= 1u << (j - 9 * off_z(j));
    return m;
}
// Cofacets of star cell j inside the star: set one zero offset to +-1.
__host__ __device__ constexpr uint32_t cofacet_mask(int j) {
    uint32_t m = 0;
    if (!off_x(j)) m |= (1u << (j - 1)) | (1u << (j + 1));
    if (!off_y(j)) m |= (1u << (j - 3)) | (1u << (j + 3));
    if (!off_z(j)) m |= (1u << (j - 9)) | (1u << (j + 9));
    return m;
}
// Destination of star cell j in the gradient words: word at centre +
// (min(ox,0), min(oy,0), min(oz,0)), nibble |ox| + 2|oy| + 4|oz|.
// Packed: bit0..2 = (ox<0, oy<0, oz<0) (also the critical corner), bits 3..5 = nibble.
__host__ __device__ constexpr uint32_t dest_desc(int j) {
    int ox = off_x(j), oy = off_y(j), oz = off_z(j);
    uint32_t corner = (ox < 0 ? 1u : 0u) | (oy < 0 ? 2u : 0u) | (oz < 0 ? 4u : 0u);
    uint32_t k = (ox ? 1u : 0u) | (oy ? 2u : 0u) | (oz ? 4u : 0u);
    return corner | (k << 3);
}

struct Tables {
    uint32_t fac[27], cof[27], desc[27];
};

__device__ __forceinline__ uint32_t float_key(uint32_t u) {
    if (u == 0x80000000u) u = 0u;  // -0.0 == +0.0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

template <int J>
struct Unroll {
    template <typename F>
    __device__ __forceinline__ static void run(F&& fn) {
        Unroll<J - 1>::run(fn);
        fn(std::integral_constant<int, J - 1>());
    }
};
template <>
struct Unroll<0> {
    template <typename F>
    __device__ __forceinline__ static void run(F&&) {}
};

// The nibbles of one lower star are collected in registers (cell j at bits
// 4j..4j+3 of a 128-bit accumulator) and OR-ed into the LDS word tile once
// per destination word at the end (flush).
template <class T>
struct Star {
    static constexpr int OX = T::OX, OY = T::OY, OZ = T::OZ;
    int lx, ly, lz;          // position in the block (0..OX etc.)
    uint32_t* words;         // LDS word tile
    const Tables* tab;
    uint64_t lo = 0, hi = 0;  // nibble of cell j: j < 16 in lo, else in hi
    __device__ void emit(uint32_t j, uint32_t nib) {
        const uint64_t v = (uint64_t)nib << (4u * (j & 15u));
        if (j < 16u) lo |= v;
        else hi |= v;
    }
    __device__ void emit_pair(uint32_t a, uint32_t b) {  // a facet, b cofacet
        int diff = (int)b - (int)a;
        int ad = diff < 0 ? -diff : diff;
        uint32_t axis = ad == 1 ? 0u : (ad == 3 ? 1u : 2u);
        uint32_t neg = diff < 0 ? 1u : 0u;
        emit(a, 1u + 2u * axis + neg);
        emit(b, 1u + 2u * axis + (1u - neg));
    }
    __device__ void emit_crit(uint32_t j) { emit(j, NB_CRIT + (tab->desc[j] & 7u)); }
    // star cell j goes to the word at corner desc(j) & 7, nibble desc(j) >> 3
    __device__ void flush() {
        uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        Unroll<27>::run([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            constexpr uint32_t d = dest_desc(j);
            const uint32_t nib = (uint32_t)((j < 16 ? lo >> (4 * j) : hi >> (4 * (j - 16))) & 15u);
            w[d & 7u] |= nib << (4u * (d >> 3));
        });
        Unroll<8>::run([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            // word (lx - a, ly - b, lz - c) of the tile, which starts one word below the block
            const int wx = lx + 1 - (c & 1), wy = ly + 1 - ((c >> 1) & 1), wz = lz + 1 - ((c >> 2) & 1);
            if (w[c]) atomicOr(&words[wx + (OX + 1) * (wy + (OY + 1) * wz)], w[c]);
        });
    }
};

__device__ __forceinline__ uint32_t ctz32(uint32_t x) { return (uint32_t)__builtin_ctz(x); }

// Rank count over the 26 neighbours: for every pair a < b of star indices
// (centre excluded), d = [K[a] > K[b]] (b precedes a) moves one unit from
// rk[b] to rk[a].  d is a compare into a lane mask that is consumed at once
// as the carry-in of an add and the borrow-in of a subtract: three plain
// VALU operations per pair.  The 325 pairs are taken in the 25 rounds of a
// round-robin schedule (13 disjoint pairs per round), four disjoint pairs
// per block with their masks in separate SGPR pairs, so one block never
// updates a rank twice and the compares of a block are issued before the
// adds that read them (at least three instructions later, more than the two
// wait states gfx950 needs between a VALU write of an SGPR and a VALU read).
struct PairSchedule {
    uint8_t a[325], b[325];
};
__host__ __device__ constexpr int star_of_player(int p) { return p < (int)CENTER ? p : p + 1; }
__host__ __device__ constexpr PairSchedule make_schedule() {
    PairSchedule s{};
    int n = 0;
    for (int r = 0; r < 25; r++) {
        // circle method: players 0..24 rotate, player 25 is fixed
        for (int k = 0; k < 13; k++) {
            int x = k == 0 ? r : (r + k) % 25;
            int y = k == 0 ? 25 : (r - k + 25) % 25;
            int u = star_of_player(x), v = star_of_player(y);
            s.a[n] = (uint8_t)(u < v ? u : v);
            s.b[n] = (uint8_t)(u < v ? v : u);
            n++;
        }
    }
    return s;
}
constexpr PairSchedule kPairs = make_schedule();

__device__ __forceinline__ void rank_pair(uint32_t ka, uint32_t kb, uint32_t& ra, uint32_t& rb) {
    uint64_t m, junk;
    asm("v_cmp_gt_u32_e64 %2, %4, %5\n\t"
        "s_nop 1\n\t"  // two wait states before a VALU reads an SGPR a VALU wrote
        "v_addc_co_u32_e64 %0, %3, %0, 0, %2\n\t"
        "v_subb_co_u32_e64 %1, %3, %1, 0, %2"
        : "+v"(ra), "+v"(rb), "=&s"(m), "=&s"(junk)
        : "v"(ka), "v"(kb));
}

// four disjoint pairs
__device__ __forceinline__ void rank_pair4(uint32_t ka0, uint32_t kb0, uint32_t& ra0, uint32_t& rb0, uint32_t ka1,
                                           uint32_t kb1, uint32_t& ra1, uint32_t& rb1, uint32_t ka2, uint32_t kb2,
                                           uint32_t& ra2, uint32_t& rb2, uint32_t ka3, uint32_t kb3, uint32_t& ra3,
                                           uint32_t& rb3) {
    uint64_t m0, m1, m2, m3, junk;
    asm("v_cmp_gt_u32_e64 %8, %13, %14\n\t"
        "v_cmp_gt_u32_e64 %9, %15, %16\n\t"
        "v_cmp_gt_u32_e64 %10, %17, %18\n\t"
        "v_cmp_gt_u32_e64 %11, %19, %20\n\t"
        "v_addc_co_u32_e64 %0, %12, %0, 0, %8\n\t"
        "v_subb_co_u32_e64 %1, %12, %1, 0, %8\n\t"
        "v_addc_co_u32_e64 %2, %12, %2, 0, %9\n\t"
        "v_subb_co_u32_e64 %3, %12, %3, 0, %9\n\t"
        "v_addc_co_u32_e64 %4, %12, %4, 0, %10\n\t"
        "v_subb_co_u32_e64 %5, %12, %5, 0, %10\n\t"
        "v_addc_co_u32_e64 %6, %12, %6, 0, %11\n\t"
        "v_subb_co_u32_e64 %7, %12, %7, 0, %11"
        : "+v"(ra0), "+v"(rb0), "+v"(ra1), "+v"(rb1), "+v"(ra2), "+v"(rb2), "+v"(ra3), "+v"(rb3), "=&s"(m0),
          "=&s"(m1), "=&s"(m2), "=&s"(m3), "=&s"(junk)
        : "v"(ka0), "v"(kb0), "v"(ka1), "v"(kb1), "v"(ka2), "v"(kb2), "v"(ka3), "v"(kb3));
}

constexpr uint32_t ALLC = ((1u << 27) - 1u) & ~(1u << CENTER);  // every star cell but the centre

// argmin of the cell keys over the set bits of m (m != 0, m within CANDS).
// The keys are packed as (key << 5) | j (keys are below 2^26 and distinct
// within a lower star), so the minimum also names the cell; the scan is
// unrolled over the candidate cells with no branch and no memory access.
template <uint32_t CANDS>
__device__ __forceinline__ uint32_t argmin_key(uint32_t m, const uint32_t (&pk)[27]) {
    uint32_t best = 0xFFFFFFFFu;
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (((CANDS >> j) & 1u) != 0) {
            const uint32_t c = pk[j] | (((m >> j) & 1u) - 1u);  // all ones when j is not in m
            best = best < c ? best : c;
        }
    });
    return best & 31u;
}

// cofacets b of x (inside the lower star, unclassified) with exactly one
// unclassified facet
__device__ __forceinline__ uint32_t ready_cofacets(uint32_t x, uint32_t LS, uint32_t C, const Tables* tab) {
    uint32_t out = 0;
    uint32_t m = tab->cof[x] & LS & ~C;
    while (m) {
        uint32_t b = ctz32(m);
        m &= m - 1;
        if (__builtin_popcount(tab->fac[b] & LS & ~C) == 1) out |= 1u << b;
    }
    return out;
}



// Number of cells in the lower star of the vertex at fidx (the same test as
// in lower_star below); used to give each wave vertices of similar work.
template <class T>
__device__ uint32_t lower_star_size(const uint32_t* fk, int fidx) {
    constexpr int FX = T::FX, FY = T::FY;
    uint32_t K[27];
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int o = off_x(j) + FX * (off_y(j) + FY * off_z(j));
        K[j] = fk[fidx + o];
    });
    const uint32_t kc = K[CENTER];
    uint32_t lower = 0;
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (j != (int)CENTER) {
            bool lw = (j < (int)CENTER) ? (K[j] <= kc) : (K[j] < kc);
            lower |= (lw ? 1u : 0u) << j;
        }
    });
    uint32_t LS = 1u << CENTER;
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (j != (int)CENTER) {
            constexpr uint32_t vm = vert_mask(j);
            LS |= ((vm & ~lower) == 0 ? 1u : 0u) << j;
        }
    });
    return (uint32_t)__builtin_popcount(LS);
}

template <class T>
__device__ void lower_star(const uint32_t* fk, int fidx, Star<T>& st) {
    constexpr int FX = T::FX, FY = T::FY;
    uint32_t K[27];
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int o = off_x(j) + FX * (off_y(j) + FY * off_z(j));
        K[j] = fk[fidx + o];
    });
    const uint32_t kc = K[CENTER];
    uint32_t lower = 0;
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (j != (int)CENTER) {
            bool lw = (j < (int)CENTER) ? (K[j] <= kc) : (K[j] < kc);
            lower |= (lw ? 1u : 0u) << j;
        }
    });
    // cells of the lower star: all their non-centre vertices are lower
    uint32_t LS = 1u << CENTER;
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (j != (int)CENTER) {
            constexpr uint32_t vm = vert_mask(j);
            LS |= ((vm & ~lower) == 0 ? 1u : 0u) << j;
        }
    });
    if ((LS & EDGES) == 0) {  // no lower neighbour: a minimum
        st.emit_crit(CENTER);
        st.flush();
        return;
    }
    // rank of every neighbour in the vertex order (ties broken by id, which
    // among the neighbours of one vertex is the order of the star index):
    // rk[b] starts at the number of non-centre indices below b, and every
    // pair a < b with K[a] > K[b] moves one unit from rk[b] to rk[a]
    uint32_t rk[27];
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        rk[j] = (uint32_t)(j > (int)CENTER ? j - 1 : j);
    });
    Unroll<25>::run([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        Unroll<3>::run([&](auto gc) {
            constexpr int p = 13 * r + 4 * decltype(gc)::value;
            rank_pair4(K[kPairs.a[p]], K[kPairs.b[p]], rk[kPairs.a[p]], rk[kPairs.b[p]], K[kPairs.a[p + 1]],
                       K[kPairs.b[p + 1]], rk[kPairs.a[p + 1]], rk[kPairs.b[p + 1]], K[kPairs.a[p + 2]],
                       K[kPairs.b[p + 2]], rk[kPairs.a[p + 2]], rk[kPairs.b[p + 2]], K[kPairs.a[p + 3]],
                       K[kPairs.b[p + 3]], rk[kPairs.a[p + 3]], rk[kPairs.b[p + 3]]);
        });
        constexpr int p = 13 * r + 12;
        rank_pair(K[kPairs.a[p]], K[kPairs.b[p]], rk[kPairs.a[p]], rk[kPairs.b[p]]);
    });
    uint32_t pk[27];
    pk[CENTER] = 0xFFFFFFFFu;
    // cell keys: bit set of the ranks of the cell's other vertices; comparing
    // them as integers is the lexicographic comparison of the descending
    // vertex lists with a proper prefix smaller
    Unroll<27>::run([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (j != (int)CENTER) {
            uint32_t key = 0;
            Unroll<27>::run([&](auto vc) {
                constexpr int v = decltype(vc)::value;
                if constexpr (((vert_mask(j) >> v) & 1u) != 0) key |= 1u << rk[v];
            });
            pk[j] = (key << 5) | (uint32_t)j;
        }
    });
    const Tables* tab = st.tab;
    uint32_t C = 1u << CENTER;  // classified cells
    uint32_t E = LS & EDGES;
    uint32_t delta = argmin_key<EDGES>(E, pk);
    st.emit_pair(CENTER, delta);
    C |= 1u << delta;
    uint32_t PZ = E & ~(1u << delta);
    uint32_t PO = ready_cofacets(delta, LS, C, tab);
    for (;;) {
        while (PO) {
            uint32_t a = argmin_key<ALLC & ~EDGES>(PO, pk);  // only quads and cubes enter PQone
            PO &= ~(1u << a);
            if (C & (1u << a)) continue;
            uint32_t uf = tab->fac[a] & LS & ~C;
            if (!uf) {
                PZ |= 1u << a;
                continue;
            }
            uint32_t p = ctz32(uf);
            st.emit_pair(p, a);
            C |= (1u << a) | (1u << p);
            PZ &= ~(1u << p);
            PO |= ready_cofacets(a, LS, C, tab) | ready_cofacets(p, LS, C, tab);
        }
        PZ &= ~C;
        if (!PZ) break;
        uint32_t g = argmin_key<ALLC>(PZ, pk);
        PZ &= ~(1u << g);
        st.emit_crit(g);
        C |= 1u << g;
        PO |= ready_cofacets(g, LS, C, tab);
    }
    st.flush();
}

// One workgroup per tile; tiles of all fields of a batch are numbered
// consecutively (tile_off: first tile of each field).
template <class T>
__global__ __launch_bounds__(THREADS) void grad_lowerstar(const float* __restrict__ f0,
                                                           const float* const* __restrict__ fptr, Geo geo,
                                                           const uint32_t* __restrict__ tile_off,
                                                           uint32_t total_tiles, uint32_t* __restrict__ grad_all,
                                                           int* __restrict__ err) {
    constexpr int OX = T::OX, OY = T::OY, OZ = T::OZ, FX = T::FX, FY = T::FY, NF = T::NF, NW = T::NW;
    constexpr int WX = T::WX, WY = T::WY, NV = T::NV;
    __shared__ uint32_t fk[NF];
    __shared__ uint32_t words[NW];
    __shared__ Tables tab;
    __shared__ uint8_t s_size[NV];
    __shared__ uint16_t s_ord[NV];
    __shared__ uint32_t s_cnt[32];
    const int tid = threadIdx.x;
    // Workgroups are dealt to the 8 XCDs round-robin; block b takes tile
    // (b % 8) * per + b / 8, so each XCD works through a contiguous slab of
    // tiles and the tiles' halos are shared in that XCD's L2.
    const uint32_t per = (total_tiles + NXCD - 1) / NXCD;
    uint32_t t = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
    if (t >= total_tiles) return;
    uint32_t fld = 0;
    if (geo.nf > 1) {
        uint32_t lo = 0, hi = geo.nf;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (tile_off[mid] <= t) lo = mid;
            else hi = mid;
        }
        fld = lo;
        t -= tile_off[fld];
    }
    const Grid g = geo.grid(fld);
    const float* __restrict__ f = fptr ? fptr[fld] : f0;
    uint32_t* __restrict__ grad = grad_all + geo.base(fld);
    const uint32_t ntx = (g.n[0] + OX - 1) / OX, nty = (g.n[1] + OY - 1) / OY;
    const uint32_t tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    const int x0 = (int)(tx * OX), y0 = (int)(ty * OY), z0 = (int)(tz * OZ);
    const int nx = (int)g.n[0], ny = (int)g.n[1], nz = (int)g.n[2];

    if (tid < 27) {
        tab.fac[tid] = facet_mask(tid);
        tab.cof[tid] = cofacet_mask(tid);
        tab.desc[tid] = dest_desc(tid);
    }
    bool bad = false;
    for (int i = tid; i < NF; i += THREADS) {
        int fx = i % FX, fy = (i / FX) % FY, fz = i / (FX * FY);
        int x = x0 - 1 + fx, y = y0 - 1 + fy, z = z0 - 1 + fz;
        uint32_t key = KEY_OUT;
        if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) {
            uint32_t u = __float_as_uint(load_global(f, (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z)));
            if ((u & 0x7F800000u) == 0x7F800000u) bad = true;
            key = float_key(u);
        }
        fk[i] = key;
    }
    if (bad) atomicOr(err, 1);
    for (int i = tid; i < NW; i += THREADS) words[i] = 0u;
    __syncthreads();

    // The pairing loop's length grows with the lower star, and a wave runs as
    // long as its largest one: order the tile's vertices by lower-star size
    // (counting sort in LDS) so that each wave gets vertices of similar size.
    // Nibbles are OR-ed into the word tile, so the order does not matter.
    if (tid < 32) s_cnt[tid] = 0;
    __syncthreads();
    for (int i = tid; i < NV; i += THREADS) {
        int lx = i % OX, ly = (i / OX) % OY, lz = i / (OX * OY);
        int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        uint32_t sz = 0;  // vertices outside the grid: size 0, skipped below
        if (x < nx && y < ny && z < nz) sz = lower_star_size<T>(fk, (lx + 1) + FX * ((ly + 1) + FY * (lz + 1)));
        s_size[i] = (uint8_t)sz;
        atomicAdd(&s_cnt[sz], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int b = 0; b < 32; b++) {
            uint32_t c = s_cnt[b];
            s_cnt[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = tid; i < NV; i += THREADS) s_ord[atomicAdd(&s_cnt[s_size[i]], 1u)] = (uint16_t)i;
    __syncthreads();
    for (int k = tid; k < NV; k += THREADS) {
        const int i = s_ord[k];
        if (s_size[i] == 0) continue;
        int lx = i % OX, ly = (i / OX) % OY, lz = i / (OX * OY);
        Star<T> st{lx, ly, lz, words, &tab};
        int fidx = (lx + 1) + FX * ((ly + 1) + FY * (lz + 1));
        lower_star(fk, fidx, st);
    }
    __syncthreads();

    for (int i = tid; i < NW; i += THREADS) {
        // tile word (wx, wy, wz) is word (x0 - 1 + wx, ...) of the grid
        int wx = i % WX, wy = (i / WX) % WY, wz = i / (WX * WY);
        int x = x0 - 1 + wx, y = y0 - 1 + wy, z = z0 - 1 + wz;
        if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) continue;
        uint32_t w = words[i];
        if (x == nx - 1) w |= 0x70707070u;  // cells with an odd X beyond the grid
        if (y == ny - 1) w |= 0x77007700u;
        if (z == nz - 1) w |= 0x77770000u;
        uint32_t* dst = &grad[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z)];
        // a word of the block's interior (its vertex and +x/+y/+z neighbours
        // all in the block) has all its nibbles here; any other word also
        // gets nibbles from a neighbouring block
        const bool whole = wx >= 1 && wx < OX && wy >= 1 && wy < OY && wz >= 1 && wz < OZ;
        if (whole) *dst = w;
        else if (w) atomicOr(dst, w);
    }
}

// Clears the gradient words (four per thread; 16-byte stores when aligned).
__global__ __launch_bounds__(THREADS) void k_zero_words(uint32_t* __restrict__ grad, uint64_t nv) {
    const uint64_t q = (uint64_t)blockIdx.x * THREADS + threadIdx.x;
    const uint64_t i = 4 * q;
    if (i >= nv) return;
    if (i + 4 <= nv && ((uintptr_t)(grad + i) & 15u) == 0) {
        *reinterpret_cast<uint4*>(grad + i) = make_uint4(0u, 0u, 0u, 0u);
    } else {
        for (uint64_t j = i; j < nv && j < i + 4; j++) grad[j] = 0u;
    }
}

using T0 = Tile<16, 8, 4>;
using T1 = Tile<32, 4, 4>;
using T2 = Tile<8, 8, 8>;
using T3 = Tile<16, 16, 2>;
using T4 = Tile<16, 8, 8>;
using T5 = Tile<16, 16, 8>;
using T6 = Tile<32, 16, 8>;

template <class T>
uint32_t tiles_of(const Grid& g) {
    return ((g.n[0] + T::OX - 1) / T::OX) * ((g.n[1] + T::OY - 1) / T::OY) * ((g.n[2] + T::OZ - 1) / T::OZ);
}

}  // namespace

// tiles of one field for tile shape `shape` (0..6)
uint32_t gradient_tiles(const Grid& g, int shape) {
    switch (shape) {
        case 1: return tiles_of<T1>(g);
        case 2: return tiles_of<T2>(g);
        case 3: return tiles_of<T3>(g);
        case 4: return tiles_of<T4>(g);
        case 5: return tiles_of<T5>(g);
        case 6: return tiles_of<T6>(g);
        default: return tiles_of<T0>(g);
    }
}

// f0: the field when fptr is null; otherwise fptr / tile_off (device arrays)
// give each field's data and first tile, and total_tiles the sum.
hipError_t launch_gradient(int shape, const float* f0, const float* const* fptr, const Geo& geo,
                           const uint32_t* tile_off, uint64_t total_tiles, uint32_t* grad, int* err, hipStream_t s) {
    if (total_tiles == 0) return hipSuccess;
    // words on block faces are OR-ed together from several blocks
    hipLaunchKernelGGL(k_zero_words, dim3(grid_blocks((geo.nv + 3) / 4, THREADS)), dim3(THREADS), 0, s, grad,
                       (uint64_t)geo.nv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t tt = (uint32_t)total_tiles;
    dim3 gd((unsigned)(NXCD * ((tt + NXCD - 1) / NXCD))), bd(THREADS);
    switch (shape) {
        case 1: hipLaunchKernelGGL(grad_lowerstar<T1>, gd, bd, 0, s, f0, fptr, geo, tile_off, tt, grad, err); break;
        case 2: hipLaunchKernelGGL(grad_lowerstar<T2>, gd, bd, 0, s, f0, fptr, geo, tile_off, tt, grad, err); break;
        case 3: hipLaunchKernelGGL(grad_lowerstar<T3>, gd, bd, 0, s, f0, fptr, geo, tile_off, tt, grad, err); break;
        case 4: hipLaunchKernelGGL(grad_lowerstar<T4>, gd, bd, 0, s, f0, fptr, geo, tile_off, tt, grad, err); break;
        case 5: hipLaunchKernelGGL(grad_lowerstar<T5>, gd, bd, 0, s, f0, fptr, geo, tile_off, tt, grad, err); break;
        case 6: hipLaunchKernelGGL(grad_lowerstar<T6>, gd, bd, 0, s, f0, fptr, geo, tile_off, tt, grad, err); break;
        default: hipLaunchKernelGGL(grad_lowerstar<T0>, gd, bd, 0, s, f0, fptr, geo, tile_off, tt, grad, err); break;
    }
    return hipGetLastError();
}

}  // namespace msc

// Pieces shared by the fused RHS + RK3 kernels: precision traits, the
// unscaled stencil sums of order 2r (Section 4, Eq. stencil-fd) and the
// per-cell 2N update with its FP32 compensated variant.
#pragma once

#include <functional>
#include <queue>
#include <vector>

#include "mhd_internal.hpp"

namespace mhd {

// T: storage type.  Rt: type of first derivatives and of the physics.
// D2: type in which second-derivative stencil sums are accumulated.
template <int PREC>
struct Prec;
template <>
struct Prec<MHD_F64> {
    using T = double;
    using Rt = double;
    using D2 = double;
};
template <>
struct Prec<MHD_F32C> {
    using T = float;
    using Rt = float;
    using D2 = double;
};
template <>
struct Prec<MHD_F32> {
    using T = float;
    using Rt = float;
    using D2 = float;
};

// First derivative times h along a stride st (radius RAD).
template <typename A, int RAD, typename T>
__device__ __forceinline__ A deriv1(const T* p, int st)
{
    A acc = A(W1(RAD, 1) / DEN1(RAD)) * (A(p[st]) - A(p[-st]));
#pragma unroll
    for (int m = 2; m <= RAD; ++m) acc += A(W1(RAD, m) / DEN1(RAD)) * (A(p[m * st]) - A(p[-m * st]));
    return acc;
}

// Pure second derivative times h^2 along a stride st.
template <typename A, int RAD, typename T>
__device__ __forceinline__ A deriv2(const T* p, int st)
{
    A acc = A(W2(RAD, 0) / DEN2(RAD)) * A(p[0]);
#pragma unroll
    for (int m = 1; m <= RAD; ++m) acc += A(W2(RAD, m) / DEN2(RAD)) * (A(p[m * st]) + A(p[-m * st]));
    return acc;
}

// Mixed second derivative times h_a h_b from the diagonals of the plane
// spanned by strides sa, sb: difference of the second differences along
// (+1, +1) and (+1, -1), divided by 4.
template <typename A, int RAD, typename T>
__device__ __forceinline__ A derivm(const T* p, int sa, int sb)
{
    const int pp = sa + sb, pm = sa - sb;
    A acc = A(0);
#pragma unroll
    for (int m = 1; m <= RAD; ++m) {
        const A e = (A(p[m * pp]) + A(p[-m * pp])) - (A(p[m * pm]) + A(p[-m * pm]));
        acc += A(W2(RAD, m) / (4.0 * DEN2(RAD))) * e;
    }
    return acc;
}

// 2N update of one cell of one field, by value: returns the new register
// value and the new state (and, for the compensated FP32 variant, updates the
// compensation c).  w_old is ignored for s == 0 (alpha_0 = 0).
template <int PREC>
__device__ __forceinline__ void rk_values(int s, typename Prec<PREC>::T f_in,
                                          typename Prec<PREC>::T w_old,
                                          typename Prec<PREC>::Rt rhs, double dt,
                                          typename Prec<PREC>::T& w_new,
                                          typename Prec<PREC>::T& f_new,
                                          typename Prec<PREC>::T& c)
{
    using T = typename Prec<PREC>::T;
    using Rt = typename Prec<PREC>::Rt;
    const Rt alpha = Rt(s == 1 ? RK_ALPHA[1] : RK_ALPHA[2]);
    const Rt beta = Rt(s == 0 ? RK_BETA[0] : (s == 1 ? RK_BETA[1] : RK_BETA[2]));
    const Rt dtr = Rt(dt);
    const Rt wn = (s == 0) ? dtr * rhs : alpha * Rt(w_old) + dtr * rhs;
    w_new = T(wn);
    if constexpr (PREC == MHD_F32C) {
        f_new = kahan_add(f_in, beta * wn, c);
    } else {
        f_new = T(f_in + beta * wn);
    }
}

// 2N update of one cell of one field with the old register value w_old
// already loaded (ignored for s == 0: alpha_0 = 0, so w is never read).
template <int PREC>
__device__ __forceinline__ void rk_update_v(int s, typename Prec<PREC>::T f_in,
                                            typename Prec<PREC>::T w_old,
                                            typename Prec<PREC>::Rt rhs, double dt,
                                            typename Prec<PREC>::T* w,
                                            typename Prec<PREC>::T* f_out,
                                            typename Prec<PREC>::T* comp)
{
    using T = typename Prec<PREC>::T;
    using Rt = typename Prec<PREC>::Rt;
    const Rt alpha = Rt(s == 1 ? RK_ALPHA[1] : RK_ALPHA[2]);
    const Rt beta = Rt(s == 0 ? RK_BETA[0] : (s == 1 ? RK_BETA[1] : RK_BETA[2]));
    const Rt dtr = Rt(dt);
    const Rt wn = (s == 0) ? dtr * rhs : alpha * Rt(w_old) + dtr * rhs;
    *w = T(wn);
    if constexpr (PREC == MHD_F32C) {
        float c = *comp;
        *f_out = kahan_add(f_in, beta * wn, c);
        *comp = c;
    } else {
        *f_out = T(f_in + beta * wn);
    }
}

// 2N update of one cell of one field.  s == 0 never reads w (alpha_0 = 0).
template <int PREC>
__device__ __forceinline__ void rk_update(int s, typename Prec<PREC>::T f_in,
                                          typename Prec<PREC>::Rt rhs, double dt,
                                          typename Prec<PREC>::T* w,
                                          typename Prec<PREC>::T* f_out,
                                          typename Prec<PREC>::T* comp)
{
    using T = typename Prec<PREC>::T;
    rk_update_v<PREC>(s, f_in, s == 0 ? T(0) : *w, rhs, dt, w, f_out, comp);
}

// ------------------------------------------------------------ tile plans
// One launch of an LDS kernel updates a set of up to MAX_BOXES disjoint
// boxes (one box, or the six slabs of the segmented iteration's outer shell
// together), each cut into TX x TY tile columns marched through z in chunks
// of zc planes.  Tiles are numbered box after box; within a box
// tile = (chunk * nty + ty) * ntx + tx.
constexpr int MAX_BOXES = 6;
constexpr int NO_TILE = -1;
constexpr int ZCHUNK_MIN = 16, WARM_PLANES = 7;

struct TilePlan {
    int nbox;
    int round;                 // workgroups resident at once (0: plain order)
    int tiles;                 // tiles of all boxes
    int first[MAX_BOXES + 1];  // first tile of each box; first[nbox] == tiles
    Box box[MAX_BOXES];
    int ntx[MAX_BOXES], nty[MAX_BOXES], nch[MAX_BOXES], zc[MAX_BOXES];
};

// Z chunks.  The hardware hands workgroups to free slots in launch order,
// so a launch lasts about the makespan of greedy list scheduling of its
// chunks (each taking its planes plus the warm-up planes) on the `round`
// resident slots; tiles are numbered longest chunk first, so that the short
// chunks (thin slabs) fill the gaps the long ones leave (for one box: whole
// rounds of equal chunks).  Thin boxes and tile counts just above a whole
// number of rounds march in the common chunk length Z of least makespan:
// every box of more than Z planes is cut into chunks of at most Z planes, no
// chunk below ZCHUNK_MIN planes unless its box is.  Candidates: each box's
// own length over 1, 2, ... chunks.
inline int64_t greedy_makespan(int n, const int64_t* jobs, const int* len, int round)
{
    std::priority_queue<int64_t, std::vector<int64_t>, std::greater<int64_t>> slots;
    for (int i = 0; i < round; ++i) slots.push(0);
    int64_t end = 0;
    for (int k = 0; k < n; ++k)
        for (int64_t i = 0; i < jobs[k]; ++i) {
            const int64_t t = slots.top() + len[k];
            slots.pop();
            slots.push(t);
            end = t > end ? t : end;
        }
    return end;
}

inline TilePlan plan_tiles_uncached(const Box* b, int n, int tx, int ty, int round)
{
    TilePlan p{};
    p.nbox = n;
    p.round = round;
    int64_t cols[MAX_BOXES];
    int nzb[MAX_BOXES], nch[MAX_BOXES], zc[MAX_BOXES], zmax = 0;
    for (int k = 0; k < n; ++k) {
        cols[k] = (int64_t)((b[k].x1 - b[k].x0 + tx - 1) / tx) * ((b[k].y1 - b[k].y0 + ty - 1) / ty);
        nzb[k] = b[k].z1 - b[k].z0;
        nch[k] = 1;
        zc[k] = nzb[k];
        zmax = nzb[k] > zmax ? nzb[k] : zmax;
    }
    // boxes in order of falling chunk length (stable), jobs and lengths per box
    auto order_of = [&](const int* z, int* ord) {
        for (int k = 0; k < n; ++k) ord[k] = k;
        for (int a = 1; a < n; ++a)
            for (int c = a; c > 0 && z[ord[c]] > z[ord[c - 1]]; --c) {
                const int t = ord[c];
                ord[c] = ord[c - 1];
                ord[c - 1] = t;
            }
    };
    if (round > 0) {
        int64_t best = -1;
        int tried[64], ntried = 0;
        for (int want = 1; want == 1 || want <= zmax / ZCHUNK_MIN; ++want) {
            for (int j = 0; j < n; ++j) {
                if (want > 1 && want > nzb[j] / ZCHUNK_MIN) continue;
                const int Z = (nzb[j] + want - 1) / want;
                bool seen = false;
                for (int t = 0; t < ntried; ++t) seen |= tried[t] == Z;
                if (seen) continue;
                if (ntried < 64) tried[ntried++] = Z;
                int cn[MAX_BOXES], cz[MAX_BOXES], ord[MAX_BOXES], len[MAX_BOXES];
                int64_t jobs[MAX_BOXES];
                for (int k = 0; k < n; ++k) {
                    cn[k] = nzb[k] > Z ? (nzb[k] + Z - 1) / Z : 1;
                    cz[k] = (nzb[k] + cn[k] - 1) / cn[k];
                }
                order_of(cz, ord);
                for (int k = 0; k < n; ++k) {
                    jobs[k] = cols[ord[k]] * cn[ord[k]];
                    len[k] = cz[ord[k]] + WARM_PLANES;
                }
                const int64_t cost = greedy_makespan(n, jobs, len, round);
                if (best < 0 || cost < best) {
                    best = cost;
                    for (int k = 0; k < n; ++k) {
                        nch[k] = cn[k];
                        zc[k] = cz[k];
                    }
                }
            }
        }
    }
    int ord[MAX_BOXES];
    order_of(zc, ord);
    p.first[0] = 0;
    for (int i = 0; i < n; ++i) {
        const int k = ord[i];
        p.box[i] = b[k];
        p.ntx[i] = (b[k].x1 - b[k].x0 + tx - 1) / tx;
        p.nty[i] = (b[k].y1 - b[k].y0 + ty - 1) / ty;
        p.nch[i] = nch[k];
        p.zc[i] = zc[k];
        p.first[i + 1] = p.first[i] + (int)(cols[k] * nch[k]);
    }
    p.tiles = p.first[n];
    return p;
}

// The plans of the last few distinct launches are kept (per host thread):
// a step driver asks for the same few box sets again and again.
inline TilePlan plan_tiles(const Box* b, int n, int tx, int ty, int round)
{
    struct Entry {
        bool used;
        int n, tx, ty, round;
        Box b[MAX_BOXES];
        TilePlan plan;
    };
    thread_local Entry cache[8] = {};
    thread_local int next = 0;
    for (Entry& e : cache) {
        if (!e.used || e.n != n || e.tx != tx || e.ty != ty || e.round != round) continue;
        bool same = true;
        for (int k = 0; k < n && same; ++k)
            same = e.b[k].x0 == b[k].x0 && e.b[k].x1 == b[k].x1 && e.b[k].y0 == b[k].y0 &&
                   e.b[k].y1 == b[k].y1 && e.b[k].z0 == b[k].z0 && e.b[k].z1 == b[k].z1;
        if (same) return e.plan;
    }
    Entry& e = cache[next];
    next = (next + 1) % 8;
    e.used = true;
    e.n = n;
    e.tx = tx;
    e.ty = ty;
    e.round = round;
    for (int k = 0; k < n; ++k) e.b[k] = b[k];
    e.plan = plan_tiles_uncached(b, n, tx, ty, round);
    return e.plan;
}

// Workgroups of a launch: with the XCD mapping the last round may name
// tiles past the end, and those workgroups exit at once.
inline int plan_blocks(const TilePlan& p)
{
    return (p.round > 0 && (p.round & 7) == 0) ? (p.tiles + p.round - 1) / p.round * p.round
                                               : p.tiles;
}

// Workgroup b -> tile.  Hardware hands consecutive workgroups to the 8 XCDs
// in turn; within one round of `round` resident workgroups, XCD k gets the
// k-th contiguous run of tiles, so the tiles that run together on one XCD
// (sharing its L2) are spatial neighbours, and a round covers a compact
// band of tile rows.
__device__ __forceinline__ int tile_of_block(int b, int tiles, int round)
{
    if (round <= 0 || (round & 7) != 0) return b < tiles ? b : NO_TILE;
    const int r = b / round, w = b - r * round;
    const int rem = min(tiles - r * round, round);  // tiles in this round
    const int per = (rem + 7) >> 3;                  // tiles per XCD in this round
    const int k = w >> 3;
    if (k >= per) return NO_TILE;
    const int t = r * round + (w & 7) * per + k;
    return t < r * round + rem ? t : NO_TILE;
}

// Whether the split kernel may fetch its halo'd planes as aligned pairs of
// x-neighbours: the padded row length is even (so are a plane and a field),
// every box starts at an even x, and f_in is aligned to two elements, so
// every pair the tiles fetch starts on a two-element boundary.
inline bool pairs_aligned(const Grid& g, const Box* bx, int nbox, const void* f_in, size_t elem)
{
    if (g.mx % 2 != 0 || g.fstride % 2 != 0) return false;
    if (reinterpret_cast<uintptr_t>(f_in) % (2 * elem) != 0) return false;
    for (int k = 0; k < nbox; ++k)
        if (bx[k].x0 % 2 != 0) return false;
    return true;
}

// One box's tile grid, as a single-box launch passes it.
struct TileMap {
    int ntx, nty;  // tiles per axis
    int nch, zc;   // z chunks per tile column, planes per chunk
    int round;     // workgroups resident at once (0: plain order)
};

__device__ __forceinline__ int tile_of_block(int b, const TileMap& m)
{
    return tile_of_block(b, m.ntx * m.nty * m.nch, m.round);
}

inline TileMap plan_map(const TilePlan& p)
{
    return TileMap{p.ntx[0], p.nty[0], p.nch[0], p.zc[0], p.round};
}

// The box of a tile (a uniform value: the whole workgroup agrees).
__device__ __forceinline__ int box_of_tile(int tile, const TilePlan& p)
{
    int k = 0;
#pragma unroll
    for (int j = 1; j < MAX_BOXES; ++j) k += (j < p.nbox && tile >= p.first[j]) ? 1 : 0;
    return k;
}

// Box kb (uniform) of a plan and the tile's index within it.  The fields
// are read through a pointer into the kernel argument with the box index as
// a scalar offset, so only the box in use occupies scalar registers.
__device__ __forceinline__ void plan_box(const TilePlan& p, int kb, int tile_g, int& x0, int& x1,
                                         int& y0, int& y1, int& z0, int& z1, int& ntx, int& nty,
                                         int& zc, int& tile)
{
    const int k = __builtin_amdgcn_readfirstlane(kb);
    const TilePlan* pp = &p;
    const Box b = pp->box[k];
    x0 = b.x0; x1 = b.x1; y0 = b.y0; y1 = b.y1; z0 = b.z0; z1 = b.z1;
    ntx = pp->ntx[k];
    nty = pp->nty[k];
    zc = pp->zc[k];
    tile = tile_g - pp->first[k];
}

}  // namespace mhd

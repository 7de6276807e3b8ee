// Fused RHS + RK3 substep, LDS-tiled z-marching kernel for gfx950, templated
// on the stencil radius RAD = 1..4 (orders 2, 4, 6, 8 of Section 4).
//
// A workgroup of 256 threads owns a TX x TY = 32 x 8 column tile (32 x 4 and
// 128 threads for FP64 at RAD = 4) and marches it through the nz planes of
// its box, one interior cell per thread per plane.
//
// On-chip data flow (sixth order, FP64: 136 KB of LDS, one workgroup per CU):
//   * LDS ring of RAD + 1 halo'd planes (t .. t+RAD) of all 8 fields, each
//     plane the tile plus a RAD-cell halo in x and y (38 x 14 cells at
//     RAD = 3).  Plane t+RAD+2 is fetched into registers while plane t is
//     computed; plane t+RAD+1 (fetched one iteration earlier) replaces plane
//     t in the ring at the end of the iteration, so the HBM stream overlaps
//     the arithmetic.
//   * x/y first, second and xy-mixed derivatives of plane t read the
//     plane-t slot (axis lines and planar diagonals of Eq. stencil-fd).
//   * z derivatives use the thread's own column: planes t-RAD..t-1 from a
//     RAD-deep register history, planes t..t+RAD from the ring.
//   * The xz / yz mixed derivatives are differences of x (or y) differences
//     taken on planes t +- m:  Dxz f(t) = sum_m w_m [d_m(t+m) - d_m(t-m)],
//     d_m(p) = f(x+m, p) - f(x-m, p).  The t+m halves come from the ring;
//     the t-m halves were formed when plane t-m was current (they are the
//     same differences D_x needs there) and are carried in RAD running
//     accumulators per mixed combination.
// Each input value is fetched from HBM once per tile plus the tile halo;
// neighbouring tiles of one round run concurrently on the same XCD (see
// tile_of_block), so halo fetches mostly hit its L2.
//
// Stencil weights are the integers W1, W2 of the central formulas of order
// 2r (exact as f64/f32 literals) with one scale factor per axis or plane:
//   D_a f  = [sum_m W1(m) d_m] / (DEN1 h_a)                 (45, -9, 1; 60 at r = 3)
//   D_aa f = [W2(0) f0 + sum_m W2(m) s_m] / (DEN2 h_a^2)    (-490, 270, -27, 2; 180)
//   D_ab f = [sum_m W2(m) e_m] / (4 DEN2 h_a h_b)
// The right-hand side assembly and the 2N update are the same as in the
// direct kernel (Appendix B; Williamson RK3).
#include <type_traits>

#include "mhd_internal.hpp"
#include "rk3_common.hpp"

namespace mhd {
namespace {

#ifndef MHD_TILED_TX
#define MHD_TILED_TX 32
#endif
constexpr int TX = MHD_TILED_TX;
// Per precision and stencil radius RAD: the tile (TX x TY cells, one thread
// each), the halo'd tile plane (38 x 14 = 532 cells at RAD = 3) and the LDS
// ring of RAD + 1 such planes of all 8 fields.  FP64 at RAD = 4 uses a
// 32 x 4 tile: its ring of five 40 x 12 planes (150 KB) fits the 160 KB of
// LDS where five 40 x 16 planes (200 KB) would not.
template <int PREC, int RAD>
struct Ring {
    static constexpr int TY = (PREC == MHD_F64 && RAD == 4) ? 128 / TX : 256 / TX;
    static constexpr int NT = TX * TY;
    static constexpr int HX = TX + 2 * RAD, HY = TY + 2 * RAD, PLANE = HX * HY;
    static constexpr int SLOT = NQ * PLANE;
    static constexpr int NSLOT = RAD + 1;
    static constexpr int FULL = PLANE / NT;   // plane elements every thread loads
    static constexpr int EXTRA = PLANE % NT;  // threads that load one more element
};
// Scheduling fences between the per-field derivative phases (bit i: after
// phase i) bound the live ranges of the LDS reads the scheduler may hoist.
#ifndef MHD_TILED_FENCES
#define MHD_TILED_FENCES 0xFF
#endif
constexpr unsigned FENCE_MASK = MHD_TILED_FENCES;
#ifndef MHD_TILED_F32_BLOCKS
#define MHD_TILED_F32_BLOCKS 1
#endif

template <int PREC, int RAD>
constexpr size_t lds_bytes()
{
    return sizeof(typename Prec<PREC>::T) * Ring<PREC, RAD>::NSLOT * Ring<PREC, RAD>::SLOT;
}

// Per-axis scale factors of the integer-weight stencils.
// (Sized by the radius: the kernel keeps these in scalar registers.)
template <int RAD>
struct Scales {
    double d1[3];     // 1/(DEN1 h_a)
    double d2[3];     // 1/(DEN2 h_a^2)
    double mxy;       // 1/(4 DEN2 h_x h_y)
    double wxz[RAD];  // W2(r, m)/(4 DEN2 h_x h_z), m = 1..r
    double wyz[RAD];  // W2(r, m)/(4 DEN2 h_y h_z)
};

// FP64 needs most of a CU's LDS for one workgroup's ring.  The FP32 rings
// are half that size, but two resident workgroups would cap a lane at 256
// registers, and the FP64 second-derivative sums of the FP32 variants then
// spill (measured at 512^3: 7.0 GCUPS with two workgroups per CU against
// 13.6 with one), so both are built for one.
template <int PREC>
constexpr int blocks_per_cu() { return PREC == MHD_F64 ? 1 : MHD_TILED_F32_BLOCKS; }

// MULTI: the launch covers the several boxes of `plan` and each workgroup
// takes its box and tile grid from there; otherwise one box, `box` and `map`
// (a separate instantiation, so that the single-box march is compiled as if
// the plan did not exist).
template <int PREC, int RAD, bool MULTI>
__global__ __launch_bounds__((Ring<PREC, RAD>::NT), blocks_per_cu<PREC>()) void k_rk3_tiled(Grid g, Phys P, Scales<RAD> sc, TileMap map, int s,
                                                     const typename Prec<PREC>::T* __restrict__ fin,
                                                     typename Prec<PREC>::T* __restrict__ fout,
                                                     typename Prec<PREC>::T* __restrict__ w,
                                                     typename Prec<PREC>::T* __restrict__ comp,
                                                     double dt, Box box, TilePlan plan)
{
    int multi_tile = 0;
    if constexpr (MULTI) {
        const int tile_g = tile_of_block(blockIdx.x, plan.tiles, plan.round);
        if (tile_g == NO_TILE) return;  // the whole workgroup exits together
        int x0, x1, y0, y1, z0, z1, ntx, nty, zc;
        plan_box(plan, box_of_tile(tile_g, plan), tile_g, x0, x1, y0, y1, z0, z1, ntx, nty, zc,
                 multi_tile);
        box = Box{x0, x1, y0, y1, z0, z1};
        map.ntx = ntx;
        map.nty = nty;
        map.zc = zc;
    }
    // the box's bounds as plain scalars (a struct captured by the lambdas
    // below costs registers)
    const int bx0 = box.x0, bx1 = box.x1, by0 = box.y0, by1 = box.y1;
    using T = typename Prec<PREC>::T;
    using Rt = typename Prec<PREC>::Rt;
    using D2 = typename Prec<PREC>::D2;
    using RG = Ring<PREC, RAD>;
    constexpr int TY = RG::TY, NT = RG::NT, HX = RG::HX, PLANE = RG::PLANE, SLOT = RG::SLOT;
    constexpr int NSLOT = RG::NSLOT, FULL = RG::FULL, EXTRA = RG::EXTRA;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* __restrict__ lds = reinterpret_cast<T*>(smem_raw);

    const int tile = MULTI ? multi_tile : tile_of_block(blockIdx.x, map);
    if (tile == NO_TILE) return;  // the whole workgroup exits together
    // tile = (chunk * nty + ty) * ntx + tx; the chunk marches its own z range
    const int per_chunk = map.ntx * map.nty, ch = tile / per_chunk, txy = tile - ch * per_chunk;
    const int tx = txy % map.ntx, ty = txy / map.ntx;
    const int bz0 = box.z0 + ch * map.zc, bz1 = min(bz0 + map.zc, box.z1);
    const int x0 = bx0 + tx * TX, y0 = by0 + ty * TY;
    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const bool active = (x0 + lx < bx1) && (y0 + ly < by1);
    const bool extra = tid < EXTRA;

    // Global addressing: a uniform field base plus a 32-bit byte offset (every
    // padded field is below 4 GiB), so loads and stores use the SGPR-base form.
    auto field_ptr = [&](auto* base, int q) { return base + q * g.fstride; };
    auto at = [](auto* p, unsigned idx) {
        using P = decltype(p);
        using C = typename std::conditional<std::is_const<typename std::remove_pointer<P>::type>::value,
                                            const char*, char*>::type;
        return reinterpret_cast<P>(reinterpret_cast<C>(p) + idx * (unsigned)sizeof(T));
    };

    // ---- per-thread load slots: elements tid, tid + 256 (and tid + 512 for
    // the first EXTRA threads) of the halo'd tile plane, clamped into the
    // padded grid for ragged tiles
    constexpr int NLOAD = FULL + (EXTRA > 0 ? 1 : 0);
    unsigned goff[NLOAD];
#pragma unroll
    for (int k = 0; k < NLOAD; ++k) {
        const int e = min(tid + k * NT, PLANE - 1);
        const int r = e / HX, c = e - r * HX;
        const int px = min(x0 + c, g.mx - 1), py = min(y0 + r, g.my - 1);
        goff[k] = (unsigned)(py * g.mx + px);
    }

    T pre[NQ][NLOAD];
    auto load_plane = [&](int t) {  // t: interior plane index, -RAD .. nz+RAD-1
        const unsigned zo = (unsigned)((t + RAD) * g.mxy);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T* f = field_ptr(fin, q);
#pragma unroll
            for (int k = 0; k < FULL; ++k) pre[q][k] = *at(f, goff[k] + zo);
        }
        if constexpr (EXTRA > 0) {
            if (extra) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) pre[q][FULL] = *at(field_ptr(fin, q), goff[FULL] + zo);
            }
        }
    };
    auto store_plane = [&](int slot) {
        T* base = lds + slot * SLOT + tid;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int k = 0; k < FULL; ++k) base[q * PLANE + k * NT] = pre[q][k];
        if constexpr (EXTRA > 0) {
            if (extra) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) base[q * PLANE + FULL * NT] = pre[q][FULL];
            }
        }
    };

    // V(slot, q, dy, dx): field q of the ring slot at offset (dx, dy) from the
    // thread's cell.  Addressed from the cell's stencil corner so that every
    // offset is a non-negative constant the LDS instructions take as an immediate.
    const int corner = ly * HX + lx;  // cell (x - RAD, y - RAD) within a plane
    auto V = [&](int slot, int q, int dy, int dx) -> T {
        return lds[(slot * SLOT + corner) + (q * PLANE + (dy + RAD) * HX + (dx + RAD))];
    };

    // ---- z state: own-column history (planes t-RAD .. t-1) and the past
    // halves of the six xz/yz mixed combinations for outputs t+1 .. t+RAD:
    //   0: Dxz uz   1: Dyz uz   2: Dxz ux + Dyz uy
    //   3: Dxz Az   4: Dyz Az   5: Dxz Ax + Dyz Ay
    T hist[RAD][NQ];
    D2 past[6][RAD];
#pragma unroll
    for (int k = 0; k < RAD; ++k)
#pragma unroll
        for (int q = 0; q < NQ; ++q) hist[k][q] = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int k = 0; k < RAD; ++k) past[c][k] = D2(0);
    // wold, cc: the 2N register and compensation of the next plane, fetched a
    // plane ahead; wnew, fnew, cnew: this plane's results
    T wold[NQ] = {}, wnew[NQ] = {}, fnew[NQ] = {}, cc[NQ] = {}, cnew[NQ] = {};

    auto cell_index = [&](int t) { return g.interior + t * g.mxy + (y0 + ly) * g.mx + (x0 + lx); };

    // ring slot of plane p: p + SOFS > 0 for every plane the march touches
    // (p >= bz0 - 2 RAD - 1), so an unsigned modulo gives the slot (an AND
    // when NSLOT is a power of two)
    constexpr int SOFS = 4 * NSLOT;
    auto slot_of = [](int p) { return (int)((unsigned)(p + SOFS) % (unsigned)NSLOT); };
    load_plane(bz0 - RAD);
    // u: plane index relative to the box start, so that the warm-up tests
    // below compare against constants.  Iterations u < -RAD only fill the
    // ring; u in [-RAD, 0) are warm-up planes.
    for (int u = -(2 * RAD + 1); u < bz1 - bz0; ++u) {
        const int t = bz0 + u;
        if (u >= -RAD) {
            int sl[RAD + 1];  // ring slots of planes t .. t+RAD
#pragma unroll
            for (int k = 0; k <= RAD; ++k) sl[k] = slot_of(t + k);
            const int s0 = sl[0];
            // warm-up planes (t < z0) run the whole computation too (branch-free
            // code schedules better); only their z state is kept

            Derivs<Rt> d;
            D2 gdu[3] = {D2(0), D2(0), D2(0)}, jmu[3] = {D2(0), D2(0), D2(0)};

            auto sum2 = [&](int q, int dir, int m) {
                return dir == 0 ? D2(V(s0, q, 0, m)) + D2(V(s0, q, 0, -m))
                                : D2(V(s0, q, m, 0)) + D2(V(s0, q, -m, 0));
            };
            auto first = [&](int q, int dir) -> Rt {  // D_x / D_y
                auto g1 = [&](int m) -> Rt {
                    return dir == 0 ? Rt(V(s0, q, 0, m)) - Rt(V(s0, q, 0, -m))
                                    : Rt(V(s0, q, m, 0)) - Rt(V(s0, q, -m, 0));
                };
                Rt acc = Rt(W1(RAD, 1)) * g1(1);
#pragma unroll
                for (int m = 2; m <= RAD; ++m) acc += Rt(W1(RAD, m)) * g1(m);
                return acc * Rt(sc.d1[dir]);
            };
            auto col = [&](int q, int k) -> T {  // own column, plane t+k, k = -RAD..RAD
                return k < 0 ? hist[k + RAD][q] : V(sl[k], q, 0, 0);
            };
            auto dz1 = [&](int q) -> Rt {
                Rt acc = Rt(W1(RAD, 1)) * (Rt(col(q, 1)) - Rt(col(q, -1)));
#pragma unroll
                for (int m = 2; m <= RAD; ++m) acc += Rt(W1(RAD, m)) * (Rt(col(q, m)) - Rt(col(q, -m)));
                return acc * Rt(sc.d1[2]);
            };
            // pure second derivatives along x, y, z
            auto second = [&](int q, D2& xx, D2& yy, D2& zz) {
                const D2 f0 = D2(W2(RAD, 0)) * D2(V(s0, q, 0, 0));
                // one axis after the other (the order the scheduler handles best)
                D2 ax = D2(W2(RAD, 1)) * sum2(q, 0, 1);
#pragma unroll
                for (int m = 2; m <= RAD; ++m) ax += D2(W2(RAD, m)) * sum2(q, 0, m);
                xx = (ax + f0) * D2(sc.d2[0]);
                D2 ay = D2(W2(RAD, 1)) * sum2(q, 1, 1);
#pragma unroll
                for (int m = 2; m <= RAD; ++m) ay += D2(W2(RAD, m)) * sum2(q, 1, m);
                yy = (ay + f0) * D2(sc.d2[1]);
                D2 az = D2(W2(RAD, 1)) * (D2(col(q, 1)) + D2(col(q, -1)));
#pragma unroll
                for (int m = 2; m <= RAD; ++m) az += D2(W2(RAD, m)) * (D2(col(q, m)) + D2(col(q, -m)));
                zz = (az + f0) * D2(sc.d2[2]);
            };
            auto dxy = [&](int q) -> D2 {
                auto e = [&](int m) {
                    return (D2(V(s0, q, m, m)) + D2(V(s0, q, -m, -m))) -
                           (D2(V(s0, q, -m, m)) + D2(V(s0, q, m, -m)));
                };
                D2 acc = D2(W2(RAD, 1)) * e(1);
#pragma unroll
                for (int m = 2; m <= RAD; ++m) acc += D2(W2(RAD, m)) * e(m);
                return acc * D2(sc.mxy);
            };
            // xz (dir 0) / yz (dir 1) mixed derivative of field q for combination
            // cb: the future half from ring planes t+1..t+RAD minus the carried
            // past half (when `first_of_combo`); then the combination's carried
            // state is advanced by plane t's own differences: past[cb][k] holds
            // the past half of output plane t+1+k.
            auto mixed = [&](int q, int dir, int cb, bool first_of_combo) -> D2 {
                const double* wm = dir == 0 ? sc.wxz : sc.wyz;
                auto dd = [&](int slot, int m) {
                    return dir == 0 ? D2(V(slot, q, 0, m)) - D2(V(slot, q, 0, -m))
                                    : D2(V(slot, q, m, 0)) - D2(V(slot, q, -m, 0));
                };
                D2 res = D2(wm[0]) * dd(sl[1], 1);
#pragma unroll
                for (int m = 2; m <= RAD; ++m) res += D2(wm[m - 1]) * dd(sl[m], m);
                if (first_of_combo) res -= past[cb][0];
                D2 c[RAD];  // this plane's half for outputs t+1 .. t+RAD
#pragma unroll
                for (int m = 1; m <= RAD; ++m) c[m - 1] = D2(wm[m - 1]) * dd(s0, m);
#pragma unroll
                for (int m = 1; m <= RAD; ++m) {
                    if (first_of_combo)
                        past[cb][m - 1] = m < RAD ? past[cb][m < RAD ? m : 0] + c[m - 1] : c[m - 1];
                    else
                        past[cb][m - 1] += c[m - 1];
                }
                return res;
            };
#define MHD_PHASE_FENCE(i) \
    if constexpr (((FENCE_MASK >> (i)) & 1) != 0) __builtin_amdgcn_sched_barrier(0)

            // ---- lnrho
            {
                d.lnrho = Rt(V(s0, 0, 0, 0));
                d.gl[0] = first(0, 0); d.gl[1] = first(0, 1); d.gl[2] = dz1(0);
                D2 xx, yy, zz;
                second(0, xx, yy, zz);
                d.lapl = Rt(xx + yy + zz);
            }
            MHD_PHASE_FENCE(0);
            // ---- ss
            {
                d.ss = Rt(V(s0, 4, 0, 0));
                d.gs[0] = first(4, 0); d.gs[1] = first(4, 1); d.gs[2] = dz1(4);
                D2 xx, yy, zz;
                second(4, xx, yy, zz);
                d.laps = Rt(xx + yy + zz);
            }
            MHD_PHASE_FENCE(1);
            // ---- ux: grad, lap; D_xx ux -> gdu_x, D_xy ux -> gdu_y, D_xz ux -> gdu_z
            {
                const D2 mz = mixed(1, 0, 2, true);
                d.ux = Rt(V(s0, 1, 0, 0));
                d.gu[0][0] = first(1, 0); d.gu[0][1] = first(1, 1); d.gu[0][2] = dz1(1);
                D2 xx, yy, zz;
                second(1, xx, yy, zz);
                d.lapu[0] = Rt(xx + yy + zz);
                gdu[0] += xx;
                gdu[1] += dxy(1);
                gdu[2] += mz;
            }
            MHD_PHASE_FENCE(2);
            // ---- uy
            {
                const D2 mz = mixed(2, 1, 2, false);
                d.uy = Rt(V(s0, 2, 0, 0));
                d.gu[1][0] = first(2, 0); d.gu[1][1] = first(2, 1); d.gu[1][2] = dz1(2);
                D2 xx, yy, zz;
                second(2, xx, yy, zz);
                d.lapu[1] = Rt(xx + yy + zz);
                gdu[1] += yy;
                gdu[0] += dxy(2);
                gdu[2] += mz;
            }
            MHD_PHASE_FENCE(3);
            // ---- uz
            {
                const D2 mx = mixed(3, 0, 0, true);
                const D2 my = mixed(3, 1, 1, true);
                d.uz = Rt(V(s0, 3, 0, 0));
                d.gu[2][0] = first(3, 0); d.gu[2][1] = first(3, 1); d.gu[2][2] = dz1(3);
                D2 xx, yy, zz;
                second(3, xx, yy, zz);
                d.lapu[2] = Rt(xx + yy + zz);
                gdu[2] += zz;
                gdu[0] += mx;
                gdu[1] += my;
            }
            MHD_PHASE_FENCE(4);
            // ---- Ax: mu0 j_x gets -(D_yy + D_zz) Ax, j_y gets D_xy Ax, j_z gets D_xz Ax
            {
                const D2 mz = mixed(5, 0, 5, true);
                d.dAx_dy = first(5, 1);
                d.dAx_dz = dz1(5);
                D2 xx, yy, zz;
                second(5, xx, yy, zz);
                d.lapA[0] = Rt(xx + yy + zz);
                jmu[0] -= yy + zz;
                jmu[1] += dxy(5);
                jmu[2] += mz;
            }
            MHD_PHASE_FENCE(5);
            // ---- Ay
            {
                const D2 mz = mixed(6, 1, 5, false);
                d.dAy_dx = first(6, 0);
                d.dAy_dz = dz1(6);
                D2 xx, yy, zz;
                second(6, xx, yy, zz);
                d.lapA[1] = Rt(xx + yy + zz);
                jmu[1] -= xx + zz;
                jmu[0] += dxy(6);
                jmu[2] += mz;
            }
            MHD_PHASE_FENCE(6);
            // ---- Az
            {
                const D2 mx = mixed(7, 0, 3, true);
                const D2 my = mixed(7, 1, 4, true);
                d.dAz_dx = first(7, 0);
                d.dAz_dy = first(7, 1);
                D2 xx, yy, zz;
                second(7, xx, yy, zz);
                d.lapA[2] = Rt(xx + yy + zz);
                jmu[2] -= xx + yy;
                jmu[0] += mx;
                jmu[1] += my;
            }
            MHD_PHASE_FENCE(7);
#undef MHD_PHASE_FENCE

#pragma unroll
            for (int a = 0; a < 3; ++a) {
                d.gdu[a] = Rt(gdu[a]);
                d.jmu[a] = Rt(jmu[a]);
            }
            Rt rhs[NQ];
            rhs_physics<Rt>(d, P, rhs);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                cnew[q] = cc[q];
                rk_values<PREC>(s, V(s0, q, 0, 0), wold[q], rhs[q], dt, wnew[q], fnew[q], cnew[q]);
            }

            // ---- advance the own-column history past plane t
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
#pragma unroll
                for (int k = 0; k + 1 < RAD; ++k) hist[k][q] = hist[k + 1][q];
                hist[RAD - 1][q] = V(s0, q, 0, 0);
            }
        }

        // ---- plane t+RAD+1 replaces plane t in the ring; then plane t+RAD+2 and the
        // next plane's register values are fetched, and only then do this
        // plane's results go out.  The vector-memory counter covers loads and
        // stores alike in issue order, so with the loads first the next
        // plane's waits for them do not also wait for these stores.
        __syncthreads();  // every read of plane t is done
        store_plane(slot_of(t + RAD + 1));
        if (t + RAD + 2 <= bz1 + RAD - 1) load_plane(t + RAD + 2);
        if (active && u + 1 >= 0 && t + 1 < bz1) {
            const unsigned c = (unsigned)cell_index(t + 1);
            if (s > 0) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) wold[q] = *at(field_ptr(w, q), c);
            }
            if constexpr (PREC == MHD_F32C) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) cc[q] = *at(field_ptr(comp, q), c);
            }
        }
        if (u >= 0 && active) {
            const unsigned c = (unsigned)cell_index(t);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                *at(field_ptr(w, q), c) = wnew[q];
                *at(field_ptr(fout, q), c) = fnew[q];
                if constexpr (PREC == MHD_F32C) *at(field_ptr(comp, q), c) = cnew[q];
            }
        }
        __syncthreads();  // plane t+RAD+1 visible to every wave
    }
}

template <int PREC, int RAD>
hipError_t launch_one(const Grid& g, const Phys& P, const Box* bx, int nbox, int s,
                      const void* f_in, void* f_out, void* w, void* comp, double dt,
                      hipStream_t st)
{
    using T = typename Prec<PREC>::T;
    constexpr size_t lds = lds_bytes<PREC, RAD>();
    constexpr int TY = Ring<PREC, RAD>::TY, NT = Ring<PREC, RAD>::NT;
    // once per instantiation (thread-safe static initialisation): the LDS
    // limit of both variants, and the workgroups resident at once (a round)
    struct Setup {
        hipError_t err;
        int round;
    };
    static const Setup setup = []() -> Setup {
        hipError_t e = hipFuncSetAttribute((const void*)k_rk3_tiled<PREC, RAD, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_rk3_tiled<PREC, RAD, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        int per_cu = 0, dev = 0, cus = 0;
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rk3_tiled<PREC, RAD, false>,
                                                             NT, lds);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        return Setup{e, per_cu * cus};
    }();
    if (setup.err != hipSuccess) return setup.err;
    const int round = setup.round;
    const TilePlan plan = plan_tiles(bx, nbox, TX, TY, round);
    Scales<RAD> sc{};
    for (int a = 0; a < 3; ++a) {
        sc.d1[a] = P.inv_h[a] / DEN1(RAD);
        sc.d2[a] = P.inv_h[a] * P.inv_h[a] / DEN2(RAD);
    }
    sc.mxy = P.inv_h[0] * P.inv_h[1] / (4.0 * DEN2(RAD));
    for (int k = 1; k <= RAD; ++k) {
        sc.wxz[k - 1] = W2(RAD, k) * P.inv_h[0] * P.inv_h[2] / (4.0 * DEN2(RAD));
        sc.wyz[k - 1] = W2(RAD, k) * P.inv_h[1] * P.inv_h[2] / (4.0 * DEN2(RAD));
    }
    if (nbox == 1)
        hipLaunchKernelGGL((k_rk3_tiled<PREC, RAD, false>), dim3(plan_blocks(plan)), dim3(NT), lds,
                           st, g, P, sc, plan_map(plan), s, (const T*)f_in, (T*)f_out, (T*)w,
                           (T*)comp, dt, plan.box[0], TilePlan{});
    else
        hipLaunchKernelGGL((k_rk3_tiled<PREC, RAD, true>), dim3(plan_blocks(plan)), dim3(NT), lds,
                           st, g, P, sc, TileMap{}, s, (const T*)f_in, (T*)f_out, (T*)w, (T*)comp,
                           dt, Box{}, plan);
    return hipGetLastError();
}

template <int RAD>
hipError_t launch_order(const Grid& g, const Phys& P, int precision, const Box* bx, int nbox,
                        int s, const void* f_in, void* f_out, void* w, void* comp, double dt,
                        hipStream_t st)
{
    switch (precision) {
    case MHD_F64:
        return launch_one<MHD_F64, RAD>(g, P, bx, nbox, s, f_in, f_out, w, nullptr, dt, st);
    case MHD_F32C:
        return launch_one<MHD_F32C, RAD>(g, P, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    default:
        return launch_one<MHD_F32, RAD>(g, P, bx, nbox, s, f_in, f_out, w, nullptr, dt, st);
    }
}

}  // namespace

// Radii 1 and 4 are instantiated in a second translation unit,
// rk3_tiled_dflt.hip (this file with MHD_DEFAULT_SCHED defined), which the
// build compiles with the default instruction scheduler: the iterative ILP
// scheduler this file is built with makes them slower (measured at 512^3).
hipError_t launch_rk3_tiled_dflt(const Grid& g, const Phys& P, int precision, const Box* bx,
                                 int nbox, int s, const void* f_in, void* f_out, void* w,
                                 void* comp, double dt, hipStream_t st);

#ifndef MHD_DEFAULT_SCHED
// The stencil radius is the grid's halo width g.r (1..4).  One launch
// updates the nbox (1..MAX_BOXES) disjoint, non-empty boxes bx.
hipError_t launch_rk3_tiled(const Grid& g, const Phys& P, int precision, const Box* bx, int nbox,
                            int s, const void* f_in, void* f_out, void* w, void* comp, double dt,
                            hipStream_t st)
{
    switch (g.r) {
    case 1:
    case 4:
        return launch_rk3_tiled_dflt(g, P, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    case 2: return launch_order<2>(g, P, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    case 3: return launch_order<3>(g, P, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    default: return hipErrorInvalidValue;
    }
}
#else
hipError_t launch_rk3_tiled_dflt(const Grid& g, const Phys& P, int precision, const Box* bx,
                                 int nbox, int s, const void* f_in, void* f_out, void* w,
                                 void* comp, double dt, hipStream_t st)
{
    switch (g.r) {
    case 1: return launch_order<1>(g, P, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    case 4: return launch_order<4>(g, P, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    default: return hipErrorInvalidValue;
    }
}
#endif

}  // namespace mhd

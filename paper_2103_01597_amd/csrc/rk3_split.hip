// Fused RHS + RK3 substep, LDS-tiled z-marching kernel with two wave groups
// per cell (gfx950).
//
// The data flow is that of the single-group tiled kernel -- a 32 x 8 column
// tile marched through z, an LDS ring of r+1 halo'd planes (t .. t+r) of all
// 8 fields for stencil radius r, an r-deep register history of the own
// column, the xz / yz mixed derivatives split into a future half read from
// the ring and a carried past half -- but each cell is served by two threads
// in different waves (figures below for r = 3, sixth order):
//   group F (waves 0-3): lnrho, ux, uy, uz -- their derivatives, Eq. B.1
//                        and Eq. B.2, and their 2N updates;
//   group M (waves 4-7): ss, Ax, Ay, Az -- their derivatives, Eqs. B.3 and
//                        B.4, and their 2N updates.
// FP64 at r = 4 uses a 32 x 4 tile (256 threads): its ring of five 40 x 12
// planes and the exchange area take the whole 160 KB of LDS.
// Each group loads, stores and differentiates only its own four fields.
// After the derivative phase the groups swap what the other side's
// equations need through LDS:
//   F -> M (10 values): lnrho, u, grad lnrho, lap lnrho, S:S, div u;
//   M -> F (7 values):  ss, grad s, j x B.
// With 512 threads per workgroup the FP64 ring (136 KB) still fits one
// workgroup per CU, so every SIMD runs two waves instead of one; a wave
// hides the LDS and barrier latency of the other.  Both hand-overs use one
// 20 KB area past the ring (M reads F's values, then writes its own into
// the same entries of its cell), so a plane costs two workgroup barriers:
//   derivatives of plane t; F writes its values
//   -- barrier (plane t read, F's values visible) --
//   plane t+4 goes into plane t's slot; M swaps the values
//   -- barrier (plane t+4 and M's values visible) --
//   physics, 2N update and stores of plane t; fetch plane t+5.
#include <type_traits>

#include "mhd_internal.hpp"
#include "rk3_common.hpp"

namespace mhd {

// FP64 at radius 4 is instantiated in a second translation unit,
// rk3_split_dflt.hip (this file with MHD_DEFAULT_SCHED defined), which the
// build compiles with the default instruction scheduler: the iterative ILP
// scheduler this file is built with makes it slower (measured at 512^3).
hipError_t launch_rk3_split_dflt(const Grid& g, const Phys& P, const Phys* P_dev, const Box* bx,
                                 int nbox, int s, const void* f_in, void* f_out, void* w, double dt,
                                 hipStream_t st);
// FP64 at radius 3 (the sixth-order default) is instantiated in a third
// translation unit, rk3_split_f64r3.hip, with the plane step compiled as a
// lambda the plane loop calls (MHD_SPLIT_BODY_LAMBDA): that form needs 197
// instead of 225 registers there and measured 1.1-1.3% faster at 512^3,
// while it measured slower for the other instantiations (FP64 at order 8
// +11%, FP32C at order 8 +4%, FP64 at order 4 +0.6%).
hipError_t launch_rk3_split_f64r3(const Grid& g, const Phys& P, const Phys* P_dev, const Box* bx,
                                  int nbox, int s, const void* f_in, void* f_out, void* w,
                                  double dt, hipStream_t st);

namespace {

#ifndef MHD_SPLIT_BODY_LAMBDA
#define MHD_SPLIT_BODY_LAMBDA 0
#endif
// The physics constants are read per plane through P_dev.  Declared
// __restrict__ (nothing the kernel stores can alias them) the reads become
// scalar-memory loads, counted apart from the vector-memory loads and
// stores; through a plain pointer they are vector loads, and the wait for
// them also waits for the next plane's prefetch issued before them (group
// M reads the constants in its derivative phase).  Scalar loads measured
// 1.2% faster for FP64 at order 6 and 1.6% at order 4 (512^3 and 256^3),
// 1.2% slower for FP64 at order 8, which rk3_split_dflt.hip builds with
// MHD_SPLIT_PHYS_SMEM 0.
#ifndef MHD_SPLIT_PHYS_SMEM
#define MHD_SPLIT_PHYS_SMEM 1
#endif
#if MHD_SPLIT_PHYS_SMEM
#define SPLIT_PHYS_PTR const Phys* __restrict__
#else
#define SPLIT_PHYS_PTR const Phys*
#endif
#ifndef MHD_SPLIT_TX
#define MHD_SPLIT_TX 32
#endif
constexpr int NXF = 10;            // values F hands to M
constexpr int NXM = 7;             // values M hands to F
// Per precision and stencil radius RAD: the tile plane of TX x TY cells
// (TY = 4 for FP64 at RAD = 4, whose 5-plane ring of a 32 x 8 tile would not
// fit the LDS; 8 otherwise), the halo'd tile plane (38 x 14 = 532 cells at
// RAD = 3) and the LDS ring of RAD + 1 such planes of all 8 fields.
template <int PREC, int RAD>
struct SRing {
    static constexpr bool SMALL = PREC == MHD_F64 && RAD == 4;
    static constexpr int TX = MHD_SPLIT_TX;
    static constexpr int TY = (SMALL ? 128 : 256) / TX;
    static constexpr int NC = TX * TY;   // cells per tile plane
    static constexpr int NTH = 2 * NC;   // threads: two groups of NC
    static constexpr int HX = TX + 2 * RAD, HY = TY + 2 * RAD, PLANE = HX * HY;
    static constexpr int SLOT = NQ * PLANE;
    static constexpr int NSLOT = RAD + 1;
};

template <int PREC, int RAD>
constexpr size_t ring_bytes()
{
    return sizeof(typename Prec<PREC>::T) * SRing<PREC, RAD>::NSLOT * SRing<PREC, RAD>::SLOT;
}
template <int PREC, int RAD>
constexpr size_t lds_bytes()
{
    return ring_bytes<PREC, RAD>() + sizeof(typename Prec<PREC>::Rt) * NXF * SRing<PREC, RAD>::NC;
}

static_assert(NXM <= NXF, "M's values reuse the entries of F's");

// Minimum waves per SIMD the kernel is built for (the second launch-bounds
// argument).  A 512-thread workgroup already puts two waves on every SIMD,
// so 1 leaves each lane up to 256 registers.  Two resident workgroups (4,
// i.e. 128 registers) would spill heavily at every radius (FP64 at r = 1:
// 203 spilled registers), and FP64's ring fills the LDS from r = 2 on.
#ifndef MHD_SPLIT_F32_BLOCKS
#define MHD_SPLIT_F32_BLOCKS 1
#endif
template <int PREC>
constexpr int blocks_per_cu() { return PREC == MHD_F64 ? 1 : MHD_SPLIT_F32_BLOCKS; }
static_assert(SRing<MHD_F64, 4>::NC % 64 == 0 && SRing<MHD_F32, 1>::NC % 64 == 0,
              "each group must be whole waves");

// Per-axis scale factors of the integer-weight stencils.
// (Sized by the radius: the kernel keeps these in scalar registers, which
// are scarce.)
template <int RAD>
struct Scales {
    double d1[3];     // 1/(DEN1 h_a)
    double d2[3];     // 1/(DEN2 h_a^2)
    double mxy;       // 1/(4 DEN2 h_x h_y)
    double wxz[RAD];  // W2(r, m)/(4 DEN2 h_x h_z), m = 1..r
    double wyz[RAD];  // W2(r, m)/(4 DEN2 h_y h_z)
};

// MULTI: the launch covers the several boxes of `plan` and each workgroup
// takes its box and tile grid from there; otherwise one box, `box` and `map`
// (a separate instantiation, so that the single-box march is compiled as if
// the plan did not exist).  PAIRS: most of each halo'd plane is fetched and
// stored into the ring as pairs of x-neighbours (one 16-byte load and LDS
// store per pair in FP64, about half the load instructions); the launch
// guarantees that every pair is aligned (even padded row length, even box x0,
// aligned f_in).
template <int PREC, int RAD, bool MULTI, bool PAIRS>
__global__ __launch_bounds__((SRing<PREC, RAD>::NTH), blocks_per_cu<PREC>()) void k_rk3_split(Grid g, SPLIT_PHYS_PTR P_dev, Scales<RAD> sc, TileMap map, int s,
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
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* __restrict__ lds = reinterpret_cast<T*>(smem_raw);
    // exchange area past the ring: F's NXF values per cell, then (in place) M's NXM
    Rt* __restrict__ xch = reinterpret_cast<Rt*>(smem_raw + ring_bytes<PREC, RAD>());  // [NXF][NC]
    using RG = SRing<PREC, RAD>;
    constexpr int TY = RG::TY, NC = RG::NC;
    constexpr int HX = RG::HX, PLANE = RG::PLANE, SLOT = RG::SLOT;
    constexpr int NSLOT = RG::NSLOT;

    const int tile = MULTI ? multi_tile : tile_of_block(blockIdx.x, map);
    if (tile == NO_TILE) return;  // the whole workgroup exits together
    // tile = (chunk * nty + ty) * ntx + tx; the chunk marches its own z range
    const int per_chunk = map.ntx * map.nty, ch = tile / per_chunk, txy = tile - ch * per_chunk;
    const int tx = txy % map.ntx, ty = txy / map.ntx;
    const int bz0 = box.z0 + ch * map.zc, bz1 = min(bz0 + map.zc, box.z1);
    constexpr int TX = RG::TX;
    const int x0 = bx0 + tx * TX, y0 = by0 + ty * TY;
    // group index, made visibly wave-uniform so that the two groups' code
    // paths (each with its own registers and the same barriers) are scalar
    // branches
    const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / NC);
    const int tid = threadIdx.x - grp * NC, lx = tid % TX, ly = tid / TX;
    const bool active = (x0 + lx < bx1) && (y0 + ly < by1);

    auto field_ptr = [&](auto* base, int q) { return base + q * g.fstride; };
    auto at = [](auto* p, unsigned idx) {
        using Pt = decltype(p);
        using C = typename std::conditional<std::is_const<typename std::remove_pointer<Pt>::type>::value,
                                            const char*, char*>::type;
        return reinterpret_cast<Pt>(reinterpret_cast<C>(p) + idx * (unsigned)sizeof(T));
    };

    // The whole march runs in one of two instantiations, one per group, so
    // that each group's registers are allocated for its own path only.  Both
    // execute the same sequence of barriers.
    auto march = [&](auto group_tag) {
        constexpr int G = decltype(group_tag)::value;
        // ---- per-thread load slots of the halo'd tile plane (clamped into the
        // padded grid for ragged tiles); each group loads its own four fields
        constexpr int q0 = 4 * G;  // first of the group's fields
        // Load units of the halo'd tile plane: with PAIRS, the first NFP * NC
        // pairs of x-neighbours (rows of HX cells are HX / 2 pairs; one 2-element
        // load and LDS store each), then the remaining cells one by one; without,
        // every cell one by one.  Offsets are clamped into the padded grid for
        // ragged tiles.
        typedef T Pair __attribute__((ext_vector_type(2)));
        constexpr int HP = HX / 2;
        constexpr int NFP = PAIRS ? (PLANE / 2) / NC : 0;   // pair slots per thread
        constexpr int CELLS0 = 2 * NFP * NC;                 // cells the pair slots cover
        constexpr int NFE = (PLANE - CELLS0) / NC, NEE = (PLANE - CELLS0) % NC;
        constexpr int NCELL = NFE + (NEE > 0 ? 1 : 0);          // cell slots per thread
        const bool extra_u = tid < NEE;
        unsigned poff[NFP > 0 ? NFP : 1], coff[NCELL > 0 ? NCELL : 1];
#pragma unroll
        for (int k = 0; k < NFP; ++k) {
            const int p = tid + k * NC, r = p / HP, c = 2 * (p - r * HP);
            const int px = min(x0 + c, g.mx - 2), py = min(y0 + r, g.my - 1);
            poff[k] = (unsigned)(py * g.mx + px);
        }
#pragma unroll
        for (int k = 0; k < NCELL; ++k) {
            const int e = min(CELLS0 + tid + k * NC, PLANE - 1);
            const int r = e / HX, c = e - r * HX;
            const int px = min(x0 + c, g.mx - 1), py = min(y0 + r, g.my - 1);
            coff[k] = (unsigned)(py * g.mx + px);
        }

        Pair prep[4][NFP > 0 ? NFP : 1];
        T prec_[4][NCELL > 0 ? NCELL : 1];
        auto load_plane = [&](int t) {
            const unsigned zo = (unsigned)((t + RAD) * g.mxy);
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const T* f = field_ptr(fin, q0 + k4);
#pragma unroll
                for (int k = 0; k < NFP; ++k) prep[k4][k] = *reinterpret_cast<const Pair*>(at(f, poff[k] + zo));
#pragma unroll
                for (int k = 0; k < NFE; ++k) prec_[k4][k] = *at(f, coff[k] + zo);
            }
            if constexpr (NEE > 0) {
                if (extra_u) {
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) prec_[k4][NFE] = *at(field_ptr(fin, q0 + k4), coff[NFE] + zo);
                }
            }
        };
        auto store_plane = [&](int slot) {
            T* base = lds + slot * SLOT + q0 * PLANE;
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
#pragma unroll
                for (int k = 0; k < NFP; ++k) reinterpret_cast<Pair*>(base + k4 * PLANE)[tid + k * NC] = prep[k4][k];
#pragma unroll
                for (int k = 0; k < NFE; ++k) base[k4 * PLANE + CELLS0 + tid + k * NC] = prec_[k4][k];
            }
            if constexpr (NEE > 0) {
                if (extra_u) {
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) base[k4 * PLANE + CELLS0 + tid + NFE * NC] = prec_[k4][NFE];
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

        // ---- z state of the group's fields: own-column history (t-RAD .. t-1),
        // indexed by field within the group, and the carried past halves of the
        // group's three xz/yz mixed combinations (past[cb][k]: output t+1+k):
        //   F: 0 Dxz uz, 1 Dyz uz, 2 Dxz ux + Dyz uy
        //   M: 0 Dxz Az, 1 Dyz Az, 2 Dxz Ax + Dyz Ay
        T hist[RAD][4];
        D2 past[3][RAD];
#pragma unroll
        for (int k = 0; k < RAD; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) hist[k][q] = T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < RAD; ++k) past[c][k] = D2(0);
        T wold[4] = {}, cc[4] = {};

        auto cell_index = [&](int t) { return g.interior + t * g.mxy + (y0 + ly) * g.mx + (x0 + lx); };

        // ring slot of plane p: p + SOFS > 0 for every plane the march touches
        // (p >= bz0 - 2 RAD - 1), so an unsigned modulo gives the slot (an AND
        // when NSLOT is a power of two)
        constexpr int SOFS = 4 * NSLOT;
        auto slot_of = [](int p) { return (int)((unsigned)(p + SOFS) % (unsigned)NSLOT); };
        load_plane(bz0 - RAD);
        // u: plane index relative to the box start, so that the warm-up tests
        // below compare against constants.  With MHD_SPLIT_BODY_LAMBDA the
        // plane step is a lambda the loop calls (FP64 at radius 3, above).
#if MHD_SPLIT_BODY_LAMBDA
        auto plane_step = [&](const int u) {
#else
        for (int u = -(2 * RAD + 1); u < bz1 - bz0; ++u) {
#endif
            const int t = bz0 + u;
            // warm-up planes (t < z0) run the whole computation too (branch-free
            // code schedules better); only their z state is kept
            const int s0 = slot_of(t);
            const bool live = u >= -RAD;  // uniform: plane t is in the ring
            Derivs<Rt> d;
            T fc[4], wnew[4], fnew[4], cnew[4];
            Rt S[3][3], divu = Rt(0), SS = Rt(0), B[3], J[3], jxB[3];
            if (live) {
                int sl[RAD + 1];  // ring slots of planes t .. t+RAD
#pragma unroll
                for (int k = 0; k <= RAD; ++k) sl[k] = slot_of(t + k);

                auto sum2 = [&](int q, int dir, int m) {
                    return dir == 0 ? D2(V(s0, q, 0, m)) + D2(V(s0, q, 0, -m))
                                    : D2(V(s0, q, m, 0)) + D2(V(s0, q, -m, 0));
                };
                auto first = [&](int q, int dir) -> Rt {
                    auto g1 = [&](int m) -> Rt {
                        return dir == 0 ? Rt(V(s0, q, 0, m)) - Rt(V(s0, q, 0, -m))
                                        : Rt(V(s0, q, m, 0)) - Rt(V(s0, q, -m, 0));
                    };
                    Rt acc = Rt(W1(RAD, 1)) * g1(1);
#pragma unroll
                    for (int m = 2; m <= RAD; ++m) acc += Rt(W1(RAD, m)) * g1(m);
                    return acc * Rt(sc.d1[dir]);
                };
                // own column of field q (group-local index k4), plane t+k, k = -RAD..RAD
                auto col = [&](int q, int k4, int k) -> T {
                    return k < 0 ? hist[k + RAD][k4] : V(sl[k], q, 0, 0);
                };
                auto dz1 = [&](int q, int k4) -> Rt {
                    Rt acc = Rt(W1(RAD, 1)) * (Rt(col(q, k4, 1)) - Rt(col(q, k4, -1)));
#pragma unroll
                    for (int m = 2; m <= RAD; ++m)
                        acc += Rt(W1(RAD, m)) * (Rt(col(q, k4, m)) - Rt(col(q, k4, -m)));
                    return acc * Rt(sc.d1[2]);
                };
                auto second = [&](int q, int k4, D2& xx, D2& yy, D2& zz) {
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
                    D2 az = D2(W2(RAD, 1)) * (D2(col(q, k4, 1)) + D2(col(q, k4, -1)));
#pragma unroll
                    for (int m = 2; m <= RAD; ++m)
                        az += D2(W2(RAD, m)) * (D2(col(q, k4, m)) + D2(col(q, k4, -m)));
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
                // xz (dir 0) / yz (dir 1) mixed derivative of field q for the
                // group's combination cb; see the single-group tiled kernel.
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
#define MHD_PHASE_FENCE() __builtin_amdgcn_sched_barrier(0)

                if constexpr (G == 0) {
                    // ================= group F: lnrho, ux, uy, uz
                    D2 gdu[3] = {D2(0), D2(0), D2(0)};
                    d.lnrho = Rt(V(s0, 0, 0, 0));
                    d.gl[0] = first(0, 0); d.gl[1] = first(0, 1); d.gl[2] = dz1(0, 0);
                    D2 xx, yy, zz;
                    second(0, 0, xx, yy, zz);
                    d.lapl = Rt(xx + yy + zz);
                    MHD_PHASE_FENCE();
                    {
                        const D2 mz = mixed(1, 0, 2, true);
                        d.ux = Rt(V(s0, 1, 0, 0));
                        d.gu[0][0] = first(1, 0); d.gu[0][1] = first(1, 1); d.gu[0][2] = dz1(1, 1);
                        D2 xx, yy, zz;
                        second(1, 1, xx, yy, zz);
                        d.lapu[0] = Rt(xx + yy + zz);
                        gdu[0] += xx;
                        gdu[1] += dxy(1);
                        gdu[2] += mz;
                    }
                    MHD_PHASE_FENCE();
                    {
                        const D2 mz = mixed(2, 1, 2, false);
                        d.uy = Rt(V(s0, 2, 0, 0));
                        d.gu[1][0] = first(2, 0); d.gu[1][1] = first(2, 1); d.gu[1][2] = dz1(2, 2);
                        D2 xx, yy, zz;
                        second(2, 2, xx, yy, zz);
                        d.lapu[1] = Rt(xx + yy + zz);
                        gdu[1] += yy;
                        gdu[0] += dxy(2);
                        gdu[2] += mz;
                    }
                    MHD_PHASE_FENCE();
                    {
                        const D2 mx = mixed(3, 0, 0, true);
                        const D2 my = mixed(3, 1, 1, true);
                        d.uz = Rt(V(s0, 3, 0, 0));
                        d.gu[2][0] = first(3, 0); d.gu[2][1] = first(3, 1); d.gu[2][2] = dz1(3, 3);
                        D2 xx, yy, zz;
                        second(3, 3, xx, yy, zz);
                        d.lapu[2] = Rt(xx + yy + zz);
                        gdu[2] += zz;
                        gdu[0] += mx;
                        gdu[1] += my;
                    }
                    MHD_PHASE_FENCE();
#pragma unroll
                    for (int a = 0; a < 3; ++a) d.gdu[a] = Rt(gdu[a]);
                } else {
                    // ================= group M: ss, Ax, Ay, Az
                    D2 jmu[3] = {D2(0), D2(0), D2(0)};
                    d.ss = Rt(V(s0, 4, 0, 0));
                    d.gs[0] = first(4, 0); d.gs[1] = first(4, 1); d.gs[2] = dz1(4, 0);
                    D2 xx, yy, zz;
                    second(4, 0, xx, yy, zz);
                    d.laps = Rt(xx + yy + zz);
                    MHD_PHASE_FENCE();
                    {
                        const D2 mz = mixed(5, 0, 2, true);
                        d.dAx_dy = first(5, 1);
                        d.dAx_dz = dz1(5, 1);
                        D2 xx, yy, zz;
                        second(5, 1, xx, yy, zz);
                        d.lapA[0] = Rt(xx + yy + zz);
                        jmu[0] -= yy + zz;
                        jmu[1] += dxy(5);
                        jmu[2] += mz;
                    }
                    MHD_PHASE_FENCE();
                    {
                        const D2 mz = mixed(6, 1, 2, false);
                        d.dAy_dx = first(6, 0);
                        d.dAy_dz = dz1(6, 2);
                        D2 xx, yy, zz;
                        second(6, 2, xx, yy, zz);
                        d.lapA[1] = Rt(xx + yy + zz);
                        jmu[1] -= xx + zz;
                        jmu[0] += dxy(6);
                        jmu[2] += mz;
                    }
                    MHD_PHASE_FENCE();
                    {
                        const D2 mx = mixed(7, 0, 0, true);
                        const D2 my = mixed(7, 1, 1, true);
                        d.dAz_dx = first(7, 0);
                        d.dAz_dy = first(7, 1);
                        D2 xx, yy, zz;
                        second(7, 3, xx, yy, zz);
                        d.lapA[2] = Rt(xx + yy + zz);
                        jmu[2] -= xx + yy;
                        jmu[0] += mx;
                        jmu[1] += my;
                    }
                    MHD_PHASE_FENCE();
#pragma unroll
                    for (int a = 0; a < 3; ++a) d.jmu[a] = Rt(jmu[a]);
                }
#undef MHD_PHASE_FENCE

                // centre values of the group's fields (the 2N update's f_in) and
                // the history shift, both before plane t's slot is reused
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    fc[k4] = V(s0, q0 + k4, 0, 0);
#pragma unroll
                    for (int k = 0; k + 1 < RAD; ++k) hist[k][k4] = hist[k + 1][k4];
                    hist[RAD - 1][k4] = fc[k4];
                }

                if constexpr (G == 0) {
                    shear(d.gu, S, divu, SS);
                    const Rt v[NXF] = {d.lnrho, d.ux, d.uy, d.uz, d.gl[0], d.gl[1], d.gl[2],
                                       d.lapl, SS, divu};
#pragma unroll
                    for (int i = 0; i < NXF; ++i) xch[i * NC + tid] = v[i];
                } else {
                    const Phys P = *P_dev;
                    magnetic(d, P, B, J, jxB);
                }
            }

            // Every read of plane t is done and F's values are visible: plane
            // t+RAD+1 replaces plane t in the ring, and M takes F's values and puts
            // its own in their place (each thread only touches the entries of
            // its own cell, so program order separates the read and the write).
            __syncthreads();
            store_plane(slot_of(t + RAD + 1));
            if constexpr (G == 1) {
                if (live) {
                    d.lnrho = xch[0 * NC + tid];
                    d.ux = xch[1 * NC + tid];
                    d.uy = xch[2 * NC + tid];
                    d.uz = xch[3 * NC + tid];
#pragma unroll
                    for (int a = 0; a < 3; ++a) d.gl[a] = xch[(4 + a) * NC + tid];
                    d.lapl = xch[7 * NC + tid];
                    SS = xch[8 * NC + tid];
                    divu = xch[9 * NC + tid];
                    const Rt v[NXM] = {d.ss, d.gs[0], d.gs[1], d.gs[2], jxB[0], jxB[1], jxB[2]};
#pragma unroll
                    for (int i = 0; i < NXM; ++i) xch[i * NC + tid] = v[i];
                }
            }
            __syncthreads();  // plane t+RAD+1 and M's values visible

            if (live) {
                // the physics constants are read here, per plane, from device
                // memory (scalar loads) rather than held in scalar registers
                // across the march, which would spill
                const Phys P = *P_dev;
                Rt rhs[4];
                if constexpr (G == 0) {
                    d.ss = xch[0 * NC + tid];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        d.gs[a] = xch[(1 + a) * NC + tid];
                        jxB[a] = xch[(4 + a) * NC + tid];
                    }
                    rhs_flow(d, P, S, divu, jxB, rhs);
                } else {
                    rhs_entropy_induction(d, P, divu, SS, B, J, rhs);
                }
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    cnew[k4] = cc[k4];
                    rk_values<PREC>(s, fc[k4], wold[k4], rhs[k4], dt, wnew[k4], fnew[k4], cnew[k4]);
                }
            }

            // plane t+RAD+2 and the next plane's register values are fetched before
            // this plane's results go out: the vector-memory counter covers loads
            // and stores alike in issue order, so the next plane's waits for the
            // loads do not also wait for these stores
            if (t + RAD + 2 <= bz1 + RAD - 1) load_plane(t + RAD + 2);
            if (active && u + 1 >= 0 && t + 1 < bz1) {
                const unsigned c = (unsigned)cell_index(t + 1);
                if (s > 0) {
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) wold[k4] = *at(field_ptr(w, q0 + k4), c);
                }
                if constexpr (PREC == MHD_F32C) {
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) cc[k4] = *at(field_ptr(comp, q0 + k4), c);
                }
            }
            if (u >= 0 && active) {
                const unsigned c = (unsigned)cell_index(t);
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    *at(field_ptr(w, q0 + k4), c) = wnew[k4];
                    *at(field_ptr(fout, q0 + k4), c) = fnew[k4];
                    if constexpr (PREC == MHD_F32C) *at(field_ptr(comp, q0 + k4), c) = cnew[k4];
                }
            }
#if MHD_SPLIT_BODY_LAMBDA
        };
        for (int u = -(2 * RAD + 1); u < bz1 - bz0; ++u) plane_step(u);
#else
        }
#endif
    };
    if (grp == 0)
        march(std::integral_constant<int, 0>{});
    else
        march(std::integral_constant<int, 1>{});
}

template <int PREC, int RAD>
hipError_t launch_one(const Grid& g, const Phys& P, const Phys* P_dev, const Box* bx, int nbox,
                      int s, const void* f_in, void* f_out, void* w, void* comp, double dt,
                      hipStream_t st)
{
    using T = typename Prec<PREC>::T;
    constexpr size_t lds = lds_bytes<PREC, RAD>();
    // pair fetches measured faster for FP64 only (the FP32 variants' 8-byte
    // pairs were no faster at order 6 and 9% slower at order 8)
    constexpr bool PAIRS_OK = PREC == MHD_F64;
    // once per instantiation (thread-safe static initialisation): the LDS
    // limit of every variant, and the workgroups resident at once (a round)
    struct Setup {
        hipError_t err;
        int round;
    };
    static const Setup setup = []() -> Setup {
        const void* kernels[4] = {(const void*)k_rk3_split<PREC, RAD, false, false>,
                                  (const void*)k_rk3_split<PREC, RAD, true, false>, nullptr,
                                  nullptr};
        if constexpr (PAIRS_OK) {
            kernels[2] = (const void*)k_rk3_split<PREC, RAD, false, PAIRS_OK>;
            kernels[3] = (const void*)k_rk3_split<PREC, RAD, true, PAIRS_OK>;
        }
        hipError_t e = hipSuccess;
        for (int k = 0; k < 4 && e == hipSuccess; ++k)
            if (kernels[k])
                e = hipFuncSetAttribute(kernels[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds);
        int per_cu = 0, dev = 0, cus = 0;
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, k_rk3_split<PREC, RAD, false, false>, SRing<PREC, RAD>::NTH, lds);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        return Setup{e, per_cu * cus};
    }();
    if (setup.err != hipSuccess) return setup.err;
    const int round = setup.round;
    const TilePlan plan =
        plan_tiles(bx, nbox, SRing<PREC, RAD>::TX, SRing<PREC, RAD>::TY, round);
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
    const dim3 grid(plan_blocks(plan)), block(SRing<PREC, RAD>::NTH);
    const bool pairs = PAIRS_OK && pairs_aligned(g, bx, nbox, f_in, sizeof(T));
#define MHD_SPLIT_LAUNCH(MULTI, PAIRS, MAP, BOX, PLAN)                                          \
    hipLaunchKernelGGL((k_rk3_split<PREC, RAD, MULTI, PAIRS>), grid, block, lds, st, g, P_dev, sc, \
                       MAP, s, (const T*)f_in, (T*)f_out, (T*)w, (T*)comp, dt, BOX, PLAN)
    if (pairs) {
        if constexpr (PAIRS_OK) {
            if (nbox == 1)
                MHD_SPLIT_LAUNCH(false, PAIRS_OK, plan_map(plan), plan.box[0], TilePlan{});
            else
                MHD_SPLIT_LAUNCH(true, PAIRS_OK, TileMap{}, Box{}, plan);
        }
    } else if (nbox == 1) {
        MHD_SPLIT_LAUNCH(false, false, plan_map(plan), plan.box[0], TilePlan{});
    } else {
        MHD_SPLIT_LAUNCH(true, false, TileMap{}, Box{}, plan);
    }
#undef MHD_SPLIT_LAUNCH
    return hipGetLastError();
}

template <int RAD>
hipError_t launch_order(const Grid& g, const Phys& P, const Phys* P_dev, int precision,
                        const Box* bx, int nbox, int s, const void* f_in, void* f_out, void* w,
                        void* comp, double dt, hipStream_t st)
{
    switch (precision) {
    case MHD_F64:
        static_assert(lds_bytes<MHD_F64, RAD>() <= 160 * 1024, "FP64 ring exceeds the LDS");
        if constexpr (RAD == 4)
            return launch_rk3_split_dflt(g, P, P_dev, bx, nbox, s, f_in, f_out, w, dt, st);
        else if constexpr (RAD == 3)
            return launch_rk3_split_f64r3(g, P, P_dev, bx, nbox, s, f_in, f_out, w, dt, st);
        else
            return launch_one<MHD_F64, RAD>(g, P, P_dev, bx, nbox, s, f_in, f_out, w, nullptr, dt,
                                            st);
    case MHD_F32C:
        return launch_one<MHD_F32C, RAD>(g, P, P_dev, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    default:
        return launch_one<MHD_F32, RAD>(g, P, P_dev, bx, nbox, s, f_in, f_out, w, nullptr, dt,
                                        st);
    }
}

}  // namespace

#if !defined(MHD_DEFAULT_SCHED) && !defined(MHD_SPLIT_F64R3)
// P (host copy) sets the stencil scales; P_dev (device copy of the same
// values) is what the kernel's physics reads.  The stencil radius is the
// grid's halo width g.r (1..4).  One launch updates the nbox (1..MAX_BOXES)
// disjoint, non-empty boxes bx.
hipError_t launch_rk3_split(const Grid& g, const Phys& P, const Phys* P_dev, int precision,
                            const Box* bx, int nbox, int s, const void* f_in, void* f_out,
                            void* w, void* comp, double dt, hipStream_t st)
{
    switch (g.r) {
    case 1: return launch_order<1>(g, P, P_dev, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    case 2: return launch_order<2>(g, P, P_dev, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    case 3: return launch_order<3>(g, P, P_dev, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    case 4: return launch_order<4>(g, P, P_dev, precision, bx, nbox, s, f_in, f_out, w, comp, dt, st);
    default: return hipErrorInvalidValue;
    }
}
#elif defined(MHD_DEFAULT_SCHED)
hipError_t launch_rk3_split_dflt(const Grid& g, const Phys& P, const Phys* P_dev, const Box* bx,
                                 int nbox, int s, const void* f_in, void* f_out, void* w, double dt,
                                 hipStream_t st)
{
    return launch_one<MHD_F64, 4>(g, P, P_dev, bx, nbox, s, f_in, f_out, w, nullptr, dt, st);
}
#else
hipError_t launch_rk3_split_f64r3(const Grid& g, const Phys& P, const Phys* P_dev, const Box* bx,
                                  int nbox, int s, const void* f_in, void* f_out, void* w,
                                  double dt, hipStream_t st)
{
    return launch_one<MHD_F64, 3>(g, P, P_dev, bx, nbox, s, f_in, f_out, w, nullptr, dt, st);
}
#endif

}  // namespace mhd

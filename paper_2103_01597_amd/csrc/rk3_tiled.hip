// Fused RHS + RK3 substep, LDS-tiled z-marching kernel for gfx950.
//
// A workgroup of 256 threads owns a TX x TY = 32 x 8 column tile and marches
// it through all nz planes, one interior cell per thread per plane.
//
// On-chip data flow (FP64: 136 KB of LDS, one workgroup per CU):
//   * LDS ring of 4 halo'd planes (t .. t+3) of all 8 fields, each plane the
//     tile plus a 3-cell halo in x and y (38 x 14 cells).  Plane t+4 is
//     fetched into registers while plane t is computed and enters the ring
//     at the next iteration, so the HBM stream overlaps the arithmetic.
//   * x/y first, second and xy-mixed derivatives of plane t read the
//     plane-t slot (axis lines and planar diagonals of Eq. stencil-fd).
//   * z derivatives use the thread's own column: planes t-3..t-1 from a
//     3-deep register history, planes t..t+3 from the ring.
//   * The xz / yz mixed derivatives are differences of x (or y) differences
//     taken on planes t +- m:  Dxz f(t) = sum_m w_m [d_m(t+m) - d_m(t-m)],
//     d_m(p) = f(x+m, p) - f(x-m, p).  The t+m halves come from the ring;
//     the t-m halves were formed when plane t-m was current (they are the
//     same differences D_x needs there) and are carried in three running
//     accumulators per mixed combination.
// Each input value is fetched from HBM once per tile plus the tile halo;
// neighbouring tiles of one round run concurrently on the same XCD (see
// tile_of_block), so halo fetches mostly hit its L2.
//
// The right-hand side assembly and the 2N update are the same as in the
// direct kernel (Appendix B; Williamson RK3).
#include "mhd_internal.hpp"
#include "rk3_common.hpp"

namespace mhd {
namespace {

constexpr int TX = 32, TY = 8, NT = TX * TY;
constexpr int HX = TX + 2 * R, HY = TY + 2 * R, PLANE = HX * HY;  // 38 x 14 = 532
constexpr int SLOT = NQ * PLANE;
constexpr int NSLOT = 4;
constexpr int LOADS = (PLANE + NT - 1) / NT;  // 3 loads per field per thread

template <typename T>
constexpr size_t lds_bytes() { return sizeof(T) * NSLOT * SLOT; }

struct TileMap {
    int ntx, nty;   // tiles per axis
    int round;      // workgroups resident at once (0: plain order)
};

constexpr int NO_TILE = -1;

// Workgroup b -> tile.  Hardware hands consecutive workgroups to the 8 XCDs
// in turn; within one round of `round` resident workgroups, XCD k gets the
// k-th contiguous run of round/8 tiles in row-major tile order, so the tiles
// that run together on one XCD (sharing its L2) are spatial neighbours, and
// a round covers a compact band of tile rows.
__device__ __forceinline__ int tile_of_block(int b, const TileMap& m)
{
    const int tiles = m.ntx * m.nty;
    if (m.round <= 0 || (m.round & 7) != 0) return b < tiles ? b : NO_TILE;
    const int r = b / m.round, w = b - r * m.round;
    const int rem = min(tiles - r * m.round, m.round);  // tiles in this round
    const int per = (rem + 7) >> 3;                      // tiles per XCD in this round
    const int k = w >> 3;
    if (k >= per) return NO_TILE;
    const int t = r * m.round + (w & 7) * per + k;
    return t < r * m.round + rem ? t : NO_TILE;
}

template <int PREC>
__global__ __launch_bounds__(NT, 1) void k_rk3_tiled(Grid g, Phys P, TileMap map, int s,
                                                     const typename Prec<PREC>::T* __restrict__ fin,
                                                     typename Prec<PREC>::T* __restrict__ fout,
                                                     typename Prec<PREC>::T* __restrict__ w,
                                                     typename Prec<PREC>::T* __restrict__ comp,
                                                     double dt)
{
    using T = typename Prec<PREC>::T;
    using Rt = typename Prec<PREC>::Rt;
    using D2 = typename Prec<PREC>::D2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* __restrict__ lds = reinterpret_cast<T*>(smem_raw);

    const int tile = tile_of_block(blockIdx.x, map);
    if (tile == NO_TILE) return;  // the whole workgroup exits together
    const int tx = tile % map.ntx, ty = tile / map.ntx;
    const int x0 = tx * TX, y0 = ty * TY;
    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const bool active = (x0 + lx < g.nx) && (y0 + ly < g.ny);

    // ---- per-thread load slots: element e of the halo'd tile plane
    unsigned goff[LOADS];
    int lofs[LOADS];
    bool lval[LOADS];
#pragma unroll
    for (int k = 0; k < LOADS; ++k) {
        const int e = tid + k * NT;
        lval[k] = e < PLANE;
        const int r = lval[k] ? e / HX : 0, c = lval[k] ? e - (e / HX) * HX : 0;
        const int px = min(x0 + c, g.mx - 1), py = min(y0 + r, g.my - 1);
        goff[k] = (unsigned)(py * g.mx + px);
        lofs[k] = lval[k] ? e : 0;
    }
    const T* fq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) fq[q] = fin + q * g.fstride;

    T pre[NQ][LOADS];
    auto load_plane = [&](int t) {  // t: interior plane index, -3 .. nz+2
        const unsigned zo = (unsigned)((t + R) * g.mxy);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int k = 0; k < LOADS; ++k)
                if (lval[k]) pre[q][k] = fq[q][goff[k] + zo];
    };
    auto store_plane = [&](int slot) {
        T* base = lds + slot * SLOT;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int k = 0; k < LOADS; ++k)
                if (lval[k]) base[q * PLANE + lofs[k]] = pre[q][k];
    };

    const int cofs = (ly + R) * HX + (lx + R);  // own cell within a plane
    auto V = [&](int slot, int q, int dy, int dx) -> T {
        return lds[slot * SLOT + q * PLANE + cofs + dy * HX + dx];
    };

    // ---- constants
    const Rt ihx = Rt(P.inv_h[0]), ihy = Rt(P.inv_h[1]), ihz = Rt(P.inv_h[2]);
    const D2 ihx2 = D2(P.inv_h[0] * P.inv_h[0]), ihy2 = D2(P.inv_h[1] * P.inv_h[1]),
             ihz2 = D2(P.inv_h[2] * P.inv_h[2]);
    const D2 ihxy = D2(P.inv_h[0] * P.inv_h[1]);
    const D2 wxz[3] = {D2(CM_1 * P.inv_h[0] * P.inv_h[2]), D2(CM_2 * P.inv_h[0] * P.inv_h[2]),
                       D2(CM_3 * P.inv_h[0] * P.inv_h[2])};
    const D2 wyz[3] = {D2(CM_1 * P.inv_h[1] * P.inv_h[2]), D2(CM_2 * P.inv_h[1] * P.inv_h[2]),
                       D2(CM_3 * P.inv_h[1] * P.inv_h[2])};

    // ---- z state: own-column history (planes t-3, t-2, t-1) and the past
    // halves of the six xz/yz mixed combinations for outputs t+1, t+2, t+3:
    //   0: Dxz uz   1: Dyz uz   2: Dxz ux + Dyz uy
    //   3: Dxz Az   4: Dyz Az   5: Dxz Ax + Dyz Ay
    T hist[3][NQ];
    D2 past[6][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int q = 0; q < NQ; ++q) hist[k][q] = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) past[c][k] = D2(0);

    const int slot_of_minus = 8;  // keeps (t + slot_of_minus) non-negative
    load_plane(-3);
    for (int t = -6; t < g.nz; ++t) {
        const int N = t + 3;  // plane entering the ring
        __syncthreads();      // slot of plane N held plane N-4, last read at t-1
        store_plane((N + slot_of_minus) & 3);
        __syncthreads();
        if (N + 1 <= g.nz + 2) load_plane(N + 1);
        if (t < -3) continue;

        const int s0 = (t + slot_of_minus) & 3, s1 = (t + 1 + slot_of_minus) & 3,
                  s2 = (t + 2 + slot_of_minus) & 3, s3 = (t + 3 + slot_of_minus) & 3;

        const int sl[4] = {s0, s1, s2, s3};
        const bool out = t >= 0;  // uniform: warm-up planes only feed the z state

        // Derivative accumulators of the output cell (filled field by field).
        Derivs<Rt> d;
        D2 gdu[3] = {D2(0), D2(0), D2(0)}, jmu[3] = {D2(0), D2(0), D2(0)};
        T wold[NQ] = {};
        const int c = g.interior + t * g.mxy + (y0 + ly) * g.mx + (x0 + lx);
        if (out && s > 0 && active) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) wold[q] = w[q * g.fstride + c];
        }

        // x (dir 0) or y (dir 1) differences d_m = f(+m) - f(-m) of plane t,
        // and the matching sums s_m = f(+m) + f(-m)
        auto diff = [&](int q, int dir, int m) {
            return dir == 0 ? D2(V(s0, q, 0, m)) - D2(V(s0, q, 0, -m))
                            : D2(V(s0, q, m, 0)) - D2(V(s0, q, -m, 0));
        };
        auto sum2 = [&](int q, int dir, int m) {
            return dir == 0 ? D2(V(s0, q, 0, m)) + D2(V(s0, q, 0, -m))
                            : D2(V(s0, q, m, 0)) + D2(V(s0, q, -m, 0));
        };
        auto first = [&](int q, int dir) -> Rt {  // D_x / D_y in the first-derivative type
            auto g1 = [&](int m) -> Rt {
                return dir == 0 ? Rt(V(s0, q, 0, m)) - Rt(V(s0, q, 0, -m))
                                : Rt(V(s0, q, m, 0)) - Rt(V(s0, q, -m, 0));
            };
            return (Rt(C1_1) * g1(1) + Rt(C1_2) * g1(2) + Rt(C1_3) * g1(3)) * (dir == 0 ? ihx : ihy);
        };
        auto col = [&](int q, int k) -> T {  // own column, plane t+k, k = -3..3
            return k < 0 ? hist[k + 3][q] : V(sl[k], q, 0, 0);
        };
        auto dz1 = [&](int q) -> Rt {
            return (Rt(C1_1) * (Rt(col(q, 1)) - Rt(col(q, -1))) +
                    Rt(C1_2) * (Rt(col(q, 2)) - Rt(col(q, -2))) +
                    Rt(C1_3) * (Rt(col(q, 3)) - Rt(col(q, -3)))) * ihz;
        };
        // second derivative D_aa along x, y, z (returned individually)
        auto second = [&](int q, D2& xx, D2& yy, D2& zz) {
            const D2 f0 = D2(C2_0) * D2(V(s0, q, 0, 0));
            xx = (D2(C2_1) * sum2(q, 0, 1) + D2(C2_2) * sum2(q, 0, 2) + D2(C2_3) * sum2(q, 0, 3) + f0) * ihx2;
            yy = (D2(C2_1) * sum2(q, 1, 1) + D2(C2_2) * sum2(q, 1, 2) + D2(C2_3) * sum2(q, 1, 3) + f0) * ihy2;
            zz = (D2(C2_1) * (D2(col(q, 1)) + D2(col(q, -1))) +
                  D2(C2_2) * (D2(col(q, 2)) + D2(col(q, -2))) +
                  D2(C2_3) * (D2(col(q, 3)) + D2(col(q, -3))) + f0) * ihz2;
        };
        auto dxy = [&](int q) -> D2 {
            const D2 cm[3] = {D2(CM_1), D2(CM_2), D2(CM_3)};
            D2 acc = D2(0);
#pragma unroll
            for (int m = 1; m <= 3; ++m)
                acc += cm[m - 1] * ((D2(V(s0, q, m, m)) + D2(V(s0, q, -m, -m))) -
                                    (D2(V(s0, q, -m, m)) + D2(V(s0, q, m, -m))));
            return acc * ihxy;
        };
        // xz (dir 0) / yz (dir 1) mixed derivative of field q for combination
        // cb: the future half from ring planes t+1..t+3 minus the carried past
        // half (when `first_of_combo`), then the combination's carried state
        // is advanced by plane t's own differences.
        auto mixed = [&](int q, int dir, int cb, bool first_of_combo) -> D2 {
            const D2* wm = dir == 0 ? wxz : wyz;
            D2 res = D2(0);
            if (out) {
#pragma unroll
                for (int m = 1; m <= 3; ++m) {
                    const int sm = sl[m];
                    const D2 dd = dir == 0 ? D2(V(sm, q, 0, m)) - D2(V(sm, q, 0, -m))
                                           : D2(V(sm, q, m, 0)) - D2(V(sm, q, -m, 0));
                    res += wm[m - 1] * dd;
                }
                if (first_of_combo) res -= past[cb][0];
            }
            const D2 c1 = wm[0] * diff(q, dir, 1), c2 = wm[1] * diff(q, dir, 2),
                     c3 = wm[2] * diff(q, dir, 3);
            if (first_of_combo) {
                past[cb][0] = past[cb][1] + c1;
                past[cb][1] = past[cb][2] + c2;
                past[cb][2] = c3;
            } else {
                past[cb][0] += c1;
                past[cb][1] += c2;
                past[cb][2] += c3;
            }
            return res;
        };
#define MHD_PHASE_FENCE() __builtin_amdgcn_sched_barrier(0)

        // ---- lnrho
        if (out) {
            d.lnrho = Rt(V(s0, 0, 0, 0));
            d.gl[0] = first(0, 0); d.gl[1] = first(0, 1); d.gl[2] = dz1(0);
            D2 xx, yy, zz;
            second(0, xx, yy, zz);
            d.lapl = Rt(xx + yy + zz);
        }
        MHD_PHASE_FENCE();
        // ---- ss
        if (out) {
            d.ss = Rt(V(s0, 4, 0, 0));
            d.gs[0] = first(4, 0); d.gs[1] = first(4, 1); d.gs[2] = dz1(4);
            D2 xx, yy, zz;
            second(4, xx, yy, zz);
            d.laps = Rt(xx + yy + zz);
        }
        MHD_PHASE_FENCE();
        // ---- ux: grad, lap; D_xx ux -> gdu_x, D_xy ux -> gdu_y, D_xz ux -> gdu_z
        {
            const D2 mz = mixed(1, 0, 2, true);
            if (out) {
                d.ux = Rt(V(s0, 1, 0, 0));
                d.gu[0][0] = first(1, 0); d.gu[0][1] = first(1, 1); d.gu[0][2] = dz1(1);
                D2 xx, yy, zz;
                second(1, xx, yy, zz);
                d.lapu[0] = Rt(xx + yy + zz);
                gdu[0] += xx;
                gdu[1] += dxy(1);
                gdu[2] += mz;
            }
        }
        MHD_PHASE_FENCE();
        // ---- uy
        {
            const D2 mz = mixed(2, 1, 2, false);
            if (out) {
                d.uy = Rt(V(s0, 2, 0, 0));
                d.gu[1][0] = first(2, 0); d.gu[1][1] = first(2, 1); d.gu[1][2] = dz1(2);
                D2 xx, yy, zz;
                second(2, xx, yy, zz);
                d.lapu[1] = Rt(xx + yy + zz);
                gdu[1] += yy;
                gdu[0] += dxy(2);
                gdu[2] += mz;
            }
        }
        MHD_PHASE_FENCE();
        // ---- uz
        {
            const D2 mx = mixed(3, 0, 0, true);
            const D2 my = mixed(3, 1, 1, true);
            if (out) {
                d.uz = Rt(V(s0, 3, 0, 0));
                d.gu[2][0] = first(3, 0); d.gu[2][1] = first(3, 1); d.gu[2][2] = dz1(3);
                D2 xx, yy, zz;
                second(3, xx, yy, zz);
                d.lapu[2] = Rt(xx + yy + zz);
                gdu[2] += zz;
                gdu[0] += mx;
                gdu[1] += my;
            }
        }
        MHD_PHASE_FENCE();
        // ---- Ax: mu0 j_x gets -(D_yy + D_zz) Ax, j_y gets D_xy Ax, j_z gets D_xz Ax
        {
            const D2 mz = mixed(5, 0, 5, true);
            if (out) {
                d.dAx_dy = first(5, 1);
                d.dAx_dz = dz1(5);
                D2 xx, yy, zz;
                second(5, xx, yy, zz);
                d.lapA[0] = Rt(xx + yy + zz);
                jmu[0] -= yy + zz;
                jmu[1] += dxy(5);
                jmu[2] += mz;
            }
        }
        MHD_PHASE_FENCE();
        // ---- Ay
        {
            const D2 mz = mixed(6, 1, 5, false);
            if (out) {
                d.dAy_dx = first(6, 0);
                d.dAy_dz = dz1(6);
                D2 xx, yy, zz;
                second(6, xx, yy, zz);
                d.lapA[1] = Rt(xx + yy + zz);
                jmu[1] -= xx + zz;
                jmu[0] += dxy(6);
                jmu[2] += mz;
            }
        }
        MHD_PHASE_FENCE();
        // ---- Az
        {
            const D2 mx = mixed(7, 0, 3, true);
            const D2 my = mixed(7, 1, 4, true);
            if (out) {
                d.dAz_dx = first(7, 0);
                d.dAz_dy = first(7, 1);
                D2 xx, yy, zz;
                second(7, xx, yy, zz);
                d.lapA[2] = Rt(xx + yy + zz);
                jmu[2] -= xx + yy;
                jmu[0] += mx;
                jmu[1] += my;
            }
        }
        MHD_PHASE_FENCE();
#undef MHD_PHASE_FENCE

        if (out && active) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                d.gdu[a] = Rt(gdu[a]);
                d.jmu[a] = Rt(jmu[a]);
            }
            Rt rhs[NQ];
            rhs_physics<Rt>(d, P, rhs);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int64_t o = q * g.fstride + c;
                rk_update_v<PREC>(s, V(s0, q, 0, 0), wold[q], rhs[q], dt, w + o, fout + o,
                                  comp ? comp + o : nullptr);
            }
        }

        // ---- advance the own-column history past plane t
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            hist[0][q] = hist[1][q];
            hist[1][q] = hist[2][q];
            hist[2][q] = V(s0, q, 0, 0);
        }
    }
}

template <int PREC>
hipError_t launch_one(const Grid& g, const Phys& P, int s, const void* f_in, void* f_out, void* w,
                      void* comp, double dt, hipStream_t st)
{
    using T = typename Prec<PREC>::T;
    static int round = -1;  // resident workgroups per round on this device
    const size_t lds = lds_bytes<T>();
    if (round < 0) {
        hipError_t e = hipFuncSetAttribute((const void*)k_rk3_tiled<PREC>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        int per_cu = 0, dev = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rk3_tiled<PREC>, NT, lds);
        if (e != hipSuccess) return e;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        round = per_cu * cus;
    }
    TileMap m;
    m.ntx = (g.nx + TX - 1) / TX;
    m.nty = (g.ny + TY - 1) / TY;
    m.round = round;
    const int tiles = m.ntx * m.nty;
    // with the XCD mapping the last round may name tiles past the end; those
    // workgroups exit at once
    const int blocks = (round > 0 && (round & 7) == 0) ? (tiles + round - 1) / round * round : tiles;
    hipLaunchKernelGGL(k_rk3_tiled<PREC>, dim3(blocks), dim3(NT), lds, st, g, P, m, s,
                       (const T*)f_in, (T*)f_out, (T*)w, (T*)comp, dt);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_rk3_tiled(const Grid& g, const Phys& P, int precision, int s, const void* f_in,
                            void* f_out, void* w, void* comp, double dt, hipStream_t st,
                            bool* launched)
{
    *launched = true;
    switch (precision) {
    case MHD_F64: return launch_one<MHD_F64>(g, P, s, f_in, f_out, w, nullptr, dt, st);
    case MHD_F32C: return launch_one<MHD_F32C>(g, P, s, f_in, f_out, w, comp, dt, st);
    default: return launch_one<MHD_F32>(g, P, s, f_in, f_out, w, nullptr, dt, st);
    }
}

}  // namespace mhd

// Fused RHS + RK3 substep, direct form: one thread per interior cell, every
// stencil point read from global memory (the L1/L2 caches catch the reuse),
// for every stencil order 2r, r = 1..4.
// It is the plain baseline next to the LDS-tiled z-marching kernels, run
// only when a caller asks for it (MHD_KERNEL_DIRECT); AUTO never picks it.
//
// Per cell it evaluates the derivatives of Section 4, Eq. (stencil-fd) --
// first and pure second derivatives on the axis lines, mixed derivatives on
// the planar diagonals -- assembles Eqs. B.1-B.4 and applies one Williamson
// 2N substep.
#include "mhd_internal.hpp"
#include "rk3_common.hpp"

namespace mhd {
namespace {

template <int PREC, int RAD>
__global__ __launch_bounds__(256) void k_rk3_direct(Grid g, Phys P, Box bx, int s,
                                                    const typename Prec<PREC>::T* __restrict__ fin,
                                                    typename Prec<PREC>::T* __restrict__ fout,
                                                    typename Prec<PREC>::T* __restrict__ w,
                                                    typename Prec<PREC>::T* __restrict__ comp,
                                                    double dt)
{
    using T = typename Prec<PREC>::T;
    using Rt = typename Prec<PREC>::Rt;
    using D2 = typename Prec<PREC>::D2;
    const int i = bx.x0 + blockIdx.x * 64 + threadIdx.x;
    const int j = bx.y0 + blockIdx.y * 4 + threadIdx.y;
    const int k = bx.z0 + blockIdx.z;
    if (i >= bx.x1 || j >= bx.y1)
        return;
    const int c = g.interior + k * g.mxy + j * g.mx + i;
    const int sx = 1, sy = g.mx, sz = g.mxy;
    const T* F[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        F[q] = fin + q * g.fstride + c;
    const Rt ihx = Rt(P.inv_h[0]), ihy = Rt(P.inv_h[1]), ihz = Rt(P.inv_h[2]);
    const D2 ih2x = D2(P.inv_h[0] * P.inv_h[0]), ih2y = D2(P.inv_h[1] * P.inv_h[1]),
             ih2z = D2(P.inv_h[2] * P.inv_h[2]);
    const D2 ihxy = D2(P.inv_h[0] * P.inv_h[1]), ihxz = D2(P.inv_h[0] * P.inv_h[2]),
             ihyz = D2(P.inv_h[1] * P.inv_h[2]);

    Derivs<Rt> d;
    d.lnrho = Rt(F[0][0]);
    d.ux = Rt(F[1][0]);
    d.uy = Rt(F[2][0]);
    d.uz = Rt(F[3][0]);
    d.ss = Rt(F[4][0]);
    const int st[3] = {sx, sy, sz};
    const Rt ih[3] = {ihx, ihy, ihz};
    const D2 ih2[3] = {ih2x, ih2y, ih2z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d.gl[a] = deriv1<Rt, RAD>(F[0], st[a]) * ih[a];
        d.gs[a] = deriv1<Rt, RAD>(F[4], st[a]) * ih[a];
#pragma unroll
        for (int b = 0; b < 3; ++b)
            d.gu[b][a] = deriv1<Rt, RAD>(F[1 + b], st[a]) * ih[a];
    }
    d.dAz_dy = deriv1<Rt, RAD>(F[7], sy) * ihy;
    d.dAy_dz = deriv1<Rt, RAD>(F[6], sz) * ihz;
    d.dAx_dz = deriv1<Rt, RAD>(F[5], sz) * ihz;
    d.dAz_dx = deriv1<Rt, RAD>(F[7], sx) * ihx;
    d.dAy_dx = deriv1<Rt, RAD>(F[6], sx) * ihx;
    d.dAx_dy = deriv1<Rt, RAD>(F[5], sy) * ihy;

    D2 sec[NQ][3];  // pure second derivatives D_aa of every field
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            sec[q][a] = deriv2<D2, RAD>(F[q], st[a]) * ih2[a];
    const D2 uxy = derivm<D2, RAD>(F[1], sx, sy) * ihxy, uyx = derivm<D2, RAD>(F[2], sx, sy) * ihxy;
    const D2 uxz = derivm<D2, RAD>(F[1], sx, sz) * ihxz, uzx = derivm<D2, RAD>(F[3], sx, sz) * ihxz;
    const D2 uyz = derivm<D2, RAD>(F[2], sy, sz) * ihyz, uzy = derivm<D2, RAD>(F[3], sy, sz) * ihyz;
    const D2 axy = derivm<D2, RAD>(F[5], sx, sy) * ihxy, ayx = derivm<D2, RAD>(F[6], sx, sy) * ihxy;
    const D2 axz = derivm<D2, RAD>(F[5], sx, sz) * ihxz, azx = derivm<D2, RAD>(F[7], sx, sz) * ihxz;
    const D2 ayz = derivm<D2, RAD>(F[6], sy, sz) * ihyz, azy = derivm<D2, RAD>(F[7], sy, sz) * ihyz;

    d.lapl = Rt(sec[0][0] + sec[0][1] + sec[0][2]);
    d.laps = Rt(sec[4][0] + sec[4][1] + sec[4][2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d.lapu[a] = Rt(sec[1 + a][0] + sec[1 + a][1] + sec[1 + a][2]);
        d.lapA[a] = Rt(sec[5 + a][0] + sec[5 + a][1] + sec[5 + a][2]);
    }
    // grad(div u): d_a (d_b u_b); the mixed terms are symmetric in (a, b)
    d.gdu[0] = Rt(sec[1][0] + uyx + uzx);
    d.gdu[1] = Rt(uxy + sec[2][1] + uzy);
    d.gdu[2] = Rt(uxz + uyz + sec[3][2]);
    // mu0 j = grad(div A) - lap A; the D_aa A_a terms cancel exactly
    d.jmu[0] = Rt((ayx + azx) - (sec[5][1] + sec[5][2]));
    d.jmu[1] = Rt((axy + azy) - (sec[6][0] + sec[6][2]));
    d.jmu[2] = Rt((axz + ayz) - (sec[7][0] + sec[7][1]));

    Rt rhs[NQ];
    rhs_physics<Rt>(d, P, rhs);

    const int64_t c64 = c;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int64_t o = q * g.fstride + c64;
        rk_update<PREC>(s, fin[o], rhs[q], dt, w + o, fout + o, comp ? comp + o : nullptr);
    }
}

template <int RAD>
void launch_order(const Grid& g, const Phys& P, int precision, const Box& bx, int s,
                  const void* f_in, void* f_out, void* w, void* comp, double dt, hipStream_t st)
{
    dim3 block(64, 4, 1);
    dim3 grid((bx.x1 - bx.x0 + 63) / 64, (bx.y1 - bx.y0 + 3) / 4, bx.z1 - bx.z0);
    switch (precision) {
    case MHD_F64:
        hipLaunchKernelGGL((k_rk3_direct<MHD_F64, RAD>), grid, block, 0, st, g, P, bx, s,
                           (const double*)f_in, (double*)f_out, (double*)w, (double*)comp, dt);
        break;
    case MHD_F32C:
        hipLaunchKernelGGL((k_rk3_direct<MHD_F32C, RAD>), grid, block, 0, st, g, P, bx, s,
                           (const float*)f_in, (float*)f_out, (float*)w, (float*)comp, dt);
        break;
    default:
        hipLaunchKernelGGL((k_rk3_direct<MHD_F32, RAD>), grid, block, 0, st, g, P, bx, s,
                           (const float*)f_in, (float*)f_out, (float*)w, (float*)nullptr, dt);
        break;
    }
}

}  // namespace

// The stencil radius is the grid's halo width g.r (1..4).
hipError_t launch_rk3_direct(const Grid& g, const Phys& P, int precision, const Box& bx, int s,
                             const void* f_in, void* f_out, void* w, void* comp, double dt,
                             hipStream_t st)
{
    switch (g.r) {
    case 1: launch_order<1>(g, P, precision, bx, s, f_in, f_out, w, comp, dt, st); break;
    case 2: launch_order<2>(g, P, precision, bx, s, f_in, f_out, w, comp, dt, st); break;
    case 3: launch_order<3>(g, P, precision, bx, s, f_in, f_out, w, comp, dt, st); break;
    case 4: launch_order<4>(g, P, precision, bx, s, f_in, f_out, w, comp, dt, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mhd

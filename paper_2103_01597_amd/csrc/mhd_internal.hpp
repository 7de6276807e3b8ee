// Internal declarations of the MHD library: launch parameters, the
// right-hand-side assembly shared by every fused kernel, and the kernel
// launchers.  gfx950 (CDNA4) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mhd.h"

namespace mhd {

constexpr int RMAX = 4;  // largest stencil radius (eighth order, Section 4)
constexpr int NQ = 8;    // fields of Table B.1

// Grid geometry as the kernels see it.  The halo is r cells wide, r the
// stencil radius (order 2r).
struct Grid {
    int nx, ny, nz;
    int mx, my, mz;   // n_i + 2r
    int64_t fstride;  // elements between fields
    int mxy;          // mx*my (one padded plane; < 2^31 for every supported size)
    int interior;     // (r*my + r)*mx + r
    int r;            // halo width = stencil radius
};

// A sub-box of the interior, half-open in interior cell indices:
// x0 <= x < x1, y0 <= y < y1, z0 <= z < z1.  The fused kernels update the
// cells of a box and leave every other cell untouched.
struct Box {
    int x0, x1, y0, y1, z0, z1;
};

__host__ __device__ inline Box full_box(const Grid& g) { return Box{0, g.nx, 0, g.ny, 0, g.nz}; }

// Physics constants and grid spacings, in double; kernels convert.
struct Phys {
    double inv_h[3];       // 1/h_i
    double cs0sq, gamma, inv_cp, lnrho0, mu0, inv_mu0, nu, zeta, eta, K;
    double bext[3];
    double gamma_m1;       // gamma - 1
    double cp_gm1;         // cp*(gamma - 1)
    double hc;             // H - C of Eq. B.3 (uniform heating minus cooling)
};

// Williamson 2N RK3 (the scheme cited in Section 4).
constexpr double RK_ALPHA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
constexpr double RK_BETA[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

// Central weights of order 2r (Section 4 lists r = 1..4), as integer
// multipliers of symmetric differences over one denominator per kind:
//   D1 f  = sum_m W1(r,m) d_m / (DEN1(r) h),             d_m = f(+m) - f(-m)
//   D2 f  = [W2(r,0) f0 + sum_m W2(r,m) s_m] / (DEN2(r) h^2),  s_m = f(+m) + f(-m)
//   Dab f = sum_m W2(r,m) e_m / (4 DEN2(r) h_a h_b),  e_m = P_m - Q_m with
//     P_m = f(+m,+m) + f(-m,-m), Q_m = f(+m,-m) + f(-m,+m) on the (a,b) plane
// (the mixed form is the difference of the second differences along the two
// diagonals of the plane, Eq. stencil-fd).  m = 1..r.
__host__ __device__ constexpr double W1(int r, int m)
{
    return r == 1 ? (m == 1 ? 1.0 : 0.0)
         : r == 2 ? (m == 1 ? 8.0 : m == 2 ? -1.0 : 0.0)
         : r == 3 ? (m == 1 ? 45.0 : m == 2 ? -9.0 : m == 3 ? 1.0 : 0.0)
                  : (m == 1 ? 672.0 : m == 2 ? -168.0 : m == 3 ? 32.0 : m == 4 ? -3.0 : 0.0);
}
__host__ __device__ constexpr double DEN1(int r)
{
    return r == 1 ? 2.0 : r == 2 ? 12.0 : r == 3 ? 60.0 : 840.0;
}
__host__ __device__ constexpr double W2(int r, int m)
{
    return r == 1 ? (m == 0 ? -2.0 : m == 1 ? 1.0 : 0.0)
         : r == 2 ? (m == 0 ? -30.0 : m == 1 ? 16.0 : m == 2 ? -1.0 : 0.0)
         : r == 3 ? (m == 0 ? -490.0 : m == 1 ? 270.0 : m == 2 ? -27.0 : m == 3 ? 2.0 : 0.0)
                  : (m == 0 ? -14350.0 : m == 1 ? 8064.0 : m == 2 ? -1008.0 : m == 3 ? 128.0
                     : m == 4 ? -9.0 : 0.0);
}
__host__ __device__ constexpr double DEN2(int r)
{
    return r == 1 ? 1.0 : r == 2 ? 12.0 : r == 3 ? 180.0 : 5040.0;
}

// Everything the right-hand side of Eqs. B.1-B.4 reads at one cell.
// R: the arithmetic type of the physics (double, or float for FP32 storage).
template <typename Rt>
struct Derivs {
    Rt lnrho, ux, uy, uz, ss;          // centre values (A enters only via derivatives)
    Rt gl[3], gs[3];                   // grad lnrho, grad s
    Rt gu[3][3];                       // gu[a][b] = d u_a / d x_b
    Rt dAz_dy, dAy_dz, dAx_dz, dAz_dx, dAy_dx, dAx_dy;
    Rt lapl, laps;                     // Laplacians of lnrho and s
    Rt lapu[3], gdu[3];                // lap u and grad(div u)
    Rt lapA[3], jmu[3];                // lap A and mu0*j = grad(div A) - lap A
};

// The right-hand side of Eqs. B.1-B.4 (uniform H and C, K constant) with the ideal
// gas closure cs^2 = cs0^2 exp(gamma s/cp + (gamma-1)(lnrho - lnrho0)),
// cp (gamma-1) T = cs^2; B = curl A + B_ext; S the traceless rate of shear.
// It is assembled from four pieces so that a kernel may split the work
// between the velocity side (B.1, B.2) and the entropy/induction side
// (B.3, B.4); rhs_physics chains them.

// Traceless rate of shear S, div u and S:S from the velocity gradient.
template <typename Rt>
__device__ __forceinline__ void shear(const Rt gu[3][3], Rt S[3][3], Rt& divu, Rt& SS)
{
    divu = gu[0][0] + gu[1][1] + gu[2][2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            S[a][b] = Rt(0.5) * (gu[a][b] + gu[b][a]);
    const Rt third_divu = divu * Rt(1.0 / 3.0);
    S[0][0] -= third_divu;
    S[1][1] -= third_divu;
    S[2][2] -= third_divu;
    SS = Rt(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            SS += S[a][b] * S[a][b];
}

// B = curl A + B_ext, J = j (current density) and the Lorentz force j x B.
template <typename Rt>
__device__ __forceinline__ void magnetic(const Derivs<Rt>& d, const Phys& P, Rt B[3], Rt J[3],
                                         Rt jxB[3])
{
    B[0] = d.dAz_dy - d.dAy_dz + Rt(P.bext[0]);
    B[1] = d.dAx_dz - d.dAz_dx + Rt(P.bext[1]);
    B[2] = d.dAy_dx - d.dAx_dy + Rt(P.bext[2]);
    const Rt inv_mu0 = Rt(P.inv_mu0);
#pragma unroll
    for (int a = 0; a < 3; ++a) J[a] = d.jmu[a] * inv_mu0;
    jxB[0] = J[1] * B[2] - J[2] * B[1];
    jxB[1] = J[2] * B[0] - J[0] * B[2];
    jxB[2] = J[0] * B[1] - J[1] * B[0];
}

// Eqs. B.1 and B.2: out[0] = d lnrho/dt, out[1..3] = du/dt.  Reads lnrho,
// ss, u, gl, gs, gu, lapu, gdu of d.
template <typename Rt>
__device__ __forceinline__ void rhs_flow(const Derivs<Rt>& d, const Phys& P, const Rt S[3][3],
                                         Rt divu, const Rt jxB[3], Rt out[4])
{
    const Rt gamma = Rt(P.gamma), inv_cp = Rt(P.inv_cp), gm1 = Rt(P.gamma_m1);
    const Rt nu = Rt(P.nu), zeta = Rt(P.zeta);
    const Rt u[3] = {d.ux, d.uy, d.uz};
    const Rt inv_rho = exp(-d.lnrho);
    const Rt cs2 = Rt(P.cs0sq) * exp(gamma * d.ss * inv_cp + gm1 * (d.lnrho - Rt(P.lnrho0)));

    out[0] = -(u[0] * d.gl[0] + u[1] * d.gl[1] + u[2] * d.gl[2]) - divu;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Rt adv = u[0] * d.gu[a][0] + u[1] * d.gu[a][1] + u[2] * d.gu[a][2];
        const Rt Sgl = S[a][0] * d.gl[0] + S[a][1] * d.gl[1] + S[a][2] * d.gl[2];
        const Rt pres = -cs2 * (d.gs[a] * inv_cp + d.gl[a]);
        const Rt visc = nu * (d.lapu[a] + d.gdu[a] * Rt(1.0 / 3.0) + Rt(2) * Sgl);
        out[1 + a] = -adv + pres + jxB[a] * inv_rho + visc + zeta * d.gdu[a];
    }
}

// Eq. B.3 divided by rho*T (out[0] = ds/dt) and Eq. B.4 (out[1..3] =
// dA/dt).  Reads lnrho, ss, u, gl, gs, lapl, laps, lapA of d.
template <typename Rt>
__device__ __forceinline__ void rhs_entropy_induction(const Derivs<Rt>& d, const Phys& P,
                                                      Rt divu, Rt SS, const Rt B[3],
                                                      const Rt J[3], Rt out[4])
{
    const Rt gamma = Rt(P.gamma), inv_cp = Rt(P.inv_cp), gm1 = Rt(P.gamma_m1);
    const Rt nu = Rt(P.nu), zeta = Rt(P.zeta), eta = Rt(P.eta);
    const Rt u[3] = {d.ux, d.uy, d.uz};
    const Rt inv_rho = exp(-d.lnrho);
    const Rt cs2 = Rt(P.cs0sq) * exp(gamma * d.ss * inv_cp + gm1 * (d.lnrho - Rt(P.lnrho0)));
    const Rt inv_T = Rt(P.cp_gm1) / cs2;

    Rt glnT2 = Rt(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Rt g = gamma * d.gs[a] * inv_cp + gm1 * d.gl[a];
        glnT2 += g * g;
    }
    const Rt laplnT = gamma * d.laps * inv_cp + gm1 * d.lapl;
    const Rt jj = J[0] * J[0] + J[1] * J[1] + J[2] * J[2];
    const Rt udgs = u[0] * d.gs[0] + u[1] * d.gs[1] + u[2] * d.gs[2];
    out[0] = -udgs + Rt(P.K) * inv_rho * (laplnT + glnT2) +
             inv_T * ((Rt(P.hc) + eta * Rt(P.mu0) * jj) * inv_rho + Rt(2) * nu * SS +
                      zeta * divu * divu);

    out[1] = u[1] * B[2] - u[2] * B[1] + eta * d.lapA[0];
    out[2] = u[2] * B[0] - u[0] * B[2] + eta * d.lapA[1];
    out[3] = u[0] * B[1] - u[1] * B[0] + eta * d.lapA[2];
}

// All of Eqs. B.1-B.4 at one cell: out[q] = d f_q / dt in field order.
template <typename Rt>
__device__ __forceinline__ void rhs_physics(const Derivs<Rt>& d, const Phys& P, Rt out[NQ])
{
    Rt S[3][3], divu, SS, B[3], J[3], jxB[3];
    shear(d.gu, S, divu, SS);
    magnetic(d, P, B, J, jxB);
    rhs_flow(d, P, S, divu, jxB, out);
    rhs_entropy_induction(d, P, divu, SS, B, J, out + 4);
}

// Kahan-compensated addition f <- f + y with running compensation c
// (FP32 storage variant).  Written with explicit round-to-nearest
// operations so the compiler cannot fuse or reassociate them.
__device__ __forceinline__ float kahan_add(float f, float y, float& c)
{
    const float yc = __fsub_rn(y, c);
    const float t = __fadd_rn(f, yc);
    c = __fsub_rn(__fsub_rn(t, f), yc);
    return t;
}

// The 6 side and 12 edge segments of a subdomain's boundary layer (the
// packed halo exchange of Section 3.3): per segment its direction d, its
// extents (r along every non-zero component of d, n_a otherwise) and its
// element offset in a packed buffer of all 8 fields.  Segment NSEG-1-k has
// direction -d of segment k.
constexpr int NSEG = 18;
struct SegTable {
    int64_t off[NSEG + 1];  // off[NSEG]: total elements
    int dir[NSEG][3];
    int len[NSEG][3];
};
SegTable seg_table(const Grid& g);

// ------------------------------------------------------------ launchers
hipError_t launch_halo(const Grid& g, void* fields, int elem_size, hipStream_t st);

// Pack (unpack false: interior boundary layer -> buf) or unpack (buf -> halo).
hipError_t launch_segments(const Grid& g, const SegTable& t, void* fields, void* buf,
                           int elem_size, bool unpack, hipStream_t st);


hipError_t launch_reduce(const Grid& g, const void* field, int elem_size, int op,
                         double* partials, int npartials, double* result, hipStream_t st);

constexpr int REDUCE_BLOCKS = 1024;

}  // namespace mhd

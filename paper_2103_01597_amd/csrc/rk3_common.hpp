// Pieces shared by the fused RHS + RK3 kernels: precision traits, the
// unscaled sixth-order stencil sums (Section 4, Eq. stencil-fd) and the
// per-cell 2N update with its FP32 compensated variant.
#pragma once

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

// First derivative times h along a stride st.
template <typename A, typename T>
__device__ __forceinline__ A deriv1(const T* p, int st)
{
    const A d1 = A(p[st]) - A(p[-st]);
    const A d2 = A(p[2 * st]) - A(p[-2 * st]);
    const A d3 = A(p[3 * st]) - A(p[-3 * st]);
    return A(C1_1) * d1 + A(C1_2) * d2 + A(C1_3) * d3;
}

// Pure second derivative times h^2 along a stride st.
template <typename A, typename T>
__device__ __forceinline__ A deriv2(const T* p, int st)
{
    const A s1 = A(p[st]) + A(p[-st]);
    const A s2 = A(p[2 * st]) + A(p[-2 * st]);
    const A s3 = A(p[3 * st]) + A(p[-3 * st]);
    return A(C2_0) * A(p[0]) + A(C2_1) * s1 + A(C2_2) * s2 + A(C2_3) * s3;
}

// Mixed second derivative times h_a h_b from the diagonals of the plane
// spanned by strides sa, sb: difference of the second differences along
// (+1, +1) and (+1, -1), divided by 4.
template <typename A, typename T>
__device__ __forceinline__ A derivm(const T* p, int sa, int sb)
{
    const int pp = sa + sb, pm = sa - sb;
    const A e1 = (A(p[pp]) + A(p[-pp])) - (A(p[pm]) + A(p[-pm]));
    const A e2 = (A(p[2 * pp]) + A(p[-2 * pp])) - (A(p[2 * pm]) + A(p[-2 * pm]));
    const A e3 = (A(p[3 * pp]) + A(p[-3 * pp])) - (A(p[3 * pm]) + A(p[-3 * pm]));
    return A(CM_1) * e1 + A(CM_2) * e2 + A(CM_3) * e3;
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

}  // namespace mhd

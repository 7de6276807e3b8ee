// Pieces shared by the fused RHS + RK3 kernels: precision traits, the
// unscaled stencil sums of order 2r (Section 4, Eq. stencil-fd) and the
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

}  // namespace mhd

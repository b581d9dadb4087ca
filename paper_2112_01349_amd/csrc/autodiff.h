// Forward-mode automatic differentiation of the reprojection residual: the
// Jacobian variant the paper calls "-a" (Sec. 5, JetVector; Sec. 6 tables),
// beside the analytic "-m" form of camera_model.h.
//
// A Dual<T, N> carries a value and N directional derivatives.  Every lane
// holds its own observation's duals in registers, so the derivative
// components of one parameter across a wavefront form the SoA vector the
// paper's JetVector stores.  The residual is written once, generically over
// the scalar type, and evaluated twice with N = 6 seeds (angle-axis and
// translation; then focal, k1, k2 and the point), which keeps the live duals
// within the register budget of FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <float.h>

namespace ba {

template <typename T, int N>
struct Dual {
    T v;
    T d[N];
};

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> dconst(T v)
{
    Dual<T, N> r;
    r.v = v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = (T)0;
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> dseed(T v, int slot)
{
    Dual<T, N> r = dconst<T, N>(v);
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = q == slot ? (T)1 : (T)0;
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b)
{
    Dual<T, N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = a.d[q] + b.d[q];
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b)
{
    Dual<T, N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = a.d[q] - b.d[q];
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator-(const Dual<T, N>& a)
{
    Dual<T, N> r;
    r.v = -a.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = -a.d[q];
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b)
{
    Dual<T, N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = a.d[q] * b.v + a.v * b.d[q];
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator*(T s, const Dual<T, N>& a)
{
    Dual<T, N> r;
    r.v = s * a.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = s * a.d[q];
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b)
{
    const T ib = (T)1 / b.v;
    Dual<T, N> r;
    r.v = a.v * ib;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = (a.d[q] - r.v * b.d[q]) * ib;
    return r;
}

template <typename T, int N>
__device__ __forceinline__ Dual<T, N> dsqrt(const Dual<T, N>& a)
{
    Dual<T, N> r;
    r.v = sqrt(a.v);
    const T h = (T)0.5 / r.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = h * a.d[q];
    return r;
}

template <typename T, int N>
__device__ __forceinline__ void dsincos(const Dual<T, N>& a, Dual<T, N>& s, Dual<T, N>& c)
{
    const T sv = sin(a.v), cv = cos(a.v);
    s.v = sv;
    c.v = cv;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        s.d[q] = cv * a.d[q];
        c.d[q] = -sv * a.d[q];
    }
}

// The BAL reprojection residual (the model of camera_model.h) over any scalar
// type S with the operators above: c = [w, t, f, k1, k2], X the point.  The
// rotation is applied to X directly by Rodrigues' formula,
//   R X = X cos th + (k x X) sin th + k (k . X)(1 - cos th),  k = w / th,
// with the first-order form X + w x X when th^2 <= DBL_EPSILON (decided on
// the value), as in the analytic form.
template <typename T, int N>
__device__ __forceinline__ void bal_residual(const Dual<T, N> c[9], const Dual<T, N> X[3], T u, T v,
                                             Dual<T, N>& e0, Dual<T, N>& e1)
{
    using D = Dual<T, N>;
    const D th2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    D P0, P1, P2;
    if ((double)th2.v > DBL_EPSILON) {
        const D th = dsqrt(th2);
        D s, co;
        dsincos(th, s, co);
        const D k0 = c[0] / th, k1 = c[1] / th, k2 = c[2] / th;
        const D kx0 = k1 * X[2] - k2 * X[1], kx1 = k2 * X[0] - k0 * X[2], kx2 = k0 * X[1] - k1 * X[0];
        const D kd = (k0 * X[0] + k1 * X[1] + k2 * X[2]) * (dconst<T, N>((T)1) - co);
        P0 = X[0] * co + kx0 * s + k0 * kd;
        P1 = X[1] * co + kx1 * s + k1 * kd;
        P2 = X[2] * co + kx2 * s + k2 * kd;
    } else {
        P0 = X[0] + (c[1] * X[2] - c[2] * X[1]);
        P1 = X[1] + (c[2] * X[0] - c[0] * X[2]);
        P2 = X[2] + (c[0] * X[1] - c[1] * X[0]);
    }
    P0 = P0 + c[3];
    P1 = P1 + c[4];
    P2 = P2 + c[5];
    const D px = -(P0 / P2), py = -(P1 / P2);
    const D r2 = px * px + py * py;
    const D fd = c[6] * (dconst<T, N>((T)1) + c[7] * r2 + c[8] * (r2 * r2));
    e0 = fd * px - dconst<T, N>(u);
    e1 = fd * py - dconst<T, N>(v);
}

// Residual and Jacobians by forward-mode differentiation: two evaluations
// with six seeds each (w, t; then f, k1, k2, X).  cam holds the FP64 camera
// parameters; Jc row-major 2x9, Jp row-major 2x3 (the layout of
// residual_jacobian).
template <typename T>
__device__ __forceinline__ void residual_jacobian_ad(const double* __restrict__ cam, T X0, T X1, T X2, T u, T v,
                                                     T& e0, T& e1, T Jc[18], T Jp[6])
{
    using D = Dual<T, 6>;
    D c[9], X[3], E0, E1;
#pragma unroll
    for (int q = 0; q < 9; ++q) c[q] = q < 6 ? dseed<T, 6>((T)cam[q], q) : dconst<T, 6>((T)cam[q]);
    X[0] = dconst<T, 6>(X0);
    X[1] = dconst<T, 6>(X1);
    X[2] = dconst<T, 6>(X2);
    bal_residual<T, 6>(c, X, u, v, E0, E1);
    e0 = E0.v;
    e1 = E1.v;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        Jc[q] = E0.d[q];
        Jc[9 + q] = E1.d[q];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) c[q] = q >= 6 ? dseed<T, 6>((T)cam[q], q - 6) : dconst<T, 6>((T)cam[q]);
    X[0] = dseed<T, 6>(X0, 3);
    X[1] = dseed<T, 6>(X1, 4);
    X[2] = dseed<T, 6>(X2, 5);
    bal_residual<T, 6>(c, X, u, v, E0, E1);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        Jc[6 + q] = E0.d[q];
        Jc[15 + q] = E1.d[q];
        Jp[q] = E0.d[3 + q];
        Jp[3 + q] = E1.d[3 + q];
    }
}

}  // namespace ba

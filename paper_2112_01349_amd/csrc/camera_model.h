// Camera model and its analytic Jacobian, shared by every kernel.
//
// Camera parameters (BAL convention of the paper's datasets, Sec. 6 dataset
// table): w (angle-axis, 3), t (3), f, k1, k2.
//   P = R(w) X + t,  p = -(Px, Py) / Pz,  d = 1 + k1 |p|^2 + k2 |p|^4,
//   u = f d p,  e = u - uv.
// Rotation: R(w) = cos(th) I + sin(th) [k]x + (1 - cos(th)) k k^T with
// th = |w|, k = w / th; when th^2 <= DBL_EPSILON the first-order form
// R = I + [w]x is used.
//
// Jacobian (the paper's analytic "-m" variant, Sec. 6):
//   de/dp   = f (d I + 2 (k1 + 2 k2 |p|^2) p p^T)          (2x2)
//   dp/dP   = -(1/Pz) [[1, 0, px], [0, 1, py]]             (2x3)
//   de/dP   = de/dp dp/dP;   de/dt = de/dP;   de/dX = de/dP R
//   de/dw   = de/dP (-[R X]x) J_l(w), J_l the left Jacobian of SO(3):
//             J_l = I + (1 - cos th)/th^2 [w]x + (th - sin th)/th^3 [w]x^2
//             (first-order branch: de/dw = de/dP (-[X]x))
//   de/df = d p,  de/dk1 = f |p|^2 p,  de/dk2 = f |p|^4 p.
#pragma once

#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

namespace ba {

// Per-camera constants, computed once per state from the FP64 parameters.
// The first 16 words are what an observation's geometry needs (one aligned
// 64-byte piece in FP32, 128 bytes in FP64); the record is 32 words.
template <typename T>
struct CamK {
    T R[9];   // row-major rotation
    T t[3];
    T f, k1, k2;
    T small;  // 1 in the first-order branch (use X instead of R X for de/dw)
    T Jl[9];  // left Jacobian of SO(3) at w; identity in the first-order branch
    T pad[7];
};
constexpr int kCamHead = 16;  // words of CamK read by observation_geometry

template <typename T>
__host__ __device__ inline void camera_constants(const double* c, CamK<T>& k)
{
    const double w0 = c[0], w1 = c[1], w2 = c[2];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    double R[9], J[9], small;
    if (th2 > DBL_EPSILON) {
        const double th = sqrt(th2);
        const double s = sin(th), co = cos(th);
        const double a0 = w0 / th, a1 = w1 / th, a2 = w2 / th;
        const double omc = 1.0 - co;
        R[0] = co + omc * a0 * a0;      R[1] = -s * a2 + omc * a0 * a1; R[2] = s * a1 + omc * a0 * a2;
        R[3] = s * a2 + omc * a1 * a0;  R[4] = co + omc * a1 * a1;      R[5] = -s * a0 + omc * a1 * a2;
        R[6] = -s * a1 + omc * a2 * a0; R[7] = s * a0 + omc * a2 * a1;  R[8] = co + omc * a2 * a2;
        const double c1 = omc / th2, c2 = (th - s) / (th2 * th);
        // [w]x^2 = w w^T - th^2 I
        const double W[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
        const double ww[9] = {w0 * w0 - th2, w0 * w1, w0 * w2, w1 * w0, w1 * w1 - th2,
                              w1 * w2, w2 * w0, w2 * w1, w2 * w2 - th2};
        for (int q = 0; q < 9; ++q) J[q] = ((q % 4) == 0 ? 1.0 : 0.0) + c1 * W[q] + c2 * ww[q];
        small = 0.0;
    } else {
        R[0] = 1.0; R[1] = -w2; R[2] = w1;
        R[3] = w2;  R[4] = 1.0; R[5] = -w0;
        R[6] = -w1; R[7] = w0;  R[8] = 1.0;
        for (int q = 0; q < 9; ++q) J[q] = (q % 4) == 0 ? 1.0 : 0.0;
        small = 1.0;
    }
    for (int q = 0; q < 9; ++q) {
        k.R[q] = (T)R[q];
        k.Jl[q] = (T)J[q];
    }
    k.t[0] = (T)c[3];
    k.t[1] = (T)c[4];
    k.t[2] = (T)c[5];
    k.f = (T)c[6];
    k.k1 = (T)c[7];
    k.k2 = (T)c[8];
    k.small = (T)small;
    for (int q = 0; q < 7; ++q) k.pad[q] = (T)0;
}

// Residual only, from the first 15 words of CamK (R, t, f, k1, k2).
template <typename T>
__device__ __forceinline__ void residual(const T* hd, T X0, T X1, T X2, T u, T v, T& e0, T& e1)
{
    const T P0 = hd[0] * X0 + hd[1] * X1 + hd[2] * X2 + hd[9];
    const T P1 = hd[3] * X0 + hd[4] * X1 + hd[5] * X2 + hd[10];
    const T P2 = hd[6] * X0 + hd[7] * X1 + hd[8] * X2 + hd[11];
    const T px = -(P0 / P2), py = -(P1 / P2);
    const T r2 = px * px + py * py;
    const T fd = hd[12] * ((T)1 + hd[13] * r2 + hd[14] * (r2 * r2));
    e0 = fd * px - u;
    e1 = fd * py - v;
}

template <typename T>
__device__ __forceinline__ void residual(const CamK<T>& k, T X0, T X1, T X2, T u, T v, T& e0, T& e1)
{
    residual<T>(k.R, X0, X1, X2, u, v, e0, e1);
}

// What the Jacobian of one observation is built from: de/dP (2x3), the
// projection p, the intrinsic factors and the lever arm of de/dw.  In terms
// of these, with J_l the camera's left Jacobian,
//   J_c = [ D (-[a]x) J_l | D | d p | f |p|^2 p | f |p|^4 p ],  J_p = D R.
template <typename T>
struct ObsGeo {
    T D[6];            // de/dP, row-major 2x3
    T px, py;          // p
    T fd;              // f d
    T d, fr2, fr4;     // d, f |p|^2, f |p|^4
    T a0, a1, a2;      // R X, or X in the first-order branch
};

// FP32 resolves P = R X + t only to ~1e-7 of |R X| + |t|: for a point within
// that of its camera's centre (a placement LM can drift into when a point's
// other views are outliers: from the centre every projection is available)
// the FP32 depth is made of rounding and the FP32 Jacobian overflows.  A
// depth is taken as resolved when it exceeds 2^-10 of the terms it is formed
// from; an unresolved one is formed again in FP64 (observation_geometry_f64).
// FP64 needs no such test.
template <typename T>
__device__ __forceinline__ bool depth_resolved(T RX2, T t2, T P2)
{
    if (sizeof(T) == 8) return true;
    return fabs(P2) > (T)(1.0 / 1024.0) * (fabs(RX2) + fabs(t2));
}

// hd: the first kCamHead words of the camera's CamK (R, t, f, k1, k2, small).
// Returns false for an unresolved FP32 depth, with every derivative set to
// zero (the caller forms the geometry in FP64 instead where it can).
template <typename T>
__device__ __forceinline__ bool observation_geometry(const T* hd, T X0, T X1, T X2, ObsGeo<T>& o)
{
    const T RX0 = hd[0] * X0 + hd[1] * X1 + hd[2] * X2;
    const T RX1 = hd[3] * X0 + hd[4] * X1 + hd[5] * X2;
    const T RX2 = hd[6] * X0 + hd[7] * X1 + hd[8] * X2;
    T P0 = RX0 + hd[9], P1 = RX1 + hd[10];
    const T P2 = RX2 + hd[11];
    const T f = hd[12], k1 = hd[13], k2 = hd[14];
    // FP32: the hardware reciprocal (1 ulp) in place of a correctly rounded
    // division, well inside the form's own rounding
    T iz = sizeof(T) == 4 ? (T)__builtin_amdgcn_rcpf((float)P2) : (T)1 / P2;
    const bool resolved = depth_resolved<T>(RX2, hd[11], P2);
    if (!resolved) P0 = P1 = iz = (T)0;  // all derivatives vanish
    const T px = -(P0 * iz), py = -(P1 * iz);
    const T r2 = px * px + py * py;
    const T d = (T)1 + k1 * r2 + k2 * (r2 * r2);
    const T fd = f * d;
    const T g = (T)2 * f * (k1 + (T)2 * k2 * r2);
    const T A00 = fd + g * px * px, A01 = g * px * py, A11 = fd + g * py * py;
    o.D[0] = -iz * A00;
    o.D[1] = -iz * A01;
    o.D[2] = -iz * (A00 * px + A01 * py);
    o.D[3] = -iz * A01;
    o.D[4] = -iz * A11;
    o.D[5] = -iz * (A01 * px + A11 * py);
    o.px = px;
    o.py = py;
    o.fd = fd;
    o.d = d;
    o.fr2 = f * r2;
    o.fr4 = o.fr2 * r2;
    const bool sm = hd[15] != (T)0;
    o.a0 = sm ? X0 : RX0;
    o.a1 = sm ? X1 : RX1;
    o.a2 = sm ? X2 : RX2;
    return resolved;
}

// The geometry formed in FP64 from the camera's FP64 constants and the FP64
// point, stored in T: the FP32 form's path for an unresolved depth (rare, so
// kept out of line).
template <typename T>
__device__ __attribute__((noinline)) ObsGeo<T> observation_geometry_f64(const CamK<double>* __restrict__ ck64,
                                                                        int32_t j, const double* __restrict__ X)
{
    ObsGeo<double> g;
    observation_geometry<double>(ck64[j].R, X[0], X[1], X[2], g);
    ObsGeo<T> o;
#pragma unroll
    for (int q = 0; q < 6; ++q) o.D[q] = (T)g.D[q];
    o.px = (T)g.px;
    o.py = (T)g.py;
    o.fd = (T)g.fd;
    o.d = (T)g.d;
    o.fr2 = (T)g.fr2;
    o.fr4 = (T)g.fr4;
    o.a0 = (T)g.a0;
    o.a1 = (T)g.a1;
    o.a2 = (T)g.a2;
    return o;
}

// The geometry of one observation in T; an unresolved FP32 depth is formed in
// FP64 when the FP64 constants are at hand (ck64), else left with zero
// derivatives.
template <typename T>
__device__ __forceinline__ void observation_geometry_checked(const T* hd, const CamK<double>* __restrict__ ck64,
                                                             int32_t j, const double* __restrict__ X, ObsGeo<T>& o)
{
    if (!observation_geometry<T>(hd, (T)X[0], (T)X[1], (T)X[2], o) && ck64) o = observation_geometry_f64<T>(ck64, j, X);
}

// Residual and Jacobians from the geometry: Jc row-major 2x9, Jp row-major
// 2x3.  R: the camera's rotation (row-major), Jl: its left Jacobian.
template <typename T>
__device__ __forceinline__ void jacobian_from_geometry(const T* R, const T* Jl, const ObsGeo<T>& o, T u, T v, T& e0,
                                                       T& e1, T Jc[18], T Jp[6])
{
    e0 = o.fd * o.px - u;
    e1 = o.fd * o.py - v;
    const T* D = o.D;
    // y_r = a x D_r  (row r of de/dP (-[a]x)), then de/dw_r = y_r J_l
    const T y00 = o.a1 * D[2] - o.a2 * D[1], y01 = o.a2 * D[0] - o.a0 * D[2], y02 = o.a0 * D[1] - o.a1 * D[0];
    const T y10 = o.a1 * D[5] - o.a2 * D[4], y11 = o.a2 * D[3] - o.a0 * D[5], y12 = o.a0 * D[4] - o.a1 * D[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Jc[c] = y00 * Jl[c] + y01 * Jl[3 + c] + y02 * Jl[6 + c];
        Jc[9 + c] = y10 * Jl[c] + y11 * Jl[3 + c] + y12 * Jl[6 + c];
        Jp[c] = D[0] * R[c] + D[1] * R[3 + c] + D[2] * R[6 + c];
        Jp[3 + c] = D[3] * R[c] + D[4] * R[3 + c] + D[5] * R[6 + c];
    }
    Jc[3] = D[0]; Jc[4] = D[1]; Jc[5] = D[2];
    Jc[12] = D[3]; Jc[13] = D[4]; Jc[14] = D[5];
    Jc[6] = o.d * o.px;
    Jc[15] = o.d * o.py;
    Jc[7] = o.fr2 * o.px;
    Jc[16] = o.fr2 * o.py;
    Jc[8] = o.fr4 * o.px;
    Jc[17] = o.fr4 * o.py;
}

template <typename T>
__device__ __forceinline__ void jacobian_from_geometry(const CamK<T>& k, const ObsGeo<T>& o, T u, T v, T& e0, T& e1,
                                                       T Jc[18], T Jp[6])
{
    jacobian_from_geometry<T>(k.R, k.Jl, o, u, v, e0, e1, Jc, Jp);
}

template <typename T>
__device__ __forceinline__ void residual_jacobian(const CamK<T>& k, T X0, T X1, T X2, T u, T v,
                                                  T& e0, T& e1, T Jc[18], T Jp[6])
{
    ObsGeo<T> o;
    observation_geometry<T>(k.R, X0, X1, X2, o);
    jacobian_from_geometry<T>(k, o, u, v, e0, e1, Jc, Jp);
}

// Huber on the 2-D residual norm, s = |e|^2: rho(s) = s for s <= delta^2,
// else 2 delta sqrt(s) - delta^2; delta <= 0 is the squared loss.  The
// IRLS weight is rho'(s).
template <typename T>
__device__ __forceinline__ T huber_rho(T s, T delta)
{
    return (delta <= (T)0 || s <= delta * delta) ? s : (T)2 * delta * sqrt(s) - delta * delta;
}

template <typename T>
__device__ __forceinline__ T huber_weight(T s, T delta)
{
    return (delta <= (T)0 || s <= delta * delta) ? (T)1 : delta / sqrt(s);
}

}  // namespace ba

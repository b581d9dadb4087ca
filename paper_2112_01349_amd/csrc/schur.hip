// Damping, block inverses and the back-substitution from stored blocks.
//
//   * k_damp_cameras: B~_j = B_j + lambda D_j and its Cholesky factor, FP64
//     (the block-Jacobi preconditioner of Alg. 2 and the B x term of Alg. 3).
//   * k_factor_schur_jacobi: the Schur-Jacobi option's preconditioner blocks
//     M_j = S_jj (per-observation terms) and their factors, replacing B~_j's.
//   * k_damp_points:  C~_i = C_i + lambda D_i and its explicit inverse (Alg. 3
//     b = C^-1 a, Eq. schur_x_p), one lane per point.
//   * k_backsub_stored: dp = C~^-1 (w - E^T x) (Eq. schur_x_p) over
//     point-aligned tiles of <= 256 observations, reading E as 27 coalesced
//     streams, for the stored-block product; the per-point sums run over the
//     point's contiguous segment in LDS.
// Damping (Reading of Sec. 3 and supplementary Sec. C): D = clamp(diag, 1e-6,
// 1e32) (Marquardt, Ceres-like) or D = I (as printed in Sec. 3).
#include "ba_internal.h"

namespace ba {

__device__ __forceinline__ double clamp_diag(double h)
{
    return h < 1e-6 ? 1e-6 : (h > 1e32 ? 1e32 : h);
}

// packed lower-triangular index (r >= c)
__host__ __device__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

// In-place Cholesky factor of a packed lower-triangular 9x9 block; false
// (with unit pivots substituted) when it is not positive definite.
__device__ __forceinline__ bool cholesky9(double L[45])
{
    bool ok = true;
    for (int c = 0; c < 9; ++c) {
        double sd = L[tri(c, c)];
        for (int t = 0; t < c; ++t) sd -= L[tri(c, t)] * L[tri(c, t)];
        if (!(sd > 0.0)) {
            ok = false;
            sd = 1.0;
        }
        const double d = sqrt(sd);
        L[tri(c, c)] = d;
        for (int r = c + 1; r < 9; ++r) {
            double x = L[tri(r, c)];
            for (int t = 0; t < c; ++t) x -= L[tri(r, t)] * L[tri(c, t)];
            L[tri(r, c)] = x / d;
        }
    }
    return ok;
}

// The factor as the PCG step applies it: the lower triangle with each
// diagonal entry replaced by its reciprocal, so the two triangular solves
// multiply instead of divide.
__device__ __forceinline__ void store_factor(const double L[45], double* __restrict__ out)
{
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) out[tri(r, c)] = r == c ? 1.0 / L[tri(r, c)] : L[tri(r, c)];
}

__global__ void k_damp_cameras(int32_t m, const double* __restrict__ hcc, double lambda, int32_t damping,
                               double* __restrict__ bd, double* __restrict__ lfac, double* __restrict__ dcam,
                               int32_t* __restrict__ flag)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const double* H = hcc + 81 * (int64_t)j;
    double L[45];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c <= r; ++c) L[tri(r, c)] = H[r * 9 + c];
    for (int a = 0; a < 9; ++a) {
        const double D = damping == 0 ? clamp_diag(H[a * 10]) : 1.0;
        dcam[9 * (int64_t)j + a] = D;
        L[tri(a, a)] += lambda * D;
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
            const double v = r >= c ? L[tri(r, c)] : L[tri(c, r)];
            bd[81 * (int64_t)j + r * 9 + c] = v;
        }
    const bool ok = cholesky9(L);
    store_factor(L, lfac + 45 * (int64_t)j);
    if (!ok) {
        atomicOr(flag, 1);
        flag[1] = j;  // one of the failing cameras (for the error message)
    }
}

// Schur-Jacobi preconditioner: M_j = B~_j + mj_j (mj holding the negated
// per-camera sums of E C~^-1 E^T) and its Cholesky factor into lfac, in
// place of the factor of B~_j.  Failure flags as the camera blocks.
__global__ void k_factor_schur_jacobi(int32_t m, const double* __restrict__ bd, const double* __restrict__ mj,
                                      double* __restrict__ lfac, int32_t* __restrict__ flag)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double L[45];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c <= r; ++c) L[tri(r, c)] = bd[81 * (int64_t)j + r * 9 + c] + mj[81 * (int64_t)j + r * 9 + c];
    const bool ok = cholesky9(L);
    store_factor(L, lfac + 45 * (int64_t)j);
    if (!ok) {
        atomicOr(flag, 1);
        flag[1] = j;
    }
}

hipError_t launch_factor_schur_jacobi(int32_t m, const double* bd, const double* mj, double* lfac, int32_t* flag,
                                      hipStream_t s)
{
    if (m > 0)
        hipLaunchKernelGGL(k_factor_schur_jacobi, dim3((m + 63) / 64), dim3(64), 0, s, m, bd, mj, lfac, flag);
    return hipGetLastError();
}

hipError_t launch_damp_cameras(int32_t m, const double* hcc, double lambda, int32_t damping, double* bd,
                               double* lfac, double* dcam, int32_t* flag, hipStream_t s)
{
    if (m > 0)
        hipLaunchKernelGGL(k_damp_cameras, dim3((m + 63) / 64), dim3(64), 0, s, m, hcc, lambda, damping, bd, lfac,
                           dcam, flag);
    return hipGetLastError();
}

// C~ = C + lambda D, inverse through its Cholesky factor; packed symmetric
// order (00, 01, 02, 11, 12, 22).
template <typename T>
__global__ void k_damp_points(int32_t n, const double* __restrict__ hpp, double lambda, int32_t damping,
                              T* __restrict__ cinv, int32_t* __restrict__ flag)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* h = hpp + 6 * (int64_t)i;
    double a00 = h[0], a01 = h[1], a02 = h[2], a11 = h[3], a12 = h[4], a22 = h[5];
    const double lam = lambda;
    if (damping == 0) {
        a00 += lam * clamp_diag(a00);
        a11 += lam * clamp_diag(a11);
        a22 += lam * clamp_diag(a22);
    } else {
        a00 += lam;
        a11 += lam;
        a22 += lam;
    }
    bool ok = a00 > 0.0;
    const double l00 = sqrt(ok ? a00 : 1.0);
    const double l10 = a01 / l00, l20 = a02 / l00;
    double s11 = a11 - l10 * l10;
    ok = ok && s11 > 0.0;
    const double l11 = sqrt(s11 > 0.0 ? s11 : 1.0);
    const double l21 = (a12 - l20 * l10) / l11;
    double s22 = a22 - l20 * l20 - l21 * l21;
    ok = ok && s22 > 0.0;
    const double l22 = sqrt(s22 > 0.0 ? s22 : 1.0);
    const double m00 = 1.0 / l00, m11 = 1.0 / l11, m22 = 1.0 / l22;
    const double m10 = -l10 * m00 * m11;
    const double m21 = -l21 * m11 * m22;
    const double m20 = -(l20 * m00 + l21 * m10) * m22;
    T* o = cinv + 6 * (int64_t)i;
    o[0] = (T)(m00 * m00 + m10 * m10 + m20 * m20);
    o[1] = (T)(m10 * m11 + m20 * m21);
    o[2] = (T)(m20 * m22);
    o[3] = (T)(m11 * m11 + m21 * m21);
    o[4] = (T)(m21 * m22);
    o[5] = (T)(m22 * m22);
    if (!ok) {
        atomicOr(flag, 2);
        flag[2] = i;  // one of the failing points (for the error message)
    }
}

template <typename T>
hipError_t launch_damp_points(int32_t n, const double* hpp, double lambda, int32_t damping, T* cinv, int32_t* flag,
                              hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL((k_damp_points<T>), dim3((n + 255) / 256), dim3(256), 0, s, n, hpp, lambda, damping, cinv,
                           flag);
    return hipGetLastError();
}

// ------------------------------------------- back-substitution (stored E)
template <typename T>
__device__ __forceinline__ void sym3_apply(const T* __restrict__ ci, T a0, T a1, T a2, T& b0, T& b1, T& b2)
{
    const T c00 = ci[0], c01 = ci[1], c02 = ci[2], c11 = ci[3], c12 = ci[4], c22 = ci[5];
    b0 = c00 * a0 + c01 * a1 + c02 * a2;
    b1 = c01 * a0 + c11 * a1 + c12 * a2;
    b2 = c02 * a0 + c12 * a1 + c22 * a2;
}

// dp_i = C~_i^-1 (w_i - sum_k E_k^T dc_j) from the stored blocks, one
// workgroup per point-aligned tile (a point longer than the tile is one tile,
// summed by a tree in LDS).
template <typename T>
__global__ __launch_bounds__(kTile) void k_backsub_stored(const int32_t* __restrict__ tile,
                                                          const int32_t* __restrict__ cam,
                                                          const int32_t* __restrict__ pt, const T* __restrict__ hcp,
                                                          const T* __restrict__ cinv, const double* __restrict__ wpt,
                                                          const T* __restrict__ xcam, double* __restrict__ dp)
{
    __shared__ T sha[3][kTile];
    __shared__ int32_t shpt[kTile];
    const int tid = threadIdx.x;
    const int32_t s = tile[blockIdx.x], e = tile[blockIdx.x + 1];
    const int32_t len = e - s;
    if (len <= kTile) {
        const bool valid = tid < len;
        const int64_t k = s + tid;
        int32_t i = -1;
        if (valid) {
            const int32_t j = cam[k];
            i = pt[k];
            T x[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) x[a] = xcam[9 * (int64_t)j + a];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                T acc = 0;
#pragma unroll
                for (int a = 0; a < 9; ++a) acc += hcp[eidx(k, a * 3 + b)] * x[a];
                sha[b][tid] = acc;
            }
        }
        shpt[tid] = i;
        __syncthreads();
        if (valid && (tid == 0 || shpt[tid - 1] != i)) {
            T a0 = 0, a1 = 0, a2 = 0;
            for (int u = tid; u < len && shpt[u] == i; ++u) {
                a0 += sha[0][u];
                a1 += sha[1][u];
                a2 += sha[2][u];
            }
            T b0, b1, b2;
            sym3_apply<T>(cinv + 6 * (int64_t)i, (T)wpt[3 * (int64_t)i] - a0, (T)wpt[3 * (int64_t)i + 1] - a1,
                          (T)wpt[3 * (int64_t)i + 2] - a2, b0, b1, b2);
            dp[3 * (int64_t)i] = (double)b0;
            dp[3 * (int64_t)i + 1] = (double)b1;
            dp[3 * (int64_t)i + 2] = (double)b2;
        }
    } else {
        // one point with more than kTile observations
        const int32_t i = pt[s];
        T a0 = 0, a1 = 0, a2 = 0;
        for (int32_t base = s; base < e; base += kTile) {
            const int64_t k = base + tid;
            if (k < e) {
                const int32_t j = cam[k];
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    T acc = 0;
#pragma unroll
                    for (int a = 0; a < 9; ++a) acc += hcp[eidx(k, a * 3 + b)] * xcam[9 * (int64_t)j + a];
                    if (b == 0) a0 += acc;
                    if (b == 1) a1 += acc;
                    if (b == 2) a2 += acc;
                }
            }
        }
        sha[0][tid] = a0;
        sha[1][tid] = a1;
        sha[2][tid] = a2;
        __syncthreads();
        for (int stride = kTile / 2; stride > 0; stride >>= 1) {
            if (tid < stride)
                for (int b = 0; b < 3; ++b) sha[b][tid] += sha[b][tid + stride];
            __syncthreads();
        }
        if (tid == 0) {
            T b0, b1, b2;
            sym3_apply<T>(cinv + 6 * (int64_t)i, (T)wpt[3 * (int64_t)i] - sha[0][0],
                          (T)wpt[3 * (int64_t)i + 1] - sha[1][0], (T)wpt[3 * (int64_t)i + 2] - sha[2][0], b0, b1,
                          b2);
            dp[3 * (int64_t)i] = (double)b0;
            dp[3 * (int64_t)i + 1] = (double)b1;
            dp[3 * (int64_t)i + 2] = (double)b2;
        }
    }
}

template <typename T>
hipError_t launch_backsub_stored(const PointMajor& pm, const T* hcp, const T* cinv, const double* wpt,
                                 const T* xcam, double* dp, hipStream_t s)
{
    if (pm.num_tiles > 0)
        hipLaunchKernelGGL((k_backsub_stored<T>), dim3(pm.num_tiles), dim3(kTile), 0, s, pm.tile, pm.cam, pm.pt, hcp,
                           cinv, wpt, xcam, dp);
    return hipGetLastError();
}

template hipError_t launch_damp_points<double>(int32_t, const double*, double, int32_t, double*, int32_t*, hipStream_t);
template hipError_t launch_damp_points<float>(int32_t, const double*, double, int32_t, float*, int32_t*, hipStream_t);
template hipError_t launch_backsub_stored<double>(const PointMajor&, const double*, const double*, const double*,
                                                  const double*, double*, hipStream_t);
template hipError_t launch_backsub_stored<float>(const PointMajor&, const float*, const float*, const double*,
                                                 const float*, double*, hipStream_t);

}  // namespace ba

// Camera-sized vector work of the PCG loop (Alg. 2 with one partition) and
// the small per-iteration kernels of the LM loop (trial state, predicted
// decrease, parameter gathers).  All vectors and scalars are FP64.  Every
// reduction writes per-block partial sums that k_sum_partials adds in a fixed
// order, so results do not depend on scheduling.
//
// PCG (Alg. 2, with the printed index slips read as: the beta branch runs for
// n >= 1, p^n = z^n + beta p^{n-1}, r^{n+1} = r^n - alpha q^n):
//   z = M^-1 r (M = blockdiag of the damped camera blocks B~_j, through their
//   Cholesky factors), rho = r^T z, p = z + beta p, q = S p,
//   alpha = rho / p^T q, x += alpha p, r -= alpha q.
#include "ba_internal.h"

namespace ba {

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block sum of up to two values into partials[blockIdx * 2 + {0,1}].
template <int NV>
__device__ __forceinline__ void block_partials(double v0, double v1, double* __restrict__ partials)
{
    __shared__ double sh[2][kRedBlock / 64];
    v0 = wave_sum64(v0);
    if (NV > 1) v1 = wave_sum64(v1);
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = v0;
        sh[1][threadIdx.x >> 6] = v1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kRedBlock / 64; ++w) {
            a += sh[0][w];
            b += sh[1][w];
        }
        partials[(int64_t)blockIdx.x * NV] = a;
        if (NV > 1) partials[(int64_t)blockIdx.x * NV + 1] = b;
    }
}

__global__ void k_zero(double* __restrict__ p, int64_t count)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0.0;
}

hipError_t launch_zero(double* p, int64_t count, hipStream_t s)
{
    if (count > 0) {
        int64_t b = (count + 255) / 256;
        if (b > 4096) b = 4096;
        hipLaunchKernelGGL(k_zero, dim3((unsigned)b), dim3(256), 0, s, p, count);
    }
    return hipGetLastError();
}

// Sums `count` rows of `stride` doubles column-wise (ncols <= stride) in a
// fixed order; one block.
__global__ __launch_bounds__(kRedBlock) void k_sum_partials(const double* __restrict__ partials, int32_t count,
                                                            int32_t stride, int32_t ncols, double* __restrict__ out)
{
    __shared__ double sh[kRedBlock / 64];
    for (int c = 0; c < ncols; ++c) {
        double acc = 0.0;
        for (int32_t t = threadIdx.x; t < count; t += kRedBlock) acc += partials[(int64_t)t * stride + c];
        acc = wave_sum64(acc);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kRedBlock / 64; ++w) t += sh[w];
            out[c] = t;
        }
        __syncthreads();
    }
}

hipError_t launch_sum_partials(const double* partials, int32_t count, int32_t stride, int32_t ncols, double* out,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRedBlock), 0, s, partials, count, stride, ncols, out);
    return hipGetLastError();
}

__global__ void k_pcg_reset(PcgScalars* __restrict__ sc, double rtol, int32_t max_iters, int32_t fixed)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc->rho = sc->rho_prev = sc->pq = sc->rr = sc->bb = sc->alpha = sc->beta = 0.0;
    sc->rtol = rtol;
    sc->max_iters = max_iters;
    sc->fixed = fixed;
    sc->iters = 0;
    sc->done = 0;
    sc->breakdown = 0;
    sc->arrive[0] = sc->arrive[1] = sc->arrive[2] = 0u;
}

hipError_t launch_pcg_reset(PcgScalars* sc, double rtol, int32_t max_iters, int32_t fixed, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_reset, dim3(1), dim3(64), 0, s, sc, rtol, max_iters, fixed);
    return hipGetLastError();
}

__host__ __device__ constexpr int tri2(int r, int c) { return r * (r + 1) / 2 + c; }

// (Unless first) x += alpha p, r -= alpha q, then z = (L L^T)^-1 r with each
// camera block's Cholesky factor.  A workgroup takes kStepCams cameras: their
// vector entries and factors are read and written in contiguous runs through
// LDS, and one lane per camera does the two triangular solves there.  The last
// block adds rho = r^T z and ||r||^2 over all blocks and takes the decision
// the next matvec depends on: stop (converged or count reached) or continue
// with beta = rho / rho_prev.
constexpr int kStepCams = 64;

__global__ __launch_bounds__(kRedBlock) void k_pcg_step(int32_t m, int first, const double* __restrict__ lfac,
                                                        const double* __restrict__ p, const double* __restrict__ q,
                                                        double* __restrict__ x, double* __restrict__ r,
                                                        double* __restrict__ z, double* __restrict__ partials,
                                                        PcgScalars* __restrict__ sc)
{
    __shared__ double sl[kStepCams * 45];
    __shared__ double sr[kStepCams * 9];
    if (sc->done) return;  // uniform: nobody writes `done` while this kernel runs
    const double alpha = first ? 0.0 : sc->alpha;
    double rz = 0.0, rr = 0.0;
    const int32_t groups = (m + kStepCams - 1) / kStepCams;
    // entries of the group's vectors and factors per thread; every load of a
    // group is issued before any is used (indices past the group's end read
    // its first entry and are not used)
    constexpr int UV = (9 * kStepCams + kRedBlock - 1) / kRedBlock;
    constexpr int UL = (45 * kStepCams + kRedBlock - 1) / kRedBlock;
    for (int32_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int32_t j0 = g * kStepCams;
        const int32_t nc = min(kStepCams, m - j0);
        const int64_t e0 = 9 * (int64_t)j0;
        const int nv = 9 * nc, nl = 45 * nc;
        double rv[UV], xv[UV], pv[UV], qv[UV], lv[UL];
#pragma unroll
        for (int u = 0; u < UV; ++u) {
            const int t = threadIdx.x + u * kRedBlock;
            const int64_t e = e0 + (t < nv ? t : 0);
            rv[u] = r[e];
            if (!first) {
                xv[u] = x[e];
                pv[u] = p[e];
                qv[u] = q[e];
            }
        }
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int t = threadIdx.x + u * kRedBlock;
            lv[u] = lfac[45 * (int64_t)j0 + (t < nl ? t : 0)];
        }
#pragma unroll
        for (int u = 0; u < UV; ++u) {
            const int t = threadIdx.x + u * kRedBlock;
            if (t < nv) {
                double v = rv[u];
                if (!first) {
                    x[e0 + t] = xv[u] + alpha * pv[u];
                    v -= alpha * qv[u];
                    r[e0 + t] = v;
                }
                sr[t] = v;
            }
        }
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int t = threadIdx.x + u * kRedBlock;
            if (t < nl) sl[t] = lv[u];
        }
        __syncthreads();
        if (threadIdx.x < nc) {
            const double* L = sl + 45 * threadIdx.x;
            double* rj = sr + 9 * threadIdx.x;
            double rv[9], y[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) rv[a] = rj[a];
            // the factor's diagonal holds reciprocals (store_factor)
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                double v = rv[a];
#pragma unroll
                for (int t = 0; t < a; ++t) v -= L[tri2(a, t)] * y[t];
                y[a] = v * L[tri2(a, a)];
            }
#pragma unroll
            for (int a = 8; a >= 0; --a) {
                double v = y[a];
#pragma unroll
                for (int t = a + 1; t < 9; ++t) v -= L[tri2(t, a)] * y[t];
                y[a] = v * L[tri2(a, a)];
            }
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                rz += rv[a] * y[a];
                rr += rv[a] * rv[a];
                rj[a] = y[a];  // z replaces r in LDS
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < UV; ++u) {
            const int t = threadIdx.x + u * kRedBlock;
            if (t < nv) z[e0 + t] = sr[t];
        }
        __syncthreads();
    }
    block_partials<2>(rz, rr, partials);
    if (!last_block_arrives(&sc->arrive[0])) return;
    __shared__ double sh2[2][kRedBlock / 64];
    double a = 0.0, b = 0.0;
    for (int32_t t = threadIdx.x; t < (int32_t)gridDim.x; t += kRedBlock) {
        a += partials[2 * (int64_t)t];
        b += partials[2 * (int64_t)t + 1];
    }
    a = wave_sum64(a);
    b = wave_sum64(b);
    if ((threadIdx.x & 63) == 0) {
        sh2[0][threadIdx.x >> 6] = a;
        sh2[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double rho = 0.0, rrs = 0.0;
        for (int w = 0; w < kRedBlock / 64; ++w) {
            rho += sh2[0][w];
            rrs += sh2[1][w];
        }
        const int32_t it = sc->iters;
        sc->rr = rrs;
        const bool stop = sc->fixed > 0 ? it >= sc->fixed
                                        : (sqrt(rrs) <= sc->rtol * sqrt(sc->bb) || it >= sc->max_iters);
        if (stop) {
            sc->done = 1;
        } else {
            sc->beta = it == 0 ? 0.0 : rho / sc->rho;
            sc->rho_prev = sc->rho;
            sc->rho = rho;
        }
        sc->arrive[0] = 0u;
    }
}

hipError_t launch_pcg_step(int32_t m, bool first, const double* lfac, const double* p, const double* q, double* x,
                           double* r, double* z, double* partials, PcgScalars* sc, hipStream_t s)
{
    // one block per group of cameras (the partial sums hold 2048 blocks;
    // beyond that each block loops over several groups)
    int32_t b = (m + kStepCams - 1) / kStepCams;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_pcg_step, dim3(b), dim3(kRedBlock), 0, s, m, first ? 1 : 0, lfac, p, q, x, r, z, partials, sc);
    return hipGetLastError();
}

// p = z (first iteration) or z + beta p; pT = (T) p.  With xf set, also the
// camera vectors the recomputing Schur product reads: [J_l p_w, p_t, p_f,
// p_k1, p_k2] in T (12 words per camera, the last three unused).  A
// workgroup takes kStepCams cameras; vectors are read and written in
// contiguous runs, the new p passing through LDS for the J_l products.
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_pcg_direction(int32_t m, int force, const double* __restrict__ z,
                                                             double* __restrict__ p, T* __restrict__ pT,
                                                             const CamK<T>* __restrict__ ck, T* __restrict__ xf,
                                                             const PcgScalars* __restrict__ sc)
{
    __shared__ double sv[kStepCams * 9];
    if (!force && sc->done) return;
    const bool first = force || sc->iters == 0;
    const double beta = first ? 0.0 : sc->beta;
    const int32_t groups = (m + kStepCams - 1) / kStepCams;
    // loads of a group issued before any is used, as in k_pcg_step
    constexpr int UV = (9 * kStepCams + kRedBlock - 1) / kRedBlock;
    constexpr int UX = (12 * kStepCams + kRedBlock - 1) / kRedBlock;
    for (int32_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int32_t j0 = g * kStepCams;
        const int32_t nc = min(kStepCams, m - j0);
        const int64_t e0 = 9 * (int64_t)j0;
        const int nv = 9 * nc, nx = 12 * nc;
        double zv[UV], pv[UV];
#pragma unroll
        for (int u = 0; u < UV; ++u) {
            const int t = threadIdx.x + u * kRedBlock;
            const int64_t e = e0 + (t < nv ? t : 0);
            zv[u] = z[e];
            pv[u] = first ? 0.0 : p[e];
        }
#pragma unroll
        for (int u = 0; u < UV; ++u) {
            const int t = threadIdx.x + u * kRedBlock;
            if (t < nv) {
                const double v = first ? zv[u] : zv[u] + beta * pv[u];
                p[e0 + t] = v;
                pT[e0 + t] = (T)v;
                sv[t] = v;
            }
        }
        if (xf) {
            // J_l rows of the lanes that form J_l p_w (a < 3), loaded before the barrier
            T J[UX][3];
#pragma unroll
            for (int u = 0; u < UX; ++u) {
                const int t = threadIdx.x + u * kRedBlock;
                const int tt = t < nx ? t : 0;
                const int c = tt / 12, a = tt - 12 * c;
                const T* Jr = ck[j0 + c].Jl + 3 * (a < 3 ? a : 0);
                J[u][0] = Jr[0];
                J[u][1] = Jr[1];
                J[u][2] = Jr[2];
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < UX; ++u) {
                const int t = threadIdx.x + u * kRedBlock;
                if (t < nx) {
                    const int c = t / 12, a = t - 12 * c;
                    const double* v = sv + 9 * c;
                    T o = (T)0;
                    if (a < 3)
                        o = (T)((double)J[u][0] * v[0] + (double)J[u][1] * v[1] + (double)J[u][2] * v[2]);
                    else if (a < 9)
                        o = (T)v[a];
                    xf[12 * (int64_t)j0 + t] = o;
                }
            }
        }
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_pcg_direction(int32_t m, bool force, const double* z, double* p, T* pT, const CamK<T>* ck, T* xf,
                                PcgScalars* sc, hipStream_t s)
{
    int32_t b = (m + kStepCams - 1) / kStepCams;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL((k_pcg_direction<T>), dim3((unsigned)b), dim3(kRedBlock), 0, s, m, force ? 1 : 0, z, p, pT,
                       ck, xf, sc);
    return hipGetLastError();
}

// ------------------------------------------------------------ LM helpers
__global__ void k_trial_state(int64_t lc, int64_t lp, const double* __restrict__ cams, const double* __restrict__ dc,
                              const double* __restrict__ pts, const double* __restrict__ dp,
                              double* __restrict__ cams_t, double* __restrict__ pts_t)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < lc + lp; t += (int64_t)gridDim.x * blockDim.x) {
        if (t < lc) cams_t[t] = cams[t] + dc[t];
        else pts_t[t - lc] = pts[t - lc] + dp[t - lc];
    }
}

hipError_t launch_trial_state(int32_t m, int32_t n, const double* cams, const double* dc, const double* pts,
                              const double* dp, double* cams_t, double* pts_t, hipStream_t s)
{
    const int64_t lc = 9 * (int64_t)m, lp = 3 * (int64_t)n;
    int64_t b = (lc + lp + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_trial_state, dim3((unsigned)b), dim3(256), 0, s, lc, lp, cams, dc, pts, dp, cams_t, pts_t);
    return hipGetLastError();
}

__device__ __forceinline__ double clamp_d(double h) { return h < 1e-6 ? 1e-6 : (h > 1e32 ? 1e32 : h); }

// pred terms: dc^T (lambda D_c dc + v) over cameras, dp^T (lambda D_p dp + w) over points
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_pred(int64_t lc, int64_t lp, const double* __restrict__ dc,
                                                    const double* __restrict__ dcam, const double* __restrict__ vcam,
                                                    const double* __restrict__ dp, const double* __restrict__ hpp,
                                                    const double* __restrict__ wpt, double lambda, int32_t damping,
                                                    double* __restrict__ partials)
{
    double a = 0.0, b = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; t < lc + lp; t += (int64_t)gridDim.x * kRedBlock) {
        if (t < lc) {
            a += dc[t] * (lambda * dcam[t] * dc[t] + vcam[t]);
        } else {
            const int64_t u = t - lc;
            const int64_t i = u / 3;
            const int c = (int)(u - 3 * i);
            const int dpos = c == 0 ? 0 : (c == 1 ? 3 : 5);
            const double D = damping == 0 ? clamp_d((double)hpp[6 * i + dpos]) : 1.0;
            b += dp[u] * (lambda * D * dp[u] + wpt[u]);
        }
    }
    block_partials<2>(a, b, partials);
}

template <typename T>
hipError_t launch_pred(int32_t m, int32_t n, const double* dc, const double* dcam, const double* vcam,
                       const double* dp, const double* hpp, const double* wpt, double lambda, int32_t damping,
                       double* partials, int32_t* nblocks, hipStream_t s)
{
    const int64_t lc = 9 * (int64_t)m, lp = 3 * (int64_t)n;
    const int32_t b = reduce_blocks(lc + lp);
    *nblocks = b;
    hipLaunchKernelGGL((k_pred<T>), dim3(b), dim3(kRedBlock), 0, s, lc, lp, dc, dcam, vcam, dp, hpp, wpt, lambda,
                       damping, partials);
    return hipGetLastError();
}

// ------------------------------------------- caller order <-> internal
__global__ void k_gather_cameras(int32_t m, int dtype, const void* __restrict__ src,
                                 const int32_t* __restrict__ old_of_new, double* __restrict__ dst)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 9 * (int64_t)m) return;
    const int64_t j = t / 9;
    const int a = (int)(t - 9 * j);
    const int64_t o = 9 * (int64_t)old_of_new[j] + a;
    dst[t] = dtype == 0 ? ((const double*)src)[o] : (double)((const float*)src)[o];
}

hipError_t launch_gather_cameras(int32_t m, int dtype, const void* src, const int32_t* old_of_new, double* dst,
                                 hipStream_t s)
{
    const int64_t len = 9 * (int64_t)m;
    if (len > 0)
        hipLaunchKernelGGL(k_gather_cameras, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, m, dtype, src,
                           old_of_new, dst);
    return hipGetLastError();
}

__global__ void k_convert_points(int64_t len, int dtype, const void* __restrict__ src, double* __restrict__ dst)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = dtype == 0 ? ((const double*)src)[t] : (double)((const float*)src)[t];
}

hipError_t launch_convert_points(int32_t n, int dtype, const void* src, double* dst, hipStream_t s)
{
    const int64_t len = 3 * (int64_t)n;
    int64_t b = (len + 255) / 256;
    if (b > 8192) b = 8192;
    if (len > 0) hipLaunchKernelGGL(k_convert_points, dim3((unsigned)b), dim3(256), 0, s, len, dtype, src, dst);
    return hipGetLastError();
}

// grad = -scale * [v; w] scattered to caller order (v, w hold -J^T W e)
__global__ void k_scatter_grad(int64_t lc, int64_t lp, int dtype, double gout, const double* __restrict__ dscale,
                               const double* __restrict__ vcam, const double* __restrict__ wpt,
                               const int32_t* __restrict__ old_of_new, void* __restrict__ gcam,
                               void* __restrict__ gpt)
{
    const double scale = dscale ? gout * dscale[0] : gout;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < lc + lp; t += (int64_t)gridDim.x * blockDim.x) {
        if (t < lc) {
            if (!gcam) continue;
            const int64_t j = t / 9;
            const int a = (int)(t - 9 * j);
            const int64_t o = 9 * (int64_t)old_of_new[j] + a;
            const double v = -scale * vcam[t];
            if (dtype == 0) ((double*)gcam)[o] = v;
            else ((float*)gcam)[o] = (float)v;
        } else {
            if (!gpt) continue;
            const int64_t u = t - lc;
            const double v = -scale * wpt[u];
            if (dtype == 0) ((double*)gpt)[u] = v;
            else ((float*)gpt)[u] = (float)v;
        }
    }
}

hipError_t launch_scatter_grad(int32_t m, int32_t n, int dtype, double scale, const double* dscale,
                               const double* vcam, const double* wpt, const int32_t* old_of_new, void* gcam, void* gpt,
                               hipStream_t s)
{
    const int64_t lc = 9 * (int64_t)m, lp = 3 * (int64_t)n;
    int64_t b = (lc + lp + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_scatter_grad, dim3((unsigned)b), dim3(256), 0, s, lc, lp, dtype, scale, dscale, vcam, wpt,
                       old_of_new, gcam, gpt);
    return hipGetLastError();
}

__global__ void k_store_cost(const double* __restrict__ sum, double* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = sum[0];
}

hipError_t launch_store_cost(const double* sum, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_store_cost, dim3(1), dim3(64), 0, s, sum, out);
    return hipGetLastError();
}

template hipError_t launch_pcg_direction<double>(int32_t, bool, const double*, double*, double*,
                                                 const CamK<double>*, double*, PcgScalars*, hipStream_t);
template hipError_t launch_pcg_direction<float>(int32_t, bool, const double*, double*, float*, const CamK<float>*,
                                                float*, PcgScalars*, hipStream_t);
template hipError_t launch_pred<double>(int32_t, int32_t, const double*, const double*, const double*, const double*,
                                        const double*, const double*, double, int32_t, double*, int32_t*, hipStream_t);
template hipError_t launch_pred<float>(int32_t, int32_t, const double*, const double*, const double*, const double*,
                                       const double*, const double*, double, int32_t, double*, int32_t*, hipStream_t);

}  // namespace ba

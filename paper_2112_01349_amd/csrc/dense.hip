// The direct option: the reduced camera system of Eq. schur_x_c written out
// as a dense FP64 matrix S [nd][nd] (nd = 9m, row-major) and solved through
// its Cholesky factor, in place of PCG, for problems with few cameras (the
// direct route the paper sets against iterative solvers in Sec. 3).
//
//   * k_dense_init: S = blockdiag(B~_j).
//   * k_dense_schur: for every point, S[cam(a), cam(b)] -= E_a C~^-1 E_b^T over
//     all pairs of its observations; E is formed from the Jacobian as in the
//     recomputing products, one observation per lane, the partner blocks
//     fetched by shuffles, the 81 terms of a block added with FP64 atomics.
//   * Cholesky, right-looking over 64 x 64 tiles: k_potrf_tile factors the
//     diagonal tile in LDS, k_trsm_tiles forms the panel below it, and
//     k_syrk_tiles updates the trailing lower tiles.
//   * k_dense_trsv: L y = g, then L^T x = y, by one workgroup, a tile at a
//     time.
#include "ba_internal.h"

namespace ba {

namespace {
constexpr int kT = 64;  // tile edge
}

__global__ void k_dense_init(int32_t m, const double* __restrict__ bd, double* __restrict__ S)
{
    const int64_t nd = 9 * (int64_t)m;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nd * nd;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / nd, c = e - r * nd;
        const int64_t jr = r / 9, jc = c / 9;
        S[e] = jr == jc ? bd[81 * jr + (r - 9 * jr) * 9 + (c - 9 * jc)] : 0.0;
    }
}

// E_k (9x3 row-major, FP64) of one observation from the geometry: E = w J_c^T J_p.
template <typename T>
__device__ __forceinline__ void coupling_block(const CamK<T>& k, const ObsGeo<T>& o, T w, double E[27])
{
    T e0, e1, Jc[18], Jp[6];
    jacobian_from_geometry<T>(k, o, (T)0, (T)0, e0, e1, Jc, Jp);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            E[a * 3 + c] = (double)w * ((double)Jc[a] * (double)Jp[c] + (double)Jc[9 + a] * (double)Jp[3 + c]);
}

// One wavefront per row of 64 observations of a segment (a short segment is a
// row; a long one, a point, is cut into rows).  Lane a pairs with every lane
// of the partner row holding the same point.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_schur(int32_t num_rows, const int4* __restrict__ rows,
                                                     const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
                                                     const T* __restrict__ wobs, const double* __restrict__ pts,
                                                     const CamK<T>* __restrict__ ck,
                                                     const CamK<double>* __restrict__ ck64,
                                                     const T* __restrict__ cinv, int32_t m, double* __restrict__ S)
{
    const int lane = threadIdx.x & 63;
    const int32_t rw = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    if (rw >= num_rows) return;  // whole wavefront leaves together
    const int64_t nd = 9 * (int64_t)m;
    // rows[rw] = {start of this row, its length, start of the partner row, its length}
    const int4 rr = rows[rw];
    const int32_t a0 = __builtin_amdgcn_readfirstlane(rr.x), alen = __builtin_amdgcn_readfirstlane(rr.y);
    const int32_t b0 = __builtin_amdgcn_readfirstlane(rr.z), blen = __builtin_amdgcn_readfirstlane(rr.w);
    const bool va = lane < alen, vb = lane < blen;
    double Ta[27], Eb[27];
    int32_t ia = -1, ja = 0, ib = -2, jb = 0;
    {
        const int64_t k = a0 + (va ? lane : 0);
        ja = cam[k];
        ia = va ? pt[k] : -1;
        const CamK<T>& kk = ck[ja];
        ObsGeo<T> o;
        observation_geometry_checked<T>(kk.R, ck64, ja, pts + 3 * (int64_t)pt[k], o);
        double E[27];
        coupling_block<T>(kk, o, wobs[k], E);
        const T* c6 = cinv + 6 * (int64_t)pt[k];
        const double C[9] = {(double)c6[0], (double)c6[1], (double)c6[2], (double)c6[1], (double)c6[3],
                             (double)c6[4], (double)c6[2], (double)c6[4], (double)c6[5]};
#pragma unroll
        for (int a = 0; a < 9; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Ta[a * 3 + c] = E[a * 3] * C[c] + E[a * 3 + 1] * C[3 + c] + E[a * 3 + 2] * C[6 + c];
    }
    {
        const int64_t k = b0 + (vb ? lane : 0);
        jb = cam[k];
        ib = vb ? pt[k] : -2;
        const CamK<T>& kk = ck[jb];
        ObsGeo<T> o;
        observation_geometry_checked<T>(kk.R, ck64, jb, pts + 3 * (int64_t)pt[k], o);
        coupling_block<T>(kk, o, wobs[k], Eb);
    }
    for (int32_t t = 0; t < blen; ++t) {  // uniform: every lane takes part in the shuffles
        const int32_t it = __shfl(ib, t, 64), jt = __shfl(jb, t, 64);
        double E[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) E[q] = __shfl(Eb[q], t, 64);
        if (va && ia == it) {
            double* blk = S + (9 * (int64_t)ja) * nd + 9 * (int64_t)jt;
#pragma unroll
            for (int a = 0; a < 9; ++a)
#pragma unroll
                for (int b = 0; b < 9; ++b) {
                    const double v = Ta[a * 3] * E[b * 3] + Ta[a * 3 + 1] * E[b * 3 + 1] + Ta[a * 3 + 2] * E[b * 3 + 2];
                    unsafeAtomicAdd(blk + a * nd + b, -v);
                }
        }
    }
}

// Factor the diagonal tile (kb, kb) in place: L L^T = A; flag on failure.
__global__ __launch_bounds__(256) void k_potrf_tile(int64_t nd, int32_t kb, double* __restrict__ S,
                                                    int32_t* __restrict__ flag)
{
    __shared__ double L[kT][kT + 1];
    const int64_t o = (int64_t)kb * kT;
    const int w = (int)(nd - o < kT ? nd - o : kT);
    for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
        const int r = e / kT, c = e % kT;
        L[r][c] = (r < w && c < w) ? S[(o + r) * nd + o + c] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int c = 0; c < w; ++c) {
        if (threadIdx.x == 0) {
            const double d = L[c][c];
            if (!(d > 0.0) || !isfinite(d)) bad = 1;
            L[c][c] = sqrt(d > 0.0 ? d : 1.0);
        }
        __syncthreads();
        const double d = L[c][c];
        for (int r = c + 1 + threadIdx.x; r < w; r += blockDim.x) L[r][c] /= d;
        __syncthreads();
        // trailing update of columns c+1.. within the tile
        for (int e = threadIdx.x; e < (w - c - 1) * (w - c - 1); e += blockDim.x) {
            const int r = c + 1 + e / (w - c - 1), q = c + 1 + e % (w - c - 1);
            if (q <= r) L[r][q] -= L[r][c] * L[q][c];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
        const int r = e / w, c = e % w;
        S[(o + r) * nd + o + c] = c <= r ? L[r][c] : 0.0;
    }
    if (threadIdx.x == 0 && bad) atomicOr(flag, 4);
}

// Panel below the diagonal tile: A[ib][kb] = A[ib][kb] L11^-T, one workgroup
// per tile row ib > kb.
__global__ __launch_bounds__(256) void k_trsm_tiles(int64_t nd, int32_t kb, double* __restrict__ S)
{
    __shared__ double L[kT][kT + 1];
    __shared__ double X[kT][kT + 1];
    const int64_t o = (int64_t)kb * kT;
    const int w = (int)(nd - o < kT ? nd - o : kT);
    const int64_t ro = o + kT * (int64_t)(1 + blockIdx.x);
    const int h = (int)(nd - ro < kT ? nd - ro : kT);
    for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
        const int r = e / kT, c = e % kT;
        L[r][c] = (r < w && c < w) ? S[(o + r) * nd + o + c] : 0.0;
        X[r][c] = (r < h && c < w) ? S[(ro + r) * nd + o + c] : 0.0;
    }
    __syncthreads();
    // X L^T = A: column c of X from columns < c; each thread owns rows
    for (int c = 0; c < w; ++c) {
        for (int r = threadIdx.x; r < h; r += blockDim.x) {
            double v = X[r][c];
            for (int t = 0; t < c; ++t) v -= X[r][t] * L[c][t];
            X[r][c] = v / L[c][c];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < h * w; e += blockDim.x) {
        const int r = e / w, c = e % w;
        S[(ro + r) * nd + o + c] = X[r][c];
    }
}

// Trailing update A[ib][jb] -= A[ib][kb] A[jb][kb]^T for kb < jb <= ib: one
// workgroup per lower tile, 16 outputs per thread.
__global__ __launch_bounds__(256) void k_syrk_tiles(int64_t nd, int32_t kb, double* __restrict__ S)
{
    __shared__ double P[kT][kT + 1];
    __shared__ double Q[kT][kT + 1];
    // blockIdx.x enumerates the lower tiles (ib, jb) of the trailing matrix
    const int32_t rem = (int32_t)((nd + kT - 1) / kT) - kb - 1;
    int32_t idx = blockIdx.x, ib = 0;
    while (idx >= ib + 1) {  // row ib holds ib + 1 tiles
        idx -= ib + 1;
        ++ib;
    }
    const int32_t jb = idx;
    if (ib >= rem) return;
    const int64_t o = (int64_t)kb * kT;
    const int64_t ro = o + kT * (int64_t)(1 + ib), co = o + kT * (int64_t)(1 + jb);
    const int h = (int)(nd - ro < kT ? nd - ro : kT), wc = (int)(nd - co < kT ? nd - co : kT);
    const int w = (int)(nd - o < kT ? nd - o : kT);
    for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
        const int r = e / kT, c = e % kT;
        P[r][c] = (r < h && c < w) ? S[(ro + r) * nd + o + c] : 0.0;
        Q[r][c] = (r < wc && c < w) ? S[(co + r) * nd + o + c] : 0.0;
    }
    __syncthreads();
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;  // 16 x 16 threads, 4 x 4 outputs each
    double acc[4][4] = {};
    for (int t = 0; t < w; ++t) {
        double p[4], q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            p[u] = P[tr * 4 + u][t];
            q[u] = Q[tc * 4 + u][t];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += p[u] * q[v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = tr * 4 + u, c = tc * 4 + v;
            if (r < h && c < wc && (ib != jb || c <= r)) S[(ro + r) * nd + co + c] -= acc[u][v];
        }
}

// x = S^-1 g with S = L L^T factored in place (lower triangle): forward then
// backward substitution by one workgroup, a tile at a time (the tile's own
// triangle by one wavefront, the coupling to the remaining rows by all).
__global__ __launch_bounds__(1024) void k_dense_trsv(int64_t nd, const double* __restrict__ L,
                                                     const double* __restrict__ g, double* __restrict__ x,
                                                     double* __restrict__ y)
{
    for (int64_t r = threadIdx.x; r < nd; r += blockDim.x) y[r] = g[r];
    __syncthreads();
    const int32_t nb = (int32_t)((nd + kT - 1) / kT);
    // forward: L y = g
    for (int32_t kb = 0; kb < nb; ++kb) {
        const int64_t o = (int64_t)kb * kT;
        const int w = (int)(nd - o < kT ? nd - o : kT);
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            double v = lane < w ? y[o + lane] : 0.0;
            for (int c = 0; c < w; ++c) {
                const double yc = __shfl(v, c, 64) / L[(o + c) * nd + o + c];
                if (lane == c) v = yc;
                if (lane > c && lane < w) v -= L[(o + lane) * nd + o + c] * yc;
            }
            if (lane < w) y[o + lane] = v;
        }
        __syncthreads();
        for (int64_t r = o + w + threadIdx.x; r < nd; r += blockDim.x) {
            double s = 0.0;
            for (int c = 0; c < w; ++c) s += L[r * nd + o + c] * y[o + c];
            y[r] -= s;
        }
        __syncthreads();
    }
    // backward: L^T x = y
    for (int64_t r = threadIdx.x; r < nd; r += blockDim.x) x[r] = y[r];
    __syncthreads();
    for (int32_t kb = nb - 1; kb >= 0; --kb) {
        const int64_t o = (int64_t)kb * kT;
        const int w = (int)(nd - o < kT ? nd - o : kT);
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            double v = lane < w ? x[o + lane] : 0.0;
            for (int c = w - 1; c >= 0; --c) {
                const double xc = __shfl(v, c, 64) / L[(o + c) * nd + o + c];
                if (lane == c) v = xc;
                if (lane < c) v -= L[(o + c) * nd + o + lane] * xc;
            }
            if (lane < w) x[o + lane] = v;
        }
        __syncthreads();
        for (int64_t r = threadIdx.x; r < o; r += blockDim.x) {
            double s = 0.0;
            for (int c = 0; c < w; ++c) s += L[(o + c) * nd + r] * x[o + c];
            x[r] -= s;
        }
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_dense_solve(const DensePlan& dp, const PointMajor& pm, const RecomputeInputs<T>& ri,
                              const T* cinv, int32_t m, const double* bd, const double* g, double* x, double* S,
                              double* ybuf, int32_t* flag, hipStream_t s)
{
    const int64_t nd = 9 * (int64_t)m;
    hipLaunchKernelGGL(k_dense_init, dim3(1024), dim3(256), 0, s, m, bd, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dp.num_rows > 0) {
        hipLaunchKernelGGL((k_dense_schur<T>), dim3((dp.num_rows + 3) / 4), dim3(256), 0, s, dp.num_rows, dp.rows,
                           pm.cam, pm.pt, ri.wobs, ri.pts, ri.ck, ri.ck64, cinv, m, S);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int32_t nb = (int32_t)((nd + kT - 1) / kT);
    for (int32_t kb = 0; kb < nb; ++kb) {
        hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(256), 0, s, nd, kb, S, flag);
        const int32_t rem = nb - kb - 1;
        if (rem > 0) {
            hipLaunchKernelGGL(k_trsm_tiles, dim3(rem), dim3(256), 0, s, nd, kb, S);
            hipLaunchKernelGGL(k_syrk_tiles, dim3(rem * (rem + 1) / 2), dim3(256), 0, s, nd, kb, S);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_dense_trsv, dim3(1), dim3(1024), 0, s, nd, S, g, x, ybuf);
    return hipGetLastError();
}

template hipError_t launch_dense_solve<float>(const DensePlan&, const PointMajor&, const RecomputeInputs<float>&,
                                              const float*, int32_t, const double*, const double*, double*, double*,
                                              double*, int32_t*, hipStream_t);
template hipError_t launch_dense_solve<double>(const DensePlan&, const PointMajor&, const RecomputeInputs<double>&,
                                               const double*, int32_t, const double*, const double*, double*,
                                               double*, double*, int32_t*, hipStream_t);

}  // namespace ba

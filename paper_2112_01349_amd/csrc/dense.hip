// The direct option: the reduced camera system of Eq. schur_x_c written out
// as a dense FP64 matrix S [nd][nd] (nd = 9m, row-major) and solved through
// its Cholesky factor, in place of PCG, for problems with few cameras (the
// direct route the paper sets against iterative solvers in Sec. 3).
//
//   * k_dense_coupling: E_k = w J_c^T J_p of every observation (FP64, from
//     the T-precision Jacobian), point-major, into a scratch stream.
//   * k_dense_rows: one workgroup per piece of a block row (camera a, at most
//     kPiece of its observations) and chunk of kChunk block columns.  It
//     walks the piece's observations; for each, the other observations of
//     the same point whose camera falls in the chunk add -E_a C~^-1 E_b^T to
//     an LDS copy of the chunk (LDS atomics).  The blocks touched are then
//     stored, or added with global atomics when the camera has several
//     pieces (the few most-seen cameras), which splits the hottest rows over
//     many workgroups.  The diagonal block starts from B~_a plus
//     the per-observation terms -sum E_k C~^-1 E_k^T (the Schur-Jacobi
//     camera-major pass), so an observation never pairs with itself here.
//   * Cholesky, blocked right-looking over 64 x 64 tiles: k_potrf_tile factors
//     the diagonal tile (one wavefront, a row per lane), k_trsm_tiles forms
//     the panel below it (a row per lane), and k_syrk_tiles updates lower
//     tiles on the FP64 matrix cores: within a super-panel of 8 tile columns
//     by each column as it is done, beyond it once per super-panel with rank
//     512, so the trailing matrix is read and written an eighth as often.
//   * k_trsv_diag / k_trsv_panel: L y = g and L^T x = y a tile at a time, the
//     tile's triangle by one wavefront and the coupling to the remaining rows
//     by many workgroups.
#include "ba_internal.h"

namespace ba {

namespace {
constexpr int kT = 64;       // factorisation tile edge
constexpr int kSuper = 8;    // tile columns per super-panel (rank of the trailing update: 64 kSuper)
constexpr int kChunk = 64;  // block columns per workgroup in k_dense_rows (41.5 KB of LDS)
}  // namespace

// E_k of every observation, [N][27] row-major 9x3.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_coupling(int64_t N, const int32_t* __restrict__ cam,
                                                        const int32_t* __restrict__ pt, const T* __restrict__ wobs,
                                                        const double* __restrict__ pts,
                                                        const CamK<T>* __restrict__ ck,
                                                        const CamK<double>* __restrict__ ck64,
                                                        double* __restrict__ E)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int32_t j = cam[k];
    const CamK<T>& kk = ck[j];
    ObsGeo<T> o;
    observation_geometry_checked<T>(kk.R, ck64, j, pts + 3 * (int64_t)pt[k], o);
    T e0, e1, Jc[18], Jp[6];
    jacobian_from_geometry<T>(kk, o, (T)0, (T)0, e0, e1, Jc, Jp);
    const double w = (double)wobs[k];
    double* out = E + 27 * k;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            out[a * 3 + c] = w * ((double)Jc[a] * (double)Jp[c] + (double)Jc[9 + a] * (double)Jp[3 + c]);
}

__global__ void k_dense_zero(int64_t len, double* __restrict__ S)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x)
        S[e] = 0.0;
}

// One workgroup per (piece, chunk): piece = {camera a, first and end
// camera-major observation, number of pieces of camera a}.  S is zero
// beforehand; blocks that received a term are stored (a camera walked by one
// piece) or added atomically (several pieces).
template <typename T>
__global__ __launch_bounds__(256) void k_dense_rows(int32_t m, int32_t nchunk, const int4* __restrict__ pieces,
                                                    const int32_t* __restrict__ cm_pm,
                                                    const int32_t* __restrict__ poff,
                                                    const int32_t* __restrict__ pm_cam,
                                                    const int32_t* __restrict__ pm_pt, const double* __restrict__ E,
                                                    const T* __restrict__ cinv, const double* __restrict__ bd,
                                                    const double* __restrict__ mj, double* __restrict__ S)
{
    __shared__ double acc[kChunk * 81];
    __shared__ int touched[kChunk];
    const int32_t pc = blockIdx.x / nchunk;
    const int4 pe = pieces[pc];
    const int32_t ja = pe.x;
    const bool first = pc == 0 || pieces[pc - 1].x != ja;  // the piece that adds the diagonal terms
    const int32_t c0 = (blockIdx.x - pc * nchunk) * kChunk;
    const int32_t cw = min(kChunk, m - c0);
    const int64_t nd = 9 * (int64_t)m;
    for (int e = threadIdx.x; e < cw * 81; e += blockDim.x) {
        const int32_t jb = c0 + e / 81;
        const int q = e % 81;
        acc[e] = (first && jb == ja) ? bd[81 * (int64_t)ja + q] + mj[81 * (int64_t)ja + q] : 0.0;
    }
    for (int c = threadIdx.x; c < kChunk; c += blockDim.x) touched[c] = (first && c0 + c == ja) ? 1 : 0;
    __syncthreads();
    for (int32_t a = pe.y + threadIdx.x; a < pe.z; a += blockDim.x) {
        const int32_t ka = cm_pm[a];
        const int32_t i = pm_pt[ka];
        const int32_t p0 = poff[i], p1 = poff[i + 1];
        bool have = false;
        double Ta[27];
        for (int32_t kb = p0; kb < p1; ++kb) {
            const int32_t jb = pm_cam[kb];
            if (kb == ka || jb < c0 || jb >= c0 + cw) continue;
            if (!have) {  // T_a = E_a C~_i^-1, formed at the first partner in the chunk
                const T* c6 = cinv + 6 * (int64_t)i;
                const double C[9] = {(double)c6[0], (double)c6[1], (double)c6[2], (double)c6[1], (double)c6[3],
                                     (double)c6[4], (double)c6[2], (double)c6[4], (double)c6[5]};
                const double* Ea = E + 27 * (int64_t)ka;
#pragma unroll
                for (int r = 0; r < 9; ++r) {
                    const double x0 = Ea[r * 3], x1 = Ea[r * 3 + 1], x2 = Ea[r * 3 + 2];
#pragma unroll
                    for (int c = 0; c < 3; ++c) Ta[r * 3 + c] = x0 * C[c] + x1 * C[3 + c] + x2 * C[6 + c];
                }
                have = true;
            }
            const double* Eb = E + 27 * (int64_t)kb;
            double eb[27];
#pragma unroll
            for (int q = 0; q < 27; ++q) eb[q] = Eb[q];
            touched[jb - c0] = 1;
            double* blk = acc + (jb - c0) * 81;
#pragma unroll
            for (int r = 0; r < 9; ++r)
#pragma unroll
                for (int c = 0; c < 9; ++c)
                    unsafeAtomicAdd(blk + r * 9 + c,
                                    -(Ta[r * 3] * eb[c * 3] + Ta[r * 3 + 1] * eb[c * 3 + 1] +
                                      Ta[r * 3 + 2] * eb[c * 3 + 2]));
        }
    }
    __syncthreads();
    // rows 9 ja .. 9 ja + 8, columns 9 c0 .. 9 (c0 + cw) - 1: contiguous per row
    const bool shared_row = pe.w > 1;
    const int rowlen = 9 * cw;
    for (int e = threadIdx.x; e < 9 * rowlen; e += blockDim.x) {
        const int r = e / rowlen, rem = e - r * rowlen;
        const int c = rem / 9, col = rem - c * 9;
        if (!touched[c]) continue;
        double* dst = S + (9 * (int64_t)ja + r) * nd + 9 * (int64_t)c0 + rem;
        const double v = acc[c * 81 + r * 9 + col];
        if (shared_row) unsafeAtomicAdd(dst, v);
        else *dst = v;
    }
}

// Factor the diagonal tile (kb, kb) in place, L L^T = A, by one wavefront
// (lane r owns row r in LDS); flag bit 2 on failure.
__global__ __launch_bounds__(64) void k_potrf_tile(int64_t nd, int32_t kb, double* __restrict__ S,
                                                   int32_t* __restrict__ flag)
{
    __shared__ double L[kT][kT + 1];
    __shared__ double col[kT];  // column c of the factor, apart from L so loads and stores do not alias
    const int r = threadIdx.x;
    const int64_t o = (int64_t)kb * kT;
    const int w = (int)(nd - o < kT ? nd - o : kT);
    // row by row, lane = column; every load reads a valid (clamped) address
    // and is selected afterwards, so the loads are issued back to back
    const int rc = r < w ? r : w - 1;
#pragma unroll 16
    for (int q = 0; q < w; ++q) {
        const double v = S[(o + q) * nd + o + rc];
        L[q][r] = r < w ? v : 0.0;  // q < w <= r: off the diagonal
    }
    for (int q = w; q < kT; ++q) L[q][r] = q == r ? 1.0 : 0.0;
    __syncthreads();
    bool bad = false;
    for (int c = 0; c < w; ++c) {
        const double dd = L[c][c];  // final: every update of column c has been applied
        if (!(dd > 0.0) || !isfinite(dd)) bad = true;
        const double d = sqrt(dd > 0.0 ? dd : 1.0);
        __syncthreads();
        double lrc = 0.0;
        if (r == c) L[c][c] = d;
        if (r > c) {
            lrc = L[r][c] / d;
            L[r][c] = lrc;
        }
        col[r] = lrc;
        __syncthreads();
        if (r > c) {
#pragma unroll 8
            for (int q = c + 1; q <= r; ++q) L[r][q] -= lrc * col[q];
        }
        __syncthreads();
    }
    for (int q = 0; q < w; ++q)
        if (r < w) S[(o + q) * nd + o + r] = r <= q ? L[q][r] : 0.0;
    if (r == 0 && bad) atomicOr(flag, 4);
}

// Panel below the diagonal tile: A[ib][kb] = A[ib][kb] L11^-T, one wavefront
// per tile row ib > kb, each lane solving its own row.
__global__ __launch_bounds__(64) void k_trsm_tiles(int64_t nd, int32_t kb, double* __restrict__ S)
{
    __shared__ double L[kT][kT + 1];
    __shared__ double X[kT][kT + 1];
    const int r = threadIdx.x;
    const int64_t o = (int64_t)kb * kT;
    const int w = (int)(nd - o < kT ? nd - o : kT);
    const int64_t ro = o + kT * (int64_t)(1 + blockIdx.x);
    const int h = (int)(nd - ro < kT ? nd - ro : kT);
    const int rc = r < w ? r : w - 1;  // row by row, lane = column, clamped loads as in k_potrf_tile
#pragma unroll 16
    for (int q = 0; q < w; ++q) {
        const double v = S[(o + q) * nd + o + rc];
        L[q][r] = r < w ? v : 0.0;
    }
#pragma unroll 16
    for (int q = 0; q < h; ++q) {
        const double v = S[(ro + q) * nd + o + rc];
        X[q][r] = r < w ? v : 0.0;
    }
    for (int q = w; q < kT; ++q) L[q][r] = 0.0;
    for (int q = h; q < kT; ++q) X[q][r] = 0.0;
    __syncthreads();
    if (r < h) {
        for (int c = 0; c < w; ++c) {
            double v0 = X[r][c], v1 = 0.0, v2 = 0.0, v3 = 0.0;  // four chains for latency
            int t = 0;
            for (; t + 4 <= c; t += 4) {
                v0 -= X[r][t] * L[c][t];
                v1 -= X[r][t + 1] * L[c][t + 1];
                v2 -= X[r][t + 2] * L[c][t + 2];
                v3 -= X[r][t + 3] * L[c][t + 3];
            }
            for (; t < c; ++t) v0 -= X[r][t] * L[c][t];
            X[r][c] = ((v0 + v1) + (v2 + v3)) / L[c][c];
        }
    }
    __syncthreads();
    for (int q = 0; q < h; ++q)
        if (r < w) S[(ro + q) * nd + o + r] = X[q][r];
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Trailing update of the lower tiles (ib, jb) with j0 <= jb < j1 and
// ib >= jb by the tile columns k0 .. k0 + kw - 1 of the factor:
// A[ib][jb] -= sum_kc A[ib][kc] A[jb][kc]^T (rank 64 kw).  One workgroup per
// tile, on the FP64 matrix cores: each wavefront forms a 32 x 32 quarter as
// 2 x 2 products of 16 x 16 x 4 (v_mfma_f64_16x16x4f64: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16] of a step, and D[4 q + l / 16][l % 16]
// in item q), accumulating over all kw panel tiles before the one
// read-modify-write of the output tile.
__global__ __launch_bounds__(256) void k_syrk_tiles(int64_t nd, int32_t k0, int32_t kw, int32_t j0,
                                                    double* __restrict__ S)
{
    __shared__ double P[kT][kT + 1];
    __shared__ double Q[kT][kT + 1];
    const int32_t nb = (int32_t)((nd + kT - 1) / kT);
    // blockIdx.x enumerates the tiles column by column: column jb holds nb - jb tiles
    int32_t idx = blockIdx.x, jb = j0;
    while (idx >= nb - jb) {
        idx -= nb - jb;
        ++jb;
    }
    const int32_t ib = jb + idx;
    const int64_t ro = kT * (int64_t)ib, co = kT * (int64_t)jb;
    const int h = (int)(nd - ro < kT ? nd - ro : kT), wc = (int)(nd - co < kT ? nd - co : kT);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = (wave >> 1) * 32, c0 = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    dbl4 acc00 = {0.0, 0.0, 0.0, 0.0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
    for (int32_t kc = k0; kc < k0 + kw; ++kc) {  // panel tiles are full: kc < jb <= nb - 1
        const int64_t o = kT * (int64_t)kc;
        __syncthreads();  // the previous panel tile has been consumed
        for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
            const int r = e / kT, c = e % kT;
            P[r][c] = r < h ? S[(ro + r) * nd + o + c] : 0.0;
            Q[r][c] = r < wc ? S[(co + r) * nd + o + c] : 0.0;
        }
        __syncthreads();
        for (int t = 0; t < kT; t += 4) {
            const double a0 = P[r0 + li][t + lk], a1 = P[r0 + 16 + li][t + lk];
            const double b0 = Q[c0 + li][t + lk], b1 = Q[c0 + 16 + li][t + lk];
            acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
            acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
            acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc10, 0, 0, 0);
            acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
        }
    }
    const dbl4 acc[2][2] = {{acc00, acc01}, {acc10, acc11}};
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + 16 * u + 4 * q + lk, c = c0 + 16 * v + li;
                if (r < h && c < wc && (ib != jb || c <= r)) S[(ro + r) * nd + co + c] -= acc[u][v][q];
            }
}

// Blocks of the lower triangle in tile columns j0 .. j1 - 1 (nb tile rows).
static unsigned column_tiles(int32_t nb, int32_t j0, int32_t j1)
{
    int64_t t = 0;
    for (int32_t j = j0; j < j1; ++j) t += nb - j;
    return (unsigned)t;
}

// The triangle of tile kb: forward (L11 y1 = y1) or backward (L11^T x1 = x1)
// in place on v[o .. o + w), one wavefront.
template <bool FORWARD>
__global__ __launch_bounds__(64) void k_trsv_diag(int64_t nd, int32_t kb, const double* __restrict__ L,
                                                  double* __restrict__ v)
{
    __shared__ double A[kT][kT + 1];
    const int lane = threadIdx.x;
    const int64_t o = (int64_t)kb * kT;
    const int w = (int)(nd - o < kT ? nd - o : kT);
    const int lc = lane < w ? lane : w - 1;
#pragma unroll 16
    for (int r = 0; r < w; ++r) {  // row r of the tile, lane = column, clamped loads
        const double v = L[(o + r) * nd + o + lc];
        A[r][lane] = lane < w ? v : 0.0;
    }
    for (int r = w; r < kT; ++r) A[r][lane] = 0.0;
    __syncthreads();
    double x = lane < w ? v[o + lane] : 0.0;
    if (FORWARD) {
        for (int c = 0; c < w; ++c) {
            const double yc = __shfl(x, c, 64) / A[c][c];
            if (lane == c) x = yc;
            if (lane > c && lane < w) x -= A[lane][c] * yc;
        }
    } else {
        for (int c = w - 1; c >= 0; --c) {
            const double xc = __shfl(x, c, 64) / A[c][c];
            if (lane == c) x = xc;
            if (lane < c) x -= A[c][lane] * xc;
        }
    }
    if (lane < w) v[o + lane] = x;
}

// The coupling of tile kb to the remaining rows: forward, v[r] -= L[r][o..]
// v[o..] for the rows below the tile; backward, v[r] -= L[o..][r] v[o..] for
// the rows above it.  A thread per row.
template <bool FORWARD>
__global__ __launch_bounds__(256) void k_trsv_panel(int64_t nd, int32_t kb, const double* __restrict__ L,
                                                    double* __restrict__ v)
{
    __shared__ double t[kT];
    const int64_t o = (int64_t)kb * kT;
    const int w = (int)(nd - o < kT ? nd - o : kT);
    if (threadIdx.x < kT) t[threadIdx.x] = threadIdx.x < w ? v[o + threadIdx.x] : 0.0;
    __syncthreads();
    const int64_t r = (FORWARD ? o + w : 0) + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= (FORWARD ? nd : o)) return;
    double s = 0.0;
    if (FORWARD) {
        const double* row = L + r * nd + o;
        for (int c = 0; c < w; ++c) s += row[c] * t[c];
    } else {
        for (int c = 0; c < w; ++c) s += L[(o + c) * nd + r] * t[c];
    }
    v[r] -= s;
}

template <typename T>
hipError_t launch_dense_solve(const DensePlan& dp, const PointMajor& pm, int64_t N, const RecomputeInputs<T>& ri,
                              const T* cinv, int32_t m, const double* bd, const double* mj, const double* g,
                              double* x, double* S, int32_t* flag, hipStream_t s)
{
    const int64_t nd = 9 * (int64_t)m;
    hipError_t e;
    if (N > 0) {
        hipLaunchKernelGGL((k_dense_coupling<T>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, pm.cam,
                           pm.pt, ri.wobs, ri.pts, ri.ck, ri.ck64, dp.E);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int32_t nchunk = (m + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_dense_zero, dim3(2048), dim3(256), 0, s, nd * nd, S);
    hipLaunchKernelGGL((k_dense_rows<T>), dim3((unsigned)(dp.num_pieces * nchunk)), dim3(256), 0, s, m, nchunk,
                       dp.pieces, dp.cm_pm, dp.poff, pm.cam, pm.pt, dp.E, cinv, bd, mj, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // Blocked right-looking Cholesky: super-panels of kSuper tile columns are
    // factored column by column (each column updating only the rest of its
    // super-panel), then the trailing matrix takes one rank-64 kSuper update.
    const int32_t nb = (int32_t)((nd + kT - 1) / kT);
    for (int32_t sb = 0; sb < nb; sb += kSuper) {
        const int32_t se = min(sb + kSuper, nb);
        for (int32_t kb = sb; kb < se; ++kb) {
            hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(64), 0, s, nd, kb, S, flag);
            const int32_t rem = nb - kb - 1;
            if (rem > 0) hipLaunchKernelGGL(k_trsm_tiles, dim3(rem), dim3(64), 0, s, nd, kb, S);
            if (kb + 1 < se)
                hipLaunchKernelGGL(k_syrk_tiles, dim3(column_tiles(nb, kb + 1, se)), dim3(256), 0, s, nd, kb, 1,
                                   kb + 1, S);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (se < nb) {
            hipLaunchKernelGGL(k_syrk_tiles, dim3(column_tiles(nb, se, nb)), dim3(256), 0, s, nd, sb, se - sb, se,
                               S);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    // x = S^-1 g: forward into x, then backward in place
    if ((e = hipMemcpyAsync(x, g, sizeof(double) * nd, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    for (int32_t kb = 0; kb < nb; ++kb) {
        hipLaunchKernelGGL((k_trsv_diag<true>), dim3(1), dim3(64), 0, s, nd, kb, S, x);
        const int64_t below = nd - (int64_t)(kb + 1) * kT;
        if (below > 0)
            hipLaunchKernelGGL((k_trsv_panel<true>), dim3((unsigned)((below + 255) / 256)), dim3(256), 0, s, nd, kb,
                               S, x);
    }
    for (int32_t kb = nb - 1; kb >= 0; --kb) {
        hipLaunchKernelGGL((k_trsv_diag<false>), dim3(1), dim3(64), 0, s, nd, kb, S, x);
        const int64_t above = (int64_t)kb * kT;
        if (above > 0)
            hipLaunchKernelGGL((k_trsv_panel<false>), dim3((unsigned)((above + 255) / 256)), dim3(256), 0, s, nd,
                               kb, S, x);
    }
    return hipGetLastError();
}

template hipError_t launch_dense_solve<float>(const DensePlan&, const PointMajor&, int64_t,
                                              const RecomputeInputs<float>&, const float*, int32_t, const double*,
                                              const double*, const double*, double*, double*, int32_t*,
                                              hipStream_t);
template hipError_t launch_dense_solve<double>(const DensePlan&, const PointMajor&, int64_t,
                                               const RecomputeInputs<double>&, const double*, int32_t,
                                               const double*, const double*, const double*, double*, double*,
                                               int32_t*, hipStream_t);

}  // namespace ba

// Implicit Schur product of Alg. 3 (DSE) with one partition, and the reduced
// right-hand side of Eq. schur_x_c that shares its second half:
//   mode 0:  c = E C~^-1 E^T x,  then q = B~ x - c   (and p^T q)
//   mode 1:  c = E C~^-1 w,      then g = v - c      (r = g, x = 0, ||g||^2)
//
// E is held as one 9x3 block per observation (27 coalesced streams) in
// point-major order.  Per point i, a_i = sum_k E_k^T x_j(k) needs all of the
// point's observations before b_i = C~_i^-1 a_i, and then every observation
// adds E_k b_i into its camera.  The camera side is Zipf-skewed (the most
// seen camera is in ~60% of the points), so the scatter is organised by
// camera popularity (cameras are relabelled most-observed first):
//
//   pass 1 (k_schur_hot): persistent workgroups, one per CU; every
//     wavefront streams its own range of line-aligned 64-observation tiles
//     (one observation per lane) with the next tile prefetched into
//     registers.  a_i is summed by a segmented scan over shuffles (points
//     that straddle tiles are carried) and b_i is formed in registers;
//     contributions to the K hottest cameras accumulate in a per-workgroup
//     LDS copy of their 9-vectors (K sized to fill the 160 KB LDS), written
//     out once at the end.  b_i of points that also have observations on
//     colder cameras is stored.
//   pass 2 (k_schur_cold): the observations on cameras >= K, from their own
//     camera-major copy of E, gather b_i and are reduced per camera by
//     wavefront chunks into fixed partial-sum slots (no atomics).
//   epilogue (k_schur_epilogue): per camera entry, sums the workgroup
//     partials (hot) or the slots (cold) in a fixed order and forms q or g.
// A point spanning more than two tiles re-reads its older blocks once (L2).
#include "ba_internal.h"

namespace ba {

// Observation 64 t + lane of line-aligned tile t.
template <typename T>
__device__ __forceinline__ void load_tile(int64_t t, int64_t N, int64_t ld, int lane, const int32_t* __restrict__ cam,
                                          const int32_t* __restrict__ pt, const T* __restrict__ hcp, int32_t& j,
                                          int32_t& i, T h[27])
{
    const int64_t k = 64 * t + lane;
    if (k < N) {
        j = cam[k];
        i = pt[k];
#pragma unroll
        for (int q = 0; q < 27; ++q) h[q] = hcp[(int64_t)q * ld + k];
    } else {
        j = 0;
        i = -1;
#pragma unroll
        for (int q = 0; q < 27; ++q) h[q] = (T)0;
    }
}

template <typename T>
__device__ __forceinline__ void add_hot(double* __restrict__ cl, int32_t j, const T h[27], T b0, T b1, T b2)
{
    double* dst = cl + 9 * j;
#pragma unroll
    for (int a = 0; a < 9; ++a)
        atomicAdd(dst + a, (double)(h[a * 3] * b0 + h[a * 3 + 1] * b1 + h[a * 3 + 2] * b2));
}

// Pass 1.  Tile t holds observations [64 t, 64 t + 64), one per lane, so
// every load is whole 128-byte lines.  Each wavefront owns the points that
// start in its range of tiles.  Per-point sums use a segmented scan over
// shuffles; a point that runs on into the next tile is carried (its partial
// sum) and finished when its
// last observation arrives (its earlier blocks are read again, from L2); the
// last point of a range is followed past the range end.  The next tile is
// loaded while the current one is processed.
// The hot-camera table is FP64 in both precisions: LDS FP64 adds issue
// without the back-pressure FP32 LDS adds show here, and the per-workgroup
// sums of the most observed cameras keep FP64 accuracy.
template <typename T, int MODE>
__global__ __launch_bounds__(HotThreads<T>::value) void k_schur_hot(
    const int32_t* __restrict__ wrange, int64_t N, int64_t ld, const int32_t* __restrict__ cam,
    const int32_t* __restrict__ pt, const T* __restrict__ hcp, const T* __restrict__ cinv,
    const double* __restrict__ wpt, const T* __restrict__ xcam, int32_t K, double* __restrict__ hot_part,
    T* __restrict__ bcold, const uint8_t* __restrict__ has_cold, const PcgScalars* __restrict__ sc)
{
    constexpr int NT = HotThreads<T>::value;
    if (MODE == 0 && sc->done) return;  // uniform over the grid
    extern __shared__ __align__(16) unsigned char smem[];
    double* cl = reinterpret_cast<double*>(smem);
    for (int q = threadIdx.x; q < K * 9; q += NT) cl[q] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int32_t gw = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    const int64_t T0 = wrange[gw], T1 = wrange[gw + 1];
    const int64_t ntiles = (N + 63) >> 6;
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    if (T0 < T1) {
        const int32_t skip_pt = T0 > 0 ? pt[64 * T0 - 1] : -1;  // owned by the previous wavefront
        int32_t carry_pt = -1;
        T cr0 = (T)0, cr1 = (T)0, cr2 = (T)0;
        int64_t carry_start = 0;
        int32_t cj, ci;
        T ch[27];
        load_tile<T>(T0, N, ld, lane, cam, pt, hcp, cj, ci, ch);
        for (int64_t t = T0; t < ntiles && (t < T1 || carry_pt >= 0); ++t) {
            int32_t nj = 0, ni = -1;
            T nh[27];
            const bool prefetch = t + 1 < T1;
            if (prefetch) load_tile<T>(t + 1, N, ld, lane, cam, pt, hcp, nj, ni, nh);
            const bool valid = 64 * t + lane < N;
            const bool owned = valid && (t < T1 ? ci != skip_pt : ci == carry_pt);
            const uint64_t om = __ballot(owned);
            if (om != 0) {
                const int32_t prev_i = __shfl_up(ci, 1, 64);
                const int prev_own = __shfl_up(owned ? 1 : 0, 1, 64);
                const bool head = owned && (lane == 0 || !prev_own || prev_i != ci);
                const uint64_t hm = __ballot(head);
                const int seg_s = 63 - __clzll((hm & upto) | 1ull);
                const int last_owned = 63 - __clzll(om);
                const uint64_t above = hm & ~upto;
                const int seg_e = above ? __ffsll((unsigned long long)above) - 2 : last_owned;
                const int first_head = __ffsll((unsigned long long)hm) - 1;
                const int last_head = 63 - __clzll(hm);
                const int32_t i_first = __shfl(ci, first_head, 64);
                const int32_t i_last = __shfl(ci, last_owned, 64);
                const bool cont = carry_pt >= 0 && i_first == carry_pt;
                int32_t inext0 = -2;
                if (last_owned == 63 && t + 1 < ntiles) inext0 = prefetch ? __shfl(ni, 0, 64) : pt[64 * (t + 1)];
                const bool last_inc = last_owned == 63 && inext0 == i_last;
                if (MODE == 0) {
                    T a0 = (T)0, a1 = (T)0, a2 = (T)0;
                    if (owned) {
                        T x[9];
#pragma unroll
                        for (int a = 0; a < 9; ++a) x[a] = xcam[9 * (int64_t)cj + a];
#pragma unroll
                        for (int a = 0; a < 9; ++a) {
                            a0 += ch[a * 3] * x[a];
                            a1 += ch[a * 3 + 1] * x[a];
                            a2 += ch[a * 3 + 2] * x[a];
                        }
                    }
#pragma unroll
                    for (int off = 1; off < 64; off <<= 1) {
                        const T u0 = __shfl_up(a0, off, 64), u1 = __shfl_up(a1, off, 64), u2 = __shfl_up(a2, off, 64);
                        if (lane - off >= seg_s) {
                            a0 += u0;
                            a1 += u1;
                            a2 += u2;
                        }
                    }
                    a0 = __shfl(a0, seg_e, 64);
                    a1 = __shfl(a1, seg_e, 64);
                    a2 = __shfl(a2, seg_e, 64);
                    if (cont && seg_s == first_head) {
                        a0 += cr0;
                        a1 += cr1;
                        a2 += cr2;
                    }
                    const bool deferred = last_inc && seg_s == last_head;
                    T b0 = (T)0, b1 = (T)0, b2 = (T)0;
                    if (owned && !deferred) {
                        const T* c6 = cinv + 6 * (int64_t)ci;
                        b0 = c6[0] * a0 + c6[1] * a1 + c6[2] * a2;
                        b1 = c6[1] * a0 + c6[3] * a1 + c6[4] * a2;
                        b2 = c6[2] * a0 + c6[4] * a1 + c6[5] * a2;
                        if (lane == seg_e && has_cold[ci]) {
                            bcold[3 * (int64_t)ci] = b0;
                            bcold[3 * (int64_t)ci + 1] = b1;
                            bcold[3 * (int64_t)ci + 2] = b2;
                        }
                        if (cj < K) add_hot<T>(cl, cj, ch, b0, b1, b2);
                    }
                    if (cont && !(last_inc && first_head == last_head)) {
                        // the carried point ends here: its observations in earlier tiles,
                        // streamed moments ago, are read again (from L2)
                        const T cb0 = __shfl(b0, first_head, 64), cb1 = __shfl(b1, first_head, 64),
                                cb2 = __shfl(b2, first_head, 64);
                        const int64_t older_end = 64 * t;
                        for (int64_t base = carry_start; base < older_end; base += 64) {
                            const int64_t kk = base + lane;
                            if (kk < older_end) {
                                const int32_t j = cam[kk];
                                if (j < K) {
                                    T h[27];
#pragma unroll
                                    for (int q = 0; q < 27; ++q) h[q] = hcp[(int64_t)q * ld + kk];
                                    add_hot<T>(cl, j, h, cb0, cb1, cb2);
                                }
                            }
                        }
                    }
                    if (last_inc) {
                        cr0 = __shfl(a0, last_head, 64);
                        cr1 = __shfl(a1, last_head, 64);
                        cr2 = __shfl(a2, last_head, 64);
                        if (!(cont && first_head == last_head)) carry_start = 64 * t + last_head;
                        carry_pt = i_last;
                    } else {
                        carry_pt = -1;
                    }
                } else {
                    if (owned) {
                        const T* c6 = cinv + 6 * (int64_t)ci;
                        const T w0 = (T)wpt[3 * (int64_t)ci], w1 = (T)wpt[3 * (int64_t)ci + 1],
                                w2 = (T)wpt[3 * (int64_t)ci + 2];
                        const T b0 = c6[0] * w0 + c6[1] * w1 + c6[2] * w2;
                        const T b1 = c6[1] * w0 + c6[3] * w1 + c6[4] * w2;
                        const T b2 = c6[2] * w0 + c6[4] * w1 + c6[5] * w2;
                        if (lane == seg_s && has_cold[ci]) {
                            bcold[3 * (int64_t)ci] = b0;
                            bcold[3 * (int64_t)ci + 1] = b1;
                            bcold[3 * (int64_t)ci + 2] = b2;
                        }
                        if (cj < K) add_hot<T>(cl, cj, ch, b0, b1, b2);
                    }
                    carry_pt = last_inc ? i_last : -1;
                }
            }
            if (prefetch) {
                cj = nj;
                ci = ni;
#pragma unroll
                for (int q = 0; q < 27; ++q) ch[q] = nh[q];
            } else if (carry_pt >= 0 && t + 1 < ntiles) {
                load_tile<T>(t + 1, N, ld, lane, cam, pt, hcp, cj, ci, ch);
            }
        }
    }
    __syncthreads();
    double* out = hot_part + (int64_t)blockIdx.x * K * 9;
    for (int q = threadIdx.x; q < K * 9; q += NT) out[q] = cl[q];
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Cold observations, camera-major: c_k = E_k b_i, reduced per camera by wave
// chunks of kColdChunk observations into slots (one per chunk and camera run).
template <typename T>
__global__ __launch_bounds__(256) void k_schur_cold(int64_t Nc, int32_t num_chunks, const int32_t* __restrict__ ccam,
                                                    const int32_t* __restrict__ cpt, const T* __restrict__ chcp,
                                                    const T* __restrict__ bcold, const int32_t* __restrict__ chunk_slot,
                                                    double* __restrict__ slots, const PcgScalars* __restrict__ sc,
                                                    int skip_if_done)
{
    if (skip_if_done && sc->done) return;
    const int lane = threadIdx.x & 63;
    const int32_t chunk = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    if (chunk >= num_chunks) return;
    const int64_t start = (int64_t)chunk * kColdChunk;
    const int64_t end = start + kColdChunk < Nc ? start + kColdChunk : Nc;
    int32_t slot = chunk_slot[chunk];
    int32_t cur = ccam[start];
    double acc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) acc[a] = 0.0;
    for (int row = 0; row < kColdRows; ++row) {
        if (start + (int64_t)row * 64 >= end) break;
        const int64_t k = start + (int64_t)row * 64 + lane;
        const bool valid = k < end;
        int32_t j = 0x7fffffff;
        T c[9];
        if (valid) {
            j = ccam[k];
            const int32_t i = cpt[k];
            const T b0 = bcold[3 * (int64_t)i], b1 = bcold[3 * (int64_t)i + 1], b2 = bcold[3 * (int64_t)i + 2];
#pragma unroll
            for (int a = 0; a < 9; ++a)
                c[a] = chcp[(int64_t)(a * 3) * Nc + k] * b0 + chcp[(int64_t)(a * 3 + 1) * Nc + k] * b1 +
                       chcp[(int64_t)(a * 3 + 2) * Nc + k] * b2;
        }
        while (true) {
            if (valid && j == cur)
#pragma unroll
                for (int a = 0; a < 9; ++a) acc[a] += (double)c[a];
            const uint64_t more = __ballot(valid && j > cur);
            if (more == 0) break;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const double v = wave_sum_d(acc[a]);
                if (lane == 0) slots[(int64_t)slot * 9 + a] = v;
                acc[a] = 0.0;
            }
            ++slot;
            cur = __shfl(j, __ffsll((unsigned long long)more) - 1, 64);
        }
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double v = wave_sum_d(acc[a]);
        if (lane == 0) slots[(int64_t)slot * 9 + a] = v;
    }
}

// Folds the per-workgroup hot partials [G][K*9] into kHotFold slices, each
// the sum of a contiguous range of workgroups in order.
__global__ __launch_bounds__(256) void k_hot_fold(int32_t K9, int32_t G, const double* __restrict__ hot_part,
                                                  double* __restrict__ fold, const PcgScalars* __restrict__ sc,
                                                  int skip_if_done)
{
    if (skip_if_done && sc->done) return;
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    const int32_t f = blockIdx.y;
    if (t >= K9) return;
    const int32_t w0 = (int32_t)((int64_t)f * G / kHotFold), w1 = (int32_t)((int64_t)(f + 1) * G / kHotFold);
    double c0 = 0.0, c1 = 0.0;
    int32_t w = w0;
    for (; w + 2 <= w1; w += 2) {
        c0 += hot_part[(int64_t)w * K9 + t];
        c1 += hot_part[(int64_t)(w + 1) * K9 + t];
    }
    if (w < w1) c0 += hot_part[(int64_t)w * K9 + t];
    fold[(int64_t)f * K9 + t] = c0 + c1;
}

// q = B~ x - c (mode 0) or g = v - c, r = g, x = 0 (mode 1); c from the hot
// slices and the cold slots.  The last block adds the per-block partial sums:
// mode 0: p^T q, then alpha = rho / p^T q and the matvec count (or a breakdown
// when p^T q <= 0); mode 1: ||b||^2.
template <int MODE>
__global__ __launch_bounds__(kRedBlock) void k_schur_epilogue(
    int32_t m, int32_t K, const double* __restrict__ hot_fold, const int32_t* __restrict__ cold_cam_slot,
    const double* __restrict__ cold_slots, const double* __restrict__ bd,
    const double* __restrict__ pvec, const double* __restrict__ vcam, double* __restrict__ out,
    double* __restrict__ xvec, double* __restrict__ rvec, double* __restrict__ partials,
    PcgScalars* __restrict__ sc)
{
    __shared__ double sh[kRedBlock / 64];
    if (MODE == 0 && sc->done) return;  // uniform over the grid
    double acc = 0.0;
    const int64_t len = 9 * (int64_t)m;
    for (int64_t t = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; t < len; t += (int64_t)gridDim.x * kRedBlock) {
        const int64_t j = t / 9;
        const int a = (int)(t - 9 * j);
        double c = 0.0;
        if (j < K) {
            const int64_t stride = (int64_t)K * 9;
#pragma unroll
            for (int f = 0; f < kHotFold; ++f) c += hot_fold[(int64_t)f * stride + t];
        } else {
            for (int32_t s = cold_cam_slot[j]; s < cold_cam_slot[j + 1]; ++s) c += cold_slots[(int64_t)s * 9 + a];
        }
        if (MODE == 0) {
            const double* B = bd + 81 * j + 9 * a;
            const double* pj = pvec + 9 * j;
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < 9; ++u) v += B[u] * pj[u];
            v -= c;
            out[t] = v;
            acc += pvec[t] * v;
        } else {
            const double v = vcam[t] - c;
            out[t] = v;
            rvec[t] = v;
            xvec[t] = 0.0;
            acc += v * v;
        }
    }
    acc = wave_sum_d(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kRedBlock / 64; ++w) s += sh[w];
        partials[blockIdx.x] = s;
    }
    if (!last_block_arrives(&sc->arrive[MODE == 0 ? 1 : 2])) return;
    double tot = 0.0;
    for (int32_t b = threadIdx.x; b < (int32_t)gridDim.x; b += kRedBlock) tot += partials[b];
    tot = wave_sum_d(tot);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kRedBlock / 64; ++w) s += sh[w];
        if (MODE == 0) {
            sc->pq = s;
            if (!(s > 0.0) || !isfinite(s)) {
                sc->breakdown = 1;
                sc->done = 1;
            } else {
                sc->alpha = sc->rho / s;
            }
            sc->iters = sc->iters + 1;
            sc->arrive[1] = 0u;
        } else {
            sc->bb = s;
            sc->rr = s;
            sc->arrive[2] = 0u;
        }
    }
}

template <typename T>
size_t hot_lds_bytes(int32_t K)
{
    return (size_t)K * 9 * sizeof(double);
}

template <typename T>
int32_t hot_max_cameras(size_t lds_limit)
{
    if (lds_limit <= 1024) return 0;
    return (int32_t)((lds_limit - 1024) / (9 * sizeof(double)));
}

template <typename T>
hipError_t prepare_schur_kernels(int32_t K)
{
    const int bytes = (int)hot_lds_bytes<T>(K);
    hipError_t e = hipFuncSetAttribute((const void*)k_schur_hot<T, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_schur_hot<T, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T>
hipError_t launch_schur_product(int mode, const SchurPlan& sp, const PointMajor& pm, int64_t N, const T* hcp,
                                const T* cinv, const double* wpt, const T* xcam, int32_t m, const double* bd,
                                const double* pvec, const double* vcam, double* out, double* xvec, double* rvec,
                                double* partials, PcgScalars* sc, hipEvent_t hot_begin, hipEvent_t hot_end,
                                hipStream_t s)
{
    hipError_t e;
    const size_t lds = hot_lds_bytes<T>(sp.K);
    if (hot_begin && (e = hipEventRecord(hot_begin, s)) != hipSuccess) return e;
    if (sp.num_wg > 0) {
        const dim3 g(sp.num_wg), b(HotThreads<T>::value);
        if (mode == 0)
            hipLaunchKernelGGL((k_schur_hot<T, 0>), g, b, lds, s, sp.wrange, N, pm.ld, pm.cam, pm.pt, hcp, cinv,
                               wpt, xcam, sp.K, (double*)sp.hot_part, (T*)sp.bcold, sp.has_cold, sc);
        else
            hipLaunchKernelGGL((k_schur_hot<T, 1>), g, b, lds, s, sp.wrange, N, pm.ld, pm.cam, pm.pt, hcp, cinv,
                               wpt, xcam, sp.K, (double*)sp.hot_part, (T*)sp.bcold, sp.has_cold, sc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (hot_end && (e = hipEventRecord(hot_end, s)) != hipSuccess) return e;
    if (sp.cold.num_chunks > 0) {
        hipLaunchKernelGGL((k_schur_cold<T>), dim3((sp.cold.num_chunks + 3) / 4), dim3(256), 0, s, sp.cold.N,
                           sp.cold.num_chunks, sp.cold.cam, sp.cold.pt, (const T*)sp.cold.hcp, (const T*)sp.bcold,
                           sp.cold.chunk_slot, sp.cold.slots, (const PcgScalars*)sc, mode == 0 ? 1 : 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (sp.K > 0 && sp.num_wg > 0) {
        const int32_t K9 = sp.K * 9;
        hipLaunchKernelGGL(k_hot_fold, dim3((K9 + 255) / 256, kHotFold), dim3(256), 0, s, K9, sp.num_wg,
                           (const double*)sp.hot_part, sp.hot_fold, (const PcgScalars*)sc, mode == 0 ? 1 : 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int32_t nb = reduce_blocks(9 * (int64_t)m);
    const int32_t Ke = sp.num_wg > 0 ? sp.K : 0;
    if (mode == 0)
        hipLaunchKernelGGL((k_schur_epilogue<0>), dim3(nb), dim3(kRedBlock), 0, s, m, Ke, sp.hot_fold,
                           sp.cold.cam_slot, sp.cold.slots, bd, pvec, vcam, out, xvec, rvec, partials, sc);
    else
        hipLaunchKernelGGL((k_schur_epilogue<1>), dim3(nb), dim3(kRedBlock), 0, s, m, Ke, sp.hot_fold,
                           sp.cold.cam_slot, sp.cold.slots, bd, pvec, vcam, out, xvec, rvec, partials, sc);
    return hipGetLastError();
}

template size_t hot_lds_bytes<float>(int32_t);
template size_t hot_lds_bytes<double>(int32_t);
template int32_t hot_max_cameras<float>(size_t);
template int32_t hot_max_cameras<double>(size_t);
template hipError_t prepare_schur_kernels<float>(int32_t);
template hipError_t prepare_schur_kernels<double>(int32_t);
template hipError_t launch_schur_product<float>(int, const SchurPlan&, const PointMajor&, int64_t, const float*,
                                                const float*, const double*, const float*, int32_t, const double*,
                                                const double*, const double*, double*, double*, double*, double*,
                                                PcgScalars*, hipEvent_t, hipEvent_t, hipStream_t);
template hipError_t launch_schur_product<double>(int, const SchurPlan&, const PointMajor&, int64_t, const double*,
                                                 const double*, const double*, const double*, int32_t, const double*,
                                                 const double*, const double*, double*, double*, double*, double*,
                                                 PcgScalars*, hipEvent_t, hipEvent_t, hipStream_t);

}  // namespace ba

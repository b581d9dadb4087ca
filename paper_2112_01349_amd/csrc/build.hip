// Residual, Jacobian and Schur block assembly (Alg. 1: residual/Jacobian and
// Hessian/constant-vector steps; Sec. 3 Eq. schur_complement), and the FP64
// cost F = 1/2 sum rho(|e|^2) (Sec. 3 Eq. obj with a Huber loss).
//
// Two passes over the observations, each with its own sorted copy of the
// index and pixel streams:
//   * point-major (k_build_points): one workgroup per point-aligned tile of
//     <= 256 observations, one thread per observation.  Writes the coupling
//     block E_k = w J_c^T J_p (tile-blocked, see eidx), and sums the
//     point blocks C_i = sum w J_p^T J_p and w_i = -sum w J_p^T e over each
//     point's run through LDS.
//   * camera-major (k_build_cameras): one wavefront per contiguous chunk of
//     2048 observations sorted by camera.  Lanes accumulate the camera terms
//     B_j = sum w J_c^T J_c and v_j = -sum w J_c^T e in registers while the
//     camera does not change and flush a wavefront-reduced partial sum into a
//     slot when it does; slots of one camera are contiguous and are summed in
//     a fixed order by k_reduce_slots, so the result is deterministic.  This
//     balances the Zipf-skewed camera segments (the most-seen camera holds
//     about 60% of all points) over the whole chip, as the paper's equal-edge
//     partition (Sec. 4.1) does over GPUs.
//   * camera-major again (k_schur_jacobi_cameras), for the Schur-Jacobi
//     preconditioner option: the same slots sum -E_k C~^-1 E_k^T per camera
//     at the damping of the current LM iteration.
#include "ba_internal.h"
#include "autodiff.h"

namespace ba {

// ------------------------------------------------------- camera constants
template <typename T>
__global__ void k_camera_constants(int32_t m, const double* __restrict__ cams, CamK<T>* __restrict__ out)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    CamK<T> k;
    camera_constants<T>(cams + 9 * (int64_t)j, k);
    out[j] = k;
}

hipError_t launch_camera_constants_f64(int32_t m, const double* cams, CamK<double>* out, hipStream_t s)
{
    if (m > 0) hipLaunchKernelGGL(k_camera_constants<double>, dim3((m + 127) / 128), dim3(128), 0, s, m, cams, out);
    return hipGetLastError();
}

hipError_t launch_camera_constants_f32(int32_t m, const double* cams, CamK<float>* out, hipStream_t s)
{
    if (m > 0) hipLaunchKernelGGL(k_camera_constants<float>, dim3((m + 127) / 128), dim3(128), 0, s, m, cams, out);
    return hipGetLastError();
}

// ------------------------------------------------------ point-major build
// Terms of one observation for its point: C (upper 6) and w (3).  Each
// product is formed in FP64 from the T-precision Jacobian; a product of two
// floats is exact there, so the sum over a point's observations is the Gram
// matrix of the float Jacobian to FP64 rounding: positive semidefinite like
// the FP64 form's, instead of carrying float rounding of order 1e-7 of its
// largest eigenvalue into its smallest (a two-view point with a narrow
// baseline has a smaller one than that).
template <typename T>
__device__ __forceinline__ void point_terms(const T Jp[6], T e0, T e1, T wt, double out[9])
{
    const double w = wt, r0 = e0, r1 = e1;
    double j[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) j[q] = Jp[q];
    out[0] = w * (j[0] * j[0] + j[3] * j[3]);
    out[1] = w * (j[0] * j[1] + j[3] * j[4]);
    out[2] = w * (j[0] * j[2] + j[3] * j[5]);
    out[3] = w * (j[1] * j[1] + j[4] * j[4]);
    out[4] = w * (j[1] * j[2] + j[4] * j[5]);
    out[5] = w * (j[2] * j[2] + j[5] * j[5]);
    out[6] = -w * (j[0] * r0 + j[3] * r1);
    out[7] = -w * (j[1] * r0 + j[4] * r1);
    out[8] = -w * (j[2] * r0 + j[5] * r1);
}

template <typename T, bool AD>
__device__ __forceinline__ void observation(int64_t k, const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
                                            const double* __restrict__ uvx, const double* __restrict__ uvy,
                                            const double* __restrict__ pts, JacSource<T> js, T delta, T& e0, T& e1,
                                            T& wt, T Jc[18], T Jp[6], int32_t& i)
{
    const int32_t j = cam[k];
    i = pt[k];
    const double* Xd = pts + 3 * (int64_t)i;
    const T X0 = (T)Xd[0], X1 = (T)Xd[1], X2 = (T)Xd[2];
    const CamK<T>& kk = js.ck[j];
    if (AD) {
        residual_jacobian_ad<T>(js.cams + 9 * (int64_t)j, X0, X1, X2, (T)uvx[k], (T)uvy[k], e0, e1, Jc, Jp);
        if (sizeof(T) == 4) {  // an unresolved FP32 depth: the analytic form from the FP64 geometry
            const T RX2 = kk.R[6] * X0 + kk.R[7] * X1 + kk.R[8] * X2;
            if (!depth_resolved<T>(RX2, kk.t[2], RX2 + kk.t[2])) {
                ObsGeo<T> o;
                observation_geometry_checked<T>(kk.R, js.ck64, j, Xd, o);
                jacobian_from_geometry<T>(kk, o, (T)uvx[k], (T)uvy[k], e0, e1, Jc, Jp);
            }
        }
    } else {
        ObsGeo<T> o;
        observation_geometry_checked<T>(kk.R, js.ck64, j, Xd, o);
        jacobian_from_geometry<T>(kk, o, (T)uvx[k], (T)uvy[k], e0, e1, Jc, Jp);
    }
    wt = huber_weight<T>(e0 * e0 + e1 * e1, delta);
}

// E_k into the tile-blocked point-major array.
template <typename T>
__device__ __forceinline__ void store_coupling_blocked(int64_t k, const T Jc[18], const T Jp[6], T wt,
                                                       T* __restrict__ hcp)
{
    T* base = hcp + eidx(k, 0);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) base[(a * 3 + b) * 64] = wt * (Jc[a] * Jp[b] + Jc[9 + a] * Jp[3 + b]);
}

// E_k into row-major streams [27][N] (the cold copy).
template <typename T>
__device__ __forceinline__ void store_coupling(int64_t k, int64_t N, const T Jc[18], const T Jp[6], T wt,
                                               T* __restrict__ hcp)
{
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            hcp[(int64_t)(a * 3 + b) * N + k] = wt * (Jc[a] * Jp[b] + Jc[9 + a] * Jp[3 + b]);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Point-major build over point-aligned tiles of <= kTile observations (a
// longer point is a tile alone).  One thread per observation computes its
// residual and Jacobian, stores its IRLS weight and, when hcp is given,
// E_k = w J_c^T J_p (27 coalesced streams);
// its terms of C_i and w_i go to LDS (FP64), and the first thread of each
// point sums the point's terms in stream order and stores C_i (upper 6) and
// w_i in FP64.  GRAD_ONLY forms w_i only.
template <typename T, bool GRAD_ONLY, bool AD>
__global__ __launch_bounds__(kTile) void k_build_points(
    const int32_t* __restrict__ tile, const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
    const double* __restrict__ uvx, const double* __restrict__ uvy, const double* __restrict__ pts,
    JacSource<T> js, T delta, int64_t ld, T* __restrict__ hcp, double* __restrict__ hpp,
    double* __restrict__ wpt, T* __restrict__ wobs)
{
    constexpr int R = GRAD_ONLY ? 3 : 9;  // terms kept: [C upper 6 |] w 3
    __shared__ double sh[R][kTile];
    __shared__ int32_t shpt[kTile];
    __shared__ double red[R][kTile / 64];
    const int tid = threadIdx.x;
    const int32_t s = tile[blockIdx.x], e = tile[blockIdx.x + 1];
    const int32_t len = e - s;
    if (len <= kTile) {
        const bool valid = tid < len;
        int32_t i = -1;
        if (valid) {
            const int64_t k = s + tid;
            T e0, e1, wt, Jc[18], Jp[6];
            observation<T, AD>(k, cam, pt, uvx, uvy, pts, js, delta, e0, e1, wt, Jc, Jp, i);
            if (!GRAD_ONLY) {
                if (hcp) store_coupling_blocked<T>(k, Jc, Jp, wt, hcp);
                wobs[k] = wt;
            }
            double v[9];
            point_terms<T>(Jp, e0, e1, wt, v);
#pragma unroll
            for (int q = 0; q < R; ++q) sh[q][tid] = v[9 - R + q];
        }
        shpt[tid] = i;
        __syncthreads();
        if (valid && (tid == 0 || shpt[tid - 1] != i)) {
            double acc[R];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = 0.0;
            for (int u = tid; u < len && shpt[u] == i; ++u)
#pragma unroll
                for (int q = 0; q < R; ++q) acc[q] += sh[q][u];
            if (!GRAD_ONLY)
#pragma unroll
                for (int q = 0; q < 6; ++q) hpp[6 * (int64_t)i + q] = acc[q];
#pragma unroll
            for (int q = 0; q < 3; ++q) wpt[3 * (int64_t)i + q] = acc[R - 3 + q];
        }
    } else {
        // one point with more than kTile observations: strided partial sums,
        // then a fixed-order reduction over the block
        const int32_t i = pt[s];
        double acc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = 0.0;
        for (int64_t k = s + tid; k < e; k += kTile) {
            T e0, e1, wt, Jc[18], Jp[6];
            int32_t ii;
            observation<T, AD>(k, cam, pt, uvx, uvy, pts, js, delta, e0, e1, wt, Jc, Jp, ii);
            if (!GRAD_ONLY) {
                if (hcp) store_coupling_blocked<T>(k, Jc, Jp, wt, hcp);
                wobs[k] = wt;
            }
            double v[9];
            point_terms<T>(Jp, e0, e1, wt, v);
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] += v[9 - R + q];
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double w = wave_sum(acc[q]);
            if ((tid & 63) == 0) red[q][tid >> 6] = w;
        }
        __syncthreads();
        if (tid == 0) {
            double tot[R];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                tot[q] = 0.0;
                for (int w = 0; w < kTile / 64; ++w) tot[q] += red[q][w];
            }
            if (!GRAD_ONLY)
#pragma unroll
                for (int q = 0; q < 6; ++q) hpp[6 * (int64_t)i + q] = tot[q];
#pragma unroll
            for (int q = 0; q < 3; ++q) wpt[3 * (int64_t)i + q] = tot[R - 3 + q];
        }
    }
}

template <typename T, bool G, bool A>
static void build_points_variant(const PointMajor& pm, const double* pts, JacSource<T> js, T delta, T* hcp,
                                 double* hpp, double* wpt, T* wobs, hipStream_t s)
{
    hipLaunchKernelGGL((k_build_points<T, G, A>), dim3((unsigned)pm.num_tiles), dim3(kTile), 0, s, pm.tile, pm.cam,
                       pm.pt, pm.uvx, pm.uvy, pts, js, delta, pm.ld, hcp, hpp, wpt, wobs);
}

template <typename T>
hipError_t launch_build_points(const PointMajor& pm, double delta, bool grad_only, const double* pts,
                               JacSource<T> js, T* hcp, double* hpp, double* wpt, T* wobs, hipStream_t s)
{
    if (pm.num_tiles <= 0) return hipGetLastError();
    const bool ad = js.cams != nullptr;
    const T d = (T)delta;
    if (grad_only) {
        if (ad) build_points_variant<T, true, true>(pm, pts, js, d, nullptr, nullptr, wpt, nullptr, s);
        else build_points_variant<T, true, false>(pm, pts, js, d, nullptr, nullptr, wpt, nullptr, s);
    } else {
        if (ad) build_points_variant<T, false, true>(pm, pts, js, d, hcp, hpp, wpt, wobs, s);
        else build_points_variant<T, false, false>(pm, pts, js, d, hcp, hpp, wpt, wobs, s);
    }
    return hipGetLastError();
}

// ----------------------------------------------------- camera-major build

// Wave sums of the W accumulated words into one slot.
template <int W>
__device__ __forceinline__ void flush_slot(double* acc, double* __restrict__ slots, int32_t slot, int lane)
{
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) slots[(int64_t)slot * kCamSlotWords + q] = v;
        acc[q] = 0.0;
    }
}

template <typename T, bool GRAD_ONLY, bool AD>
__global__ __launch_bounds__(256) void k_build_cameras(
    int64_t N, int32_t num_chunks, const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
    const double* __restrict__ uvx, const double* __restrict__ uvy, const double* __restrict__ pts,
    JacSource<T> js, T delta, const int32_t* __restrict__ chunk_slot, double* __restrict__ slots,
    int64_t Nc, T* __restrict__ chcp, T* __restrict__ cw)
{
    constexpr int W = GRAD_ONLY ? 9 : kCamSlotWords;
    const int64_t cold0 = N - Nc;  // the cold cameras' observations are the stream's tail
    const int lane = threadIdx.x & 63;
    const int32_t chunk = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    if (chunk >= num_chunks) return;  // whole wavefront leaves together
    const int64_t start = (int64_t)chunk * kCmChunk;
    const int64_t end = start + kCmChunk < N ? start + kCmChunk : N;
    int32_t slot = chunk_slot[chunk];
    int32_t cur = cam[start];
    double acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0.0;
    for (int row = 0; row < kCmRows; ++row) {
        const int64_t k = start + (int64_t)row * 64 + lane;
        if (start + (int64_t)row * 64 >= end) break;
        const bool valid = k < end;
        T e0 = 0, e1 = 0, wt = 0, Jc[18], Jp[6];
        int32_t j = 0x7fffffff;
        if (valid) {
            int32_t i;
            j = cam[k];
            observation<T, AD>(k, cam, pt, uvx, uvy, pts, js, delta, e0, e1, wt, Jc, Jp, i);
            if (!GRAD_ONLY && k >= cold0) {
                if (chcp) store_coupling<T>(k - cold0, Nc, Jc, Jp, wt, chcp);
                if (cw) cw[k - cold0] = wt;
            }
        }
        while (true) {
            if (valid && j == cur) {
                // FP64 products of the T-precision Jacobian (exact for
                // float), as in point_terms: B_j stays a Gram matrix
                const double w = wt, r0 = e0, r1 = e1;
                double jc[18];
#pragma unroll
                for (int a = 0; a < 18; ++a) jc[a] = Jc[a];
                int q = 0;
                if (!GRAD_ONLY) {
#pragma unroll
                    for (int a = 0; a < 9; ++a)
#pragma unroll
                        for (int b = a; b < 9; ++b) acc[q++] += w * (jc[a] * jc[b] + jc[9 + a] * jc[9 + b]);
                }
#pragma unroll
                for (int a = 0; a < 9; ++a) acc[q++] += -w * (jc[a] * r0 + jc[9 + a] * r1);
            }
            // lanes not yet consumed hold larger camera ids (the chunk is sorted)
            const uint64_t more = __ballot(valid && j > cur);
            if (more == 0) break;
            flush_slot<W>(acc, slots, slot, lane);
            ++slot;
            const int first = __ffsll((unsigned long long)more) - 1;
            cur = __shfl(j, first, 64);  // strictly larger: the loop ends
        }
    }
    flush_slot<W>(acc, slots, slot, lane);
}

// One wavefront per segment of <= kSlotSeg consecutive slots of one camera
// (lanes = the 54 terms).  A camera with one segment is written directly;
// otherwise the last of its segments to finish (device-scope counter) adds
// the segment sums in segment order, so the result is deterministic.
// MODE 0: the 45 upper-triangle B terms and the 9 v terms into hcc and vcam;
// MODE 1: the 9 v terms only; MODE 2: 45 upper-triangle terms only, into hcc.
template <int MODE>
__global__ __launch_bounds__(256) void k_reduce_slots(int32_t num_segs, const int32_t* __restrict__ seg_cam,
                                                      const int32_t* __restrict__ seg_slot,
                                                      const int32_t* __restrict__ cam_slot,
                                                      const int32_t* __restrict__ cam_seg,
                                                      const double* __restrict__ slots,
                                                      double* __restrict__ seg_part, uint32_t* __restrict__ arrive,
                                                      double* __restrict__ hcc, double* __restrict__ vcam)
{
    const int lane = threadIdx.x & 63;
    const int32_t sg = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    if (sg >= num_segs) return;
    const int32_t j = seg_cam[sg];
    const int32_t s0 = seg_slot[sg];
    const int32_t s1 = min(s0 + kSlotSeg, cam_slot[j + 1]);
    const int W = MODE == 1 ? 9 : (MODE == 2 ? 45 : kCamSlotWords);
    double acc = 0.0;
    if (lane < W)
        for (int32_t sl = s0; sl < s1; ++sl) acc += slots[(int64_t)sl * kCamSlotWords + lane];
    const int32_t g0 = cam_seg[j], g1 = cam_seg[j + 1];
    if (g1 - g0 > 1) {
        if (lane < W) seg_part[(int64_t)sg * kCamSlotWords + lane] = acc;
        __threadfence();
        uint32_t prev = 0;
        if (lane == 0) prev = atomicAdd(arrive + j, 1u);
        prev = __shfl(prev, 0, 64);
        if (prev != (uint32_t)(g1 - g0 - 1)) return;
        __threadfence();
        acc = 0.0;
        if (lane < W)
            for (int32_t g = g0; g < g1; ++g) acc += seg_part[(int64_t)g * kCamSlotWords + lane];
        if (lane == 0) arrive[j] = 0u;
    }
    if (lane >= W) return;
    const int q = MODE == 1 ? 45 + lane : lane;
    if (q < 45) {
        // upper-triangle index q -> (a, b), a <= b
        int a = 0, rem = q;
        while (rem >= 9 - a) {
            rem -= 9 - a;
            ++a;
        }
        const int b = a + rem;
        hcc[81 * (int64_t)j + a * 9 + b] = acc;
        hcc[81 * (int64_t)j + b * 9 + a] = acc;
    } else {
        vcam[9 * (int64_t)j + (q - 45)] = acc;
    }
}

template <typename T, bool G, bool A>
static void build_cameras_variant(const CameraMajor& cm, int64_t N, const double* pts, JacSource<T> js, T delta,
                                  int64_t Nc, T* chcp, T* cw, hipStream_t s)
{
    hipLaunchKernelGGL((k_build_cameras<T, G, A>), dim3((cm.num_chunks + 3) / 4), dim3(256), 0, s, N, cm.num_chunks,
                       cm.cam, cm.pt, cm.uvx, cm.uvy, pts, js, delta, cm.chunk_slot, cm.slots, Nc, chcp, cw);
}

template <typename T>
hipError_t launch_build_cameras(const CameraMajor& cm, int32_t m, int64_t N, const double* pts, JacSource<T> js,
                                double delta, bool grad_only, double* hcc, double* vcam, int64_t Nc, T* chcp,
                                T* cw, hipStream_t s)
{
    if (cm.num_chunks > 0) {
        const bool ad = js.cams != nullptr;
        const T d = (T)delta;
        if (grad_only) {
            if (ad) build_cameras_variant<T, true, true>(cm, N, pts, js, d, 0, nullptr, nullptr, s);
            else build_cameras_variant<T, true, false>(cm, N, pts, js, d, 0, nullptr, nullptr, s);
        } else {
            if (ad) build_cameras_variant<T, false, true>(cm, N, pts, js, d, Nc, chcp, cw, s);
            else build_cameras_variant<T, false, false>(cm, N, pts, js, d, Nc, chcp, cw, s);
        }
    }
    if (cm.num_segs > 0) {
        const int blocks = (cm.num_segs + 3) / 4;
        if (grad_only)
            hipLaunchKernelGGL((k_reduce_slots<1>), dim3(blocks), dim3(256), 0, s, cm.num_segs, cm.seg_cam,
                               cm.seg_slot, cm.cam_slot, cm.cam_seg, cm.slots, cm.seg_part, cm.arrive, hcc, vcam);
        else
            hipLaunchKernelGGL((k_reduce_slots<0>), dim3(blocks), dim3(256), 0, s, cm.num_segs, cm.seg_cam,
                               cm.seg_slot, cm.cam_slot, cm.cam_seg, cm.slots, cm.seg_part, cm.arrive, hcc, vcam);
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- FP64 cost
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_cost(int64_t N, const int32_t* __restrict__ cam,
                                                    const int32_t* __restrict__ pt, const double* __restrict__ uvx,
                                                    const double* __restrict__ uvy, const double* __restrict__ pts,
                                                    const CamK<T>* __restrict__ ck, T delta,
                                                    double* __restrict__ partials)
{
    __shared__ double sh[kRedBlock / 64];
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; k < N; k += (int64_t)gridDim.x * kRedBlock) {
        const int32_t j = cam[k], i = pt[k];
        const CamK<T> kk = ck[j];
        T e0, e1;
        residual<T>(kk, (T)pts[3 * (int64_t)i], (T)pts[3 * (int64_t)i + 1], (T)pts[3 * (int64_t)i + 2], (T)uvx[k],
                    (T)uvy[k], e0, e1);
        acc += 0.5 * (double)huber_rho<T>(e0 * e0 + e1 * e1, delta);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kRedBlock / 64; ++w) t += sh[w];
        partials[blockIdx.x] = t;
    }
}

int32_t reduce_blocks(int64_t count)
{
    int64_t b = (count + kRedBlock - 1) / kRedBlock;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int32_t)b;
}

template <typename T>
hipError_t launch_cost_t(const PointMajor& pm, int64_t N, const double* pts, const CamK<T>* ck, double delta,
                         double* partials, int32_t* nblocks, hipStream_t s)
{
    const int32_t b = reduce_blocks(N);
    *nblocks = b;
    hipLaunchKernelGGL((k_cost<T>), dim3(b), dim3(kRedBlock), 0, s, N, pm.cam, pm.pt, pm.uvx, pm.uvy, pts, ck,
                       (T)delta, partials);
    return hipGetLastError();
}

hipError_t launch_cost(const PointMajor& pm, int64_t N, const double* pts, const CamK<double>* ck, double delta,
                       double* partials, int32_t* nblocks, hipStream_t s)
{
    return launch_cost_t<double>(pm, N, pts, ck, delta, partials, nblocks, s);
}

// Schur-Jacobi preconditioner terms: per camera, the sum over its
// observations of E_k C~_i^-1 E_k^T (E_k = w J_c^T J_p, the damped point
// inverse of the current lambda), negated, camera-major as the B_j build.
// Products in FP64 from the T-precision Jacobian.
template <typename T, bool AD>
__global__ __launch_bounds__(256) void k_schur_jacobi_cameras(
    int64_t N, int32_t num_chunks, const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
    const double* __restrict__ uvx, const double* __restrict__ uvy, const double* __restrict__ pts,
    JacSource<T> js, T delta, const T* __restrict__ cinv, const int32_t* __restrict__ chunk_slot,
    double* __restrict__ slots)
{
    constexpr int W = 45;
    const int lane = threadIdx.x & 63;
    const int32_t chunk = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    if (chunk >= num_chunks) return;  // whole wavefront leaves together
    const int64_t start = (int64_t)chunk * kCmChunk;
    const int64_t end = start + kCmChunk < N ? start + kCmChunk : N;
    int32_t slot = chunk_slot[chunk];
    int32_t cur = cam[start];
    double acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0.0;
    for (int row = 0; row < kCmRows; ++row) {
        const int64_t k = start + (int64_t)row * 64 + lane;
        if (start + (int64_t)row * 64 >= end) break;
        const bool valid = k < end;
        T e0 = 0, e1 = 0, wt = 0, Jc[18], Jp[6];
        int32_t j = 0x7fffffff, i = 0;
        if (valid) {
            j = cam[k];
            observation<T, AD>(k, cam, pt, uvx, uvy, pts, js, delta, e0, e1, wt, Jc, Jp, i);
        }
        while (true) {
            if (valid && j == cur) {
                const double w = wt;
                double E[27], Tm[27];
#pragma unroll
                for (int a = 0; a < 9; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        E[a * 3 + c] = w * ((double)Jc[a] * (double)Jp[c] + (double)Jc[9 + a] * (double)Jp[3 + c]);
                const T* c6 = cinv + 6 * (int64_t)i;
                const double C[9] = {(double)c6[0], (double)c6[1], (double)c6[2], (double)c6[1], (double)c6[3],
                                     (double)c6[4], (double)c6[2], (double)c6[4], (double)c6[5]};
#pragma unroll
                for (int a = 0; a < 9; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        Tm[a * 3 + c] = E[a * 3] * C[c] + E[a * 3 + 1] * C[3 + c] + E[a * 3 + 2] * C[6 + c];
                int q = 0;
#pragma unroll
                for (int a = 0; a < 9; ++a)
#pragma unroll
                    for (int b = a; b < 9; ++b)
                        acc[q++] -= Tm[a * 3] * E[b * 3] + Tm[a * 3 + 1] * E[b * 3 + 1] + Tm[a * 3 + 2] * E[b * 3 + 2];
            }
            const uint64_t more = __ballot(valid && j > cur);
            if (more == 0) break;
            flush_slot<W>(acc, slots, slot, lane);
            ++slot;
            const int first = __ffsll((unsigned long long)more) - 1;
            cur = __shfl(j, first, 64);
        }
    }
    flush_slot<W>(acc, slots, slot, lane);
}

template <typename T>
hipError_t launch_schur_jacobi_terms(const CameraMajor& cm, int64_t N, const double* pts, JacSource<T> js,
                                     double delta, const T* cinv, double* mj, hipStream_t s)
{
    if (cm.num_chunks > 0) {
        const dim3 grid((cm.num_chunks + 3) / 4);
        if (js.cams)
            hipLaunchKernelGGL((k_schur_jacobi_cameras<T, true>), grid, dim3(256), 0, s, N, cm.num_chunks, cm.cam,
                               cm.pt, cm.uvx, cm.uvy, pts, js, (T)delta, cinv, cm.chunk_slot, cm.slots);
        else
            hipLaunchKernelGGL((k_schur_jacobi_cameras<T, false>), grid, dim3(256), 0, s, N, cm.num_chunks, cm.cam,
                               cm.pt, cm.uvx, cm.uvy, pts, js, (T)delta, cinv, cm.chunk_slot, cm.slots);
    }
    if (cm.num_segs > 0)
        hipLaunchKernelGGL((k_reduce_slots<2>), dim3((cm.num_segs + 3) / 4), dim3(256), 0, s, cm.num_segs,
                           cm.seg_cam, cm.seg_slot, cm.cam_slot, cm.cam_seg, cm.slots, cm.seg_part, cm.arrive, mj,
                           (double*)nullptr);
    return hipGetLastError();
}

template hipError_t launch_schur_jacobi_terms<double>(const CameraMajor&, int64_t, const double*,
                                                      JacSource<double>, double, const double*, double*,
                                                      hipStream_t);
template hipError_t launch_schur_jacobi_terms<float>(const CameraMajor&, int64_t, const double*, JacSource<float>,
                                                     double, const float*, double*, hipStream_t);
template hipError_t launch_build_points<double>(const PointMajor&, double, bool, const double*, JacSource<double>,
                                                double*, double*, double*, double*, hipStream_t);
template hipError_t launch_build_points<float>(const PointMajor&, double, bool, const double*, JacSource<float>,
                                               float*, double*, double*, float*, hipStream_t);
template hipError_t launch_build_cameras<double>(const CameraMajor&, int32_t, int64_t, const double*,
                                                 JacSource<double>, double, bool, double*, double*, int64_t,
                                                 double*, double*, hipStream_t);
template hipError_t launch_build_cameras<float>(const CameraMajor&, int32_t, int64_t, const double*,
                                                JacSource<float>, double, bool, double*, double*, int64_t, float*,
                                                float*, hipStream_t);
template hipError_t launch_cost_t<float>(const PointMajor&, int64_t, const double*, const CamK<float>*, double,
                                         double*, int32_t*, hipStream_t);

}  // namespace ba

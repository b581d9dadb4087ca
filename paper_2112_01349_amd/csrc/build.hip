// Residual, Jacobian and Schur block assembly (Alg. 1: residual/Jacobian and
// Hessian/constant-vector steps; Sec. 3 Eq. schur_complement), and the FP64
// cost F = 1/2 sum rho(|e|^2) (Sec. 3 Eq. obj with a Huber loss).
//
// Two passes over the observations, each with its own sorted copy of the
// index and pixel streams:
//   * point-major (k_build_points): one wavefront per point-aligned segment
//     of <= 64 observations, one lane per observation.  Writes the coupling
//     block E_k = w J_c^T J_p (tile-blocked, see eidx) when E is stored, and
//     sums the point blocks C_i = sum w J_p^T J_p and w_i = -sum w J_p^T e
//     over each point's run of lanes by a segmented scan.
//   * camera-major (k_build_cameras): one wavefront per chunk of 32 rows of
//     the camera-sorted stream, each row up to 64 observations of one camera,
//     software-pipelined.  Lanes accumulate the camera terms
//     B_j = sum w J_c^T J_c and v_j = -sum w J_c^T e in registers while the
//     camera does not change and flush a wavefront-reduced partial sum into a
//     slot at the first row of the next; slots of one camera are contiguous
//     and are summed in a fixed order by k_reduce_slots, so the result is
//     deterministic.  This
//     balances the Zipf-skewed camera segments (the most-seen camera holds
//     about 60% of all points) over the whole chip, as the paper's equal-edge
//     partition (Sec. 4.1) does over GPUs.
//   * camera-major again (k_schur_jacobi_cameras), for the Schur-Jacobi
//     preconditioner option: the same slots sum -E_k C~^-1 E_k^T per camera
//     at the damping of the current LM iteration.
#include "ba_internal.h"
#include "autodiff.h"
#include "camera_cache.h"
#include "wave_ops.h"

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

// Point-major build, one wavefront per point-aligned segment.  A short
// segment (up to 64 observations of whole points) has one observation per
// lane: each lane computes its residual and Jacobian, stores its IRLS weight
// and, when E is stored, E_k = w J_c^T J_p (27 coalesced rows); its terms of
// C_i and w_i (FP64) are summed over each point's run of lanes by a
// segmented scan, and the run's last lane stores C_i (upper 6) and w_i.  A
// long segment (one point of more than 64 observations) is walked in rows of
// 64 with per-lane partial sums reduced over the wavefront at the end.  Both
// sums have a fixed order.  GRAD_ONLY forms w_i only; without STORE_E the
// camera half of the Jacobian is never formed.
template <typename T, bool GRAD_ONLY, bool AD, bool STORE_E>
__global__ __launch_bounds__(256) void k_build_points(
    int32_t num_short, const int2* __restrict__ sseg, int32_t num_long, const int2* __restrict__ lseg,
    const int32_t* __restrict__ cam, const int32_t* __restrict__ pt, const double* __restrict__ uvx,
    const double* __restrict__ uvy, const double* __restrict__ pts, JacSource<T> js, T delta,
    T* __restrict__ hcp, double* __restrict__ hpp, double* __restrict__ wpt, T* __restrict__ wobs)
{
    constexpr int R = GRAD_ONLY ? 3 : 9;  // terms kept: [C upper 6 |] w 3
    const int lane = threadIdx.x & 63;
    const int32_t w = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (w < num_short) {
        const int2 be = sseg[w];
        const int32_t b = __builtin_amdgcn_readfirstlane(be.x);
        const int32_t len = __builtin_amdgcn_readfirstlane(be.y) - b;
        const bool valid = lane < len;
        const int64_t k = b + (valid ? lane : 0);
        T e0, e1, wt, Jc[18], Jp[6];
        int32_t i;
        observation<T, AD>(k, cam, pt, uvx, uvy, pts, js, delta, e0, e1, wt, Jc, Jp, i);
        if (!GRAD_ONLY && valid) {
            if (STORE_E) store_coupling_blocked<T>(k, Jc, Jp, wt, hcp);
            wobs[k] = wt;
        }
        double v[9];
        point_terms<T>(Jp, e0, e1, wt, v);
        double a[R];
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] = v[9 - R + q];
        // runs of one point: lane 0 and every lane whose point differs from
        // the lane before start one; lanes past the segment start none and
        // only ever follow the valid ones
        const int32_t prev = lane_before(i, -1);
        const uint64_t heads = __ballot(valid && (lane == 0 || i != prev));
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
        const int seg_s = 63 - __clzll((heads & upto) | 1ull);
        // (a non-finite term spreads to the other points of its segment, whose
        // blocks the solve then rejects as it rejects that point's)
        run_prefix<double, R>(a, lane, seg_s);
        const bool last = valid && (lane == len - 1 || ((heads >> (lane + 1)) & 1ull));
        if (last) {
            if (!GRAD_ONLY)
#pragma unroll
                for (int q = 0; q < 6; ++q) hpp[6 * (int64_t)i + q] = a[q];
#pragma unroll
            for (int q = 0; q < 3; ++q) wpt[3 * (int64_t)i + q] = a[R - 3 + q];
        }
    } else if (w < num_short + num_long) {
        const int2 be = lseg[w - num_short];
        const int32_t s0 = __builtin_amdgcn_readfirstlane(be.x), s1 = __builtin_amdgcn_readfirstlane(be.y);
        const int32_t i = __builtin_amdgcn_readfirstlane(pt[s0]);
        double acc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = 0.0;
        for (int64_t r = s0; r < s1; r += 64) {
            const bool valid = r + lane < s1;
            const int64_t k = valid ? r + lane : r;
            T e0, e1, wt, Jc[18], Jp[6];
            int32_t ii;
            observation<T, AD>(k, cam, pt, uvx, uvy, pts, js, delta, e0, e1, wt, Jc, Jp, ii);
            if (!GRAD_ONLY && valid) {
                if (STORE_E) store_coupling_blocked<T>(k, Jc, Jp, wt, hcp);
                wobs[k] = wt;
            }
            double v[9];
            point_terms<T>(Jp, e0, e1, wt, v);
            if (valid)
#pragma unroll
                for (int q = 0; q < R; ++q) acc[q] += v[9 - R + q];
        }
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = wave_sum(acc[q]);
        if (lane == 0) {
            if (!GRAD_ONLY)
#pragma unroll
                for (int q = 0; q < 6; ++q) hpp[6 * (int64_t)i + q] = acc[q];
#pragma unroll
            for (int q = 0; q < 3; ++q) wpt[3 * (int64_t)i + q] = acc[R - 3 + q];
        }
    }
}

template <typename T, bool G, bool A, bool S>
static void build_points_variant(const PointMajor& pm, const double* pts, JacSource<T> js, T delta, T* hcp,
                                 double* hpp, double* wpt, T* wobs, hipStream_t s)
{
    const int64_t waves = (int64_t)pm.num_short + pm.num_long;
    hipLaunchKernelGGL((k_build_points<T, G, A, S>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s,
                       pm.num_short, pm.sseg, pm.num_long, pm.lseg, pm.cam, pm.pt, pm.uvx, pm.uvy, pts, js, delta,
                       hcp, hpp, wpt, wobs);
}

template <typename T>
hipError_t launch_build_points(const PointMajor& pm, double delta, bool grad_only, const double* pts,
                               JacSource<T> js, T* hcp, double* hpp, double* wpt, T* wobs, hipStream_t s)
{
    if ((int64_t)pm.num_short + pm.num_long <= 0) return hipGetLastError();
    const bool ad = js.cams != nullptr;
    const T d = (T)delta;
    if (grad_only) {
        if (ad) build_points_variant<T, true, true, false>(pm, pts, js, d, nullptr, nullptr, wpt, nullptr, s);
        else build_points_variant<T, true, false, false>(pm, pts, js, d, nullptr, nullptr, wpt, nullptr, s);
    } else if (hcp) {
        if (ad) build_points_variant<T, false, true, true>(pm, pts, js, d, hcp, hpp, wpt, wobs, s);
        else build_points_variant<T, false, false, true>(pm, pts, js, d, hcp, hpp, wpt, wobs, s);
    } else {
        if (ad) build_points_variant<T, false, true, false>(pm, pts, js, d, nullptr, hpp, wpt, wobs, s);
        else build_points_variant<T, false, false, false>(pm, pts, js, d, nullptr, hpp, wpt, wobs, s);
    }
    return hipGetLastError();
}

// ----------------------------------------------------- camera-major build

// Wave exchanges of the slot flush.  swap_add32(lo, hi): lanes 0-31 get
// lo(l) + lo(l + 32), lanes 32-63 get hi(l - 32) + hi(l) (v_permlane32_swap
// trades the upper half of its first operand for the lower half of its
// second); swap_add16 does the same between rows 0|1 and 2|3 of 16 lanes
// (v_permlane16_swap).  xor_step<M>: lanes with bit M clear get lo(l) +
// lo(l ^ M), the others hi(l ^ M) + hi(l).
__device__ __forceinline__ double pair_double(uint32_t lo, uint32_t hi)
{
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double swap_add32(double lo, double hi)
{
    const uint64_t a = (uint64_t)__double_as_longlong(lo), b = (uint64_t)__double_as_longlong(hi);
    const auto x = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
    const auto y = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
    return pair_double(x[0], y[0]) + pair_double(x[1], y[1]);
}

__device__ __forceinline__ double swap_add16(double lo, double hi)
{
    const uint64_t a = (uint64_t)__double_as_longlong(lo), b = (uint64_t)__double_as_longlong(hi);
    const auto x = __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
    const auto y = __builtin_amdgcn_permlane16_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
    return pair_double(x[0], y[0]) + pair_double(x[1], y[1]);
}

template <int M>
__device__ __forceinline__ double xor_step(double lo, double hi, int lane)
{
    const bool up = (lane & M) != 0;
    return (up ? hi : lo) + __shfl_xor(up ? lo : hi, M, 64);
}

// Sums each of the W accumulated words over the wavefront into word q of
// the slot, then clears them.  Recursive halving: at each of the six
// exchanges the lanes with the distance bit clear keep the lower half of the
// words and the others the upper half, adding the partner's copy, so lane q
// ends with word q (words from W on are zero).  63 pair exchanges replace
// six shuffles per word, and the slot is written by one coalesced store.
template <int W>
__device__ __forceinline__ void flush_slot(double* acc, double* __restrict__ slots, int32_t slot, int lane)
{
    static_assert(W <= 64, "one word per lane");
    double v32[32], v16[16], v8[8], v4[4], v2[2];
#pragma unroll
    for (int t = 0; t < 32; ++t) v32[t] = t < W ? swap_add32(acc[t], t + 32 < W ? acc[t + 32] : 0.0) : 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) v16[t] = t < W ? swap_add16(v32[t], v32[t + 16]) : 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t) v8[t] = t < W ? xor_step<8>(v16[t], v16[t + 8], lane) : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) v4[t] = t < W ? xor_step<4>(v8[t], v8[t + 4], lane) : 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) v2[t] = xor_step<2>(v4[t], v4[t + 2], lane);
    const double v = xor_step<1>(v2[0], v2[1], lane);
    if (lane < W) slots[(int64_t)slot * kCamSlotWords + lane] = v;
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0.0;
}

// One row (up to 64 consecutive observations of one camera, one per lane)
// of a camera-major chunk: the streamed words, then what they point at.  The
// chunk's rows are software-pipelined: while row r is computed, the point and
// camera loads of row r + 1 and the streamed words of row r + 2 are in
// flight.  A row holds one camera: its index is wave-uniform.
template <typename T>
struct CmRow {
    int32_t k0, len;    // first observation and length (uniform)
    int32_t j;          // the row's camera (uniform)
    int32_t jv;         // the same, loaded per lane (FP32: the camera gathers stay vector loads)
    int32_t i;          // point (lanes past the row's end: the row's first observation's)
    double u, v;        // pixel
    double X[3];        // point (gathered)
    T hd[kCamHead];     // camera constants R, t, f, k1, k2, small
    T Jl[9];            // camera left Jacobian
};

template <typename T>
__device__ __forceinline__ void cm_stream(const int32_t* __restrict__ rows, int32_t row, int lane,
                                          const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
                                          const double* __restrict__ uvx, const double* __restrict__ uvy,
                                          CmRow<T>& r)
{
    r.k0 = __builtin_amdgcn_readfirstlane(rows[row]);
    r.len = __builtin_amdgcn_readfirstlane(rows[row + 1]) - r.k0;
    const int64_t kk = r.k0 + (lane < r.len ? lane : 0);
    r.j = __builtin_amdgcn_readfirstlane(cam[r.k0]);
    if (sizeof(T) == 4) r.jv = cam[kk];
    r.i = pt[kk];
    r.u = uvx[kk];
    r.v = uvy[kk];
}

template <typename T>
__device__ __forceinline__ void cm_gather(const double* __restrict__ pts, const CamK<T>* __restrict__ ck, CmRow<T>& r)
{
    const double* X = pts + 3 * (int64_t)r.i;
    r.X[0] = X[0];
    r.X[1] = X[1];
    r.X[2] = X[2];
    // FP64: scalar loads of the uniform camera (fewer vector registers: two
    // wavefronts per SIMD); FP32: per-lane loads (the scalar form's 42
    // registers of camera words for two rows overflow the scalar file)
    const int32_t j = sizeof(T) == 8 ? r.j : r.jv;
    const T* c = reinterpret_cast<const T*>(ck + j);
#pragma unroll
    for (int q = 0; q < kCamHead; ++q) r.hd[q] = c[q];
#pragma unroll
    for (int q = 0; q < 9; ++q) r.Jl[q] = ck[j].Jl[q];
}

// Residual, Jacobian and IRLS weight of one gathered observation (the
// analytic form from the constants, or forward-mode differentiation).
template <typename T, bool AD>
__device__ __forceinline__ void cm_observation(const CmRow<T>& r, const double* __restrict__ pts, JacSource<T> js,
                                               T delta, T& e0, T& e1, T& wt, T Jc[18], T Jp[6])
{
    const T X0 = (T)r.X[0], X1 = (T)r.X[1], X2 = (T)r.X[2];
    bool done = false;
    if (AD) {
        residual_jacobian_ad<T>(js.cams + 9 * (int64_t)r.j, X0, X1, X2, (T)r.u, (T)r.v, e0, e1, Jc, Jp);
        // an unresolved FP32 depth: the analytic form from the FP64 geometry
        done = sizeof(T) == 8 || depth_resolved<T>(r.hd[6] * X0 + r.hd[7] * X1 + r.hd[8] * X2, r.hd[11],
                                                   r.hd[6] * X0 + r.hd[7] * X1 + r.hd[8] * X2 + r.hd[11]);
    }
    if (!done) {
        ObsGeo<T> o;
        if (!observation_geometry<T>(r.hd, X0, X1, X2, o) && js.ck64)
            o = observation_geometry_f64<T>(js.ck64, r.j, pts + 3 * (int64_t)r.i);
        jacobian_from_geometry<T>(r.hd, r.Jl, o, (T)r.u, (T)r.v, e0, e1, Jc, Jp);
    }
    wt = huber_weight<T>(e0 * e0 + e1 * e1, delta);
}

// Walks the rows [r0, r1) of one camera-major chunk through the pipeline
// above and calls body(r) for each (uniform over the wave).
template <typename T, class Body>
__device__ __forceinline__ void cm_rows(int32_t r0, int32_t r1, int lane, const int32_t* __restrict__ rows,
                                        const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
                                        const double* __restrict__ uvx, const double* __restrict__ uvy,
                                        const double* __restrict__ pts, const CamK<T>* __restrict__ ck, Body&& body)
{
    CmRow<T> a, b;
    cm_stream<T>(rows, r0, lane, cam, pt, uvx, uvy, a);
    cm_gather<T>(pts, ck, a);
    if (r0 + 1 < r1) cm_stream<T>(rows, r0 + 1, lane, cam, pt, uvx, uvy, b);
    for (int32_t row = r0; row < r1; ++row) {
        const CmRow<T> c = a;
        if (row + 1 < r1) {
            a = b;
            cm_gather<T>(pts, ck, a);
        }
        if (row + 2 < r1) cm_stream<T>(rows, row + 2, lane, cam, pt, uvx, uvy, b);
        body(c);
    }
}

template <typename T, bool GRAD_ONLY, bool AD>
__global__ __launch_bounds__(256) void k_build_cameras(
    int64_t N, int32_t num_rows, const int32_t* __restrict__ rows, const int32_t* __restrict__ cam,
    const int32_t* __restrict__ pt, const double* __restrict__ uvx, const double* __restrict__ uvy,
    const double* __restrict__ pts, JacSource<T> js, T delta, const int32_t* __restrict__ chunk_slot,
    double* __restrict__ slots, int64_t Nc, T* __restrict__ chcp, T* __restrict__ cw)
{
    constexpr int W = GRAD_ONLY ? 9 : kCamSlotWords;
    const int64_t cold0 = N - Nc;  // the cold cameras' observations are the stream's tail
    const int lane = threadIdx.x & 63;
    const int32_t chunk = __builtin_amdgcn_readfirstlane((int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int32_t r0 = chunk * kCmRows;
    if (r0 >= num_rows) return;  // whole wavefront leaves together
    const int32_t r1 = min(r0 + kCmRows, num_rows);
    int32_t slot = chunk_slot[chunk];
    int32_t cur = cam[rows[r0]];
    double acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0.0;
    cm_rows<T>(r0, r1, lane, rows, cam, pt, uvx, uvy, pts, js.ck, [&](const CmRow<T>& r) {
        const int64_t k = (int64_t)r.k0 + lane;
        const bool valid = lane < r.len;
        T e0, e1, wt, Jc[18], Jp[6];
        cm_observation<T, AD>(r, pts, js, delta, e0, e1, wt, Jc, Jp);
        if (!GRAD_ONLY && valid && k >= cold0) {
            if (chcp) store_coupling<T>(k - cold0, Nc, Jc, Jp, wt, chcp);
            if (cw) cw[k - cold0] = wt;
        }
        // a row holds one camera: the previous camera's sums leave at its first row
        if (r.j != cur) {
            flush_slot<W>(acc, slots, slot, lane);
            ++slot;
            cur = r.j;
        }
        if (valid) {
            // FP64 terms: the weighted Jacobian entry w J_c[r][a] (exact for
            // float operands) times J_c[r][b], fused into the accumulator
            const double w = wt, re0 = e0, re1 = e1;
            double jc[18];
#pragma unroll
            for (int a = 0; a < 18; ++a) jc[a] = Jc[a];
            int q = 0;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const double w0 = w * jc[a], w1 = w * jc[9 + a];
                if (!GRAD_ONLY) {
#pragma unroll
                    for (int b = a; b < 9; ++b) {
                        acc[q] = fma(w0, jc[b], fma(w1, jc[9 + b], acc[q]));
                        ++q;
                    }
                }
                acc[W - 9 + a] = fma(-w0, re0, fma(-w1, re1, acc[W - 9 + a]));
            }
        }
    });
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
    hipLaunchKernelGGL((k_build_cameras<T, G, A>), dim3((cm.num_chunks + 3) / 4), dim3(256), 0, s, N, cm.num_rows,
                       cm.row, cm.cam, cm.pt, cm.uvx, cm.uvy, pts, js, delta, cm.chunk_slot, cm.slots, Nc, chcp, cw);
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
// Persistent workgroups of kCostThreads over the point-major stream; the
// camera heads of the most observed cameras are read from an LDS copy.
constexpr int kCostThreads = 1024;
constexpr int kCostCacheCameras = 1024;

template <typename T>
__global__ __launch_bounds__(kCostThreads) void k_cost(int64_t N, const int32_t* __restrict__ cam,
                                                       const int32_t* __restrict__ pt, const double* __restrict__ uvx,
                                                       const double* __restrict__ uvy, const double* __restrict__ pts,
                                                       const CamK<T>* __restrict__ ck, T delta, int32_t Kc,
                                                       double* __restrict__ partials)
{
    constexpr int S = sizeof(CamK<T>) / sizeof(T);
    extern __shared__ __align__(16) unsigned char smem[];
    T* cache = reinterpret_cast<T*>(smem);
    __shared__ double sh[kCostThreads / 64];
    fill_camera_cache<T, kCamHead, S, kCostThreads>(reinterpret_cast<const T*>(ck), Kc, cache);
    __syncthreads();
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kCostThreads + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * kCostThreads) {
        const int32_t j = cam[k], i = pt[k];
        T hd[kCamHead], e0, e1;
        camera_words<T, kCamHead, kCamHead, S>(j, Kc, cache, reinterpret_cast<const T*>(ck), hd);
        residual<T>(hd, (T)pts[3 * (int64_t)i], (T)pts[3 * (int64_t)i + 1], (T)pts[3 * (int64_t)i + 2], (T)uvx[k],
                    (T)uvy[k], e0, e1);
        acc += 0.5 * (double)huber_rho<T>(e0 * e0 + e1 * e1, delta);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kCostThreads / 64; ++w) t += sh[w];
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
    int64_t b = (N + kCostThreads - 1) / kCostThreads;
    if (b > kPersistentBlocks) b = kPersistentBlocks;
    if (b < 1) b = 1;
    *nblocks = (int32_t)b;
    const int32_t Kc = pm.num_cameras < kCostCacheCameras ? pm.num_cameras : kCostCacheCameras;
    hipLaunchKernelGGL((k_cost<T>), dim3((unsigned)b), dim3(kCostThreads), (size_t)Kc * kCamHead * sizeof(T), s, N,
                       pm.cam, pm.pt, pm.uvx, pm.uvy, pts, ck, (T)delta, Kc, partials);
    return hipGetLastError();
}

// Dynamic LDS beyond the default limit for the cost kernels above.
hipError_t prepare_cost_kernels()
{
    hipError_t e = hipFuncSetAttribute((const void*)k_cost<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(kCostCacheCameras * kCamHead * sizeof(double)));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_cost<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kCostCacheCameras * kCamHead * sizeof(float)));
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
    int32_t num_rows, const int32_t* __restrict__ rows, const int32_t* __restrict__ cam,
    const int32_t* __restrict__ pt, const double* __restrict__ uvx, const double* __restrict__ uvy,
    const double* __restrict__ pts, JacSource<T> js, T delta, const T* __restrict__ cinv,
    const int32_t* __restrict__ chunk_slot, double* __restrict__ slots)
{
    constexpr int W = 45;
    const int lane = threadIdx.x & 63;
    const int32_t chunk = __builtin_amdgcn_readfirstlane((int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int32_t r0 = chunk * kCmRows;
    if (r0 >= num_rows) return;  // whole wavefront leaves together
    const int32_t r1 = min(r0 + kCmRows, num_rows);
    int32_t slot = chunk_slot[chunk];
    int32_t cur = cam[rows[r0]];
    double acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0.0;
    cm_rows<T>(r0, r1, lane, rows, cam, pt, uvx, uvy, pts, js.ck, [&](const CmRow<T>& r) {
        const bool valid = lane < r.len;
        T e0, e1, wt, Jc[18], Jp[6];
        cm_observation<T, AD>(r, pts, js, delta, e0, e1, wt, Jc, Jp);
        if (r.j != cur) {
            flush_slot<W>(acc, slots, slot, lane);
            ++slot;
            cur = r.j;
        }
        if (valid) {
            const double w = wt;
            double E[27], Tm[27];
#pragma unroll
            for (int a = 0; a < 9; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    E[a * 3 + c] = w * ((double)Jc[a] * (double)Jp[c] + (double)Jc[9 + a] * (double)Jp[3 + c]);
            const T* c6 = cinv + 6 * (int64_t)r.i;
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
    });
    flush_slot<W>(acc, slots, slot, lane);
}

template <typename T>
hipError_t launch_schur_jacobi_terms(const CameraMajor& cm, int64_t /* N: the rows bound the stream */,
                                     const double* pts, JacSource<T> js, double delta, const T* cinv, double* mj,
                                     hipStream_t s)
{
    if (cm.num_chunks > 0) {
        const dim3 grid((cm.num_chunks + 3) / 4);
        if (js.cams)
            hipLaunchKernelGGL((k_schur_jacobi_cameras<T, true>), grid, dim3(256), 0, s, cm.num_rows, cm.row, cm.cam,
                               cm.pt, cm.uvx, cm.uvy, pts, js, (T)delta, cinv, cm.chunk_slot, cm.slots);
        else
            hipLaunchKernelGGL((k_schur_jacobi_cameras<T, false>), grid, dim3(256), 0, s, cm.num_rows, cm.row, cm.cam,
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

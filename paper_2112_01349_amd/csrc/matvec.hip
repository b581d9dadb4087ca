// Implicit Schur product of Alg. 3 (DSE) with one partition, and the reduced
// right-hand side of Eq. schur_x_c that shares its second half:
//   mode 0:  c = E C~^-1 E^T x,  then q = B~ x - c   (and p^T q)
//   mode 1:  c = E C~^-1 w,      then g = v - c      (r = g, x = 0, ||g||^2)
//
// E is held as one 9x3 block per observation in point-major order, stored
// tile-blocked (the 27 rows of a 64-observation tile are contiguous).  Per point i, a_i = sum_k E_k^T x_j(k) needs all of the
// point's observations before b_i = C~_i^-1 a_i, and then every observation
// adds E_k b_i into its camera.  The camera side is Zipf-skewed (the most
// seen camera is in ~60% of the points), so the scatter is organised by
// camera popularity (cameras are relabelled most-observed first):
//
//   pass 1 (k_schur_hot, or k_schur_rhs for mode 1): persistent
//     workgroups, one per CU; every wavefront streams its own range of
//     line-aligned 64-observation tiles (one observation per lane) with the
//     next tile prefetched into registers.  a_i is summed by a segmented scan
//     over shuffles (a point that runs on into the next tile is finished from
//     the prefetched registers) and b_i is formed in registers; contributions
//     to the K hottest cameras accumulate in a per-workgroup LDS copy of their
//     9-vectors (K sized to fill the LDS), written out once at the
//     end.  b_i of points that also have observations on colder cameras is
//     stored.
//   pass 2 (k_schur_cold): the observations on cameras >= K, from their own
//     camera-major copy of E, gather b_i and are reduced per camera by
//     wavefront chunks into fixed partial-sum slots (no atomics).
//   fold + epilogue (k_hot_fold, k_schur_epilogue): per camera entry, sums
//     the workgroup partials (hot) or the slots (cold) in a fixed order and
//     forms q or g.
//
// That is the stored-block design.  The default product stores no E: its
// point-major pass (k_schur_free) and cold pass (k_schur_cold_free) form
// each block again from the Jacobian's geometry, and the point-major pass
// shares its LDS between the hot table and a copy of the most observed
// cameras' records (camera_cache.h).
#include "ba_internal.h"
#include "camera_cache.h"
#include "wave_ops.h"

namespace ba {

// Observation 64 t + lane of tile t, for t uniform over the wavefront and at
// most the tile count: the point-major arrays end with a padding tile (point
// index -1), so no lane needs a bounds test, and the tile's 27 rows are one
// contiguous run.  The streams are read with non-temporal loads: each byte is
// used once, and keeping them out of the caches leaves L1/L2 to the camera
// vectors, C~^-1 and the flags that are gathered per lane (0.83 -> 0.78 ms per
// pass at 29M observations in FP32).
template <typename T>
__device__ __forceinline__ void load_tile(int64_t t, int lane, const int32_t* __restrict__ cam,
                                          const int32_t* __restrict__ pt, const T* __restrict__ hcp, int32_t& j,
                                          int32_t& i, T h[27])
{
    const int64_t k0 = 64 * t;
    j = __builtin_nontemporal_load(cam + k0 + lane);
    i = __builtin_nontemporal_load(pt + k0 + lane);
    const T* e = hcp + t * (27 * 64) + lane;
#pragma unroll
    for (int q = 0; q < 27; ++q) h[q] = __builtin_nontemporal_load(e + q * 64);
}

template <typename T>
__device__ __forceinline__ void add_hot(double* __restrict__ cl, int32_t j, const T h[27], T b0, T b1, T b2)
{
    double* dst = cl + 9 * j;
#pragma unroll
    for (int a = 0; a < 9; ++a)
        atomicAdd(dst + a, (double)(h[a * 3] * b0 + h[a * 3 + 1] * b1 + h[a * 3 + 2] * b2));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// a = E_k^T x_j for one observation's 9x3 block.
template <typename T>
__device__ __forceinline__ void block_t_times_x(const T h[27], const T* __restrict__ xcam, int32_t j, T& a0, T& a1,
                                                T& a2)
{
    T x[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) x[a] = xcam[9 * (int64_t)j + a];
    a0 = (T)0;
    a1 = (T)0;
    a2 = (T)0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        a0 += h[a * 3] * x[a];
        a1 += h[a * 3 + 1] * x[a];
        a2 += h[a * 3 + 2] * x[a];
    }
}

// Pass 1 of the matvec.  Tile t holds observations [64 t, 64 t + 64), one
// per lane.  A point belongs to the tile that holds its first observation,
// and each wavefront takes the points that start in its range of tiles.
// Per iteration the wave gathers what this tile needs per lane (camera
// vectors, C~^-1, the cold flag), then prefetches the next tile, then
// finishes every point that ends inside this tile.  A wave's loads complete
// in issue order, so only the tile's last point, which may run on into the
// next tile, waits for the prefetch: it is finished from the prefetched
// registers and no block is read twice.  A point that fills the whole next
// tile and goes on (longer than the point lengths of the usual workloads) is
// finished by a second walk over its further tiles.
// The hot-camera table is FP64 in both precisions: LDS FP64 adds issue
// without the back-pressure FP32 LDS adds show here, and the per-workgroup
// sums of the most observed cameras keep FP64 accuracy.
template <typename T>
__global__ __launch_bounds__(HotThreads<T>::value) void k_schur_hot(
    const int32_t* __restrict__ wrange, int64_t N, const int32_t* __restrict__ cam,
    const int32_t* __restrict__ pt, const T* __restrict__ hcp, const T* __restrict__ cinv,
    const T* __restrict__ xcam, int32_t K, double* __restrict__ hot_part, T* __restrict__ bcold,
    const int32_t* __restrict__ crec, const PcgScalars* __restrict__ sc)
{
    constexpr int NT = HotThreads<T>::value;
    if (sc->done) return;  // uniform over the grid
    extern __shared__ __align__(16) unsigned char smem[];
    double* cl = reinterpret_cast<double*>(smem);
    for (int q = threadIdx.x; q < K * 9; q += NT) cl[q] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int32_t gw = __builtin_amdgcn_readfirstlane(blockIdx.x * (NT / 64) + (threadIdx.x >> 6));
    const int64_t T0 = wrange[gw], T1 = wrange[gw + 1];
    const int64_t ntiles = (N + 63) >> 6;
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    if (T0 < T1) {
        int32_t before = T0 > 0 ? pt[64 * T0 - 1] : -1;  // point of the observation just before tile t
        int32_t cj, ci;
        T ch[27];
        load_tile<T>(T0, lane, cam, pt, hcp, cj, ci, ch);
        int64_t t = T0;
        while (t < T1) {
            const int32_t prev = __shfl_up(ci, 1, 64);
            const int32_t last_i = __builtin_amdgcn_readlane(ci, 63);
            const bool valid = ci >= 0;
            const bool head = valid && ci != (lane == 0 ? before : prev);
            const uint64_t hm = __ballot(head);
            const int first_head = hm ? __ffsll((unsigned long long)hm) - 1 : 64;
            const bool owned = valid && lane >= first_head;
            // this tile's gathers first, then the next tile's prefetch: loads complete
            // in issue order, so waiting for these never waits for the prefetch
            T x[9], c6[6];
            const int64_t ii = ci >= 0 ? ci : 0;
#pragma unroll
            for (int a = 0; a < 9; ++a) x[a] = xcam[9 * (int64_t)cj + a];
#pragma unroll
            for (int a = 0; a < 6; ++a) c6[a] = cinv[6 * ii + a];
            const bool hc = crec[ii] >= 0;  // (this design's records are indexed by point)
            __builtin_amdgcn_sched_barrier(0);
            int32_t nj, ni;
            T nh[27];
            load_tile<T>(t + 1, lane, cam, pt, hcp, nj, ni, nh);  // the padding tile when t + 1 = ntiles
            __builtin_amdgcn_sched_barrier(0);
            if (hm != 0) {
                const int last_owned = 63 - __clzll(__ballot(owned));
                const int last_head = 63 - __clzll(hm);
                const int seg_s = 63 - __clzll((hm & upto) | 1ull);
                const uint64_t above = hm & ~upto;
                const int seg_e = above ? __ffsll((unsigned long long)above) - 2 : last_owned;
                const int32_t s_pt = last_owned == 63 ? last_i : -2;  // the last point reaches lane 63
                T a0 = (T)0, a1 = (T)0, a2 = (T)0;
                if (owned) {
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
                const bool strad = owned && s_pt >= 0 && seg_s == last_head;  // the last point's lanes
                // the points that end inside this tile
                if (owned && !strad) {
                    const T b0 = c6[0] * a0 + c6[1] * a1 + c6[2] * a2;
                    const T b1 = c6[1] * a0 + c6[3] * a1 + c6[4] * a2;
                    const T b2 = c6[2] * a0 + c6[4] * a1 + c6[5] * a2;
                    if (lane == seg_e && hc) {
                        bcold[kBcold * ii] = b0;
                        bcold[kBcold * ii + 1] = b1;
                        bcold[kBcold * ii + 2] = b2;
                    }
                    if (cj < K) add_hot<T>(cl, cj, ch, b0, b1, b2);
                }
                if (s_pt >= 0) {
                    // the last point, which may run on into the next tile: this is
                    // where the wave waits for the prefetched tile
                    const bool cn = ni == s_pt;  // a prefix of the next tile
                    const uint64_t cm = __ballot(cn);
                    T c0 = (T)0, c1 = (T)0, c2 = (T)0;
                    if (cm != 0) {
                        if (cn) block_t_times_x<T>(nh, xcam, nj, c0, c1, c2);
                        c0 = wave_sum(c0);
                        c1 = wave_sum(c1);
                        c2 = wave_sum(c2);
                    }
                    a0 += c0;
                    a1 += c1;
                    a2 += c2;
                    if (cm == ~0ull && t + 2 < ntiles && pt[64 * (t + 2)] == s_pt) {
                        // it fills the next tile and goes on: add its further tiles,
                        // then walk all of its tiles again for the camera side
                        T p0 = __shfl(a0, 63, 64), p1 = __shfl(a1, 63, 64), p2 = __shfl(a2, 63, 64);
                        int64_t u = t + 2;
                        while (true) {
                            int32_t j, i;
                            T h[27];
                            load_tile<T>(u, lane, cam, pt, hcp, j, i, h);
                            const bool in = i == s_pt;
                            T d0 = (T)0, d1 = (T)0, d2 = (T)0;
                            if (in) block_t_times_x<T>(h, xcam, j, d0, d1, d2);
                            p0 += wave_sum(d0);
                            p1 += wave_sum(d1);
                            p2 += wave_sum(d2);
                            if (__ballot(in) != ~0ull || u + 1 >= ntiles || pt[64 * (u + 1)] != s_pt) break;
                            ++u;
                        }
                        const T* q6 = cinv + 6 * (int64_t)s_pt;
                        const T s0 = q6[0] * p0 + q6[1] * p1 + q6[2] * p2;
                        const T s1 = q6[1] * p0 + q6[3] * p1 + q6[4] * p2;
                        const T s2 = q6[2] * p0 + q6[4] * p1 + q6[5] * p2;
                        if (lane == 0 && crec[s_pt] >= 0) {
                            bcold[kBcold * (int64_t)s_pt] = s0;
                            bcold[kBcold * (int64_t)s_pt + 1] = s1;
                            bcold[kBcold * (int64_t)s_pt + 2] = s2;
                        }
                        if (K > 0)  // with no hot camera the cold pass does the camera side
                            for (int64_t v = t; v <= u; ++v) {
                                int32_t j, i;
                                T h[27];
                                load_tile<T>(v, lane, cam, pt, hcp, j, i, h);
                                if (i == s_pt && j < K) add_hot<T>(cl, j, h, s0, s1, s2);
                            }
                        // tiles t + 1 .. u - 1 hold only this point; go on at tile u
                        before = s_pt;
                        t = u;
                        if (t < T1) load_tile<T>(t, lane, cam, pt, hcp, cj, ci, ch);
                        continue;
                    }
                    T b0 = (T)0, b1 = (T)0, b2 = (T)0;
                    if (strad) {
                        b0 = c6[0] * a0 + c6[1] * a1 + c6[2] * a2;
                        b1 = c6[1] * a0 + c6[3] * a1 + c6[4] * a2;
                        b2 = c6[2] * a0 + c6[4] * a1 + c6[5] * a2;
                        if (lane == 63 && hc) {
                            bcold[kBcold * ii] = b0;
                            bcold[kBcold * ii + 1] = b1;
                            bcold[kBcold * ii + 2] = b2;
                        }
                        if (cj < K) add_hot<T>(cl, cj, ch, b0, b1, b2);
                    }
                    if (cm != 0) {
                        const T s0 = __shfl(b0, 63, 64), s1 = __shfl(b1, 63, 64), s2 = __shfl(b2, 63, 64);
                        if (cn && nj < K) add_hot<T>(cl, nj, nh, s0, s1, s2);
                    }
                }
            }
            before = last_i;
            cj = nj;
            ci = ni;
#pragma unroll
            for (int q = 0; q < 27; ++q) ch[q] = nh[q];
            ++t;
        }
    }
    __syncthreads();
    double* out = hot_part + (int64_t)blockIdx.x * K * 9;
    for (int q = threadIdx.x; q < K * 9; q += NT) out[q] = cl[q];
}

// ------------------------------------------------- product without stored E
// The coupling block of an observation factors as E_k = w J_c^T J_p, and its
// Jacobian costs ~100 arithmetic operations to form again from the camera
// constants and the point, against 108 bytes (FP32) of HBM to read it.  In
// terms of observation_geometry's D = de/dP, p and lever arm a:
//   J_c x  = D (x_t + u x a) + p (d x_f + f|p|^2 x_k1 + f|p|^4 x_k2),
//            u = J_l x_w (per camera, in xf);
//   J_p^T z = R^T (D^T z);
//   J_p b  = D (R b);
//   J_c^T y = [J_l^T (a x g), g, d p.y, f|p|^2 p.y, f|p|^4 p.y],  g = D^T y.
// So E_k^T x = J_p^T (w J_c x) and E_k b = J_c^T (w J_p b); the J_l^T of the
// camera side is applied once per hot camera when the table is written out.

// Slice f of the fold of the per-workgroup hot partials [G][K*9]: the sum of a
// contiguous range of workgroups, in order, for entry t.
__device__ __forceinline__ void fold_slice(int32_t t, int32_t f, int32_t K9, int32_t G,
                                           const double* __restrict__ hot_part, double* __restrict__ fold)
{
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

template <typename T>
__device__ __forceinline__ void load_head(const CamK<T>* __restrict__ ck, int32_t j, T hd[kCamHead])
{
    const T* src = reinterpret_cast<const T*>(ck + j);
#pragma unroll
    for (int q = 0; q < kCamHead; ++q) hd[q] = src[q];
}

// Element `e` of an array at a 32-bit byte offset from a wave-uniform base:
// the load takes the base in scalar registers and one 32-bit vector offset,
// with no 64-bit address arithmetic per lane.  Offsets stay below 4 GB: a
// camera record times the camera count (checked when the problem is made),
// or the records of the points inside one segment.
template <typename E>
__device__ __forceinline__ const E* at_bytes(const void* base, uint32_t off)
{
    return reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + off);
}

// The camera record the product reads per observation, kept in LDS for the
// hot cameras (camera_cache.h): the first kCamHead words of CamK (R, t, f,
// k1, k2, small) and the camera's direction record from
// launch_pcg_direction (12 words, 9 used).

// Camera j's head and (XV) direction words: from the workgroup's LDS copy
// when j < Kc, else from memory.  The LDS reads are issued first: both
// branches fill the same registers, so the memory loads of the other lanes
// wait only for those short reads, never the reverse.
template <typename T, bool XV>
__device__ __forceinline__ void camera_inputs(int32_t j, int32_t Kc, const T* cache, const CamK<T>* __restrict__ ck,
                                              const T* __restrict__ xf, T hd[kCamHead], T xv[9])
{
    if (j < Kc) {
        const T* c = cache + kCamRec * j;
        load_words16<T, kCamHead>(c, hd);
        if (XV) load_words16<T, 9>(c + kCamHead, xv);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (j >= Kc) {
        const uint32_t uj = (uint32_t)j;
        load_words16<T, kCamHead>(at_bytes<T>(ck, uj * (uint32_t)sizeof(CamK<T>)), hd);
        if (XV) load_words16<T, 9>(at_bytes<T>(xf, uj * (uint32_t)(12 * sizeof(T))), xv);
    }
}

// E_k^T x for one observation (3 values in the point's frame).
template <typename T>
__device__ __forceinline__ void free_et_x(const ObsGeo<T>& o, const T hd[kCamHead], const T xv[9], T w, T& e0,
                                          T& e1, T& e2)
{
    const T v0 = xv[3] + (xv[1] * o.a2 - xv[2] * o.a1);
    const T v1 = xv[4] + (xv[2] * o.a0 - xv[0] * o.a2);
    const T v2 = xv[5] + (xv[0] * o.a1 - xv[1] * o.a0);
    const T sc = o.d * xv[6] + o.fr2 * xv[7] + o.fr4 * xv[8];
    const T z0 = w * (o.D[0] * v0 + o.D[1] * v1 + o.D[2] * v2 + o.px * sc);
    const T z1 = w * (o.D[3] * v0 + o.D[4] * v1 + o.D[5] * v2 + o.py * sc);
    const T h0 = o.D[0] * z0 + o.D[3] * z1, h1 = o.D[1] * z0 + o.D[4] * z1, h2 = o.D[2] * z0 + o.D[5] * z1;
    e0 = hd[0] * h0 + hd[3] * h1 + hd[6] * h2;
    e1 = hd[1] * h0 + hd[4] * h1 + hd[7] * h2;
    e2 = hd[2] * h0 + hd[5] * h1 + hd[8] * h2;
}

// Camera side of E_k b for one observation, before J_l^T.
template <typename T>
__device__ __forceinline__ void free_camera_side(const ObsGeo<T>& o, const T hd[kCamHead], T w, T b0, T b1, T b2,
                                                 T c[9])
{
    const T r0 = hd[0] * b0 + hd[1] * b1 + hd[2] * b2;
    const T r1 = hd[3] * b0 + hd[4] * b1 + hd[5] * b2;
    const T r2 = hd[6] * b0 + hd[7] * b1 + hd[8] * b2;
    const T y0 = w * (o.D[0] * r0 + o.D[1] * r1 + o.D[2] * r2);
    const T y1 = w * (o.D[3] * r0 + o.D[4] * r1 + o.D[5] * r2);
    const T g0 = o.D[0] * y0 + o.D[3] * y1, g1 = o.D[1] * y0 + o.D[4] * y1, g2 = o.D[2] * y0 + o.D[5] * y1;
    const T pyv = o.px * y0 + o.py * y1;
    c[0] = o.a1 * g2 - o.a2 * g1;
    c[1] = o.a2 * g0 - o.a0 * g2;
    c[2] = o.a0 * g1 - o.a1 * g0;
    c[3] = g0;
    c[4] = g1;
    c[5] = g2;
    c[6] = o.d * pyv;
    c[7] = o.fr2 * pyv;
    c[8] = o.fr4 * pyv;
}

// ... added to the workgroup's FP64 table of hot cameras.
template <typename T>
__device__ __forceinline__ void free_add_hot(double* __restrict__ cl, int32_t j, const ObsGeo<T>& o,
                                             const T hd[kCamHead], T w, T b0, T b1, T b2)
{
    T c[9];
    free_camera_side<T>(o, hd, w, b0, b1, b2, c);
    double* dst = cl + 9 * j;
#pragma unroll
    for (int a = 0; a < 9; ++a) atomicAdd(dst + a, (double)c[a]);
}

// Everything one observation needs: its camera's constants and vector, its
// point and its weight.
template <typename T, bool XV>
__device__ __forceinline__ void free_observation(int64_t k, const int32_t* __restrict__ cam,
                                                 const int32_t* __restrict__ pt, const T* __restrict__ wobs,
                                                 const double* __restrict__ pts, const CamK<T>* __restrict__ ck,
                                                 const CamK<double>* __restrict__ ck64, const T* __restrict__ xf,
                                                 int32_t Kc, const T* cache, int32_t& j, int32_t& i, T& w,
                                                 T hd[kCamHead], T xv[9], ObsGeo<T>& o)
{
    j = cam[k];
    i = pt[k];
    w = wobs[k];
    camera_inputs<T, XV>(j, Kc, cache, ck, xf, hd, xv);
    observation_geometry_checked<T>(hd, ck64, j, pts + 3 * (int64_t)i, o);
}

// A short segment in flight: its streamed indices and weight (stage 1), then
// what they point at (stage 2).
template <typename T>
struct FreeRow {
    int32_t b, len;  // segment start and length (uniform)
    int32_t i0;      // point of the segment's first observation (uniform)
    int32_t j, i;
    T w;
};


template <typename T>
struct FreeData {
    T hd[kCamHead];
    T xv[9];   // modes 0 and 2
    T X[3];
    T c6[6];
    T wv[3];   // w_i, modes 1 and 2
    int32_t rec;  // the point's cold-pass record or -1 (modes 0 and 1)
};

template <typename T>
__device__ __forceinline__ void free_stream(const int2* __restrict__ sseg, int32_t q, int lane,
                                            const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
                                            const T* __restrict__ wobs, FreeRow<T>& r)
{
    const int2 be = sseg[q];
    r.b = __builtin_amdgcn_readfirstlane(be.x);
    r.len = __builtin_amdgcn_readfirstlane(be.y) - r.b;
    const uint32_t l = (uint32_t)(lane < r.len ? lane : 0);
    r.j = (cam + r.b)[l];
    r.i = (pt + r.b)[l];
    r.w = (wobs + r.b)[l];
    r.i0 = __builtin_amdgcn_readfirstlane(r.i);  // lane 0 always holds an observation
}

template <typename T, int MODE>
__device__ __forceinline__ void free_gather(const FreeRow<T>& r, const double* __restrict__ pts,
                                            const CamK<T>* __restrict__ ck, const T* __restrict__ xf,
                                            int32_t Kc, const T* cache, const T* __restrict__ cinv,
                                            const int32_t* __restrict__ crec, const double* __restrict__ wpt,
                                            FreeData<T>& d)
{
    const uint32_t di = (uint32_t)(r.i - r.i0);
    camera_inputs<T, MODE != 1>(r.j, Kc, cache, ck, xf, d.hd, d.xv);
    const int64_t i0 = r.i0;
    const double* X = at_bytes<double>(pts + 3 * i0, di * 24u);
#pragma unroll
    for (int a = 0; a < 3; ++a) d.X[a] = (T)X[a];
    const T* c6 = at_bytes<T>(cinv + 6 * i0, di * (uint32_t)(6 * sizeof(T)));
#pragma unroll
    for (int a = 0; a < 6; ++a) d.c6[a] = c6[a];
    if (MODE != 0) {
        const double* wv = at_bytes<double>(wpt + 3 * i0, di * 24u);
#pragma unroll
        for (int a = 0; a < 3; ++a) d.wv[a] = (T)wv[a];
    }
    if (MODE != 2) d.rec = *at_bytes<int32_t>(crec + i0, di * 4u);
}

// One short segment.  Mode 0 (product): E^T x per lane, a_i per point run
// by a segmented scan, b_i = C~_i^-1 a_i, then the camera side of the hot
// cameras.  Mode 1 (reduced right-hand side): b_i = C~_i^-1 w_i and the
// camera side.  Mode 2 (back-substitution): a_i as in mode 0, then
// dp_i = C~_i^-1 (w_i - a_i).
template <typename T, int MODE>
__device__ __forceinline__ void free_short(const FreeRow<T>& r, const FreeData<T>& d, int lane,
                                           int32_t K, double* __restrict__ cl, T* __restrict__ bcold,
                                           double* __restrict__ dp, const double* __restrict__ pts,
                                           const CamK<double>* __restrict__ ck64)
{
    const bool valid = lane < r.len;
    ObsGeo<T> o;
    if (!observation_geometry<T>(d.hd, d.X[0], d.X[1], d.X[2], o) && ck64)
        o = observation_geometry_f64<T>(ck64, r.j, pts + 3 * (int64_t)r.i);
    T a0, a1, a2;
    int seg_e = lane;
    if (MODE == 1) {
        a0 = d.wv[0];
        a1 = d.wv[1];
        a2 = d.wv[2];
        const int32_t next = __shfl_down(r.i, 1, 64);
        seg_e = (lane == r.len - 1 || r.i != next) ? lane : -1;  // the last lane of each point run
    } else {
        free_et_x<T>(o, d.hd, d.xv, r.w, a0, a1, a2);
        if (!valid) a0 = a1 = a2 = (T)0;
        const int32_t prev = lane_before(r.i, -1);
        const bool head = valid && (lane == 0 || r.i != prev);
        const uint64_t hm = __ballot(head);
        // the run's first lane: the highest head at or below this lane (lane
        // 0 is always one); its last: the lane before the next head above
        const int seg_s = lane - __clzll((hm | 1ull) << (63 - lane));
        const uint64_t above = lane < 63 ? hm >> (lane + 1) : 0ull;
        seg_e = above ? __ffsll((unsigned long long)above) + lane - 1 : r.len - 1;
        run_prefix3<T>(a0, a1, a2, lane, seg_s);
        a0 = __shfl(a0, seg_e, 64);
        a1 = __shfl(a1, seg_e, 64);
        a2 = __shfl(a2, seg_e, 64);
        if (MODE == 2) {
            a0 = d.wv[0] - a0;
            a1 = d.wv[1] - a1;
            a2 = d.wv[2] - a2;
        }
    }
    // formed on every lane, so the gathered C~^-1 is not sunk into a branch
    // (a load there would be waited for on its own)
    const T b0 = d.c6[0] * a0 + d.c6[1] * a1 + d.c6[2] * a2;
    const T b1 = d.c6[1] * a0 + d.c6[3] * a1 + d.c6[4] * a2;
    const T b2 = d.c6[2] * a0 + d.c6[4] * a1 + d.c6[5] * a2;
    const uint32_t di = (uint32_t)(r.i - r.i0);
    if (MODE == 2) {
        if (valid && lane == seg_e) {
            double* o = const_cast<double*>(at_bytes<double>(dp + 3 * (int64_t)r.i0, di * 24u));
            o[0] = (double)b0;
            o[1] = (double)b1;
            o[2] = (double)b2;
        }
        return;
    }
    if (valid && lane == seg_e && d.rec >= 0) {
        T* o = bcold + kBcold * (int64_t)d.rec;
        o[0] = b0;
        o[1] = b1;
        o[2] = b2;
    }
    if (valid && r.j < K) free_add_hot<T>(cl, r.j, o, d.hd, r.w, b0, b1, b2);
}

// A unit of the workgroup's shared work list for the calling wavefront
// (wave-uniform; every lane must be active).
__device__ __forceinline__ int32_t grab_unit(int32_t* counter, int lane)
{
    int32_t v = 0;
    if (lane == 0) v = atomicAdd(counter, 1);
    return __builtin_amdgcn_readfirstlane(v);
}

// The point-major pass without stored blocks, in the three modes of
// free_short (0: product, 1: reduced right-hand side, 2: back-substitution).
// Work units are point-aligned segments: short ones (up to 64 observations of
// whole points, one per lane) and long ones (one point of more than 64
// observations, in rows of 64, walked a second time for its camera side);
// each workgroup has a range of each kind, which its wavefronts share.  Hot
// cameras accumulate in the workgroup's LDS table as in k_schur_hot; b_i of
// points with cold observations goes into their cold-pass records
// (k_schur_cold_free).  Mode 2 has no camera side (K = 0).  Every mode keeps
// an LDS copy of the camera records of cameras [0, Kc) (kCamRec words each,
// after the hot table), so all three run one workgroup per CU.
template <typename T, int MODE>
struct FreeThreads {
    static constexpr int value = FreeWgThreads<T>::value;
};

// Bytes of the hot table (K cameras, FP64), rounded to 16 for the records
// after it.
__host__ __device__ __forceinline__ size_t free_table_bytes(int32_t K)
{
    return ((size_t)K * 9 * sizeof(double) + 15) & ~(size_t)15;
}

template <typename T, int MODE>
__global__ __launch_bounds__((FreeThreads<T, MODE>::value)) void k_schur_free(
    const int32_t* __restrict__ frange, const int2* __restrict__ sseg, const int32_t* __restrict__ lrange,
    const int2* __restrict__ lseg, const int32_t* __restrict__ cam, const int32_t* __restrict__ pt,
    const T* __restrict__ wobs, const double* __restrict__ pts, const CamK<T>* __restrict__ ck,
    const CamK<double>* __restrict__ ck64, const T* __restrict__ xf, const T* __restrict__ cinv,
    const double* __restrict__ wpt, int32_t K, int32_t Kc, double* __restrict__ hot_part, T* __restrict__ bcold,
    const int32_t* __restrict__ crec, double* __restrict__ dp, const PcgScalars* __restrict__ sc)
{
    constexpr int NT = FreeThreads<T, MODE>::value;
    if (MODE == 0 && sc->done) return;  // uniform over the grid
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t next_unit[2];  // next short batch, next long segment of the workgroup
    double* cl = reinterpret_cast<double*>(smem);
    for (int q = threadIdx.x; q < K * 9; q += NT) cl[q] = 0.0;
    // the hot cameras' records, 16 bytes per thread and step (the right-hand
    // side reads no direction words)
    T* cache = reinterpret_cast<T*>(smem + free_table_bytes(K));
    {
        constexpr int RC = kCamRec * (int)sizeof(T) / 16, HC = kCamHead * (int)sizeof(T) / 16;
        uint4* dst = reinterpret_cast<uint4*>(cache);
        for (int q = threadIdx.x; q < Kc * RC; q += NT) {
            const int32_t j = q / RC, c = q - j * RC;
            if (c < HC) dst[q] = reinterpret_cast<const uint4*>(ck + j)[c];
            else if (MODE != 1) dst[q] = reinterpret_cast<const uint4*>(xf + 12 * (int64_t)j)[c - HC];
        }
    }
    if (threadIdx.x == 0) {
        next_unit[0] = 0;
        next_unit[1] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    // The workgroup's segments (the host's split over its wavefronts, taken
    // together) are handed out to its wavefronts one unit at a time from LDS
    // counters: the SIMDs issue their oldest wavefront first, so equal static
    // shares ended 270 us (first of four per SIMD) to 370 us (last) into a
    // 29M-observation pass, the last ones at low occupancy.  Long segments
    // (the largest units) go first.
    constexpr int WPG = NT / 64;
    const int32_t wg = blockIdx.x;
    {
        const int32_t L0 = lrange[wg * WPG], L1 = lrange[(wg + 1) * WPG];
        for (int32_t q = L0 + grab_unit(&next_unit[1], lane); q < L1; q = L0 + grab_unit(&next_unit[1], lane)) {
            const int2 be = lseg[q];
            const int32_t s0 = __builtin_amdgcn_readfirstlane(be.x), s1 = __builtin_amdgcn_readfirstlane(be.y);
            const int32_t i = __builtin_amdgcn_readfirstlane(pt[s0]);
            T s_0 = (T)0, s_1 = (T)0, s_2 = (T)0;
            if (MODE != 1)
                for (int32_t r = s0; r < s1; r += 64) {
                    const bool valid = r + lane < s1;
                    const int64_t k = valid ? r + lane : r;
                    int32_t j, ii;
                    T w, hd[kCamHead], xv[9];
                    ObsGeo<T> o;
                    free_observation<T, MODE != 1>(k, cam, pt, wobs, pts, ck, ck64, xf, Kc, cache, j, ii, w, hd, xv, o);
                    T e0, e1, e2;
                    free_et_x<T>(o, hd, xv, w, e0, e1, e2);
                    if (!valid) e0 = e1 = e2 = (T)0;
                    s_0 += wave_sum(e0);
                    s_1 += wave_sum(e1);
                    s_2 += wave_sum(e2);
                }
            if (MODE != 0) {
                const T w0 = (T)wpt[3 * (int64_t)i], w1 = (T)wpt[3 * (int64_t)i + 1], w2 = (T)wpt[3 * (int64_t)i + 2];
                s_0 = MODE == 1 ? w0 : w0 - s_0;
                s_1 = MODE == 1 ? w1 : w1 - s_1;
                s_2 = MODE == 1 ? w2 : w2 - s_2;
            }
            const T* c6 = cinv + 6 * (int64_t)i;
            const T b0 = c6[0] * s_0 + c6[1] * s_1 + c6[2] * s_2;
            const T b1 = c6[1] * s_0 + c6[3] * s_1 + c6[4] * s_2;
            const T b2 = c6[2] * s_0 + c6[4] * s_1 + c6[5] * s_2;
            if (MODE == 2) {
                if (lane == 0) {
                    dp[3 * (int64_t)i] = (double)b0;
                    dp[3 * (int64_t)i + 1] = (double)b1;
                    dp[3 * (int64_t)i + 2] = (double)b2;
                }
                continue;
            }
            const int32_t rec = crec[i];
            if (lane == 0 && rec >= 0) {
                bcold[kBcold * (int64_t)rec] = b0;
                bcold[kBcold * (int64_t)rec + 1] = b1;
                bcold[kBcold * (int64_t)rec + 2] = b2;
            }
            if (K > 0)
                for (int32_t r = s0; r < s1; r += 64) {
                    const bool valid = r + lane < s1;
                    const int64_t k = valid ? r + lane : r;
                    int32_t j, ii;
                    T w, hd[kCamHead], xv[9];
                    ObsGeo<T> o;
                    free_observation<T, MODE != 1>(k, cam, pt, wobs, pts, ck, ck64, xf, Kc, cache, j, ii, w, hd, xv, o);
                    if (valid && j < K) free_add_hot<T>(cl, j, o, hd, w, b0, b1, b2);
                }
        }
    }
    {
        // Batches of NB short segments: the loads of all of them are issued
        // before any is computed; the next batch is claimed before this one
        // is computed.  (FP64 and the back-substitution take one at a time,
        // to stay within the registers of sixteen wavefronts per CU)
        constexpr int NB = MODE == 2 || sizeof(T) == 8 ? 1 : 2;  // three spill in FP32
        const int32_t S0 = frange[wg * WPG], S1 = frange[(wg + 1) * WPG];
        const int32_t nbat = (S1 - S0) / NB;
        int32_t bt = grab_unit(&next_unit[0], lane);
        while (bt < nbat) {
            const int32_t next = grab_unit(&next_unit[0], lane);
            FreeRow<T> r[NB];
            FreeData<T> d[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) free_stream<T>(sseg, S0 + NB * bt + u, lane, cam, pt, wobs, r[u]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < NB; ++u) free_gather<T, MODE>(r[u], pts, ck, xf, Kc, cache, cinv, crec, wpt, d[u]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < NB; ++u) free_short<T, MODE>(r[u], d[u], lane, K, cl, bcold, dp, pts, ck64);
            bt = next;
        }
        // the segments past the last whole batch go to the wavefront that claims batch nbat
        if (bt == nbat)
            for (int32_t q = S0 + NB * nbat; q < S1; ++q) {
                FreeRow<T> r;
                FreeData<T> d;
                free_stream<T>(sseg, q, lane, cam, pt, wobs, r);
                free_gather<T, MODE>(r, pts, ck, xf, Kc, cache, cinv, crec, wpt, d);
                free_short<T, MODE>(r, d, lane, K, cl, bcold, dp, pts, ck64);
            }
    }
    __syncthreads();
    // out: the table with J_l^T applied to each camera's rotation part
    double* out = hot_part + (int64_t)blockIdx.x * K * 9;
    for (int q = threadIdx.x; q < K * 9; q += NT) {
        const int32_t j = q / 9;
        const int a = q - 9 * j;
        double v = cl[q];
        if (a < 3) {
            const T* J = ck[j].Jl;
            const double* g = cl + 9 * j;
            v = (double)J[a] * g[0] + (double)J[3 + a] * g[1] + (double)J[6 + a] * g[2];
        }
        out[q] = v;
    }
}

// Point-major pass of the reduced right-hand side: every observation adds
// E_k C~_i^-1 w_i into its camera (hot cameras into the LDS table), and the
// first lane of each point run in a tile stores b_i for the cold pass (runs
// of one point in several tiles store the same value).  Observations are
// independent here, so the tiles need no ownership rule.
template <typename T>
__global__ __launch_bounds__(HotThreads<T>::value) void k_schur_rhs(
    const int32_t* __restrict__ wrange, int64_t N, const int32_t* __restrict__ cam,
    const int32_t* __restrict__ pt, const T* __restrict__ hcp, const T* __restrict__ cinv,
    const double* __restrict__ wpt, int32_t K, double* __restrict__ hot_part, T* __restrict__ bcold,
    const int32_t* __restrict__ crec)
{
    constexpr int NT = HotThreads<T>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    double* cl = reinterpret_cast<double*>(smem);
    for (int q = threadIdx.x; q < K * 9; q += NT) cl[q] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int32_t gw = __builtin_amdgcn_readfirstlane(blockIdx.x * (NT / 64) + (threadIdx.x >> 6));
    const int64_t T0 = wrange[gw], T1 = wrange[gw + 1];
    for (int64_t t = T0; t < T1; ++t) {
        int32_t j, i;
        T h[27];
        load_tile<T>(t, lane, cam, pt, hcp, j, i, h);
        const int32_t prev = __shfl_up(i, 1, 64);
        if (i >= 0) {
            const T* c6 = cinv + 6 * (int64_t)i;
            const T w0 = (T)wpt[3 * (int64_t)i], w1 = (T)wpt[3 * (int64_t)i + 1], w2 = (T)wpt[3 * (int64_t)i + 2];
            const T b0 = c6[0] * w0 + c6[1] * w1 + c6[2] * w2;
            const T b1 = c6[1] * w0 + c6[3] * w1 + c6[4] * w2;
            const T b2 = c6[2] * w0 + c6[4] * w1 + c6[5] * w2;
            if ((lane == 0 || prev != i) && crec[i] >= 0) {
                bcold[kBcold * (int64_t)i] = b0;
                bcold[kBcold * (int64_t)i + 1] = b1;
                bcold[kBcold * (int64_t)i + 2] = b2;
            }
            if (j < K) add_hot<T>(cl, j, h, b0, b1, b2);
        }
    }
    __syncthreads();
    double* out = hot_part + (int64_t)blockIdx.x * K * 9;
    for (int q = threadIdx.x; q < K * 9; q += NT) out[q] = cl[q];
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
            const T b0 = bcold[kBcold * (int64_t)i], b1 = bcold[kBcold * (int64_t)i + 1], b2 = bcold[kBcold * (int64_t)i + 2];
#pragma unroll
            for (int a = 0; a < 9; ++a)
                c[a] = __builtin_nontemporal_load(chcp + (int64_t)(a * 3) * Nc + k) * b0 +
                       __builtin_nontemporal_load(chcp + (int64_t)(a * 3 + 1) * Nc + k) * b1 +
                       __builtin_nontemporal_load(chcp + (int64_t)(a * 3 + 2) * Nc + k) * b2;
        }
        while (true) {
            if (valid && j == cur)
#pragma unroll
                for (int a = 0; a < 9; ++a) acc[a] += (double)c[a];
            const uint64_t more = __ballot(valid && j > cur);
            if (more == 0) break;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const double v = wave_sum(acc[a]);
                if (lane == 0) slots[(int64_t)slot * 9 + a] = v;
                acc[a] = 0.0;
            }
            ++slot;
            cur = __shfl(j, __ffsll((unsigned long long)more) - 1, 64);
        }
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double v = wave_sum(acc[a]);
        if (lane == 0) slots[(int64_t)slot * 9 + a] = v;
    }
}

// Cold observations without stored blocks: as k_schur_cold, with E_k b
// formed from the camera constants, the point and the observation's weight
// (cw, in cold-stream order).  The camera is uniform over a slot, so J_l^T of
// the rotation part is applied once per slot.
template <typename T>
__global__ __launch_bounds__(256) void k_schur_cold_free(int64_t Nc, int32_t num_chunks,
                                                         const int32_t* __restrict__ ccam,
                                                         const int32_t* __restrict__ cpt, const T* __restrict__ cw,
                                                         const double* __restrict__ pts,
                                                         const CamK<T>* __restrict__ ck,
                                                         const CamK<double>* __restrict__ ck64,
                                                         const T* __restrict__ bcold,
                                                         const int32_t* __restrict__ rec_pt,
                                                         const int32_t* __restrict__ chunk_slot,
                                                         double* __restrict__ slots, const PcgScalars* __restrict__ sc,
                                                         int skip_if_done, int32_t cold_blocks, int32_t K9,
                                                         int32_t G, const double* __restrict__ hot_part,
                                                         double* __restrict__ hot_fold)
{
    if (skip_if_done && sc->done) return;
    if ((int32_t)blockIdx.x >= cold_blocks) {  // trailing blocks fold the hot partials meanwhile
        const int32_t fx = (K9 + 255) / 256;
        const int32_t fb = (int32_t)blockIdx.x - cold_blocks;
        const int32_t f = fb / fx;
        fold_slice((fb - f * fx) * 256 + (int32_t)threadIdx.x, f, K9, G, hot_part, hot_fold);
        return;
    }
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
    auto flush = [&](int32_t camj) {
        double v[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            v[a] = wave_sum(acc[a]);
            acc[a] = 0.0;
        }
        if (lane == 0) {
            const T* J = ck[camj].Jl;
            double* o = slots + (int64_t)slot * 9;
#pragma unroll
            for (int a = 0; a < 3; ++a) o[a] = (double)J[a] * v[0] + (double)J[3 + a] * v[1] + (double)J[6 + a] * v[2];
#pragma unroll
            for (int a = 3; a < 9; ++a) o[a] = v[a];
        }
    };
    // rows two at a time: both rows' loads are issued before either is used
    for (int row = 0; row < kColdRows; row += 2) {
        if (start + (int64_t)row * 64 >= end) break;
        int32_t j[2], i[2];
        T w[2], hd[2][kCamHead], X[2][3], b[2][3];
        bool valid[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t k = start + (int64_t)(row + u) * 64 + lane;
            valid[u] = k < end;
            const int64_t kk = valid[u] ? k : start;
            j[u] = ccam[kk];
            i[u] = cpt[kk];
            w[u] = cw[kk];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            load_head<T>(ck, j[u], hd[u]);
            const T* bp = bcold + kBcold * (int64_t)i[u];  // b_i and the point: one record
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                b[u][a] = bp[a];
                X[u][a] = bp[3 + a];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            ObsGeo<T> o;
            // an unresolved FP32 depth: the geometry from the FP64 point of the record
            if (!observation_geometry<T>(hd[u], X[u][0], X[u][1], X[u][2], o) && ck64)
                o = observation_geometry_f64<T>(ck64, j[u], pts + 3 * (int64_t)rec_pt[i[u]]);
            T c[9];
            free_camera_side<T>(o, hd[u], w[u], b[u][0], b[u][1], b[u][2], c);
            const int32_t jj = valid[u] ? j[u] : 0x7fffffff;
            while (true) {
                if (valid[u] && jj == cur)
#pragma unroll
                    for (int a = 0; a < 9; ++a) acc[a] += (double)c[a];
                const uint64_t more = __ballot(valid[u] && jj > cur);
                if (more == 0) break;
                flush(cur);
                ++slot;
                cur = __shfl(jj, __ffsll((unsigned long long)more) - 1, 64);
            }
        }
    }
    flush(cur);
}

// Folds the per-workgroup hot partials [G][K*9] into kHotFold slices, each
// the sum of a contiguous range of workgroups in order.
__global__ __launch_bounds__(256) void k_hot_fold(int32_t K9, int32_t G, const double* __restrict__ hot_part,
                                                  double* __restrict__ fold, const PcgScalars* __restrict__ sc,
                                                  int skip_if_done)
{
    if (skip_if_done && sc->done) return;
    fold_slice(blockIdx.x * 256 + threadIdx.x, blockIdx.y, K9, G, hot_part, fold);
}

// q = B~ x - c (mode 0) or g = v - c, r = g, x = 0 (mode 1); c from the hot
// slices and the cold slots.  The last block adds the per-block partial sums:
// mode 0: p^T q, then alpha = rho / p^T q and the matvec count (or a breakdown
// when p^T q <= 0); mode 1: ||b||^2.
template <int MODE>
__global__ __launch_bounds__(kEpiThreads) void k_schur_epilogue(
    int32_t m, int32_t K, const double* __restrict__ hot_fold, const int32_t* __restrict__ cold_cam_slot,
    const double* __restrict__ cold_slots, const double* __restrict__ bd,
    const double* __restrict__ pvec, const double* __restrict__ vcam, double* __restrict__ out,
    double* __restrict__ xvec, double* __restrict__ rvec, double* __restrict__ partials,
    PcgScalars* __restrict__ sc)
{
    __shared__ double sh[kEpiThreads / 64];
    if (MODE == 0 && sc->done) return;  // uniform over the grid
    double acc = 0.0;
    const int64_t len = 9 * (int64_t)m;
    for (int64_t t = blockIdx.x * (int64_t)kEpiThreads + threadIdx.x; t < len; t += (int64_t)gridDim.x * kEpiThreads) {
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
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kEpiThreads / 64; ++w) s += sh[w];
        partials[blockIdx.x] = s;
    }
    if (!last_block_arrives(&sc->arrive[MODE == 0 ? 1 : 2])) return;
    double tot = 0.0;
    for (int32_t b = threadIdx.x; b < (int32_t)gridDim.x; b += kEpiThreads) tot += partials[b];
    tot = wave_sum(tot);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kEpiThreads / 64; ++w) s += sh[w];
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
size_t hot_lds_bytes(int32_t K, int32_t Kc)
{
    return free_table_bytes(K) + (size_t)Kc * kCamRec * sizeof(T);
}

template <typename T>
int32_t hot_max_cameras(size_t lds_limit, int32_t Kc)
{
    const size_t rec = (size_t)Kc * kCamRec * sizeof(T) + 1024 + 16;
    if (lds_limit <= rec) return 0;
    return (int32_t)((lds_limit - rec) / (9 * sizeof(double)));
}

template <typename T>
hipError_t prepare_schur_kernels(int32_t K, int32_t Kc, bool recompute)
{
    const int bytes = (int)hot_lds_bytes<T>(K, recompute ? Kc : 0);
    hipError_t e;
    if (recompute) {
        e = hipFuncSetAttribute((const void*)k_schur_free<T, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)k_schur_free<T, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute((const void*)k_schur_free<T, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    }
    e = hipFuncSetAttribute((const void*)k_schur_hot<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_schur_rhs<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// The point half of the cold pass's per-point records: the point cast to T
// (words 3-5), for points with a cold observation.  Points change only with
// the state, so this runs with the build; the product passes write the b_i
// half (words 0-2).
template <typename T>
__global__ void k_cold_points(int32_t n, const double* __restrict__ pts, const int32_t* __restrict__ crec,
                              T* __restrict__ bcold)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = crec[i];
    if (r < 0) return;
    T* rec = bcold + kBcold * (int64_t)r;
    rec[3] = (T)pts[3 * (int64_t)i];
    rec[4] = (T)pts[3 * (int64_t)i + 1];
    rec[5] = (T)pts[3 * (int64_t)i + 2];
}

template <typename T>
hipError_t launch_cold_points(const SchurPlan& sp, int32_t n, const double* pts, hipStream_t s)
{
    if (n > 0 && sp.cold.N > 0)
        hipLaunchKernelGGL((k_cold_points<T>), dim3((n + 255) / 256), dim3(256), 0, s, n, pts, sp.crec,
                           (T*)sp.bcold);
    return hipGetLastError();
}

template hipError_t launch_cold_points<float>(const SchurPlan&, int32_t, const double*, hipStream_t);
template hipError_t launch_cold_points<double>(const SchurPlan&, int32_t, const double*, hipStream_t);

template <typename T>
hipError_t launch_schur_product(int mode, const SchurPlan& sp, const PointMajor& pm, int64_t N, const T* hcp,
                                const T* cinv, const double* wpt, const T* xcam, const RecomputeInputs<T>* ri,
                                int32_t m, const double* bd, const double* pvec, const double* vcam, double* out,
                                double* xvec, double* rvec, double* partials, PcgScalars* sc, hipEvent_t hot_begin,
                                hipEvent_t hot_end, hipStream_t s)
{
    hipError_t e;
    const size_t lds = hot_lds_bytes<T>(sp.K, sp.recompute && ri ? sp.Kc : 0);
    if (hot_begin && (e = hipEventRecord(hot_begin, s)) != hipSuccess) return e;
    if (sp.num_wg > 0) {
        const dim3 g(sp.num_wg), b(sp.recompute && ri ? FreeWgThreads<T>::value : HotThreads<T>::value);
        if (mode == 0 && sp.recompute && ri)
            hipLaunchKernelGGL((k_schur_free<T, 0>), g, b, lds, s, sp.frange, sp.sseg, sp.lrange, sp.lseg, pm.cam,
                               pm.pt, ri->wobs, ri->pts, ri->ck, ri->ck64, ri->xf, cinv, nullptr, sp.K, sp.Kc, (double*)sp.hot_part,
                               (T*)sp.bcold, sp.crec, nullptr, sc);
        else if (mode == 1 && sp.recompute && ri)
            hipLaunchKernelGGL((k_schur_free<T, 1>), g, b, lds, s, sp.frange, sp.sseg, sp.lrange, sp.lseg, pm.cam,
                               pm.pt, ri->wobs, ri->pts, ri->ck, ri->ck64, nullptr, cinv, wpt, sp.K, sp.Kc, (double*)sp.hot_part,
                               (T*)sp.bcold, sp.crec, nullptr, nullptr);
        else if (mode == 0)
            hipLaunchKernelGGL((k_schur_hot<T>), g, b, lds, s, sp.wrange, N, pm.cam, pm.pt, hcp, cinv, xcam,
                               sp.K, (double*)sp.hot_part, (T*)sp.bcold, sp.crec, sc);
        else
            hipLaunchKernelGGL((k_schur_rhs<T>), g, b, lds, s, sp.wrange, N, pm.cam, pm.pt, hcp, cinv, wpt,
                               sp.K, (double*)sp.hot_part, (T*)sp.bcold, sp.crec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (hot_end && (e = hipEventRecord(hot_end, s)) != hipSuccess) return e;
    const int32_t K9 = sp.K * 9;
    const bool fold = sp.K > 0 && sp.num_wg > 0;
    bool folded = false;
    if (sp.cold.num_chunks > 0) {
        if (sp.recompute && ri) {
            // the fold of the hot partials rides in the same launch as extra blocks
            const int32_t cold_blocks = (sp.cold.num_chunks + 3) / 4;
            const int32_t fold_blocks = fold ? (K9 + 255) / 256 * kHotFold : 0;
            hipLaunchKernelGGL((k_schur_cold_free<T>), dim3(cold_blocks + fold_blocks), dim3(256), 0, s, sp.cold.N,
                               sp.cold.num_chunks, sp.cold.cam, sp.cold.pt, (const T*)sp.cold.w, ri->pts, ri->ck,
                               ri->ck64, (const T*)sp.bcold, sp.rec_pt, sp.cold.chunk_slot, sp.cold.slots,
                               (const PcgScalars*)sc, mode == 0 ? 1 : 0, cold_blocks, K9, sp.num_wg,
                               (const double*)sp.hot_part, sp.hot_fold);
            folded = fold;
        } else
            hipLaunchKernelGGL((k_schur_cold<T>), dim3((sp.cold.num_chunks + 3) / 4), dim3(256), 0, s, sp.cold.N,
                               sp.cold.num_chunks, sp.cold.cam, sp.cold.pt, (const T*)sp.cold.hcp,
                               (const T*)sp.bcold, sp.cold.chunk_slot, sp.cold.slots, (const PcgScalars*)sc,
                               mode == 0 ? 1 : 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (fold && !folded) {
        hipLaunchKernelGGL(k_hot_fold, dim3((K9 + 255) / 256, kHotFold), dim3(256), 0, s, K9, sp.num_wg,
                           (const double*)sp.hot_part, sp.hot_fold, (const PcgScalars*)sc, mode == 0 ? 1 : 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // one entry per thread where the blocks allow; few blocks, since the
    // last-block reduction serialises one device-scope atomic per block
    int64_t nb64 = (9 * (int64_t)m + kEpiThreads - 1) / kEpiThreads;
    const int32_t nb = (int32_t)(nb64 < 1 ? 1 : (nb64 > kSmallBlocks ? kSmallBlocks : nb64));
    const int32_t Ke = sp.num_wg > 0 ? sp.K : 0;
    if (mode == 0)
        hipLaunchKernelGGL((k_schur_epilogue<0>), dim3(nb), dim3(kEpiThreads), 0, s, m, Ke, sp.hot_fold,
                           sp.cold.cam_slot, sp.cold.slots, bd, pvec, vcam, out, xvec, rvec, partials, sc);
    else
        hipLaunchKernelGGL((k_schur_epilogue<1>), dim3(nb), dim3(kEpiThreads), 0, s, m, Ke, sp.hot_fold,
                           sp.cold.cam_slot, sp.cold.slots, bd, pvec, vcam, out, xvec, rvec, partials, sc);
    return hipGetLastError();
}

template size_t hot_lds_bytes<float>(int32_t, int32_t);
template size_t hot_lds_bytes<double>(int32_t, int32_t);
template int32_t hot_max_cameras<float>(size_t, int32_t);
template int32_t hot_max_cameras<double>(size_t, int32_t);
template hipError_t prepare_schur_kernels<float>(int32_t, int32_t, bool);
template hipError_t prepare_schur_kernels<double>(int32_t, int32_t, bool);
template <typename T>
hipError_t launch_backsub_free(const SchurPlan& sp, const PointMajor& pm, const RecomputeInputs<T>& ri, const T* cinv,
                               const double* wpt, double* dp, hipStream_t s)
{
    if (sp.num_wg <= 0) return hipGetLastError();
    constexpr int NT = FreeThreads<T, 2>::value;  // the same waves as the product, NT / 64 per workgroup
    // no hot table (K = 0), the same camera records
    const size_t lds = hot_lds_bytes<T>(0, sp.Kc);
    hipLaunchKernelGGL((k_schur_free<T, 2>), dim3(sp.num_wg * (FreeWgThreads<T>::value / NT)), dim3(NT), lds, s,
                       sp.frange, sp.sseg, sp.lrange, sp.lseg, pm.cam, pm.pt, ri.wobs, ri.pts, ri.ck, ri.ck64, ri.xf,
                       cinv, wpt, 0, sp.Kc, nullptr, nullptr, sp.crec, dp, nullptr);
    return hipGetLastError();
}

template hipError_t launch_backsub_free<float>(const SchurPlan&, const PointMajor&, const RecomputeInputs<float>&,
                                               const float*, const double*, double*, hipStream_t);
template hipError_t launch_backsub_free<double>(const SchurPlan&, const PointMajor&, const RecomputeInputs<double>&,
                                                const double*, const double*, double*, hipStream_t);
template hipError_t launch_schur_product<float>(int, const SchurPlan&, const PointMajor&, int64_t, const float*,
                                                const float*, const double*, const float*,
                                                const RecomputeInputs<float>*, int32_t, const double*, const double*,
                                                const double*, double*, double*, double*, double*, PcgScalars*,
                                                hipEvent_t, hipEvent_t, hipStream_t);
template hipError_t launch_schur_product<double>(int, const SchurPlan&, const PointMajor&, int64_t, const double*,
                                                 const double*, const double*, const double*,
                                                 const RecomputeInputs<double>*, int32_t, const double*,
                                                 const double*, const double*, double*, double*, double*, double*,
                                                 PcgScalars*, hipEvent_t, hipEvent_t, hipStream_t);

}  // namespace ba

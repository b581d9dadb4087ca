// Internal declarations of the bundle-adjustment library: device workspace
// layout and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "camera_model.h"

namespace ba {

constexpr int kTile = 256;      // observations per point-aligned tile (one workgroup)
constexpr int kCmRows = 32;     // rows of <= 64 observations of one camera per camera-major wave chunk
constexpr int kColdRows = 8;    // rows of 64 observations per cold-stream wave chunk
constexpr int kColdChunk = 64 * kColdRows;
constexpr int kRedBlock = 256;  // threads of reduction blocks
constexpr int kCamSlotWords = 54;  // 45 upper-triangle B terms + 9 v terms
constexpr int kSlotSeg = 32;       // slots summed by one wavefront before the per-camera combine
constexpr int kHotFold = 8;        // slices the per-workgroup hot partials are folded into
constexpr int kBcold = 6;          // words of T per point record read by the cold pass
constexpr int kEpiThreads = 1024;  // threads of the product's epilogue blocks
constexpr int kSmallBlocks = 192;  // at most this many epilogue blocks (its last-block reduction
                                   // serialises one device-scope atomic per block)

// Scalars of one PCG run, kept on the device.  Kernels of the PCG loop read
// `done` first and do nothing once it is set, so the host can enqueue
// iterations ahead and read the flag only now and then.
struct PcgScalars {
    double rho;         // r^T z of the current iteration
    double rho_prev;    // r^T z of the previous iteration
    double pq;          // p^T q
    double rr;          // ||r||^2 of the current residual
    double bb;          // ||b||^2
    double alpha, beta;
    double rtol;        // stop when ||r|| <= rtol ||b|| ...
    int32_t max_iters;  // ... or when this many matvecs ran
    int32_t fixed;      // > 0: run exactly this many matvecs instead
    int32_t iters;      // matvecs executed
    int32_t done;       // loop finished (converged, count reached or breakdown)
    int32_t breakdown;  // p^T q <= 0 or non-finite
    uint32_t arrive[3]; // arrival counters of last-block reductions
};

// Last-block reduction: every block stores its partial sums, then the last
// block to arrive (device-scope counter) adds all partials in block order.
__device__ __forceinline__ bool last_block_arrives(uint32_t* counter)
{
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(counter, 1u);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// The point-major coupling blocks E are stored tile-blocked: the 27 rows of
// each 64-observation tile are contiguous ([tile][27][64] of T), so one tile
// is a single run of memory (6.9 KB in FP32) and every row is a 256-byte
// (FP32) or 512-byte (FP64) aligned piece of it.
__host__ __device__ __forceinline__ int64_t eidx(int64_t k, int q) { return ((k >> 6) * 27 + q) * 64 + (k & 63); }

// Point-major observation stream (sorted by point, then camera).
struct PointMajor {
    int32_t* cam;      // [ld] internal camera id
    int32_t* pt;       // [ld]
    double* uvx;       // [N]
    double* uvy;       // [N]
    int32_t* tile;     // [num_tiles + 1] observation offsets of point-aligned tiles
    int32_t num_tiles;
    int64_t ld;        // stream length: N rounded up to 64 plus one padding tile
                       // (cam 0, pt -1), so tile t + 1 always exists; E holds 27 ld
    // point-aligned segments as [begin, end) observation ranges: short ones
    // (<= 64 observations of whole points) and long ones (one longer point)
    const int2* sseg;
    const int2* lseg;
    int32_t num_short, num_long;
    int32_t num_cameras;
};

// Workgroups of the persistent streaming kernels (the cost pass):
// one per CU of the MI355X.
constexpr int kPersistentBlocks = 256;
// Sets the dynamic LDS limits of the cost kernels (once per process
// is enough; called when a problem is made).
hipError_t prepare_cost_kernels();

// Camera-major observation stream (sorted by camera, then point).
struct CameraMajor {
    int32_t* cam;         // [N]
    int32_t* pt;          // [N]
    double* uvx;          // [N]
    double* uvy;          // [N]
    int32_t* row;         // [num_rows + 1] first observation of each row: <= 64 of one camera
    int32_t num_rows;
    int32_t* chunk_slot;  // [num_chunks + 1] first partial-sum slot of each wave chunk (kCmRows rows)
    int32_t* cam_slot;    // [m + 1] slots of each camera (contiguous)
    int32_t num_chunks;
    int32_t num_slots;
    double* slots;        // [num_slots][54]
    // per-camera reduction of the slots in segments of <= kSlotSeg
    int32_t num_segs;
    int32_t* seg_cam;     // [num_segs] camera of each segment
    int32_t* seg_slot;    // [num_segs] first slot of each segment
    int32_t* cam_seg;     // [m + 1] segments of each camera (contiguous)
    double* seg_part;     // [num_segs][54]
    uint32_t* arrive;     // [m] arrival counters (zero between calls)
};

// Words of the camera record the recomputing product keeps in LDS for its
// hot cameras: the head of CamK and the 12-word direction record.
constexpr int kCamRec = kCamHead + 12;
// records kept (most observed cameras first), FP32-mixed / FP64
constexpr int kCacheCamerasF32 = 512;
constexpr int kCacheCamerasF64 = 256;
template <typename T>
constexpr size_t kCamRecBytes()
{
    return kCamRec * sizeof(T);
}

// Threads per workgroup of the hot-camera Schur pass (one workgroup per CU).
template <typename T>
struct HotThreads;
template <>
struct HotThreads<float> {
    static constexpr int value = 1024;
};
template <>
struct HotThreads<double> {
    static constexpr int value = 512;
};

// Threads per workgroup of the recomputing product's point-major pass (one
// workgroup per CU, like the stored-block pass): sixteen wavefronts in both
// precisions.  FP64 takes one segment at a time to fit them (at 29M
// observations 0.524 ms per pass, against 0.554 ms for eight wavefronts
// with two segments in flight and 0.533 ms for twelve with one).
template <typename T>
struct FreeWgThreads;
template <>
struct FreeWgThreads<float> {
    static constexpr int value = 1024;
};
template <>
struct FreeWgThreads<double> {
    static constexpr int value = 1024;
};

// Observations on cameras outside the hot set, in camera-major order.
struct ColdStream {
    int64_t N = 0;
    int32_t* cam = nullptr;         // [N]
    int32_t* pt = nullptr;          // [N] the observation's point record (crec)
    void* hcp = nullptr;            // [27][N] of T (stored-block product)
    void* w = nullptr;              // [N] of T: IRLS weights (recomputing product)
    int32_t* chunk_slot = nullptr;  // [num_chunks + 1]
    int32_t* cam_slot = nullptr;    // [m + 1]
    int32_t num_chunks = 0;
    int32_t num_slots = 0;
    double* slots = nullptr;        // [num_slots][9]
};

// Schedule of the implicit Schur product (see matvec.hip).
struct SchurPlan {
    int32_t K = 0;                  // hot cameras: internal ids [0, K)
    int32_t Kc = 0;                 // recomputing product: cameras [0, Kc) whose records the
                                    // point-major pass keeps in LDS
    int32_t num_wg = 0;             // persistent workgroups of the hot pass
    int32_t* wrange = nullptr;      // [num_wg * waves per workgroup + 1] ranges of 64-observation
                                    // tiles per wavefront
    int32_t* crec = nullptr;        // [n] the point's record in bcold, -1 when it has no cold
                                    // observation (the stored-block design: the point's own index;
                                    // the recomputing one: records in order of first use by the
                                    // camera-major cold stream, so they are read mostly in sequence)
    void* hot_part = nullptr;       // [num_wg][K][9] FP64
    double* hot_fold = nullptr;     // [kHotFold][K][9] FP64
    void* bcold = nullptr;          // [n][kBcold] of T: b_i for the cold pass (words 0-2), and
                                    // (recomputing product) the point cast to T (words 3-5), one
                                    // record per point with a cold observation (crec)
    int32_t* rec_pt = nullptr;      // recomputing product: the point of each record
    ColdStream cold;
    // the recomputing product (mode 0 when set): point-aligned segments, short
    // (<= 64 observations of whole points) and long (one longer point), as
    // [begin, end) observation ranges, and their ranges per wavefront
    bool recompute = false;
    int32_t num_short = 0, num_long = 0;
    int2* sseg = nullptr;           // [num_short]
    int2* lseg = nullptr;           // [num_long]
    int32_t* frange = nullptr;      // [num_wg * waves per workgroup + 1] short-segment ranges, split
                                    // by observation count; a workgroup's share runs from its first
                                    // wavefront's start to the next workgroup's
    int32_t* lrange = nullptr;      // [num_wg * waves per workgroup + 1] long-segment ranges, alike
};

// What the recomputing product reads besides the streams of PointMajor.
template <typename T>
struct RecomputeInputs {
    const T* wobs;       // [ld] IRLS weight per point-major observation
    const double* pts;   // [n][3] point coordinates
    const CamK<T>* ck;   // [m] camera constants
    const T* xf;         // [m][12] camera vectors from launch_pcg_direction
    const CamK<double>* ck64;  // [m] FP64 constants (FP32 form: unresolved depths), nullable
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipGetLastError().
hipError_t launch_camera_constants_f64(int32_t m, const double* cams, CamK<double>* out, hipStream_t s);
hipError_t launch_camera_constants_f32(int32_t m, const double* cams, CamK<float>* out, hipStream_t s);

// Where the build's Jacobians come from: the per-camera constants of the
// analytic form (ck), or, when cams is set, forward-mode differentiation of
// the residual at the FP64 camera parameters cams [m][9] (internal order).
// ck64 (nullable): FP64 constants of the same cameras, for the FP32 form's
// observations whose depth FP32 cannot resolve.
template <typename T>
struct JacSource {
    const CamK<T>* ck;
    const double* cams;
    const CamK<double>* ck64;
};

// Point-major build: E_k into hcp, C_i into hpp and each observation's IRLS
// weight into wobs (all unless grad_only), and w_i into wpt.
template <typename T>
hipError_t launch_build_points(const PointMajor& pm, double delta, bool grad_only, const double* pts,
                               JacSource<T> js, T* hcp, double* hpp, double* wpt, T* wobs, hipStream_t s);
// Camera-major build: B_j (unless grad_only) and v_j; for the last Nc
// observations of the camera-major stream (the cold cameras) also, when
// given, E_k into chcp[q * Nc + k - (N - Nc)] and the weight into
// cw[k - (N - Nc)].
template <typename T>
hipError_t launch_build_cameras(const CameraMajor& cm, int32_t m, int64_t N, const double* pts,
                                JacSource<T> js, double delta, bool grad_only, double* hcc,
                                double* vcam, int64_t Nc, T* chcp, T* cw, hipStream_t s);

// Schur-Jacobi preconditioner option: mj [m][81] = -sum_k E_k C~^-1 E_k^T per
// camera (camera-major pass at the current state and damping), then
// lfac = chol(B~_j + mj_j) with failure flags as launch_damp_cameras.
template <typename T>
hipError_t launch_schur_jacobi_terms(const CameraMajor& cm, int64_t N, const double* pts, JacSource<T> js,
                                     double delta, const T* cinv, double* mj, hipStream_t s);
hipError_t launch_factor_schur_jacobi(int32_t m, const double* bd, const double* mj, double* lfac, int32_t* flag,
                                      hipStream_t s);

hipError_t launch_damp_cameras(int32_t m, const double* hcc, double lambda, int32_t damping,
                               double* bd, double* lfac, double* dcam, int32_t* flag, hipStream_t s);
template <typename T>
hipError_t launch_damp_points(int32_t n, const double* hpp, double lambda, int32_t damping, T* cinv,
                              int32_t* flag, hipStream_t s);

// The direct option's plan: the camera-major walk (pieces of at most
// kDensePiece observations of one camera, and per camera-major entry its
// point-major index), the point
// offsets of the point-major stream, and an FP64 scratch stream of E_k.
constexpr int32_t kDensePiece = 4096;  // camera-major observations per piece of a block row

struct DensePlan {
    int32_t num_pieces = 0;
    int4* pieces = nullptr;    // {camera, first, end, pieces of this camera}, camera order
    int32_t* coff = nullptr;   // [m + 1]
    int32_t* cm_pm = nullptr;  // [N]
    int32_t* poff = nullptr;   // [n + 1]
    double* E = nullptr;       // [N][27]
};

// x = S^-1 g for the reduced camera system written out (S [9m][9m] FP64,
// formed from B~ (bd), the per-camera self terms mj and the cross terms of
// shared points, then factored in place); flag bit 2 when S is not positive
// definite.
template <typename T>
hipError_t launch_dense_solve(const DensePlan& dp, const PointMajor& pm, int64_t N, const RecomputeInputs<T>& ri,
                              const T* cinv, int32_t m, const double* bd, const double* mj, const double* g,
                              double* x, double* S, int32_t* flag, hipStream_t s);

// Back-substitution from the stored blocks (BA_SCHUR_STORED=1):
// dp = C~^-1 (w - E^T x), x in T (xcam).
template <typename T>
hipError_t launch_backsub_stored(const PointMajor& pm, const T* hcp, const T* cinv, const double* wpt,
                                 const T* xcam, double* dp, hipStream_t s);

// Writes the point half of the cold pass's per-point records (the point cast
// to T) for the current state; run whenever the points change.
template <typename T>
hipError_t launch_cold_points(const SchurPlan& sp, int32_t n, const double* pts, hipStream_t s);

// Full implicit Schur product.  mode 0: out = q = B~ x - E C~^-1 E^T x, then
// p^T q, alpha and the matvec count into sc (skipped once sc->done);
// mode 1: out = g = v - E C~^-1 w, r = g, x = 0 and ||g||^2 into sc.
// xcam: x in T and pvec: x in FP64 (mode 0).  With sp.recompute and ri set,
// mode 0 forms E from the Jacobian instead of reading hcp.  hot_begin/hot_end
// (nullable) bracket the point-major pass.
template <typename T>
hipError_t launch_schur_product(int mode, const SchurPlan& sp, const PointMajor& pm, int64_t N, const T* hcp,
                                const T* cinv, const double* wpt, const T* xcam, const RecomputeInputs<T>* ri,
                                int32_t m, const double* bd, const double* pvec, const double* vcam, double* out,
                                double* xvec, double* rvec, double* partials, PcgScalars* sc, hipEvent_t hot_begin,
                                hipEvent_t hot_end, hipStream_t s);
// Back-substitution without stored blocks (sp.recompute): dp_i =
// C~_i^-1 (w_i - sum_k E_k^T dc_j), with dc in ri.xf (launch_pcg_direction).
template <typename T>
hipError_t launch_backsub_free(const SchurPlan& sp, const PointMajor& pm, const RecomputeInputs<T>& ri, const T* cinv,
                               const double* wpt, double* dp, hipStream_t s);
// LDS of the point-major pass for K hot cameras: their FP64 table, and with
// the recomputing product the records of cameras [0, Kc).
template <typename T>
size_t hot_lds_bytes(int32_t K, int32_t Kc);
// The largest hot set whose table fits beside Kc camera records.
template <typename T>
int32_t hot_max_cameras(size_t lds_limit, int32_t Kc);
template <typename T>
hipError_t prepare_schur_kernels(int32_t K, int32_t Kc, bool recompute);

hipError_t launch_zero(double* p, int64_t count, hipStream_t s);
hipError_t launch_sum_partials(const double* partials, int32_t count, int32_t stride, int32_t ncols,
                               double* out, hipStream_t s);
// Resets the PCG scalars with the stopping rule of this run.
hipError_t launch_pcg_reset(PcgScalars* sc, double rtol, int32_t max_iters, int32_t fixed, hipStream_t s);
// One PCG step on the camera vectors: (unless first) x += alpha p, r -= alpha q;
// z = M^-1 r; then rho, ||r||^2, the stopping test and beta (last block).
hipError_t launch_pcg_step(int32_t m, bool first, const double* lfac, const double* p, const double* q,
                           double* x, double* r, double* z, double* partials, PcgScalars* sc, hipStream_t s);
// p = z (first iteration) or z + beta p; pT = (T) p; with xf set also the
// recomputing product's camera vectors [J_l p_w, p_t, p_f, p_k1, p_k2] (12
// words per camera, J_l from ck).  With force, runs even after the loop
// stopped (used to hand x to the back-substitution).
template <typename T>
hipError_t launch_pcg_direction(int32_t m, bool force, const double* z, double* p, T* pT, const CamK<T>* ck, T* xf,
                                PcgScalars* sc, hipStream_t s);
hipError_t launch_trial_state(int32_t m, int32_t n, const double* cams, const double* dc, const double* pts,
                              const double* dp, double* cams_t, double* pts_t, hipStream_t s);
hipError_t launch_cost(const PointMajor& pm, int64_t N, const double* pts, const CamK<double>* ck,
                       double delta, double* partials, int32_t* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_cost_t(const PointMajor& pm, int64_t N, const double* pts, const CamK<T>* ck,
                         double delta, double* partials, int32_t* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_pred(int32_t m, int32_t n, const double* dc, const double* dcam, const double* vcam,
                       const double* dp, const double* hpp, const double* wpt, double lambda, int32_t damping,
                       double* partials, int32_t* nblocks, hipStream_t s);

// caller order <-> internal order, with dtype conversion
hipError_t launch_gather_cameras(int32_t m, int dtype, const void* src, const int32_t* old_of_new, double* dst,
                                 hipStream_t s);
hipError_t launch_convert_points(int32_t n, int dtype, const void* src, double* dst, hipStream_t s);
// scale (times *dscale when dscale is set) times -v and -w into caller order
hipError_t launch_scatter_grad(int32_t m, int32_t n, int dtype, double scale, const double* dscale,
                               const double* vcam, const double* wpt, const int32_t* old_of_new, void* gcam,
                               void* gpt, hipStream_t s);
hipError_t launch_store_cost(const double* sum, double* out, hipStream_t s);

int32_t reduce_blocks(int64_t count);

}  // namespace ba

// Internal declarations of the bundle-adjustment library: device workspace
// layout and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "camera_model.h"

namespace ba {

constexpr int kTile = 256;      // observations per point-aligned tile (one workgroup)
constexpr int kCmRows = 32;     // rows of 64 observations per camera-major wave chunk
constexpr int kCmChunk = 64 * kCmRows;
constexpr int kRedBlock = 256;  // threads of reduction blocks
constexpr int kCamSlotWords = 54;  // 45 upper-triangle B terms + 9 v terms

// Scalars of one PCG run, kept on the device.
struct PcgScalars {
    double rho;       // r^T z of the current iteration
    double rho_prev;  // r^T z of the previous iteration
    double pq;        // p^T q
    double rr;        // ||r||^2 after the last update
    double bb;        // ||b||^2
    double alpha, beta;
    int32_t breakdown;  // set when p^T q <= 0 or non-finite; later updates are skipped
    int32_t pad;
};

// Point-major observation stream (sorted by point, then camera).
struct PointMajor {
    int32_t* cam;      // [N] internal camera id
    int32_t* pt;       // [N]
    double* uvx;       // [N]
    double* uvy;       // [N]
    int32_t* tile;     // [num_tiles + 1] observation offsets of point-aligned tiles
    int32_t num_tiles;
};

// Camera-major observation stream (sorted by camera, then point).
struct CameraMajor {
    int32_t* cam;         // [N]
    int32_t* pt;          // [N]
    double* uvx;          // [N]
    double* uvy;          // [N]
    int32_t* chunk_slot;  // [num_chunks + 1] first partial-sum slot of each wave chunk
    int32_t* cam_slot;    // [m + 1] slots of each camera (contiguous)
    int32_t num_chunks;
    int32_t num_slots;
    double* slots;        // [num_slots][54]
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipGetLastError().
hipError_t launch_camera_constants_f64(int32_t m, const double* cams, CamK<double>* out, hipStream_t s);
hipError_t launch_camera_constants_f32(int32_t m, const double* cams, CamK<float>* out, hipStream_t s);

template <typename T>
hipError_t launch_build_points(const PointMajor& pm, int64_t N, const double* pts, const CamK<T>* ck,
                               double delta, bool grad_only, T* hcp, T* hpp, double* wpt, hipStream_t s);
template <typename T>
hipError_t launch_build_cameras(const CameraMajor& cm, int32_t m, int64_t N, const double* pts,
                                const CamK<T>* ck, double delta, bool grad_only, double* hcc,
                                double* vcam, hipStream_t s);

hipError_t launch_damp_cameras(int32_t m, const double* hcc, double lambda, int32_t damping,
                               double* bd, double* lfac, double* dcam, int32_t* flag, hipStream_t s);
template <typename T>
hipError_t launch_damp_points(int32_t n, const T* hpp, double lambda, int32_t damping, T* cinv,
                              int32_t* flag, hipStream_t s);

// mode 0: c = E C^-1 E^T x    (implicit Schur product without the B term)
// mode 1: c = E C^-1 w        (reduced right-hand side)
// mode 2: dp = C^-1 (w - E^T x)  (back-substitution)
template <typename T>
hipError_t launch_schur_tiles(int mode, const PointMajor& pm, int64_t N, const T* hcp, const T* cinv,
                              const double* wpt, const T* xcam, double* cacc, double* dp, hipStream_t s);

hipError_t launch_zero(double* p, int64_t count, hipStream_t s);
hipError_t launch_rhs_combine(int32_t m, const double* vcam, const double* cacc, double* g, double* x,
                              double* r, double* partials, int32_t* nblocks, hipStream_t s);
hipError_t launch_sum_partials(const double* partials, int32_t count, int32_t stride, int32_t ncols,
                               double* out, hipStream_t s);
hipError_t launch_pcg_precond(int32_t m, const double* lfac, const double* r, double* z, double* partials,
                              int32_t* nblocks, const PcgScalars* sc, hipStream_t s);
template <typename T>
hipError_t launch_pcg_direction(int32_t m, bool first, const double* z, double* p, T* pT, PcgScalars* sc,
                                hipStream_t s);
hipError_t launch_matvec_combine(int32_t m, const double* bd, const double* p, const double* cacc, double* q,
                                 double* partials, int32_t* nblocks, const PcgScalars* sc, hipStream_t s);
hipError_t launch_pcg_update(int32_t m, const double* p, const double* q, double* x, double* r,
                             double* partials, int32_t* nblocks, PcgScalars* sc, hipStream_t s);
hipError_t launch_pcg_finish_scalars(PcgScalars* sc, const double* sums, int which, hipStream_t s);

hipError_t launch_trial_state(int32_t m, int32_t n, const double* cams, const double* dc, const double* pts,
                              const double* dp, double* cams_t, double* pts_t, hipStream_t s);
hipError_t launch_cost(const PointMajor& pm, int64_t N, const double* pts, const CamK<double>* ck,
                       double delta, double* partials, int32_t* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_cost_t(const PointMajor& pm, int64_t N, const double* pts, const CamK<T>* ck,
                         double delta, double* partials, int32_t* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_pred(int32_t m, int32_t n, const double* dc, const double* dcam, const double* vcam,
                       const double* dp, const T* hpp, const double* wpt, double lambda, int32_t damping,
                       double* partials, int32_t* nblocks, hipStream_t s);

// caller order <-> internal order, with dtype conversion
hipError_t launch_gather_cameras(int32_t m, int dtype, const void* src, const int32_t* old_of_new, double* dst,
                                 hipStream_t s);
hipError_t launch_convert_points(int32_t n, int dtype, const void* src, double* dst, hipStream_t s);
hipError_t launch_scatter_grad(int32_t m, int32_t n, int dtype, double scale, const double* vcam,
                               const double* wpt, const int32_t* old_of_new, void* gcam, void* gpt,
                               hipStream_t s);
hipError_t launch_store_cost(const double* sum, double* out, hipStream_t s);

int32_t reduce_blocks(int64_t count);

}  // namespace ba

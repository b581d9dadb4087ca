// Robust reprojection cost from caller device arrays with no handle and no
// allocation: F = 1/2 sum_k rho(|e_k|^2) (Sec. 3, Eq. obj, with the Huber
// reading of the robust loss), the quantity ba_cost_fwd_device computes for a
// handle.  Its only scratch is the per-block partial sums, held in a
// file-scope device array: each device keeps its own copy of the array for
// the life of the process, and every call on that device shares it, so two
// calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ba.h"
#include "ba_internal.h"

namespace ba {

constexpr int kNoAllocBlocks = 2048;  // partial sums: 16 KB of scratch per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocBlocks];

// Device address of `scratch` on each device, looked up once per device with
// that device current (the array's name is only a host-side stand-in).
static double* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mutex;

static hipError_t scratch_for_current_device(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// One thread per observation (grid-stride): the camera's constants are formed
// from its nine parameters in FP64 (rounded to T for the FP32 form, as the
// handle's path does), then the residual in T and 1/2 rho in FP64.  An index
// outside [0, m) or [0, n) contributes NaN, so a bad graph shows in the
// result instead of reading out of bounds.
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_cost_raw(int64_t N, int32_t m, int32_t n,
                                                        const T* __restrict__ cams, const T* __restrict__ pts,
                                                        const int32_t* __restrict__ oc, const int32_t* __restrict__ op,
                                                        const double* __restrict__ uv, T delta,
                                                        double* __restrict__ partials)
{
    __shared__ double sh[kRedBlock / 64];
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; k < N; k += (int64_t)gridDim.x * kRedBlock) {
        const int32_t j = oc[k], i = op[k];
        if (j < 0 || j >= m || i < 0 || i >= n) {
            acc += __builtin_nan("");
            continue;
        }
        double c[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) c[a] = (double)cams[9 * (int64_t)j + a];
        CamK<T> kk;
        camera_constants<T>(c, kk);
        T e0, e1;
        residual<T>(kk, pts[3 * (int64_t)i], pts[3 * (int64_t)i + 1], pts[3 * (int64_t)i + 2], (T)uv[2 * k],
                    (T)uv[2 * k + 1], e0, e1);
        acc += 0.5 * (double)huber_rho<T>(e0 * e0 + e1 * e1, delta);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kRedBlock / 64; ++w) t += sh[w];
        partials[blockIdx.x] = t;
    }
}

}  // namespace ba

using namespace ba;

extern "C" ba_status ba_cost_device_noalloc(int32_t num_cameras, int32_t num_points, int64_t num_obs,
                                            int32_t dtype, const void* d_cams, const void* d_pts,
                                            const int32_t* d_obs_camera, const int32_t* d_obs_point,
                                            const double* d_obs_uv, double huber_delta, double* d_cost_f64,
                                            void* hip_stream)
{
    if (num_cameras < 1 || num_points < 0 || num_obs < 0 || (dtype != 0 && dtype != 1) || !d_cams ||
        (num_points > 0 && !d_pts) || !d_cost_f64 || !(huber_delta == huber_delta) ||
        (num_obs > 0 && (!d_obs_camera || !d_obs_point || !d_obs_uv)))
        return BA_EINVAL;
    double* partials = nullptr;
    if (scratch_for_current_device(&partials) != hipSuccess) return BA_EDEVICE;
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t blocks = reduce_blocks(num_obs);
    if (blocks > kNoAllocBlocks) blocks = kNoAllocBlocks;
    if (dtype == 0)
        hipLaunchKernelGGL((k_cost_raw<double>), dim3(blocks), dim3(kRedBlock), 0, s, num_obs, num_cameras,
                           num_points, (const double*)d_cams, (const double*)d_pts, d_obs_camera, d_obs_point,
                           d_obs_uv, huber_delta, partials);
    else
        hipLaunchKernelGGL((k_cost_raw<float>), dim3(blocks), dim3(kRedBlock), 0, s, num_obs, num_cameras,
                           num_points, (const float*)d_cams, (const float*)d_pts, d_obs_camera, d_obs_point,
                           d_obs_uv, (float)huber_delta, partials);
    if (hipGetLastError() != hipSuccess) return BA_EDEVICE;
    // the blocks' partial sums added in block order into the caller's double
    if (launch_sum_partials(partials, blocks, 1, 1, d_cost_f64, s) != hipSuccess) return BA_EDEVICE;
    return BA_OK;
}

// C ABI and host driver: problem set-up (validation, sorting, workspace) and
// the Levenberg-Marquardt loop of Alg. 1 (one partition) inside the
// trust-region wrapper of the supplementary Sec. C.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"

using namespace ba;

namespace {

thread_local std::string g_create_error;

struct DevAlloc {
    std::vector<void*> ptrs;
    int64_t bytes = 0;
    hipError_t err = hipSuccess;
    template <typename T>
    T* get(int64_t count)
    {
        if (err != hipSuccess) return nullptr;
        if (count <= 0) count = 1;
        void* p = nullptr;
        const size_t sz = (size_t)count * sizeof(T);
        err = hipMalloc(&p, sz);
        if (err != hipSuccess) return nullptr;
        ptrs.push_back(p);
        bytes += (int64_t)sz;
        return (T*)p;
    }
    void release()
    {
        for (void* p : ptrs) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
};

}  // namespace

struct ba_problem {
    int32_t m = 0, n = 0;
    int64_t N = 0;
    ba_options opt{};
    hipStream_t stream = nullptr;
    std::string last_error;
    std::vector<int32_t> old_of_new, new_of_old;

    DevAlloc mem;
    // state (internal camera order)
    double *cams = nullptr, *pts = nullptr, *cams_t = nullptr, *pts_t = nullptr;
    CamK<double>*ck64 = nullptr, *ck64_t = nullptr;
    CamK<float>* ck32 = nullptr;
    int32_t* d_old_of_new = nullptr;
    PointMajor pm{};
    CameraMajor cm{};
    SchurPlan sp{};
    // blocks
    void* hcp = nullptr;   // [27][N] of T
    void* hpp = nullptr;   // [n][6] FP64 (summed and inverted in FP64 in both forms)
    void* cinv = nullptr;  // [n][6] of T
    double* wpt = nullptr; // [n][3]
    double *hcc = nullptr, *vcam = nullptr, *bd = nullptr, *lfac = nullptr, *dcam = nullptr;
    double* mj = nullptr;  // [m][81]: Schur-Jacobi terms (preconditioner option)
    // PCG
    double *g = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *cacc = nullptr;
    void* pT = nullptr;
    void* wobs = nullptr;  // [ld] of T: IRLS weight per point-major observation
    void* xf = nullptr;    // [m][12] of T: camera vectors of the recomputing product
    double* dp = nullptr;
    double *partials = nullptr, *sums = nullptr;
    PcgScalars* sc = nullptr;
    int32_t* flag = nullptr;
    // direct option: S [9m][9m] FP64 factored in place and the formation plan
    double* S = nullptr;
    DensePlan dense{};
    // pinned host scratch
    double* h_scalars = nullptr;
    hipEvent_t sync_ev = nullptr;  // polled by wait_stream
    bool is_f32() const { return opt.precision == BA_FP32_MIXED; }
};

#define BA_TRY(prob, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            (prob)->last_error = std::string(#expr) + ": " + hipGetErrorString(e_);         \
            return BA_EDEVICE;                                                               \
        }                                                                                    \
    } while (0)

// Text for a failed damped-block factorisation from the device flag words:
// bit 0 of flag[0] is set by the camera blocks, bit 1 by the point blocks;
// flag[1] and flag[2] name one failing camera and point, whose undamped block
// diagonal is quoted.
static std::string not_pd_message(ba_problem* P, const int32_t* flag, double lambda, bool schur_jacobi = false)
{
    char buf[256];
    std::string msg = "damped";
    if (flag[0] & 1) {
        if (schur_jacobi) msg += " Schur-Jacobi";
        double d[81] = {0};
        const int32_t j = flag[1];
        if (j >= 0 && j < P->m && hipMemcpy(d, P->hcc + 81 * (int64_t)j, sizeof d, hipMemcpyDeviceToHost) == hipSuccess)
            std::snprintf(buf, sizeof buf, " camera block %d (diagonal %.3e .. %.3e)", (int)P->old_of_new[j],
                          *std::min_element(d, d + 81, [](double a, double b) { return a < b; }),
                          *std::max_element(d, d + 81, [](double a, double b) { return a < b; }));
        else
            std::snprintf(buf, sizeof buf, " camera block");
        msg += buf;
    }
    if (flag[0] & 2) {
        double c[6] = {0};
        const int32_t i = flag[2];
        if (i >= 0 && i < P->n && hipMemcpy(c, (const double*)P->hpp + 6 * (int64_t)i, sizeof c, hipMemcpyDeviceToHost) == hipSuccess)
            std::snprintf(buf, sizeof buf, "%s point block %d (C = %.3e %.3e %.3e %.3e %.3e %.3e)",
                          (flag[0] & 1) ? " and" : "", (int)i, c[0], c[1], c[2], c[3], c[4], c[5]);
        else
            std::snprintf(buf, sizeof buf, "%s point block", (flag[0] & 1) ? " and" : "");
        msg += buf;
    }
    std::snprintf(buf, sizeof buf, " not positive definite at lambda %.3e", lambda);
    return msg + buf;
}

static bool finite_all(const double* a, int64_t len)
{
    for (int64_t t = 0; t < len; ++t)
        if (!std::isfinite(a[t])) return false;
    return true;
}

static ba_status check_options(const ba_options* o, std::string& msg)
{
    if (o->struct_size != sizeof(ba_options)) {
        msg = "ba_options.struct_size mismatch";
        return BA_EINVAL;
    }
    if (o->precision != BA_FP64 && o->precision != BA_FP32_MIXED) {
        msg = "unknown precision";
        return BA_EINVAL;
    }
    if (o->damping != BA_DAMP_MARQUARDT && o->damping != BA_DAMP_IDENTITY) {
        msg = "unknown damping";
        return BA_EINVAL;
    }
    if (o->jacobian != BA_JACOBIAN_ANALYTIC && o->jacobian != BA_JACOBIAN_AUTODIFF) {
        msg = "unknown jacobian";
        return BA_EINVAL;
    }
    if (o->solver != BA_SOLVER_PCG && o->solver != BA_SOLVER_DENSE) {
        msg = "unknown solver";
        return BA_EINVAL;
    }
    if (o->preconditioner != BA_PRECOND_CAMERA_BLOCKS && o->preconditioner != BA_PRECOND_SCHUR_JACOBI) {
        msg = "unknown preconditioner";
        return BA_EINVAL;
    }
    if (o->max_lm_iters < 0 || o->max_pcg_iters < 0 || o->pcg_fixed_iters < 0 || !std::isfinite(o->pcg_rtol) ||
        !(o->lambda_init > 0.0) || !std::isfinite(o->lambda_init) || !std::isfinite(o->min_relative_decrease) ||
        !std::isfinite(o->huber_delta)) {
        msg = "invalid option value";
        return BA_EINVAL;
    }
    if (o->pcg_schedule)
        for (int32_t t = 0; t < o->max_lm_iters; ++t)
            if (o->pcg_schedule[t] < 0) {
                msg = "negative pcg_schedule entry";
                return BA_EINVAL;
            }
    return BA_OK;
}

extern "C" {

ba_status ba_options_default(ba_options* opt)
{
    if (!opt) return BA_EINVAL;
    std::memset(opt, 0, sizeof(*opt));
    opt->struct_size = sizeof(ba_options);
    opt->precision = BA_FP64;
    opt->damping = BA_DAMP_MARQUARDT;
    opt->huber_delta = 0.0;
    opt->max_lm_iters = 10;
    opt->max_pcg_iters = 50;
    opt->pcg_rtol = 1e-8;
    opt->pcg_fixed_iters = 0;
    opt->pcg_schedule = nullptr;
    opt->lambda_init = 1e-4;
    opt->min_relative_decrease = 1e-3;
    opt->time_kernels = 0;
    opt->jacobian = BA_JACOBIAN_ANALYTIC;
    opt->solver = BA_SOLVER_PCG;
    opt->preconditioner = BA_PRECOND_CAMERA_BLOCKS;
    return BA_OK;
}

const char* ba_status_str(ba_status s)
{
    switch (s) {
    case BA_OK: return "BA_OK";
    case BA_EINVAL: return "BA_EINVAL";
    case BA_ENOMEM: return "BA_ENOMEM";
    case BA_EDEVICE: return "BA_EDEVICE";
    case BA_ENUMERIC: return "BA_ENUMERIC";
    }
    return "BA_UNKNOWN";
}

const char* ba_last_error(const ba_problem* prob)
{
    if (!prob) return g_create_error.c_str();
    return prob->last_error.c_str();
}

void ba_destroy(ba_problem* prob)
{
    if (!prob) return;
    if (prob->stream) (void)hipStreamSynchronize(prob->stream);
    else (void)hipDeviceSynchronize();
    prob->mem.release();
    if (prob->h_scalars) (void)hipHostFree(prob->h_scalars);
    if (prob->sync_ev) (void)hipEventDestroy(prob->sync_ev);
    delete prob;
}

ba_status ba_memory_bytes(const ba_problem* prob, int64_t* bytes)
{
    if (!prob || !bytes) return BA_EINVAL;
    *bytes = prob->mem.bytes;
    return BA_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ set-up
// Partial-sum slots of a camera-sorted stream (observations, or rows of one
// camera each) cut into wave chunks of `chunk` entries: one slot per (chunk,
// camera run); a camera's slots are contiguous.  Returns the slot count.
static int32_t plan_slots(const std::vector<int32_t>& cam_sorted, int32_t m, int32_t chunk,
                          std::vector<int32_t>& chunk_slot, std::vector<int32_t>& cam_slot)
{
    const int64_t len = (int64_t)cam_sorted.size();
    const int32_t num_chunks = (int32_t)((len + chunk - 1) / chunk);
    chunk_slot.assign((size_t)num_chunks + 1, 0);
    std::vector<int32_t> per_cam((size_t)m, 0);
    int32_t slot = 0;
    for (int32_t c = 0; c < num_chunks; ++c) {
        chunk_slot[c] = slot;
        const int64_t s = (int64_t)c * chunk, e = std::min<int64_t>(len, s + chunk);
        for (int64_t t = s; t < e; ++t)
            if (t == s || cam_sorted[(size_t)t] != cam_sorted[(size_t)t - 1]) {
                per_cam[cam_sorted[(size_t)t]]++;
                ++slot;
            }
    }
    chunk_slot[num_chunks] = slot;
    cam_slot.assign((size_t)m + 1, 0);
    for (int32_t j = 0; j < m; ++j) cam_slot[(size_t)j + 1] = cam_slot[j] + per_cam[j];
    return slot;
}

static ba_status upload_state(ba_problem* P, const double* cameras, const double* points)
{
    const int32_t m = P->m, n = P->n;
    if (cameras) {
        std::vector<double> c((size_t)9 * m);
        for (int32_t j = 0; j < m; ++j)
            std::memcpy(&c[(size_t)9 * j], cameras + (size_t)9 * P->old_of_new[j], 9 * sizeof(double));
        BA_TRY(P, hipMemcpyAsync(P->cams, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, P->stream));
        BA_TRY(P, launch_camera_constants_f64(m, P->cams, P->ck64, P->stream));
        BA_TRY(P, hipStreamSynchronize(P->stream));
    }
    if (points && n > 0) {
        BA_TRY(P, hipMemcpyAsync(P->pts, points, (size_t)3 * n * sizeof(double), hipMemcpyHostToDevice, P->stream));
        BA_TRY(P, hipStreamSynchronize(P->stream));
    }
    return BA_OK;
}

extern "C" ba_status ba_create(int32_t m, int32_t n, int64_t N, const double* cameras, const double* points,
                               const int32_t* obs_camera, const int32_t* obs_point, const double* obs_uv,
                               const ba_options* opt_in, void* hip_stream, ba_problem** out)
{
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is NULL";
        return BA_EINVAL;
    }
    *out = nullptr;
    ba_options opt;
    if (opt_in) opt = *opt_in;
    else ba_options_default(&opt);
    std::string msg;
    if (check_options(&opt, msg) != BA_OK) {
        g_create_error = msg;
        return BA_EINVAL;
    }
    if (m < 1 || n < 0 || N < 0 || N >= ((int64_t)1 << 31)) {
        g_create_error = "invalid counts";
        return BA_EINVAL;
    }
    if (opt.solver == BA_SOLVER_DENSE && m > BA_DENSE_MAX_CAMERAS) {
        g_create_error = "the dense solver takes at most " + std::to_string(BA_DENSE_MAX_CAMERAS) + " cameras";
        return BA_EINVAL;
    }
    if (!cameras || (n > 0 && !points) || (N > 0 && (!obs_camera || !obs_point || !obs_uv))) {
        g_create_error = "NULL input array";
        return BA_EINVAL;
    }
    if (!finite_all(cameras, 9 * (int64_t)m) || (n > 0 && !finite_all(points, 3 * (int64_t)n)) ||
        (N > 0 && !finite_all(obs_uv, 2 * N))) {
        g_create_error = "non-finite input";
        return BA_EINVAL;
    }
    for (int64_t k = 0; k < N; ++k)
        if (obs_camera[k] < 0 || obs_camera[k] >= m || obs_point[k] < 0 || obs_point[k] >= n) {
            g_create_error = "observation index out of range at " + std::to_string(k);
            return BA_EINVAL;
        }

    ba_problem* P = new (std::nothrow) ba_problem();
    if (!P) {
        g_create_error = "host allocation failed";
        return BA_ENOMEM;
    }
    P->m = m;
    P->n = n;
    P->N = N;
    P->opt = opt;
    P->opt.pcg_schedule = nullptr;  // a create-time schedule pointer is not retained
    P->stream = (hipStream_t)hip_stream;

    // Cameras relabelled by popularity (most observed first), ties by id.
    std::vector<int64_t> ccount(m, 0);
    for (int64_t k = 0; k < N; ++k) ccount[obs_camera[k]]++;
    P->old_of_new.resize(m);
    P->new_of_old.resize(m);
    for (int32_t j = 0; j < m; ++j) P->old_of_new[j] = j;
    std::stable_sort(P->old_of_new.begin(), P->old_of_new.end(),
                     [&](int32_t a, int32_t b) { return ccount[a] > ccount[b]; });
    for (int32_t j = 0; j < m; ++j) P->new_of_old[P->old_of_new[j]] = j;

    // Point-major order: counting sort by point, then by camera within a point.
    std::vector<int64_t> poff((size_t)n + 1, 0);
    for (int64_t k = 0; k < N; ++k) poff[(size_t)obs_point[k] + 1]++;
    for (int32_t i = 0; i < n; ++i) poff[(size_t)i + 1] += poff[i];
    std::vector<int32_t> pm_order((size_t)N);
    {
        std::vector<int64_t> fill(poff.begin(), poff.end() - 1);
        for (int64_t k = 0; k < N; ++k) pm_order[(size_t)fill[obs_point[k]]++] = (int32_t)k;
    }
    std::vector<int32_t> h_pm_cam((size_t)N), h_pm_pt((size_t)N);
    for (int32_t i = 0; i < n; ++i) {
        auto b = pm_order.begin() + poff[i], e = pm_order.begin() + poff[(size_t)i + 1];
        std::stable_sort(b, e, [&](int32_t u, int32_t v) {
            return P->new_of_old[obs_camera[u]] < P->new_of_old[obs_camera[v]];
        });
    }
    std::vector<double> h_uvx((size_t)N), h_uvy((size_t)N);
    for (int64_t t = 0; t < N; ++t) {
        const int32_t k = pm_order[(size_t)t];
        h_pm_cam[(size_t)t] = P->new_of_old[obs_camera[k]];
        h_pm_pt[(size_t)t] = obs_point[k];
        h_uvx[(size_t)t] = obs_uv[2 * (int64_t)k];
        h_uvy[(size_t)t] = obs_uv[2 * (int64_t)k + 1];
    }
    // Point-aligned tiles of <= kTile observations; a longer point is a tile alone.
    std::vector<int32_t> tiles;
    tiles.push_back(0);
    {
        int64_t cur = 0;  // start of the open tile
        for (int32_t i = 0; i < n; ++i) {
            const int64_t a = poff[i], b = poff[(size_t)i + 1];
            if (b == a) continue;
            if (b - cur > kTile && a > cur) {
                tiles.push_back((int32_t)a);
                cur = a;
            }
            if (b - a > kTile) {  // long point: its own tile
                tiles.push_back((int32_t)b);
                cur = b;
            }
        }
        if (cur < N) tiles.push_back((int32_t)N);
    }
    P->pm.num_tiles = (int32_t)tiles.size() - 1;

    // Camera-major order: stable counting sort of the point-major stream by camera.
    std::vector<int64_t> coff((size_t)m + 1, 0);
    for (int64_t t = 0; t < N; ++t) coff[(size_t)h_pm_cam[(size_t)t] + 1]++;
    for (int32_t j = 0; j < m; ++j) coff[(size_t)j + 1] += coff[j];
    std::vector<int32_t> h_cm_cam((size_t)N), h_cm_pt((size_t)N);
    std::vector<double> h_cm_uvx((size_t)N), h_cm_uvy((size_t)N);
    {
        std::vector<int64_t> fill(coff.begin(), coff.end() - 1);
        for (int64_t t = 0; t < N; ++t) {
            const int32_t j = h_pm_cam[(size_t)t];
            const int64_t d = fill[j]++;
            h_cm_cam[(size_t)d] = j;
            h_cm_pt[(size_t)d] = h_pm_pt[(size_t)t];
            h_cm_uvx[(size_t)d] = h_uvx[(size_t)t];
            h_cm_uvy[(size_t)d] = h_uvy[(size_t)t];
        }
    }
    // rows of <= 64 observations that never span two cameras (a camera's
    // last row may be short), so a camera changes only between rows
    std::vector<int32_t> h_cm_row;
    for (int32_t j = 0; j < m; ++j)
        for (int64_t t = coff[j]; t < coff[(size_t)j + 1]; t += 64) h_cm_row.push_back((int32_t)t);
    h_cm_row.push_back((int32_t)N);
    P->cm.num_rows = (int32_t)h_cm_row.size() - 1;
    std::vector<int32_t> chunk_slot, cam_slot;
    {
        std::vector<int32_t> row_cam((size_t)P->cm.num_rows);
        for (int32_t r = 0; r < P->cm.num_rows; ++r) row_cam[(size_t)r] = h_cm_cam[(size_t)h_cm_row[(size_t)r]];
        P->cm.num_slots = plan_slots(row_cam, m, kCmRows, chunk_slot, cam_slot);
    }
    const int32_t num_chunks = (int32_t)chunk_slot.size() - 1;
    P->cm.num_chunks = num_chunks;
    std::vector<int32_t> seg_cam, seg_slot, cam_seg((size_t)m + 1, 0);
    for (int32_t j = 0; j < m; ++j) {
        for (int32_t sl = cam_slot[j]; sl < cam_slot[(size_t)j + 1]; sl += kSlotSeg) {
            seg_cam.push_back(j);
            seg_slot.push_back(sl);
        }
        cam_seg[(size_t)j + 1] = (int32_t)seg_cam.size();
    }
    P->cm.num_segs = (int32_t)seg_cam.size();

    // Schur-product schedule: hot cameras held in LDS, persistent workgroups
    // over short tiles, long tiles apart, cold observations camera-major.
    int dev = 0, cus = 0, lds_limit = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        g_create_error = "cannot query the HIP device";
        delete P;
        return BA_EDEVICE;
    }
    SchurPlan& sp = P->sp;
    {
        const char* stored = std::getenv("BA_SCHUR_STORED");
        sp.recompute = !(stored && std::atoi(stored) != 0);
        // recomputing product: the LDS holds the records of cameras [0, Kc)
        // and the hot table in the rest.  More records shorten the
        // point-major pass and fewer hot cameras lengthen the cold pass; at
        // 29M observations (Zipf) the PCG iteration took 0.462 / 0.444 /
        // 0.441 / 0.441 ms FP32 and 0.636 / 0.636 / 0.639 / 0.654 ms FP64
        // with 128 / 256 / 384 / 512 records.
        const size_t rec = P->is_f32() ? kCamRecBytes<float>() : kCamRecBytes<double>();
        const char* env_c = std::getenv("BA_CACHE_CAMERAS");
        const int32_t kc_default = P->is_f32() ? kCacheCamerasF32 : kCacheCamerasF64;
        if (!sp.recompute) sp.Kc = 0;
        else sp.Kc = std::max(0, std::min(m, env_c ? std::atoi(env_c) : kc_default));
        if (sp.Kc > 0 && (size_t)sp.Kc * rec + 1040 > (size_t)lds_limit)
            sp.Kc = (int32_t)(((size_t)lds_limit - 1040) / rec);
        int32_t kmax = P->is_f32() ? hot_max_cameras<float>((size_t)lds_limit, sp.Kc)
                                   : hot_max_cameras<double>((size_t)lds_limit, sp.Kc);
        const char* env = std::getenv("BA_HOT_CAMERAS");
        if (env) kmax = std::min(kmax, std::max(0, std::atoi(env)));
        sp.K = std::max(0, std::min(m, kmax));
        if (sp.K > 0 && !env) {
            // Keep the hot set only when it costs fewer observation visits per
            // product than none: N + rewalk + cold < 2N.  With a hot set, a long
            // point is walked again for its camera side: the stored-block pass
            // re-reads every tile it touches (plus the tile it resumes at); the
            // recomputing pass walks a point of more than 64 observations twice.
            // With none, that walk is skipped and the cold pass takes every
            // observation.
            int64_t rewalk = 0, cold = 0;
            for (int32_t i = 0; i < n; ++i) {
                const int64_t a = poff[i], b = poff[(size_t)i + 1];
                if (sp.recompute) {
                    if (b - a > 64) rewalk += b - a;
                } else if (b - a > 0 && ((b - 1) >> 6) >= (a >> 6) + 2) {
                    rewalk += (((b - 1) >> 6) - (a >> 6) + 2) * 64;
                }
            }
            for (int32_t j = sp.K; j < m; ++j) cold += coff[(size_t)j + 1] - coff[j];
            if (rewalk + cold > N) sp.K = 0;
        }
    }
    // line-aligned 64-observation tiles split evenly over the hot pass's
    // wavefronts; the point-major arrays end with one padding tile (point -1)
    P->pm.ld = ((N + 63) / 64 + 1) * 64;
    const int64_t ntiles64 = (N + 63) / 64;
    const int32_t waves_per_wg = sp.recompute
                                     ? (P->is_f32() ? FreeWgThreads<float>::value : FreeWgThreads<double>::value) / 64
                                     : (P->is_f32() ? HotThreads<float>::value : HotThreads<double>::value) / 64;
    sp.num_wg = 0;
    if (ntiles64 > 0)
        sp.num_wg = (int32_t)std::max<int64_t>(1, std::min<int64_t>(std::max(1, cus),
                                                                   (ntiles64 + waves_per_wg - 1) / waves_per_wg));
    const int32_t num_waves = sp.num_wg * waves_per_wg;
    std::vector<int32_t> wrange((size_t)num_waves + 1, 0);
    for (int32_t w = 0; w <= num_waves; ++w) wrange[(size_t)w] = (int32_t)((int64_t)w * ntiles64 / num_waves);
    // recomputing product: point-aligned segments, short (<= 64 observations of
    // whole points) and long (one point of more observations); each kind is
    // split over the wavefronts by observation count
    const int32_t free_waves = num_waves;
    std::vector<int2> sseg, lseg;
    std::vector<int32_t> frange((size_t)free_waves + 1, 0), lrange((size_t)free_waves + 1, 0);
    {
        int64_t open = -1, open_len = 0;  // the short segment being filled
        for (int32_t i = 0; i < n; ++i) {
            const int64_t a = poff[i], b = poff[(size_t)i + 1];
            if (b == a) continue;
            if (b - a > 64) {
                lseg.push_back(make_int2((int32_t)a, (int32_t)b));
                continue;
            }
            if (open >= 0 && open_len + (b - a) > 64) {
                sseg.push_back(make_int2((int32_t)open, (int32_t)(open + open_len)));
                open = -1;
            }
            if (open < 0) {
                open = a;
                open_len = 0;
            }
            // points of one short segment are contiguous: a long point closes it
            if (open + open_len != a) {
                sseg.push_back(make_int2((int32_t)open, (int32_t)(open + open_len)));
                open = a;
                open_len = 0;
            }
            open_len += b - a;
        }
        if (open >= 0) sseg.push_back(make_int2((int32_t)open, (int32_t)(open + open_len)));
        sp.num_short = (int32_t)sseg.size();
        sp.num_long = (int32_t)lseg.size();
        auto split = [&](const std::vector<int2>& v, std::vector<int32_t>& range) {
            std::vector<int64_t> cum(v.size() + 1, 0);
            for (size_t q = 0; q < v.size(); ++q) cum[q + 1] = cum[q] + (v[q].y - v[q].x);
            for (int32_t w = 0; w <= free_waves; ++w) {
                const int64_t target = cum.back() * w / std::max(1, free_waves);
                range[(size_t)w] = (int32_t)(std::lower_bound(cum.begin(), cum.end(), target) - cum.begin());
            }
            range[(size_t)free_waves] = (int32_t)v.size();
        };
        split(sseg, frange);
        split(lseg, lrange);
    }
    // the build: 32 wavefronts per CU over the same tiles
    // cold stream: observations on cameras >= K, camera-major
    // Each point with a cold observation has one record the cold pass gathers
    // (b_i, and for the recomputing product the point).  The recomputing
    // product numbers the records in order of first use by the cold stream,
    // so a point whose cold observations are few (most are) is read in
    // sequence with its neighbours in that stream (at 29M: 0.61 instead of
    // one 128-byte line per cold observation); the stored design keeps the
    // point's own index.
    std::vector<int32_t> h_cold_cam, h_cold_pt;
    std::vector<int32_t> crec((size_t)(n > 0 ? n : 1), -1);
    int32_t num_rec = 0;
    for (int64_t d = 0; d < N; ++d) {
        if (h_cm_cam[(size_t)d] >= sp.K) {
            const int32_t i = h_cm_pt[(size_t)d];
            if (crec[(size_t)i] < 0) crec[(size_t)i] = sp.recompute ? num_rec++ : i;
            h_cold_cam.push_back(h_cm_cam[(size_t)d]);
            h_cold_pt.push_back(crec[(size_t)i]);
        }
    }
    sp.cold.N = (int64_t)h_cold_cam.size();
    if (std::getenv("BA_VERBOSE"))
        std::fprintf(stderr,
                     "[ba] m=%d n=%d N=%lld cus=%d lds/block=%d hot K=%d wg=%d tiles=%lld cold obs=%lld (%.2f%%) "
                     "product=%s segments=%d\n",
                     m, n, (long long)N, cus, lds_limit, sp.K, sp.num_wg, (long long)ntiles64, (long long)sp.cold.N,
                     N > 0 ? 100.0 * (double)sp.cold.N / (double)N : 0.0, sp.recompute ? "recompute" : "stored",
                     sp.num_short + sp.num_long);
    std::vector<int32_t> cold_chunk_slot, cold_cam_slot;
    sp.cold.num_slots = plan_slots(h_cold_cam, m, kColdChunk, cold_chunk_slot, cold_cam_slot);
    sp.cold.num_chunks = (int32_t)cold_chunk_slot.size() - 1;

    // Workspace: everything the solve needs, sized once.
    DevAlloc& A = P->mem;
    const size_t tsz = P->is_f32() ? sizeof(float) : sizeof(double);
    P->cams = A.get<double>(9 * (int64_t)m);
    P->cams_t = A.get<double>(9 * (int64_t)m);
    P->pts = A.get<double>(3 * (int64_t)n);
    P->pts_t = A.get<double>(3 * (int64_t)n);
    P->ck64 = A.get<CamK<double>>(m);
    P->ck64_t = A.get<CamK<double>>(m);
    P->ck32 = A.get<CamK<float>>(m);
    P->d_old_of_new = A.get<int32_t>(m);
    P->pm.cam = A.get<int32_t>(P->pm.ld);
    P->pm.pt = A.get<int32_t>(P->pm.ld);
    P->pm.uvx = A.get<double>(N);
    P->pm.uvy = A.get<double>(N);
    P->pm.tile = A.get<int32_t>((int64_t)tiles.size());
    P->cm.cam = A.get<int32_t>(N);
    P->cm.pt = A.get<int32_t>(N);
    P->cm.uvx = A.get<double>(N);
    P->cm.uvy = A.get<double>(N);
    P->cm.row = A.get<int32_t>((int64_t)P->cm.num_rows + 1);
    P->cm.chunk_slot = A.get<int32_t>((int64_t)num_chunks + 1);
    P->cm.cam_slot = A.get<int32_t>((int64_t)m + 1);
    P->cm.slots = A.get<double>((int64_t)P->cm.num_slots * kCamSlotWords);
    P->cm.seg_cam = A.get<int32_t>(P->cm.num_segs);
    P->cm.seg_slot = A.get<int32_t>(P->cm.num_segs);
    P->cm.cam_seg = A.get<int32_t>((int64_t)m + 1);
    P->cm.seg_part = A.get<double>((int64_t)P->cm.num_segs * kCamSlotWords);
    P->cm.arrive = A.get<uint32_t>(m);
    // point-major E is stored only for the stored-block product
    P->hcp = sp.recompute ? nullptr : A.get<char>(27 * P->pm.ld * (int64_t)tsz);
    P->hpp = A.get<char>(6 * (int64_t)n * (int64_t)sizeof(double));
    P->cinv = A.get<char>(6 * (int64_t)n * (int64_t)tsz);
    P->wpt = A.get<double>(3 * (int64_t)n);
    P->hcc = A.get<double>(81 * (int64_t)m);
    P->vcam = A.get<double>(9 * (int64_t)m);
    P->bd = A.get<double>(81 * (int64_t)m);
    P->lfac = A.get<double>(45 * (int64_t)m);
    P->mj = A.get<double>(81 * (int64_t)m);
    P->dcam = A.get<double>(9 * (int64_t)m);
    for (double** v : {&P->g, &P->x, &P->r, &P->z, &P->p, &P->q, &P->cacc}) *v = A.get<double>(9 * (int64_t)m);
    P->pT = A.get<char>(9 * (int64_t)m * (int64_t)tsz);
    sp.wrange = A.get<int32_t>((int64_t)wrange.size());
    sp.sseg = A.get<int2>(std::max<int64_t>(1, (int64_t)sseg.size()));
    sp.lseg = A.get<int2>(std::max<int64_t>(1, (int64_t)lseg.size()));
    P->pm.sseg = sp.sseg;
    P->pm.lseg = sp.lseg;
    P->pm.num_short = sp.num_short;
    P->pm.num_long = sp.num_long;
    P->pm.num_cameras = m;
    sp.frange = A.get<int32_t>((int64_t)frange.size());
    sp.lrange = A.get<int32_t>((int64_t)lrange.size());
    P->wobs = A.get<char>(P->pm.ld * (int64_t)tsz);
    P->xf = A.get<char>(12 * (int64_t)m * (int64_t)tsz);
    sp.crec = A.get<int32_t>(std::max<int64_t>(1, n));
    sp.rec_pt = A.get<int32_t>(std::max<int64_t>(1, n));
    sp.hot_part = A.get<double>((int64_t)sp.num_wg * sp.K * 9);
    sp.hot_fold = A.get<double>((int64_t)kHotFold * sp.K * 9);
    sp.bcold = A.get<char>(kBcold * (int64_t)n * (int64_t)tsz);
    sp.cold.cam = A.get<int32_t>(sp.cold.N);
    sp.cold.pt = A.get<int32_t>(sp.cold.N);
    sp.cold.hcp = sp.recompute ? nullptr : A.get<char>(27 * sp.cold.N * (int64_t)tsz);
    sp.cold.w = sp.recompute ? A.get<char>(sp.cold.N * (int64_t)tsz) : nullptr;
    sp.cold.chunk_slot = A.get<int32_t>((int64_t)sp.cold.num_chunks + 1);
    sp.cold.cam_slot = A.get<int32_t>((int64_t)m + 1);
    sp.cold.slots = A.get<double>((int64_t)sp.cold.num_slots * 9);
    P->dp = A.get<double>(3 * (int64_t)n);
    P->partials = A.get<double>(2 * 2048);
    P->sums = A.get<double>(8);
    P->sc = A.get<PcgScalars>(1);
    P->flag = A.get<int32_t>(4);  // [failure bits, a failing camera, a failing point, unused]
    if (opt.solver == BA_SOLVER_DENSE) {
        P->S = A.get<double>(81 * (int64_t)m * m);
        int64_t np = 0;
        for (int32_t j = 0; j < m; ++j)
            np += std::max<int64_t>(1, (coff[(size_t)j + 1] - coff[j] + kDensePiece - 1) / kDensePiece);
        P->dense.num_pieces = (int32_t)np;
        P->dense.pieces = A.get<int4>(np);
        P->dense.coff = A.get<int32_t>((int64_t)m + 1);
        P->dense.cm_pm = A.get<int32_t>(N);
        P->dense.poff = A.get<int32_t>((int64_t)n + 1);
        P->dense.E = A.get<double>(27 * N);
    }
    if (A.err != hipSuccess) {
        g_create_error = std::string("device allocation failed: ") + hipGetErrorString(A.err);
        const bool oom = A.err == hipErrorOutOfMemory || A.err == hipErrorMemoryAllocation;
        A.release();
        delete P;
        return oom ? BA_ENOMEM : BA_EDEVICE;
    }
    if (hipHostMalloc((void**)&P->h_scalars, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        g_create_error = "pinned host allocation failed";
        A.release();
        delete P;
        return BA_ENOMEM;
    }
    if (hipEventCreateWithFlags(&P->sync_ev, hipEventDisableTiming) != hipSuccess) {
        g_create_error = "event creation failed";
        A.release();
        (void)hipHostFree(P->h_scalars);
        delete P;
        return BA_EDEVICE;
    }
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(P->d_old_of_new, P->old_of_new.data(), sizeof(int32_t) * m);
    h_pm_cam.resize((size_t)P->pm.ld, 0);
    h_pm_pt.resize((size_t)P->pm.ld, -1);
    if (e == hipSuccess) e = up(P->pm.cam, h_pm_cam.data(), sizeof(int32_t) * (size_t)P->pm.ld);
    if (e == hipSuccess) e = up(P->pm.pt, h_pm_pt.data(), sizeof(int32_t) * (size_t)P->pm.ld);
    if (e == hipSuccess && P->hcp) e = hipMemset(P->hcp, 0, 27 * (size_t)P->pm.ld * tsz);
    if (e == hipSuccess) e = up(P->pm.uvx, h_uvx.data(), sizeof(double) * N);
    if (e == hipSuccess) e = up(P->pm.uvy, h_uvy.data(), sizeof(double) * N);
    if (e == hipSuccess) e = up(P->pm.tile, tiles.data(), sizeof(int32_t) * tiles.size());
    if (e == hipSuccess) e = up(P->cm.cam, h_cm_cam.data(), sizeof(int32_t) * N);
    if (e == hipSuccess) e = up(P->cm.pt, h_cm_pt.data(), sizeof(int32_t) * N);
    if (e == hipSuccess) e = up(P->cm.uvx, h_cm_uvx.data(), sizeof(double) * N);
    if (e == hipSuccess) e = up(P->cm.uvy, h_cm_uvy.data(), sizeof(double) * N);
    if (e == hipSuccess) e = up(P->cm.row, h_cm_row.data(), sizeof(int32_t) * h_cm_row.size());
    if (e == hipSuccess) e = up(P->cm.chunk_slot, chunk_slot.data(), sizeof(int32_t) * chunk_slot.size());
    if (e == hipSuccess) e = up(P->cm.cam_slot, cam_slot.data(), sizeof(int32_t) * cam_slot.size());
    if (e == hipSuccess) e = up(P->cm.seg_cam, seg_cam.data(), sizeof(int32_t) * seg_cam.size());
    if (e == hipSuccess) e = up(P->cm.seg_slot, seg_slot.data(), sizeof(int32_t) * seg_slot.size());
    if (e == hipSuccess) e = up(P->cm.cam_seg, cam_seg.data(), sizeof(int32_t) * cam_seg.size());
    if (e == hipSuccess) e = hipMemset(P->cm.arrive, 0, sizeof(uint32_t) * (size_t)m);
    if (e == hipSuccess) e = hipMemset(P->hcc, 0, sizeof(double) * 81 * (size_t)m);
    if (e == hipSuccess) e = hipMemset(P->mj, 0, sizeof(double) * 81 * (size_t)m);  // unseen cameras: no term
    if (e == hipSuccess) e = hipMemset(P->vcam, 0, sizeof(double) * 9 * (size_t)m);
    if (e == hipSuccess) e = up(sp.wrange, wrange.data(), sizeof(int32_t) * wrange.size());
    if (e == hipSuccess && !sseg.empty()) e = up(sp.sseg, sseg.data(), sizeof(int2) * sseg.size());
    if (e == hipSuccess && !lseg.empty()) e = up(sp.lseg, lseg.data(), sizeof(int2) * lseg.size());
    if (e == hipSuccess) e = up(sp.frange, frange.data(), sizeof(int32_t) * frange.size());
    if (e == hipSuccess) e = up(sp.lrange, lrange.data(), sizeof(int32_t) * lrange.size());
    if (e == hipSuccess && opt.solver == BA_SOLVER_DENSE) {
        // camera-major entry d holds point-major observation cm_pm[d]
        std::vector<int32_t> h_coff((size_t)m + 1), h_cm_pm((size_t)N), h_poff((size_t)n + 1);
        for (int32_t j = 0; j <= m; ++j) h_coff[(size_t)j] = (int32_t)coff[(size_t)j];
        for (int32_t i = 0; i <= n; ++i) h_poff[(size_t)i] = (int32_t)poff[(size_t)i];
        std::vector<int64_t> fill(coff.begin(), coff.end() - 1);
        for (int64_t t = 0; t < N; ++t) h_cm_pm[(size_t)fill[h_pm_cam[(size_t)t]]++] = (int32_t)t;
        std::vector<int4> h_pieces;
        for (int32_t j = 0; j < m; ++j) {
            const int32_t a = h_coff[(size_t)j], b = h_coff[(size_t)j + 1];
            const int32_t np = std::max(1, (b - a + kDensePiece - 1) / kDensePiece);
            for (int32_t q = 0; q < np; ++q)
                h_pieces.push_back(make_int4(j, a + q * kDensePiece, std::min(b, a + (q + 1) * kDensePiece), np));
        }
        e = up(P->dense.coff, h_coff.data(), sizeof(int32_t) * h_coff.size());
        if (e == hipSuccess) e = up(P->dense.pieces, h_pieces.data(), sizeof(int4) * h_pieces.size());
        if (e == hipSuccess) e = up(P->dense.cm_pm, h_cm_pm.data(), sizeof(int32_t) * h_cm_pm.size());
        if (e == hipSuccess) e = up(P->dense.poff, h_poff.data(), sizeof(int32_t) * h_poff.size());
    }
    if (e == hipSuccess) e = hipMemset(P->wobs, 0, (size_t)P->pm.ld * tsz);
    if (e == hipSuccess) e = hipMemset(P->xf, 0, 12 * (size_t)m * tsz);
    if (e == hipSuccess && n > 0) e = up(sp.crec, crec.data(), sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess && n > 0) {
        std::vector<int32_t> rec_pt((size_t)n, 0);
        for (int32_t i = 0; i < n; ++i)
            if (crec[(size_t)i] >= 0) rec_pt[(size_t)crec[(size_t)i]] = i;
        e = up(sp.rec_pt, rec_pt.data(), sizeof(int32_t) * (size_t)n);
    }
    if (e == hipSuccess) e = up(sp.cold.cam, h_cold_cam.data(), sizeof(int32_t) * h_cold_cam.size());
    if (e == hipSuccess) e = up(sp.cold.pt, h_cold_pt.data(), sizeof(int32_t) * h_cold_pt.size());
    if (e == hipSuccess) e = up(sp.cold.chunk_slot, cold_chunk_slot.data(), sizeof(int32_t) * cold_chunk_slot.size());
    if (e == hipSuccess) e = up(sp.cold.cam_slot, cold_cam_slot.data(), sizeof(int32_t) * cold_cam_slot.size());
    if (e == hipSuccess)
        e = P->is_f32() ? prepare_schur_kernels<float>(sp.K, sp.Kc, sp.recompute)
                        : prepare_schur_kernels<double>(sp.K, sp.Kc, sp.recompute);
    if (e == hipSuccess) e = prepare_cost_kernels();
    if (e == hipSuccess) e = hipMemset(P->hpp, 0, 6 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    if (e == hipSuccess) e = hipMemset(P->wpt, 0, 3 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    // the back-substitution writes only points with observations: the step
    // of a point with none stays zero (its C_i and w_i are zero)
    if (e == hipSuccess) e = hipMemset(P->dp, 0, 3 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    if (e == hipSuccess) e = hipMemset(P->sc, 0, sizeof(PcgScalars));
    if (e == hipSuccess) e = hipMemset(P->flag, 0, 4 * sizeof(int32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        g_create_error = std::string("device upload failed: ") + hipGetErrorString(e);
        ba_destroy(P);
        return BA_EDEVICE;
    }
    ba_status st = upload_state(P, cameras, points);
    if (st != BA_OK) {
        g_create_error = P->last_error;
        ba_destroy(P);
        return st;
    }
    *out = P;
    return BA_OK;
}

extern "C" ba_status ba_set_params(ba_problem* P, const double* cameras, const double* points)
{
    if (!P) return BA_EINVAL;
    if ((cameras && !finite_all(cameras, 9 * (int64_t)P->m)) || (points && !finite_all(points, 3 * (int64_t)P->n))) {
        P->last_error = "non-finite parameters";
        return BA_EINVAL;
    }
    return upload_state(P, cameras, points);
}

extern "C" ba_status ba_get_params(const ba_problem* Pc, double* cameras, double* points)
{
    if (!Pc) return BA_EINVAL;
    ba_problem* P = const_cast<ba_problem*>(Pc);
    BA_TRY(P, hipStreamSynchronize(P->stream));
    if (cameras) {
        std::vector<double> c((size_t)9 * P->m);
        BA_TRY(P, hipMemcpy(c.data(), P->cams, c.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int32_t j = 0; j < P->m; ++j)
            std::memcpy(cameras + (size_t)9 * P->old_of_new[j], &c[(size_t)9 * j], 9 * sizeof(double));
    }
    if (points && P->n > 0)
        BA_TRY(P, hipMemcpy(points, P->pts, (size_t)3 * P->n * sizeof(double), hipMemcpyDeviceToHost));
    return BA_OK;
}

// ------------------------------------------------------------- helpers
// Waits for everything queued so far on the problem's stream by polling an
// event: a blocking synchronisation wakes the host some 30 us after the
// work ends, and the solve waits once per batch of PCG iterations and a few
// times per LM iteration, with the GPU idle until the next launch.
static hipError_t wait_stream(ba_problem* P)
{
    hipError_t e = hipEventRecord(P->sync_ev, P->stream);
    if (e != hipSuccess) return e;
    while ((e = hipEventQuery(P->sync_ev)) == hipErrorNotReady) {
    }
    return e;
}

static ba_status read_scalars(ba_problem* P, const void* dev, size_t bytes)
{
    BA_TRY(P, hipMemcpyAsync(P->h_scalars, dev, bytes, hipMemcpyDeviceToHost, P->stream));
    BA_TRY(P, wait_stream(P));
    return BA_OK;
}

// F at (pts, ck) summed in FP64 into P->sums[0]
template <typename T>
static ba_status cost_into_sums(ba_problem* P, const double* pts, const CamK<T>* ck, hipStream_t s)
{
    int32_t nb = 0;
    if (P->N == 0) {
        BA_TRY(P, launch_zero(P->sums, 1, s));
        return BA_OK;
    }
    BA_TRY(P, launch_cost_t<T>(P->pm, P->N, pts, ck, P->opt.huber_delta, P->partials, &nb, s));
    BA_TRY(P, launch_sum_partials(P->partials, nb, 1, 1, P->sums, s));
    return BA_OK;
}

// Camera constants of the current state in T (FP32: refreshed by each build).
template <typename T>
static const CamK<T>* state_ck(const ba_problem* P)
{
    if constexpr (sizeof(T) == 4)
        return (const CamK<T>*)P->ck32;
    else
        return (const CamK<T>*)P->ck64;
}

template <typename T>
static RecomputeInputs<T> recompute_inputs(const ba_problem* P)
{
    return RecomputeInputs<T>{(const T*)P->wobs, P->pts, state_ck<T>(P), (const T*)P->xf,
                              sizeof(T) == 4 ? P->ck64 : nullptr};
}

// Where the Jacobian comes from at the current state (the build refreshes
// the FP32 camera constants first).
template <typename T>
static JacSource<T> jac_source(const ba_problem* P)
{
    return JacSource<T>{state_ck<T>(P), P->opt.jacobian == BA_JACOBIAN_AUTODIFF ? P->cams : nullptr,
                        sizeof(T) == 4 ? P->ck64 : nullptr};
}

template <typename T>
static ba_status build_system(ba_problem* P)
{
    hipStream_t s = P->stream;
    const CamK<T>* ck;
    if constexpr (sizeof(T) == 4) {
        BA_TRY(P, launch_camera_constants_f32(P->m, P->cams, P->ck32, s));
        ck = (const CamK<T>*)P->ck32;
    } else {
        ck = (const CamK<T>*)P->ck64;
    }
    const JacSource<T> js{ck, P->opt.jacobian == BA_JACOBIAN_AUTODIFF ? P->cams : nullptr,
                          sizeof(T) == 4 ? P->ck64 : nullptr};
    BA_TRY(P, launch_build_points<T>(P->pm, P->opt.huber_delta, false, P->pts, js, (T*)P->hcp, (double*)P->hpp,
                                     P->wpt, (T*)P->wobs, s));
    BA_TRY(P, launch_build_cameras<T>(P->cm, P->m, P->N, P->pts, js, P->opt.huber_delta, false, P->hcc, P->vcam,
                                      P->sp.cold.N, (T*)P->sp.cold.hcp, (T*)P->sp.cold.w, s));
    if (P->sp.recompute) BA_TRY(P, launch_cold_points<T>(P->sp, P->n, P->pts, s));
    return BA_OK;
}

// With time_kernels, the PCG loop brackets every kTimedStride-th matvec with events.
constexpr int32_t kTimedStride = 8;

struct PcgTimer {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    ~PcgTimer()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipError_t next(hipEvent_t* a, hipEvent_t* b)
    {
        while (ev.size() < used + 2) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev.push_back(e);
        }
        *a = ev[used];
        *b = ev[used + 1];
        used += 2;
        return hipSuccess;
    }
};

// PCG on the reduced camera system (Alg. 2, one partition); dc = x.  The
// stopping test runs on the device before every matvec (the loop test of Alg. 2);
// the host enqueues iterations in batches and reads the `done` flag between
// batches.  With a fixed count everything is enqueued at once.
template <typename T>
static ba_status run_pcg(ba_problem* P, const ba_options& o, int32_t fixed, int32_t* iters, int32_t* stop,
                         PcgTimer* tm, double* matvec_ms, double* hot_ms, int64_t* launches)
{
    hipStream_t s = P->stream;
    const int32_t m = P->m;
    const int32_t cap = fixed > 0 ? fixed : o.max_pcg_iters;
    BA_TRY(P, launch_pcg_reset(P->sc, o.pcg_rtol, o.max_pcg_iters, fixed, s));
    // b = v - E C^-1 w; x = 0; r = b; ||b||^2; then z = M^-1 r and the first test
    const RecomputeInputs<T> ri = recompute_inputs<T>(P);
    T* xf = P->sp.recompute ? (T*)P->xf : nullptr;
    BA_TRY(P, launch_schur_product<T>(1, P->sp, P->pm, P->N, (const T*)P->hcp, (const T*)P->cinv, P->wpt, nullptr,
                                      &ri, m, P->bd, nullptr, P->vcam, P->g, P->x, P->r, P->partials, P->sc,
                                      nullptr, nullptr, s));
    BA_TRY(P, launch_pcg_step(m, true, P->lfac, P->p, P->q, P->x, P->r, P->z, P->partials, P->sc, s));
    // timed matvecs: every kTimedStride-th (each event marker costs the stream
    // a few microseconds: timing all of them made a PCG iteration 3% longer)
    struct Mark {
        int32_t iter;
        std::array<hipEvent_t, 4> ev;
    };
    std::vector<Mark> marks;
    const int32_t batch = fixed > 0 ? std::max(1, cap) : 8;
    int32_t enqueued = 0;
    while (enqueued < cap) {
        const int32_t nb = std::min(batch, cap - enqueued);
        for (int32_t b = 0; b < nb; ++b) {
            BA_TRY(P, launch_pcg_direction<T>(m, false, P->z, P->p, (T*)P->pT, ri.ck, xf, P->sc, s));
            const bool timed = tm && enqueued % kTimedStride == 0;
            std::array<hipEvent_t, 4> ev{nullptr, nullptr, nullptr, nullptr};
            if (timed) {
                BA_TRY(P, tm->next(&ev[0], &ev[1]));
                BA_TRY(P, tm->next(&ev[2], &ev[3]));
                BA_TRY(P, hipEventRecord(ev[0], s));
            }
            BA_TRY(P, launch_schur_product<T>(0, P->sp, P->pm, P->N, (const T*)P->hcp, (const T*)P->cinv, P->wpt,
                                              (const T*)P->pT, &ri, m, P->bd, P->p, nullptr, P->q, nullptr, nullptr,
                                              P->partials, P->sc, ev[2], ev[3], s));
            if (timed) {
                BA_TRY(P, hipEventRecord(ev[1], s));
                marks.push_back(Mark{enqueued, ev});
            }
            BA_TRY(P, launch_pcg_step(m, false, P->lfac, P->p, P->q, P->x, P->r, P->z, P->partials, P->sc, s));
            ++enqueued;
        }
        ba_status st = read_scalars(P, P->sc, sizeof(PcgScalars));
        if (st != BA_OK) return st;
        if (((const PcgScalars*)P->h_scalars)->done) break;
    }
    ba_status st = read_scalars(P, P->sc, sizeof(PcgScalars));
    if (st != BA_OK) return st;
    const PcgScalars* h = (const PcgScalars*)P->h_scalars;
    *iters = h->iters;
    if (h->breakdown)
        *stop = BA_PCG_BREAKDOWN;
    else if (fixed > 0)
        *stop = BA_PCG_FIXED;
    else
        *stop = h->iters >= o.max_pcg_iters ? BA_PCG_CAP : BA_PCG_CONVERGED;
    // A breakdown (p^T q <= 0 or non-finite) stops the loop before that
    // update, so x holds the last iterate: it is used as the step (truncated CG).
    // matvecs run in order: those enqueued before the count reached did real work
    for (size_t u = 0; u < marks.size() && marks[u].iter < h->iters; ++u) {
        float ms = 0.0f, hms = 0.0f;
        BA_TRY(P, hipEventElapsedTime(&ms, marks[u].ev[0], marks[u].ev[1]));
        BA_TRY(P, hipEventElapsedTime(&hms, marks[u].ev[2], marks[u].ev[3]));
        *matvec_ms += ms;
        *hot_ms += hms;
        *launches += 1;
    }
    if (tm) tm->used = 0;
    return BA_OK;
}

// The direct option: g = v - E C~^-1 w by the same product as PCG's right-hand
// side, then dc = x = S^-1 g with S written out and factored.  A reduced system
// that is not positive definite ends the solve (BA_ENUMERIC).
template <typename T>
static ba_status run_dense(ba_problem* P, double lambda)
{
    hipStream_t s = P->stream;
    const RecomputeInputs<T> ri = recompute_inputs<T>(P);
    BA_TRY(P, launch_pcg_reset(P->sc, 0.0, 0, 0, s));
    BA_TRY(P, launch_schur_product<T>(1, P->sp, P->pm, P->N, (const T*)P->hcp, (const T*)P->cinv, P->wpt, nullptr,
                                      &ri, P->m, P->bd, nullptr, P->vcam, P->g, P->x, P->r, P->partials, P->sc,
                                      nullptr, nullptr, s));
    // the per-observation (diagonal) terms come from the camera-major pass
    BA_TRY(P, launch_schur_jacobi_terms<T>(P->cm, P->N, P->pts, jac_source<T>(P), P->opt.huber_delta,
                                           (const T*)P->cinv, P->mj, s));
    BA_TRY(P, launch_dense_solve<T>(P->dense, P->pm, P->N, ri, (const T*)P->cinv, P->m, P->bd, P->mj, P->g, P->x,
                                    P->S, P->flag, s));
    BA_TRY(P, hipMemcpyAsync(P->h_scalars, P->flag, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BA_TRY(P, hipStreamSynchronize(s));
    if (*(const int32_t*)P->h_scalars & 4) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "damped reduced camera system not positive definite at lambda %.3e", lambda);
        P->last_error = buf;
        BA_TRY(P, hipMemsetAsync(P->flag, 0, 4 * sizeof(int32_t), s));
        return BA_ENUMERIC;
    }
    return BA_OK;
}

template <typename T>
static ba_status lm_solve_t(ba_problem* P, const ba_options& o, ba_report* rep)
{
    using clock = std::chrono::steady_clock;
    hipStream_t s = P->stream;
    const int32_t m = P->m, n = P->n;
    const auto t_start = clock::now();
    ba_status st;
    BA_TRY(P, hipStreamSynchronize(s));
    if ((st = cost_into_sums<double>(P, P->pts, P->ck64, s)) != BA_OK) return st;
    if ((st = read_scalars(P, P->sums, sizeof(double))) != BA_OK) return st;
    double F = P->h_scalars[0];
    double lambda = o.lambda_init, nu = 2.0;
    bool need_build = true;
    double pcg_ms = 0.0, matvec_ms = 0.0, hot_ms = 0.0;
    int64_t pcg_total = 0, launches = 0;
    PcgTimer timer;
    if (rep) {
        rep->initial_cost = F;
        rep->iters_run = 0;
    }
    int32_t it = 0;
    ba_status result = BA_OK;
    for (it = 0; it < o.max_lm_iters; ++it) {
        const auto t_it = clock::now();
        if (need_build) {
            if ((st = build_system<T>(P)) != BA_OK) return st;
            need_build = false;
        }
        BA_TRY(P, launch_damp_cameras(m, P->hcc, lambda, o.damping, P->bd, P->lfac, P->dcam, P->flag, s));
        BA_TRY(P, launch_damp_points<T>(n, (const double*)P->hpp, lambda, o.damping, (T*)P->cinv, P->flag, s));
        if (P->opt.solver == BA_SOLVER_PCG && o.preconditioner == BA_PRECOND_SCHUR_JACOBI) {
            BA_TRY(P, launch_schur_jacobi_terms<T>(P->cm, P->N, P->pts, jac_source<T>(P), o.huber_delta,
                                                   (const T*)P->cinv, P->mj, s));
            BA_TRY(P, launch_factor_schur_jacobi(m, P->bd, P->mj, P->lfac, P->flag, s));
        }
        BA_TRY(P, hipMemcpyAsync(P->h_scalars, P->flag, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BA_TRY(P, wait_stream(P));
        if (*(const int32_t*)P->h_scalars != 0) {
            P->last_error = not_pd_message(P, (const int32_t*)P->h_scalars, lambda,
                                           P->opt.solver == BA_SOLVER_PCG && o.preconditioner == BA_PRECOND_SCHUR_JACOBI);
            BA_TRY(P, hipMemsetAsync(P->flag, 0, 4 * sizeof(int32_t), s));
            result = BA_ENUMERIC;
            break;
        }
        const int32_t fixed = o.pcg_schedule ? o.pcg_schedule[it] : o.pcg_fixed_iters;
        int32_t npcg = 0, stop = BA_PCG_DIRECT;
        const auto t_pcg = clock::now();
        if (P->opt.solver == BA_SOLVER_DENSE)
            st = run_dense<T>(P, lambda);
        else
            st = run_pcg<T>(P, o, fixed, &npcg, &stop, o.time_kernels ? &timer : nullptr, &matvec_ms, &hot_ms,
                            &launches);
        pcg_ms += std::chrono::duration<double, std::milli>(clock::now() - t_pcg).count();
        pcg_total += npcg;
        if (st != BA_OK) {
            if (rep && rep->pcg_iters && it < rep->capacity) rep->pcg_iters[it] = npcg;
            result = st;
            break;
        }
        // dp = C~^-1 (w - E^T dc); trial state; F(x + dx); predicted decrease
        if (P->sp.recompute) {
            const RecomputeInputs<T> ri = recompute_inputs<T>(P);
            BA_TRY(P, launch_pcg_direction<T>(m, true, P->x, P->p, (T*)P->pT, ri.ck, (T*)P->xf, P->sc, s));
            BA_TRY(P, launch_backsub_free<T>(P->sp, P->pm, ri, (const T*)P->cinv, P->wpt, P->dp, s));
        } else {
            BA_TRY(P, launch_pcg_direction<T>(m, true, P->x, P->p, (T*)P->pT, nullptr, nullptr, P->sc, s));
            BA_TRY(P, launch_backsub_stored<T>(P->pm, (const T*)P->hcp, (const T*)P->cinv, P->wpt,
                                               (const T*)P->pT, P->dp, s));
        }
        BA_TRY(P, launch_trial_state(m, n, P->cams, P->x, P->pts, P->dp, P->cams_t, P->pts_t, s));
        BA_TRY(P, launch_camera_constants_f64(m, P->cams_t, P->ck64_t, s));
        if ((st = cost_into_sums<double>(P, P->pts_t, P->ck64_t, s)) != BA_OK) return st;
        int32_t nb = 0;
        BA_TRY(P, launch_pred<T>(m, n, P->x, P->dcam, P->vcam, P->dp, (const double*)P->hpp, P->wpt, lambda, o.damping,
                                 P->partials, &nb, s));
        BA_TRY(P, launch_sum_partials(P->partials, nb, 2, 2, P->sums + 1, s));
        if ((st = read_scalars(P, P->sums, 3 * sizeof(double))) != BA_OK) return st;
        const double Ft = P->h_scalars[0];
        const double pred = 0.5 * (P->h_scalars[1] + P->h_scalars[2]);
        const double gain = (F - Ft) / pred;
        const bool acc = pred > 0.0 && std::isfinite(Ft) && gain > o.min_relative_decrease;
        if (rep) {
            if (it < rep->capacity) {
                if (rep->lambda) rep->lambda[it] = lambda;
                if (rep->trial_cost) rep->trial_cost[it] = Ft;
                if (rep->pred) rep->pred[it] = pred;
                if (rep->pcg_iters) rep->pcg_iters[it] = npcg;
                if (rep->accepted) rep->accepted[it] = acc ? 1 : 0;
                if (rep->pcg_stop) rep->pcg_stop[it] = stop;
            }
        }
        if (acc) {
            std::swap(P->cams, P->cams_t);
            std::swap(P->pts, P->pts_t);
            std::swap(P->ck64, P->ck64_t);
            F = Ft;
            const double t = 2.0 * gain - 1.0;
            const double f = 1.0 - t * t * t;
            lambda *= (f > 1.0 / 3.0 ? f : 1.0 / 3.0);
            nu = 2.0;
            need_build = true;
        } else {
            lambda *= nu;
            nu *= 2.0;
        }
        if (rep && it < rep->capacity) {
            if (rep->cost) rep->cost[it] = F;
            if (rep->ms) rep->ms[it] = std::chrono::duration<double, std::milli>(clock::now() - t_it).count();
        }
        if (lambda > 1e32) {  // no further progress possible: normal end
            ++it;
            break;
        }
    }
    if (rep) {
        rep->iters_run = it;
        rep->final_cost = F;
        rep->total_ms = std::chrono::duration<double, std::milli>(clock::now() - t_start).count();
        rep->pcg_ms = pcg_ms;
        rep->pcg_iters_total = pcg_total;
        rep->matvec_ms = matvec_ms;
        rep->matvec_launches = launches;
        rep->schur_hot_ms = hot_ms;
    }
    return result;
}

extern "C" ba_status ba_lm_solve(ba_problem* P, const ba_options* opt, ba_report* rep)
{
    if (!P) return BA_EINVAL;
    ba_options o = opt ? *opt : P->opt;
    std::string msg;
    if (check_options(&o, msg) != BA_OK) {
        P->last_error = msg;
        return BA_EINVAL;
    }
    if (o.precision != P->opt.precision) {
        P->last_error = "precision differs from the create-time precision";
        return BA_EINVAL;
    }
    if (o.solver != P->opt.solver) {
        P->last_error = "solver differs from the create-time solver";
        return BA_EINVAL;
    }
    if (rep && rep->capacity < 0) {
        P->last_error = "negative report capacity";
        return BA_EINVAL;
    }
    const double delta_saved = P->opt.huber_delta;
    const int32_t jacobian_saved = P->opt.jacobian;
    P->opt.huber_delta = o.huber_delta;
    P->opt.jacobian = o.jacobian;
    ba_status st = P->is_f32() ? lm_solve_t<float>(P, o, rep) : lm_solve_t<double>(P, o, rep);
    P->opt.huber_delta = delta_saved;
    P->opt.jacobian = jacobian_saved;
    return st;
}

// --------------------------------------------------- cost and gradients
template <typename T>
static ba_status grad_into(ba_problem* P, const double* cams, const double* pts, const CamK<T>* ck,
                           const CamK<double>* ck64, hipStream_t s)
{
    const JacSource<T> js{ck, P->opt.jacobian == BA_JACOBIAN_AUTODIFF ? cams : nullptr, ck64};
    BA_TRY(P, launch_build_points<T>(P->pm, P->opt.huber_delta, true, pts, js, nullptr, nullptr, P->wpt, nullptr, s));
    BA_TRY(P, launch_build_cameras<T>(P->cm, P->m, P->N, pts, js, P->opt.huber_delta, true, nullptr, P->vcam, 0,
                                      nullptr, nullptr, s));
    return BA_OK;
}

extern "C" ba_status ba_eval_cost_grad(ba_problem* P, double* cost, double* grad_cameras, double* grad_points)
{
    if (!P) return BA_EINVAL;
    hipStream_t s = P->stream;
    ba_status st;
    if (cost) {
        if ((st = cost_into_sums<double>(P, P->pts, P->ck64, s)) != BA_OK) return st;
        if ((st = read_scalars(P, P->sums, sizeof(double))) != BA_OK) return st;
        *cost = P->h_scalars[0];
    }
    if (grad_cameras || grad_points) {
        if ((st = grad_into<double>(P, P->cams, P->pts, P->ck64, nullptr, s)) != BA_OK) return st;
        // gradients land in cams_t / pts_t (caller order), then to the host
        BA_TRY(P, launch_scatter_grad(P->m, P->n, 0, 1.0, nullptr, P->vcam, P->wpt, P->d_old_of_new,
                                      grad_cameras ? (void*)P->cams_t : nullptr,
                                      grad_points ? (void*)P->pts_t : nullptr, s));
        BA_TRY(P, hipStreamSynchronize(s));
        if (grad_cameras)
            BA_TRY(P, hipMemcpy(grad_cameras, P->cams_t, sizeof(double) * 9 * (size_t)P->m, hipMemcpyDeviceToHost));
        if (grad_points && P->n > 0)
            BA_TRY(P, hipMemcpy(grad_points, P->pts_t, sizeof(double) * 3 * (size_t)P->n, hipMemcpyDeviceToHost));
    }
    return BA_OK;
}

template <typename T>
static ba_status device_form(ba_problem* P, int32_t dtype, const void* d_cams, const void* d_pts, bool backward,
                             double gout, const double* d_gout, void* d_cost, void* d_gc, void* d_gp, hipStream_t s)
{
    BA_TRY(P, launch_gather_cameras(P->m, dtype, d_cams, P->d_old_of_new, P->cams_t, s));
    BA_TRY(P, launch_convert_points(P->n, dtype, d_pts, P->pts_t, s));
    const CamK<T>* ck;
    BA_TRY(P, launch_camera_constants_f64(P->m, P->cams_t, P->ck64_t, s));
    if constexpr (sizeof(T) == 4) {
        BA_TRY(P, launch_camera_constants_f32(P->m, P->cams_t, P->ck32, s));
        ck = (const CamK<T>*)P->ck32;
    } else {
        ck = (const CamK<T>*)P->ck64_t;
    }
    ba_status st;
    if (!backward) {
        if ((st = cost_into_sums<T>(P, P->pts_t, ck, s)) != BA_OK) return st;
        BA_TRY(P, launch_store_cost(P->sums, (double*)d_cost, s));
        return BA_OK;
    }
    if ((st = grad_into<T>(P, P->cams_t, P->pts_t, ck, sizeof(T) == 4 ? P->ck64_t : nullptr, s)) != BA_OK)
        return st;
    BA_TRY(P, launch_scatter_grad(P->m, P->n, dtype, gout, d_gout, P->vcam, P->wpt, P->d_old_of_new, d_gc, d_gp,
                                  s));
    return BA_OK;
}

extern "C" ba_status ba_cost_fwd_device(ba_problem* P, int32_t dtype, const void* d_cams, const void* d_pts,
                                        void* d_cost_f64, void* hip_stream)
{
    if (!P || (dtype != 0 && dtype != 1) || !d_cams || (P->n > 0 && !d_pts) || !d_cost_f64) {
        if (P) P->last_error = "invalid argument";
        return BA_EINVAL;
    }
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : P->stream;
    return dtype == 0
               ? device_form<double>(P, dtype, d_cams, d_pts, false, 0.0, nullptr, d_cost_f64, nullptr, nullptr, s)
               : device_form<float>(P, dtype, d_cams, d_pts, false, 0.0, nullptr, d_cost_f64, nullptr, nullptr, s);
}

extern "C" ba_status ba_cost_bwd_device(ba_problem* P, int32_t dtype, const void* d_cams, const void* d_pts,
                                        double gout, const double* d_gout, void* d_grad_cams, void* d_grad_pts,
                                        void* hip_stream)
{
    if (!P || (dtype != 0 && dtype != 1) || !d_cams || (P->n > 0 && !d_pts) || !std::isfinite(gout)) {
        if (P) P->last_error = "invalid argument";
        return BA_EINVAL;
    }
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : P->stream;
    return dtype == 0 ? device_form<double>(P, dtype, d_cams, d_pts, true, gout, d_gout, nullptr, d_grad_cams,
                                            d_grad_pts, s)
                      : device_form<float>(P, dtype, d_cams, d_pts, true, gout, d_gout, nullptr, d_grad_cams,
                                           d_grad_pts, s);
}

// ------------------------------------------------ reduced-system operator
template <typename T>
static ba_status schur_matvec_t(ba_problem* P, double lambda, int32_t damping, const double* x, double* q)
{
    hipStream_t s = P->stream;
    const int32_t m = P->m, n = P->n;
    ba_status st;
    if ((st = build_system<T>(P)) != BA_OK) return st;
    BA_TRY(P, launch_damp_cameras(m, P->hcc, lambda, damping, P->bd, P->lfac, P->dcam, P->flag, s));
    BA_TRY(P, launch_damp_points<T>(n, (const double*)P->hpp, lambda, damping, (T*)P->cinv, P->flag, s));
    std::vector<double> xi((size_t)9 * m), qi((size_t)9 * m);
    for (int32_t j = 0; j < m; ++j)
        std::memcpy(&xi[(size_t)9 * j], x + (size_t)9 * P->old_of_new[j], 9 * sizeof(double));
    BA_TRY(P, hipMemcpyAsync(P->x, xi.data(), xi.size() * sizeof(double), hipMemcpyHostToDevice, s));
    BA_TRY(P, launch_pcg_reset(P->sc, 0.0, 1, 0, s));
    const RecomputeInputs<T> ri = recompute_inputs<T>(P);
    BA_TRY(P, launch_pcg_direction<T>(m, true, P->x, P->p, (T*)P->pT, ri.ck, P->sp.recompute ? (T*)P->xf : nullptr,
                                      P->sc, s));
    BA_TRY(P, launch_schur_product<T>(0, P->sp, P->pm, P->N, (const T*)P->hcp, (const T*)P->cinv, P->wpt,
                                      (const T*)P->pT, &ri, m, P->bd, P->p, nullptr, P->q, nullptr, nullptr, P->partials,
                                      P->sc, nullptr, nullptr, s));
    BA_TRY(P, hipMemcpyAsync(qi.data(), P->q, qi.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    BA_TRY(P, hipMemcpyAsync(P->h_scalars, P->flag, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BA_TRY(P, hipStreamSynchronize(s));
    if (*(const int32_t*)P->h_scalars != 0) {
        P->last_error = not_pd_message(P, (const int32_t*)P->h_scalars, lambda);
        BA_TRY(P, hipMemset(P->flag, 0, 4 * sizeof(int32_t)));
        return BA_ENUMERIC;
    }
    for (int32_t j = 0; j < m; ++j)
        std::memcpy(q + (size_t)9 * P->old_of_new[j], &qi[(size_t)9 * j], 9 * sizeof(double));
    return BA_OK;
}

extern "C" ba_status ba_schur_matvec(ba_problem* P, double lambda, int32_t damping, const double* x, double* q)
{
    if (!P) return BA_EINVAL;
    if (!x || !q || !(lambda >= 0.0) || !std::isfinite(lambda) ||
        (damping != BA_DAMP_MARQUARDT && damping != BA_DAMP_IDENTITY) || !finite_all(x, 9 * (int64_t)P->m)) {
        P->last_error = "invalid argument";
        return BA_EINVAL;
    }
    return P->is_f32() ? schur_matvec_t<float>(P, lambda, damping, x, q)
                       : schur_matvec_t<double>(P, lambda, damping, x, q);
}

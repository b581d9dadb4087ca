/* ba.h - C ABI of the MI355X bundle-adjustment LM step.
 *
 * The library solves the bundle-adjustment objective of MegBA (arXiv
 * 2112.01349), Sec. 3 Eq. (obj): x* = argmin sum_k rho(|e_k|^2), one residual
 * e_k per observation (graph edge) between a camera and a point, with the
 * Levenberg-Marquardt method.  Each LM iteration runs, on one GPU:
 *   - the per-observation residual and Jacobian (Alg. 1, first step);
 *   - Schur block assembly B (camera 9x9), C (point 3x3) and the vectors v, w
 *     (Alg. 1, second step; Eq. schur_complement); the camera-point blocks E
 *     (9x3 per observation) are formed again from the Jacobian inside every
 *     product that uses them rather than stored (BA_SCHUR_STORED=1 in the
 *     environment at ba_create stores and streams them instead);
 *   - the reduced camera system (Eq. schur_x_c) solved by block-Jacobi PCG
 *     (Alg. 2) whose matrix-vector products are implicit Schur products
 *     (Alg. 3); options: the Schur-Jacobi blocks as the preconditioner, or
 *     the system written out and Cholesky-factored (ba_options.solver);
 *   - point back-substitution (Eq. schur_x_p) and the additive update
 *     (Alg. 1, last step), inside a trust-region accept/reject loop
 *     (supplementary Sec. C: LM with a Ceres-like trust region).
 *
 * Conventions shared by every call:
 *   - Cameras are [m][9] rows: wx wy wz (angle-axis), tx ty tz, f, k1, k2,
 *     the BAL convention of the paper's datasets (Sec. 6, dataset table):
 *     P = R(w) X + t, p = -(Px, Py)/Pz, u = f (1 + k1|p|^2 + k2|p|^4) p,
 *     residual e = u - uv.
 *   - Points are [n][3] rows; observations are (camera, point, uv) triples.
 *   - All host arrays are row-major, caller-owned, and only read or written
 *     during the call.  Arrays come and go in the caller's camera and point
 *     order, whatever order the library uses inside.
 *   - Every call returns a ba_status; none aborts or exits.  On failure the
 *     handle keeps its last valid state and ba_last_error() describes the
 *     failure.  A handle is not thread-safe; distinct handles are independent.
 */
#ifndef BA_H
#define BA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_problem ba_problem; /* opaque handle */

typedef enum {
    BA_OK = 0,
    BA_EINVAL = 1,   /* bad count, index out of range, non-finite input, bad option */
    BA_ENOMEM = 2,   /* device workspace does not fit */
    BA_EDEVICE = 3,  /* HIP runtime error (message in ba_last_error) */
    BA_ENUMERIC = 4  /* a damped block (or, with BA_SOLVER_DENSE, the damped reduced
                        camera system) that is not positive definite */
} ba_status;

typedef enum {
    BA_FP64 = 0,       /* every step in FP64 */
    BA_FP32_MIXED = 1  /* Jacobians, coupling blocks E, C~^-1 and matvecs in FP32;
                          cost sums, PCG vectors/dots/scalars, the 9x9 camera-block
                          factorisations, the 3x3 point-block sums and inversions
                          and the products forming B and C in FP64 (paper Sec. 6,
                          Table float); an observation whose point sits within
                          FP32 resolution of its camera's centre has its
                          geometry formed in FP64 */
} ba_precision;

typedef enum {
    BA_DAMP_MARQUARDT = 0, /* lambda * clamp(diag(H), 1e-6, 1e32), Ceres-like (supp. Sec. C) */
    BA_DAMP_IDENTITY = 1   /* lambda * I, as printed in Sec. 3 */
} ba_damping;

typedef enum {
    BA_JACOBIAN_ANALYTIC = 0, /* closed-form Jacobian (the paper's "-m" variant, Sec. 6) */
    BA_JACOBIAN_AUTODIFF = 1  /* forward-mode automatic differentiation of the residual
                                 (the paper's "-a" variant, Sec. 5 JetVector) */
} ba_jacobian;

typedef enum {
    BA_SOLVER_PCG = 0,   /* block-Jacobi PCG on implicit Schur products (Alg. 2 and 3) */
    BA_SOLVER_DENSE = 1  /* the reduced camera system (Eq. schur_x_c) written out as a dense
                            FP64 [9m][9m] matrix and solved through its Cholesky factor, the
                            direct route of Sec. 3, for m <= BA_DENSE_MAX_CAMERAS; needs
                            (9m)^2 * 8 bytes more device memory, allocated at ba_create */
} ba_solver;

#define BA_DENSE_MAX_CAMERAS 2048

typedef enum {
    BA_PRECOND_CAMERA_BLOCKS = 0, /* M_j = B~_j, the damped camera blocks (Alg. 2) */
    BA_PRECOND_SCHUR_JACOBI = 1   /* M_j = B~_j - sum_{k in obs(j)} E_k C~^-1 E_k^T: the block
                                     diagonal of the reduced system (Eq. schur_x_c), summed
                                     per observation (a repeated (camera, point) pair adds no
                                     cross term); formed once per LM iteration */
} ba_preconditioner;

/* How one iteration's PCG solve ended (Alg. 2 with the stopping rule of
 * ba_options; the paper leaves the stopping rule open). */
typedef enum {
    BA_PCG_CONVERGED = 0, /* ||r|| <= pcg_rtol ||b|| before a matvec */
    BA_PCG_CAP = 1,       /* max_pcg_iters matvecs ran (the residual test may also hold there) */
    BA_PCG_BREAKDOWN = 2, /* p^T q <= 0 or non-finite: the last iterate is the step */
    BA_PCG_FIXED = 3,     /* a fixed count (pcg_fixed_iters or pcg_schedule) ran to its end */
    BA_PCG_DIRECT = 4     /* BA_SOLVER_DENSE: no PCG */
} ba_pcg_stop;

typedef struct {
    uint32_t struct_size;          /* sizeof(ba_options) */
    int32_t precision;             /* ba_precision; fixed at ba_create */
    int32_t damping;               /* ba_damping */
    double huber_delta;            /* Huber threshold in pixels on |e|; <= 0: squared loss */
    int32_t max_lm_iters;          /* LM iterations; accepted and rejected ones both count */
    int32_t max_pcg_iters;         /* cap on Schur matvecs per LM iteration */
    double pcg_rtol;               /* stop PCG when ||r||_2 <= pcg_rtol * ||b||_2 */
    int32_t pcg_fixed_iters;       /* > 0: run exactly this many matvecs per LM iteration */
    int32_t jacobian;              /* ba_jacobian: how J_c and J_p are formed */
    const int32_t *pcg_schedule;   /* nullable [max_lm_iters]: exact matvec count per LM
                                      iteration; overrides pcg_fixed_iters and pcg_rtol */
    double lambda_init;            /* initial LM damping, default 1e-4 */
    double min_relative_decrease;  /* accept a step iff gain ratio > this, default 1e-3 */
    int32_t time_kernels;          /* != 0: time every 8th Schur matvec of each PCG solve with
                                      HIP events (the events lengthen the matvecs they bracket) */
    int32_t solver;                /* ba_solver; fixed at ba_create.  With BA_SOLVER_DENSE
                                      the PCG fields are ignored and pcg_iters reports 0;
                                      a reduced system that is not positive definite
                                      ends the solve with BA_ENUMERIC */
    int32_t preconditioner;        /* ba_preconditioner of PCG; may change between solves */
} ba_options;

typedef struct {
    /* caller-owned arrays, each nullable, of length >= capacity */
    int32_t capacity;
    int32_t iters_run;             /* LM iterations executed */
    double initial_cost;           /* F at entry, F = 1/2 sum rho(|e|^2) */
    double final_cost;             /* F of the last accepted state */
    double *cost;                  /* F after each iteration's accept/reject */
    double *trial_cost;            /* F(x + dx) of each iteration's trial step */
    double *lambda;                /* damping used by each iteration */
    double *pred;                  /* predicted (model) decrease of each step */
    double *ms;                    /* wall time of each iteration, ms */
    int32_t *pcg_iters;            /* Schur matvecs of each iteration */
    int32_t *accepted;             /* 1 if the step was accepted */
    int32_t *pcg_stop;             /* ba_pcg_stop of each iteration's solve */
    /* totals, always filled */
    double total_ms;               /* whole solve */
    double pcg_ms;                 /* time inside the PCG loops */
    int64_t pcg_iters_total;       /* Schur matvecs executed */
    double matvec_ms;              /* sum of timed matvec kernel durations (time_kernels) */
    int64_t matvec_launches;       /* number of timed matvec launches (time_kernels) */
    double schur_hot_ms;           /* of matvec_ms: the point-major pass over all
                                      observations (time_kernels) */
} ba_report;

/* Fills *opt with defaults: FP64, Marquardt damping, squared loss, 10 LM
 * iterations, PCG max 50 / rtol 1e-8, lambda 1e-4, min decrease 1e-3. */
ba_status ba_options_default(ba_options *opt);

/* Creates a problem from a graph of cameras, points and observations (Sec. 3:
 * nodes and edges; Sec. 5.3 addNode/addEdge taken in bulk).
 *   num_cameras m >= 1, num_points n >= 0, num_obs N >= 0 (N < 2^31)
 *   cameras [m][9], points [n][3]: initial state, FP64, finite
 *   obs_camera[N] in [0,m), obs_point[N] in [0,n), obs_uv [N][2] finite pixels
 *   opt: nullable (defaults); its precision selects the workspace type
 *   hip_stream: hipStream_t to order all work on; NULL = the default stream
 * The library copies everything to device memory in its own layout and sizes
 * the whole workspace here (the paper's memory pool, Sec. 5.2); later calls
 * allocate nothing.  Duplicate (camera, point) pairs are allowed (their terms
 * add); points with fewer than two observations and cameras with none are
 * allowed.  Errors: BA_EINVAL (handle not created; also for BA_SOLVER_DENSE
 * with m > BA_DENSE_MAX_CAMERAS), BA_ENOMEM, BA_EDEVICE. */
ba_status ba_create(int32_t num_cameras, int32_t num_points, int64_t num_obs,
                    const double *cameras, const double *points,
                    const int32_t *obs_camera, const int32_t *obs_point,
                    const double *obs_uv, const ba_options *opt, void *hip_stream,
                    ba_problem **out);

/* Replaces the current state (caller order, FP64).  BA_EINVAL on non-finite input. */
ba_status ba_set_params(ba_problem *prob, const double *cameras, const double *points);

/* Copies the current state out (caller order, FP64); either pointer may be NULL. */
ba_status ba_get_params(const ba_problem *prob, double *cameras, double *points);

/* F = 1/2 sum rho(|e|^2) at the current state in FP64, and optionally its
 * gradient sum rho'(|e|^2) J^T e (Sec. 3: g = -J^T Sigma r) per camera
 * [m][9] and per point [n][3], caller order.  Gradients are computed in FP64. */
ba_status ba_eval_cost_grad(ba_problem *prob, double *cost, double *grad_cameras,
                            double *grad_points);

/* Runs the LM loop from the current state (Alg. 1 with one partition inside
 * the trust-region wrapper) and leaves the last accepted state in the handle.
 * opt: NULL = the create-time options; opt->precision and opt->solver must
 * equal the create-time values.  rep: nullable.  A PCG breakdown (p^T q <= 0 or
 * non-finite, possible in the FP32 products near a gauge direction once
 * lambda is small) ends that PCG run with its last iterate as the step
 * (truncated CG) and the loop goes on.  BA_ENUMERIC stops the loop and keeps
 * the last accepted state; the report holds the iterations run. */
ba_status ba_lm_solve(ba_problem *prob, const ba_options *opt, ba_report *rep);

/* Applies the damped reduced camera system of the current state,
 *   q = (B~ - E C~^-1 E^T) x      (Eq. schur_x_c, computed as in Alg. 3),
 * with B~ = B + lambda D_c, C~ = C + lambda D_p (damping: ba_damping) and
 * the create-time Huber threshold and precision.  x and q are [m][9] host
 * arrays in caller camera order.  The system is assembled at the current
 * state first.  BA_ENUMERIC if a damped block is not positive definite. */
ba_status ba_schur_matvec(ba_problem *prob, double lambda, int32_t damping, const double *x,
                          double *q);

/* Device-pointer forms for a torch.autograd.Function, ordered on hip_stream
 * (NULL = the handle's stream).  dtype: 0 = FP64, 1 = FP32 for the parameter
 * and gradient arrays and for the Jacobian arithmetic; the cost is always
 * summed and returned in FP64.  d_cams [m][9] and d_pts [n][3] are device
 * arrays in caller order; d_cost_f64 is one device double.  The calls borrow
 * the arrays only for their duration and use the handle's observation graph
 * and Huber threshold. */
ba_status ba_cost_fwd_device(ba_problem *prob, int32_t dtype, const void *d_cams,
                             const void *d_pts, void *d_cost_f64, void *hip_stream);

/* d_grad_cams [m][9], d_grad_pts [n][3] (dtype, caller order) receive
 * s * sum rho'(|e|^2) J^T e at (d_cams, d_pts), s = gout times the device
 * double *d_gout when d_gout is not NULL (read on the stream, so a caller
 * holding the upstream gradient on the device need not synchronise); either
 * output may be NULL. */
ba_status ba_cost_bwd_device(ba_problem *prob, int32_t dtype, const void *d_cams,
                             const void *d_pts, double gout, const double *d_gout,
                             void *d_grad_cams, void *d_grad_pts, void *hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the cost of
 * ba_cost_fwd_device from caller device arrays, with no handle and no
 * allocation.  F = 1/2 sum rho(|e|^2) over num_obs observations, written to
 * the device double d_cost_f64, ordered on hip_stream (NULL = the default
 * stream).  d_cams [m][9] and d_pts [n][3] are dtype arrays (0 = FP64, 1 =
 * FP32; FP32 also computes the residuals in FP32, the sum is FP64);
 * d_obs_camera, d_obs_point [N] int32 and d_obs_uv [N][2] FP64 are device
 * arrays; huber_delta <= 0 selects the squared loss.  The reduction's only
 * scratch is a fixed 2048-entry FP64 array in device memory, one per device
 * for the life of the process, so any N is accepted; calls that overlap on
 * one device share that array and race (order them on one stream).  An
 * observation index out of range makes the result NaN.  Errors: BA_EINVAL
 * (bad count, dtype, NULL array or NaN delta), BA_EDEVICE (launch failure). */
ba_status ba_cost_device_noalloc(int32_t num_cameras, int32_t num_points, int64_t num_obs,
                                 int32_t dtype, const void *d_cams, const void *d_pts,
                                 const int32_t *d_obs_camera, const int32_t *d_obs_point,
                                 const double *d_obs_uv, double huber_delta, double *d_cost_f64,
                                 void *hip_stream);

/* Bytes of device memory the handle holds. */
ba_status ba_memory_bytes(const ba_problem *prob, int64_t *bytes);

/* Releases the handle and all its device memory; NULL is ignored. */
void ba_destroy(ba_problem *prob);

const char *ba_status_str(ba_status status);

/* Message for the last failing call on this handle ("" if none); for a NULL
 * handle, the message of the last failed ba_create on this thread. */
const char *ba_last_error(const ba_problem *prob);

#ifdef __cplusplus
}
#endif
#endif /* BA_H */

/* Bundle-adjustment oracle: plain, single-threaded FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The solver library
 * never links it, and this header is not shared with the solver.
 *
 * Every routine sums in observation order and follows the paper (MegBA,
 * arXiv 2112.01349) as cited per function.  Readings where the paper is
 * silent are marked "Reading".
 *
 * Layouts (all row-major, FP64 unless stated):
 *   cameras [m][9] = wx wy wz tx ty tz f k1 k2   (angle-axis, translation,
 *                                                focal, radial k1, k2)
 *   points  [n][3]
 *   obs_cam[N], obs_pt[N] int32; obs_uv [N][2] pixels
 *   B  [m][81]  camera blocks (9x9)     C  [n][9]  point blocks (3x3)
 *   E  [N][27]  coupling block per observation, 9x3, E[k][a*3+b]
 *   v  [m][9]   w  [n][3]               gradient-side vectors (-J^T W e)
 */
#ifndef BA_ORACLE_H
#define BA_ORACLE_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_ENUMERIC 4
#define ORC_BREAKDOWN 5   /* orc_pcg: p^T q <= 0 or non-finite; x holds the last iterate */

typedef struct {
    double huber_delta;        /* <= 0: squared loss */
    int32_t damping;           /* 0: lambda*clamp(diag H); 1: lambda*I */
    int32_t max_lm_iters;
    int32_t max_pcg_iters;
    double pcg_rtol;
    const int32_t *pcg_schedule; /* nullable [max_lm_iters]: exact PCG counts */
    double lambda_init;
    double min_relative_decrease;
    int32_t preconditioner;    /* 0: damped camera blocks B~_j (Alg. 2); 1: Schur-Jacobi */
    int32_t solver;            /* 0: PCG (Alg. 2); 1: the reduced camera system written out
                                  and factored (the direct option for small problems) */
} orc_options;

/* How a PCG solve ended (Alg. 2 with the stopping readings): */
#define ORC_PCG_CONVERGED 0   /* ||r|| <= rtol ||b|| before a matvec */
#define ORC_PCG_CAP 1         /* the matvec cap was reached first */
#define ORC_PCG_BREAKDOWN 2   /* p^T q <= 0 or non-finite; x holds the last iterate */
#define ORC_PCG_FIXED 3       /* a fixed count (schedule) was run to its end */
#define ORC_PCG_DIRECT 4      /* no PCG: the reduced system was factored */

typedef struct {               /* caller-owned arrays of length max_lm_iters */
    int32_t iters_run;
    double initial_cost, final_cost;
    double *cost, *trial_cost, *lambda, *pred;
    int32_t *pcg_iters, *accepted;
    int32_t *pcg_stop;         /* nullable: ORC_PCG_* per iteration */
} orc_trace;

int orc_project(const double cam[9], const double X[3], double uv[2]);
int orc_residual_jacobian(const double cam[9], const double X[3], const double uv[2],
                          double e[2], double Jc[18], double Jp[6]);
double orc_rho(double s, double delta);
double orc_rho_prime(double s, double delta);

double orc_cost(int64_t N, const double *cams, const double *pts, const int32_t *oc,
                const int32_t *op, const double *uv, double delta);
double orc_cost_subset(const int64_t *list, int64_t count, const double *cams,
                       const double *pts, const int32_t *oc, const int32_t *op,
                       const double *uv, double delta);
double orc_gradient(int32_t m, int32_t n, int64_t N, const double *cams, const double *pts,
                    const int32_t *oc, const int32_t *op, const double *uv, double delta,
                    double *grad_cams, double *grad_pts);

int orc_assemble(int32_t m, int32_t n, int64_t N, const double *cams, const double *pts,
                 const int32_t *oc, const int32_t *op, const double *uv, double delta,
                 double *B, double *C, double *E, double *v, double *w, double *cost);
void orc_subset_sums(const int64_t *list, int64_t count, const double *cams,
                     const double *pts, const int32_t *oc, const int32_t *op,
                     const double *uv, double delta, double Bs[81], double vs[9],
                     double Cs[9], double ws[3], double *cost);

void orc_damp(int32_t m, int32_t n, const double *B, const double *C, double lambda,
              int32_t damping, double *Bd, double *Cd, double *Dc, double *Dp);
int orc_invert_points(int32_t n, const double *Cd, double *Cinv);

void orc_schur_matvec(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
                      const double *Bd, const double *E, const double *Cinv,
                      const double *x, double *out, double *work_a, double *work_b);
void orc_reduced_rhs(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
                     const double *v, const double *w, const double *E, const double *Cinv,
                     double *g, double *work_b);
void orc_schur_jacobi(int32_t m, int64_t N, const int32_t *oc, const int32_t *op,
                      const double *Bd, const double *E, const double *Cinv, double *M);
int orc_pcg_m(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
              const double *Bd, const double *E, const double *Cinv, const double *Mblk,
              const double *b, double rtol, int32_t max_iters, int32_t fixed_iters, double *x,
              int32_t *iters);
int orc_pcg(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
            const double *Bd, const double *E, const double *Cinv, const double *b,
            double rtol, int32_t max_iters, int32_t fixed_iters, double *x, int32_t *iters);
void orc_back_substitute(int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
                         const double *E, const double *Cinv, const double *w,
                         const double *dc, double *dp);

int orc_schur_dense(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
                    const double *Bd, const double *E, const double *Cinv, double *S);
int orc_dense_solve(int64_t nd, const double *A, const double *b, double *x);
int orc_lm_solve(int32_t m, int32_t n, int64_t N, double *cams, double *pts,
                 const int32_t *oc, const int32_t *op, const double *uv,
                 const orc_options *opt, orc_trace *trace);

double orc_schur_row(int32_t j, const double *cams, const double *pts,
                     const int32_t *oc, const int32_t *op, const double *uv, double delta,
                     double lambda, int32_t damping,
                     const int64_t *cam_off, const int64_t *cam_obs,
                     const int64_t *pt_off, const int64_t *pt_obs,
                     const double *x, double q[9]);
#endif

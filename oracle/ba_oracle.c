/* Bundle-adjustment oracle: plain, single-threaded FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the solver library.  It shares no
 * code, header or table with the HIP path.
 *
 * The method is MegBA (arXiv 2112.01349): the least-squares objective of
 * Sec. 3 (Eq. obj), the Gauss-Newton/LM normal equations of Sec. 3, the Schur
 * block system (Eq. schur_complement), the reduced camera system (Eq.
 * schur_x_c), point back-substitution (Eq. schur_x_p), and Algorithms 1-3
 * (distributed BA, DPCG, DSE) taken with a single partition, so that every
 * all-reduce is the identity.  The LM wrapper is the trust-region scheme the
 * supplementary Sec. C names ("same as Ceres").
 *
 * Jacobians come from forward-mode dual numbers (one value plus twelve
 * partials: nine camera and three point parameters), independent of any
 * closed-form derivative.
 *
 * Build: gcc -O2 -std=c99 -fPIC -shared -ffp-contract=off (no fast-math).
 */
#include "ba_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ duals */
#define NPART 12
typedef struct {
    double v;
    double d[NPART];
} dual;

static dual d_const(double c)
{
    dual r;
    r.v = c;
    memset(r.d, 0, sizeof r.d);
    return r;
}

static dual d_var(double x, int slot)
{
    dual r = d_const(x);
    r.d[slot] = 1.0;
    return r;
}

static dual d_add(dual a, dual b)
{
    dual r;
    r.v = a.v + b.v;
    for (int i = 0; i < NPART; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}

static dual d_sub(dual a, dual b)
{
    dual r;
    r.v = a.v - b.v;
    for (int i = 0; i < NPART; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}

static dual d_mul(dual a, dual b)
{
    dual r;
    r.v = a.v * b.v;
    for (int i = 0; i < NPART; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}

static dual d_div(dual a, dual b)
{
    dual r;
    r.v = a.v / b.v;
    for (int i = 0; i < NPART; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r;
}

static dual d_neg(dual a)
{
    dual r;
    r.v = -a.v;
    for (int i = 0; i < NPART; ++i) r.d[i] = -a.d[i];
    return r;
}

static dual d_sqrt(dual a)
{
    dual r;
    r.v = sqrt(a.v);
    for (int i = 0; i < NPART; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
    return r;
}

static dual d_sin(dual a)
{
    dual r;
    double c = cos(a.v);
    r.v = sin(a.v);
    for (int i = 0; i < NPART; ++i) r.d[i] = c * a.d[i];
    return r;
}

static dual d_cos(dual a)
{
    dual r;
    double s = sin(a.v);
    r.v = cos(a.v);
    for (int i = 0; i < NPART; ++i) r.d[i] = -s * a.d[i];
    return r;
}

/* ------------------------------------------------- camera model (Sec. 6)
 * Reading: the BAL camera convention of the paper's datasets (Sec. 6 dataset
 * table).  P = R(w) X + t, p = -(P_x, P_y)/P_z, d = 1 + k1 |p|^2 + k2 |p|^4,
 * u = f d p, residual e = u - uv (information matrix = identity, Sec. 4.1).
 * Rotation: Rodrigues' formula; when |w|^2 <= DBL_EPSILON the first-order
 * form R X = X + w x X is used (Reading). */
static void rotate_dual(const dual w[3], const dual X[3], dual out[3])
{
    dual t2 = d_add(d_add(d_mul(w[0], w[0]), d_mul(w[1], w[1])), d_mul(w[2], w[2]));
    if (t2.v > DBL_EPSILON) {
        dual th = d_sqrt(t2);
        dual c = d_cos(th), s = d_sin(th);
        dual k[3] = {d_div(w[0], th), d_div(w[1], th), d_div(w[2], th)};
        dual kx[3] = {d_sub(d_mul(k[1], X[2]), d_mul(k[2], X[1])),
                      d_sub(d_mul(k[2], X[0]), d_mul(k[0], X[2])),
                      d_sub(d_mul(k[0], X[1]), d_mul(k[1], X[0]))};
        dual kd = d_add(d_add(d_mul(k[0], X[0]), d_mul(k[1], X[1])), d_mul(k[2], X[2]));
        dual omc = d_sub(d_const(1.0), c);
        for (int a = 0; a < 3; ++a)
            out[a] = d_add(d_add(d_mul(X[a], c), d_mul(kx[a], s)), d_mul(d_mul(k[a], kd), omc));
    } else {
        dual wx[3] = {d_sub(d_mul(w[1], X[2]), d_mul(w[2], X[1])),
                      d_sub(d_mul(w[2], X[0]), d_mul(w[0], X[2])),
                      d_sub(d_mul(w[0], X[1]), d_mul(w[1], X[0]))};
        for (int a = 0; a < 3; ++a) out[a] = d_add(X[a], wx[a]);
    }
}

static void project_dual(const dual c[9], const dual X[3], dual u[2])
{
    dual RX[3];
    rotate_dual(c, X, RX);
    dual P0 = d_add(RX[0], c[3]), P1 = d_add(RX[1], c[4]), P2 = d_add(RX[2], c[5]);
    dual px = d_neg(d_div(P0, P2)), py = d_neg(d_div(P1, P2));
    dual r2 = d_add(d_mul(px, px), d_mul(py, py));
    dual dist = d_add(d_add(d_const(1.0), d_mul(c[7], r2)), d_mul(c[8], d_mul(r2, r2)));
    dual fd = d_mul(c[6], dist);
    u[0] = d_mul(fd, px);
    u[1] = d_mul(fd, py);
}

/* Plain FP64 projection: the same formula as project_dual with values only. */
int orc_project(const double cam[9], const double X[3], double uv[2])
{
    double RX[3];
    double t2 = cam[0] * cam[0] + cam[1] * cam[1] + cam[2] * cam[2];
    if (t2 > DBL_EPSILON) {
        double th = sqrt(t2);
        double c = cos(th), s = sin(th);
        double k[3] = {cam[0] / th, cam[1] / th, cam[2] / th};
        double kx[3] = {k[1] * X[2] - k[2] * X[1], k[2] * X[0] - k[0] * X[2],
                        k[0] * X[1] - k[1] * X[0]};
        double kd = k[0] * X[0] + k[1] * X[1] + k[2] * X[2];
        double omc = 1.0 - c;
        for (int a = 0; a < 3; ++a) RX[a] = X[a] * c + kx[a] * s + k[a] * kd * omc;
    } else {
        double wx[3] = {cam[1] * X[2] - cam[2] * X[1], cam[2] * X[0] - cam[0] * X[2],
                        cam[0] * X[1] - cam[1] * X[0]};
        for (int a = 0; a < 3; ++a) RX[a] = X[a] + wx[a];
    }
    double P0 = RX[0] + cam[3], P1 = RX[1] + cam[4], P2 = RX[2] + cam[5];
    double px = -(P0 / P2), py = -(P1 / P2);
    double r2 = px * px + py * py;
    double dist = 1.0 + cam[7] * r2 + cam[8] * (r2 * r2);
    double fd = cam[6] * dist;
    uv[0] = fd * px;
    uv[1] = fd * py;
    return ORC_OK;
}

/* Residual and Jacobians of one observation: J_c = de/dc (2x9, row-major),
 * J_p = de/dX (2x3), by forward-mode duals (Alg. 1, residual/Jacobian step). */
int orc_residual_jacobian(const double cam[9], const double X[3], const double uv[2],
                          double e[2], double Jc[18], double Jp[6])
{
    dual c[9], P[3], u[2];
    for (int a = 0; a < 9; ++a) c[a] = d_var(cam[a], a);
    for (int a = 0; a < 3; ++a) P[a] = d_var(X[a], 9 + a);
    project_dual(c, P, u);
    for (int r = 0; r < 2; ++r) {
        e[r] = u[r].v - uv[r];
        for (int a = 0; a < 9; ++a) Jc[r * 9 + a] = u[r].d[a];
        for (int b = 0; b < 3; ++b) Jp[r * 3 + b] = u[r].d[9 + b];
    }
    return ORC_OK;
}

/* ---------------------------------------------------------- robust loss
 * Reading: Huber on the 2-D residual norm, s = |e|^2:
 *   rho(s) = s (s <= delta^2),  2 delta sqrt(s) - delta^2 otherwise;
 * delta <= 0 selects the squared loss of Eq. obj.  The IRLS weight is
 * rho'(s) and no second-order correction is used. */
double orc_rho(double s, double delta)
{
    if (delta <= 0.0 || s <= delta * delta) return s;
    return 2.0 * delta * sqrt(s) - delta * delta;
}

double orc_rho_prime(double s, double delta)
{
    if (delta <= 0.0 || s <= delta * delta) return 1.0;
    return delta / sqrt(s);
}

/* F = 1/2 sum rho(|e|^2) in observation order (Eq. obj; the factor 1/2 is a
 * Reading that only rescales F). */
double orc_cost(int64_t N, const double *cams, const double *pts, const int32_t *oc,
                const int32_t *op, const double *uv, double delta)
{
    double F = 0.0;
    for (int64_t k = 0; k < N; ++k) {
        double u[2];
        orc_project(cams + 9 * (int64_t)oc[k], pts + 3 * (int64_t)op[k], u);
        double e0 = u[0] - uv[2 * k], e1 = u[1] - uv[2 * k + 1];
        F += 0.5 * orc_rho(e0 * e0 + e1 * e1, delta);
    }
    return F;
}

double orc_cost_subset(const int64_t *list, int64_t count, const double *cams,
                       const double *pts, const int32_t *oc, const int32_t *op,
                       const double *uv, double delta)
{
    double F = 0.0;
    for (int64_t t = 0; t < count; ++t) {
        int64_t k = list[t];
        double u[2];
        orc_project(cams + 9 * (int64_t)oc[k], pts + 3 * (int64_t)op[k], u);
        double e0 = u[0] - uv[2 * k], e1 = u[1] - uv[2 * k + 1];
        F += 0.5 * orc_rho(e0 * e0 + e1 * e1, delta);
    }
    return F;
}

/* grad F = sum rho'(s) J^T e (Sec. 3: g = -J^T Sigma r, with IRLS weights).
 * Returns F. */
double orc_gradient(int32_t m, int32_t n, int64_t N, const double *cams, const double *pts,
                    const int32_t *oc, const int32_t *op, const double *uv, double delta,
                    double *grad_cams, double *grad_pts)
{
    memset(grad_cams, 0, sizeof(double) * 9 * (size_t)m);
    memset(grad_pts, 0, sizeof(double) * 3 * (size_t)n);
    double F = 0.0;
    for (int64_t k = 0; k < N; ++k) {
        double e[2], Jc[18], Jp[6];
        int64_t j = oc[k], i = op[k];
        orc_residual_jacobian(cams + 9 * j, pts + 3 * i, uv + 2 * k, e, Jc, Jp);
        double s = e[0] * e[0] + e[1] * e[1];
        double wt = orc_rho_prime(s, delta);
        F += 0.5 * orc_rho(s, delta);
        for (int a = 0; a < 9; ++a) grad_cams[9 * j + a] += wt * (Jc[a] * e[0] + Jc[9 + a] * e[1]);
        for (int b = 0; b < 3; ++b) grad_pts[3 * i + b] += wt * (Jp[b] * e[0] + Jp[3 + b] * e[1]);
    }
    return F;
}

/* ------------------------------------------------------------- assembly
 * Alg. 1 (Hessian and constant vector step) with one partition:
 *   B_j  = sum_{k in obs(j)} w J_c^T J_c          (9x9)
 *   C_i  = sum_{k in obs(i)} w J_p^T J_p          (3x3)
 *   E_k  = w J_c^T J_p                            (9x3, one block per edge;
 *                                                  Sec. 4.1: E has one
 *                                                  non-zero block per edge)
 *   v_j  = -sum w J_c^T e,   w_i = -sum w J_p^T e  (Sec. 3, g = -J^T r)
 * with w = rho'(|e|^2).  Returns the cost at the same state. */
static void add_observation(const double e[2], const double Jc[18], const double Jp[6],
                            double wt, double *Bj, double *Ci, double *Ek, double *vj,
                            double *wi)
{
    for (int a = 0; a < 9; ++a) {
        for (int b = 0; b < 9; ++b)
            Bj[a * 9 + b] += wt * (Jc[a] * Jc[b] + Jc[9 + a] * Jc[9 + b]);
        for (int b = 0; b < 3; ++b) {
            double h = wt * (Jc[a] * Jp[b] + Jc[9 + a] * Jp[3 + b]);
            if (Ek) Ek[a * 3 + b] += h;
        }
        vj[a] -= wt * (Jc[a] * e[0] + Jc[9 + a] * e[1]);
    }
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) Ci[a * 3 + b] += wt * (Jp[a] * Jp[b] + Jp[3 + a] * Jp[3 + b]);
        wi[a] -= wt * (Jp[a] * e[0] + Jp[3 + a] * e[1]);
    }
}

int orc_assemble(int32_t m, int32_t n, int64_t N, const double *cams, const double *pts,
                 const int32_t *oc, const int32_t *op, const double *uv, double delta,
                 double *B, double *C, double *E, double *v, double *w, double *cost)
{
    memset(B, 0, sizeof(double) * 81 * (size_t)m);
    memset(C, 0, sizeof(double) * 9 * (size_t)n);
    memset(E, 0, sizeof(double) * 27 * (size_t)N);
    memset(v, 0, sizeof(double) * 9 * (size_t)m);
    memset(w, 0, sizeof(double) * 3 * (size_t)n);
    double F = 0.0;
    for (int64_t k = 0; k < N; ++k) {
        double e[2], Jc[18], Jp[6];
        int64_t j = oc[k], i = op[k];
        orc_residual_jacobian(cams + 9 * j, pts + 3 * i, uv + 2 * k, e, Jc, Jp);
        double s = e[0] * e[0] + e[1] * e[1];
        double wt = orc_rho_prime(s, delta);
        F += 0.5 * orc_rho(s, delta);
        add_observation(e, Jc, Jp, wt, B + 81 * j, C + 9 * i, E + 27 * k, v + 9 * j, w + 3 * i);
    }
    if (cost) *cost = F;
    return ORC_OK;
}

/* Sums of the assembly terms over a list of observations: with the list of
 * one camera's observations Bs, vs are that camera's B_j, v_j; with one
 * point's list Cs, ws are C_i, w_i. */
void orc_subset_sums(const int64_t *list, int64_t count, const double *cams,
                     const double *pts, const int32_t *oc, const int32_t *op,
                     const double *uv, double delta, double Bs[81], double vs[9],
                     double Cs[9], double ws[3], double *cost)
{
    memset(Bs, 0, sizeof(double) * 81);
    memset(vs, 0, sizeof(double) * 9);
    memset(Cs, 0, sizeof(double) * 9);
    memset(ws, 0, sizeof(double) * 3);
    double F = 0.0;
    for (int64_t t = 0; t < count; ++t) {
        int64_t k = list[t];
        double e[2], Jc[18], Jp[6];
        orc_residual_jacobian(cams + 9 * (int64_t)oc[k], pts + 3 * (int64_t)op[k], uv + 2 * k,
                              e, Jc, Jp);
        double s = e[0] * e[0] + e[1] * e[1];
        double wt = orc_rho_prime(s, delta);
        F += 0.5 * orc_rho(s, delta);
        add_observation(e, Jc, Jp, wt, Bs, Cs, NULL, vs, ws);
    }
    if (cost) *cost = F;
}

/* -------------------------------------------------------------- damping
 * Sec. 3 writes the LM matrix as J^T J + lambda I; the supplementary Sec. C
 * says the trust region follows Ceres.  Reading: damping = 0 uses
 * lambda * D with D = clamp(diag(H), 1e-6, 1e32) on both the camera and the
 * point blocks; damping = 1 uses lambda * I as printed. */
static double clamp_diag(double h)
{
    if (h < 1e-6) return 1e-6;
    if (h > 1e32) return 1e32;
    return h;
}

void orc_damp(int32_t m, int32_t n, const double *B, const double *C, double lambda,
              int32_t damping, double *Bd, double *Cd, double *Dc, double *Dp)
{
    for (int64_t j = 0; j < m; ++j) {
        for (int a = 0; a < 81; ++a) Bd[81 * j + a] = B[81 * j + a];
        for (int a = 0; a < 9; ++a) {
            double D = damping == 0 ? clamp_diag(B[81 * j + a * 10]) : 1.0;
            Dc[9 * j + a] = D;
            Bd[81 * j + a * 10] += lambda * D;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 9; ++a) Cd[9 * i + a] = C[9 * i + a];
        for (int a = 0; a < 3; ++a) {
            double D = damping == 0 ? clamp_diag(C[9 * i + a * 4]) : 1.0;
            Dp[3 * i + a] = D;
            Cd[9 * i + a * 4] += lambda * D;
        }
    }
}

/* Cholesky A = L L^T of a k x k SPD matrix; returns 0 on success. */
static int cholesky(const double *A, int k, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)(k * k));
    for (int c = 0; c < k; ++c) {
        double s = A[c * k + c];
        for (int t = 0; t < c; ++t) s -= L[c * k + t] * L[c * k + t];
        if (!(s > 0.0)) return -1;
        double d = sqrt(s);
        L[c * k + c] = d;
        for (int r = c + 1; r < k; ++r) {
            double x = A[r * k + c];
            for (int t = 0; t < c; ++t) x -= L[r * k + t] * L[c * k + t];
            L[r * k + c] = x / d;
        }
    }
    return 0;
}

static void chol_solve(const double *L, int k, const double *rhs, double *x)
{
    double y[9];
    for (int r = 0; r < k; ++r) {
        double s = rhs[r];
        for (int t = 0; t < r; ++t) s -= L[r * k + t] * y[t];
        y[r] = s / L[r * k + r];
    }
    for (int r = k - 1; r >= 0; --r) {
        double s = y[r];
        for (int t = r + 1; t < k; ++t) s -= L[t * k + r] * x[t];
        x[r] = s / L[r * k + r];
    }
}

/* C~_i^{-1} formed explicitly per point through its Cholesky factor (used by
 * Alg. 3's b = C^{-1} a and Eq. schur_x_p). */
int orc_invert_points(int32_t n, const double *Cd, double *Cinv)
{
    for (int64_t i = 0; i < n; ++i) {
        double L[9];
        if (cholesky(Cd + 9 * i, 3, L)) return ORC_ENUMERIC;
        for (int c = 0; c < 3; ++c) {
            double unit[3] = {0.0, 0.0, 0.0}, col[3];
            unit[c] = 1.0;
            chol_solve(L, 3, unit, col);
            for (int r = 0; r < 3; ++r) Cinv[9 * i + r * 3 + c] = col[r];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------- Alg. 3 (DSE), K = 1
 *   a = E^T x;  b = C^{-1} a;  c = E b;  d = B x;  return d - c.
 * E^T x gathers per point over its observations; E b scatters per camera. */
void orc_schur_matvec(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
                      const double *Bd, const double *E, const double *Cinv,
                      const double *x, double *out, double *work_a, double *work_b)
{
    memset(work_a, 0, sizeof(double) * 3 * (size_t)n);
    for (int64_t k = 0; k < N; ++k) {
        const double *Ek = E + 27 * k;
        const double *xj = x + 9 * (int64_t)oc[k];
        double *ai = work_a + 3 * (int64_t)op[k];
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int a = 0; a < 9; ++a) s += Ek[a * 3 + b] * xj[a];
            ai[b] += s;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Cinv[9 * i + r * 3 + c] * work_a[3 * i + c];
            work_b[3 * i + r] = s;
        }
    for (int64_t j = 0; j < m; ++j)
        for (int r = 0; r < 9; ++r) {
            double s = 0.0;
            for (int c = 0; c < 9; ++c) s += Bd[81 * j + r * 9 + c] * x[9 * j + c];
            out[9 * j + r] = s;
        }
    for (int64_t k = 0; k < N; ++k) {
        const double *Ek = E + 27 * k;
        const double *bi = work_b + 3 * (int64_t)op[k];
        double *oj = out + 9 * (int64_t)oc[k];
        for (int a = 0; a < 9; ++a)
            oj[a] -= Ek[a * 3] * bi[0] + Ek[a * 3 + 1] * bi[1] + Ek[a * 3 + 2] * bi[2];
    }
}

/* Alg. 1, reduced constant vector: g = v - E C^{-1} w (Eq. schur_x_c). */
void orc_reduced_rhs(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
                     const double *v, const double *w, const double *E, const double *Cinv,
                     double *g, double *work_b)
{
    for (int64_t i = 0; i < n; ++i)
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Cinv[9 * i + r * 3 + c] * w[3 * i + c];
            work_b[3 * i + r] = s;
        }
    memcpy(g, v, sizeof(double) * 9 * (size_t)m);
    for (int64_t k = 0; k < N; ++k) {
        const double *Ek = E + 27 * k;
        const double *bi = work_b + 3 * (int64_t)op[k];
        double *gj = g + 9 * (int64_t)oc[k];
        for (int a = 0; a < 9; ++a)
            gj[a] -= Ek[a * 3] * bi[0] + Ek[a * 3 + 1] * bi[1] + Ek[a * 3 + 2] * bi[2];
    }
}

static double dot(const double *a, const double *b, int64_t len)
{
    double s = 0.0;
    for (int64_t t = 0; t < len; ++t) s += a[t] * b[t];
    return s;
}

/* ------------------------------------------------- Alg. 2 (DPCG), K = 1
 * Printed index slips read as: the beta branch runs for n >= 1, the update is
 * p^n = z^n + beta p^{n-1}, and the residual update uses q^n.  x^0 = 0 (Alg. 1
 * passes 0), so r^0 = b.  Preconditioner: the damped camera blocks B~_j.
 * Stopping (Reading): before each matvec, stop when ||r|| <= rtol ||b|| or
 * when the matvec count reaches max_iters; fixed_iters > 0 runs exactly that
 * many matvecs.  p^T q <= 0 (or non-finite) is a breakdown (Reading, the
 * paper is silent): the loop stops with x at the last iterate, as truncated
 * CG does on a direction of non-positive curvature, and returns
 * ORC_BREAKDOWN; the failed matvec counts. */
int orc_pcg(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
            const double *Bd, const double *E, const double *Cinv, const double *b,
            double rtol, int32_t max_iters, int32_t fixed_iters, double *x, int32_t *iters)
{
    return orc_pcg_m(m, n, N, oc, op, Bd, E, Cinv, Bd, b, rtol, max_iters, fixed_iters, x, iters);
}

/* Schur-Jacobi preconditioner blocks, an option beside Alg. 2's damped camera
 * blocks (the paper's Sec. 3 names iterative solvers on the reduced system and
 * leaves the preconditioner to Alg. 2; this is the block diagonal of S itself):
 *   M_j = B~_j - sum_{k in obs(j)} E_k C~_{i(k)}^{-1} E_k^T,
 * summed per observation, which is the diagonal block S_jj exactly when no
 * camera sees a point twice (with a repeated pair the cross terms are left out;
 * every term stays positive semi-definite, so M_j >= lambda D_j). */
void orc_schur_jacobi(int32_t m, int64_t N, const int32_t *oc, const int32_t *op,
                      const double *Bd, const double *E, const double *Cinv, double *M)
{
    memcpy(M, Bd, sizeof(double) * 81 * (size_t)m);
    for (int64_t k = 0; k < N; ++k) {
        const double *Ek = E + 27 * k;
        const double *Ci = Cinv + 9 * (int64_t)op[k];
        double T[27];   /* E_k C~^{-1}, 9x3 */
        for (int a = 0; a < 9; ++a)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d) s += Ek[a * 3 + d] * Ci[d * 3 + c];
                T[a * 3 + c] = s;
            }
        double *Mj = M + 81 * (int64_t)oc[k];
        for (int a = 0; a < 9; ++a)
            for (int b2 = 0; b2 < 9; ++b2) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += T[a * 3 + c] * Ek[b2 * 3 + c];
                Mj[a * 9 + b2] -= s;
            }
    }
}

/* The reduced camera system written out, dense [9m][9m] row-major (Eq.
 * schur_x_c): S = blockdiag(B~_j) - sum over points i of E_a C~_i^-1 E_b^T for
 * every ordered pair (a, b) of the point's observations, placed at the block
 * of cameras (cam(a), cam(b)).  This is the matrix the direct option for small
 * problems factors (Sec. 3, direct against iterative solvers). */
int orc_schur_dense(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
                    const double *Bd, const double *E, const double *Cinv, double *S)
{
    const int64_t nd = 9 * (int64_t)m;
    memset(S, 0, sizeof(double) * (size_t)(nd * nd));
    for (int64_t j = 0; j < m; ++j)
        for (int a = 0; a < 9; ++a)
            for (int b = 0; b < 9; ++b) S[(9 * j + a) * nd + 9 * j + b] = Bd[81 * j + a * 9 + b];
    /* the observations of each point, in observation order */
    int64_t *start = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *list = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!start || !list || !fill) {
        free(start); free(list); free(fill);
        return ORC_ENUMERIC;
    }
    for (int64_t k = 0; k < N; ++k) start[op[k] + 1]++;
    for (int32_t i = 0; i < n; ++i) start[i + 1] += start[i];
    for (int32_t i = 0; i < n; ++i) fill[i] = start[i];
    for (int64_t k = 0; k < N; ++k) list[fill[op[k]]++] = k;
    for (int32_t i = 0; i < n; ++i) {
        const double *Ci = Cinv + 9 * (int64_t)i;
        for (int64_t u = start[i]; u < start[i + 1]; ++u) {
            const int64_t ka = list[u];
            const double *Ea = E + 27 * ka;
            double T[27]; /* E_a C~^-1 */
            for (int a = 0; a < 9; ++a)
                for (int c = 0; c < 3; ++c) {
                    double t = 0.0;
                    for (int d = 0; d < 3; ++d) t += Ea[a * 3 + d] * Ci[d * 3 + c];
                    T[a * 3 + c] = t;
                }
            for (int64_t v = start[i]; v < start[i + 1]; ++v) {
                const int64_t kb = list[v];
                const double *Eb = E + 27 * kb;
                double *blk = S + (9 * (int64_t)oc[ka]) * nd + 9 * (int64_t)oc[kb];
                for (int a = 0; a < 9; ++a)
                    for (int b = 0; b < 9; ++b) {
                        double t = 0.0;
                        for (int c = 0; c < 3; ++c) t += T[a * 3 + c] * Eb[b * 3 + c];
                        blk[a * nd + b] -= t;
                    }
            }
        }
    }
    free(start); free(list); free(fill);
    return ORC_OK;
}

/* x = A^-1 b for a dense symmetric positive definite A [nd][nd] (row-major)
 * by its Cholesky factor and two triangular solves; ORC_ENUMERIC when A is
 * not positive definite. */
int orc_dense_solve(int64_t nd, const double *A, const double *b, double *x)
{
    double *L = malloc(sizeof(double) * (size_t)(nd * nd > 0 ? nd * nd : 1));
    double *y = malloc(sizeof(double) * (size_t)(nd > 0 ? nd : 1));
    if (!L || !y) {
        free(L); free(y);
        return ORC_ENUMERIC;
    }
    int status = cholesky(A, (int)nd, L) ? ORC_ENUMERIC : ORC_OK;
    if (status == ORC_OK) {
        for (int64_t r = 0; r < nd; ++r) {
            double t = b[r];
            for (int64_t c = 0; c < r; ++c) t -= L[r * nd + c] * y[c];
            y[r] = t / L[r * nd + r];
        }
        for (int64_t r = nd - 1; r >= 0; --r) {
            double t = y[r];
            for (int64_t c = r + 1; c < nd; ++c) t -= L[c * nd + r] * x[c];
            x[r] = t / L[r * nd + r];
        }
    }
    free(L); free(y);
    return status;
}

/* PCG of Alg. 2 with the preconditioner blocks Mblk (Bd for Alg. 2 itself). */
int orc_pcg_m(int32_t m, int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
              const double *Bd, const double *E, const double *Cinv, const double *Mblk,
              const double *b, double rtol, int32_t max_iters, int32_t fixed_iters, double *x,
              int32_t *iters)
{
    int64_t len = 9 * (int64_t)m;
    double *r = malloc(sizeof(double) * (size_t)len);
    double *z = malloc(sizeof(double) * (size_t)len);
    double *p = malloc(sizeof(double) * (size_t)len);
    double *q = malloc(sizeof(double) * (size_t)len);
    double *wa = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *wb = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *L = malloc(sizeof(double) * 81 * (size_t)(m > 0 ? m : 1));
    int status = ORC_OK;
    for (int64_t j = 0; j < m; ++j)
        if (cholesky(Mblk + 81 * j, 9, L + 81 * j)) status = ORC_ENUMERIC;
    memset(x, 0, sizeof(double) * (size_t)len);
    memcpy(r, b, sizeof(double) * (size_t)len);
    double bnorm = sqrt(dot(b, b, len));
    double rho_prev = 0.0;
    int32_t it = 0;
    while (status == ORC_OK) {
        if (fixed_iters > 0) {
            if (it >= fixed_iters) break;
        } else {
            if (sqrt(dot(r, r, len)) <= rtol * bnorm || it >= max_iters) break;
        }
        for (int64_t j = 0; j < m; ++j) chol_solve(L + 81 * j, 9, r + 9 * j, z + 9 * j);
        double rho = dot(r, z, len);
        if (it >= 1) {
            double beta = rho / rho_prev;
            for (int64_t t = 0; t < len; ++t) p[t] = z[t] + beta * p[t];
        } else {
            memcpy(p, z, sizeof(double) * (size_t)len);
        }
        orc_schur_matvec(m, n, N, oc, op, Bd, E, Cinv, p, q, wa, wb);
        ++it;
        double pq = dot(p, q, len);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = ORC_BREAKDOWN;
            break;
        }
        double alpha = rho / pq;
        for (int64_t t = 0; t < len; ++t) {
            x[t] += alpha * p[t];
            r[t] -= alpha * q[t];
        }
        rho_prev = rho;
    }
    *iters = it;
    free(r);
    free(z);
    free(p);
    free(q);
    free(wa);
    free(wb);
    free(L);
    return status;
}

/* Eq. schur_x_p: dx_p = C^{-1} (w - E^T dx_c). */
void orc_back_substitute(int32_t n, int64_t N, const int32_t *oc, const int32_t *op,
                         const double *E, const double *Cinv, const double *w,
                         const double *dc, double *dp)
{
    double *t = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    memcpy(t, w, sizeof(double) * 3 * (size_t)n);
    for (int64_t k = 0; k < N; ++k) {
        const double *Ek = E + 27 * k;
        const double *xj = dc + 9 * (int64_t)oc[k];
        double *ti = t + 3 * (int64_t)op[k];
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int a = 0; a < 9; ++a) s += Ek[a * 3 + b] * xj[a];
            ti[b] -= s;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Cinv[9 * i + r * 3 + c] * t[3 * i + c];
            dp[3 * i + r] = s;
        }
    free(t);
}

/* ------------------------------------------------------------ LM loop
 * Alg. 1 with K = 1 (build, reduced system, DPCG, back-substitution, additive
 * update) inside the trust-region wrapper of the supplementary Sec. C.
 * Reading (Ceres-like, Madsen-Nielsen-Tingleff schedule): lambda_0 from the
 * options, nu = 2; predicted decrease
 *   pred = 1/2 [dc^T (lambda D_c dc + v) + dp^T (lambda D_p dp + w)];
 * gain = (F - F') / pred; accept iff pred > 0, F' finite and
 * gain > min_relative_decrease; then lambda *= max(1/3, 1 - (2 gain - 1)^3),
 * nu = 2; otherwise lambda *= nu, nu *= 2.  Every iteration counts; the loop
 * stops after max_lm_iters, or (normally, keeping the last accepted state)
 * when lambda exceeds 1e32.  A rejected step keeps
 * the assembled system and only re-damps it. */
int orc_lm_solve(int32_t m, int32_t n, int64_t N, double *cams, double *pts,
                 const int32_t *oc, const int32_t *op, const double *uv,
                 const orc_options *opt, orc_trace *trace)
{
    size_t M = (size_t)(m > 0 ? m : 1), P = (size_t)(n > 0 ? n : 1), K = (size_t)(N > 0 ? N : 1);
    double *B = malloc(sizeof(double) * 81 * M), *Bd = malloc(sizeof(double) * 81 * M);
    double *C = malloc(sizeof(double) * 9 * P), *Cd = malloc(sizeof(double) * 9 * P);
    double *Ci = malloc(sizeof(double) * 9 * P);
    double *E = malloc(sizeof(double) * 27 * K);
    double *v = malloc(sizeof(double) * 9 * M), *w = malloc(sizeof(double) * 3 * P);
    double *Dc = malloc(sizeof(double) * 9 * M), *Dp = malloc(sizeof(double) * 3 * P);
    double *g = malloc(sizeof(double) * 9 * M), *dc = malloc(sizeof(double) * 9 * M);
    double *dp = malloc(sizeof(double) * 3 * P), *wb = malloc(sizeof(double) * 3 * P);
    double *cams_t = malloc(sizeof(double) * 9 * M), *pts_t = malloc(sizeof(double) * 3 * P);
    double *Mj = malloc(sizeof(double) * 81 * M);
    int status = ORC_OK;
    double delta = opt->huber_delta;
    double F = orc_cost(N, cams, pts, oc, op, uv, delta);
    double lambda = opt->lambda_init, nu = 2.0;
    int need_build = 1;
    int32_t it;
    trace->initial_cost = F;
    for (it = 0; it < opt->max_lm_iters; ++it) {
        if (need_build) {
            double Fb;
            orc_assemble(m, n, N, cams, pts, oc, op, uv, delta, B, C, E, v, w, &Fb);
            need_build = 0;
        }
        orc_damp(m, n, B, C, lambda, opt->damping, Bd, Cd, Dc, Dp);
        if (orc_invert_points(n, Cd, Ci)) {
            status = ORC_ENUMERIC;
            break;
        }
        orc_reduced_rhs(m, n, N, oc, op, v, w, E, Ci, g, wb);
        int32_t fixed = opt->pcg_schedule ? opt->pcg_schedule[it] : 0;
        int32_t npcg = 0;
        int pst;
        if (opt->solver == 1) {
            /* the reduced camera system written out and factored */
            const int64_t nd = 9 * (int64_t)m;
            double *S = malloc(sizeof(double) * (size_t)(nd * nd));
            pst = S ? orc_schur_dense(m, n, N, oc, op, Bd, E, Ci, S) : ORC_ENUMERIC;
            if (pst == ORC_OK) pst = orc_dense_solve(nd, S, g, dc);
            free(S);
        } else {
            if (opt->preconditioner == 1) orc_schur_jacobi(m, N, oc, op, Bd, E, Ci, Mj);
            /* a breakdown leaves dc at the last iterate, which is still a step */
            pst = orc_pcg_m(m, n, N, oc, op, Bd, E, Ci, opt->preconditioner == 1 ? Mj : Bd, g, opt->pcg_rtol,
                            opt->max_pcg_iters, fixed, dc, &npcg);
        }
        if (pst != ORC_OK && pst != ORC_BREAKDOWN) {
            trace->pcg_iters[it] = npcg;
            status = ORC_ENUMERIC;
            break;
        }
        if (trace->pcg_stop) {
            int32_t stop;
            if (opt->solver == 1) stop = ORC_PCG_DIRECT;
            else if (pst == ORC_BREAKDOWN) stop = ORC_PCG_BREAKDOWN;
            else if (fixed > 0) stop = ORC_PCG_FIXED;
            else stop = npcg >= opt->max_pcg_iters ? ORC_PCG_CAP : ORC_PCG_CONVERGED;
            trace->pcg_stop[it] = stop;
        }
        orc_back_substitute(n, N, oc, op, E, Ci, w, dc, dp);
        for (size_t t = 0; t < 9 * (size_t)m; ++t) cams_t[t] = cams[t] + dc[t];
        for (size_t t = 0; t < 3 * (size_t)n; ++t) pts_t[t] = pts[t] + dp[t];
        double Ft = orc_cost(N, cams_t, pts_t, oc, op, uv, delta);
        double pred = 0.0;
        for (size_t t = 0; t < 9 * (size_t)m; ++t) pred += dc[t] * (lambda * Dc[t] * dc[t] + v[t]);
        for (size_t t = 0; t < 3 * (size_t)n; ++t) pred += dp[t] * (lambda * Dp[t] * dp[t] + w[t]);
        pred *= 0.5;
        double gain = (F - Ft) / pred;
        int acc = pred > 0.0 && isfinite(Ft) && gain > opt->min_relative_decrease;
        trace->lambda[it] = lambda;
        trace->trial_cost[it] = Ft;
        trace->pred[it] = pred;
        trace->pcg_iters[it] = npcg;
        trace->accepted[it] = acc;
        if (acc) {
            memcpy(cams, cams_t, sizeof(double) * 9 * (size_t)m);
            memcpy(pts, pts_t, sizeof(double) * 3 * (size_t)n);
            F = Ft;
            double t = 2.0 * gain - 1.0;
            double f = 1.0 - t * t * t;
            lambda *= (f > 1.0 / 3.0 ? f : 1.0 / 3.0);
            nu = 2.0;
            need_build = 1;
        } else {
            lambda *= nu;
            nu *= 2.0;
        }
        trace->cost[it] = F;
        if (lambda > 1e32) {   /* no further progress possible: normal end */
            ++it;
            break;
        }
    }
    trace->iters_run = it;
    trace->final_cost = F;
    free(B); free(Bd); free(C); free(Cd); free(Ci); free(E); free(v); free(w);
    free(Dc); free(Dp); free(g); free(dc); free(dp); free(wb); free(cams_t); free(pts_t); free(Mj);
    return status;
}

/* One row block of the reduced camera system computed from scratch:
 *   q_j = B~_j x_j - sum_{k in obs(j)} E_k C~_{i(k)}^{-1} sum_{k' in obs(i(k))} E_k'^T x_{j(k')}
 * (Alg. 3 restricted to camera j).  cam_obs[cam_off[j]..cam_off[j+1]) lists
 * camera j's observations and pt_obs[pt_off[i]..pt_off[i+1]) point i's.
 * Returns 0, or -1 if a damped point block is not positive definite. */
double orc_schur_row(int32_t j, const double *cams, const double *pts,
                     const int32_t *oc, const int32_t *op, const double *uv, double delta,
                     double lambda, int32_t damping,
                     const int64_t *cam_off, const int64_t *cam_obs,
                     const int64_t *pt_off, const int64_t *pt_obs,
                     const double *x, double q[9])
{
    double Bs[81], vs[9], Cs[9], ws[3], F;
    orc_subset_sums(cam_obs + cam_off[j], cam_off[j + 1] - cam_off[j], cams, pts, oc, op, uv,
                    delta, Bs, vs, Cs, ws, &F);
    for (int a = 0; a < 9; ++a) Bs[a * 10] += lambda * (damping == 0 ? clamp_diag(Bs[a * 10]) : 1.0);
    for (int r = 0; r < 9; ++r) {
        double s = 0.0;
        for (int c = 0; c < 9; ++c) s += Bs[r * 9 + c] * x[9 * (int64_t)j + c];
        q[r] = s;
    }
    for (int64_t t = cam_off[j]; t < cam_off[j + 1]; ++t) {
        int64_t k = cam_obs[t];
        int64_t i = op[k];
        double Ci[9] = {0}, a[3] = {0}, Ekk[27] = {0};
        for (int64_t u = pt_off[i]; u < pt_off[i + 1]; ++u) {
            int64_t k2 = pt_obs[u];
            double e[2], Jc[18], Jp[6];
            orc_residual_jacobian(cams + 9 * (int64_t)oc[k2], pts + 3 * i, uv + 2 * k2, e, Jc, Jp);
            double wt = orc_rho_prime(e[0] * e[0] + e[1] * e[1], delta);
            const double *xj = x + 9 * (int64_t)oc[k2];
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c) Ci[r * 3 + c] += wt * (Jp[r] * Jp[c] + Jp[3 + r] * Jp[3 + c]);
            }
            for (int aa = 0; aa < 9; ++aa)
                for (int b = 0; b < 3; ++b) {
                    double h = wt * (Jc[aa] * Jp[b] + Jc[9 + aa] * Jp[3 + b]);
                    a[b] += h * xj[aa];
                    if (k2 == k) Ekk[aa * 3 + b] = h;
                }
        }
        for (int r = 0; r < 3; ++r) Ci[r * 4] += lambda * (damping == 0 ? clamp_diag(Ci[r * 4]) : 1.0);
        double L[9], b[3];
        if (cholesky(Ci, 3, L)) return -1.0;
        chol_solve(L, 3, a, b);
        for (int r = 0; r < 9; ++r) q[r] -= Ekk[r * 3] * b[0] + Ekk[r * 3 + 1] * b[1] + Ekk[r * 3 + 2] * b[2];
    }
    return 0.0;
}

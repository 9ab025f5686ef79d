/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * Plain FP64 CPU implementation of pose graph optimisation (PGO) with the
 * same Levenberg-Marquardt iteration as the bundle-adjustment oracle (the
 * paper's second workload, Sec. IV-D, Eq. 4 and Eq. 5):
 *
 *   Z* = argmin_Z 1/2 sum_(i,j) r_ij^T Omega_ij r_ij,
 *   r_ij = Log(zeta_i^-1 zeta_j T_ij^-1)            (in se(3), R^6)
 *
 * Conventions (shared with the bundle-adjustment oracle where they apply):
 *   pose     [tx ty tz qx qy qz qw], the 4x4 transform [R(q) t; 0 1];
 *   tangent  delta = (rho, phi), left update zeta <- Exp(delta) zeta with
 *            Exp(rho, phi) = [Exp_SO3(phi)  V(phi) rho; 0 1];
 *   Log      the inverse of that Exp (phi from the rotation, rho = V^-1 t);
 *   Jacobian with E = zeta_i^-1 zeta_j T_ij^-1 and r = Log(E),
 *              d r / d delta_j =  Jl^-1(r) Ad(zeta_i^-1),
 *              d r / d delta_i = -Jl^-1(r) Ad(zeta_i^-1),
 *            where Ad(R, t) = [R  t^ R; 0  R] and Jl^-1(xi) is the inverse
 *            left Jacobian, evaluated here by its power series in ad_xi
 *            (ad_xi = [phi^  rho^; 0  phi^]): Jl^-1 = sum_n B_n / n! ad^n,
 *            the Bernoulli numbers B_n of x / (e^x - 1);
 *   solve    Gauss-Newton system H = sum J^T Omega J, g = sum J^T Omega r,
 *            clamped diagonal damping, block-Jacobi PCG on the 6x6 block
 *            pattern of the edges (x0 = 0, relative tolerance), or dense
 *            Cholesky; trust-region rule and acceptance as for bundle
 *            adjustment (orc_lambda_update).
 * Fixed poses (gauge anchors) have zero Jacobian blocks and a zero step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

double orc_lambda_update(int accepted, double ratio, double lambda, double lambda_min,
                         double lambda_max);

typedef struct {
    double cg_rtol;
    int32_t cg_maxiter;
    double lambda0, lambda_min, lambda_max;
    double diag_min, diag_max;
    int32_t solver; /* 0 PCG, 1 dense Cholesky */
} pgo_options;

typedef struct {
    double cost_before, cost_after, lambda_used, lambda_next;
    double cg_rel_resid, pred, grad_inf;
    int32_t accepted, cg_iters, cg_breakdown, status;
} pgo_step_info;

typedef struct {
    pgo_options o;
    int32_t n, m;            /* poses, edges */
    int32_t *ei, *ej;
    double *T;               /* [m][7] measurements */
    double *Om;              /* [m][36] information */
    uint8_t *fixed;
    double *Z, *Znew;        /* [n][7] */
    double lambda;
    /* block pattern of H: upper blocks (a, b), a <= b, diagonal first */
    int64_t *H_ptr, nnzb;
    int32_t *H_col;
    double *H, *g, *dx;      /* [nnzb][36], [n][6], [n][6] */
    double *r, *J;           /* [m][6], [m][36] (d r / d delta_j) */
    double F;
} pgo_ctx;

/* ------------------------------------------------------------------------ */
/* small SE(3) helpers (4x4 transforms as R[9], t[3])                        */
/* ------------------------------------------------------------------------ */

static void hat3(const double v[3], double M[9])
{
    M[0] = 0;     M[1] = -v[2]; M[2] = v[1];
    M[3] = v[2];  M[4] = 0;     M[5] = -v[0];
    M[6] = -v[1]; M[7] = v[0];  M[8] = 0;
}

static void mat3_mul(const double A[9], const double B[9], double C[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

static void pose_to_Rt(const double *p, double R[9], double t[3])
{
    const double x = p[3], y = p[4], z = p[5], w = p[6];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
    R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
    R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
    t[0] = p[0]; t[1] = p[1]; t[2] = p[2];
}

/* inverse of (R, t): (R^T, -R^T t) */
static void inv_Rt(const double R[9], const double t[3], double Ri[9], double ti[3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Ri[3 * i + j] = R[3 * j + i];
    for (int i = 0; i < 3; ++i) ti[i] = -(Ri[3 * i] * t[0] + Ri[3 * i + 1] * t[1] + Ri[3 * i + 2] * t[2]);
}

/* (R1, t1) (R2, t2) */
static void compose(const double R1[9], const double t1[3], const double R2[9], const double t2[3],
                    double R[9], double t[3])
{
    mat3_mul(R1, R2, R);
    for (int i = 0; i < 3; ++i)
        t[i] = R1[3 * i] * t2[0] + R1[3 * i + 1] * t2[1] + R1[3 * i + 2] * t2[2] + t1[i];
}

/* Log of (R, t): xi = (rho, phi) with Exp(xi) = (R, t) */
static void se3_log(const double R[9], const double t[3], double xi[6])
{
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    const double th = acos(c);
    const double w[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    /* phi = th / (2 sin th) (R - R^T)^v; series 1/2 + th^2/12 below 1e-4 */
    const double s = th < 1e-4 ? 0.5 + th * th / 12.0 : th / (2.0 * sin(th));
    double phi[3] = {s * w[0], s * w[1], s * w[2]};
    /* rho = V^-1 t, V^-1 = I - 1/2 phi^ + a phi^2, a = (1 - th sin th / (2 (1 - cos th))) / th^2 */
    const double a = th < 1e-4 ? 1.0 / 12.0 + th * th / 720.0
                               : (1.0 - th * sin(th) / (2.0 * (1.0 - cos(th)))) / (th * th);
    double P[9], P2[9];
    hat3(phi, P);
    mat3_mul(P, P, P2);
    for (int i = 0; i < 3; ++i) {
        double v = t[i];
        for (int k = 0; k < 3; ++k) v += (-0.5 * P[3 * i + k] + a * P2[3 * i + k]) * t[k];
        xi[i] = v;
    }
    xi[3] = phi[0];
    xi[4] = phi[1];
    xi[5] = phi[2];
}

/* Ad(R, t) = [R  t^ R; 0  R] (6x6 row-major, acting on (rho, phi)) */
static void adjoint6(const double R[9], const double t[3], double A[36])
{
    double Th[9], TR[9];
    hat3(t, Th);
    mat3_mul(Th, R, TR);
    memset(A, 0, 36 * sizeof(double));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            A[6 * i + j] = R[3 * i + j];
            A[6 * i + 3 + j] = TR[3 * i + j];
            A[6 * (3 + i) + 3 + j] = R[3 * i + j];
        }
}

static void mat6_mul(const double *A, const double *B, double *C)
{
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += A[6 * i + k] * B[6 * k + j];
            C[6 * i + j] = s;
        }
}

/* Jl^-1(xi) = sum_n c_n ad_xi^n with c_n = B_n / n! the coefficients of
 * x / (e^x - 1) (Bernoulli numbers, B_1 = -1/2): from (e^x - 1) / x times
 * that series being 1, c_0 = 1 and c_n = -sum_{k<n} c_k / (n - k + 1)!.
 * Forty terms (the series converges for |phi| < 2 pi). */
void orc_se3_jl_inv(const double xi[6], double Jinv[36])
{
    enum { NT = 40 };
    double cf[NT], inv_fact[NT + 2];
    inv_fact[0] = 1.0;
    for (int k = 1; k < NT + 2; ++k) inv_fact[k] = inv_fact[k - 1] / k;
    cf[0] = 1.0;
    for (int n = 1; n < NT; ++n) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += cf[k] * inv_fact[n - k + 1];
        cf[n] = -s;
    }
    const int nterms = NT;
    const double *bern_over_fact = cf;
    double ad[36], pw[36], tmp[36];
    double ph[9], rh[9];
    hat3(xi + 3, ph);
    hat3(xi, rh);
    memset(ad, 0, sizeof ad);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            ad[6 * i + j] = ph[3 * i + j];
            ad[6 * i + 3 + j] = rh[3 * i + j];
            ad[6 * (3 + i) + 3 + j] = ph[3 * i + j];
        }
    memset(pw, 0, sizeof pw);
    for (int i = 0; i < 6; ++i) pw[7 * i] = 1.0;
    memset(Jinv, 0, 36 * sizeof(double));
    for (int n = 0; n < nterms; ++n) {
        for (int q = 0; q < 36; ++q) Jinv[q] += bern_over_fact[n] * pw[q];
        mat6_mul(pw, ad, tmp);
        memcpy(pw, tmp, sizeof pw);
    }
}

/* residual and d r / d delta_j of one edge at poses Zi, Zj with measurement T */
void orc_pgo_edge(const double *Zi, const double *Zj, const double *T, double r[6], double Jj[36])
{
    double Ri[9], ti[3], Rj[9], tj[3], RT[9], tT[3];
    pose_to_Rt(Zi, Ri, ti);
    pose_to_Rt(Zj, Rj, tj);
    pose_to_Rt(T, RT, tT);
    double Rii[9], tii[3], RTi[9], tTi[3], Ra[9], ta[3], Re[9], te[3];
    inv_Rt(Ri, ti, Rii, tii);
    inv_Rt(RT, tT, RTi, tTi);
    compose(Rii, tii, Rj, tj, Ra, ta);
    compose(Ra, ta, RTi, tTi, Re, te);
    se3_log(Re, te, r);
    if (Jj) {
        double Jl[36], Ad[36];
        orc_se3_jl_inv(r, Jl);
        adjoint6(Rii, tii, Ad);
        mat6_mul(Jl, Ad, Jj);
    }
}

/* left retraction of a pose by delta = (rho, phi): exact SE(3) exponential */
static void retract(const double *Z, const double *d, double *out)
{
    const double *rho = d, *phi = d + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], th = sqrt(th2);
    double A, B, C; /* sin th / th, (1 - cos th) / th^2, (th - sin th) / th^3 */
    if (th < 1e-5) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double P[9], P2[9], Rd[9], V[9];
    hat3(phi, P);
    mat3_mul(P, P, P2);
    for (int q = 0; q < 9; ++q) {
        const double I = (q % 4 == 0) ? 1.0 : 0.0;
        Rd[q] = I + A * P[q] + B * P2[q];
        V[q] = I + B * P[q] + C * P2[q];
    }
    double td[3];
    for (int i = 0; i < 3; ++i) td[i] = V[3 * i] * rho[0] + V[3 * i + 1] * rho[1] + V[3 * i + 2] * rho[2];
    double R[9], t[3], Rn[9], tn[3];
    pose_to_Rt(Z, R, t);
    compose(Rd, td, R, t, Rn, tn);
    /* rotation matrix -> quaternion (largest-component branch), normalised */
    double q[4];
    const double tr = Rn[0] + Rn[4] + Rn[8];
    if (tr > 0) {
        const double s = 2.0 * sqrt(tr + 1.0);
        q[3] = 0.25 * s;
        q[0] = (Rn[7] - Rn[5]) / s;
        q[1] = (Rn[2] - Rn[6]) / s;
        q[2] = (Rn[3] - Rn[1]) / s;
    } else if (Rn[0] > Rn[4] && Rn[0] > Rn[8]) {
        const double s = 2.0 * sqrt(1.0 + Rn[0] - Rn[4] - Rn[8]);
        q[3] = (Rn[7] - Rn[5]) / s;
        q[0] = 0.25 * s;
        q[1] = (Rn[1] + Rn[3]) / s;
        q[2] = (Rn[2] + Rn[6]) / s;
    } else if (Rn[4] > Rn[8]) {
        const double s = 2.0 * sqrt(1.0 + Rn[4] - Rn[0] - Rn[8]);
        q[3] = (Rn[2] - Rn[6]) / s;
        q[0] = (Rn[1] + Rn[3]) / s;
        q[1] = 0.25 * s;
        q[2] = (Rn[5] + Rn[7]) / s;
    } else {
        const double s = 2.0 * sqrt(1.0 + Rn[8] - Rn[0] - Rn[4]);
        q[3] = (Rn[3] - Rn[1]) / s;
        q[0] = (Rn[2] + Rn[6]) / s;
        q[1] = (Rn[5] + Rn[7]) / s;
        q[2] = 0.25 * s;
    }
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (q[3] < 0) {
        for (int k = 0; k < 4; ++k) q[k] = -q[k];
    }
    out[0] = tn[0];
    out[1] = tn[1];
    out[2] = tn[2];
    for (int k = 0; k < 4; ++k) out[3 + k] = q[k] / qn;
}

void orc_pgo_retract(const double *Z, const double *d, double *out) { retract(Z, d, out); }

/* ------------------------------------------------------------------------ */
/* context                                                                   */
/* ------------------------------------------------------------------------ */

static void *zalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

static int cmp_int(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

pgo_ctx *orc_pgo_create(const pgo_options *o, int32_t n, int32_t m, const int32_t *ei,
                        const int32_t *ej, const double *T, const double *omega, const uint8_t *fixed)
{
    pgo_ctx *c = zalloc(1, sizeof(pgo_ctx));
    c->o = *o;
    c->n = n;
    c->m = m;
    c->ei = zalloc((size_t)m, sizeof(int32_t));
    c->ej = zalloc((size_t)m, sizeof(int32_t));
    memcpy(c->ei, ei, sizeof(int32_t) * m);
    memcpy(c->ej, ej, sizeof(int32_t) * m);
    c->T = zalloc((size_t)m * 7, sizeof(double));
    memcpy(c->T, T, sizeof(double) * 7 * m);
    c->Om = zalloc((size_t)m * 36, sizeof(double));
    for (int32_t e = 0; e < m; ++e)
        for (int q = 0; q < 36; ++q) c->Om[36 * e + q] = omega ? omega[36 * e + q] : (q % 7 == 0 ? 1.0 : 0.0);
    c->fixed = zalloc((size_t)n, 1);
    if (fixed) memcpy(c->fixed, fixed, n);
    c->Z = zalloc((size_t)n * 7, sizeof(double));
    c->Znew = zalloc((size_t)n * 7, sizeof(double));
    c->lambda = o->lambda0;
    /* pattern: diagonal plus (min, max) of every edge, sorted, unique */
    int32_t *cnt = zalloc((size_t)n, sizeof(int32_t));
    for (int32_t e = 0; e < m; ++e) cnt[ei[e] < ej[e] ? ei[e] : ej[e]]++;
    int64_t *ptr = zalloc((size_t)n + 1, sizeof(int64_t));
    for (int32_t a = 0; a < n; ++a) ptr[a + 1] = ptr[a] + 1 + cnt[a];
    int32_t *cols = zalloc((size_t)ptr[n], sizeof(int32_t));
    int64_t *fill = zalloc((size_t)n, sizeof(int64_t));
    for (int32_t a = 0; a < n; ++a) cols[ptr[a] + fill[a]++] = a;
    for (int32_t e = 0; e < m; ++e) {
        const int32_t a = ei[e] < ej[e] ? ei[e] : ej[e], b = ei[e] < ej[e] ? ej[e] : ei[e];
        cols[ptr[a] + fill[a]++] = b;
    }
    c->H_ptr = zalloc((size_t)n + 1, sizeof(int64_t));
    c->H_col = zalloc((size_t)ptr[n], sizeof(int32_t));
    for (int32_t a = 0; a < n; ++a) {
        int32_t *row = cols + ptr[a];
        const int64_t len = ptr[a + 1] - ptr[a];
        qsort(row, (size_t)len, sizeof(int32_t), cmp_int);
        int64_t u = 0;
        for (int64_t k = 0; k < len; ++k)
            if (u == 0 || row[k] != row[u - 1]) row[u++] = row[k];
        c->H_ptr[a + 1] = c->H_ptr[a] + u;
        memcpy(c->H_col + c->H_ptr[a], row, sizeof(int32_t) * u);
    }
    c->nnzb = c->H_ptr[n];
    free(cnt);
    free(ptr);
    free(cols);
    free(fill);
    c->H = zalloc((size_t)c->nnzb * 36, sizeof(double));
    c->g = zalloc((size_t)n * 6, sizeof(double));
    c->dx = zalloc((size_t)n * 6, sizeof(double));
    c->r = zalloc((size_t)m * 6, sizeof(double));
    c->J = zalloc((size_t)m * 36, sizeof(double));
    return c;
}

void orc_pgo_destroy(pgo_ctx *c)
{
    if (!c) return;
    void *p[] = {c->ei, c->ej, c->T, c->Om, c->fixed, c->Z, c->Znew, c->H_ptr, c->H_col,
                 c->H, c->g, c->dx, c->r, c->J};
    for (size_t i = 0; i < sizeof p / sizeof p[0]; ++i) free(p[i]);
    free(c);
}

void orc_pgo_set_poses(pgo_ctx *c, const double *Z) { memcpy(c->Z, Z, sizeof(double) * 7 * c->n); }
void orc_pgo_get_poses(const pgo_ctx *c, double *Z) { memcpy(Z, c->Z, sizeof(double) * 7 * c->n); }
void orc_pgo_set_lambda(pgo_ctx *c, double l) { c->lambda = l; }
int64_t orc_pgo_nnzb(const pgo_ctx *c) { return c->nnzb; }

static double edge_cost(const double *Om, const double r[6])
{
    double s = 0.0;
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) s += r[a] * Om[6 * a + b] * r[b];
    return 0.5 * s;
}

/* F = 1/2 sum r^T Omega r at poses Z (Eq. 4 with the conventional 1/2) */
double orc_pgo_cost(const pgo_ctx *c, const double *Z)
{
    double F = 0.0;
    for (int32_t e = 0; e < c->m; ++e) {
        double r[6];
        orc_pgo_edge(Z + 7 * (int64_t)c->ei[e], Z + 7 * (int64_t)c->ej[e], c->T + 7 * (int64_t)e, r, NULL);
        F += edge_cost(c->Om + 36 * (int64_t)e, r);
    }
    return F;
}

static int64_t find_blk(const pgo_ctx *c, int32_t a, int32_t b)
{
    for (int64_t k = c->H_ptr[a]; k < c->H_ptr[a + 1]; ++k)
        if (c->H_col[k] == b) return k;
    return -1;
}

/* J of the edge with respect to delta_i (-Jj) and delta_j (Jj), fixed poses zeroed */
static void edge_blocks(const pgo_ctx *c, int32_t e, double Ji[36], double Jj[36])
{
    const double *J = c->J + 36 * (int64_t)e;
    for (int q = 0; q < 36; ++q) {
        Ji[q] = c->fixed[c->ei[e]] ? 0.0 : -J[q];
        Jj[q] = c->fixed[c->ej[e]] ? 0.0 : J[q];
    }
}

/* H = sum J^T Omega J, g = sum J^T Omega r (upper blocks), edge by edge */
static void linearize(pgo_ctx *c)
{
    memset(c->H, 0, sizeof(double) * 36 * c->nnzb);
    memset(c->g, 0, sizeof(double) * 6 * c->n);
    double F = 0.0;
    for (int32_t e = 0; e < c->m; ++e) {
        double *r = c->r + 6 * (int64_t)e;
        orc_pgo_edge(c->Z + 7 * (int64_t)c->ei[e], c->Z + 7 * (int64_t)c->ej[e], c->T + 7 * (int64_t)e, r,
                     c->J + 36 * (int64_t)e);
        const double *Om = c->Om + 36 * (int64_t)e;
        F += edge_cost(Om, r);
        double Jb[2][36];
        edge_blocks(c, e, Jb[0], Jb[1]);
        const int32_t v[2] = {c->ei[e], c->ej[e]};
        double OJ[2][36], Or[6];
        for (int s = 0; s < 2; ++s)
            for (int a = 0; a < 6; ++a)
                for (int k = 0; k < 6; ++k) {
                    double t = 0.0;
                    for (int b = 0; b < 6; ++b) t += Om[6 * a + b] * Jb[s][6 * b + k];
                    OJ[s][6 * a + k] = t;
                }
        for (int a = 0; a < 6; ++a) {
            double t = 0.0;
            for (int b = 0; b < 6; ++b) t += Om[6 * a + b] * r[b];
            Or[a] = t;
        }
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < 6; ++k) {
                double t = 0.0;
                for (int a = 0; a < 6; ++a) t += Jb[s][6 * a + k] * Or[a];
                c->g[6 * v[s] + k] += t;
            }
        for (int s = 0; s < 2; ++s)
            for (int u = 0; u < 2; ++u) {
                if (v[s] > v[u] || (v[s] == v[u] && s != u)) continue;
                double *B = c->H + 36 * find_blk(c, v[s], v[u]);
                for (int k = 0; k < 6; ++k)
                    for (int l = 0; l < 6; ++l) {
                        double t = 0.0;
                        for (int a = 0; a < 6; ++a) t += Jb[s][6 * a + k] * OJ[u][6 * a + l];
                        B[6 * k + l] += t;
                    }
            }
    }
    c->F = F;
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

static void spmv(const pgo_ctx *c, const double *H, const double *x, double *y)
{
    memset(y, 0, sizeof(double) * 6 * c->n);
    for (int32_t a = 0; a < c->n; ++a)
        for (int64_t e = c->H_ptr[a]; e < c->H_ptr[a + 1]; ++e) {
            const int32_t b = c->H_col[e];
            const double *B = H + 36 * e;
            for (int i = 0; i < 6; ++i)
                for (int k = 0; k < 6; ++k) y[6 * a + i] += B[6 * i + k] * x[6 * b + k];
            if (b != a)
                for (int i = 0; i < 6; ++i)
                    for (int k = 0; k < 6; ++k) y[6 * b + k] += B[6 * i + k] * x[6 * a + i];
        }
}

static double dotn(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static int chol(int n, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            if (i == j) {
                if (!(s > 0)) return -1;
                L[i * n + i] = sqrt(s);
            } else {
                L[i * n + j] = s / L[j * n + j];
            }
        }
    return 0;
}

static void chol_solve(int n, const double *L, const double *b, double *x)
{
    double *y = zalloc((size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
        y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
    free(y);
}

/* (H + lambda diag(clamp(diag H))) dx = -g: block-Jacobi PCG or dense Cholesky */
static int solve(pgo_ctx *c, double rtol, int32_t maxiter, pgo_step_info *info)
{
    const int64_t nn = 6 * (int64_t)c->n;
    double *Hd = zalloc((size_t)c->nnzb * 36, sizeof(double));
    memcpy(Hd, c->H, sizeof(double) * 36 * c->nnzb);
    for (int32_t a = 0; a < c->n; ++a) {
        double *D = Hd + 36 * c->H_ptr[a];
        for (int i = 0; i < 6; ++i) D[7 * i] += c->lambda * clampd(D[7 * i], c->o.diag_min, c->o.diag_max);
    }
    double *b = zalloc((size_t)nn, sizeof(double));
    for (int64_t i = 0; i < nn; ++i) b[i] = -c->g[i];
    double *x = c->dx;
    memset(x, 0, sizeof(double) * nn);
    int st = 0;
    const double bn = sqrt(dotn(nn, b, b));
    if (c->o.solver == 1) {
        double *A = zalloc((size_t)(nn * nn), sizeof(double)), *L = zalloc((size_t)(nn * nn), sizeof(double));
        for (int32_t a = 0; a < c->n; ++a)
            for (int64_t e = c->H_ptr[a]; e < c->H_ptr[a + 1]; ++e) {
                const int32_t bb = c->H_col[e];
                for (int i = 0; i < 6; ++i)
                    for (int k = 0; k < 6; ++k) {
                        A[(6 * a + i) * nn + 6 * bb + k] = Hd[36 * e + 6 * i + k];
                        A[(6 * bb + k) * nn + 6 * a + i] = Hd[36 * e + 6 * i + k];
                    }
            }
        st = chol((int)nn, A, L);
        if (!st) chol_solve((int)nn, L, b, x);
        info->cg_iters = 0;
        free(A);
        free(L);
        double *q = zalloc((size_t)nn, sizeof(double));
        spmv(c, Hd, x, q);
        for (int64_t i = 0; i < nn; ++i) q[i] = b[i] - q[i];
        info->cg_rel_resid = bn > 0 ? sqrt(dotn(nn, q, q)) / bn : 0.0;
        free(q);
    } else {
        double *Lb = zalloc((size_t)c->n * 36, sizeof(double));
        for (int32_t a = 0; a < c->n && !st; ++a) st = chol(6, Hd + 36 * c->H_ptr[a], Lb + 36 * a);
        double *r = zalloc((size_t)nn, sizeof(double)), *z = zalloc((size_t)nn, sizeof(double));
        double *p = zalloc((size_t)nn, sizeof(double)), *q = zalloc((size_t)nn, sizeof(double));
        memcpy(r, b, sizeof(double) * nn);
        int32_t it = 0, brk = 0;
        double rn = bn;
        if (!st && bn > 0) {
            for (int32_t a = 0; a < c->n; ++a) chol_solve(6, Lb + 36 * a, r + 6 * a, z + 6 * a);
            memcpy(p, z, sizeof(double) * nn);
            double rz = dotn(nn, r, z);
            for (int32_t k = 1; k <= maxiter; ++k) {
                spmv(c, Hd, p, q);
                const double pq = dotn(nn, p, q);
                if (!(pq > 0)) {
                    brk = 1;
                    break;
                }
                const double al = rz / pq;
                for (int64_t i = 0; i < nn; ++i) {
                    x[i] += al * p[i];
                    r[i] -= al * q[i];
                }
                it = k;
                rn = sqrt(dotn(nn, r, r));
                if (rn <= rtol * bn) break;
                for (int32_t a = 0; a < c->n; ++a) chol_solve(6, Lb + 36 * a, r + 6 * a, z + 6 * a);
                const double rz2 = dotn(nn, r, z);
                const double be = rz2 / rz;
                rz = rz2;
                for (int64_t i = 0; i < nn; ++i) p[i] = z[i] + be * p[i];
            }
        }
        info->cg_iters = it;
        info->cg_breakdown = brk;
        info->cg_rel_resid = bn > 0 ? rn / bn : 0.0;
        free(Lb);
        free(r);
        free(z);
        free(p);
        free(q);
    }
    free(Hd);
    free(b);
    return st;
}

/* One LM iteration (Alg. 1) of PGO: linearise, damp, solve, candidate
 * poses, cost, acceptance and the damping update.  rtol / maxiter < 0 take
 * the options' values. */
int orc_pgo_lm_step(pgo_ctx *c, double rtol, int32_t maxiter, pgo_step_info *info)
{
    memset(info, 0, sizeof *info);
    linearize(c);
    info->cost_before = c->F;
    info->lambda_used = c->lambda;
    double gi = 0.0;
    for (int64_t i = 0; i < 6 * (int64_t)c->n; ++i) gi = fmax(gi, fabs(c->g[i]));
    info->grad_inf = gi;
    if (solve(c, rtol < 0 ? c->o.cg_rtol : rtol, maxiter < 0 ? c->o.cg_maxiter : maxiter, info))
        return info->status = -2;
    /* predicted reduction of the Gauss-Newton model: -g.dx - 1/2 |J dx|_Omega^2 */
    double lin = dotn(6 * (int64_t)c->n, c->g, c->dx), quad = 0.0;
    for (int32_t e = 0; e < c->m; ++e) {
        double Jb[2][36];
        edge_blocks(c, e, Jb[0], Jb[1]);
        const double *di = c->dx + 6 * (int64_t)c->ei[e], *dj = c->dx + 6 * (int64_t)c->ej[e];
        double u[6];
        for (int a = 0; a < 6; ++a) {
            double t = 0.0;
            for (int k = 0; k < 6; ++k) t += Jb[0][6 * a + k] * di[k] + Jb[1][6 * a + k] * dj[k];
            u[a] = t;
        }
        quad += 2.0 * edge_cost(c->Om + 36 * (int64_t)e, u);
    }
    info->pred = -lin - 0.5 * quad;
    for (int32_t a = 0; a < c->n; ++a) {
        if (c->fixed[a]) memcpy(c->Znew + 7 * a, c->Z + 7 * a, sizeof(double) * 7);
        else retract(c->Z + 7 * a, c->dx + 6 * a, c->Znew + 7 * a);
    }
    const double Fn = orc_pgo_cost(c, c->Znew);
    info->cost_after = Fn;
    const double ratio = (c->F - Fn) / info->pred;
    const int acc = isfinite(Fn) && Fn < c->F && info->pred > 0;
    info->accepted = acc;
    c->lambda = orc_lambda_update(acc, ratio, c->lambda, c->o.lambda_min, c->o.lambda_max);
    info->lambda_next = c->lambda;
    if (acc) {
        double *t = c->Z;
        c->Z = c->Znew;
        c->Znew = t;
    }
    return 0;
}

/* read-back for tests: H (upper blocks, undamped), g, the last step dx */
void orc_pgo_get_system(const pgo_ctx *c, int64_t *H_ptr, int32_t *H_col, double *H, double *g, double *dx)
{
    if (H_ptr) memcpy(H_ptr, c->H_ptr, sizeof(int64_t) * (c->n + 1));
    if (H_col) memcpy(H_col, c->H_col, sizeof(int32_t) * c->nnzb);
    if (H) memcpy(H, c->H, sizeof(double) * 36 * c->nnzb);
    if (g) memcpy(g, c->g, sizeof(double) * 6 * c->n);
    if (dx) memcpy(dx, c->dx, sizeof(double) * 6 * c->n);
}

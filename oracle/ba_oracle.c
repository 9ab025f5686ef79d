/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of one
 * Levenberg-Marquardt iteration of bundle adjustment, written to be checked
 * against the paper by eye.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may build, load or call it; the GPU
 * library shares no code with it.
 *
 * What it computes (paper: "Bundle Adjustment in the Eager Mode"):
 *   - the BA objective over observed (camera, point) pairs only (Eq. 1 and the
 *     Notation paragraph of Sec. III-A);
 *   - one LM iteration (Alg. 1, Eq. 2): Jacobian, A = J^T J, damping
 *     A + lambda diag(A) with diagonal clamping (Sec. IV-B-3), solve, strategy
 *     update of lambda from the ratio of actual to predicted reduction
 *     (Sec. V, TrustRegion(up=2, down=1/16));
 *   - the linear solve by PCG with a block-diagonal preconditioner
 *     (Sec. IV-C-2), applied to the Schur complement of the damped system on
 *     the cameras (the paper does not name the Schur complement; this oracle
 *     eliminates the points exactly, which yields the same step as solving
 *     the damped full system).
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   camera model  BAL pinhole with radial distortion, 9 tangent parameters
 *                 (6 pose + f, k1, k2) or 6 (pose only); pose stored as
 *                 [tx ty tz qx qy qz qw], world->camera, Y = R X + t,
 *                 pixel = f D(s) (-Yx/Yz, -Yy/Yz), D = 1 + k1 s + k2 s^2.
 *   retraction    left update T <- Exp(delta) T on SE(3), delta = (rho, phi);
 *                 intrinsics and points additive.
 *   loss          Huber on the squared residual norm, F = 1/2 sum w rho(s);
 *                 Gauss-Newton weights w_k rho'(s_k).
 *   damping       D = clamp(diag A, dmin, dmax), A* = A + lambda diag(D).
 *   LM control    accept iff F' < F, F' finite, pred > 0;
 *                 ratio > 0.75 -> lambda/2; ratio <= 0.25 or reject -> 16 lambda.
 *   PCG           x0 = 0, relative tolerance on the recursively updated residual.
 *   direct solve  the paper's Cholesky alternative (Sec. IV-C-1) applied to the
 *                 reduced camera system, assembled dense: S = L L^T.
 *   stopping      orc_solve: lambda_max rejection, plateau of relative decrease,
 *                 gradient norm, iteration cap (Sec. V, StopOnPlateau).
 *
 * Threads: loops over independent units (observations, points, cameras, rows
 * of the reduced system) run under OpenMP; every sum keeps one fixed order
 * (each output accumulated by one thread in the order of the sequential
 * loop, scalar totals summed sequentially from per-unit terms), so results
 * are bitwise the same for every thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t d;            /* camera tangent dimension: 9 or 6 */
    double huber_delta;   /* <= 0 selects the plain squared loss */
    double cg_rtol;
    int32_t cg_maxiter;
    double lambda0, lambda_min, lambda_max;
    double diag_min, diag_max;
    int32_t solver;       /* 0: block-Jacobi PCG; 1: dense Cholesky of the
                             reduced camera system (Sec. IV-C-1) */
} orc_options;

typedef struct {
    double cost_before, cost_after, lambda_used, lambda_next;
    double cg_rel_resid, pred, grad_inf;
    int32_t accepted, cg_iters, cg_breakdown, status;
} orc_step_info;

typedef struct orc_ctx {
    orc_options o;
    int32_t nc, np;
    int64_t no;
    int32_t *cidx, *pidx;
    double *obs, *ow;
    uint8_t *fixed;
    double *cams, *pts;
    double lambda;
    /* observation lists per point and per camera, in input order; and per
     * camera ordered by (point, input order), the order in which the
     * point-by-point Schur accumulation reaches a camera's blocks */
    int64_t *pt_ptr, *pt_obs, *cam_ptr, *cam_obs, *cam_obs_pt;
    /* transposed pattern: for column b the upper blocks (a, b), a < b,
     * ascending a */
    int64_t *T_ptr, *T_blk;
    int32_t *T_row;
    double *term; /* per-observation scratch for sequential totals */
    /* linearisation at the current parameters */
    int have_lin;
    double F;
    double *r, *w, *Jc, *Jp;
    double *U, *V, *gc, *gp;
    /* reduced camera system, upper block triangle, row-major blocks */
    int64_t *S_ptr, nnzb;
    int32_t *S_col;
    double *S, *bS;
    double *Vinv;
    double *dc, *dp;
    double *cams_new, *pts_new;
} orc_ctx;

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                       */
/* ------------------------------------------------------------------------ */

static void quat_to_rot(const double q[4], double R[9])
{
    const double x = q[0], y = q[1], z = q[2], w = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
    R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
    R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Cholesky factor L (lower, row-major n x n) of SPD A; returns 0 on success. */
static int cholesky(int n, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i) {
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
    }
    return 0;
}

/* solve L L^T x = b */
static void cholesky_solve(int n, const double *L, const double *b, double *x)
{
    double y[16];
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
}

/* inverse of a 3x3 matrix by the adjugate; returns the determinant */
static double inverse3(const double A[9], double Ai[9])
{
    const double c00 = A[4] * A[8] - A[5] * A[7];
    const double c01 = A[5] * A[6] - A[3] * A[8];
    const double c02 = A[3] * A[7] - A[4] * A[6];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    const double id = 1.0 / det;
    Ai[0] = c00 * id;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    Ai[3] = c01 * id;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    Ai[6] = c02 * id;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return det;
}

/* ------------------------------------------------------------------------ */
/* camera model (Eq. 1) and its Jacobian                                     */
/* ------------------------------------------------------------------------ */

/* Pixel of world point X in camera `cam`; when Jc/Jp are given also the
 * derivatives of the pixel w.r.t. the camera tangent (2 x d, row-major; left
 * SE(3) perturbation, then f, k1, k2) and the point (2 x 3).  Returns Y_z. */
double orc_project(const double *cam, const double *X, int32_t d, double *pix,
                   double *Jc, double *Jp)
{
    double R[9];
    quat_to_rot(cam + 3, R);
    double Y[3];
    for (int i = 0; i < 3; ++i)
        Y[i] = R[3 * i] * X[0] + R[3 * i + 1] * X[1] + R[3 * i + 2] * X[2] + cam[i];
    const double f = cam[7], k1 = cam[8], k2 = cam[9];
    const double u = -Y[0] / Y[2], v = -Y[1] / Y[2];
    const double s = u * u + v * v;
    const double D = 1.0 + k1 * s + k2 * s * s;
    pix[0] = f * D * u;
    pix[1] = f * D * v;
    if (!Jc && !Jp) return Y[2];

    /* d pixel / d(u,v) */
    const double dD = 2.0 * (k1 + 2.0 * k2 * s);
    const double A[4] = {f * (D + dD * u * u), f * dD * u * v,
                         f * dD * u * v,       f * (D + dD * v * v)};
    /* d(u,v) / dY */
    const double iz = -1.0 / Y[2];
    const double B[6] = {iz, 0.0, iz * (-Y[0] / Y[2]),
                         0.0, iz, iz * (-Y[1] / Y[2])};
    double AB[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            AB[i * 3 + j] = A[i * 2] * B[j] + A[i * 2 + 1] * B[3 + j];
    if (Jp) {
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j)
                Jp[i * 3 + j] = AB[i * 3] * R[j] + AB[i * 3 + 1] * R[3 + j] + AB[i * 3 + 2] * R[6 + j];
    }
    if (Jc) {
        /* dY/d(rho, phi) = [ I | -[Y]x ] */
        const double negYx[9] = {0.0, Y[2], -Y[1],
                                 -Y[2], 0.0, Y[0],
                                 Y[1], -Y[0], 0.0};
        for (int i = 0; i < 2; ++i) {
            for (int j = 0; j < 3; ++j) Jc[i * d + j] = AB[i * 3 + j];
            for (int j = 0; j < 3; ++j)
                Jc[i * d + 3 + j] = AB[i * 3] * negYx[j] + AB[i * 3 + 1] * negYx[3 + j] +
                                    AB[i * 3 + 2] * negYx[6 + j];
        }
        if (d == 9) {
            const double uv[2] = {u, v};
            for (int i = 0; i < 2; ++i) {
                Jc[i * d + 6] = D * uv[i];
                Jc[i * d + 7] = f * s * uv[i];
                Jc[i * d + 8] = f * s * s * uv[i];
            }
        }
    }
    return Y[2];
}

/* T <- Exp(delta) T with delta = (rho, phi), then f, k1, k2 additive (d = 9). */
void orc_retract_camera(const double *cam, const double *delta, int32_t d, double *out)
{
    const double *rho = delta, *phi = delta + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    double a, b, c, hs, hc; /* sin(th)/th, (1-cos)/th^2, (th-sin)/th^3, sin(th/2)/th, cos(th/2) */
    if (th < 1e-5) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
        c = 1.0 / 6.0 - th2 / 120.0;
        hs = 0.5 - th2 / 48.0;
        hc = 1.0 - th2 / 8.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
        c = (th - sin(th)) / (th2 * th);
        hs = sin(0.5 * th) / th;
        hc = cos(0.5 * th);
    }
    const double K[9] = {0.0, -phi[2], phi[1],
                         phi[2], 0.0, -phi[0],
                         -phi[1], phi[0], 0.0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[i * 3 + j] = K[i * 3] * K[j] + K[i * 3 + 1] * K[3 + j] + K[i * 3 + 2] * K[6 + j];
    double Rp[9], Vm[9];
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        Rp[i] = I + a * K[i] + b * K2[i];
        Vm[i] = I + b * K[i] + c * K2[i];
    }
    const double *t = cam;
    for (int i = 0; i < 3; ++i)
        out[i] = Rp[3 * i] * t[0] + Rp[3 * i + 1] * t[1] + Rp[3 * i + 2] * t[2] +
                 Vm[3 * i] * rho[0] + Vm[3 * i + 1] * rho[1] + Vm[3 * i + 2] * rho[2];
    /* q' = q_phi (x) q, Hamilton product, scalar last */
    const double p[4] = {hs * phi[0], hs * phi[1], hs * phi[2], hc};
    const double *q = cam + 3;
    double qn[4];
    qn[0] = p[3] * q[0] + p[0] * q[3] + p[1] * q[2] - p[2] * q[1];
    qn[1] = p[3] * q[1] - p[0] * q[2] + p[1] * q[3] + p[2] * q[0];
    qn[2] = p[3] * q[2] + p[0] * q[1] - p[1] * q[0] + p[2] * q[3];
    qn[3] = p[3] * q[3] - p[0] * q[0] - p[1] * q[1] - p[2] * q[2];
    const double nq = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int i = 0; i < 4; ++i) out[3 + i] = qn[i] / nq;
    for (int i = 7; i < 10; ++i) out[i] = cam[i] + (d == 9 ? delta[6 + (i - 7)] : 0.0);
}

/* Huber on the squared norm s: rho(s), and rho'(s). */
static void robust(double s, double delta, double *rho, double *drho)
{
    if (delta <= 0.0 || s <= delta * delta) {
        *rho = s;
        *drho = 1.0;
    } else {
        const double rs = sqrt(s);
        *rho = 2.0 * delta * rs - delta * delta;
        *drho = delta / rs;
    }
}

/* ------------------------------------------------------------------------ */
/* context                                                                   */
/* ------------------------------------------------------------------------ */

static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

static void bucket(int64_t n, int32_t nkeys, const int32_t *key, int64_t **ptr_out,
                   int64_t **lst_out)
{
    int64_t *ptr = xcalloc((size_t)nkeys + 1, sizeof(int64_t));
    int64_t *lst = xcalloc((size_t)n, sizeof(int64_t));
    for (int64_t k = 0; k < n; ++k) ptr[key[k] + 1]++;
    for (int32_t i = 0; i < nkeys; ++i) ptr[i + 1] += ptr[i];
    int64_t *fill = xcalloc((size_t)nkeys, sizeof(int64_t));
    for (int64_t k = 0; k < n; ++k) lst[ptr[key[k]] + fill[key[k]]++] = k;
    free(fill);
    *ptr_out = ptr;
    *lst_out = lst;
}

static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* upper-triangular block pattern of the reduced camera system: (a, b), a <= b,
 * whenever a point is seen by both cameras; every diagonal block is present. */
static void build_pattern(orc_ctx *c)
{
    int32_t *cnt = xcalloc((size_t)c->nc, sizeof(int32_t));
    int32_t **cols = xcalloc((size_t)c->nc, sizeof(int32_t *));
    int32_t *cap = xcalloc((size_t)c->nc, sizeof(int32_t));
    for (int32_t a = 0; a < c->nc; ++a) {
        cap[a] = 8;
        cols[a] = malloc(sizeof(int32_t) * 8);
        cols[a][cnt[a]++] = a;
    }
    for (int32_t j = 0; j < c->np; ++j) {
        for (int64_t x = c->pt_ptr[j]; x < c->pt_ptr[j + 1]; ++x) {
            const int32_t a = c->cidx[c->pt_obs[x]];
            for (int64_t y = c->pt_ptr[j]; y < c->pt_ptr[j + 1]; ++y) {
                const int32_t b = c->cidx[c->pt_obs[y]];
                if (b <= a) continue;
                if (cnt[a] == cap[a]) {
                    cap[a] *= 2;
                    cols[a] = realloc(cols[a], sizeof(int32_t) * cap[a]);
                }
                cols[a][cnt[a]++] = b;
            }
        }
    }
    c->S_ptr = xcalloc((size_t)c->nc + 1, sizeof(int64_t));
    for (int32_t a = 0; a < c->nc; ++a) {
        qsort(cols[a], cnt[a], sizeof(int32_t), cmp_i32);
        int32_t u = 0;
        for (int32_t i = 0; i < cnt[a]; ++i)
            if (u == 0 || cols[a][i] != cols[a][u - 1]) cols[a][u++] = cols[a][i];
        cnt[a] = u;
        c->S_ptr[a + 1] = c->S_ptr[a] + u;
    }
    c->nnzb = c->S_ptr[c->nc];
    c->S_col = xcalloc((size_t)c->nnzb, sizeof(int32_t));
    for (int32_t a = 0; a < c->nc; ++a) {
        memcpy(c->S_col + c->S_ptr[a], cols[a], sizeof(int32_t) * cnt[a]);
        free(cols[a]);
    }
    free(cols);
    free(cnt);
    free(cap);
    /* column lists of the off-diagonal upper blocks, rows ascending */
    c->T_ptr = xcalloc((size_t)c->nc + 1, sizeof(int64_t));
    for (int32_t a = 0; a < c->nc; ++a)
        for (int64_t e = c->S_ptr[a] + 1; e < c->S_ptr[a + 1]; ++e) c->T_ptr[c->S_col[e] + 1]++;
    for (int32_t b = 0; b < c->nc; ++b) c->T_ptr[b + 1] += c->T_ptr[b];
    c->T_blk = xcalloc((size_t)c->T_ptr[c->nc], sizeof(int64_t));
    c->T_row = xcalloc((size_t)c->T_ptr[c->nc], sizeof(int32_t));
    int64_t *fill = xcalloc((size_t)c->nc, sizeof(int64_t));
    for (int32_t a = 0; a < c->nc; ++a)
        for (int64_t e = c->S_ptr[a] + 1; e < c->S_ptr[a + 1]; ++e) {
            const int32_t b = c->S_col[e];
            c->T_blk[c->T_ptr[b] + fill[b]] = e;
            c->T_row[c->T_ptr[b] + fill[b]++] = a;
        }
    free(fill);
    /* per camera, its observations by (point, input order) */
    c->cam_obs_pt = xcalloc((size_t)c->no, sizeof(int64_t));
    fill = xcalloc((size_t)c->nc, sizeof(int64_t));
    for (int32_t j = 0; j < c->np; ++j)
        for (int64_t x = c->pt_ptr[j]; x < c->pt_ptr[j + 1]; ++x) {
            const int64_t k = c->pt_obs[x];
            const int32_t a = c->cidx[k];
            c->cam_obs_pt[c->cam_ptr[a] + fill[a]++] = k;
        }
    free(fill);
}

static int64_t find_block(const orc_ctx *c, int32_t a, int32_t b)
{
    int64_t lo = c->S_ptr[a], hi = c->S_ptr[a + 1] - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) / 2;
        if (c->S_col[mid] == b) return mid;
        if (c->S_col[mid] < b) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

orc_ctx *orc_create(const orc_options *o, int32_t nc, int32_t np, int64_t no,
                    const int32_t *cidx, const int32_t *pidx, const double *obs,
                    const double *ow, const uint8_t *fixed)
{
    orc_ctx *c = xcalloc(1, sizeof(orc_ctx));
    c->o = *o;
    c->nc = nc;
    c->np = np;
    c->no = no;
    const int d = o->d;
    c->cidx = xcalloc((size_t)no, sizeof(int32_t));
    c->pidx = xcalloc((size_t)no, sizeof(int32_t));
    c->obs = xcalloc((size_t)no * 2, sizeof(double));
    c->ow = xcalloc((size_t)no, sizeof(double));
    c->fixed = xcalloc((size_t)nc, 1);
    memcpy(c->cidx, cidx, sizeof(int32_t) * no);
    memcpy(c->pidx, pidx, sizeof(int32_t) * no);
    memcpy(c->obs, obs, sizeof(double) * 2 * no);
    for (int64_t k = 0; k < no; ++k) c->ow[k] = ow ? ow[k] : 1.0;
    if (fixed) memcpy(c->fixed, fixed, nc);
    c->cams = xcalloc((size_t)nc * 10, sizeof(double));
    c->pts = xcalloc((size_t)np * 3, sizeof(double));
    c->cams_new = xcalloc((size_t)nc * 10, sizeof(double));
    c->pts_new = xcalloc((size_t)np * 3, sizeof(double));
    c->lambda = o->lambda0;
    bucket(no, np, pidx, &c->pt_ptr, &c->pt_obs);
    bucket(no, nc, cidx, &c->cam_ptr, &c->cam_obs);
    c->r = xcalloc((size_t)no * 2, sizeof(double));
    c->w = xcalloc((size_t)no, sizeof(double));
    c->Jc = xcalloc((size_t)no * 2 * d, sizeof(double));
    c->Jp = xcalloc((size_t)no * 6, sizeof(double));
    c->U = xcalloc((size_t)nc * d * d, sizeof(double));
    c->V = xcalloc((size_t)np * 9, sizeof(double));
    c->gc = xcalloc((size_t)nc * d, sizeof(double));
    c->gp = xcalloc((size_t)np * 3, sizeof(double));
    c->Vinv = xcalloc((size_t)np * 9, sizeof(double));
    c->term = xcalloc((size_t)no, sizeof(double));
    build_pattern(c);
    c->S = xcalloc((size_t)c->nnzb * d * d, sizeof(double));
    c->bS = xcalloc((size_t)nc * d, sizeof(double));
    c->dc = xcalloc((size_t)nc * d, sizeof(double));
    c->dp = xcalloc((size_t)np * 3, sizeof(double));
    return c;
}

void orc_destroy(orc_ctx *c)
{
    if (!c) return;
    void *p[] = {c->cidx, c->pidx, c->obs, c->ow, c->fixed, c->cams, c->pts, c->pt_ptr,
                 c->pt_obs, c->cam_ptr, c->cam_obs, c->r, c->w, c->Jc, c->Jp, c->U, c->V,
                 c->gc, c->gp, c->S_ptr, c->S_col, c->S, c->bS, c->Vinv, c->dc, c->dp,
                 c->cams_new, c->pts_new, c->cam_obs_pt, c->T_ptr, c->T_blk, c->T_row,
                 c->term};
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) free(p[i]);
    free(c);
}

void orc_set_params(orc_ctx *c, const double *cams, const double *pts)
{
    memcpy(c->cams, cams, sizeof(double) * 10 * c->nc);
    memcpy(c->pts, pts, sizeof(double) * 3 * c->np);
    c->have_lin = 0;
}

void orc_get_params(const orc_ctx *c, double *cams, double *pts)
{
    memcpy(cams, c->cams, sizeof(double) * 10 * c->nc);
    memcpy(pts, c->pts, sizeof(double) * 3 * c->np);
}

void orc_set_lambda(orc_ctx *c, double lambda) { c->lambda = lambda; }
double orc_get_lambda(const orc_ctx *c) { return c->lambda; }
int64_t orc_nnzb(const orc_ctx *c) { return c->nnzb; }

/* ------------------------------------------------------------------------ */
/* objective and linearisation                                               */
/* ------------------------------------------------------------------------ */

/* F = 1/2 sum_k omega_k rho(|r_k|^2) at the given parameters (Eq. 1). */
double orc_cost(const orc_ctx *c, const double *cams, const double *pts)
{
    double *term = c->term;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < c->no; ++k) {
        double pix[2];
        orc_project(cams + 10 * (int64_t)c->cidx[k], pts + 3 * (int64_t)c->pidx[k], c->o.d, pix,
                    NULL, NULL);
        const double rx = pix[0] - c->obs[2 * k], ry = pix[1] - c->obs[2 * k + 1];
        double rho, drho;
        robust(rx * rx + ry * ry, c->o.huber_delta, &rho, &drho);
        term[k] = 0.5 * c->ow[k] * rho;
    }
    double F = 0.0;
    for (int64_t k = 0; k < c->no; ++k) F += term[k];
    return F;
}

/* Alg. 1, first two lines: J at theta, then the blocks of A = J^T W J and the
 * gradient g = J^T W r (W: Gauss-Newton weights of the robust loss). */
static void linearize(orc_ctx *c)
{
    const int d = c->o.d;
    double *term = c->term;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < c->no; ++k) {
        double pix[2];
        double *Jc = c->Jc + (size_t)k * 2 * d, *Jp = c->Jp + (size_t)k * 6;
        orc_project(c->cams + 10 * (int64_t)c->cidx[k], c->pts + 3 * (int64_t)c->pidx[k], d, pix,
                    Jc, Jp);
        if (c->fixed[c->cidx[k]]) memset(Jc, 0, sizeof(double) * 2 * d);
        c->r[2 * k] = pix[0] - c->obs[2 * k];
        c->r[2 * k + 1] = pix[1] - c->obs[2 * k + 1];
        double rho, drho;
        robust(c->r[2 * k] * c->r[2 * k] + c->r[2 * k + 1] * c->r[2 * k + 1], c->o.huber_delta,
               &rho, &drho);
        term[k] = 0.5 * c->ow[k] * rho;
        c->w[k] = c->ow[k] * drho;
    }
    double F = 0.0;
    for (int64_t k = 0; k < c->no; ++k) F += term[k];
    c->F = F;
    /* camera blocks U_a and gradients g_a: sums over the camera's
     * observations in input order */
#pragma omp parallel for schedule(dynamic, 8)
    for (int32_t a = 0; a < c->nc; ++a) {
        double *U = c->U + (size_t)a * d * d, *gc = c->gc + (size_t)a * d;
        memset(U, 0, sizeof(double) * d * d);
        memset(gc, 0, sizeof(double) * d);
        for (int64_t x = c->cam_ptr[a]; x < c->cam_ptr[a + 1]; ++x) {
            const int64_t k = c->cam_obs[x];
            const double *Jc = c->Jc + (size_t)k * 2 * d;
            const double *r = c->r + 2 * k, w = c->w[k];
            for (int i = 0; i < d; ++i) {
                for (int j = 0; j < d; ++j) U[i * d + j] += w * (Jc[i] * Jc[j] + Jc[d + i] * Jc[d + j]);
                gc[i] += w * (Jc[i] * r[0] + Jc[d + i] * r[1]);
            }
        }
    }
    /* point blocks V_j and gradients g_j: sums over the point's track in
     * input order */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < c->np; ++j) {
        double *V = c->V + (size_t)j * 9, *gp = c->gp + (size_t)j * 3;
        memset(V, 0, sizeof(double) * 9);
        memset(gp, 0, sizeof(double) * 3);
        for (int64_t x = c->pt_ptr[j]; x < c->pt_ptr[j + 1]; ++x) {
            const int64_t k = c->pt_obs[x];
            const double *Jp = c->Jp + (size_t)k * 6;
            const double *r = c->r + 2 * k, w = c->w[k];
            for (int i = 0; i < 3; ++i) {
                for (int m = 0; m < 3; ++m) V[i * 3 + m] += w * (Jp[i] * Jp[m] + Jp[3 + i] * Jp[3 + m]);
                gp[i] += w * (Jp[i] * r[0] + Jp[3 + i] * r[1]);
            }
        }
    }
    c->have_lin = 1;
}

/* W_k = w_k Jc_k^T Jp_k  (d x 3) */
static void block_W(const orc_ctx *c, int64_t k, double *W)
{
    const int d = c->o.d;
    const double *Jc = c->Jc + (size_t)k * 2 * d, *Jp = c->Jp + (size_t)k * 6;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < 3; ++j) W[i * 3 + j] = c->w[k] * (Jc[i] * Jp[j] + Jc[d + i] * Jp[3 + j]);
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* ------------------------------------------------------------------------ */
/* damped system, Schur complement, PCG, back-substitution                  */
/* ------------------------------------------------------------------------ */

/* S = blockdiag(U*) - sum_j W_j V*_j^{-1} W_j^T,  b_S = -g_c + sum_j W_j V*_j^{-1} g_p,j
 *
 * Each row a of S (and b_S[a]) is built by one thread, visiting the
 * camera's observations by (point, input order) and each observed point's
 * track in input order: the order in which a loop over the points,
 * ascending, reaches the blocks of row a. */
static int schur(orc_ctx *c, double lambda)
{
    const int d = c->o.d, dd = d * d;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int32_t j = 0; j < c->np; ++j) {
        double Vs[9];
        memcpy(Vs, c->V + (size_t)j * 9, sizeof Vs);
        for (int i = 0; i < 3; ++i)
            Vs[i * 4] += lambda * clampd(Vs[i * 4], c->o.diag_min, c->o.diag_max);
        const double det = inverse3(Vs, c->Vinv + (size_t)j * 9);
        if (!(det > 0) || !isfinite(det)) bad = 1;
    }
    if (bad) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t a = 0; a < c->nc; ++a) {
        memset(c->S + (size_t)c->S_ptr[a] * dd, 0, sizeof(double) * (c->S_ptr[a + 1] - c->S_ptr[a]) * dd);
        double *Saa = c->S + (size_t)c->S_ptr[a] * dd; /* the diagonal is a row's first block */
        const double *U = c->U + (size_t)a * dd;
        for (int i = 0; i < dd; ++i) Saa[i] = U[i];
        for (int i = 0; i < d; ++i)
            Saa[i * d + i] += lambda * clampd(U[i * d + i], c->o.diag_min, c->o.diag_max);
        for (int i = 0; i < d; ++i) c->bS[a * d + i] = -c->gc[a * d + i];
        double W[16 * 3], W2[16 * 3], Y[16 * 3];
        for (int64_t q = c->cam_ptr[a]; q < c->cam_ptr[a + 1]; ++q) {
            const int64_t k = c->cam_obs_pt[q];
            const int32_t j = c->pidx[k];
            const double *Vi = c->Vinv + (size_t)j * 9;
            const double *gp = c->gp + (size_t)j * 3;
            block_W(c, k, W);
            /* Y = W V*^{-1} */
            for (int i = 0; i < d; ++i)
                for (int m = 0; m < 3; ++m)
                    Y[i * 3 + m] = W[i * 3] * Vi[m] + W[i * 3 + 1] * Vi[3 + m] + W[i * 3 + 2] * Vi[6 + m];
            for (int i = 0; i < d; ++i)
                c->bS[a * d + i] += Y[i * 3] * gp[0] + Y[i * 3 + 1] * gp[1] + Y[i * 3 + 2] * gp[2];
            for (int64_t y = c->pt_ptr[j]; y < c->pt_ptr[j + 1]; ++y) {
                const int64_t k2 = c->pt_obs[y];
                const int32_t b = c->cidx[k2];
                if (b < a) continue; /* only the upper block triangle is stored */
                block_W(c, k2, W2);
                double *Sab = c->S + (size_t)find_block(c, a, b) * dd;
                for (int i = 0; i < d; ++i)
                    for (int m = 0; m < d; ++m)
                        Sab[i * d + m] -= Y[i * 3] * W2[m * 3] + Y[i * 3 + 1] * W2[m * 3 + 1] +
                                          Y[i * 3 + 2] * W2[m * 3 + 2];
            }
        }
    }
    return 0;
}

/* y = S x using the stored upper block triangle and its transpose.  Output
 * block a is summed by one thread: first S_ra^T x_r for the blocks (r, a),
 * r < a, ascending r, then S_ab x_b along row a -- the order in which a loop
 * over the rows, ascending, reaches y_a. */
static void spmv(const orc_ctx *c, const double *x, double *y)
{
    const int d = c->o.d, dd = d * d;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t a = 0; a < c->nc; ++a) {
        double *ya = y + (size_t)a * d;
        memset(ya, 0, sizeof(double) * d);
        for (int64_t t = c->T_ptr[a]; t < c->T_ptr[a + 1]; ++t) {
            const double *B = c->S + (size_t)c->T_blk[t] * dd;
            const double *xr = x + (size_t)c->T_row[t] * d;
            for (int i = 0; i < d; ++i)
                for (int m = 0; m < d; ++m) ya[m] += B[i * d + m] * xr[i];
        }
        for (int64_t e = c->S_ptr[a]; e < c->S_ptr[a + 1]; ++e) {
            const int32_t b = c->S_col[e];
            const double *B = c->S + (size_t)e * dd;
            for (int i = 0; i < d; ++i)
                for (int m = 0; m < d; ++m) ya[i] += B[i * d + m] * x[b * d + m];
        }
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Preconditioned conjugate gradients on S x = b_S with M = blockdiag(S_aa). */
static int pcg(orc_ctx *c, double rtol, int32_t maxiter, orc_step_info *info)
{
    const int d = c->o.d, dd = d * d;
    const int64_t n = (int64_t)c->nc * d;
    double *L = malloc(sizeof(double) * c->nc * dd);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int32_t a = 0; a < c->nc; ++a)
        if (cholesky(d, c->S + (size_t)c->S_ptr[a] * dd, L + (size_t)a * dd)) bad = 1;
    if (bad) {
        free(L);
        return -1;
    }
    double *x = c->dc, *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    memset(x, 0, sizeof(double) * n);
    memcpy(r, c->bS, sizeof(double) * n);
    const double bnorm = sqrt(dot(n, c->bS, c->bS));
    int32_t it = 0, breakdown = 0;
    double rnorm = bnorm;
    if (bnorm > 0) {
#pragma omp parallel for schedule(static)
        for (int32_t a = 0; a < c->nc; ++a) cholesky_solve(d, L + (size_t)a * dd, r + a * d, z + a * d);
        memcpy(p, z, sizeof(double) * n);
        double rz = dot(n, r, z);
        for (int32_t k = 1; k <= maxiter; ++k) {
            spmv(c, p, q);
            const double pq = dot(n, p, q);
            if (!(pq > 0)) {
                breakdown = 1;
                break;
            }
            const double alpha = rz / pq;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            it = k;
            rnorm = sqrt(dot(n, r, r));
            if (rnorm <= rtol * bnorm) break;
#pragma omp parallel for schedule(static)
            for (int32_t a = 0; a < c->nc; ++a)
                cholesky_solve(d, L + (size_t)a * dd, r + a * d, z + a * d);
            const double rz_new = dot(n, r, z);
            const double beta = rz_new / rz;
            rz = rz_new;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
    }
    info->cg_iters = it;
    info->cg_breakdown = breakdown;
    info->cg_rel_resid = bnorm > 0 ? rnorm / bnorm : 0.0;
    free(L);
    free(r);
    free(z);
    free(p);
    free(q);
    return 0;
}

/* dp_j = V*_j^{-1} (-g_p,j - sum_k W_k^T dc_{c_k}) */
static void back_substitute(orc_ctx *c)
{
    const int d = c->o.d;
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < c->np; ++j) {
        double W[16 * 3];
        double t[3] = {-c->gp[j * 3], -c->gp[j * 3 + 1], -c->gp[j * 3 + 2]};
        for (int64_t x = c->pt_ptr[j]; x < c->pt_ptr[j + 1]; ++x) {
            const int64_t k = c->pt_obs[x];
            block_W(c, k, W);
            const double *dc = c->dc + (size_t)c->cidx[k] * d;
            for (int m = 0; m < 3; ++m)
                for (int i = 0; i < d; ++i) t[m] -= W[i * 3 + m] * dc[i];
        }
        const double *Vi = c->Vinv + (size_t)j * 9;
        for (int m = 0; m < 3; ++m)
            c->dp[j * 3 + m] = Vi[m * 3] * t[0] + Vi[m * 3 + 1] * t[1] + Vi[m * 3 + 2] * t[2];
    }
}

/* pred = F - m(delta) for the Gauss-Newton model m(delta) = F + g^T delta + 1/2 |J delta|_W^2 */
static double predicted_reduction(orc_ctx *c)
{
    const int d = c->o.d;
    double lin = dot((int64_t)c->nc * d, c->gc, c->dc) + dot((int64_t)c->np * 3, c->gp, c->dp);
    double *term = c->term;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < c->no; ++k) {
        const double *Jc = c->Jc + (size_t)k * 2 * d, *Jp = c->Jp + (size_t)k * 6;
        const double *dc = c->dc + (size_t)c->cidx[k] * d, *dp = c->dp + (size_t)c->pidx[k] * 3;
        double e[2];
        for (int i = 0; i < 2; ++i) {
            e[i] = 0.0;
            for (int m = 0; m < d; ++m) e[i] += Jc[i * d + m] * dc[m];
            for (int m = 0; m < 3; ++m) e[i] += Jp[i * 3 + m] * dp[m];
        }
        term[k] = c->w[k] * (e[0] * e[0] + e[1] * e[1]);
    }
    double quad = 0.0;
    for (int64_t k = 0; k < c->no; ++k) quad += term[k];
    return -lin - 0.5 * quad;
}

static double grad_inf(const orc_ctx *c)
{
    double g = 0.0;
    for (int64_t i = 0; i < (int64_t)c->nc * c->o.d; ++i) g = fmax(g, fabs(c->gc[i]));
    for (int64_t i = 0; i < (int64_t)c->np * 3; ++i) g = fmax(g, fabs(c->gp[i]));
    return g;
}

static int dense_spd_solve(int n, const double *A, const double *b, double *x);

/* The reduced camera system solved by factorisation instead of PCG (the
 * paper's Cholesky alternative, Sec. IV-C-1): S assembled dense from its
 * upper blocks and their transposes, S = L L^T, then L y = b_S and
 * L^T dc = y.  Reports |b_S - S dc| / |b_S| as the relative residual. */
static int dense_step(orc_ctx *c, orc_step_info *info)
{
    const int d = c->o.d, dd = d * d;
    const int64_t n = (int64_t)c->nc * d;
    double *A = xcalloc((size_t)(n * n), sizeof(double));
    for (int32_t a = 0; a < c->nc; ++a)
        for (int64_t e = c->S_ptr[a]; e < c->S_ptr[a + 1]; ++e) {
            const int32_t b = c->S_col[e];
            const double *B = c->S + (size_t)e * dd;
            for (int i = 0; i < d; ++i)
                for (int m = 0; m < d; ++m) {
                    A[(size_t)(a * d + i) * n + b * d + m] = B[i * d + m];
                    A[(size_t)(b * d + m) * n + a * d + i] = B[i * d + m];
                }
        }
    const int st = dense_spd_solve((int)n, A, c->bS, c->dc);
    double rr = 0.0, bb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = c->bS[i];
        for (int64_t q = 0; q < n; ++q) s -= A[(size_t)(i * n + q)] * c->dc[q];
        rr += s * s;
        bb += c->bS[i] * c->bS[i];
    }
    info->cg_iters = 0;
    info->cg_breakdown = 0;
    info->cg_rel_resid = bb > 0 ? sqrt(rr / bb) : 0.0;
    free(A);
    return st;
}

/* The step of one LM iteration at the current lambda, without accepting it:
 * linearise (if needed), damp, reduce onto the cameras, PCG, back-substitute,
 * predicted reduction.  rtol < 0 / maxiter < 0 take the options' values. */
int orc_compute_step(orc_ctx *c, double rtol, int32_t maxiter, orc_step_info *info)
{
    memset(info, 0, sizeof *info);
    if (!c->have_lin) linearize(c);
    info->cost_before = c->F;
    info->lambda_used = c->lambda;
    info->grad_inf = grad_inf(c);
    if (!isfinite(c->F)) return info->status = -2;
    if (schur(c, c->lambda)) return info->status = -2;
    if (c->o.solver == 1) {
        if (dense_step(c, info)) return info->status = -2;
    } else if (pcg(c, rtol < 0 ? c->o.cg_rtol : rtol, maxiter < 0 ? c->o.cg_maxiter : maxiter, info)) {
        return info->status = -2;
    }
    back_substitute(c);
    info->pred = predicted_reduction(c);
    return 0;
}

/* Trust-region update of the damping (Sec. V: TrustRegion(up=2, down=0.5**4)
 * acting on the trust radius 1/lambda): a step whose actual reduction is
 * more than 3/4 of the predicted one doubles the radius (lambda / 2, not
 * below lambda_min); a rejected step, or a ratio of at most 1/4, shrinks it
 * sixteen-fold (16 lambda, not above lambda_max); in between lambda stays.
 * The 1/4 and 3/4 thresholds are this oracle's reading (the paper gives
 * only the factors). */
double orc_lambda_update(int accepted, double ratio, double lambda, double lambda_min,
                         double lambda_max)
{
    if (!accepted || !(ratio > 0.25)) return fmin(16.0 * lambda, lambda_max);
    if (ratio > 0.75) return fmax(0.5 * lambda, lambda_min);
    return lambda;
}

/* One LM iteration (Alg. 1): step, candidate theta' = theta (+) delta, its
 * cost, acceptance and the trust-region update of lambda. */
int orc_lm_step(orc_ctx *c, double rtol, int32_t maxiter, orc_step_info *info)
{
    int st = orc_compute_step(c, rtol, maxiter, info);
    if (st) return st;
    const int d = c->o.d;
#pragma omp parallel for schedule(static)
    for (int32_t a = 0; a < c->nc; ++a) {
        if (c->fixed[a]) memcpy(c->cams_new + 10 * a, c->cams + 10 * a, sizeof(double) * 10);
        else orc_retract_camera(c->cams + 10 * a, c->dc + (size_t)a * d, d, c->cams_new + 10 * a);
    }
    for (int64_t i = 0; i < (int64_t)c->np * 3; ++i) c->pts_new[i] = c->pts[i] + c->dp[i];
    const double Fn = orc_cost(c, c->cams_new, c->pts_new);
    info->cost_after = Fn;
    const double ratio = (c->F - Fn) / info->pred;
    const int accept = isfinite(Fn) && Fn < c->F && info->pred > 0;
    info->accepted = accept;
    c->lambda = orc_lambda_update(accept, ratio, c->lambda, c->o.lambda_min, c->o.lambda_max);
    info->lambda_next = c->lambda;
    if (accept) {
        double *t = c->cams;
        c->cams = c->cams_new;
        c->cams_new = t;
        t = c->pts;
        c->pts = c->pts_new;
        c->pts_new = t;
        c->have_lin = 0;
    }
    return 0;
}

/* Repeated LM iterations with the stopping rules of Sec. V (StopOnPlateau):
 * after each iteration, in this order,
 *   - a rejected step whose damping was lambda_max already: stop, -4 ("not
 *     converged", reason 4);
 *   - plateau_steps consecutive iterations whose relative decrease
 *     (F - F') / F is below rel_tol (a rejected step decreases by 0): stop,
 *     reason 2;
 *   - |g|_inf <= 1e-12 (1 + F) at the iteration's linearisation point: stop,
 *     reason 3;
 *   - max_iters iterations: stop, reason 1.
 * infos (max_iters entries, may be NULL) receive each iteration's report;
 * *done the number of iterations run, *reason the rule that stopped. */
int orc_solve(orc_ctx *c, int32_t max_iters, double rel_tol, int32_t plateau_steps, double rtol,
              int32_t maxiter, orc_step_info *infos, int32_t *done, int32_t *reason)
{
    int32_t n = 0, flat = 0, why = 0;
    int ret = 0;
    for (int32_t it = 0; it < max_iters && why == 0; ++it) {
        orc_step_info info;
        const int st = orc_lm_step(c, rtol, maxiter, &info);
        if (infos) infos[it] = info;
        if (st) {
            ret = st;
            why = 5;
            break;
        }
        ++n;
        const double dec = info.accepted ? (info.cost_before - info.cost_after) / info.cost_before : 0.0;
        flat = dec < rel_tol ? flat + 1 : 0;
        if (!info.accepted && info.lambda_used >= c->o.lambda_max) {
            ret = -4;
            why = 4;
        } else if (flat >= plateau_steps) {
            why = 2;
        } else if (info.grad_inf <= 1e-12 * (1.0 + info.cost_before)) {
            why = 3;
        } else if (it + 1 == max_iters) {
            why = 1;
        }
    }
    if (done) *done = n;
    if (reason) *reason = why;
    return ret;
}

/* Number of threads of the parallel loops (n >= 1). */
void orc_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
int32_t orc_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* read-back of intermediate quantities (for parity tests)                   */
/* ------------------------------------------------------------------------ */

void orc_get_linearization(orc_ctx *c, double *r, double *w, double *Jc, double *Jp, double *F)
{
    if (!c->have_lin) linearize(c);
    const int d = c->o.d;
    if (r) memcpy(r, c->r, sizeof(double) * 2 * c->no);
    if (w) memcpy(w, c->w, sizeof(double) * c->no);
    if (Jc) memcpy(Jc, c->Jc, sizeof(double) * 2 * d * c->no);
    if (Jp) memcpy(Jp, c->Jp, sizeof(double) * 6 * c->no);
    if (F) *F = c->F;
}

void orc_get_normal(orc_ctx *c, double *U, double *V, double *gc, double *gp)
{
    if (!c->have_lin) linearize(c);
    const int d = c->o.d;
    if (U) memcpy(U, c->U, sizeof(double) * d * d * c->nc);
    if (V) memcpy(V, c->V, sizeof(double) * 9 * c->np);
    if (gc) memcpy(gc, c->gc, sizeof(double) * d * c->nc);
    if (gp) memcpy(gp, c->gp, sizeof(double) * 3 * c->np);
}

void orc_get_schur(const orc_ctx *c, int64_t *S_ptr, int32_t *S_col, double *S, double *bS)
{
    const int d = c->o.d;
    if (S_ptr) memcpy(S_ptr, c->S_ptr, sizeof(int64_t) * (c->nc + 1));
    if (S_col) memcpy(S_col, c->S_col, sizeof(int32_t) * c->nnzb);
    if (S) memcpy(S, c->S, sizeof(double) * d * d * c->nnzb);
    if (bS) memcpy(bS, c->bS, sizeof(double) * d * c->nc);
}

void orc_get_step(const orc_ctx *c, double *dc, double *dp, double *Vinv)
{
    if (dc) memcpy(dc, c->dc, sizeof(double) * c->o.d * c->nc);
    if (dp) memcpy(dp, c->dp, sizeof(double) * 3 * c->np);
    if (Vinv) memcpy(Vinv, c->Vinv, sizeof(double) * 9 * c->np);
}

/* ------------------------------------------------------------------------ */
/* implicit-function adjoint at a stationary point                           */
/*                                                                            */
/* The paper uses the solver inside learning pipelines, where a loss on the   */
/* optimum theta* is differentiated with respect to the observations          */
/* (Sec. VI-D and App. A: bilevel use).  At theta* the tangent gradient      */
/* G(theta, x, omega) = sum_k omega_k J_k^T r_k vanishes; the implicit        */
/* function theorem gives d theta* / d x_k = H^-1 omega_k J_k^T and          */
/* d theta* / d omega_k = -H^-1 J_k^T r_k, with H the exact Hessian of        */
/* delta -> F(Retract(theta*, delta)) at delta = 0:                           */
/*   H = sum_k omega_k (J_k^T J_k + sum_m r_km Hess(pi_km)).                  */
/* With v = H^-1 dL/dtheta:                                                   */
/*   dL/dx_k = omega_k J_k v,   dL/domega_k = -r_k . (J_k v).                 */
/* Squared loss only.  Fixed cameras are constrained: their tangent is zero.  */
/* The linear system is solved exactly: points eliminated block by block,     */
/* the reduced camera system by a dense Cholesky factorisation.               */
/* ------------------------------------------------------------------------ */

/* hyper-dual numbers a + b e1 + c e2 + d e1 e2 with e1^2 = e2^2 = 0: for
 * f(x + e1 u + e2 w) the e1 part is f'(x) u and the e1 e2 part u^T f''(x) w. */
typedef struct { double a, b, c, d; } hd;

static hd hd_k(double a) { hd r = {a, 0.0, 0.0, 0.0}; return r; }
static hd hd_add(hd x, hd y) { hd r = {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; return r; }
static hd hd_sub(hd x, hd y) { hd r = {x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d}; return r; }
static hd hd_scale(double s, hd x) { hd r = {s * x.a, s * x.b, s * x.c, s * x.d}; return r; }
static hd hd_mul(hd x, hd y)
{
    hd r = {x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a,
            x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a};
    return r;
}
static hd hd_div(hd x, hd y)
{
    /* 1/y = 1/a - b/a^2 e1 - c/a^2 e2 + (2bc/a^3 - d/a^2) e1 e2 */
    const double i = 1.0 / y.a;
    const hd inv = {i, -y.b * i * i, -y.c * i * i, (2.0 * y.b * y.c * i - y.d) * i * i};
    return hd_mul(x, inv);
}
static void hd_cross(const hd a[3], const hd b[3], hd out[3])
{
    out[0] = hd_sub(hd_mul(a[1], b[2]), hd_mul(a[2], b[1]));
    out[1] = hd_sub(hd_mul(a[2], b[0]), hd_mul(a[0], b[2]));
    out[2] = hd_sub(hd_mul(a[0], b[1]), hd_mul(a[1], b[0]));
}

/* Pixel of the point X + dX seen by the camera retracted along the tangent
 * dt = [rho, phi, (df, dk1, dk2), dX] (hyper-dual, zero value part).  The
 * SE(3) exponential acting on a point is I + xi^ + xi^2/2 here: every product
 * of three tangent components vanishes in this algebra, so the series is
 * exact.  xi^ [Y; 1] = phi x Y + rho. */
static void project_hd(const double *cam, const double *X, int d, const hd *dt, hd pix[2])
{
    double R[9];
    quat_to_rot(cam + 3, R);
    const hd *rho = dt, *phi = dt + 3, *dX = dt + d;
    hd Yp[3];
    for (int i = 0; i < 3; ++i) {
        hd s = hd_k(cam[i]);
        for (int j = 0; j < 3; ++j) s = hd_add(s, hd_scale(R[3 * i + j], hd_add(hd_k(X[j]), dX[j])));
        Yp[i] = s;
    }
    hd a[3], b[3], Y[3];
    hd_cross(phi, Yp, a);
    for (int i = 0; i < 3; ++i) a[i] = hd_add(a[i], rho[i]);
    hd_cross(phi, a, b);
    for (int i = 0; i < 3; ++i) Y[i] = hd_add(hd_add(Yp[i], a[i]), hd_scale(0.5, b[i]));
    hd f = hd_k(cam[7]), k1 = hd_k(cam[8]), k2 = hd_k(cam[9]);
    if (d == 9) {
        f = hd_add(f, dt[6]);
        k1 = hd_add(k1, dt[7]);
        k2 = hd_add(k2, dt[8]);
    }
    const hd u = hd_scale(-1.0, hd_div(Y[0], Y[2]));
    const hd v = hd_scale(-1.0, hd_div(Y[1], Y[2]));
    const hd s = hd_add(hd_mul(u, u), hd_mul(v, v));
    const hd D = hd_add(hd_k(1.0), hd_add(hd_mul(k1, s), hd_mul(k2, hd_mul(s, s))));
    const hd fD = hd_mul(f, D);
    pix[0] = hd_mul(fD, u);
    pix[1] = hd_mul(fD, v);
}

/* For observation k: residual r (2), J (2 x n, tangent order [camera d,
 * point 3], n = d + 3) and C = sum_m r_m Hess(pi_m) (n x n), all from the
 * hyper-dual evaluation of the projection. */
void orc_obs_second_order(const orc_ctx *c, int64_t k, double *r, double *J, double *C)
{
    const int d = c->o.d, n = d + 3;
    const double *cam = c->cams + 10 * (int64_t)c->cidx[k];
    const double *X = c->pts + 3 * (int64_t)c->pidx[k];
    double H0[144], H1[144];
    hd pix[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    for (int i = 0; i < n; ++i) {
        for (int j = i; j < n; ++j) {
            hd dt[12];
            for (int q = 0; q < 12; ++q) dt[q] = hd_k(0.0);
            dt[i].b = 1.0;
            dt[j].c = 1.0;
            project_hd(cam, X, d, dt, pix);
            if (j == i) {
                J[i] = pix[0].b;
                J[n + i] = pix[1].b;
            }
            H0[i * n + j] = H0[j * n + i] = pix[0].d;
            H1[i * n + j] = H1[j * n + i] = pix[1].d;
        }
    }
    r[0] = pix[0].a - c->obs[2 * k];
    r[1] = pix[1].a - c->obs[2 * k + 1];
    for (int q = 0; q < n * n; ++q) C[q] = r[0] * H0[q] + r[1] * H1[q];
}

/* Dense Cholesky solve of an SPD system of any size: returns 0 on success. */
static int dense_spd_solve(int n, const double *A, const double *b, double *x)
{
    double *L = xcalloc((size_t)n * n, sizeof(double));
    double *y = xcalloc((size_t)n, sizeof(double));
    int st = cholesky(n, A, L);
    if (st == 0) {
        for (int i = 0; i < n; ++i) {
            double s = b[i];
            for (int q = 0; q < i; ++q) s -= L[(size_t)i * n + q] * y[q];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int q = i + 1; q < n; ++q) s -= L[(size_t)q * n + i] * x[q];
            x[i] = s / L[(size_t)i * n + i];
        }
    }
    free(L);
    free(y);
    return st;
}

/* Adjoint at the current parameters (assumed stationary).  gLc: dL/dtheta
 * for the cameras (nc x d, tangent), gLp: for the points (np x 3).  Outputs
 * dLdx (no x 2), dLdw (no, may be NULL), and the adjoint vector v (vc: nc x d,
 * vp: np x 3, either may be NULL).  Returns 0, -1 for a Huber loss
 * (unsupported), -2 when H is not positive definite on the free variables. */
int orc_backward(orc_ctx *c, const double *gLc, const double *gLp, double *dLdx, double *dLdw,
                 double *vc_out, double *vp_out)
{
    if (c->o.huber_delta > 0.0) return -1;
    const int d = c->o.d, n = d + 3;
    const int64_t no = c->no;
    const int nc = c->nc, np = c->np;
    double *J = xcalloc((size_t)no * 2 * n, sizeof(double));
    double *r = xcalloc((size_t)no * 2, sizeof(double));
    double *U = xcalloc((size_t)nc * d * d, sizeof(double));
    double *V = xcalloc((size_t)np * 9, sizeof(double));
    double *W = xcalloc((size_t)no * d * 3, sizeof(double));
    double *Vi = xcalloc((size_t)np * 9, sizeof(double));
    double C[144], A[144];
    for (int64_t k = 0; k < no; ++k) {
        double *Jk = J + (size_t)k * 2 * n;
        orc_obs_second_order(c, k, r + 2 * k, Jk, C);
        if (c->fixed[c->cidx[k]]) { /* constrained camera: no camera tangent */
            for (int m = 0; m < 2; ++m)
                for (int i = 0; i < d; ++i) Jk[m * n + i] = 0.0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    if (i < d || j < d) C[i * n + j] = 0.0;
        }
        const double wk = c->ow[k];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                A[i * n + j] = wk * (Jk[i] * Jk[j] + Jk[n + i] * Jk[n + j] + C[i * n + j]);
        double *Ua = U + (size_t)c->cidx[k] * d * d;
        double *Vj = V + (size_t)c->pidx[k] * 9;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) Ua[i * d + j] += A[i * n + j];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Vj[i * 3 + j] += A[(d + i) * n + d + j];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < 3; ++j) W[(size_t)k * d * 3 + i * 3 + j] = A[i * n + d + j];
    }
    int st = 0;
    for (int j = 0; j < np && st == 0; ++j) {
        if (c->pt_ptr[j + 1] == c->pt_ptr[j]) continue; /* unobserved: v_p = dL/dp / 0 undefined */
        const double det = inverse3(V + 9 * (size_t)j, Vi + 9 * (size_t)j);
        if (!(det > 0.0)) st = -2;
    }
    const int ns = d * nc;
    double *S = xcalloc((size_t)ns * ns, sizeof(double));
    double *b = xcalloc((size_t)ns, sizeof(double));
    double *vc = xcalloc((size_t)ns, sizeof(double));
    double *vp = xcalloc((size_t)np * 3, sizeof(double));
    if (st == 0) {
        for (int a = 0; a < nc; ++a)
            for (int i = 0; i < d; ++i) {
                b[a * d + i] = gLc[a * d + i];
                for (int j = 0; j < d; ++j)
                    S[(size_t)(a * d + i) * ns + a * d + j] = U[(size_t)a * d * d + i * d + j];
            }
        for (int j = 0; j < np; ++j) {
            const double *Vij = Vi + 9 * (size_t)j;
            for (int64_t xi = c->pt_ptr[j]; xi < c->pt_ptr[j + 1]; ++xi) {
                const int64_t x = c->pt_obs[xi];
                const double *Wx = W + (size_t)x * d * 3;
                double Y[27]; /* Y = W_x V_j^-1 (d x 3) */
                for (int i = 0; i < d; ++i)
                    for (int q = 0; q < 3; ++q)
                        Y[i * 3 + q] = Wx[i * 3] * Vij[q] + Wx[i * 3 + 1] * Vij[3 + q] +
                                       Wx[i * 3 + 2] * Vij[6 + q];
                const int ax = c->cidx[x];
                for (int i = 0; i < d; ++i)
                    b[ax * d + i] -= Y[i * 3] * gLp[3 * j] + Y[i * 3 + 1] * gLp[3 * j + 1] +
                                     Y[i * 3 + 2] * gLp[3 * j + 2];
                for (int64_t yi = c->pt_ptr[j]; yi < c->pt_ptr[j + 1]; ++yi) {
                    const int64_t y = c->pt_obs[yi];
                    const double *Wy = W + (size_t)y * d * 3;
                    const int ay = c->cidx[y];
                    for (int i = 0; i < d; ++i)
                        for (int q = 0; q < d; ++q)
                            S[(size_t)(ax * d + i) * ns + ay * d + q] -=
                                Y[i * 3] * Wy[q * 3] + Y[i * 3 + 1] * Wy[q * 3 + 1] +
                                Y[i * 3 + 2] * Wy[q * 3 + 2];
                }
            }
        }
        for (int a = 0; a < nc; ++a) {
            if (!c->fixed[a]) continue;
            for (int i = 0; i < d; ++i) {
                const int row = a * d + i;
                for (int q = 0; q < ns; ++q) S[(size_t)row * ns + q] = S[(size_t)q * ns + row] = 0.0;
                S[(size_t)row * ns + row] = 1.0;
                b[row] = 0.0;
            }
        }
        if (dense_spd_solve(ns, S, b, vc) != 0) st = -2;
    }
    if (st == 0) {
        for (int j = 0; j < np; ++j) {
            double s[3] = {gLp[3 * j], gLp[3 * j + 1], gLp[3 * j + 2]};
            for (int64_t xi = c->pt_ptr[j]; xi < c->pt_ptr[j + 1]; ++xi) {
                const int64_t x = c->pt_obs[xi];
                const double *Wx = W + (size_t)x * d * 3;
                const double *va = vc + (size_t)c->cidx[x] * d;
                for (int q = 0; q < 3; ++q)
                    for (int i = 0; i < d; ++i) s[q] -= Wx[i * 3 + q] * va[i];
            }
            const double *Vij = Vi + 9 * (size_t)j;
            for (int q = 0; q < 3; ++q)
                vp[3 * j + q] = Vij[3 * q] * s[0] + Vij[3 * q + 1] * s[1] + Vij[3 * q + 2] * s[2];
        }
        for (int64_t k = 0; k < no; ++k) {
            const double *Jk = J + (size_t)k * 2 * n;
            const double *va = vc + (size_t)c->cidx[k] * d, *vq = vp + 3 * (size_t)c->pidx[k];
            double e[2];
            for (int m = 0; m < 2; ++m) {
                double s = 0.0;
                for (int i = 0; i < d; ++i) s += Jk[m * n + i] * va[i];
                for (int i = 0; i < 3; ++i) s += Jk[m * n + d + i] * vq[i];
                e[m] = s;
            }
            dLdx[2 * k] = c->ow[k] * e[0];
            dLdx[2 * k + 1] = c->ow[k] * e[1];
            if (dLdw) dLdw[k] = -(r[2 * k] * e[0] + r[2 * k + 1] * e[1]);
        }
        if (vc_out) memcpy(vc_out, vc, sizeof(double) * ns);
        if (vp_out) memcpy(vp_out, vp, sizeof(double) * 3 * np);
    }
    void *p[] = {J, r, U, V, W, Vi, S, b, vc, vp};
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) free(p[i]);
    return st;
}

/* Host-only driver of the C oracle for sanitizer builds (no Python in the
 * process, so AddressSanitizer and UBSan see every access of the oracle's
 * own code).  Reads a scene written by the test, runs LM iterations of both
 * solvers, the adjoint and a pose graph, and prints one line per result.
 *
 * usage: oracle_drive <prefix>
 *   <prefix>.hdr  int64 nc, np, no, n_poses, n_edges
 *   <prefix>.cam/.pt int32 [no]; .obs f64 [no][2]; .cams f64 [nc][10]; .pts f64 [np][3]
 *   <prefix>.ei/.ej int32 [n_edges]; .T f64 [n_edges][7]; .om f64 [n_edges][36]; .Z f64 [n_poses][7]
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t d;
    double huber_delta, cg_rtol;
    int32_t cg_maxiter;
    double lambda0, lambda_min, lambda_max, diag_min, diag_max;
    int32_t solver;
} orc_options;
typedef struct {
    double cost_before, cost_after, lambda_used, lambda_next, cg_rel_resid, pred, grad_inf;
    int32_t accepted, cg_iters, cg_breakdown, status;
} orc_step_info;
typedef struct orc_ctx orc_ctx;
orc_ctx *orc_create(const orc_options *o, int32_t nc, int32_t np, int64_t no, const int32_t *cidx,
                    const int32_t *pidx, const double *obs, const double *ow, const uint8_t *fixed);
void orc_destroy(orc_ctx *c);
void orc_set_params(orc_ctx *c, const double *cams, const double *pts);
int orc_lm_step(orc_ctx *c, double rtol, int32_t maxiter, orc_step_info *info);
int orc_solve(orc_ctx *c, int32_t max_iters, double rel_tol, int32_t plateau_steps, double rtol,
              int32_t maxiter, orc_step_info *infos, int32_t *done, int32_t *reason);
int orc_backward(orc_ctx *c, const double *gLc, const double *gLp, double *dLdx, double *dLdw,
                 double *vc, double *vp);

typedef struct {
    double cg_rtol;
    int32_t cg_maxiter;
    double lambda0, lambda_min, lambda_max, diag_min, diag_max;
    int32_t solver;
} pgo_options;
typedef struct pgo_ctx pgo_ctx;
pgo_ctx *orc_pgo_create(const pgo_options *o, int32_t n, int32_t m, const int32_t *ei, const int32_t *ej,
                        const double *T, const double *omega, const uint8_t *fixed);
void orc_pgo_destroy(pgo_ctx *c);
void orc_pgo_set_poses(pgo_ctx *c, const double *Z);
int orc_pgo_lm_step(pgo_ctx *c, double rtol, int32_t maxiter, orc_step_info *info);

static void *load(const char *pre, const char *ext, size_t bytes)
{
    char fn[1024];
    snprintf(fn, sizeof fn, "%s.%s", pre, ext);
    FILE *f = fopen(fn, "rb");
    if (!f) {
        fprintf(stderr, "missing %s\n", fn);
        exit(2);
    }
    void *p = malloc(bytes ? bytes : 1);
    if (fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short %s\n", fn);
        exit(2);
    }
    fclose(f);
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    const char *pre = argv[1];
    int64_t *h = load(pre, "hdr", 5 * sizeof(int64_t));
    const int32_t nc = (int32_t)h[0], np = (int32_t)h[1];
    const int64_t no = h[2];
    const int32_t nz = (int32_t)h[3], ne = (int32_t)h[4];
    int32_t *cam = load(pre, "cam", 4 * no), *pt = load(pre, "pt", 4 * no);
    double *obs = load(pre, "obs", 16 * no), *cams = load(pre, "cams", 80 * (size_t)nc);
    double *pts = load(pre, "pts", 24 * (size_t)np);
    uint8_t *fixed = calloc((size_t)nc, 1);
    fixed[0] = fixed[1] = 1;
    for (int solver = 0; solver < 2; ++solver) {
        orc_options o = {9, solver ? 0.0 : 1.0, 1e-10, 500, 1e-4, 1e-12, 1e12, 1e-6, 1e32, solver};
        orc_ctx *c = orc_create(&o, nc, np, no, cam, pt, obs, NULL, fixed);
        orc_set_params(c, cams, pts);
        orc_step_info inf[40];
        int32_t done = 0, why = 0;
        const int st = orc_solve(c, 40, 1e-12, 3, -1.0, -1, inf, &done, &why);
        printf("ba solver %d status %d iters %d reason %d cost %.17g\n", solver, st, done, why,
               inf[done - 1].accepted ? inf[done - 1].cost_after : inf[done - 1].cost_before);
        if (solver == 1) {
            /* adjoint of L = sum of the camera translations */
            double *gLc = calloc((size_t)nc * 9, sizeof(double)), *gLp = calloc((size_t)np * 3, sizeof(double));
            double *dx = calloc((size_t)no * 2, sizeof(double)), *dw = calloc((size_t)no, sizeof(double));
            double *vc = calloc((size_t)nc * 9, sizeof(double)), *vp = calloc((size_t)np * 3, sizeof(double));
            for (int32_t i = 0; i < nc; ++i) gLc[9 * i] = 1.0;
            const int sb = orc_backward(c, gLc, gLp, dx, dw, vc, vp);
            double s = 0.0;
            for (int64_t k = 0; k < 2 * no; ++k) s += dx[k];
            printf("adjoint status %d sum %.17g\n", sb, s);
            free(gLc);
            free(gLp);
            free(dx);
            free(dw);
            free(vc);
            free(vp);
        }
        orc_destroy(c);
    }
    int32_t *ei = load(pre, "ei", 4 * (size_t)ne), *ej = load(pre, "ej", 4 * (size_t)ne);
    double *T = load(pre, "T", 56 * (size_t)ne), *om = load(pre, "om", 288 * (size_t)ne);
    double *Z = load(pre, "Z", 56 * (size_t)nz);
    uint8_t *pf = calloc((size_t)nz, 1);
    pf[0] = 1;
    for (int solver = 0; solver < 2; ++solver) {
        pgo_options po = {1e-10, 1000, 1e-4, 1e-12, 1e12, 1e-6, 1e32, solver};
        pgo_ctx *g = orc_pgo_create(&po, nz, ne, ei, ej, T, om, pf);
        orc_pgo_set_poses(g, Z);
        orc_step_info info;
        double F = 0.0;
        for (int it = 0; it < 6; ++it) {
            orc_pgo_lm_step(g, -1.0, -1, &info);
            F = info.accepted ? info.cost_after : info.cost_before;
        }
        printf("pgo solver %d cost %.17g\n", solver, F);
        orc_pgo_destroy(g);
    }
    free(h); free(cam); free(pt); free(obs); free(cams); free(pts); free(fixed);
    free(ei); free(ej); free(T); free(om); free(Z); free(pf);
    return 0;
}

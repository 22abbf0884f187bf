/*
 * Plain FP64 CPU oracle for the OCP-QP primal-dual interior-point method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU path.
 *
 * What it computes (paper: "HPIPM: a high-performance quadratic programming
 * framework for model predictive control", Frison and Diehl):
 *   - the OCP QP of Section 2.2 (stage-wise cost, dynamics, two-sided box and
 *     general constraints), cast into the generic QP form of eq:alg:pdipm:qp
 *     with the two-sided rows stacked as  C = [G; -G],  d = [lo; -hi];
 *   - the residual function of eq:alg:pdipm:delta (r_g, r_b, r_d, r_m);
 *   - the Newton step of eq:alg:pdipm:delta, obtained by eliminating dt and
 *     then dlam (the reduced system eq:alg:kkt) and factorizing that system
 *     with the CLASSICAL Riccati recursion (Section 3.3, variant (a));
 *   - the infeasible-start Mehrotra predictor-corrector IPM in the delta
 *     formulation (Section 4.2, mode "speed"), with the conditional
 *     corrector, the optional primal regularization and the lower clamp on
 *     the multipliers and slacks (Section 4.2, common choices).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   Riccati equations are derived from eq:alg:kkt by dynamic programming:
 *     M_n = Phi_n + F_n' P_{n+1} F_n,  F_n = [B_n A_n],
 *     m_n = gt_n + F_n' (P_{n+1} rb_n + p_{n+1}),
 *     P_n = M_xx - M_xu M_uu^{-1} M_ux,  p_n = m_x - M_xu M_uu^{-1} m_u,
 *     du_n = -M_uu^{-1} (M_ux dx_n + m_u),  dx_{n+1} = F_n dz_n + rb_n,
 *     dpi_{n+1} = P_{n+1} dx_{n+1} + p_{n+1},  dx_0 = -P_0^{-1} p_0.
 *   Init: y = 0, pi = 0, t = max(C y - d, 1), lam = 1.
 *   sigma = (mu_aff / mu)^3; fraction to the boundary gamma; one step length
 *   for primal and dual; the corrector is rejected when the duality measure
 *   after it exceeds corr_ratio times the affine one.
 *
 * No BLAS, no SIMD intrinsics, no threads.  Dense loops only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int N;
    const int *nx, *nu, *nbu, *nbx, *ng; /* length N+1 each */
    const double *A, *B, *b;             /* stages 0..N-1, concatenated, col-major */
    const double *Q, *S, *R, *q, *r;     /* stages 0..N, concatenated, col-major; S is nu x nx */
    const int *idxbu, *idxbx;            /* concatenated index lists */
    const double *lbu, *ubu, *lbx, *ubx;
    const double *D, *C, *lg, *ug;       /* D: ng x nu, C: ng x nx, col-major */
} orc_qp;

typedef struct {
    double tol_stat, tol_eq, tol_ineq, tol_comp;
    int iter_max;
    double alpha_min, gamma, lam_min, t_min, reg_prim, corr_ratio;
    int warm_start; /* 0 cold; 1 primal guess (u, x); 2 primal and dual guess (Section 4.2) */
    int abs_form;   /* 1: absolute formulation (eq:alg:pdipm:abs), exit on the duality measure */
} orc_arg;

/* An iterate, a step or a residual in the user layout: u (sum nu), x (sum nx),
 * pi (sum over n<N of nx[n+1]), and per-stage constraint vectors ordered
 * [box u, box x, general] (sum over n of nbu+nbx+ng). */
typedef struct {
    double *u, *x, *pi, *lam_l, *lam_u, *t_l, *t_u;
} orc_vec;

enum { ORC_SUCCESS = 0, ORC_MAX_ITER = 1, ORC_MIN_STEP = 2, ORC_NAN = 3, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

/* ------------------------------------------------------------------------ */
/* Expanded stage data                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nx, nu, nz, nc, nxn;    /* nxn: nx of stage n+1 (0 at the last stage) */
    double *H;                  /* nz x nz: [[R, S], [S', Q]] */
    double *g;                  /* nz: [r; q] */
    double *F;                  /* nxn x nz: [B A] */
    double *bb;                 /* nxn */
    double *G;                  /* nc x nz: rows [J^{b,u} 0; 0 J^{b,x}; D C] */
    double *lo, *hi;            /* nc */
} stage_t;

typedef struct {
    int N;
    stage_t *st;
    int *zoff, *poff, *coff, *uoff, *xoff;
    int nv, neq, ncon;          /* sizes of y, pi, and of the one-sided constraint count / 2 */
} prob_t;

#define IX(i, j, ld) ((size_t)(j) * (size_t)(ld) + (size_t)(i))

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

static void prob_free(prob_t *p)
{
    if (!p->st) return;
    for (int n = 0; n <= p->N; ++n) {
        stage_t *s = &p->st[n];
        free(s->H); free(s->g); free(s->F); free(s->bb); free(s->G); free(s->lo); free(s->hi);
    }
    free(p->st); free(p->zoff); free(p->poff); free(p->coff); free(p->uoff); free(p->xoff);
    memset(p, 0, sizeof(*p));
}

static int prob_build(const orc_qp *qp, prob_t *p)
{
    memset(p, 0, sizeof(*p));
    int N = qp->N;
    if (N < 0) return ORC_EINVAL;
    p->N = N;
    p->st = (stage_t *)xcalloc((size_t)N + 1, sizeof(stage_t));
    p->zoff = (int *)xcalloc((size_t)N + 2, sizeof(int));
    p->poff = (int *)xcalloc((size_t)N + 2, sizeof(int));
    p->coff = (int *)xcalloc((size_t)N + 2, sizeof(int));
    p->uoff = (int *)xcalloc((size_t)N + 2, sizeof(int));
    p->xoff = (int *)xcalloc((size_t)N + 2, sizeof(int));
    size_t oA = 0, oB = 0, ob = 0, oQ = 0, oS = 0, oR = 0, oq = 0, or_ = 0;
    size_t oiu = 0, oix = 0, oD = 0, oC = 0, og = 0;
    for (int n = 0; n <= N; ++n) {
        stage_t *s = &p->st[n];
        int nx = qp->nx[n], nu = qp->nu[n], nbu = qp->nbu[n], nbx = qp->nbx[n], ng = qp->ng[n];
        if (nx < 0 || nu < 0 || nbu < 0 || nbx < 0 || ng < 0) { prob_free(p); return ORC_EINVAL; }
        s->nx = nx; s->nu = nu; s->nz = nx + nu; s->nc = nbu + nbx + ng;
        s->nxn = (n < N) ? qp->nx[n + 1] : 0;
        int nz = s->nz, nxn = s->nxn, nc = s->nc;
        s->H = (double *)xcalloc((size_t)nz * nz, sizeof(double));
        s->g = (double *)xcalloc((size_t)nz, sizeof(double));
        s->F = (double *)xcalloc((size_t)nxn * nz, sizeof(double));
        s->bb = (double *)xcalloc((size_t)nxn, sizeof(double));
        s->G = (double *)xcalloc((size_t)nc * nz, sizeof(double));
        s->lo = (double *)xcalloc((size_t)nc, sizeof(double));
        s->hi = (double *)xcalloc((size_t)nc, sizeof(double));
        /* Hessian [[R, S], [S', Q]] and gradient [r; q] */
        for (int j = 0; j < nu; ++j)
            for (int i = 0; i < nu; ++i) s->H[IX(i, j, nz)] = qp->R[oR + IX(i, j, nu)];
        for (int j = 0; j < nx; ++j)
            for (int i = 0; i < nu; ++i) {
                double v = qp->S[oS + IX(i, j, nu)];
                s->H[IX(i, nu + j, nz)] = v;
                s->H[IX(nu + j, i, nz)] = v;
            }
        for (int j = 0; j < nx; ++j)
            for (int i = 0; i < nx; ++i) s->H[IX(nu + i, nu + j, nz)] = qp->Q[oQ + IX(i, j, nx)];
        for (int i = 0; i < nu; ++i) s->g[i] = qp->r[or_ + i];
        for (int i = 0; i < nx; ++i) s->g[nu + i] = qp->q[oq + i];
        oR += (size_t)nu * nu; oS += (size_t)nu * nx; oQ += (size_t)nx * nx; or_ += nu; oq += nx;
        /* dynamics F = [B A] */
        if (n < N) {
            for (int j = 0; j < nu; ++j)
                for (int i = 0; i < nxn; ++i) s->F[IX(i, j, nxn)] = qp->B[oB + IX(i, j, nxn)];
            for (int j = 0; j < nx; ++j)
                for (int i = 0; i < nxn; ++i) s->F[IX(i, nu + j, nxn)] = qp->A[oA + IX(i, j, nxn)];
            for (int i = 0; i < nxn; ++i) s->bb[i] = qp->b[ob + i];
            oB += (size_t)nxn * nu; oA += (size_t)nxn * nx; ob += nxn;
        }
        /* constraint rows */
        int row = 0;
        for (int k = 0; k < nbu; ++k, ++row) {
            int j = qp->idxbu[oiu + k];
            if (j < 0 || j >= nu) { prob_free(p); return ORC_EINVAL; }
            s->G[IX(row, j, nc)] = 1.0;
            s->lo[row] = qp->lbu[oiu + k]; s->hi[row] = qp->ubu[oiu + k];
        }
        for (int k = 0; k < nbx; ++k, ++row) {
            int j = qp->idxbx[oix + k];
            if (j < 0 || j >= nx) { prob_free(p); return ORC_EINVAL; }
            s->G[IX(row, nu + j, nc)] = 1.0;
            s->lo[row] = qp->lbx[oix + k]; s->hi[row] = qp->ubx[oix + k];
        }
        for (int k = 0; k < ng; ++k, ++row) {
            for (int j = 0; j < nu; ++j) s->G[IX(row, j, nc)] = qp->D[oD + IX(k, j, ng)];
            for (int j = 0; j < nx; ++j) s->G[IX(row, nu + j, nc)] = qp->C[oC + IX(k, j, ng)];
            s->lo[row] = qp->lg[og + k]; s->hi[row] = qp->ug[og + k];
        }
        for (int k = 0; k < nc; ++k)
            if (!(s->lo[k] <= s->hi[k])) { prob_free(p); return ORC_EINVAL; }
        oiu += nbu; oix += nbx; oD += (size_t)ng * nu; oC += (size_t)ng * nx; og += ng;
        p->zoff[n + 1] = p->zoff[n] + nz;
        p->poff[n + 1] = p->poff[n] + nxn;
        p->coff[n + 1] = p->coff[n] + nc;
        p->uoff[n + 1] = p->uoff[n] + nu;
        p->xoff[n + 1] = p->xoff[n] + nx;
    }
    p->nv = p->zoff[N + 1];
    p->neq = p->poff[N + 1];
    p->ncon = p->coff[N + 1];
    return 0;
}

/* Internal vectors: y (nv, stage-wise [u; x]), pi (neq, pi_{n+1} for n<N),
 * and four constraint vectors (ncon each). */
typedef struct {
    double *y, *pi, *ll, *lu, *tl, *tu;
} ivec_t;

static int ivec_alloc(const prob_t *p, ivec_t *v)
{
    v->y = (double *)xcalloc((size_t)p->nv, sizeof(double));
    v->pi = (double *)xcalloc((size_t)p->neq, sizeof(double));
    v->ll = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    v->lu = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    v->tl = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    v->tu = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    return (v->y && v->pi && v->ll && v->lu && v->tl && v->tu) ? 0 : ORC_ENOMEM;
}

static void ivec_free(ivec_t *v)
{
    free(v->y); free(v->pi); free(v->ll); free(v->lu); free(v->tl); free(v->tu);
    memset(v, 0, sizeof(*v));
}

static void ivec_from_user(const prob_t *p, const orc_vec *in, ivec_t *v)
{
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        for (int i = 0; i < s->nu; ++i) v->y[p->zoff[n] + i] = in->u[p->uoff[n] + i];
        for (int i = 0; i < s->nx; ++i) v->y[p->zoff[n] + s->nu + i] = in->x[p->xoff[n] + i];
    }
    memcpy(v->pi, in->pi, sizeof(double) * (size_t)p->neq);
    memcpy(v->ll, in->lam_l, sizeof(double) * (size_t)p->ncon);
    memcpy(v->lu, in->lam_u, sizeof(double) * (size_t)p->ncon);
    memcpy(v->tl, in->t_l, sizeof(double) * (size_t)p->ncon);
    memcpy(v->tu, in->t_u, sizeof(double) * (size_t)p->ncon);
}

static void ivec_to_user(const prob_t *p, const ivec_t *v, orc_vec *out)
{
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        for (int i = 0; i < s->nu; ++i) out->u[p->uoff[n] + i] = v->y[p->zoff[n] + i];
        for (int i = 0; i < s->nx; ++i) out->x[p->xoff[n] + i] = v->y[p->zoff[n] + s->nu + i];
    }
    memcpy(out->pi, v->pi, sizeof(double) * (size_t)p->neq);
    memcpy(out->lam_l, v->ll, sizeof(double) * (size_t)p->ncon);
    memcpy(out->lam_u, v->lu, sizeof(double) * (size_t)p->ncon);
    memcpy(out->t_l, v->tl, sizeof(double) * (size_t)p->ncon);
    memcpy(out->t_u, v->tu, sizeof(double) * (size_t)p->ncon);
}

/* ------------------------------------------------------------------------ */
/* Residual function, eq:alg:pdipm:delta right-hand side                     */
/*   r_g = H y + g - A' pi - C' lam                                           */
/*   r_b = -A y + b                                                           */
/*   r_d = -C y + t + d        (lower rows: -G z + t_l + lo;                  */
/*                              upper rows:  G z + t_u - hi)                  */
/* Here the r_g / r_b / r_d "constants" are passed in, so that the same code  */
/* also evaluates the iterative-refinement residual K*step + r, Section 3.4.  */
/* ------------------------------------------------------------------------ */

/* out_g = H y + cg - A' pi - C' lam  (per stage)
 * out_b = -A y + cb
 * out_dl = -G z + tl + cdl ;  out_du = G z + tu + cdu */
static void kkt_apply(const prob_t *p, const ivec_t *v, int with_H,
                      const double *cg, const double *cb, const double *cdl, const double *cdu,
                      double *og, double *ob, double *odl, double *odu)
{
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        const double *z = v->y + p->zoff[n];
        double *rg = og + p->zoff[n];
        for (int i = 0; i < s->nz; ++i) {
            double acc = cg ? cg[p->zoff[n] + i] : 0.0;
            if (with_H)
                for (int j = 0; j < s->nz; ++j) acc += s->H[IX(i, j, s->nz)] * z[j];
            rg[i] = acc;
        }
        /* -A' pi : +F' pi_{n+1} on z_n, -pi_n on x_n */
        if (n < p->N) {
            const double *pin = v->pi + p->poff[n];
            for (int j = 0; j < s->nz; ++j) {
                double acc = 0.0;
                for (int i = 0; i < s->nxn; ++i) acc += s->F[IX(i, j, s->nxn)] * pin[i];
                rg[j] += acc;
            }
        }
        if (n > 0) {
            const double *pin = v->pi + p->poff[n - 1];
            for (int i = 0; i < s->nx; ++i) rg[s->nu + i] -= pin[i];
        }
        /* -C' lam = -G'(lam_l - lam_u) */
        const double *ll = v->ll + p->coff[n], *lu = v->lu + p->coff[n];
        for (int j = 0; j < s->nz; ++j) {
            double acc = 0.0;
            for (int k = 0; k < s->nc; ++k) acc += s->G[IX(k, j, s->nc)] * (ll[k] - lu[k]);
            rg[j] -= acc;
        }
        /* r_b,n = F z_n + cb_n - x_{n+1}    (that is -A y + b) */
        if (n < p->N) {
            const double *zn1 = v->y + p->zoff[n + 1] + p->st[n + 1].nu;
            double *rb = ob + p->poff[n];
            for (int i = 0; i < s->nxn; ++i) {
                double acc = cb ? cb[p->poff[n] + i] : 0.0;
                for (int j = 0; j < s->nz; ++j) acc += s->F[IX(i, j, s->nxn)] * z[j];
                rb[i] = acc - zn1[i];
            }
        }
        /* r_d */
        const double *tl = v->tl + p->coff[n], *tu = v->tu + p->coff[n];
        for (int k = 0; k < s->nc; ++k) {
            double gz = 0.0;
            for (int j = 0; j < s->nz; ++j) gz += s->G[IX(k, j, s->nc)] * z[j];
            odl[p->coff[n] + k] = -gz + tl[k] + (cdl ? cdl[p->coff[n] + k] : 0.0);
            odu[p->coff[n] + k] = gz + tu[k] + (cdu ? cdu[p->coff[n] + k] : 0.0);
        }
    }
}

/* The constant part of the residual function: g, b and d = [lo; -hi]
 * (the residual at y = 0, pi = 0, lam = 0, t = 0). */
static void data_terms(const prob_t *p, double *cg, double *cb, double *cdl, double *cdu)
{
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        for (int i = 0; i < s->nz; ++i) cg[p->zoff[n] + i] = s->g[i];
        for (int i = 0; i < s->nxn; ++i) cb[p->poff[n] + i] = s->bb[i];
        for (int k = 0; k < s->nc; ++k) {
            cdl[p->coff[n] + k] = s->lo[k];
            cdu[p->coff[n] + k] = -s->hi[k];
        }
    }
}

/* IPM residuals at an iterate: constants g, b, d = [lo; -hi]. */
static void residuals(const prob_t *p, const ivec_t *v, double *rg, double *rb, double *rdl, double *rdu)
{
    double *cg = (double *)xcalloc((size_t)p->nv, sizeof(double));
    double *cb = (double *)xcalloc((size_t)p->neq, sizeof(double));
    double *cdl = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    double *cdu = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    data_terms(p, cg, cb, cdl, cdu);
    kkt_apply(p, v, 1, cg, cb, cdl, cdu, rg, rb, rdl, rdu);
    free(cg); free(cb); free(cdl); free(cdu);
}

static double inf_norm(const double *v, int n)
{
    double m = 0.0;
    for (int i = 0; i < n; ++i) {
        double a = fabs(v[i]);
        if (a != a) return a; /* NaN propagates */
        if (a > m) m = a;
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (column-major, in place)                   */
/* ------------------------------------------------------------------------ */

static int lu_factor(int n, double *a, int lda, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int pk = k;
        double best = fabs(a[IX(k, k, lda)]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(a[IX(i, k, lda)]) > best) { best = fabs(a[IX(i, k, lda)]); pk = i; }
        piv[k] = pk;
        if (best == 0.0) return -1;
        if (pk != k)
            for (int j = 0; j < n; ++j) {
                double t = a[IX(k, j, lda)]; a[IX(k, j, lda)] = a[IX(pk, j, lda)]; a[IX(pk, j, lda)] = t;
            }
        double d = a[IX(k, k, lda)];
        for (int i = k + 1; i < n; ++i) a[IX(i, k, lda)] /= d;
        for (int j = k + 1; j < n; ++j) {
            double akj = a[IX(k, j, lda)];
            for (int i = k + 1; i < n; ++i) a[IX(i, j, lda)] -= a[IX(i, k, lda)] * akj;
        }
    }
    return 0;
}

/* Solve (LU) X = B for nrhs columns of B (col-major, ldb). */
static void lu_solve(int n, const double *a, int lda, const int *piv, double *bm, int ldb, int nrhs)
{
    for (int c = 0; c < nrhs; ++c) {
        double *x = bm + (size_t)c * ldb;
        for (int k = 0; k < n; ++k)
            if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
        for (int k = 0; k < n; ++k)
            for (int i = k + 1; i < n; ++i) x[i] -= a[IX(i, k, lda)] * x[k];
        for (int k = n - 1; k >= 0; --k) {
            x[k] /= a[IX(k, k, lda)];
            for (int i = 0; i < k; ++i) x[i] -= a[IX(i, k, lda)] * x[k];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Classical Riccati factorization of the reduced system eq:alg:kkt          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *M;    /* nz x nz, the full stage matrix M_n (kept whole) */
    double *Luu;  /* nu x nu LU factors of M_uu */
    int *piv;     /* nu */
    double *K;    /* nu x nx : M_uu^{-1} M_ux */
    double *P;    /* nx x nx */
} fac_stage_t;

typedef struct {
    int N;
    fac_stage_t *fs;
    double *LP0;  /* LU of P_0 */
    int *piv0;
} fac_t;

static void fac_free(fac_t *f)
{
    if (!f->fs) return;
    for (int n = 0; n <= f->N; ++n) {
        free(f->fs[n].M); free(f->fs[n].Luu); free(f->fs[n].piv); free(f->fs[n].K); free(f->fs[n].P);
    }
    free(f->fs); free(f->LP0); free(f->piv0);
    memset(f, 0, sizeof(*f));
}

/* Phi_n = H_n + G_n' diag(wl + wu) G_n + reg I.  Backward recursion. */
static int factorize(const prob_t *p, const double *wl, const double *wu, double reg, fac_t *f)
{
    int N = p->N;
    f->N = N;
    f->fs = (fac_stage_t *)xcalloc((size_t)N + 1, sizeof(fac_stage_t));
    for (int n = N; n >= 0; --n) {
        const stage_t *s = &p->st[n];
        fac_stage_t *fs = &f->fs[n];
        int nz = s->nz, nu = s->nu, nx = s->nx, nxn = s->nxn, nc = s->nc;
        fs->M = (double *)xcalloc((size_t)nz * nz, sizeof(double));
        fs->Luu = (double *)xcalloc((size_t)nu * nu, sizeof(double));
        fs->piv = (int *)xcalloc((size_t)nu, sizeof(int));
        fs->K = (double *)xcalloc((size_t)nu * nx, sizeof(double));
        fs->P = (double *)xcalloc((size_t)nx * nx, sizeof(double));
        double *M = fs->M;
        for (int j = 0; j < nz; ++j)
            for (int i = 0; i < nz; ++i) M[IX(i, j, nz)] = s->H[IX(i, j, nz)];
        for (int i = 0; i < nz; ++i) M[IX(i, i, nz)] += reg;
        const double *wln = wl + p->coff[n], *wun = wu + p->coff[n];
        for (int k = 0; k < nc; ++k) {
            double w = wln[k] + wun[k];
            for (int j = 0; j < nz; ++j)
                for (int i = 0; i < nz; ++i) M[IX(i, j, nz)] += s->G[IX(k, i, nc)] * w * s->G[IX(k, j, nc)];
        }
        if (n < N) {
            const double *Pn1 = f->fs[n + 1].P;
            /* M += F' P_{n+1} F */
            double *PF = (double *)xcalloc((size_t)nxn * nz, sizeof(double));
            for (int j = 0; j < nz; ++j)
                for (int i = 0; i < nxn; ++i) {
                    double acc = 0.0;
                    for (int k = 0; k < nxn; ++k) acc += Pn1[IX(i, k, nxn)] * s->F[IX(k, j, nxn)];
                    PF[IX(i, j, nxn)] = acc;
                }
            for (int j = 0; j < nz; ++j)
                for (int i = 0; i < nz; ++i) {
                    double acc = 0.0;
                    for (int k = 0; k < nxn; ++k) acc += s->F[IX(k, i, nxn)] * PF[IX(k, j, nxn)];
                    M[IX(i, j, nz)] += acc;
                }
            free(PF);
        }
        /* M_uu factor, K = M_uu^{-1} M_ux, P = M_xx - M_xu K */
        for (int j = 0; j < nu; ++j)
            for (int i = 0; i < nu; ++i) fs->Luu[IX(i, j, nu)] = M[IX(i, j, nz)];
        if (nu > 0 && lu_factor(nu, fs->Luu, nu, fs->piv) != 0) return -1;
        for (int j = 0; j < nx; ++j)
            for (int i = 0; i < nu; ++i) fs->K[IX(i, j, nu)] = M[IX(i, nu + j, nz)];
        if (nu > 0) lu_solve(nu, fs->Luu, nu, fs->piv, fs->K, nu, nx);
        for (int j = 0; j < nx; ++j)
            for (int i = 0; i < nx; ++i) {
                double acc = M[IX(nu + i, nu + j, nz)];
                for (int k = 0; k < nu; ++k) acc -= M[IX(nu + i, k, nz)] * fs->K[IX(k, j, nu)];
                fs->P[IX(i, j, nx)] = acc;
            }
    }
    int nx0 = p->st[0].nx;
    f->LP0 = (double *)xcalloc((size_t)nx0 * nx0, sizeof(double));
    f->piv0 = (int *)xcalloc((size_t)nx0, sizeof(int));
    memcpy(f->LP0, f->fs[0].P, sizeof(double) * (size_t)nx0 * nx0);
    if (nx0 > 0 && lu_factor(nx0, f->LP0, nx0, f->piv0) != 0) return -1;
    return 0;
}

/* Solve  [Phi -A'; -A 0][dy; dpi] = -[gt; rb]  with the stored recursion. */
static void riccati_solve(const prob_t *p, const fac_t *f, const double *gt, const double *rb,
                          double *dy, double *dpi)
{
    int N = p->N;
    double **pv = (double **)xcalloc((size_t)N + 1, sizeof(double *));
    double **kv = (double **)xcalloc((size_t)N + 1, sizeof(double *));
    /* backward: m_n, k_n = M_uu^{-1} m_u, p_n = m_x - M_xu k_n */
    for (int n = N; n >= 0; --n) {
        const stage_t *s = &p->st[n];
        const fac_stage_t *fs = &f->fs[n];
        int nz = s->nz, nu = s->nu, nx = s->nx, nxn = s->nxn;
        double *m = (double *)xcalloc((size_t)nz, sizeof(double));
        for (int i = 0; i < nz; ++i) m[i] = gt[p->zoff[n] + i];
        if (n < N) {
            const double *Pn1 = f->fs[n + 1].P;
            double *v = (double *)xcalloc((size_t)nxn, sizeof(double));
            for (int i = 0; i < nxn; ++i) {
                double acc = pv[n + 1][i];
                for (int k = 0; k < nxn; ++k) acc += Pn1[IX(i, k, nxn)] * rb[p->poff[n] + k];
                v[i] = acc;
            }
            for (int j = 0; j < nz; ++j) {
                double acc = 0.0;
                for (int i = 0; i < nxn; ++i) acc += s->F[IX(i, j, nxn)] * v[i];
                m[j] += acc;
            }
            free(v);
        }
        kv[n] = (double *)xcalloc((size_t)nu, sizeof(double));
        for (int i = 0; i < nu; ++i) kv[n][i] = m[i];
        if (nu > 0) lu_solve(nu, fs->Luu, nu, fs->piv, kv[n], nu, 1);
        pv[n] = (double *)xcalloc((size_t)nx, sizeof(double));
        for (int i = 0; i < nx; ++i) {
            double acc = m[nu + i];
            for (int k = 0; k < nu; ++k) acc -= fs->M[IX(nu + i, k, nz)] * kv[n][k];
            pv[n][i] = acc;
        }
        free(m);
    }
    /* dx_0 = -P_0^{-1} p_0 */
    int nx0 = p->st[0].nx;
    double *dx = (double *)xcalloc((size_t)nx0, sizeof(double));
    for (int i = 0; i < nx0; ++i) dx[i] = -pv[0][i];
    if (nx0 > 0) lu_solve(nx0, f->LP0, nx0, f->piv0, dx, nx0, 1);
    /* forward */
    for (int n = 0; n <= N; ++n) {
        const stage_t *s = &p->st[n];
        const fac_stage_t *fs = &f->fs[n];
        int nu = s->nu, nx = s->nx, nxn = s->nxn, nz = s->nz;
        double *dz = dy + p->zoff[n];
        for (int i = 0; i < nu; ++i) {
            double acc = kv[n][i];
            for (int k = 0; k < nx; ++k) acc += fs->K[IX(i, k, nu)] * dx[k];
            dz[i] = -acc;
        }
        for (int i = 0; i < nx; ++i) dz[nu + i] = dx[i];
        if (n < N) {
            const double *Pn1 = f->fs[n + 1].P;
            double *dxn = (double *)xcalloc((size_t)nxn, sizeof(double));
            for (int i = 0; i < nxn; ++i) {
                double acc = rb[p->poff[n] + i];
                for (int j = 0; j < nz; ++j) acc += s->F[IX(i, j, nxn)] * dz[j];
                dxn[i] = acc;
            }
            for (int i = 0; i < nxn; ++i) {
                double acc = pv[n + 1][i];
                for (int k = 0; k < nxn; ++k) acc += Pn1[IX(i, k, nxn)] * dxn[k];
                dpi[p->poff[n] + i] = acc;
            }
            free(dx);
            dx = dxn;
        }
    }
    free(dx);
    for (int n = 0; n <= N; ++n) { free(pv[n]); free(kv[n]); }
    free(pv); free(kv);
}

/* Full Newton step of eq:alg:pdipm:delta given the residuals (rg, rb, rdl,
 * rdu, rml, rmu) at iterate v and a factorization built from w = lam / t.
 * Elimination of dt then dlam (Section 3.3):
 *   gt = rg - C'(W rd - T^{-1} rm)
 *   dt = C dy - rd,    dlam = -T^{-1}(rm + Lam dt). */
static void newton_solve(const prob_t *p, const fac_t *f, const ivec_t *v,
                         const double *rg, const double *rb, const double *rdl, const double *rdu,
                         const double *rml, const double *rmu, ivec_t *d)
{
    double *gt = (double *)xcalloc((size_t)p->nv, sizeof(double));
    for (int i = 0; i < p->nv; ++i) gt[i] = rg[i];
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        int c0 = p->coff[n];
        for (int k = 0; k < s->nc; ++k) {
            int c = c0 + k;
            double el = (v->ll[c] / v->tl[c]) * rdl[c] - rml[c] / v->tl[c];
            double eu = (v->lu[c] / v->tu[c]) * rdu[c] - rmu[c] / v->tu[c];
            /* C'(e) with C = [G; -G]: G'(el) - G'(eu) */
            for (int j = 0; j < s->nz; ++j) gt[p->zoff[n] + j] -= s->G[IX(k, j, s->nc)] * (el - eu);
        }
    }
    riccati_solve(p, f, gt, rb, d->y, d->pi);
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        const double *dz = d->y + p->zoff[n];
        for (int k = 0; k < s->nc; ++k) {
            int c = p->coff[n] + k;
            double gdz = 0.0;
            for (int j = 0; j < s->nz; ++j) gdz += s->G[IX(k, j, s->nc)] * dz[j];
            d->tl[c] = gdz - rdl[c];
            d->tu[c] = -gdz - rdu[c];
            d->ll[c] = -(rml[c] + v->ll[c] * d->tl[c]) / v->tl[c];
            d->lu[c] = -(rmu[c] + v->lu[c] * d->tu[c]) / v->tu[c];
        }
    }
    free(gt);
}

/* Newton step in the absolute formulation (Section 3.2, eq:alg:pdipm:abs):
 * the same matrix with right-hand side -[g; b; d; rm - 2 Lam T e] (the
 * first three blocks linear in the iterate, so only their constant part
 * remains; rm is the delta formulation's complementarity term, e.g. lam.*t -
 * tau), whose solution is the full-step iterate; the step is its difference
 * with the current iterate (eq:alg:pdipm:step). */
static void newton_solve_abs(const prob_t *p, const fac_t *f, const ivec_t *v, const double *rml, const double *rmu,
                             ivec_t *d)
{
    int nc = p->ncon;
    double *cg = (double *)xcalloc((size_t)p->nv, sizeof(double));
    double *cb = (double *)xcalloc((size_t)p->neq, sizeof(double));
    double *cdl = (double *)xcalloc((size_t)nc, sizeof(double));
    double *cdu = (double *)xcalloc((size_t)nc, sizeof(double));
    double *al = (double *)xcalloc((size_t)nc, sizeof(double));
    double *au = (double *)xcalloc((size_t)nc, sizeof(double));
    data_terms(p, cg, cb, cdl, cdu);
    for (int i = 0; i < nc; ++i) {
        al[i] = rml[i] - 2.0 * v->ll[i] * v->tl[i];
        au[i] = rmu[i] - 2.0 * v->lu[i] * v->tu[i];
    }
    newton_solve(p, f, v, cg, cb, cdl, cdu, al, au, d);
    for (int i = 0; i < p->nv; ++i) d->y[i] -= v->y[i];
    for (int i = 0; i < p->neq; ++i) d->pi[i] -= v->pi[i];
    for (int i = 0; i < nc; ++i) {
        d->ll[i] -= v->ll[i];
        d->lu[i] -= v->lu[i];
        d->tl[i] -= v->tl[i];
        d->tu[i] -= v->tu[i];
    }
    free(cg); free(cb); free(cdl); free(cdu); free(al); free(au);
}

/* Largest alpha (uncapped; HUGE_VAL if no component blocks) keeping
 * lam + alpha dlam >= 0 and t + alpha dt >= 0. */
static double max_step(const prob_t *p, const ivec_t *v, const ivec_t *d)
{
    double a = HUGE_VAL;
    const double *vv[4] = {v->ll, v->lu, v->tl, v->tu};
    const double *dd[4] = {d->ll, d->lu, d->tl, d->tu};
    for (int s = 0; s < 4; ++s)
        for (int i = 0; i < p->ncon; ++i)
            if (dd[s][i] < 0.0) {
                double r = -vv[s][i] / dd[s][i];
                if (r < a) a = r;
            }
    return a;
}

static double mu_after(const prob_t *p, const ivec_t *v, const ivec_t *d, double alpha)
{
    double acc = 0.0;
    for (int i = 0; i < p->ncon; ++i) {
        acc += (v->ll[i] + alpha * d->ll[i]) * (v->tl[i] + alpha * d->tl[i]);
        acc += (v->lu[i] + alpha * d->lu[i]) * (v->tu[i] + alpha * d->tu[i]);
    }
    return acc / (2.0 * p->ncon);
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                      */
/* ------------------------------------------------------------------------ */

/* Residuals at a user-layout iterate.  Outputs in the user layout of a
 * step (u / x slots hold r_g split by stage, pi slot holds r_b, lam_l/lam_u
 * slots hold r_d lower / upper, t_l/t_u slots hold lam_l*t_l, lam_u*t_u).
 * norms: inf-norms of r_g, r_b, r_d and lam.*t; mu = lam't / n_c. */
int orc_residuals(const orc_qp *qp, const orc_vec *it, orc_vec *res, double *norms, double *mu)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    ivec_t v, r;
    ivec_alloc(&p, &v); ivec_alloc(&p, &r);
    ivec_from_user(&p, it, &v);
    residuals(&p, &v, r.y, r.pi, r.ll, r.lu);
    double comp = 0.0, lt = 0.0;
    for (int i = 0; i < p.ncon; ++i) {
        r.tl[i] = v.ll[i] * v.tl[i];
        r.tu[i] = v.lu[i] * v.tu[i];
        lt += r.tl[i] + r.tu[i];
    }
    comp = inf_norm(r.tl, p.ncon);
    double cu = inf_norm(r.tu, p.ncon);
    if (cu > comp || cu != cu) comp = cu;
    if (norms) {
        double dl = inf_norm(r.ll, p.ncon), du = inf_norm(r.lu, p.ncon);
        norms[0] = inf_norm(r.y, p.nv);
        norms[1] = inf_norm(r.pi, p.neq);
        norms[2] = (du > dl || du != du) ? du : dl;
        norms[3] = comp;
    }
    if (mu) *mu = p.ncon ? lt / (2.0 * p.ncon) : 0.0;
    if (res) ivec_to_user(&p, &r, res);
    ivec_free(&v); ivec_free(&r);
    prob_free(&p);
    return 0;
}

/* Newton step of eq:alg:pdipm:delta at the iterate `it` with r_m = lam.*t - tau,
 * factorized with regularization `reg`; with abs_form, the same step through
 * the absolute formulation.  Returns the step in user layout. */
int orc_newton_step(const orc_qp *qp, const orc_vec *it, double tau, double reg, int abs_form, orc_vec *step)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    ivec_t v, r, d;
    ivec_alloc(&p, &v); ivec_alloc(&p, &r); ivec_alloc(&p, &d);
    ivec_from_user(&p, it, &v);
    residuals(&p, &v, r.y, r.pi, r.ll, r.lu);
    double *wl = (double *)xcalloc((size_t)p.ncon, sizeof(double));
    double *wu = (double *)xcalloc((size_t)p.ncon, sizeof(double));
    for (int i = 0; i < p.ncon; ++i) {
        wl[i] = v.ll[i] / v.tl[i];
        wu[i] = v.lu[i] / v.tu[i];
        r.tl[i] = v.ll[i] * v.tl[i] - tau;
        r.tu[i] = v.lu[i] * v.tu[i] - tau;
    }
    fac_t f;
    memset(&f, 0, sizeof(f));
    rc = factorize(&p, wl, wu, reg, &f);
    if (rc == 0) {
        if (abs_form) newton_solve_abs(&p, &f, &v, r.tl, r.tu, &d);
        else newton_solve(&p, &f, &v, r.y, r.pi, r.ll, r.lu, r.tl, r.tu, &d);
        ivec_to_user(&p, &d, step);
    }
    fac_free(&f);
    free(wl); free(wu);
    ivec_free(&v); ivec_free(&r); ivec_free(&d);
    prob_free(&p);
    return rc ? ORC_NAN : 0;
}

/* The IPM.  On return `sol` holds the final iterate; iters, the number of
 * iterations taken; res_norms the four residual inf-norms at the final
 * iterate; mu_out the final duality measure.  The return value is the
 * solver status (>= 0) or a usage error (< 0). */
int orc_solve(const orc_qp *qp, const orc_arg *arg, orc_vec *sol, int *iters, double *res_norms, double *mu_out)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    ivec_t v, r, d, dc;
    ivec_alloc(&p, &v); ivec_alloc(&p, &r); ivec_alloc(&p, &d); ivec_alloc(&p, &dc);
    int nc = p.ncon;
    double *wl = (double *)xcalloc((size_t)nc, sizeof(double));
    double *wu = (double *)xcalloc((size_t)nc, sizeof(double));
    double *rml = (double *)xcalloc((size_t)nc, sizeof(double));
    double *rmu = (double *)xcalloc((size_t)nc, sizeof(double));

    /* Initial point.  Cold start: y = 0, pi = 0, t = max(C y - d, 1), lam = 1.
     * Warm start (Section 4.2) from the iterate passed in `sol`: with a primal
     * guess, y is the guess and the rest is set as in the cold start at that
     * y; with a primal and dual guess, every block is the guess, multipliers
     * and slacks clamped below as in the iterate update. */
    if (arg->warm_start != 0) ivec_from_user(&p, sol, &v);
    if (arg->warm_start == 2) {
        for (int i = 0; i < nc; ++i) {
            if (v.ll[i] < arg->lam_min) v.ll[i] = arg->lam_min;
            if (v.lu[i] < arg->lam_min) v.lu[i] = arg->lam_min;
            if (v.tl[i] < arg->t_min) v.tl[i] = arg->t_min;
            if (v.tu[i] < arg->t_min) v.tu[i] = arg->t_min;
        }
    } else {
        if (arg->warm_start == 0)
            for (int i = 0; i < p.nv; ++i) v.y[i] = 0.0;
        for (int i = 0; i < p.neq; ++i) v.pi[i] = 0.0;
        for (int n = 0; n <= p.N; ++n) {
            const stage_t *s = &p.st[n];
            const double *z = v.y + p.zoff[n];
            for (int k = 0; k < s->nc; ++k) {
                int c = p.coff[n] + k;
                double gz = 0.0;
                for (int j = 0; j < s->nz; ++j) gz += s->G[IX(k, j, s->nc)] * z[j];
                double tl0 = gz - s->lo[k], tu0 = s->hi[k] - gz;
                v.tl[c] = tl0 > 1.0 ? tl0 : 1.0;
                v.tu[c] = tu0 > 1.0 ? tu0 : 1.0;
                v.ll[c] = 1.0;
                v.lu[c] = 1.0;
            }
        }
    }

    int status = ORC_MAX_ITER, k = 0;
    double norms[4] = {0, 0, 0, 0}, mu = 0.0;
    const int absf = arg->abs_form != 0;
    for (k = 0;; ++k) {
        /* absolute formulation (Section 4.2, mode speed_abs): no residuals in
         * the loop, exit on the duality measure alone */
        if (!absf) residuals(&p, &v, r.y, r.pi, r.ll, r.lu);
        double lt = 0.0, comp = 0.0;
        for (int i = 0; i < nc; ++i) {
            double a = v.ll[i] * v.tl[i], b2 = v.lu[i] * v.tu[i];
            lt += a + b2;
            if (a > comp) comp = a;
            if (b2 > comp) comp = b2;
        }
        mu = nc ? lt / (2.0 * nc) : 0.0;
        if (absf) {
            if (mu != mu) { status = ORC_NAN; break; }
            if (mu <= arg->tol_comp) { status = ORC_SUCCESS; break; }
        } else {
            double dl = inf_norm(r.ll, nc), du = inf_norm(r.lu, nc);
            norms[0] = inf_norm(r.y, p.nv);
            norms[1] = inf_norm(r.pi, p.neq);
            norms[2] = du > dl ? du : dl;
            norms[3] = comp;
            if (norms[0] != norms[0] || norms[1] != norms[1] || norms[2] != norms[2] || mu != mu) {
                status = ORC_NAN;
                break;
            }
            if (norms[0] <= arg->tol_stat && norms[1] <= arg->tol_eq && norms[2] <= arg->tol_ineq &&
                norms[3] <= arg->tol_comp) {
                status = ORC_SUCCESS;
                break;
            }
        }
        if (k >= arg->iter_max) { status = ORC_MAX_ITER; break; }

        for (int i = 0; i < nc; ++i) { wl[i] = v.ll[i] / v.tl[i]; wu[i] = v.lu[i] / v.tu[i]; }
        fac_t f;
        memset(&f, 0, sizeof(f));
        if (factorize(&p, wl, wu, arg->reg_prim, &f) != 0) { fac_free(&f); status = ORC_NAN; break; }

        /* predictor (affine): r_m = lam.*t */
        for (int i = 0; i < nc; ++i) { rml[i] = v.ll[i] * v.tl[i]; rmu[i] = v.lu[i] * v.tu[i]; }
        if (absf) newton_solve_abs(&p, &f, &v, rml, rmu, &d);
        else newton_solve(&p, &f, &v, r.y, r.pi, r.ll, r.lu, rml, rmu, &d);
        ivec_t *step = &d;
        if (nc > 0) {
            double a_aff = max_step(&p, &v, &d);
            if (a_aff > 1.0) a_aff = 1.0;
            double mu_aff = mu_after(&p, &v, &d, a_aff);
            double sigma = mu > 0.0 ? (mu_aff / mu) * (mu_aff / mu) * (mu_aff / mu) : 0.0;
            /* corrector: r_m = lam.*t + dlam_aff.*dt_aff - sigma mu */
            for (int i = 0; i < nc; ++i) {
                rml[i] = v.ll[i] * v.tl[i] + d.ll[i] * d.tl[i] - sigma * mu;
                rmu[i] = v.lu[i] * v.tu[i] + d.lu[i] * d.tu[i] - sigma * mu;
            }
            if (absf) newton_solve_abs(&p, &f, &v, rml, rmu, &dc);
            else newton_solve(&p, &f, &v, r.y, r.pi, r.ll, r.lu, rml, rmu, &dc);
            double a_c = max_step(&p, &v, &dc);
            if (a_c > 1.0) a_c = 1.0;
            double mu_c = mu_after(&p, &v, &dc, a_c);
            if (mu_c > arg->corr_ratio * mu_aff) {
                /* conditional corrector rejected: predictor-centering step */
                for (int i = 0; i < nc; ++i) {
                    rml[i] = v.ll[i] * v.tl[i] - sigma * mu;
                    rmu[i] = v.lu[i] * v.tu[i] - sigma * mu;
                }
                if (absf) newton_solve_abs(&p, &f, &v, rml, rmu, &dc);
                else newton_solve(&p, &f, &v, r.y, r.pi, r.ll, r.lu, rml, rmu, &dc);
            }
            step = &dc;
        }
        fac_free(&f);

        double amax = max_step(&p, &v, step);
        double alpha = arg->gamma * amax;
        if (alpha > 1.0) alpha = 1.0;
        for (int i = 0; i < p.nv; ++i) v.y[i] += alpha * step->y[i];
        for (int i = 0; i < p.neq; ++i) v.pi[i] += alpha * step->pi[i];
        for (int i = 0; i < nc; ++i) {
            v.ll[i] += alpha * step->ll[i];
            v.lu[i] += alpha * step->lu[i];
            v.tl[i] += alpha * step->tl[i];
            v.tu[i] += alpha * step->tu[i];
            if (v.ll[i] < arg->lam_min) v.ll[i] = arg->lam_min;
            if (v.lu[i] < arg->lam_min) v.lu[i] = arg->lam_min;
            if (v.tl[i] < arg->t_min) v.tl[i] = arg->t_min;
            if (v.tu[i] < arg->t_min) v.tu[i] = arg->t_min;
        }
        if (alpha < arg->alpha_min) {
            /* report the residuals at the point reached */
            residuals(&p, &v, r.y, r.pi, r.ll, r.lu);
            double lt2 = 0.0, comp2 = 0.0;
            for (int i = 0; i < nc; ++i) {
                double a = v.ll[i] * v.tl[i], b2 = v.lu[i] * v.tu[i];
                lt2 += a + b2;
                if (a > comp2) comp2 = a;
                if (b2 > comp2) comp2 = b2;
            }
            mu = nc ? lt2 / (2.0 * nc) : 0.0;
            double dl2 = inf_norm(r.ll, nc), du2 = inf_norm(r.lu, nc);
            norms[0] = inf_norm(r.y, p.nv);
            norms[1] = inf_norm(r.pi, p.neq);
            norms[2] = du2 > dl2 ? du2 : dl2;
            norms[3] = comp2;
            status = ORC_MIN_STEP;
            ++k;
            break;
        }
    }
    if (absf && status != ORC_NAN) {
        /* residuals only before returning */
        residuals(&p, &v, r.y, r.pi, r.ll, r.lu);
        double comp3 = 0.0;
        for (int i = 0; i < nc; ++i) {
            double a = v.ll[i] * v.tl[i], b2 = v.lu[i] * v.tu[i];
            if (a > comp3) comp3 = a;
            if (b2 > comp3) comp3 = b2;
        }
        double dl3 = inf_norm(r.ll, nc), du3 = inf_norm(r.lu, nc);
        norms[0] = inf_norm(r.y, p.nv);
        norms[1] = inf_norm(r.pi, p.neq);
        norms[2] = du3 > dl3 ? du3 : dl3;
        norms[3] = comp3;
        if (norms[0] != norms[0] || norms[1] != norms[1] || norms[2] != norms[2] || norms[3] != norms[3])
            status = ORC_NAN;
    }
    if (iters) *iters = k;
    if (res_norms) for (int i = 0; i < 4; ++i) res_norms[i] = norms[i];
    if (mu_out) *mu_out = mu;
    ivec_to_user(&p, &v, sol);
    free(wl); free(wu); free(rml); free(rmu);
    ivec_free(&v); ivec_free(&r); ivec_free(&d); ivec_free(&dc);
    prob_free(&p);
    return status;
}

/* Iterative-refinement residual of Section 3.4 at iterate `it` for a step
 * `step` and right-hand side r = (rg, rb, rd, rm) given in `rhs` (user
 * layout, lam_l/lam_u slots = rd lower/upper, t_l/t_u slots = rm lower/upper):
 *   r_ir = K step + r. */
int orc_ir_residual(const orc_qp *qp, const orc_vec *it, const orc_vec *step, const orc_vec *rhs, orc_vec *out)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    ivec_t v, d, c, o;
    ivec_alloc(&p, &v); ivec_alloc(&p, &d); ivec_alloc(&p, &c); ivec_alloc(&p, &o);
    ivec_from_user(&p, it, &v);
    ivec_from_user(&p, step, &d);
    ivec_from_user(&p, rhs, &c);
    kkt_apply(&p, &d, 1, c.y, c.pi, c.ll, c.lu, o.y, o.pi, o.ll, o.lu);
    for (int i = 0; i < p.ncon; ++i) {
        o.tl[i] = v.tl[i] * d.ll[i] + v.ll[i] * d.tl[i] + c.tl[i];
        o.tu[i] = v.tu[i] * d.lu[i] + v.lu[i] * d.tu[i] + c.tu[i];
    }
    ivec_to_user(&p, &o, out);
    ivec_free(&v); ivec_free(&d); ivec_free(&c); ivec_free(&o);
    prob_free(&p);
    return 0;
}

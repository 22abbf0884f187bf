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
    /* Soft constraints (Section 2.2, the slack variables): stage n has ns[n]
     * slacks; slack j relaxes row idxs[j] of the stage's rows [box u, box x,
     * general] on both sides (lower row + s^l, upper row - s^u), with
     * diagonal Hessians Zl, Zu, gradients zl, zu and lower bounds lls, lus
     * (s^l >= lls, s^u >= lus).  ns == NULL: no slacks. */
    const int *ns;
    const int *idxs;
    const double *Zl, *Zu, *zl, *zu, *lls, *lus;
} orc_qp;

typedef struct {
    double tol_stat, tol_eq, tol_ineq, tol_comp;
    int iter_max;
    double alpha_min, gamma, lam_min, t_min, reg_prim, corr_ratio;
    int warm_start; /* 0 cold; 1 primal guess (u, x); 2 primal and dual guess (Section 4.2) */
    int abs_form;   /* 1: absolute formulation (eq:alg:pdipm:abs), exit on the duality measure */
    /* Iterative refinement of the prediction-centering-correction direction
     * (Section 3.4; Section 4.2 refines that direction "in case this is not
     * accurate enough"): up to ir_max corrections, each solving the Newton
     * system again with the refinement residual K d + r as right-hand side,
     * until ||K d + r||_inf <= ir_tol * max(1, largest residual norm at the
     * iterate).  A correction that does not lower the refinement residual is
     * taken back.  ir_max = 0: no refinement (mode speed). */
    int ir_max;
    double ir_tol;
} orc_arg;

/* An iterate, a step or a residual in the user layout: u (sum nu), x (sum nx),
 * pi (sum over n<N of nx[n+1]), and per-stage constraint vectors ordered
 * [box u, box x, general] (sum over n of nbu+nbx+ng). */
typedef struct {
    double *u, *x, *pi, *lam_l, *lam_u, *t_l, *t_u;
    /* slacks s^l, s^u and the multipliers and slacks of their lower bounds
     * (sum over n of ns); may be NULL when the problem has no slacks */
    double *s_l, *s_u, *lam_sl, *lam_su, *t_sl, *t_su;
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
    int ns;                     /* slacks of the stage */
    int *srow;                  /* nc: slack of row k, -1 for a hard row */
    double *Zl, *Zu, *zl, *zu, *lls, *lus; /* ns */
} stage_t;

typedef struct {
    int N;
    stage_t *st;
    int *zoff, *poff, *coff, *uoff, *xoff, *soff;
    int nv, neq, ncon;          /* sizes of y, pi, and of the one-sided constraint count / 2 */
    int nsoft;                  /* number of slacks (each with a lower and an upper copy) */
} prob_t;

#define IX(i, j, ld) ((size_t)(j) * (size_t)(ld) + (size_t)(i))

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

static void prob_free(prob_t *p)
{
    if (!p->st) return;
    for (int n = 0; n <= p->N; ++n) {
        stage_t *s = &p->st[n];
        free(s->H); free(s->g); free(s->F); free(s->bb); free(s->G); free(s->lo); free(s->hi);
        free(s->srow); free(s->Zl); free(s->Zu); free(s->zl); free(s->zu); free(s->lls); free(s->lus);
    }
    free(p->st); free(p->zoff); free(p->poff); free(p->coff); free(p->uoff); free(p->xoff); free(p->soff);
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
    p->soff = (int *)xcalloc((size_t)N + 2, sizeof(int));
    size_t os = 0;
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
        /* slacks */
        int ns = qp->ns ? qp->ns[n] : 0;
        if (ns < 0 || ns > nc) { prob_free(p); return ORC_EINVAL; }
        s->ns = ns;
        s->srow = (int *)xcalloc((size_t)nc, sizeof(int));
        for (int k = 0; k < nc; ++k) s->srow[k] = -1;
        s->Zl = (double *)xcalloc((size_t)ns, sizeof(double));
        s->Zu = (double *)xcalloc((size_t)ns, sizeof(double));
        s->zl = (double *)xcalloc((size_t)ns, sizeof(double));
        s->zu = (double *)xcalloc((size_t)ns, sizeof(double));
        s->lls = (double *)xcalloc((size_t)ns, sizeof(double));
        s->lus = (double *)xcalloc((size_t)ns, sizeof(double));
        for (int j = 0; j < ns; ++j) {
            int k = qp->idxs[os + j];
            if (k < 0 || k >= nc || s->srow[k] >= 0) { prob_free(p); return ORC_EINVAL; }
            s->srow[k] = j;
            s->Zl[j] = qp->Zl[os + j]; s->Zu[j] = qp->Zu[os + j];
            s->zl[j] = qp->zl[os + j]; s->zu[j] = qp->zu[os + j];
            s->lls[j] = qp->lls[os + j]; s->lus[j] = qp->lus[os + j];
            if (!(s->Zl[j] >= 0.0) || !(s->Zu[j] >= 0.0)) { prob_free(p); return ORC_EINVAL; }
        }
        os += ns;
        p->soff[n + 1] = p->soff[n] + ns;
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
    p->nsoft = p->soff[N + 1];
    return 0;
}

/* Internal vectors: y (nv, stage-wise [u; x]), pi (neq, pi_{n+1} for n<N),
 * and four constraint vectors (ncon each). */
typedef struct {
    double *y, *pi, *ll, *lu, *tl, *tu;
    /* slacks (nsoft each): s^l, s^u, multipliers and slacks of s^l >= lls,
     * s^u >= lus */
    double *sl, *su, *lsl, *lsu, *tsl, *tsu;
} ivec_t;

static int ivec_alloc(const prob_t *p, ivec_t *v)
{
    v->y = (double *)xcalloc((size_t)p->nv, sizeof(double));
    v->pi = (double *)xcalloc((size_t)p->neq, sizeof(double));
    v->ll = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    v->lu = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    v->tl = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    v->tu = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    v->sl = (double *)xcalloc((size_t)p->nsoft, sizeof(double));
    v->su = (double *)xcalloc((size_t)p->nsoft, sizeof(double));
    v->lsl = (double *)xcalloc((size_t)p->nsoft, sizeof(double));
    v->lsu = (double *)xcalloc((size_t)p->nsoft, sizeof(double));
    v->tsl = (double *)xcalloc((size_t)p->nsoft, sizeof(double));
    v->tsu = (double *)xcalloc((size_t)p->nsoft, sizeof(double));
    return (v->y && v->pi && v->ll && v->lu && v->tl && v->tu && v->sl && v->su && v->lsl && v->lsu && v->tsl &&
            v->tsu) ? 0 : ORC_ENOMEM;
}

static void ivec_free(ivec_t *v)
{
    free(v->y); free(v->pi); free(v->ll); free(v->lu); free(v->tl); free(v->tu);
    free(v->sl); free(v->su); free(v->lsl); free(v->lsu); free(v->tsl); free(v->tsu);
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
    if (p->nsoft > 0) {
        size_t b = sizeof(double) * (size_t)p->nsoft;
        memcpy(v->sl, in->s_l, b); memcpy(v->su, in->s_u, b);
        memcpy(v->lsl, in->lam_sl, b); memcpy(v->lsu, in->lam_su, b);
        memcpy(v->tsl, in->t_sl, b); memcpy(v->tsu, in->t_su, b);
    }
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
    if (p->nsoft > 0) {
        size_t b = sizeof(double) * (size_t)p->nsoft;
        memcpy(out->s_l, v->sl, b); memcpy(out->s_u, v->su, b);
        memcpy(out->lam_sl, v->lsl, b); memcpy(out->lam_su, v->lsu, b);
        memcpy(out->t_sl, v->tsl, b); memcpy(out->t_su, v->tsu, b);
    }
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
        /* r_d; a soft row holds its slack: lower row G z + s^l, upper row
         * -G z + s^u */
        const double *tl = v->tl + p->coff[n], *tu = v->tu + p->coff[n];
        for (int k = 0; k < s->nc; ++k) {
            double gz = 0.0;
            for (int j = 0; j < s->nz; ++j) gz += s->G[IX(k, j, s->nc)] * z[j];
            const int js = s->srow[k];
            const double sl = js >= 0 ? v->sl[p->soff[n] + js] : 0.0;
            const double su = js >= 0 ? v->su[p->soff[n] + js] : 0.0;
            odl[p->coff[n] + k] = -gz - sl + tl[k] + (cdl ? cdl[p->coff[n] + k] : 0.0);
            odu[p->coff[n] + k] = gz - su + tu[k] + (cdu ? cdu[p->coff[n] + k] : 0.0);
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

/* Slack rows of the residual function (soft constraints, Section 2.2):
 *   r_s^l = Z^l s^l + z^l - lam_l(row) - lam_sl,
 *   r_s^u = Z^u s^u + z^u - lam_u(row) - lam_su,
 *   r_d of the slack bounds: -s^l + t_sl + lls,  -s^u + t_su + lus.
 * Written to r->sl, r->su (stationarity) and r->lsl, r->lsu (r_d). */
static void soft_residuals(const prob_t *p, const ivec_t *v, ivec_t *r)
{
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        for (int k = 0; k < s->nc; ++k) {
            const int js = s->srow[k];
            if (js < 0) continue;
            const int J = p->soff[n] + js, c = p->coff[n] + k;
            r->sl[J] = s->Zl[js] * v->sl[J] + s->zl[js] - v->ll[c] - v->lsl[J];
            r->su[J] = s->Zu[js] * v->su[J] + s->zu[js] - v->lu[c] - v->lsu[J];
            r->lsl[J] = -v->sl[J] + v->tsl[J] + s->lls[js];
            r->lsu[J] = -v->su[J] + v->tsu[J] + s->lus[js];
        }
    }
}

/* IPM residuals at an iterate: constants g, b, d = [lo; -hi]; r_g, r_b,
 * r_d in r->y, r->pi, r->ll, r->lu, the slack rows as in soft_residuals. */
static void residuals(const prob_t *p, const ivec_t *v, ivec_t *r)
{
    double *cg = (double *)xcalloc((size_t)p->nv, sizeof(double));
    double *cb = (double *)xcalloc((size_t)p->neq, sizeof(double));
    double *cdl = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    double *cdu = (double *)xcalloc((size_t)p->ncon, sizeof(double));
    data_terms(p, cg, cb, cdl, cdu);
    kkt_apply(p, v, 1, cg, cb, cdl, cdu, r->y, r->pi, r->ll, r->lu);
    soft_residuals(p, v, r);
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

static double max2(double a, double b) { return (b > a || b != b) ? b : a; }

/* Duality measure mu = lam't / (2 (ncon + nsoft)) over every one-sided row
 * (the two sides of each constraint row and of each slack bound), and the
 * largest lam_i t_i. */
static double duality(const prob_t *p, const ivec_t *v, double *comp)
{
    double lt = 0.0, cm = 0.0;
    for (int i = 0; i < p->ncon; ++i) {
        double a = v->ll[i] * v->tl[i], b = v->lu[i] * v->tu[i];
        lt += a + b;
        cm = max2(max2(cm, a), b);
    }
    for (int i = 0; i < p->nsoft; ++i) {
        double a = v->lsl[i] * v->tsl[i], b = v->lsu[i] * v->tsu[i];
        lt += a + b;
        cm = max2(max2(cm, a), b);
    }
    if (comp) *comp = cm;
    int m = p->ncon + p->nsoft;
    return m ? lt / (2.0 * m) : 0.0;
}

/* The four residual inf-norms (stationarity incl. the slack rows, equality,
 * inequality incl. the slack bounds, complementarity) and mu at iterate v
 * with residuals r. */
static double norms_at(const prob_t *p, const ivec_t *v, const ivec_t *r, double *norms)
{
    double comp = 0.0;
    double mu = duality(p, v, &comp);
    norms[0] = max2(inf_norm(r->y, p->nv), max2(inf_norm(r->sl, p->nsoft), inf_norm(r->su, p->nsoft)));
    norms[1] = inf_norm(r->pi, p->neq);
    norms[2] = max2(max2(inf_norm(r->ll, p->ncon), inf_norm(r->lu, p->ncon)),
                    max2(inf_norm(r->lsl, p->nsoft), inf_norm(r->lsu, p->nsoft)));
    norms[3] = comp;
    return mu;
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

/* Barrier weights of the reduced system eq:alg:kkt per constraint row: w =
 * lam / t on each side.  A soft row's slack is eliminated together with its
 * lower bound (a diagonal block, so the cost is linear in the number of
 * slacks, Section 2.2): with D = Z + w + w_s, w_s = lam_s / t_s, the weight
 * the row puts on G z becomes w - w^2 / D = w (Z + w_s) / D. */
static void barrier_weights(const prob_t *p, const ivec_t *v, double *wl, double *wu)
{
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        for (int k = 0; k < s->nc; ++k) {
            const int c = p->coff[n] + k, js = s->srow[k];
            wl[c] = v->ll[c] / v->tl[c];
            wu[c] = v->lu[c] / v->tu[c];
            if (js < 0) continue;
            const int J = p->soff[n] + js;
            const double wsl = v->lsl[J] / v->tsl[J], wsu = v->lsu[J] / v->tsu[J];
            wl[c] = wl[c] * (s->Zl[js] + wsl) / (s->Zl[js] + wl[c] + wsl);
            wu[c] = wu[c] * (s->Zu[js] + wsu) / (s->Zu[js] + wu[c] + wsu);
        }
    }
}

/* Slack elimination terms of soft row c (slack J of the stage): the
 * diagonals D = Z + w + w_s and the slack rows of the reduced gradient
 * g_s = r_s - e - e_s, with e = w r_d - r_m / t of the row side and e_s the
 * same of the slack bound. */
static void soft_terms(const stage_t *s, int js, int J, int c, const ivec_t *v, const ivec_t *r, double *Dl,
                       double *gl, double *Du, double *gu)
{
    const double wl = v->ll[c] / v->tl[c], wu = v->lu[c] / v->tu[c];
    const double el = wl * r->ll[c] - r->tl[c] / v->tl[c];
    const double eu = wu * r->lu[c] - r->tu[c] / v->tu[c];
    const double wsl = v->lsl[J] / v->tsl[J], wsu = v->lsu[J] / v->tsu[J];
    const double esl = wsl * r->lsl[J] - r->tsl[J] / v->tsl[J];
    const double esu = wsu * r->lsu[J] - r->tsu[J] / v->tsu[J];
    *Dl = s->Zl[js] + wl + wsl;
    *gl = r->sl[J] - el - esl;
    *Du = s->Zu[js] + wu + wsu;
    *gu = r->su[J] - eu - esu;
}

/* Full Newton step of eq:alg:pdipm:delta at iterate v, given the right-hand
 * side r (r_g, r_b, r_d in r->y, r->pi, r->ll/lu; r_m in r->tl/tu; the slack
 * rows r_s in r->sl/su, r_d of the slack bounds in r->lsl/lsu and their r_m
 * in r->tsl/tsu) and a factorization built from barrier_weights.
 * Elimination of dt then dlam (Section 3.3):
 *   gt = rg - C'(W rd - T^{-1} rm)
 *   dt = C dy - rd,    dlam = -T^{-1}(rm + Lam dt).
 * A soft row first eliminates its slack: the slack rows read
 *   D ds^l + w G dz = -g_s^l,  D ds^u - w G dz = -g_s^u,
 * so the row's term e becomes e + w g_s / D (the weight change is in the
 * factorization), and after the Riccati solve ds = -(g_s +- w G dz) / D. */
static void newton_solve(const prob_t *p, const fac_t *f, const ivec_t *v, const ivec_t *r, ivec_t *d)
{
    double *gt = (double *)xcalloc((size_t)p->nv, sizeof(double));
    for (int i = 0; i < p->nv; ++i) gt[i] = r->y[i];
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        int c0 = p->coff[n];
        for (int k = 0; k < s->nc; ++k) {
            int c = c0 + k;
            double wl = v->ll[c] / v->tl[c], wu = v->lu[c] / v->tu[c];
            double el = wl * r->ll[c] - r->tl[c] / v->tl[c];
            double eu = wu * r->lu[c] - r->tu[c] / v->tu[c];
            const int js = s->srow[k];
            if (js >= 0) {
                double Dl, gl, Du, gu;
                soft_terms(s, js, p->soff[n] + js, c, v, r, &Dl, &gl, &Du, &gu);
                el += wl * gl / Dl;
                eu += wu * gu / Du;
            }
            /* C'(e) with C = [G; -G]: G'(el) - G'(eu) */
            for (int j = 0; j < s->nz; ++j) gt[p->zoff[n] + j] -= s->G[IX(k, j, s->nc)] * (el - eu);
        }
    }
    riccati_solve(p, f, gt, r->pi, d->y, d->pi);
    for (int n = 0; n <= p->N; ++n) {
        const stage_t *s = &p->st[n];
        const double *dz = d->y + p->zoff[n];
        for (int k = 0; k < s->nc; ++k) {
            int c = p->coff[n] + k;
            double gdz = 0.0;
            for (int j = 0; j < s->nz; ++j) gdz += s->G[IX(k, j, s->nc)] * dz[j];
            double dsl = 0.0, dsu = 0.0;
            const int js = s->srow[k];
            if (js >= 0) {
                const int J = p->soff[n] + js;
                double Dl, gl, Du, gu;
                soft_terms(s, js, J, c, v, r, &Dl, &gl, &Du, &gu);
                dsl = -(gl + (v->ll[c] / v->tl[c]) * gdz) / Dl;
                dsu = -(gu - (v->lu[c] / v->tu[c]) * gdz) / Du;
                d->sl[J] = dsl;
                d->su[J] = dsu;
                d->tsl[J] = dsl - r->lsl[J];
                d->tsu[J] = dsu - r->lsu[J];
                d->lsl[J] = -(r->tsl[J] + v->lsl[J] * d->tsl[J]) / v->tsl[J];
                d->lsu[J] = -(r->tsu[J] + v->lsu[J] * d->tsu[J]) / v->tsu[J];
            }
            d->tl[c] = gdz + dsl - r->ll[c];
            d->tu[c] = -gdz + dsu - r->lu[c];
            d->ll[c] = -(r->tl[c] + v->ll[c] * d->tl[c]) / v->tl[c];
            d->lu[c] = -(r->tu[c] + v->lu[c] * d->tu[c]) / v->tu[c];
        }
    }
    free(gt);
}

/* Newton step in the absolute formulation (Section 3.2, eq:alg:pdipm:abs):
 * the same matrix with right-hand side -[g; b; d; rm - 2 Lam T e] (the
 * first three blocks linear in the iterate, so only their constant part
 * remains; rm is the delta formulation's complementarity term, e.g. lam.*t -
 * tau, passed in r->tl/tu), whose solution is the full-step iterate; the
 * step is its difference with the current iterate (eq:alg:pdipm:step).
 * Problems with slacks are not taken by this formulation. */
static void newton_solve_abs(const prob_t *p, const fac_t *f, const ivec_t *v, const ivec_t *rm, ivec_t *d)
{
    int nc = p->ncon;
    ivec_t c;
    ivec_alloc(p, &c);
    data_terms(p, c.y, c.pi, c.ll, c.lu);
    for (int i = 0; i < nc; ++i) {
        c.tl[i] = rm->tl[i] - 2.0 * v->ll[i] * v->tl[i];
        c.tu[i] = rm->tu[i] - 2.0 * v->lu[i] * v->tu[i];
    }
    newton_solve(p, f, v, &c, d);
    for (int i = 0; i < p->nv; ++i) d->y[i] -= v->y[i];
    for (int i = 0; i < p->neq; ++i) d->pi[i] -= v->pi[i];
    for (int i = 0; i < nc; ++i) {
        d->ll[i] -= v->ll[i];
        d->lu[i] -= v->lu[i];
        d->tl[i] -= v->tl[i];
        d->tu[i] -= v->tu[i];
    }
    ivec_free(&c);
}

/* Largest alpha (uncapped; HUGE_VAL if no component blocks) keeping every
 * lam + alpha dlam >= 0 and t + alpha dt >= 0 (constraint rows and slack
 * bounds). */
static double max_step(const prob_t *p, const ivec_t *v, const ivec_t *d)
{
    double a = HUGE_VAL;
    const double *vv[8] = {v->ll, v->lu, v->tl, v->tu, v->lsl, v->lsu, v->tsl, v->tsu};
    const double *dd[8] = {d->ll, d->lu, d->tl, d->tu, d->lsl, d->lsu, d->tsl, d->tsu};
    for (int s = 0; s < 8; ++s) {
        const int m = s < 4 ? p->ncon : p->nsoft;
        for (int i = 0; i < m; ++i)
            if (dd[s][i] < 0.0) {
                double r = -vv[s][i] / dd[s][i];
                if (r < a) a = r;
            }
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
    for (int i = 0; i < p->nsoft; ++i) {
        acc += (v->lsl[i] + alpha * d->lsl[i]) * (v->tsl[i] + alpha * d->tsl[i]);
        acc += (v->lsu[i] + alpha * d->lsu[i]) * (v->tsu[i] + alpha * d->tsu[i]);
    }
    return acc / (2.0 * (p->ncon + p->nsoft));
}

/* r_m = lam.*t + a.*b - shift on every one-sided row, written to r->tl/tu
 * and r->tsl/tsu (a, b: the affine step's dlam and dt for the corrector, or
 * NULL), summed in that order. */
static void set_rm(const prob_t *p, const ivec_t *v, const ivec_t *aff, double shift, ivec_t *r)
{
    for (int i = 0; i < p->ncon; ++i) {
        r->tl[i] = (aff ? v->ll[i] * v->tl[i] + aff->ll[i] * aff->tl[i] : v->ll[i] * v->tl[i]) - shift;
        r->tu[i] = (aff ? v->lu[i] * v->tu[i] + aff->lu[i] * aff->tu[i] : v->lu[i] * v->tu[i]) - shift;
    }
    for (int i = 0; i < p->nsoft; ++i) {
        r->tsl[i] = (aff ? v->lsl[i] * v->tsl[i] + aff->lsl[i] * aff->tsl[i] : v->lsl[i] * v->tsl[i]) - shift;
        r->tsu[i] = (aff ? v->lsu[i] * v->tsu[i] + aff->lsu[i] * aff->tsu[i] : v->lsu[i] * v->tsu[i]) - shift;
    }
}


/* Refinement residual of eq:alg:itref at iterate v for step d and
 * right-hand side r (r_g, r_b, r_d in r->y, r->pi, r->ll/lu; r_m in
 * r->tl/tu):  o = K d + r.  Returns ||o||_inf.  Problems without slacks. */
static double ir_apply(const prob_t *p, const ivec_t *v, const ivec_t *d, const ivec_t *r, ivec_t *o)
{
    kkt_apply(p, d, 1, r->y, r->pi, r->ll, r->lu, o->y, o->pi, o->ll, o->lu);
    for (int i = 0; i < p->ncon; ++i) {
        o->tl[i] = v->tl[i] * d->ll[i] + v->ll[i] * d->tl[i] + r->tl[i];
        o->tu[i] = v->tu[i] * d->lu[i] + v->lu[i] * d->tu[i] + r->tu[i];
    }
    double m = max2(inf_norm(o->y, p->nv), inf_norm(o->pi, p->neq));
    m = max2(m, max2(inf_norm(o->ll, p->ncon), inf_norm(o->lu, p->ncon)));
    return max2(m, max2(inf_norm(o->tl, p->ncon), inf_norm(o->tu, p->ncon)));
}

/* d += s * e on every block (problems without slacks) */
static void step_axpy(const prob_t *p, double s, const ivec_t *e, ivec_t *d)
{
    for (int i = 0; i < p->nv; ++i) d->y[i] += s * e->y[i];
    for (int i = 0; i < p->neq; ++i) d->pi[i] += s * e->pi[i];
    for (int i = 0; i < p->ncon; ++i) {
        d->ll[i] += s * e->ll[i];
        d->lu[i] += s * e->lu[i];
        d->tl[i] += s * e->tl[i];
        d->tu[i] += s * e->tu[i];
    }
}

/* Iterative refinement (Section 3.4) of the step d solving K d = -r with
 * the factorization f: each correction e solves K e = -(K d + r) with the
 * same factors.  Stops when ||K d + r||_inf <= tol, after max_steps
 * corrections, or when a correction did not lower the residual (that
 * correction is then taken back).  Returns the corrections kept. */
static int refine_step(const prob_t *p, const fac_t *f, const ivec_t *v, const ivec_t *r, int max_steps, double tol,
                       ivec_t *d)
{
    ivec_t ri, e;
    ivec_alloc(p, &ri);
    ivec_alloc(p, &e);
    int kept = 0;
    double prev = HUGE_VAL;
    for (int it = 0;; ++it) {
        double nr = ir_apply(p, v, d, r, &ri);
        if (it > 0 && !(nr < prev)) {
            step_axpy(p, -1.0, &e, d);
            --kept;
            break;
        }
        if (nr <= tol || it == max_steps) break;
        prev = nr;
        newton_solve(p, f, v, &ri, &e);
        step_axpy(p, 1.0, &e, d);
        ++kept;
    }
    ivec_free(&ri);
    ivec_free(&e);
    return kept;
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                      */
/* ------------------------------------------------------------------------ */

/* Residuals at a user-layout iterate.  Outputs in the user layout of a
 * step (u / x slots hold r_g split by stage, pi slot holds r_b, lam_l/lam_u
 * slots hold r_d lower / upper, t_l/t_u slots hold lam_l*t_l, lam_u*t_u;
 * with slacks, s_l/s_u hold r_s, lam_sl/lam_su the r_d of the slack bounds
 * and t_sl/t_su their lam*t).  norms: inf-norms of r_g (with r_s), r_b, r_d
 * (with the slack bounds) and lam.*t; mu = lam't / n_c over every one-sided
 * row. */
int orc_residuals(const orc_qp *qp, const orc_vec *it, orc_vec *res, double *norms, double *mu)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    ivec_t v, r;
    ivec_alloc(&p, &v); ivec_alloc(&p, &r);
    ivec_from_user(&p, it, &v);
    residuals(&p, &v, &r);
    double nrm[4];
    double m = norms_at(&p, &v, &r, nrm);
    set_rm(&p, &v, NULL, 0.0, &r);
    if (norms) for (int i = 0; i < 4; ++i) norms[i] = nrm[i];
    if (mu) *mu = m;
    if (res) ivec_to_user(&p, &r, res);
    ivec_free(&v); ivec_free(&r);
    prob_free(&p);
    return 0;
}

/* Newton step of eq:alg:pdipm:delta at the iterate `it` with r_m = lam.*t - tau,
 * factorized with regularization `reg`; with abs_form, the same step through
 * the absolute formulation (not for problems with slacks).  Returns the step
 * in user layout. */
int orc_newton_step(const orc_qp *qp, const orc_vec *it, double tau, double reg, int abs_form, orc_vec *step)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    if (abs_form && p.nsoft > 0) { prob_free(&p); return ORC_EINVAL; }
    ivec_t v, r, d;
    ivec_alloc(&p, &v); ivec_alloc(&p, &r); ivec_alloc(&p, &d);
    ivec_from_user(&p, it, &v);
    residuals(&p, &v, &r);
    set_rm(&p, &v, NULL, tau, &r);
    double *wl = (double *)xcalloc((size_t)p.ncon, sizeof(double));
    double *wu = (double *)xcalloc((size_t)p.ncon, sizeof(double));
    barrier_weights(&p, &v, wl, wu);
    fac_t f;
    memset(&f, 0, sizeof(f));
    rc = factorize(&p, wl, wu, reg, &f);
    if (rc == 0) {
        if (abs_form) newton_solve_abs(&p, &f, &v, &r, &d);
        else newton_solve(&p, &f, &v, &r, &d);
        ivec_to_user(&p, &d, step);
    }
    fac_free(&f);
    free(wl); free(wu);
    ivec_free(&v); ivec_free(&r); ivec_free(&d);
    prob_free(&p);
    return rc ? ORC_NAN : 0;
}

/* Newton step of orc_newton_step (delta formulation, no slacks) followed by
 * up to ir_max refinement corrections (Section 3.4) until ||K d + r||_inf <=
 * ir_tol * max(1, largest residual norm at the iterate); the factorization
 * takes the regularization reg, the refinement residual the matrix K without
 * it (Section 4.2: the effect of the regularization can be offset by
 * refinement).  *kept: the corrections kept. */
int orc_newton_step_ir(const orc_qp *qp, const orc_vec *it, double tau, double reg, int ir_max, double ir_tol,
                       orc_vec *step, int *kept)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    if (p.nsoft > 0 || ir_max < 0) { prob_free(&p); return ORC_EINVAL; }
    ivec_t v, r, d;
    ivec_alloc(&p, &v); ivec_alloc(&p, &r); ivec_alloc(&p, &d);
    ivec_from_user(&p, it, &v);
    residuals(&p, &v, &r);
    double norms[4];
    norms_at(&p, &v, &r, norms);
    set_rm(&p, &v, NULL, tau, &r);
    double *wl = (double *)xcalloc((size_t)p.ncon, sizeof(double));
    double *wu = (double *)xcalloc((size_t)p.ncon, sizeof(double));
    barrier_weights(&p, &v, wl, wu);
    fac_t f;
    memset(&f, 0, sizeof(f));
    rc = factorize(&p, wl, wu, reg, &f);
    if (rc == 0) {
        newton_solve(&p, &f, &v, &r, &d);
        const double tol = ir_tol * max2(1.0, max2(max2(norms[0], norms[1]), max2(norms[2], norms[3])));
        int k = refine_step(&p, &f, &v, &r, ir_max, tol, &d);
        if (kept) *kept = k;
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
 * solver status (>= 0) or a usage error (< 0); ir_steps (may be NULL) the
 * refinement corrections kept in total.  Problems with slacks take the delta
 * formulation without refinement. */
int orc_solve(const orc_qp *qp, const orc_arg *arg, orc_vec *sol, int *iters, double *res_norms, double *mu_out,
              int *ir_steps)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    if (p.nsoft > 0 && arg->abs_form != 0) { prob_free(&p); return ORC_EINVAL; }
    /* refinement: delta formulation without slacks */
    if (arg->ir_max < 0 || (arg->ir_max > 0 && (p.nsoft > 0 || arg->abs_form != 0))) { prob_free(&p); return ORC_EINVAL; }
    ivec_t v, r, d, dc;
    ivec_alloc(&p, &v); ivec_alloc(&p, &r); ivec_alloc(&p, &d); ivec_alloc(&p, &dc);
    int nc = p.ncon, nsf = p.nsoft;
    double *wl = (double *)xcalloc((size_t)nc, sizeof(double));
    double *wu = (double *)xcalloc((size_t)nc, sizeof(double));

    /* Initial point.  Cold start: y = 0, pi = 0, t = max(C y - d, 1), lam = 1
     * (slacks s = 0, their bounds' t = max(s - ls, 1), lam = 1).
     * Warm start (Section 4.2) from the iterate passed in `sol`: with a primal
     * guess, y and the slacks s are the guess and the rest is set as in the
     * cold start at that point; with a primal and dual guess, every block is
     * the guess, multipliers and slacks clamped below as in the iterate
     * update. */
    if (arg->warm_start != 0) ivec_from_user(&p, sol, &v);
    if (arg->warm_start == 2) {
        for (int i = 0; i < nc; ++i) {
            if (v.ll[i] < arg->lam_min) v.ll[i] = arg->lam_min;
            if (v.lu[i] < arg->lam_min) v.lu[i] = arg->lam_min;
            if (v.tl[i] < arg->t_min) v.tl[i] = arg->t_min;
            if (v.tu[i] < arg->t_min) v.tu[i] = arg->t_min;
        }
        for (int i = 0; i < nsf; ++i) {
            if (v.lsl[i] < arg->lam_min) v.lsl[i] = arg->lam_min;
            if (v.lsu[i] < arg->lam_min) v.lsu[i] = arg->lam_min;
            if (v.tsl[i] < arg->t_min) v.tsl[i] = arg->t_min;
            if (v.tsu[i] < arg->t_min) v.tsu[i] = arg->t_min;
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
                /* slacks of a soft row: zero, or the guess */
                const int js = s->srow[k];
                const int J = js >= 0 ? p.soff[n] + js : 0;
                const double sl0 = (js >= 0 && arg->warm_start == 1) ? v.sl[J] : 0.0;
                const double su0 = (js >= 0 && arg->warm_start == 1) ? v.su[J] : 0.0;
                double tl0 = gz + sl0 - s->lo[k], tu0 = s->hi[k] - gz + su0;
                v.tl[c] = tl0 > 1.0 ? tl0 : 1.0;
                v.tu[c] = tu0 > 1.0 ? tu0 : 1.0;
                v.ll[c] = 1.0;
                v.lu[c] = 1.0;
                if (js >= 0) {
                    const double tsl0 = sl0 - s->lls[js], tsu0 = su0 - s->lus[js];
                    v.sl[J] = sl0;
                    v.su[J] = su0;
                    v.tsl[J] = tsl0 > 1.0 ? tsl0 : 1.0;
                    v.tsu[J] = tsu0 > 1.0 ? tsu0 : 1.0;
                    v.lsl[J] = 1.0;
                    v.lsu[J] = 1.0;
                }
            }
        }
    }

    int status = ORC_MAX_ITER, k = 0, ir_total = 0;
    double norms[4] = {0, 0, 0, 0}, mu = 0.0;
    const int absf = arg->abs_form != 0;
    for (k = 0;; ++k) {
        /* absolute formulation (Section 4.2, mode speed_abs): no residuals in
         * the loop, exit on the duality measure alone */
        if (absf) {
            mu = duality(&p, &v, NULL);
            if (mu != mu) { status = ORC_NAN; break; }
            if (mu <= arg->tol_comp) { status = ORC_SUCCESS; break; }
        } else {
            residuals(&p, &v, &r);
            mu = norms_at(&p, &v, &r, norms);
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

        /* refinement tolerance relative to the residuals at this iterate */
        const int refine = arg->ir_max > 0;
        const double ir_tol = arg->ir_tol * max2(1.0, max2(max2(norms[0], norms[1]), max2(norms[2], norms[3])));
        barrier_weights(&p, &v, wl, wu);
        fac_t f;
        memset(&f, 0, sizeof(f));
        if (factorize(&p, wl, wu, arg->reg_prim, &f) != 0) { fac_free(&f); status = ORC_NAN; break; }

        /* predictor (affine): r_m = lam.*t */
        set_rm(&p, &v, NULL, 0.0, &r);
        if (absf) newton_solve_abs(&p, &f, &v, &r, &d);
        else newton_solve(&p, &f, &v, &r, &d);
        ivec_t *step = &d;
        if (nc + nsf > 0) {
            double a_aff = max_step(&p, &v, &d);
            if (a_aff > 1.0) a_aff = 1.0;
            double mu_aff = mu_after(&p, &v, &d, a_aff);
            double sigma = mu > 0.0 ? (mu_aff / mu) * (mu_aff / mu) * (mu_aff / mu) : 0.0;
            /* corrector: r_m = lam.*t + dlam_aff.*dt_aff - sigma mu */
            set_rm(&p, &v, &d, sigma * mu, &r);
            if (absf) newton_solve_abs(&p, &f, &v, &r, &dc);
            else newton_solve(&p, &f, &v, &r, &dc);
            if (refine) ir_total += refine_step(&p, &f, &v, &r, arg->ir_max, ir_tol, &dc);
            double a_c = max_step(&p, &v, &dc);
            if (a_c > 1.0) a_c = 1.0;
            double mu_c = mu_after(&p, &v, &dc, a_c);
            if (mu_c > arg->corr_ratio * mu_aff) {
                /* conditional corrector rejected: predictor-centering step */
                set_rm(&p, &v, NULL, sigma * mu, &r);
                if (absf) newton_solve_abs(&p, &f, &v, &r, &dc);
                else newton_solve(&p, &f, &v, &r, &dc);
                if (refine) ir_total += refine_step(&p, &f, &v, &r, arg->ir_max, ir_tol, &dc);
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
        for (int i = 0; i < nsf; ++i) {
            v.sl[i] += alpha * step->sl[i];
            v.su[i] += alpha * step->su[i];
            v.lsl[i] += alpha * step->lsl[i];
            v.lsu[i] += alpha * step->lsu[i];
            v.tsl[i] += alpha * step->tsl[i];
            v.tsu[i] += alpha * step->tsu[i];
            if (v.lsl[i] < arg->lam_min) v.lsl[i] = arg->lam_min;
            if (v.lsu[i] < arg->lam_min) v.lsu[i] = arg->lam_min;
            if (v.tsl[i] < arg->t_min) v.tsl[i] = arg->t_min;
            if (v.tsu[i] < arg->t_min) v.tsu[i] = arg->t_min;
        }
        if (alpha < arg->alpha_min) {
            /* report the residuals at the point reached */
            residuals(&p, &v, &r);
            mu = norms_at(&p, &v, &r, norms);
            status = ORC_MIN_STEP;
            ++k;
            break;
        }
    }
    if (absf && status != ORC_NAN) {
        /* residuals only before returning */
        residuals(&p, &v, &r);
        double mu3 = norms_at(&p, &v, &r, norms);
        (void)mu3;
        if (norms[0] != norms[0] || norms[1] != norms[1] || norms[2] != norms[2] || norms[3] != norms[3])
            status = ORC_NAN;
    }
    if (iters) *iters = k;
    if (ir_steps) *ir_steps = ir_total;
    if (res_norms) for (int i = 0; i < 4; ++i) res_norms[i] = norms[i];
    if (mu_out) *mu_out = mu;
    ivec_to_user(&p, &v, sol);
    free(wl); free(wu);
    ivec_free(&v); ivec_free(&r); ivec_free(&d); ivec_free(&dc);
    prob_free(&p);
    return status;
}

/* Iterative-refinement residual of Section 3.4 at iterate `it` for a step
 * `step` and right-hand side r = (rg, rb, rd, rm) given in `rhs` (user
 * layout, lam_l/lam_u slots = rd lower/upper, t_l/t_u slots = rm lower/upper):
 *   r_ir = K step + r.  Not for problems with slacks. */
int orc_ir_residual(const orc_qp *qp, const orc_vec *it, const orc_vec *step, const orc_vec *rhs, orc_vec *out)
{
    prob_t p;
    int rc = prob_build(qp, &p);
    if (rc) return rc;
    if (p.nsoft > 0) { prob_free(&p); return ORC_EINVAL; }
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

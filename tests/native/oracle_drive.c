/* Drives every entry point of the CPU oracle on small random OCP QPs with
 * stage-varying sizes, box and general rows and soft rows, for a build under
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure: the
 * oracle is compiled into this program).  Prints "ok" and exits 0 when every
 * call returns its expected code; the sanitizers abort on a memory or
 * undefined-behaviour error. */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/oqp_oracle.c"

static unsigned long long g_state = 88172645463325252ull;

static double urand(void) /* xorshift64, uniform in [0, 1) */
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }
static int *ialloc(size_t n) { return (int *)calloc(n ? n : 1, sizeof(int)); }

typedef struct {
    orc_qp q;
    int nu_tot, nx_tot, npi, nc_tot, ns_tot;
    void *owned[40];
    int nown;
} qp_t;

static void *own(qp_t *t, void *p)
{
    t->owned[t->nown++] = p;
    return p;
}

/* random strictly convex OCP QP with N stages; soft: slacks on some rows */
static void make_qp(qp_t *t, int N, int soft)
{
    memset(t, 0, sizeof(*t));
    orc_qp *q = &t->q;
    q->N = N;
    int *nx = own(t, ialloc(N + 1)), *nu = own(t, ialloc(N + 1)), *nbu = own(t, ialloc(N + 1));
    int *nbx = own(t, ialloc(N + 1)), *ng = own(t, ialloc(N + 1)), *ns = own(t, ialloc(N + 1));
    for (int n = 0; n <= N; ++n) {
        nx[n] = 1 + (int)(urand() * 4);
        nu[n] = n < N ? (int)(urand() * 3) : 0;
        nbu[n] = nu[n];
        nbx[n] = n == 0 ? nx[n] : (int)(urand() * (nx[n] + 1));
        ng[n] = n < N ? (int)(urand() * 3) : 0;
        const int nc = nbu[n] + nbx[n] + ng[n];
        ns[n] = (soft && n > 0) ? (int)(urand() * (nc + 1)) : 0;
    }
    size_t sA = 0, sB = 0, sb = 0, sQ = 0, sS = 0, sR = 0, sq = 0, sr = 0, su = 0, sx = 0, sD = 0, sC = 0, sg = 0, ss = 0;
    for (int n = 0; n <= N; ++n) {
        if (n < N) {
            sA += (size_t)nx[n + 1] * nx[n];
            sB += (size_t)nx[n + 1] * nu[n];
            sb += nx[n + 1];
        }
        sQ += (size_t)nx[n] * nx[n];
        sS += (size_t)nu[n] * nx[n];
        sR += (size_t)nu[n] * nu[n];
        sq += nx[n];
        sr += nu[n];
        su += nbu[n];
        sx += nbx[n];
        sD += (size_t)ng[n] * nu[n];
        sC += (size_t)ng[n] * nx[n];
        sg += ng[n];
        ss += ns[n];
        t->nu_tot += nu[n];
        t->nx_tot += nx[n];
        if (n > 0) t->npi += nx[n];
        t->nc_tot += nbu[n] + nbx[n] + ng[n];
    }
    t->ns_tot = (int)ss;
    double *A = own(t, dalloc(sA)), *B = own(t, dalloc(sB)), *b = own(t, dalloc(sb));
    double *Q = own(t, dalloc(sQ)), *S = own(t, dalloc(sS)), *R = own(t, dalloc(sR));
    double *qv = own(t, dalloc(sq)), *rv = own(t, dalloc(sr));
    int *ibu = own(t, ialloc(su)), *ibx = own(t, ialloc(sx));
    double *lbu = own(t, dalloc(su)), *ubu = own(t, dalloc(su)), *lbx = own(t, dalloc(sx)), *ubx = own(t, dalloc(sx));
    double *D = own(t, dalloc(sD)), *C = own(t, dalloc(sC)), *lg = own(t, dalloc(sg)), *ug = own(t, dalloc(sg));
    int *idxs = own(t, ialloc(ss));
    double *Zl = own(t, dalloc(ss)), *Zu = own(t, dalloc(ss)), *zl = own(t, dalloc(ss)), *zu = own(t, dalloc(ss));
    double *lls = own(t, dalloc(ss)), *lus = own(t, dalloc(ss));
    size_t oA = 0, oB = 0, ob = 0, oQ = 0, oS = 0, oR = 0, oq = 0, orr = 0, ou = 0, ox = 0, oD = 0, oC = 0, og = 0, os = 0;
    for (int n = 0; n <= N; ++n) {
        if (n < N) {
            for (int k = 0; k < nx[n + 1] * nx[n]; ++k) A[oA + k] = 0.6 * (urand() - 0.5);
            for (int k = 0; k < nx[n + 1] * nu[n]; ++k) B[oB + k] = urand() - 0.5;
            for (int k = 0; k < nx[n + 1]; ++k) b[ob + k] = 0.1 * (urand() - 0.5);
            oA += (size_t)nx[n + 1] * nx[n];
            oB += (size_t)nx[n + 1] * nu[n];
            ob += nx[n + 1];
        }
        for (int i = 0; i < nx[n]; ++i) Q[oQ + i + i * nx[n]] = 1.0 + urand();
        for (int i = 0; i < nu[n]; ++i) R[oR + i + i * nu[n]] = 0.5 + urand();
        for (int k = 0; k < nx[n]; ++k) qv[oq + k] = 0.2 * (urand() - 0.5);
        for (int k = 0; k < nu[n]; ++k) rv[orr + k] = 0.2 * (urand() - 0.5);
        oQ += (size_t)nx[n] * nx[n];
        oS += (size_t)nu[n] * nx[n];
        oR += (size_t)nu[n] * nu[n];
        oq += nx[n];
        orr += nu[n];
        for (int k = 0; k < nbu[n]; ++k) {
            ibu[ou + k] = k;
            lbu[ou + k] = -1.0 - urand();
            ubu[ou + k] = 1.0 + urand();
        }
        ou += nbu[n];
        for (int k = 0; k < nbx[n]; ++k) {
            ibx[ox + k] = k;
            if (n == 0) {
                lbx[ox + k] = ubx[ox + k] = urand() - 0.5;
            } else {
                lbx[ox + k] = -2.0 - urand();
                ubx[ox + k] = 2.0 + urand();
            }
        }
        ox += nbx[n];
        for (int k = 0; k < ng[n] * nu[n]; ++k) D[oD + k] = urand() - 0.5;
        for (int k = 0; k < ng[n] * nx[n]; ++k) C[oC + k] = urand() - 0.5;
        for (int k = 0; k < ng[n]; ++k) {
            lg[og + k] = -1.0 - urand();
            ug[og + k] = 1.0 + urand();
        }
        oD += (size_t)ng[n] * nu[n];
        oC += (size_t)ng[n] * nx[n];
        og += ng[n];
        for (int k = 0; k < ns[n]; ++k) {
            idxs[os + k] = k; /* rows 0..ns-1 of the stage, each once */
            Zl[os + k] = Zu[os + k] = 0.5 + urand();
            zl[os + k] = zu[os + k] = urand();
            lls[os + k] = lus[os + k] = 0.0;
        }
        os += ns[n];
    }
    q->nx = nx; q->nu = nu; q->nbu = nbu; q->nbx = nbx; q->ng = ng;
    q->A = A; q->B = B; q->b = b; q->Q = Q; q->S = S; q->R = R; q->q = qv; q->r = rv;
    q->idxbu = ibu; q->idxbx = ibx; q->lbu = lbu; q->ubu = ubu; q->lbx = lbx; q->ubx = ubx;
    q->D = D; q->C = C; q->lg = lg; q->ug = ug;
    if (soft) {
        q->ns = ns; q->idxs = idxs; q->Zl = Zl; q->Zu = Zu; q->zl = zl; q->zu = zu; q->lls = lls; q->lus = lus;
    }
}

static void vec_alloc(orc_vec *v, const qp_t *t)
{
    v->u = dalloc(t->nu_tot); v->x = dalloc(t->nx_tot); v->pi = dalloc(t->npi);
    v->lam_l = dalloc(t->nc_tot); v->lam_u = dalloc(t->nc_tot); v->t_l = dalloc(t->nc_tot); v->t_u = dalloc(t->nc_tot);
    v->s_l = dalloc(t->ns_tot); v->s_u = dalloc(t->ns_tot); v->lam_sl = dalloc(t->ns_tot);
    v->lam_su = dalloc(t->ns_tot); v->t_sl = dalloc(t->ns_tot); v->t_su = dalloc(t->ns_tot);
}

static void vec_free(orc_vec *v)
{
    double *p[13] = {v->u, v->x, v->pi, v->lam_l, v->lam_u, v->t_l, v->t_u, v->s_l, v->s_u, v->lam_sl, v->lam_su,
                     v->t_sl, v->t_su};
    for (int k = 0; k < 13; ++k) free(p[k]);
}

static void interior(orc_vec *v, const qp_t *t)
{
    for (int i = 0; i < t->nu_tot; ++i) v->u[i] = urand() - 0.5;
    for (int i = 0; i < t->nx_tot; ++i) v->x[i] = urand() - 0.5;
    for (int i = 0; i < t->npi; ++i) v->pi[i] = urand() - 0.5;
    for (int i = 0; i < t->nc_tot; ++i) {
        v->lam_l[i] = 0.1 + urand(); v->lam_u[i] = 0.1 + urand();
        v->t_l[i] = 0.1 + urand(); v->t_u[i] = 0.1 + urand();
    }
    for (int i = 0; i < t->ns_tot; ++i) {
        v->s_l[i] = urand(); v->s_u[i] = urand();
        v->lam_sl[i] = 0.1 + urand(); v->lam_su[i] = 0.1 + urand();
        v->t_sl[i] = 0.1 + urand(); v->t_su[i] = 0.1 + urand();
    }
}

static int failures = 0;
#define EXPECT(cond, what)                                   \
    do {                                                     \
        if (!(cond)) {                                       \
            fprintf(stderr, "FAIL %s (case %d)\n", what, c); \
            ++failures;                                      \
        }                                                    \
    } while (0)

int main(void)
{
    for (int c = 0; c < 24; ++c) {
        const int soft = c % 3 == 2;
        qp_t t;
        make_qp(&t, 1 + c % 5, soft);
        orc_vec it, out, st, sol;
        vec_alloc(&it, &t); vec_alloc(&out, &t); vec_alloc(&st, &t); vec_alloc(&sol, &t);
        interior(&it, &t);
        double norms[4], mu;
        EXPECT(orc_residuals(&t.q, &it, &out, norms, &mu) == 0, "residuals");
        EXPECT(orc_newton_step(&t.q, &it, 0.1, 0.0, 0, &st) == 0, "newton_step");
        if (!soft) {
            int kept = -1;
            EXPECT(orc_newton_step(&t.q, &it, 0.1, 0.0, 1, &st) == 0, "newton_step abs");
            EXPECT(orc_newton_step_ir(&t.q, &it, 0.1, 1e-3, 5, 1e-12, &st, &kept) == 0 && kept >= 0, "newton_step_ir");
            EXPECT(orc_ir_residual(&t.q, &it, &st, &out, &sol) == 0, "ir_residual");
        } else {
            int kept = 0;
            EXPECT(orc_newton_step_ir(&t.q, &it, 0.1, 0.0, 2, 1e-10, &st, &kept) == ORC_EINVAL, "newton_step_ir soft");
            EXPECT(orc_ir_residual(&t.q, &it, &st, &out, &sol) == ORC_EINVAL, "ir_residual soft");
        }
        orc_arg a = {1e-8, 1e-8, 1e-8, 1e-8, 60, 1e-10, 0.995, 1e-16, 1e-16, 0.0, 10.0, 0, 0, 0, 1e-10};
        int iters = 0, irs = 0;
        double res[4];
        int rc = orc_solve(&t.q, &a, &sol, &iters, res, &mu, &irs);
        EXPECT(rc >= 0 && rc <= ORC_NAN, "solve");
        if (!soft) {
            a.ir_max = 3;
            rc = orc_solve(&t.q, &a, &sol, &iters, res, &mu, &irs);
            EXPECT(rc >= 0 && rc <= ORC_NAN, "solve refined");
            a.ir_max = 0;
            a.abs_form = 1;
            rc = orc_solve(&t.q, &a, &sol, &iters, res, &mu, &irs);
            EXPECT(rc >= 0 && rc <= ORC_NAN, "solve abs");
            a.abs_form = 0;
        } else {
            a.ir_max = 3;
            EXPECT(orc_solve(&t.q, &a, &sol, &iters, res, &mu, &irs) == ORC_EINVAL, "solve refined soft");
            a.ir_max = 0;
        }
        /* warm starts from the last point */
        a.warm_start = 1;
        rc = orc_solve(&t.q, &a, &sol, &iters, res, &mu, &irs);
        EXPECT(rc >= 0 && rc <= ORC_NAN, "solve warm primal");
        a.warm_start = 2;
        rc = orc_solve(&t.q, &a, &sol, &iters, res, &mu, &irs);
        EXPECT(rc >= 0 && rc <= ORC_NAN, "solve warm primal-dual");
        vec_free(&it); vec_free(&out); vec_free(&st); vec_free(&sol);
        for (int k = 0; k < t.nown; ++k) free(t.owned[k]);
    }
    if (failures) return 1;
    printf("ok\n");
    return 0;
}

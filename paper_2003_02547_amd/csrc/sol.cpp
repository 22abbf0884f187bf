// Solution object with per-stage getters (Section 1: getters over an
// internal layout, memory provided by the caller).  Filled from a finished
// batch instance or server request; the getters copy one stage's block of
// the primal solution, the dynamics multipliers, or the multipliers and
// slacks of one kind of constraint.
#include <cstring>

#include "../../include/oqp.h"
#include "internal.h"

struct oqp_sol {
    const oqp_dims* dims;
    int filled;
    oqp_stat stat;
    int64_t* ou;   // N+2 offsets into u
    int64_t* ox;   // into x
    int64_t* op;   // into pi (stage n < N: the multiplier of the dynamics n -> n+1)
    int64_t* oc;   // into the constraint vectors
    double *u, *x, *pi, *ll, *lu, *tl, *tu;
};

namespace {

struct SolSizes {
    int64_t nu, nx, npi, nc;
};

SolSizes sol_sizes(const oqp_dims* d)
{
    SolSizes s{0, 0, 0, 0};
    for (int n = 0; n <= d->N; ++n) {
        s.nu += d->nu[n];
        s.nx += d->nx[n];
        if (n < d->N) s.npi += d->nx[n + 1];
        s.nc += d->nbu[n] + d->nbx[n] + d->ng[n];
    }
    return s;
}

size_t sol_layout(const oqp_dims* d, size_t* off_idx, size_t* off_dbl)
{
    const SolSizes s = sol_sizes(d);
    size_t o = align_up(sizeof(oqp_sol), 16);
    *off_idx = o;
    o = align_up(o + sizeof(int64_t) * 4 * (size_t)(d->N + 2), 16);
    *off_dbl = o;
    o += sizeof(double) * (size_t)(s.nu + s.nx + s.npi + 4 * s.nc + 7);
    return o;
}

enum SolField { S_U, S_X, S_PI, S_LLB_U, S_LUB_U, S_LLB_X, S_LUB_X, S_LLG, S_LUG, S_TLB_U, S_TUB_U, S_TLB_X,
                S_TUB_X, S_TLG, S_TUG };

int sol_get(const oqp_sol* s, int field, int n, double* out)
{
    if (!s || !out) return fail(OQP_EINVAL, "oqp_sol_get: NULL argument");
    const oqp_dims* d = s->dims;
    if (n < 0 || n > d->N) return fail(OQP_EINVAL, "oqp_sol_get: stage %d out of range", n);
    if (!s->filled) return fail(OQP_ESTATE, "oqp_sol_get: solution not filled");
    const double* src = nullptr;
    int64_t cnt = 0;
    const int64_t c0 = s->oc[n];
    const int nbu = d->nbu[n], nbx = d->nbx[n], ng = d->ng[n];
    switch (field) {
    case S_U: src = s->u + s->ou[n]; cnt = d->nu[n]; break;
    case S_X: src = s->x + s->ox[n]; cnt = d->nx[n]; break;
    case S_PI:
        if (n == d->N) return fail(OQP_EINVAL, "oqp_sol_get_pi: stage N has no dynamics");
        src = s->pi + s->op[n];
        cnt = d->nx[n + 1];
        break;
    case S_LLB_U: src = s->ll + c0; cnt = nbu; break;
    case S_LUB_U: src = s->lu + c0; cnt = nbu; break;
    case S_LLB_X: src = s->ll + c0 + nbu; cnt = nbx; break;
    case S_LUB_X: src = s->lu + c0 + nbu; cnt = nbx; break;
    case S_LLG: src = s->ll + c0 + nbu + nbx; cnt = ng; break;
    case S_LUG: src = s->lu + c0 + nbu + nbx; cnt = ng; break;
    case S_TLB_U: src = s->tl + c0; cnt = nbu; break;
    case S_TUB_U: src = s->tu + c0; cnt = nbu; break;
    case S_TLB_X: src = s->tl + c0 + nbu; cnt = nbx; break;
    case S_TUB_X: src = s->tu + c0 + nbu; cnt = nbx; break;
    case S_TLG: src = s->tl + c0 + nbu + nbx; cnt = ng; break;
    case S_TUG: src = s->tu + c0 + nbu + nbx; cnt = ng; break;
    default: return fail(OQP_EINVAL, "oqp_sol_get: bad field");
    }
    if (cnt > 0) std::memcpy(out, src, sizeof(double) * (size_t)cnt);
    return OQP_OK;
}

}  // namespace

extern "C" size_t oqp_sol_bytes(const oqp_dims* dims)
{
    if (!dims) return 0;
    size_t a, b;
    return sol_layout(dims, &a, &b);
}

extern "C" int oqp_sol_init(const oqp_dims* dims, void* mem, size_t bytes, oqp_sol** out)
{
    if (!dims || !mem || !out) return fail(OQP_EINVAL, "oqp_sol_init: NULL argument");
    if ((uintptr_t)mem % 16) return fail(OQP_EINVAL, "oqp_sol_init: memory not 16-byte aligned");
    size_t oi, od;
    const size_t need = sol_layout(dims, &oi, &od);
    if (bytes < need) return fail(OQP_ENOMEM, "oqp_sol_init: %zu < %zu bytes", bytes, need);
    char* m = (char*)mem;
    std::memset(m, 0, need);
    oqp_sol* s = (oqp_sol*)m;
    s->dims = dims;
    const int N = dims->N;
    int64_t* idx = (int64_t*)(m + oi);
    s->ou = idx;
    s->ox = idx + (N + 2);
    s->op = idx + 2 * (N + 2);
    s->oc = idx + 3 * (N + 2);
    int64_t au = 0, ax = 0, ap = 0, ac = 0;
    for (int n = 0; n <= N; ++n) {
        s->ou[n] = au;
        s->ox[n] = ax;
        s->op[n] = ap;
        s->oc[n] = ac;
        au += dims->nu[n];
        ax += dims->nx[n];
        if (n < N) ap += dims->nx[n + 1];
        ac += dims->nbu[n] + dims->nbx[n] + dims->ng[n];
    }
    s->ou[N + 1] = au;
    s->ox[N + 1] = ax;
    s->op[N + 1] = ap;
    s->oc[N + 1] = ac;
    double* dd = (double*)(m + od);
    s->u = dd;
    s->x = s->u + au + 1;
    s->pi = s->x + ax + 1;
    s->ll = s->pi + ap + 1;
    s->lu = s->ll + ac + 1;
    s->tl = s->lu + ac + 1;
    s->tu = s->tl + ac + 1;
    *out = s;
    return OQP_OK;
}

extern "C" int oqp_batch_fill_sol(const oqp_batch* batch, int i, oqp_sol* sol)
{
    if (!batch || !sol) return fail(OQP_EINVAL, "oqp_batch_fill_sol: NULL argument");
    const oqp_dims* d = sol->dims;
    oqp_stat st;
    int rc = oqp_batch_get_stat(batch, i, &st);
    if (rc) return rc;
    if (!batch_dims_match(batch, i, d)) return fail(OQP_EINVAL, "oqp_batch_fill_sol: dims differ from instance %d", i);
    rc = oqp_batch_get_sol(batch, i, sol->u, sol->x, sol->pi, sol->ll, sol->lu, sol->tl, sol->tu);
    if (rc) return rc;
    sol->stat = st;
    sol->filled = 1;
    return OQP_OK;
}

extern "C" int oqp_server_fill_sol(oqp_server* server, uint64_t ticket, oqp_sol* sol)
{
    if (!server || !sol) return fail(OQP_EINVAL, "oqp_server_fill_sol: NULL argument");
    oqp_stat st;
    int rc = oqp_server_poll(server, ticket, &st);
    if (rc < 0) return rc;
    if (rc == OQP_PENDING) return fail(OQP_ESTATE, "oqp_server_fill_sol: request not finished");
    if (!server_dims_match(server, ticket, sol->dims))
        return fail(OQP_EINVAL, "oqp_server_fill_sol: dims differ from the request");
    rc = oqp_server_get_sol(server, ticket, sol->u, sol->x, sol->pi, sol->ll, sol->lu, sol->tl, sol->tu);
    if (rc) return rc;
    sol->stat = st;
    sol->filled = 1;
    return OQP_OK;
}

extern "C" int oqp_sol_get_stat(const oqp_sol* sol, oqp_stat* stat)
{
    if (!sol || !stat) return fail(OQP_EINVAL, "oqp_sol_get_stat: NULL argument");
    if (!sol->filled) return fail(OQP_ESTATE, "oqp_sol_get_stat: solution not filled");
    *stat = sol->stat;
    return OQP_OK;
}

extern "C" int oqp_res_get_norms(const oqp_sol* sol, double* out)
{
    if (!sol || !out) return fail(OQP_EINVAL, "oqp_res_get_norms: NULL argument");
    if (!sol->filled) return fail(OQP_ESTATE, "oqp_res_get_norms: solution not filled");
    for (int k = 0; k < 4; ++k) out[k] = sol->stat.res[k];
    return OQP_OK;
}

#define OQP_SOL_GETTER(name, field) \
    extern "C" int oqp_sol_get_##name(const oqp_sol* sol, int n, double* out) { return sol_get(sol, field, n, out); }
OQP_SOL_GETTER(u, S_U)
OQP_SOL_GETTER(x, S_X)
OQP_SOL_GETTER(pi, S_PI)
OQP_SOL_GETTER(lam_lb_u, S_LLB_U)
OQP_SOL_GETTER(lam_ub_u, S_LUB_U)
OQP_SOL_GETTER(lam_lb_x, S_LLB_X)
OQP_SOL_GETTER(lam_ub_x, S_LUB_X)
OQP_SOL_GETTER(lam_lg, S_LLG)
OQP_SOL_GETTER(lam_ug, S_LUG)
OQP_SOL_GETTER(t_lb_u, S_TLB_U)
OQP_SOL_GETTER(t_ub_u, S_TUB_U)
OQP_SOL_GETTER(t_lb_x, S_TLB_X)
OQP_SOL_GETTER(t_ub_x, S_TUB_X)
OQP_SOL_GETTER(t_lg, S_TLG)
OQP_SOL_GETTER(t_ug, S_TUG)
#undef OQP_SOL_GETTER
